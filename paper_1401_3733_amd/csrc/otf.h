// Links in a higher representation formed on the fly from the fundamental
// link (the gauge field holds only the N x N matrices U, the field content the
// paper counts, Section II.A), applied without building the d_R x d_R matrix
// R(U):
//
//   two-index (sym SG = +1, asym SG = -1): a colour vector v is the matrix
//     S = sum_A v_A e_A  (e_(aa) = E_aa, e_(ab) = (E_ab + SG E_ba)/sqrt2),
//     and R(U) v is the vector of V S V^T with V = U, i.e. out_(aa) = S'_aa,
//     out_(ab) = sqrt2 S'_ab (S' has the symmetry of S);
//   adjoint: v is X = sum_a v_a T_a (generalised Gell-Mann / 2), R(U) v is
//     the vector of X' = V X V^dag, out_a = 2 Tr(T_a X').
//
// The backward hop needs R(U)^dag = R(U^dag): the same with V = U^dag.
// These are the definitions R_AB = Tr(e_A^dag U e_B U^T) and
// R_ab = 2 Tr(T_a U T_b U^dag) applied to v, so the result equals R(U) v up
// to rounding.  Basis order as in the representation kernel: pairs a <= b
// (a < b) lexicographic; adjoint pairs j < k lexicographic, symmetric then
// antisymmetric generator of each pair, then the N - 1 diagonal ones.
#pragma once
#include "bsm_internal.h"

namespace bsm {

// (rep, N) of an on-the-fly operator packed as RN = rep * 16 + N (0: links
// stored in the representation)
constexpr int otf_rn(int rep, int N) { return rep * 16 + N; }
constexpr int otf_rep(int rn) { return rn >> 4; }
constexpr int otf_n(int rn) { return rn & 15; }
constexpr int otf_dim(int rn) {
    return otf_rep(rn) == BSM_REP_ADJ ? otf_n(rn) * otf_n(rn) - 1
         : otf_rep(rn) == BSM_REP_SYM ? otf_n(rn) * (otf_n(rn) + 1) / 2
         : otf_rep(rn) == BSM_REP_ASYM ? otf_n(rn) * (otf_n(rn) - 1) / 2
                                       : otf_n(rn);
}

// V_ij = U_ij (forward) or conj(U_ji) (backward)
template <int N, bool BACK, class T>
__device__ inline cx<T> vmat(const cx<T> (&u)[N * N], int i, int j) {
    if constexpr (!BACK) return u[i * N + j];
    else return mk<T>(u[j * N + i].re, -u[j * N + i].im);
}

template <int N, int SG, bool BACK, class T>
__device__ inline void twoindex_apply(const cx<T> (&u)[N * N], const cx<T> *h, cx<T> *out) {
    constexpr T w = (T)0.70710678118654752440;
    constexpr T r2 = (T)1.41421356237309504880;
    cx<T> S[N * N];
    {
        int A = 0;
#pragma unroll
        for (int a = 0; a < N; a++) {
            S[a * N + a] = mk<T>(0, 0);
#pragma unroll
            for (int b = a; b < N; b++) {
                if (a == b && SG < 0) continue;
                if (a == b) {
                    S[a * N + a] = h[A];
                } else {
                    S[a * N + b] = w * h[A];
                    S[b * N + a] = (SG > 0 ? w : -w) * h[A];
                }
                A++;
            }
        }
    }
    // T1 = V S
    cx<T> T1[N * N];
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int k = 0; k < N; k++) {
            cx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int j = 0; j < N; j++) acc = cfma(vmat<N, BACK, T>(u, i, j), S[j * N + k], acc);
            T1[i * N + k] = acc;
        }
    // out from S' = T1 V^T: S'_ab = sum_k T1_ak V_bk
    int A = 0;
#pragma unroll
    for (int a = 0; a < N; a++)
#pragma unroll
        for (int b = a; b < N; b++) {
            if (a == b && SG < 0) continue;
            cx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int k = 0; k < N; k++) acc = cfma(T1[a * N + k], vmat<N, BACK, T>(u, b, k), acc);
            out[A] = a == b ? acc : r2 * acc;
            A++;
        }
}

template <int N, bool BACK, class T>
__device__ inline void adjoint_apply(const cx<T> (&u)[N * N], const cx<T> *h, cx<T> *out) {
    constexpr int NP = N * (N - 1) / 2;
    // X = sum_a h_a T_a
    cx<T> X[N * N];
#pragma unroll
    for (int e = 0; e < N * N; e++) X[e] = mk<T>(0, 0);
    {
        int pair = 0;
#pragma unroll
        for (int j = 0; j < N; j++)
#pragma unroll
            for (int k = j + 1; k < N; k++) {
                const cx<T> s = h[2 * pair], a = h[2 * pair + 1];
                // (E_jk + E_kj)/2 s + (-i E_jk + i E_kj)/2 a
                X[j * N + k] = mk<T>((T)0.5 * (s.re + a.im), (T)0.5 * (s.im - a.re));
                X[k * N + j] = mk<T>((T)0.5 * (s.re - a.im), (T)0.5 * (s.im + a.re));
                pair++;
            }
#pragma unroll
        for (int l = 1; l < N; l++) {
            const T nrm = (T)(1.0 / __builtin_sqrt(2.0 * l * (l + 1)));
            const cx<T> c = h[2 * NP + l - 1];
#pragma unroll
            for (int m = 0; m < l; m++) X[m * N + m] = X[m * N + m] + nrm * c;
            X[l * N + l] = X[l * N + l] - (T)l * nrm * c;
        }
    }
    // Y = V X
    cx<T> Y[N * N];
#pragma unroll
    for (int i = 0; i < N; i++)
#pragma unroll
        for (int k = 0; k < N; k++) {
            cx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int j = 0; j < N; j++) acc = cfma(vmat<N, BACK, T>(u, i, j), X[j * N + k], acc);
            Y[i * N + k] = acc;
        }
    // X'_ij = sum_k Y_ik conj(V_jk), consumed entry by entry
    auto xp = [&](int i, int j) {
        cx<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int k = 0; k < N; k++) acc = cfma_conj(vmat<N, BACK, T>(u, j, k), Y[i * N + k], acc);
        return acc;
    };
    {
        int pair = 0;
#pragma unroll
        for (int j = 0; j < N; j++)
#pragma unroll
            for (int k = j + 1; k < N; k++) {
                const cx<T> xjk = xp(j, k), xkj = xp(k, j);
                out[2 * pair] = xjk + xkj;                                    // 2 Tr(T_sym X')
                out[2 * pair + 1] = mk<T>(xkj.im - xjk.im, xjk.re - xkj.re);  // i (X'_jk - X'_kj)
                pair++;
            }
    }
    cx<T> diag[N];
#pragma unroll
    for (int m = 0; m < N; m++) diag[m] = xp(m, m);
#pragma unroll
    for (int l = 1; l < N; l++) {
        const T nrm = (T)(2.0 / __builtin_sqrt(2.0 * l * (l + 1)));
        cx<T> s = mk<T>(0, 0);
#pragma unroll
        for (int m = 0; m < l; m++) s = s + diag[m];
        s = s - (T)l * diag[l];
        out[2 * NP + l - 1] = nrm * s;
    }
}

// g = R(U) h (forward) or R(U)^dag h (backward) for the representation RN
template <int RN, bool BACK, class T>
__device__ inline void rep_apply(const cx<T> (&u)[otf_n(RN) * otf_n(RN)], const cx<T> *h, cx<T> *g) {
    constexpr int N = otf_n(RN);
    if constexpr (otf_rep(RN) == BSM_REP_SYM) twoindex_apply<N, 1, BACK, T>(u, h, g);
    else if constexpr (otf_rep(RN) == BSM_REP_ASYM) twoindex_apply<N, -1, BACK, T>(u, h, g);
    else if constexpr (otf_rep(RN) == BSM_REP_ADJ) adjoint_apply<N, BACK, T>(u, h, g);
    else {
#pragma unroll
        for (int i = 0; i < N; i++) {
            cx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int j = 0; j < N; j++) acc = cfma(vmat<N, BACK, T>(u, i, j), h[j], acc);
            g[i] = acc;
        }
    }
}

}  // namespace bsm
