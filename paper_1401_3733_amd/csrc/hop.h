// Wilson hopping term on the even-odd lattice, one thread per output site.
//
//   (H psi)(x) = sum_mu s+ (1 - g_mu) U_mu(x) psi(x+mu) + s- (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)
//
// With g_mu = [[0, A_mu], [A_mu^dag, 0]] (A_0 = 1, A_k = -i sigma_k), the
// projector (1 - sg g_mu) has rank 2: its upper spin pair is
//   h = psi_up - sg A_mu psi_dn
// and its lower pair is -sg A_mu^dag h.  So each of the 8 hops loads the
// neighbour's 4 d components, forms the 2 d-component half spinor h, multiplies
// only h by the d x d link, and rebuilds the lower pair from the product:
// half the link arithmetic of the naive form.  sg = +1 for forward hops and -1
// for backward ones; the adjoint operator flips both.  The boundary sign of
// wrapping hops is folded into the reconstruction coefficients.
#pragma once
#include "dispatch.h"
#include "spinor_io.h"

namespace bsm {

template <int MU, int D, class T>
__device__ inline void project(const cx<T> (&s)[4 * D], T sg, cx<T> (&h0)[D], cx<T> (&h1)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) {
        cx<T> s0 = s[i], s1 = s[D + i], s2 = s[2 * D + i], s3 = s[3 * D + i];
        if constexpr (MU == 0) {          // A psi_dn = (s2, s3)
            h0[i] = mk<T>(fma(-sg, s2.re, s0.re), fma(-sg, s2.im, s0.im));
            h1[i] = mk<T>(fma(-sg, s3.re, s1.re), fma(-sg, s3.im, s1.im));
        } else if constexpr (MU == 1) {   // A psi_dn = (-i s3, -i s2)
            h0[i] = mk<T>(fma(-sg, s3.im, s0.re), fma(sg, s3.re, s0.im));
            h1[i] = mk<T>(fma(-sg, s2.im, s1.re), fma(sg, s2.re, s1.im));
        } else if constexpr (MU == 2) {   // A psi_dn = (-s3, s2)
            h0[i] = mk<T>(fma(sg, s3.re, s0.re), fma(sg, s3.im, s0.im));
            h1[i] = mk<T>(fma(-sg, s2.re, s1.re), fma(-sg, s2.im, s1.im));
        } else {                          // A psi_dn = (-i s2, i s3)
            h0[i] = mk<T>(fma(-sg, s2.im, s0.re), fma(sg, s2.re, s0.im));
            h1[i] = mk<T>(fma(sg, s3.im, s1.re), fma(-sg, s3.re, s1.im));
        }
    }
}

// acc_up += w g ;  acc_dn += -sg w A_mu^dag g
template <int MU, int D, class T>
__device__ inline void reconstruct(cx<T> (&acc)[4 * D], T sg, T w, const cx<T> (&g0)[D],
                                   const cx<T> (&g1)[D]) {
    const T v = -sg * w;
#pragma unroll
    for (int i = 0; i < D; i++) {
        acc[i].re = fma(w, g0[i].re, acc[i].re);
        acc[i].im = fma(w, g0[i].im, acc[i].im);
        acc[D + i].re = fma(w, g1[i].re, acc[D + i].re);
        acc[D + i].im = fma(w, g1[i].im, acc[D + i].im);
        cx<T> &a2 = acc[2 * D + i];
        cx<T> &a3 = acc[3 * D + i];
        if constexpr (MU == 0) {          // A^dag g = (g0, g1)
            a2.re = fma(v, g0[i].re, a2.re); a2.im = fma(v, g0[i].im, a2.im);
            a3.re = fma(v, g1[i].re, a3.re); a3.im = fma(v, g1[i].im, a3.im);
        } else if constexpr (MU == 1) {   // A^dag g = (i g1, i g0)
            a2.re = fma(-v, g1[i].im, a2.re); a2.im = fma(v, g1[i].re, a2.im);
            a3.re = fma(-v, g0[i].im, a3.re); a3.im = fma(v, g0[i].re, a3.im);
        } else if constexpr (MU == 2) {   // A^dag g = (g1, -g0)
            a2.re = fma(v, g1[i].re, a2.re); a2.im = fma(v, g1[i].im, a2.im);
            a3.re = fma(-v, g0[i].re, a3.re); a3.im = fma(-v, g0[i].im, a3.im);
        } else {                          // A^dag g = (i g0, -i g1)
            a2.re = fma(-v, g0[i].im, a2.re); a2.im = fma(v, g0[i].re, a2.im);
            a3.re = fma(v, g1[i].im, a3.re); a3.im = fma(-v, g1[i].re, a3.im);
        }
    }
}

// g = U h (forward) or U^dag h (backward) for both spin components
template <int D, bool REAL, int LP, bool BACK, class T>
__device__ inline void link_mul(const void *blk, int64_t stride, uint32_t hl, const cx<T> (&h0)[D],
                                const cx<T> (&h1)[D], cx<T> (&g0)[D], cx<T> (&g1)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) { g0[i] = mk<T>(0, 0); g1[i] = mk<T>(0, 0); }
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            cx<T> u = load_link<LP, REAL, T>(blk, stride, i * D + j, hl);
            if constexpr (REAL) {
                // real link: U_ij (forward) and U^T_ji (backward) are the same number
                if constexpr (!BACK) {
                    g0[i].re = fma(u.re, h0[j].re, g0[i].re); g0[i].im = fma(u.re, h0[j].im, g0[i].im);
                    g1[i].re = fma(u.re, h1[j].re, g1[i].re); g1[i].im = fma(u.re, h1[j].im, g1[i].im);
                } else {
                    g0[j].re = fma(u.re, h0[i].re, g0[j].re); g0[j].im = fma(u.re, h0[i].im, g0[j].im);
                    g1[j].re = fma(u.re, h1[i].re, g1[j].re); g1[j].im = fma(u.re, h1[i].im, g1[j].im);
                }
            } else {
                if constexpr (!BACK) {
                    g0[i] = cfma(u, h0[j], g0[i]);
                    g1[i] = cfma(u, h1[j], g1[i]);
                } else {
                    // (U^dag h)_j += conj(U_ij) h_i
                    g0[j] = cfma_conj(u, h0[i], g0[j]);
                    g1[j] = cfma_conj(u, h1[i], g1[j]);
                }
            }
        }
}

template <int MU, int D, bool REAL, int SP, int LP, class T>
__device__ inline void hop_dir(const Geom &g, const Coords &c, int p, uint32_t h, const char *U,
                               size_t lblk, const char *in, T eta, cx<T> (&acc)[4 * D]) {
    const int64_t S = g.Vh_pad;
    // coordinates in direction mu, extent
    const int Lmu = g.L[MU];
    const int xm = MU == 0 ? c.t : MU == 1 ? c.x : MU == 2 ? c.y : c.z;
    const bool ap = (g.apbc >> MU) & 1;
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        const bool back = dir == 1;
        int xn = back ? xm - 1 : xm + 1;
        T w = (T)1;
        if (xn == Lmu) { xn = 0; if (ap) w = (T)-1; }
        if (xn < 0) { xn = Lmu - 1; if (ap) w = (T)-1; }
        uint32_t hn;
        if constexpr (MU == 1) {
            hn = (uint32_t)c.row * g.LXh + (xn >> 1);
        } else {
            int t = c.t, z = c.z, y = c.y;
            if (MU == 0) t = xn;
            if (MU == 2) y = xn;
            if (MU == 3) z = xn;
            uint32_t row = ((uint32_t)t * g.L[3] + z) * g.L[2] + y;
            hn = row * g.LXh + c.xh;
        }
        cx<T> s[4 * D];
        load_spinor<SP, D, T>(in, S, hn, s);
        const T sg = back ? -eta : eta;
        cx<T> h0[D], h1[D], g0[D], g1[D];
        project<MU, D, T>(s, sg, h0, h1);
        if (!back) {
            const char *blk = U + (size_t)(p * 4 + MU) * lblk;
            link_mul<D, REAL, LP, false, T>(blk, S, h, h0, h1, g0, g1);
        } else {
            const char *blk = U + (size_t)((1 - p) * 4 + MU) * lblk;
            link_mul<D, REAL, LP, true, T>(blk, S, hn, h0, h1, g0, g1);
        }
        reconstruct<MU, D, T>(acc, sg, w, g0, g1);
    }
}

template <int D, bool REAL, int SP, int LP>
__global__ __launch_bounds__(256) void k_hop(Geom g, HopArgs a, int nblk) {
    using T = typename Compute<SP>::T;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int pi = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t h = (lb - pi * nblk) * 256 + threadIdx.x;
    const int p = a.p0 + pi;
    const bool active = h < (uint32_t)g.Vh;
    const size_t lblk = link_block_bytes(LP, REAL, D, g.Vh_pad);
    double nrm = 0.0;
    if (active) {
        cx<T> acc[4 * D];
#pragma unroll
        for (int k = 0; k < 4 * D; k++) acc[k] = mk<T>(0, 0);
        Coords c = decode(g, h, p);
        const char *in = (const char *)a.in[p];
        const char *U = (const char *)a.U;
        const T eta = a.dagger ? (T)-1 : (T)1;
        hop_dir<0, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        hop_dir<1, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        hop_dir<2, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        hop_dir<3, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        const T bb = (T)a.b;
#pragma unroll
        for (int k = 0; k < 4 * D; k++) acc[k] = bb * acc[k];
        if (a.a != 0.0) {
            cx<T> xs[4 * D];
            load_spinor<SP, D, T>(a.x[p], g.Vh_pad, h, xs);
            const T aa = (T)a.a;
#pragma unroll
            for (int k = 0; k < 4 * D; k++) {
                acc[k].re = fma(aa, xs[k].re, acc[k].re);
                acc[k].im = fma(aa, xs[k].im, acc[k].im);
            }
        }
        store_spinor<SP, D, T>(a.out[p], g.Vh_pad, h, acc);
        if (a.norm_partials) {
#pragma unroll
            for (int k = 0; k < 4 * D; k++)
                nrm += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
        }
    }
    if (a.norm_partials) {
        double s = block_sum_256(nrm);
        if (threadIdx.x == 0) a.norm_partials[lb] = s;
    }
}

// Launch for one (spinor precision, link precision, d_R); the definitions are
// explicitly instantiated in the hop_*.hip sources (split so they build in
// parallel).
template <int SP, int LP, int D>
bsm_status hop_run(const Geom &g, bool real, const HopArgs &a, hipStream_t st) {
    int nblk = (g.Vh + 255) / 256;
    dim3 grid(nblk * a.np);
    if (real) {
        if constexpr (D == 3 || D == 8 || D == 15)
            k_hop<D, true, SP, LP><<<grid, 256, 0, st>>>(g, a, nblk);
        else
            return fail(BSM_ERR_UNSUPPORTED, "real links only for adjoint d_R 3, 8, 15");
    } else {
        k_hop<D, false, SP, LP><<<grid, 256, 0, st>>>(g, a, nblk);
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

#define BSM_HOP_INSTANTIATE(SP, LP, D) \
    template bsm_status hop_run<SP, LP, D>(const Geom &, bool, const HopArgs &, hipStream_t);


}  // namespace bsm
