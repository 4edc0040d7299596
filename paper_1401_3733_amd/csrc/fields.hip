// Layout conversion (canonical complex128 <-> internal even-odd SoA) and the
// representation map of the links.
#include "dispatch.h"
#include "spinor_io.h"

namespace bsm {

// ----------------------------------------------------------------- spinors
template <int P, int D>
__global__ __launch_bounds__(256) void k_pack_spinor(Geom g, const double2 *canon, char *internal,
                                                     size_t field_bytes, size_t block_bytes) {
    uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    int p = blockIdx.y;
    int r = blockIdx.z;
    if (h >= (uint32_t)g.Vh_pad) return;
    using T = double;
    cx<T> s[4 * D];
    if (h < (uint32_t)g.Vh) {
        Coords c = decode(g, h, p);
        int64_t lex = (int64_t)c.row * g.L[1] + c.x;
        const double2 *src = canon + ((int64_t)r * 2 * g.Vh + lex) * 4 * D;
#pragma unroll
        for (int k = 0; k < 4 * D; k++) s[k] = mk<T>(src[k].x, src[k].y);
    } else {
#pragma unroll
        for (int k = 0; k < 4 * D; k++) s[k] = mk<T>(0.0, 0.0);
    }
    store_spinor<P, D, T>(internal + r * field_bytes + p * block_bytes, g.Vh_pad, h, s);
}

template <int P, int D>
__global__ __launch_bounds__(256) void k_unpack_spinor(Geom g, const char *internal, double2 *canon,
                                                       size_t field_bytes, size_t block_bytes) {
    uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    int p = blockIdx.y;
    int r = blockIdx.z;
    if (h >= (uint32_t)g.Vh) return;
    using T = double;
    cx<T> s[4 * D];
    load_spinor<P, D, T>(internal + r * field_bytes + p * block_bytes, g.Vh_pad, h, s);
    Coords c = decode(g, h, p);
    int64_t lex = (int64_t)c.row * g.L[1] + c.x;
    double2 *dst = canon + ((int64_t)r * 2 * g.Vh + lex) * 4 * D;
#pragma unroll
    for (int k = 0; k < 4 * D; k++) dst[k] = make_double2(s[k].re, s[k].im);
}

template <int P, int D>
struct PackLaunch {
    static bsm_status run(Geom g, int n_rhs, const void *canon, void *internal, hipStream_t st,
                          bool unpack) {
        size_t bb = spinor_block_bytes(P, D, g.Vh_pad);
        dim3 grid((g.Vh_pad + 255) / 256, 2, n_rhs);
        if (!unpack)
            k_pack_spinor<P, D><<<grid, 256, 0, st>>>(g, (const double2 *)canon, (char *)internal,
                                                      2 * bb, bb);
        else
            k_unpack_spinor<P, D><<<grid, 256, 0, st>>>(g, (const char *)internal, (double2 *)canon,
                                                        2 * bb, bb);
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
};

template <int D>
struct PackByD {
    static bsm_status run(int prec, Geom g, int n_rhs, const void *canon, void *internal,
                          hipStream_t st, bool unpack) {
        switch (prec) {
        case BSM_F64: return PackLaunch<BSM_F64, D>::run(g, n_rhs, canon, internal, st, unpack);
        case BSM_F32: return PackLaunch<BSM_F32, D>::run(g, n_rhs, canon, internal, st, unpack);
        case BSM_F16S: return PackLaunch<BSM_F16S, D>::run(g, n_rhs, canon, internal, st, unpack);
        }
        return fail(BSM_ERR_ARG, "bad spinor precision");
    }
};

bsm_status launch_pack_spinor(const Geom &g, int d, int prec, int n_rhs, const void *canon,
                              void *internal, hipStream_t st, bool unpack) {
    return dispatch_d<PackByD>(d, prec, g, n_rhs, canon, internal, st, unpack);
}

// ----------------------------------------------------------- representation
// Generators of su(N) in the adjoint basis: for each pair j<k the symmetric
// (E_jk + E_kj)/2 and antisymmetric (-i E_jk + i E_kj)/2 matrix, then the
// diagonal diag(1,..,1,-l,0..)/sqrt(2 l (l+1)), l = 1..N-1.  A generator is
// returned as its (at most N) nonzero entries.
struct Sparse {
    int n;
    int r[16], c[16];
    double re[16], im[16];
};

__device__ inline void adj_generator(int N, int a, Sparse &s) {
    int npair = N * (N - 1) / 2;
    s.n = 0;
    if (a < 2 * npair) {
        int pair = a >> 1, type = a & 1;
        int j = 0, k = 1, cnt = 0;
        for (j = 0; j < N; j++) {
            bool found = false;
            for (k = j + 1; k < N; k++) {
                if (cnt == pair) { found = true; break; }
                cnt++;
            }
            if (found) break;
        }
        s.n = 2;
        s.r[0] = j; s.c[0] = k;
        s.r[1] = k; s.c[1] = j;
        if (type == 0) {
            s.re[0] = 0.5; s.im[0] = 0; s.re[1] = 0.5; s.im[1] = 0;
        } else {
            s.re[0] = 0; s.im[0] = -0.5; s.re[1] = 0; s.im[1] = 0.5;
        }
    } else {
        int l = a - 2 * npair + 1;
        double nrm = 1.0 / sqrt(2.0 * l * (l + 1));
        for (int m = 0; m <= l; m++) {
            s.r[m] = m; s.c[m] = m;
            s.re[m] = (m < l) ? nrm : -l * nrm;
            s.im[m] = 0;
        }
        s.n = l + 1;
    }
}

// two-index basis element A for sym (sg = +1) / asym (sg = -1)
__device__ inline void twoindex_basis(int N, int sg, int A, Sparse &s) {
    int cnt = 0;
    for (int a = 0; a < N; a++)
        for (int b = a; b < N; b++) {
            if (a == b && sg < 0) continue;
            if (cnt == A) {
                if (a == b) {
                    s.n = 1; s.r[0] = a; s.c[0] = a; s.re[0] = 1; s.im[0] = 0;
                } else {
                    double w = 0.70710678118654752440;
                    s.n = 2;
                    s.r[0] = a; s.c[0] = b; s.re[0] = w; s.im[0] = 0;
                    s.r[1] = b; s.c[1] = a; s.re[1] = sg * w; s.im[1] = 0;
                }
                return;
            }
            cnt++;
        }
    s.n = 0;
}

template <int LP, bool REAL>
__device__ inline void store_link(void *blk, int64_t stride, int e, uint32_t h, double re, double im) {
    if constexpr (REAL) {
        if constexpr (LP == BSM_F64) ((double *)blk)[e * stride + h] = re;
        else if constexpr (LP == BSM_F32) ((float *)blk)[e * stride + h] = (float)re;
        else ((__half *)blk)[e * stride + h] = __float2half_rn((float)re);
    } else {
        if constexpr (LP == BSM_F64) ((double2 *)blk)[e * stride + h] = make_double2(re, im);
        else if constexpr (LP == BSM_F32) ((float2 *)blk)[e * stride + h] = make_float2((float)re, (float)im);
        else ((__half2 *)blk)[e * stride + h] = __halves2half2(__float2half_rn((float)re), __float2half_rn((float)im));
    }
}

// One thread per (link, column b of R(U)).  Links: block (p, mu) for
// blockIdx.y = p*4 + mu; canonical input U_mu(x) at [lex][mu].
template <int LP, bool REAL>
__global__ __launch_bounds__(128) void k_represent(Geom g, int N, int rep, int d,
                                                   const double2 *Uc, char *out) {
    uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    int p = blockIdx.y >> 2, mu = blockIdx.y & 3;
    int b = blockIdx.z;
    if (h >= (uint32_t)g.Vh_pad) return;
    size_t blk_bytes = link_elem_bytes(LP, REAL) * d * d * g.Vh_pad;
    char *blk = out + (size_t)(p * 4 + mu) * blk_bytes;
    if (h >= (uint32_t)g.Vh) {
        for (int a = 0; a < d; a++) store_link<LP, REAL>(blk, g.Vh_pad, a * d + b, h, 0.0, 0.0);
        return;
    }
    Coords c = decode(g, h, p);
    int64_t lex = (int64_t)c.row * g.L[1] + c.x;
    const double2 *u = Uc + (lex * 4 + mu) * N * N;
    if (rep == BSM_REP_FUND) {
        for (int a = 0; a < d; a++) {
            double2 v = u[a * N + b];
            store_link<LP, REAL>(blk, g.Vh_pad, a * d + b, h, v.x, v.y);
        }
        return;
    }
    // X = U e_b U^dag (adj) or U e_b U^T (two-index), e_b sparse; N <= 6
    double Xr[36], Xi[36];
    Sparse eb;
    if (rep == BSM_REP_ADJ) adj_generator(N, b, eb);
    else twoindex_basis(N, rep == BSM_REP_SYM ? 1 : -1, b, eb);
    for (int m = 0; m < N; m++)
        for (int n = 0; n < N; n++) {
            double sr = 0, si = 0;
            for (int q = 0; q < eb.n; q++) {
                double2 um = u[m * N + eb.r[q]];     // U_{m, r}
                double2 un = u[n * N + eb.c[q]];     // U_{n, c}
                if (rep == BSM_REP_ADJ) un.y = -un.y;   // conj for U^dag
                // e * U_{m r} * (U_{n c} or conj)
                double pr = um.x * un.x - um.y * un.y, pi = um.x * un.y + um.y * un.x;
                sr += eb.re[q] * pr - eb.im[q] * pi;
                si += eb.re[q] * pi + eb.im[q] * pr;
            }
            Xr[m * N + n] = sr;
            Xi[m * N + n] = si;
        }
    for (int a = 0; a < d; a++) {
        Sparse ea;
        if (rep == BSM_REP_ADJ) adj_generator(N, a, ea);
        else twoindex_basis(N, rep == BSM_REP_SYM ? 1 : -1, a, ea);
        double rr = 0, ri = 0;
        for (int q = 0; q < ea.n; q++) {
            int i = ea.r[q], j = ea.c[q];
            if (rep == BSM_REP_ADJ) {
                // 2 Tr(T_a X) = 2 sum (T_a)_{ij} X_{ji}
                double xr = Xr[j * N + i], xi = Xi[j * N + i];
                rr += 2 * (ea.re[q] * xr - ea.im[q] * xi);
                ri += 2 * (ea.re[q] * xi + ea.im[q] * xr);
            } else {
                // Tr(e_a^dag X) = sum conj((e_a)_{ij}) X_{ij}
                double xr = Xr[i * N + j], xi = Xi[i * N + j];
                rr += ea.re[q] * xr + ea.im[q] * xi;
                ri += ea.re[q] * xi - ea.im[q] * xr;
            }
        }
        store_link<LP, REAL>(blk, g.Vh_pad, a * d + b, h, rr, ri);
    }
}

template <int LP, bool REAL>
__global__ __launch_bounds__(128) void k_unpack_gauge(Geom g, int d, const char *in, double2 *canon) {
    uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    int p = blockIdx.y >> 2, mu = blockIdx.y & 3;
    if (h >= (uint32_t)g.Vh) return;
    size_t blk_bytes = link_elem_bytes(LP, REAL) * d * d * g.Vh_pad;
    const char *blk = in + (size_t)(p * 4 + mu) * blk_bytes;
    Coords c = decode(g, h, p);
    int64_t lex = (int64_t)c.row * g.L[1] + c.x;
    double2 *dst = canon + (lex * 4 + mu) * d * d;
    for (int e = 0; e < d * d; e++) {
        cx<double> v = load_link<LP, REAL, double>(blk, g.Vh_pad, e, h);
        dst[e] = make_double2(v.re, v.im);
    }
}

template <int LP, bool REAL>
static bsm_status rep_launch(const Geom &g, int N, int rep, int d, const void *Uc, void *out,
                             hipStream_t st) {
    dim3 grid((g.Vh_pad + 127) / 128, 8, d);
    k_represent<LP, REAL><<<grid, 128, 0, st>>>(g, N, rep, d, (const double2 *)Uc, (char *)out);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status launch_represent(const Geom &g, int N, int rep, int d, int link_prec, const void *Uc,
                            void *out, hipStream_t st) {
    bool real = rep == BSM_REP_ADJ;
    switch (link_prec) {
    case BSM_F64: return real ? rep_launch<BSM_F64, true>(g, N, rep, d, Uc, out, st)
                              : rep_launch<BSM_F64, false>(g, N, rep, d, Uc, out, st);
    case BSM_F32: return real ? rep_launch<BSM_F32, true>(g, N, rep, d, Uc, out, st)
                              : rep_launch<BSM_F32, false>(g, N, rep, d, Uc, out, st);
    case BSM_F16S: return real ? rep_launch<BSM_F16S, true>(g, N, rep, d, Uc, out, st)
                               : rep_launch<BSM_F16S, false>(g, N, rep, d, Uc, out, st);
    }
    return fail(BSM_ERR_ARG, "bad link precision");
}

template <int LP, bool REAL>
static bsm_status unpack_g(const Geom &g, int d, const void *in, void *canon, hipStream_t st) {
    dim3 grid((g.Vh + 127) / 128, 8, 1);
    k_unpack_gauge<LP, REAL><<<grid, 128, 0, st>>>(g, d, (const char *)in, (double2 *)canon);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status launch_unpack_gauge(const Geom &g, int d, bool real, int link_prec, const void *in,
                               void *canon, hipStream_t st) {
    switch (link_prec) {
    case BSM_F64: return real ? unpack_g<BSM_F64, true>(g, d, in, canon, st)
                              : unpack_g<BSM_F64, false>(g, d, in, canon, st);
    case BSM_F32: return real ? unpack_g<BSM_F32, true>(g, d, in, canon, st)
                              : unpack_g<BSM_F32, false>(g, d, in, canon, st);
    case BSM_F16S: return real ? unpack_g<BSM_F16S, true>(g, d, in, canon, st)
                               : unpack_g<BSM_F16S, false>(g, d, in, canon, st);
    }
    return fail(BSM_ERR_ARG, "bad link precision");
}

// links stored in one precision -> another (elementwise over all planes)
template <int SRC, int DST, bool REAL>
__global__ __launch_bounds__(256) void k_convert_links(size_t nelem, const char *src, char *dst) {
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nelem; e += (size_t)gridDim.x * 256) {
        const int64_t i = (int64_t)e;
        // read element i of the flat plane array
        double re, im = 0.0;
        if constexpr (REAL) {
            if constexpr (SRC == BSM_F64) re = ((const double *)src)[i];
            else if constexpr (SRC == BSM_F32) re = ((const float *)src)[i];
            else re = __half2float(((const __half *)src)[i]);
        } else {
            if constexpr (SRC == BSM_F64) { double2 t = ((const double2 *)src)[i]; re = t.x; im = t.y; }
            else if constexpr (SRC == BSM_F32) { float2 t = ((const float2 *)src)[i]; re = t.x; im = t.y; }
            else { float2 t = __half22float2(((const __half2 *)src)[i]); re = t.x; im = t.y; }
        }
        store_link<DST, REAL>(dst, 0, 0, (uint32_t)i, re, im);
    }
}

template <int SRC, int DST>
static bsm_status conv2(size_t n, bool real, const void *src, void *dst, hipStream_t st) {
    size_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (real) k_convert_links<SRC, DST, true><<<(int)nb, 256, 0, st>>>(n, (const char *)src, (char *)dst);
    else k_convert_links<SRC, DST, false><<<(int)nb, 256, 0, st>>>(n, (const char *)src, (char *)dst);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status launch_convert_links(const Geom &g, int d, bool real, int src_prec, int dst_prec, const void *src,
                                void *dst, hipStream_t st) {
    const size_t n = (size_t)8 * d * d * g.Vh_pad;
    if (src_prec == BSM_F64 && dst_prec == BSM_F32) return conv2<BSM_F64, BSM_F32>(n, real, src, dst, st);
    if (src_prec == BSM_F64 && dst_prec == BSM_F16S) return conv2<BSM_F64, BSM_F16S>(n, real, src, dst, st);
    if (src_prec == BSM_F32 && dst_prec == BSM_F16S) return conv2<BSM_F32, BSM_F16S>(n, real, src, dst, st);
    return fail(BSM_ERR_UNSUPPORTED, "link conversion");
}

}  // namespace bsm
