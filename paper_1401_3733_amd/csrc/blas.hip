// Krylov vector kernels: linear combinations, dots and norms with FP64
// accumulation, on internal spinor fields of any storage precision.  One
// thread per site (grid-stride), components handled in chunks of 4 complex
// numbers; F16S outputs are requantised per site after the whole site is
// formed.
#include "blas.h"
#include "dispatch.h"
#include "spinor_io.h"

namespace bsm {

// one site per thread (grid-stride only beyond kMaxPartials workgroups):
// a grid-stride loop over few workgroups streams measurably slower
constexpr int kBlasMaxBlocks = kMaxPartials;

// chunk k = complex components 4k..4k+3 of one site, as 8 doubles
template <int P, int D>
struct Field {
    const char *blk;
    int64_t S;
    float sc;
    __device__ inline void open(const void *base, int b, uint32_t h, int64_t S_) {
        S = S_;
        blk = (const char *)base + (size_t)b * spinor_block_bytes(P, D, S_);
        if constexpr (P == BSM_F16S) sc = ((const float *)(blk + (size_t)D * S * 16))[h];
    }
    __device__ inline void load(uint32_t h, int k, double (&v)[8]) const {
        if constexpr (P == BSM_F64) {
            const double2 *b = (const double2 *)blk;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                double2 t = b[(4 * k + q) * S + h];
                v[2 * q] = t.x; v[2 * q + 1] = t.y;
            }
        } else if constexpr (P == BSM_F32) {
            const float4 *b = (const float4 *)blk;
#pragma unroll
            for (int q = 0; q < 2; q++) {
                float4 t = b[(2 * k + q) * S + h];
                v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
            }
        } else {
            const uint4 *b = (const uint4 *)blk;
            uint4 t = b[k * S + h];
            uint32_t w[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                float2 f = __half22float2(*reinterpret_cast<__half2 *>(&w[q]));
                v[2 * q] = (double)(f.x * sc);
                v[2 * q + 1] = (double)(f.y * sc);
            }
        }
    }
    // F64 / F32 only
    __device__ inline void store(uint32_t h, int k, const double (&v)[8]) const {
        if constexpr (P == BSM_F64) {
            double2 *b = (double2 *)blk;
#pragma unroll
            for (int q = 0; q < 4; q++) b[(4 * k + q) * S + h] = make_double2(v[2 * q], v[2 * q + 1]);
        } else if constexpr (P == BSM_F32) {
            float4 *b = (float4 *)blk;
#pragma unroll
            for (int q = 0; q < 2; q++)
                b[(2 * k + q) * S + h] = make_float4((float)v[4 * q], (float)v[4 * q + 1],
                                                     (float)v[4 * q + 2], (float)v[4 * q + 3]);
        }
    }
};

// whole-site store for F16S: buf holds 8 D reals as float
template <int D>
__device__ inline void store_f16s(const char *blk, int64_t S, uint32_t h, const float (&f)[8 * D]) {
    uint4 *b = (uint4 *)blk;
    float mx = 0.f;
#pragma unroll
    for (int c = 0; c < 8 * D; c++) mx = fmaxf(mx, fabsf(f[c]));
    float inv = mx > 0.f ? 1.0f / mx : 0.f;
#pragma unroll
    for (int k = 0; k < D; k++) {
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            __half2 hh = __floats2half2_rn(f[8 * k + 2 * q] * inv, f[8 * k + 2 * q + 1] * inv);
            w[q] = *reinterpret_cast<uint32_t *>(&hh);
        }
        b[k * S + h] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    ((float *)(b + D * S))[h] = mx;
}

// Sites of nblk parity blocks: i < n maps to block i / S, plane index
// i % S; plane indices at or above live (= Vh) are padding, which kernels
// skip: no operator writes it, and scratch reused across precisions can hold
// any bytes there.
struct SiteIter {
    uint32_t n;       // nblk * Vh_pad
    int64_t S;
    uint32_t live;
};

__device__ inline void site_of(uint32_t i, int64_t S, int &b, uint32_t &h) {
    b = (int)(i / (uint32_t)S);
    h = i - (uint32_t)b * (uint32_t)S;
}

// out = a A + b B
template <int D, int PO, int PA, int PB, bool HASB, bool NORM>
__global__ __launch_bounds__(256) void k_axpby(SiteIter it, void *out, const void *A, const void *B,
                                               double a, double bcoef, double *partials) {
    double nrm = 0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < it.n; i += gridDim.x * 256) {
        int b; uint32_t h;
        site_of(i, it.S, b, h);
        if (h >= it.live) continue;
        Field<PA, D> fa; fa.open(A, b, h, it.S);
        Field<PB, D> fb;
        if constexpr (HASB) fb.open(B, b, h, it.S);
        Field<PO, D> fo; fo.open(out, b, h, it.S);
        float buf[PO == BSM_F16S ? 8 * D : 1];
#pragma unroll
        for (int k = 0; k < D; k++) {
            double va[8], vb[8], vo[8];
            fa.load(h, k, va);
            if constexpr (HASB) fb.load(h, k, vb);
#pragma unroll
            for (int q = 0; q < 8; q++) {
                vo[q] = a * va[q];
                if constexpr (HASB) vo[q] = fma(bcoef, vb[q], vo[q]);
                if constexpr (NORM) nrm += vo[q] * vo[q];
            }
            if constexpr (PO == BSM_F16S) {
#pragma unroll
                for (int q = 0; q < 8; q++) buf[8 * k + q] = (float)vo[q];
            } else {
                fo.store(h, k, vo);
            }
        }
        if constexpr (PO == BSM_F16S) store_f16s<D>(fo.blk, it.S, h, buf);
    }
    if constexpr (NORM) {
        double s = block_sum_256(nrm);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

// partials of |A|^2 (DOT = false) or Re <A, B>
template <int D, int PA, int PB, bool DOT>
__global__ __launch_bounds__(256) void k_dot(SiteIter it, const void *A, const void *B, double *partials) {
    double acc = 0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < it.n; i += gridDim.x * 256) {
        int b; uint32_t h;
        site_of(i, it.S, b, h);
        if (h >= it.live) continue;
        Field<PA, D> fa; fa.open(A, b, h, it.S);
        Field<PB, D> fb;
        if constexpr (DOT) fb.open(B, b, h, it.S);
#pragma unroll
        for (int k = 0; k < D; k++) {
            double va[8], vb[8];
            fa.load(h, k, va);
            if constexpr (DOT) fb.load(h, k, vb);
#pragma unroll
            for (int q = 0; q < 8; q++) acc += DOT ? va[q] * vb[q] : va[q] * va[q];
        }
    }
    double s = block_sum_256(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// x += alpha p ; r -= alpha q ; partials |r|^2   (x, r in F64 or F32; x null:
// r only, the solution is formed later from the kept directions)
template <int D, int PX, int PP, int PR, int PQ>
__global__ __launch_bounds__(256) void k_cg_update(SiteIter it, void *x, const void *p, void *r,
                                                   const void *q, const double *scal, int ia,
                                                   double *partials) {
    const double alpha = scal[ia];
    const bool hx = x != nullptr;
    double nrm = 0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < it.n; i += gridDim.x * 256) {
        int b; uint32_t h;
        site_of(i, it.S, b, h);
        if (h >= it.live) continue;
        Field<PX, D> fx;
        Field<PP, D> fp;
        if (hx) {
            fx.open(x, b, h, it.S);
            fp.open(p, b, h, it.S);
        }
        Field<PR, D> fr; fr.open(r, b, h, it.S);
        Field<PQ, D> fq; fq.open(q, b, h, it.S);
#pragma unroll
        for (int k = 0; k < D; k++) {
            double vx[8], vp[8], vr[8], vq[8];
            if (hx) { fx.load(h, k, vx); fp.load(h, k, vp); }
            fr.load(h, k, vr); fq.load(h, k, vq);
#pragma unroll
            for (int c = 0; c < 8; c++) {
                if (hx) vx[c] = fma(alpha, vp[c], vx[c]);
                vr[c] = fma(-alpha, vq[c], vr[c]);
            }
            if (hx) fx.store(h, k, vx);
            if constexpr (PR == BSM_F32) {
#pragma unroll
                for (int c = 0; c < 8; c++) { double t = (double)(float)vr[c]; nrm += t * t; }
            } else {
#pragma unroll
                for (int c = 0; c < 8; c++) nrm += vr[c] * vr[c];
            }
            fr.store(h, k, vr);
        }
    }
    double s = block_sum_256(nrm);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// p = r + beta p_in  (p_in = p in place)
template <int D, int PP, int PR>
__global__ __launch_bounds__(256) void k_cg_xpay(SiteIter it, void *p, const void *r, const double *scal,
                                                 int ib, const void *p_in) {
    const double beta = scal[ib];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < it.n; i += gridDim.x * 256) {
        int b; uint32_t h;
        site_of(i, it.S, b, h);
        if (h >= it.live) continue;
        Field<PP, D> fp; fp.open(p, b, h, it.S);
        Field<PP, D> fi; fi.open(p_in, b, h, it.S);
        Field<PR, D> fr; fr.open(r, b, h, it.S);
        float buf[PP == BSM_F16S ? 8 * D : 1];
#pragma unroll
        for (int k = 0; k < D; k++) {
            double vp[8], vr[8];
            fi.load(h, k, vp); fr.load(h, k, vr);
#pragma unroll
            for (int c = 0; c < 8; c++) vp[c] = fma(beta, vp[c], vr[c]);
            if constexpr (PP == BSM_F16S) {
#pragma unroll
                for (int c = 0; c < 8; c++) buf[8 * k + c] = (float)vp[c];
            } else {
                fp.store(h, k, vp);
            }
        }
        if constexpr (PP == BSM_F16S) store_f16s<D>(fp.blk, it.S, h, buf);
    }
}

// ---------------------------------------------------------------- launchers
int blas_blocks(const Geom &g, int nblk) {
    int64_t n = (int64_t)nblk * g.Vh_pad;
    int64_t b = (n + 255) / 256;
    return (int)(b < kBlasMaxBlocks ? b : kBlasMaxBlocks);
}

static SiteIter iter_of(const Geom &g, int nblk) {
    SiteIter it;
    it.n = (uint32_t)((int64_t)nblk * g.Vh_pad);
    it.S = g.Vh_pad;
    it.live = (uint32_t)g.Vh;
    return it;
}

template <int D>
struct AxpbyByD {
    template <int PO, int PA, int PB>
    static bsm_status go(const Geom &g, int nblk, Vec out, double a, Vec A, double b, Vec B,
                         double *partials, hipStream_t st) {
        SiteIter it = iter_of(g, nblk);
        int nb = blas_blocks(g, nblk);
        bool hasb = B.ptr != nullptr, norm = partials != nullptr;
        if (hasb && norm) k_axpby<D, PO, PA, PB, true, true><<<nb, 256, 0, st>>>(it, out.ptr, A.ptr, B.ptr, a, b, partials);
        else if (hasb) k_axpby<D, PO, PA, PB, true, false><<<nb, 256, 0, st>>>(it, out.ptr, A.ptr, B.ptr, a, b, partials);
        else if (norm) k_axpby<D, PO, PA, PA, false, true><<<nb, 256, 0, st>>>(it, out.ptr, A.ptr, nullptr, a, b, partials);
        else k_axpby<D, PO, PA, PA, false, false><<<nb, 256, 0, st>>>(it, out.ptr, A.ptr, nullptr, a, b, partials);
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
    // supported combinations: all operands of one precision; conversions
    // (no B); and F64 = F64 + F32 (folding a low-precision solution in)
    static bsm_status run(const Geom &g, int nblk, Vec out, double a, Vec A, double b, Vec B,
                          double *partials, hipStream_t st) {
        const int po = out.prec, pa = A.prec, pb = B.ptr ? B.prec : A.prec;
#define SAME(P) if (po == P && pa == P && pb == P) return go<P, P, P>(g, nblk, out, a, A, b, B, partials, st);
        SAME(BSM_F64) SAME(BSM_F32) SAME(BSM_F16S)
#undef SAME
        if (!B.ptr) {
#define CONV(O, I) if (po == O && pa == I) return go<O, I, I>(g, nblk, out, a, A, b, B, partials, st);
            CONV(BSM_F64, BSM_F32) CONV(BSM_F64, BSM_F16S) CONV(BSM_F32, BSM_F64)
            CONV(BSM_F32, BSM_F16S) CONV(BSM_F16S, BSM_F64) CONV(BSM_F16S, BSM_F32)
#undef CONV
        }
        if (po == BSM_F64 && pa == BSM_F64 && pb == BSM_F32)
            return go<BSM_F64, BSM_F64, BSM_F32>(g, nblk, out, a, A, b, B, partials, st);
        return fail(BSM_ERR_UNSUPPORTED, "axpby precision combination");
    }
};

bsm_status blas_axpby(const Geom &g, int d, int nblk, Vec out, double a, Vec A, double b, Vec B,
                      double *partials, hipStream_t st) {
    return dispatch_d<AxpbyByD>(d, g, nblk, out, a, A, b, B, partials, st);
}

template <int D>
struct DotByD {
    static bsm_status run(const Geom &g, int nblk, Vec A, Vec B, double *partials, hipStream_t st) {
        SiteIter it = iter_of(g, nblk);
        int nb = blas_blocks(g, nblk);
        if (B.ptr && B.prec != A.prec) return fail(BSM_ERR_UNSUPPORTED, "dot of mixed precisions");
        switch (A.prec) {
        case BSM_F64:
            if (B.ptr) k_dot<D, BSM_F64, BSM_F64, true><<<nb, 256, 0, st>>>(it, A.ptr, B.ptr, partials);
            else k_dot<D, BSM_F64, BSM_F64, false><<<nb, 256, 0, st>>>(it, A.ptr, nullptr, partials);
            break;
        case BSM_F32:
            if (B.ptr) k_dot<D, BSM_F32, BSM_F32, true><<<nb, 256, 0, st>>>(it, A.ptr, B.ptr, partials);
            else k_dot<D, BSM_F32, BSM_F32, false><<<nb, 256, 0, st>>>(it, A.ptr, nullptr, partials);
            break;
        default:
            if (B.ptr) k_dot<D, BSM_F16S, BSM_F16S, true><<<nb, 256, 0, st>>>(it, A.ptr, B.ptr, partials);
            else k_dot<D, BSM_F16S, BSM_F16S, false><<<nb, 256, 0, st>>>(it, A.ptr, nullptr, partials);
        }
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
};

bsm_status blas_dot(const Geom &g, int d, int nblk, Vec A, Vec B, double *partials, hipStream_t st) {
    return dispatch_d<DotByD>(d, g, nblk, A, B, partials, st);
}

// CG kernels: the precision combinations the solvers use
//   F64 : x, p, r, q all F64
//   F32 : x, p, r, q all F32
//   F16S: x, r F32; p, q F16S
template <int D>
struct CgByD {
    static bsm_status run(const Geom &g, int nblk, Vec x, Vec p, Vec r, Vec q, const double *scal,
                          int ia, double *partials, hipStream_t st, int mode, int ib) {
        SiteIter it = iter_of(g, nblk);
        int nb = blas_blocks(g, nblk);
        if (mode == 0) {
            if (x.prec == BSM_F64 && p.prec == BSM_F64 && r.prec == BSM_F64 && q.prec == BSM_F64)
                k_cg_update<D, BSM_F64, BSM_F64, BSM_F64, BSM_F64><<<nb, 256, 0, st>>>(it, x.ptr, p.ptr, r.ptr, q.ptr, scal, ia, partials);
            else if (x.prec == BSM_F32 && p.prec == BSM_F32 && r.prec == BSM_F32 && q.prec == BSM_F32)
                k_cg_update<D, BSM_F32, BSM_F32, BSM_F32, BSM_F32><<<nb, 256, 0, st>>>(it, x.ptr, p.ptr, r.ptr, q.ptr, scal, ia, partials);
            else if (x.prec == BSM_F32 && p.prec == BSM_F16S && r.prec == BSM_F32 && q.prec == BSM_F16S)
                k_cg_update<D, BSM_F32, BSM_F16S, BSM_F32, BSM_F16S><<<nb, 256, 0, st>>>(it, x.ptr, p.ptr, r.ptr, q.ptr, scal, ia, partials);
            else
                return fail(BSM_ERR_UNSUPPORTED, "cg_update precision combination");
        } else {
            // p = r + beta p
            if (p.prec == BSM_F64 && r.prec == BSM_F64)
                k_cg_xpay<D, BSM_F64, BSM_F64><<<nb, 256, 0, st>>>(it, p.ptr, r.ptr, scal, ib, x.ptr ? x.ptr : p.ptr);
            else if (p.prec == BSM_F32 && r.prec == BSM_F32)
                k_cg_xpay<D, BSM_F32, BSM_F32><<<nb, 256, 0, st>>>(it, p.ptr, r.ptr, scal, ib, x.ptr ? x.ptr : p.ptr);
            else if (p.prec == BSM_F16S && r.prec == BSM_F32)
                k_cg_xpay<D, BSM_F16S, BSM_F32><<<nb, 256, 0, st>>>(it, p.ptr, r.ptr, scal, ib, x.ptr ? x.ptr : p.ptr);
            else
                return fail(BSM_ERR_UNSUPPORTED, "cg_xpay precision combination");
        }
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
};

bsm_status blas_cg_update(const Geom &g, int d, int nblk, Vec x, Vec p, Vec r, Vec q,
                          const double *scal, int ia, double *partials, hipStream_t st) {
    return dispatch_d<CgByD>(d, g, nblk, x, p, r, q, scal, ia, partials, st, 0, 0);
}

bsm_status blas_cg_xpay(const Geom &g, int d, int nblk, Vec p, Vec r, const double *scal, int ib,
                        hipStream_t st) {
    Vec none{nullptr, BSM_F64};
    return dispatch_d<CgByD>(d, g, nblk, none, p, r, none, scal, 0, (double *)nullptr, st, 1, ib);
}

bsm_status blas_cg_xpay_to(const Geom &g, int d, int nblk, Vec p_out, Vec p_in, Vec r, const double *scal, int ib,
                           hipStream_t st) {
    if (p_in.prec != p_out.prec) return fail(BSM_ERR_ARG, "cg_xpay: p_in and p_out differ in precision");
    Vec none{nullptr, BSM_F64};
    // the kernel takes p_in through the (otherwise unused) x slot
    return dispatch_d<CgByD>(d, g, nblk, p_in, p_out, r, none, scal, 0, (double *)nullptr, st, 1, ib);
}

// x += sum_k alphas[k] p_k over kn kept directions, p_k the ring slot
// (slot0 + k) % ring, slots pstride bytes apart
template <int D, int PX, int PP>
__global__ __launch_bounds__(256) void k_x_flush(SiteIter it, void *x, const char *pbase, size_t pstride, int ring,
                                                 int slot0, int kn, const double *alphas) {
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < it.n; i += gridDim.x * 256) {
        int b; uint32_t h;
        site_of(i, it.S, b, h);
        if (h >= it.live) continue;
        Field<PX, D> fx; fx.open(x, b, h, it.S);
        for (int k = 0; k < D; k++) {
            double vx[8];
            fx.load(h, k, vx);
            for (int j = 0; j < kn; j++) {
                Field<PP, D> fp; fp.open(pbase + (size_t)((slot0 + j) % ring) * pstride, b, h, it.S);
                double vp[8];
                fp.load(h, k, vp);
                const double a = alphas[j];
#pragma unroll
                for (int c = 0; c < 8; c++) vx[c] = fma(a, vp[c], vx[c]);
            }
            fx.store(h, k, vx);
        }
    }
}

template <int D>
struct XFlushByD {
    static bsm_status run(const Geom &g, int nblk, Vec x, const char *pbase, int pprec, size_t pstride, int ring,
                          int slot0, int kn, const double *alphas, hipStream_t st) {
        SiteIter it = iter_of(g, nblk);
        const int nb = blas_blocks(g, nblk);
        if (x.prec == BSM_F32 && pprec == BSM_F32)
            k_x_flush<D, BSM_F32, BSM_F32><<<nb, 256, 0, st>>>(it, x.ptr, pbase, pstride, ring, slot0, kn, alphas);
        else if (x.prec == BSM_F32 && pprec == BSM_F16S)
            k_x_flush<D, BSM_F32, BSM_F16S><<<nb, 256, 0, st>>>(it, x.ptr, pbase, pstride, ring, slot0, kn, alphas);
        else
            return fail(BSM_ERR_UNSUPPORTED, "x_flush precision combination");
        BSM_HIP(hipGetLastError());
        return BSM_OK;
    }
};

bsm_status blas_x_flush(const Geom &g, int d, int nblk, Vec x, const char *pbase, int pprec, size_t pstride,
                        int ring, int slot0, int kn, const double *alphas, hipStream_t st) {
    if (kn <= 0) return BSM_OK;
    return dispatch_d<XFlushByD>(d, g, nblk, x, pbase, pprec, pstride, ring, slot0, kn, alphas, st);
}

// ------------------------------------------------------------- reductions
__device__ inline double fixed_sum(const double *partials, int n) {
    double acc = 0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partials[i];
    return block_sum_256(acc);
}

__global__ __launch_bounds__(256) void k_reduce(const double *partials, int n, double *dst) {
    double s = fixed_sum(partials, n);
    if (threadIdx.x == 0) dst[0] = s;
}

__global__ __launch_bounds__(256) void k_cg_scalars(const double *partials, int n, double *scal, int op,
                                                    int it) {
    double s = fixed_sum(partials, n);
    if (threadIdx.x != 0) return;
    if (op == 0) {
        scal[S_PAP] = s;
        double rr = scal[S_RR];
        double al = rr / s;
        scal[S_ALPHA] = (s > 0 && isfinite(al)) ? al : 0.0;
        if (it >= 0 && it < kAlphaHist) scal[S_AHIST + it] = scal[S_ALPHA];
    } else if (op == 1) {
        double rr = scal[S_RR];
        double be = s / rr;
        scal[S_BETA] = (rr > 0 && isfinite(be)) ? be : 0.0;
        scal[S_RR] = s;
        scal[S_HIST + it] = s;
    } else {
        scal[S_RR] = s;
        scal[S_HIST + it] = s;
    }
}

bsm_status reduce_into(const double *partials, int n, double *dst, hipStream_t st) {
    k_reduce<<<1, 256, 0, st>>>(partials, n, dst);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status cg_scalars(const double *partials, int n, double *scal, int op, int it, hipStream_t st) {
    k_cg_scalars<<<1, 256, 0, st>>>(partials, n, scal, op, it);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
