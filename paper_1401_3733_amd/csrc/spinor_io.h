// Device-side access to internal spinor and link storage.
#pragma once
#include "bsm_internal.h"

namespace bsm {

// Load the 4d complex components of site h from one parity block.
template <int P, int D, class T>
__device__ inline void load_spinor(const void *blk, int64_t stride, uint32_t h, cx<T> (&s)[4 * D]) {
    if constexpr (P == BSM_F64) {
        const double2 *b = (const double2 *)blk;
#pragma unroll
        for (int c = 0; c < 4 * D; c++) {
            double2 v = b[c * stride + h];
            s[c] = mk<T>((T)v.x, (T)v.y);
        }
    } else if constexpr (P == BSM_F32) {
        const float4 *b = (const float4 *)blk;
#pragma unroll
        for (int k = 0; k < 2 * D; k++) {
            float4 v = b[k * stride + h];
            s[2 * k] = mk<T>(v.x, v.y);
            s[2 * k + 1] = mk<T>(v.z, v.w);
        }
    } else {
        const uint4 *b = (const uint4 *)blk;
        const float sc = ((const float *)(b + D * stride))[h];
#pragma unroll
        for (int k = 0; k < D; k++) {
            uint4 v = b[k * stride + h];
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                __half2 hh = *reinterpret_cast<__half2 *>(&w[q]);
                float2 f = __half22float2(hh);
                s[4 * k + q] = mk<T>(f.x * sc, f.y * sc);
            }
        }
    }
}

// Store the 4d complex components of site h.  F16S: per-site scale
// s = max |component| (float32), codes = rne_f16(float32(v * float32(1/s))).
template <int P, int D, class T>
__device__ inline void store_spinor(void *blk, int64_t stride, uint32_t h, const cx<T> (&s)[4 * D]) {
    if constexpr (P == BSM_F64) {
        double2 *b = (double2 *)blk;
#pragma unroll
        for (int c = 0; c < 4 * D; c++) b[c * stride + h] = make_double2((double)s[c].re, (double)s[c].im);
    } else if constexpr (P == BSM_F32) {
        float4 *b = (float4 *)blk;
#pragma unroll
        for (int k = 0; k < 2 * D; k++)
            b[k * stride + h] = make_float4((float)s[2 * k].re, (float)s[2 * k].im,
                                            (float)s[2 * k + 1].re, (float)s[2 * k + 1].im);
    } else {
        uint4 *b = (uint4 *)blk;
        float f[8 * D];
#pragma unroll
        for (int c = 0; c < 4 * D; c++) {
            f[2 * c] = (float)s[c].re;
            f[2 * c + 1] = (float)s[c].im;
        }
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
            b[k * stride + h] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        ((float *)(b + D * stride))[h] = mx;
    }
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

// store_spinor with streaming (non-temporal) stores for F32 and F64
template <int P, int D, class T>
__device__ inline void store_spinor_nt(void *blk, int64_t stride, uint32_t h, const cx<T> (&s)[4 * D]) {
    if constexpr (P == BSM_F32) {
        f32x4v *b = (f32x4v *)blk;
#pragma unroll
        for (int k = 0; k < 2 * D; k++) {
            f32x4v v = {(float)s[2 * k].re, (float)s[2 * k].im, (float)s[2 * k + 1].re, (float)s[2 * k + 1].im};
            __builtin_nontemporal_store(v, b + k * stride + h);
        }
    } else if constexpr (P == BSM_F64) {
        typedef double f64x2v __attribute__((ext_vector_type(2)));
        f64x2v *b = (f64x2v *)blk;
#pragma unroll
        for (int c = 0; c < 4 * D; c++) {
            f64x2v v = {(double)s[c].re, (double)s[c].im};
            __builtin_nontemporal_store(v, b + c * stride + h);
        }
    } else {
        store_spinor<P, D, T>(blk, stride, h, s);
    }
}
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Link element (i, j) of a link block (complex or real) as cx<T>; NT: a
// non-temporal (streaming) load.
template <int LP, bool REAL, class T, bool NT = false>
__device__ inline cx<T> load_link(const void *blk, int64_t stride, int e, uint32_t h) {
    if constexpr (NT && !REAL && LP == BSM_F32) {
        f32x2 v = __builtin_nontemporal_load((const f32x2 *)blk + e * stride + h);
        return mk<T>((T)v.x, (T)v.y);
    } else if constexpr (NT && !REAL && LP == BSM_F64) {
        f64x2 v = __builtin_nontemporal_load((const f64x2 *)blk + e * stride + h);
        return mk<T>((T)v.x, (T)v.y);
    } else if constexpr (NT && REAL && LP == BSM_F32) {
        float v = __builtin_nontemporal_load((const float *)blk + e * stride + h);
        return mk<T>((T)v, (T)0);
    } else if constexpr (NT && REAL && LP == BSM_F64) {
        double v = __builtin_nontemporal_load((const double *)blk + e * stride + h);
        return mk<T>((T)v, (T)0);
    } else if constexpr (NT && !REAL && LP == BSM_F16S) {
        uint32_t v = __builtin_nontemporal_load((const uint32_t *)blk + e * stride + h);
        float2 f = __half22float2(*reinterpret_cast<__half2 *>(&v));
        return mk<T>((T)f.x, (T)f.y);
    } else if constexpr (REAL) {
        if constexpr (LP == BSM_F64) return mk<T>((T)((const double *)blk)[e * stride + h], (T)0);
        else if constexpr (LP == BSM_F32) return mk<T>((T)((const float *)blk)[e * stride + h], (T)0);
        else return mk<T>((T)__half2float(((const __half *)blk)[e * stride + h]), (T)0);
    } else {
        if constexpr (LP == BSM_F64) {
            double2 v = ((const double2 *)blk)[e * stride + h];
            return mk<T>((T)v.x, (T)v.y);
        } else if constexpr (LP == BSM_F32) {
            float2 v = ((const float2 *)blk)[e * stride + h];
            return mk<T>((T)v.x, (T)v.y);
        } else {
            float2 v = __half22float2(((const __half2 *)blk)[e * stride + h]);
            return mk<T>((T)v.x, (T)v.y);
        }
    }
}

// neighbour of c one step along +mu (back = false) or -mu: half index and the
// boundary factor of the hop
template <int MU>
__device__ inline uint32_t neighbour(const Geom &g, const Coords &c, bool back, float &w) {
    const int Lmu = g.L[MU];
    const int xm = MU == 0 ? c.t : MU == 1 ? c.x : MU == 2 ? c.y : c.z;
    int xn = back ? xm - 1 : xm + 1;
    w = 1.f;
    const bool ap = (g.apbc >> MU) & 1;
    if (xn == Lmu) { xn = 0; if (ap) w = -1.f; }
    if (xn < 0) { xn = Lmu - 1; if (ap) w = -1.f; }
    if constexpr (MU == 1) {
        return (uint32_t)c.row * g.LXh + (xn >> 1);
    } else {
        int t = c.t, z = c.z, y = c.y;
        if (MU == 0) t = xn;
        if (MU == 2) y = xn;
        if (MU == 3) z = xn;
        uint32_t row = ((uint32_t)t * g.L[3] + z) * g.L[2] + y;
        return row * g.LXh + c.xh;
    }
}

// Non-temporal link loads per spinor precision (bit SP of BSM_LINK_NT).
#ifndef BSM_LINK_NT
#define BSM_LINK_NT 0x7
#endif

// Sum over a 256-thread workgroup in a fixed order (valid on thread 0):
// xor-shuffles inside each 64-wide wavefront, then the 4 wavefronts in order.
__device__ inline double block_sum_256(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __shared__ double ws[4];
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) ws[w] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0) s = (ws[0] + ws[1]) + (ws[2] + ws[3]);
    return s;
}

}  // namespace bsm
