// Internal definitions shared by the libbsm HIP sources (not part of the ABI).
//
// Internal field layout: even-odd checkerboarded structure-of-arrays.
//   Sites of one parity are numbered by their half index h = lex / 2 with
//   lex = ((t*LZ + z)*LY + y)*LX + x (LX even, so the two sites x = 2k, 2k+1
//   of a row share h and have opposite parity).  Each parity block stores
//   component planes of Vh_pad sites (V/2 rounded up to a multiple of 64,
//   plus 256 when that is a multiple of 1024, so that planes do not start a
//   large power of two apart), so lane i of a wavefront touches site i of a
//   plane and every load is coalesced.  Sites h >= Vh of a plane are padding.
//   Spinor (4 d complex per site, component c = spin*d + colour):
//     F64  : 4d planes of double2 (one complex)           16 B per site-plane
//     F32  : 2d planes of float4  (complex 2k, 2k+1)      16 B
//     F16S : d  planes of uint4   (complex 4k..4k+3 as half2), then one float
//            plane with the per-site scale
//   Links, per (parity q, mu) block, U_mu(x) for x of parity q at index h:
//     complex: d*d planes of double2 / float2 / half2 (element (i,j) at plane i*d+j)
//     real   : d*d planes of double / float / half
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <string>

#include "../../include/bsm.h"

namespace bsm {

constexpr int kXcds = 8;        // gfx950: 8 XCDs, each with its own L2

// -------------------------------------------------------------- fast division
// Exact unsigned division by a runtime constant for n < 2^31
// (Granlund & Montgomery 1994): q = (umulhi(n, m) + n) >> l.
struct FastDiv {
    uint32_t d, m, l;
    FastDiv() : d(1), m(1), l(0) {}
    explicit FastDiv(uint32_t d_) : d(d_) {
        l = 0;
        while ((1u << l) < d) l++;
        uint64_t two32 = 1ull << 32;
        m = (uint32_t)((two32 * ((1ull << l) - d)) / d + 1);
    }
    __host__ __device__ inline uint32_t div(uint32_t n) const {
#ifdef __HIP_DEVICE_COMPILE__
        uint32_t hi = __umulhi(n, m);
#else
        uint32_t hi = (uint32_t)(((uint64_t)n * m) >> 32);
#endif
        return (hi + n) >> l;
    }
};

// -------------------------------------------------------------- geometry
struct Geom {
    int32_t L[4];          // T, LX, LY, LZ
    int32_t LXh;           // LX / 2
    int32_t Vh;            // sites per parity
    int32_t Vh_pad;        // plane stride (sites)
    int32_t apbc;          // bit mu set: antiperiodic in mu
    FastDiv div_xh, div_y, div_z;
};

struct Coords { int32_t t, x, y, z, xh, row; };

// half index h of parity p -> coordinates; row = (t*LZ + z)*LY + y
__device__ inline Coords decode(const Geom &g, uint32_t h, int p) {
    Coords c;
    uint32_t row = g.div_xh.div(h);
    c.xh = h - row * g.LXh;
    uint32_t r2 = g.div_y.div(row);
    c.y = row - r2 * g.L[2];
    uint32_t t = g.div_z.div(r2);
    c.z = r2 - t * g.L[3];
    c.t = t;
    c.row = row;
    c.x = 2 * c.xh + ((c.t + c.z + c.y + p) & 1);
    return c;
}

// -------------------------------------------------------------- storage traits
// number of 16-byte planes of a spinor site
__host__ __device__ constexpr int spinor_planes(int prec, int d) {
    return prec == BSM_F64 ? 4 * d : prec == BSM_F32 ? 2 * d : d;
}
// bytes of one parity block of a spinor field
__host__ __device__ inline size_t spinor_block_bytes(int prec, int d, int64_t Vh_pad) {
    size_t b = (size_t)spinor_planes(prec, d) * 16 * Vh_pad;
    if (prec == BSM_F16S) b += (size_t)4 * Vh_pad;
    return b;
}
__host__ __device__ inline size_t link_elem_bytes(int prec, bool real) {
    size_t r = prec == BSM_F64 ? 8 : prec == BSM_F32 ? 4 : 2;
    return real ? r : 2 * r;
}
__host__ __device__ inline size_t link_block_bytes(int prec, bool real, int d, int64_t Vh_pad) {
    return link_elem_bytes(prec, real) * d * d * Vh_pad;
}

// compute type of the operator for a spinor precision
template <int P> struct Compute { using T = float; };
template <> struct Compute<BSM_F64> { using T = double; };

// -------------------------------------------------------------- complex
template <class T> struct cx { T re, im; };
template <class T> __device__ __host__ inline cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T> __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// a * b
template <class T> __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a * b
template <class T> __device__ inline cx<T> cfma(cx<T> a, cx<T> b, cx<T> acc) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}
// acc + conj(a) * b
template <class T> __device__ inline cx<T> cfma_conj(cx<T> a, cx<T> b, cx<T> acc) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
    return acc;
}
// i * a
template <class T> __device__ inline cx<T> times_i(cx<T> a) { return {-a.im, a.re}; }

// -------------------------------------------------------------- errors
void set_error(const std::string &msg);
bsm_status fail(bsm_status st, const std::string &msg);
bsm_status hip_check(hipError_t e, const char *what);

#define BSM_HIP(call)                                                     \
    do {                                                                  \
        hipError_t _e = (call);                                           \
        if (_e != hipSuccess) return ::bsm::hip_check(_e, #call);         \
    } while (0)

// XCD-aware block order: the hardware hands consecutive workgroups to the
// 8 XCDs in turn; remap so each XCD walks one contiguous range of sites and
// neighbour re-reads stay inside that XCD's L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nblk) {
    uint32_t full = nblk / kXcds * kXcds;
    if (b >= full) return b;
    uint32_t per = full / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Workgroup order across the XCDs with a run length: c = 0 is xcd_remap (each
// XCD one contiguous share of the grid); c > 0 deals each XCD runs of c
// consecutive logical workgroups, so all XCDs work on nearby parts of the grid
// at the same time and share the memory-side cache (c = 1: the hardware's own
// round-robin order).  A bijection on [0, nblk).
__device__ inline uint32_t xcd_chunk_remap(uint32_t b, uint32_t nblk, uint32_t c) {
    if (c == 0) return xcd_remap(b, nblk);
    const uint32_t span = c * kXcds, full = nblk / span * span;
    if (b >= full) return b;
    const uint32_t x = b % kXcds, k = b / kXcds;
    return (k / c) * span + x * c + k % c;
}

// ------------------------------------------------------------ link storage
// Internal link code of a descriptor: the link precision (bits 0-1), and for
// fundamental storage of a higher representation (BSM_LINKS_FUNDAMENTAL) the
// flag kLinkOtf with (rep, N) in bits 8-11 and 12-15; the operator then forms
// R(U) from U inside the hop.  Fundamental fermions with the flag are the
// plain stored case.
constexpr int kLinkOtf = BSM_LINKS_FUNDAMENTAL;
__host__ __device__ inline int link_base(int lc) { return lc & 3; }
__host__ __device__ inline bool link_is_otf(int lc) { return (lc & kLinkOtf) != 0; }
// (rep, N) of an on-the-fly code as rep * 16 + N, 0 for stored links
__host__ __device__ inline int link_rn(int lc) { return link_is_otf(lc) ? ((lc >> 8) & 15) * 16 + ((lc >> 12) & 15) : 0; }
inline int link_code(const bsm_field_desc *d) {
    const int base = d->link_prec & 3;
    if (!(d->link_prec & kLinkOtf) || d->rep == BSM_REP_FUND) return base;
    return base | kLinkOtf | (d->rep << 8) | (d->N << 12);
}
// dimension of the stored link matrices (N for on-the-fly codes)
inline int link_dim(const bsm_field_desc *d) { return link_is_otf(link_code(d)) ? d->N : d->d_R; }
// real stored links (adjoint representation stored as R(U))
inline bool link_real(const bsm_field_desc *d) { return d->rep == BSM_REP_ADJ && !link_is_otf(link_code(d)); }

// hop traversal plan, chosen per (d_R, link type, precisions) by bsm_autotune
struct HopPlan {
    int order = 0, tchunk = 1;
    float us = 0.f;   // measured time per hop when tuned (0: default plan)
};

// multi-RHS hop plan per d_R (sites per wavefront, wavefronts per workgroup)
struct BlockPlan {
    int spw = 1, wpb = 4;
    int tiled = 0;    // 1: tiled site order (block_tile_for)
    int xchunk = 0;   // workgroup run length per XCD (xcd_chunk_remap)
    float us = 0.f;   // measured time per hop when tuned (0: default plan)
};

}  // namespace bsm

// context (defined in api.cpp)
struct bsm_ctx_s {
    bsm::Geom g;
    bsm_lattice lat;
    int device;
    // reduction scratch
    double *partials;       // device, n_partials doubles
    int64_t n_partials;     // reduction_slots(Vh): room for every fused-norm launch
    double *scal;           // device scalars for solvers (kScalars)
    double *host_scal;      // pinned host mirror
    // scratch buffers (lazily grown, zero-filled when allocated):
    //   0: solvers, 1: FGCR (its fall back CG uses 0), 2: network layers
    void *work[3];
    size_t work_bytes[3];
    // pinned host scratch (lazily grown) and the batched solver's private
    // stream (created on first use, default priority), kept for the
    // context's lifetime so a solve allocates nothing after warm-up
    void *pinned;
    size_t pinned_bytes;
    hipStream_t solver_stream;
    bsm::HopPlan plans[16][2][3][6];   // [d_R][adjoint][spinor prec][link prec (+3: on the fly)]
    bsm::BlockPlan block_plans[16][2];  // [d_R][FP16 block fields]
};

namespace bsm {
constexpr int kMaxPartials = 1 << 16;
constexpr int kScalars = 4096;
// FP64 reduction slots of a context for Vh sites per parity: the vector
// kernels cap their grids at kMaxPartials workgroups, a fused-norm hop writes
// one partial per workgroup of both parities, and its smallest workgroups
// (the FP64 colour split with four threads per site) cover 64 sites
inline int64_t reduction_slots(int64_t Vh) {
    const int64_t hop = 2 * ((Vh + 63) / 64);
    return hop > kMaxPartials ? hop : kMaxPartials;
}
// scratch that persists across calls, zero-filled when (re)allocated; slot 0
// is the solvers' buffer, slot 1 FGCR's, slot 2 the network layers
bsm_status ctx_work(bsm_ctx ctx, size_t bytes, void **out);
bsm_status ctx_work_slot(bsm_ctx ctx, int slot, size_t bytes, void **out);
// pinned host scratch of at least bytes (contents undefined after growth)
bsm_status ctx_pinned(bsm_ctx ctx, size_t bytes, void **out);
// the context's non-blocking solver stream
bsm_status ctx_solver_stream(bsm_ctx ctx, hipStream_t *out);
// device address of the allocation-free network's static scratch on this
// device (the device must be current); once per device, at context creation
bsm_status noalloc_scratch_init(int device);
}
