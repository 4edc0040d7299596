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
#include "otf.h"
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

// Links small enough to be loaded whole before the multiply (all loads of a
// hop in flight together); larger ones stream row by row.
template <int D> constexpr bool kLinkWhole = D * D <= 16;

template <int D, bool REAL, int LP, bool NT, class T>
struct LinkRegs {
    cx<T> u[kLinkWhole<D> ? D * D : 1];
    __device__ inline void load(const void *blk, int64_t stride, uint32_t hl) {
        if constexpr (kLinkWhole<D>) {
#pragma unroll
            for (int e = 0; e < D * D; e++) u[e] = load_link<LP, REAL, T, NT>(blk, stride, e, hl);
        }
    }
};

// g = U h (forward) or U^dag h (backward) for both spin components; the link
// comes from L (whole-matrix case) or is streamed from blk
template <int D, bool REAL, int LP, bool BACK, bool NT, class T>
__device__ inline void link_mul(const LinkRegs<D, REAL, LP, NT, T> &L, const void *blk, int64_t stride,
                                uint32_t hl, const cx<T> (&h0)[D], const cx<T> (&h1)[D], cx<T> (&g0)[D],
                                cx<T> (&g1)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) { g0[i] = mk<T>(0, 0); g1[i] = mk<T>(0, 0); }
#pragma unroll
    for (int i = 0; i < D; i++) {
        cx<T> row[D];
#pragma unroll
        for (int j = 0; j < D; j++) {
            if constexpr (kLinkWhole<D>) row[j] = L.u[i * D + j];
            else row[j] = load_link<LP, REAL, T, NT>(blk, stride, i * D + j, hl);
        }
#pragma unroll
        for (int j = 0; j < D; j++) {
            const cx<T> u = row[j];
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
}

// link block and site of a hop: forward uses U_mu(x) (this site, parity p),
// backward U_mu(x - mu) stored at the neighbour (parity 1-p)
template <int MU, bool BACK>
__device__ inline const char *link_block(const char *U, size_t lblk, int p) {
    return U + (size_t)((BACK ? 1 - p : p) * 4 + MU) * lblk;
}

// one hop with the neighbour's half spinor already projected: link multiply
// (forward link of this site, or the daggered link of the neighbour) and
// reconstruction into acc
template <int MU, int D, bool REAL, int LP, bool BACK, class T, bool NT = true>
__device__ inline void hop_half(const Geom &g, const LinkRegs<D, REAL, LP, NT, T> &L, const char *blk,
                                uint32_t hl, T sg, T w, const cx<T> (&h0)[D], const cx<T> (&h1)[D],
                                cx<T> (&acc)[4 * D]) {
    cx<T> g0[D], g1[D];
    link_mul<D, REAL, LP, BACK, NT, T>(L, blk, g.Vh_pad, hl, h0, h1, g0, g1);
    reconstruct<MU, D, T>(acc, sg, w, g0, g1);
}

// both hops along mu, loading the neighbour spinors
template <int MU, int D, bool REAL, int SP, int LP, class T>
__device__ inline void hop_dir(const Geom &g, const Coords &c, int p, uint32_t h, const char *U,
                               size_t lblk, const char *in, T eta, cx<T> (&acc)[4 * D]) {
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        const bool back = dir == 1;
        float wf;
        const uint32_t hn = neighbour<MU>(g, c, back, wf);
        constexpr bool NT = (BSM_LINK_NT >> SP) & 1;
        // issue the spinor and link loads of this hop before any arithmetic
        cx<T> s[4 * D];
        load_spinor<SP, D, T>(in, g.Vh_pad, hn, s);
        LinkRegs<D, REAL, LP, NT, T> L;
        const char *blk = back ? link_block<MU, true>(U, lblk, p) : link_block<MU, false>(U, lblk, p);
        const uint32_t hl = back ? hn : h;
        L.load(blk, g.Vh_pad, hl);
        const T sg = back ? -eta : eta;
        cx<T> h0[D], h1[D];
        project<MU, D, T>(s, sg, h0, h1);
        if (!back) hop_half<MU, D, REAL, LP, false, T, NT>(g, L, blk, hl, sg, (T)wf, h0, h1, acc);
        else hop_half<MU, D, REAL, LP, true, T, NT>(g, L, blk, hl, sg, (T)wf, h0, h1, acc);
    }
}

// Hops with on-the-fly links: the accumulators are pinned after each hop (an
// empty statement that holds them in registers there) and the scheduler may
// not move instructions across, so later directions' neighbour loads are not
// hoisted over this one's arithmetic.  Without it the F16 spinor forms issued
// all eight directions' loads first and held 256 registers (one wavefront per
// SIMD).  Measured per form on 32^3 x 64: pinned is faster for F16 spinors
// (2S SU(3) 432 -> 172 us), FP32 (2S SU(3) 295 -> 257 us, 2S SU(2)
// 147 -> 112 us; the SU(2) adjoint loses 3 %) and FP64 at d_R >= 6 (2S SU(3)
// 520 -> 486 us), and slower for FP64 at d_R = 3 (2S SU(2) 209 -> 262 us).
template <int SP, int RN>
constexpr bool kOtfPin = SP == BSM_F16S ||
                         (SP == BSM_F32 && !(otf_rep(RN) == BSM_REP_ADJ && otf_n(RN) == 2)) ||
                         (SP == BSM_F64 && otf_dim(RN) >= 6);

template <int SP, int RN, class T>
__device__ inline void otf_pin(cx<T> (&acc)[4 * otf_dim(RN)]) {
    if constexpr (kOtfPin<SP, RN>) {
#pragma unroll
        for (int k = 0; k < 4 * otf_dim(RN); k++) {
            asm volatile("" : "+v"(acc[k].re));
            asm volatile("" : "+v"(acc[k].im));
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// both hops along mu with fundamental links: R(U) (or R(U)^dag) applied to
// the projected half spinor on the fly
template <int MU, int RN, int SP, int LP, class T>
__device__ inline void hop_dir_otf(const Geom &g, const Coords &c, int p, uint32_t h, const char *U,
                                   size_t lblk, const char *in, T eta, cx<T> (&acc)[4 * otf_dim(RN)]) {
    constexpr int D = otf_dim(RN), N = otf_n(RN);
    constexpr bool NT = (BSM_LINK_NT >> SP) & 1;
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        const bool back = dir == 1;
        float wf;
        const uint32_t hn = neighbour<MU>(g, c, back, wf);
        cx<T> s[4 * D];
        load_spinor<SP, D, T>(in, g.Vh_pad, hn, s);
        const char *blk = back ? link_block<MU, true>(U, lblk, p) : link_block<MU, false>(U, lblk, p);
        const uint32_t hl = back ? hn : h;
        cx<T> u[N * N];
#pragma unroll
        for (int e = 0; e < N * N; e++) u[e] = load_link<LP, false, T, NT>(blk, g.Vh_pad, e, hl);
        const T sg = back ? -eta : eta;
        cx<T> h0[D], h1[D], g0[D], g1[D];
        project<MU, D, T>(s, sg, h0, h1);
        if (!back) {
            rep_apply<RN, false, T>(u, h0, g0);
            rep_apply<RN, false, T>(u, h1, g1);
        } else {
            rep_apply<RN, true, T>(u, h0, g0);
            rep_apply<RN, true, T>(u, h1, g1);
        }
        reconstruct<MU, D, T>(acc, sg, (T)wf, g0, g1);
        otf_pin<SP, RN>(acc);
    }
}

// out = a x + b acc, stored; returns |out|^2 contribution when asked
template <int D, int SP, class T>
__device__ inline double hop_epilogue(const Geom &g, const HopArgs &a, int p, uint32_t h, cx<T> (&acc)[4 * D]) {
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
    // streaming stores: the output is not read again by this launch, and
    // keeping it out of L2 leaves room for the input's neighbour re-reads
    store_spinor_nt<SP, D, T>(a.out[p], g.Vh_pad, h, acc);
    double nrm = 0.0;
    if (a.norm_partials) {
#pragma unroll
        for (int k = 0; k < 4 * D; k++)
            nrm += (double)acc[k].re * acc[k].re + (double)acc[k].im * acc[k].im;
    }
    return nrm;
}

// site handled by this thread under the traversal plan (see HopArgs)
__device__ inline uint32_t plan_site(const HopArgs &a, uint32_t bl, uint32_t S3, uint32_t ntile) {
    if (a.order != 1) return bl * 256 + threadIdx.x;
    const uint32_t tc = (uint32_t)a.tchunk;
    const uint32_t per_chunk = ntile * tc;
    const uint32_t chunk = bl / per_chunk;
    const uint32_t rem = bl - chunk * per_chunk;
    const uint32_t tile = rem / tc;
    const uint32_t t = chunk * tc + (rem - tile * tc);
    return t * S3 + tile * 256 + threadIdx.x;
}

// Waves per SIMD the compiler must allow for (caps registers); 0 = its choice.
#ifndef BSM_HOP_WAVES
#define BSM_HOP_WAVES 0
#endif
#if BSM_HOP_WAVES > 0
#define BSM_HOP_ATTR __attribute__((amdgpu_waves_per_eu(BSM_HOP_WAVES)))
#elif defined(BSM_HOP_VGPR)
#define BSM_HOP_ATTR __attribute__((amdgpu_num_vgpr(BSM_HOP_VGPR)))
#else
#define BSM_HOP_ATTR
#endif

// one output site per thread (plans 0, 1, 2, 4); RN != 0: fundamental links,
// representation RN formed on the fly
template <int D, bool REAL, int SP, int LP, int RN>
__device__ inline void hop_body(const Geom &g, const HopArgs &a, int nblk) {
    using T = typename Compute<SP>::T;
    const uint32_t S3 = (uint32_t)g.Vh / (uint32_t)g.L[0];
    uint32_t lb;
    int pi;
    uint32_t h;
    if (a.order == 4) {
        // XCD bands: XCD e (the hardware deals workgroups to the 8 XCDs in
        // turn) owns the band [e B/8, (e+1) B/8) of the B tiles of every time
        // slice and walks it t-major, so a time neighbour was fetched by the
        // same XCD a few workgroups earlier and is still in its L2
        const uint32_t e = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
        const uint32_t B = S3 / 256, B8 = B / kXcds, per_par = (uint32_t)g.L[0] * B8;
        pi = (int)(k / per_par);
        const uint32_t r = k - pi * per_par, t = r / B8, j = r - t * B8;
        lb = blockIdx.x;
        h = (t * B + e * B8 + j) * 256 + threadIdx.x;
    } else {
        lb = a.order == 2 ? blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
        pi = lb >= (uint32_t)nblk ? 1 : 0;
        h = plan_site(a, lb - pi * nblk, S3, S3 / 256);
    }
    const int p = a.p0 + pi;
    const bool active = h < (uint32_t)g.Vh;
    const size_t lblk = RN ? link_block_bytes(LP, false, otf_n(RN), g.Vh_pad) : link_block_bytes(LP, REAL, D, g.Vh_pad);
    double nrm = 0.0;
    if (active) {
        cx<T> acc[4 * D];
#pragma unroll
        for (int k = 0; k < 4 * D; k++) acc[k] = mk<T>(0, 0);
        Coords c = decode(g, h, p);
        const char *in = (const char *)a.in[p];
        const char *U = (const char *)a.U;
        const T eta = a.dagger ? (T)-1 : (T)1;
        if constexpr (RN != 0) {
            static_assert(otf_dim(RN) == D, "on-the-fly representation does not match d_R");
            hop_dir_otf<0, RN, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir_otf<1, RN, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir_otf<2, RN, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir_otf<3, RN, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        } else {
            hop_dir<0, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir<1, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir<2, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir<3, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        }
        nrm = hop_epilogue<D, SP, T>(g, a, p, h, acc);
    }
    if (a.norm_partials) {
        double s = block_sum_256(nrm);
        if (threadIdx.x == 0) a.norm_partials[lb] = s;
    }
}

template <int D, bool REAL, int SP, int LP>
__global__ __launch_bounds__(256) BSM_HOP_ATTR void k_hop(Geom g, HopArgs a, int nblk) {
    hop_body<D, REAL, SP, LP, 0>(g, a, nblk);
}

// the on-the-fly form (fundamental links, representation formed per hop)
template <int D, int SP, int LP, int RN>
__global__ __launch_bounds__(256) void k_hop_otf(
    Geom g, HopArgs a, int nblk) {
    hop_body<D, false, SP, LP, RN>(g, a, nblk);
}

// Column sweep (plan 3).  A thread owns one spatial half site s and walks
// tchunk consecutive time slices t (output site h = t S3 + s).  Its two time
// neighbours are the input sites (t +- 1) S3 + s of the same column, so every
// input spinor of the column is loaded once and serves the forward hop of
// output t-1 and the backward hop of output t+1: the backward projection is
// kept in a two-deep register ring.  Workgroups cover 256 consecutive s with
// the spatial tile fastest, so the spatial neighbours of a time slice are
// read by workgroups running at the same time, from contiguous memory.
// RN != 0: fundamental links, the representation formed on the fly in the
// time hops as in hop_dir_otf (and there for the spatial directions).
template <int D, bool REAL, int SP, int LP, int RN>
__device__ inline void hop_col_body(const Geom &g, const HopArgs &a, int nblk) {
    using T = typename Compute<SP>::T;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int pi = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t bl = lb - pi * nblk;
    const int p = a.p0 + pi;
    const uint32_t S3 = (uint32_t)g.Vh / (uint32_t)g.L[0];
    const uint32_t ntile = S3 / 256;
    const uint32_t chunk = bl / ntile;
    const uint32_t s = (bl - chunk * ntile) * 256 + threadIdx.x;
    const int T0 = (int)chunk * a.tchunk;
    const int LT = g.L[0];
    const size_t lblk = RN ? link_block_bytes(LP, false, otf_n(RN), g.Vh_pad) : link_block_bytes(LP, REAL, D, g.Vh_pad);
    const char *in = (const char *)a.in[p];
    const char *U = (const char *)a.U;
    const T eta = a.dagger ? (T)-1 : (T)1;
    const bool apt = g.apbc & 1;
    // spatial coordinates of the column
    Coords c0 = decode(g, s, 0);
    // ring: backward projections (sg = -eta) of in(t-1) and in(t)
    cx<T> r0a[D], r0b[D], r1a[D], r1b[D];
    {
        cx<T> sp[4 * D];
        const int tm = T0 == 0 ? LT - 1 : T0 - 1;
        load_spinor<SP, D, T>(in, g.Vh_pad, (uint32_t)tm * S3 + s, sp);
        project<0, D, T>(sp, -eta, r0a, r0b);
        load_spinor<SP, D, T>(in, g.Vh_pad, (uint32_t)T0 * S3 + s, sp);
        project<0, D, T>(sp, -eta, r1a, r1b);
    }
    double nrm = 0.0;
    for (int k = 0; k < a.tchunk; k++) {
        const int t = T0 + k;
        const uint32_t h = (uint32_t)t * S3 + s;
        Coords c = c0;
        c.t = t;
        c.row = ((uint32_t)t * g.L[3] + c0.z) * g.L[2] + c0.y;
        c.x = 2 * c0.xh + ((t + c0.z + c0.y + p) & 1);
        cx<T> acc[4 * D];
#pragma unroll
        for (int q = 0; q < 4 * D; q++) acc[q] = mk<T>(0, 0);
        // time: forward neighbour in(t+1), backward from the ring
        const int tp = t + 1 == LT ? 0 : t + 1;
        const uint32_t hp = (uint32_t)tp * S3 + s;
        const uint32_t hm = (uint32_t)(t == 0 ? LT - 1 : t - 1) * S3 + s;
        cx<T> nb0[D], nb1[D];
        const T wf = (apt && t + 1 == LT) ? (T)-1 : (T)1;
        const T wb = (apt && t == 0) ? (T)-1 : (T)1;
        if constexpr (RN != 0) {
            constexpr int N = otf_n(RN);
            constexpr bool NT = (BSM_LINK_NT >> SP) & 1;
            {
                cx<T> sp[4 * D], f0[D], f1[D], g0[D], g1[D];
                load_spinor<SP, D, T>(in, g.Vh_pad, hp, sp);
                const char *blk = link_block<0, false>(U, lblk, p);
                cx<T> u[N * N];
#pragma unroll
                for (int e = 0; e < N * N; e++) u[e] = load_link<LP, false, T, NT>(blk, g.Vh_pad, e, h);
                project<0, D, T>(sp, eta, f0, f1);
                project<0, D, T>(sp, -eta, nb0, nb1);
                rep_apply<RN, false, T>(u, f0, g0);
                rep_apply<RN, false, T>(u, f1, g1);
                reconstruct<0, D, T>(acc, eta, wf, g0, g1);
                otf_pin<SP, RN>(acc);
            }
            {
                cx<T> g0[D], g1[D];
                const char *blk = link_block<0, true>(U, lblk, p);
                cx<T> u[N * N];
#pragma unroll
                for (int e = 0; e < N * N; e++) u[e] = load_link<LP, false, T, NT>(blk, g.Vh_pad, e, hm);
                rep_apply<RN, true, T>(u, r0a, g0);
                rep_apply<RN, true, T>(u, r0b, g1);
                reconstruct<0, D, T>(acc, -eta, wb, g0, g1);
                otf_pin<SP, RN>(acc);
            }
        } else {
            {
                cx<T> sp[4 * D], f0[D], f1[D];
                load_spinor<SP, D, T>(in, g.Vh_pad, hp, sp);
                const char *blk = link_block<0, false>(U, lblk, p);
                LinkRegs<D, REAL, LP, true, T> L;
                L.load(blk, g.Vh_pad, h);
                project<0, D, T>(sp, eta, f0, f1);
                project<0, D, T>(sp, -eta, nb0, nb1);
                hop_half<0, D, REAL, LP, false, T>(g, L, blk, h, eta, wf, f0, f1, acc);
            }
            {
                const char *blk = link_block<0, true>(U, lblk, p);
                LinkRegs<D, REAL, LP, true, T> L;
                L.load(blk, g.Vh_pad, hm);
                hop_half<0, D, REAL, LP, true, T>(g, L, blk, hm, -eta, wb, r0a, r0b, acc);
            }
        }
#pragma unroll
        for (int i = 0; i < D; i++) {
            r0a[i] = r1a[i]; r0b[i] = r1b[i];
            r1a[i] = nb0[i]; r1b[i] = nb1[i];
        }
        if constexpr (RN != 0) {
            hop_dir_otf<1, RN, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir_otf<2, RN, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir_otf<3, RN, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        } else {
            hop_dir<1, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir<2, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
            hop_dir<3, D, REAL, SP, LP, T>(g, c, p, h, U, lblk, in, eta, acc);
        }
        nrm += hop_epilogue<D, SP, T>(g, a, p, h, acc);
    }
    if (a.norm_partials) {
        double sum = block_sum_256(nrm);
        if (threadIdx.x == 0) a.norm_partials[lb] = sum;
    }
}

template <int D, bool REAL, int SP, int LP>
__global__ __launch_bounds__(256) void k_hop_col(Geom g, HopArgs a, int nblk) {
    hop_col_body<D, REAL, SP, LP, 0>(g, a, nblk);
}

// the column sweep with fundamental links
template <int D, int SP, int LP, int RN>
__global__ __launch_bounds__(256) void k_hop_col_otf(Geom g, HopArgs a, int nblk) {
    hop_col_body<D, false, SP, LP, RN>(g, a, nblk);
}

// Launch for one (spinor precision, link precision, d_R); the definitions are
// explicitly instantiated in the hop_*.hip sources (split so they build in
// parallel).
// ------------------------------------------------------------ colour split
// FP64 spinors with large d_R: one thread per site would hold 4d complex
// accumulators, 4d complex neighbour components and a link row in FP64 and
// spill.  Here G threads share a site: thread (g, site) loads colours
// j = g, g+G, ... of each neighbour, projects them (the projection is
// colour-diagonal) into LDS, and after a barrier forms rows i = g, g+G, ...
// of U h from the whole half spinor, accumulating its own output colours.
// A workgroup holds 256/G sites; each wavefront has one colour group and 64
// consecutive sites, so every plane access is coalesced.
template <int MU>
__device__ inline void project1(const double2 (&s)[4], double sg, double2 &h0, double2 &h1) {
    const double2 s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3];
    if constexpr (MU == 0) {
        h0 = make_double2(fma(-sg, s2.x, s0.x), fma(-sg, s2.y, s0.y));
        h1 = make_double2(fma(-sg, s3.x, s1.x), fma(-sg, s3.y, s1.y));
    } else if constexpr (MU == 1) {
        h0 = make_double2(fma(-sg, s3.y, s0.x), fma(sg, s3.x, s0.y));
        h1 = make_double2(fma(-sg, s2.y, s1.x), fma(sg, s2.x, s1.y));
    } else if constexpr (MU == 2) {
        h0 = make_double2(fma(sg, s3.x, s0.x), fma(sg, s3.y, s0.y));
        h1 = make_double2(fma(-sg, s2.x, s1.x), fma(-sg, s2.y, s1.y));
    } else {
        h0 = make_double2(fma(-sg, s2.y, s0.x), fma(sg, s2.x, s0.y));
        h1 = make_double2(fma(sg, s3.y, s1.x), fma(-sg, s3.x, s1.y));
    }
}

// acc (4 spins of one colour) += reconstruction of (g0, g1)
template <int MU>
__device__ inline void reconstruct1(cx<double> (&acc)[4], double sg, double w, cx<double> g0, cx<double> g1) {
    const double v = -sg * w;
    acc[0].re = fma(w, g0.re, acc[0].re); acc[0].im = fma(w, g0.im, acc[0].im);
    acc[1].re = fma(w, g1.re, acc[1].re); acc[1].im = fma(w, g1.im, acc[1].im);
    cx<double> &a2 = acc[2], &a3 = acc[3];
    if constexpr (MU == 0) {
        a2.re = fma(v, g0.re, a2.re); a2.im = fma(v, g0.im, a2.im);
        a3.re = fma(v, g1.re, a3.re); a3.im = fma(v, g1.im, a3.im);
    } else if constexpr (MU == 1) {
        a2.re = fma(-v, g1.im, a2.re); a2.im = fma(v, g1.re, a2.im);
        a3.re = fma(-v, g0.im, a3.re); a3.im = fma(v, g0.re, a3.im);
    } else if constexpr (MU == 2) {
        a2.re = fma(v, g1.re, a2.re); a2.im = fma(v, g1.im, a2.im);
        a3.re = fma(-v, g0.re, a3.re); a3.im = fma(-v, g0.im, a3.im);
    } else {
        a2.re = fma(-v, g0.im, a2.re); a2.im = fma(v, g0.re, a2.im);
        a3.re = fma(v, g1.im, a3.re); a3.im = fma(-v, g1.re, a3.im);
    }
}

template <int MU, int D, bool REAL, int LP, int G>
__device__ inline void hop_dir_wide(const Geom &g, const Coords &c, bool active, int p, uint32_t h, const char *U,
                                    size_t lblk, const char *in, double eta, int gi, int sl, double2 *hs,
                                    cx<double> (&acc)[(D + G - 1) / G][4]) {
    constexpr int NC = (D + G - 1) / G, SPW = 256 / G;
#pragma unroll
    for (int dir = 0; dir < 2; dir++) {
        const bool back = dir == 1;
        float wf = 1.f;
        const uint32_t hn = active ? neighbour<MU>(g, c, back, wf) : 0u;
        const double sg = back ? -eta : eta;
        const double2 *sp = (const double2 *)in;
        // my colours of the neighbour, projected, into LDS [half][colour][site]
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const int j = gi + G * k;
            if (j < D) {
                double2 sv[4], h0 = make_double2(0.0, 0.0), h1 = h0;
                if (active) {
#pragma unroll
                    for (int s4 = 0; s4 < 4; s4++) sv[s4] = sp[(size_t)(s4 * D + j) * g.Vh_pad + hn];
                    project1<MU>(sv, sg, h0, h1);
                }
                hs[(0 * D + j) * SPW + sl] = h0;
                hs[(1 * D + j) * SPW + sl] = h1;
            }
        }
        __syncthreads();
        const char *blk = back ? link_block<MU, true>(U, lblk, p) : link_block<MU, false>(U, lblk, p);
        const uint32_t hl = back ? hn : h;
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const int i = gi + G * k;
            if (i < D && active) {
                // the whole link row (forward) or column (backward) in flight first
                cx<double> u[D];
#pragma unroll
                for (int j = 0; j < D; j++)
                    u[j] = load_link<LP, REAL, double, true>(blk, g.Vh_pad, back ? j * D + i : i * D + j, hl);
                cx<double> g0 = mk<double>(0.0, 0.0), g1 = g0;
#pragma unroll
                for (int j = 0; j < D; j++) {
                    const double2 a0 = hs[(0 * D + j) * SPW + sl], a1 = hs[(1 * D + j) * SPW + sl];
                    const cx<double> h0 = mk<double>(a0.x, a0.y), h1 = mk<double>(a1.x, a1.y);
                    if (!back) {
                        g0 = cfma(u[j], h0, g0);
                        g1 = cfma(u[j], h1, g1);
                    } else {
                        // (U^dag h)_i = sum_j conj(U_ji) h_j
                        g0 = cfma_conj(u[j], h0, g0);
                        g1 = cfma_conj(u[j], h1, g1);
                    }
                }
                reconstruct1<MU>(acc[k], sg, (double)wf, g0, g1);
            }
        }
        __syncthreads();
    }
}

template <int D, bool REAL, int LP, int G>
__global__ __launch_bounds__(256) void k_hop_wide(Geom g, HopArgs a, int nblk) {
    constexpr int NC = (D + G - 1) / G, SPW = 256 / G;
    __shared__ double2 hs[2 * D * SPW];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int pi = lb >= (uint32_t)nblk ? 1 : 0;
    const int p = a.p0 + pi;
    const int gi = threadIdx.x / SPW, sl = threadIdx.x % SPW;
    const uint32_t h = (lb - pi * nblk) * SPW + sl;
    const bool active = h < (uint32_t)g.Vh;
    const size_t lblk = link_block_bytes(LP, REAL, D, g.Vh_pad);
    cx<double> acc[NC][4];
#pragma unroll
    for (int k = 0; k < NC; k++)
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++) acc[k][s4] = mk<double>(0.0, 0.0);
    Coords c{};
    if (active) c = decode(g, h, p);
    const char *in = (const char *)a.in[p];
    const char *U = (const char *)a.U;
    const double eta = a.dagger ? -1.0 : 1.0;
    hop_dir_wide<0, D, REAL, LP, G>(g, c, active, p, h, U, lblk, in, eta, gi, sl, hs, acc);
    hop_dir_wide<1, D, REAL, LP, G>(g, c, active, p, h, U, lblk, in, eta, gi, sl, hs, acc);
    hop_dir_wide<2, D, REAL, LP, G>(g, c, active, p, h, U, lblk, in, eta, gi, sl, hs, acc);
    hop_dir_wide<3, D, REAL, LP, G>(g, c, active, p, h, U, lblk, in, eta, gi, sl, hs, acc);
    double nrm = 0.0;
    if (active) {
        const double bb = a.b, aa = a.a;
        const double2 *x = (const double2 *)a.x[p];
        double2 *o = (double2 *)a.out[p];
#pragma unroll
        for (int k = 0; k < NC; k++) {
            const int i = gi + G * k;
            if (i >= D) continue;
#pragma unroll
            for (int s4 = 0; s4 < 4; s4++) {
                const size_t e = (size_t)(s4 * D + i) * g.Vh_pad + h;
                double re = bb * acc[k][s4].re, im = bb * acc[k][s4].im;
                if (aa != 0.0) {
                    const double2 xv = x[e];
                    re = fma(aa, xv.x, re);
                    im = fma(aa, xv.y, im);
                }
                typedef double f64x2w __attribute__((ext_vector_type(2)));
                f64x2w v = {re, im};
                __builtin_nontemporal_store(v, (f64x2w *)o + e);
                nrm += re * re + im * im;
            }
        }
    }
    if (a.norm_partials) {
        const double s = block_sum_256(nrm);
        if (threadIdx.x == 0) a.norm_partials[lb] = s;
    }
}

template <int SP, int LP, int D>
bsm_status hop_run(const Geom &g, bool real, const HopArgs &a, hipStream_t st) {
    const int grid = hop_grid(g, a);
    const int nblk = grid / a.np;
    if (a.norm_partials && (int64_t)grid > a.norm_cap)
        return fail(BSM_ERR_ARG, "fused-norm hop needs " + std::to_string(grid) + " reduction slots, " +
                                     std::to_string(a.norm_cap) + " available");
    if (real && !(D == 3 || D == 8 || D == 15))
        return fail(BSM_ERR_UNSUPPORTED, "real links only for adjoint d_R 3, 8, 15");
    if (a.wide > 0) {
        if constexpr (SP == BSM_F64 && D >= 5) {
            if (a.wide != (D <= 8 ? 2 : 4)) return fail(BSM_ERR_ARG, "colour split does not match d_R");
            constexpr int G = D <= 8 ? 2 : 4;
            if (real) {
                if constexpr (D == 8 || D == 15) k_hop_wide<D, true, LP, G><<<grid, 256, 0, st>>>(g, a, nblk);
            } else {
                k_hop_wide<D, false, LP, G><<<grid, 256, 0, st>>>(g, a, nblk);
            }
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        } else {
            return fail(BSM_ERR_ARG, "colour split only for FP64 spinors with d_R >= 5");
        }
    }
    if (a.order == 3) {
        if constexpr (D <= kColMaxD) {
            if (real) {
                if constexpr (D == 3 || D == 8 || D == 15) k_hop_col<D, true, SP, LP><<<grid, 256, 0, st>>>(g, a, nblk);
            } else {
                k_hop_col<D, false, SP, LP><<<grid, 256, 0, st>>>(g, a, nblk);
            }
        } else {
            return fail(BSM_ERR_UNSUPPORTED, "column plan only for d_R <= 6");
        }
    } else if (real) {
        if constexpr (D == 3 || D == 8 || D == 15) k_hop<D, true, SP, LP><<<grid, 256, 0, st>>>(g, a, nblk);
    } else {
        k_hop<D, false, SP, LP><<<grid, 256, 0, st>>>(g, a, nblk);
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// fundamental links, representation RN formed on the fly (one thread per
// site, or the column sweep for d_R <= 6; no colour split)
template <int SP, int LP, int RN>
bsm_status hop_run_otf(const Geom &g, const HopArgs &a, hipStream_t st) {
    constexpr int D = otf_dim(RN);
    if (a.wide > 0 || (a.order == 3 && D > kColMaxD)) return fail(BSM_ERR_ARG, "on-the-fly hop: plan not available");
    const int grid = hop_grid(g, a);
    const int nblk = grid / a.np;
    if (a.norm_partials && (int64_t)grid > a.norm_cap)
        return fail(BSM_ERR_ARG, "fused-norm hop needs " + std::to_string(grid) + " reduction slots, " +
                                     std::to_string(a.norm_cap) + " available");
    if (a.order == 3) {
        if constexpr (D <= kColMaxD) k_hop_col_otf<D, SP, LP, RN><<<grid, 256, 0, st>>>(g, a, nblk);
    } else {
        k_hop_otf<D, SP, LP, RN><<<grid, 256, 0, st>>>(g, a, nblk);
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

#define BSM_HOP_INSTANTIATE(SP, LP, D) \
    template bsm_status hop_run<SP, LP, D>(const Geom &, bool, const HopArgs &, hipStream_t);


}  // namespace bsm
