// Multi-RHS Wilson hop on FP16 block fields and FP16 matrix cores, and the
// F16S vector kernels of the batched solver's inner recurrence.
//
// The hop of 16 right-hand sides at one site and direction is, as in the FP32
// block kernel, the d x d real (adjoint) link times the d x 64 matrix of
// projected half spinors, here as four v_mfma_f32_16x16x16_f16 (one per spin
// component and re/im part; the whole colour sum, d <= 15 padded to 16, in
// one instruction) with FP32 accumulation:
//   A[i][k] = U_ik (forward; U^T stored for the backward hop),  lane l: i = l%16, k = 4(l/16) + 0..3
//   B[k][j] = h[colour k][rhs j],                                 lane l: k = 4(l/16) + 0..3, j = l%16
//   D[i][j] -> lane l holds rows 4(l/16) + v, v < 4, column j = l%16.
// Lane l therefore loads, for RHS l%16, the four colours 4(l/16) + 0..3 of its
// neighbour (one 16-byte load per colour: the four spins), and the link row
// i = l%16, columns 4(l/16) + 0..3 (one 8-byte load).  The per-RHS scale of
// the neighbour multiplies column j of the product, i.e. one factor per lane.
// Products of FP16 operands are exact in FP32; the projected half spinor is
// rounded to FP16 (relative 2^-11), the same order as the storage rounding.
#include <type_traits>

#include "block.h"
#include "block_dev.h"
#include "dispatch.h"
#include "spinor_io.h"

namespace bsm {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline float2 half2_to_f(uint32_t w) {
    __half2 hh = *reinterpret_cast<__half2 *>(&w);
    return __half22float2(hh);
}
__device__ inline uint32_t f_to_half2(float a, float b) {
    __half2 hh = __floats2half2_rn(a, b);
    return *reinterpret_cast<uint32_t *>(&hh);
}

// largest |re|, |im| of the values of one RHS over the four lanes that hold
// it (lanes r, r + 16, r + 32, r + 48)
__device__ inline float rhs_max(float m) {
    m = fmaxf(m, __shfl_xor(m, 16, 64));
    return fmaxf(m, __shfl_xor(m, 32, 64));
}

// Quantise and store the colours 4q + v (v < 4, < D) of one site and RHS held
// by this lane as v[colour slot][spin]; returns the lane's share of |stored|^2.
template <int D>
__device__ inline double store_site_h(char *blk, size_t scale_off, uint32_t h, int r, int q,
                                      const float2 (&v)[4][4]) {
    float m = 0.f;
#pragma unroll
    for (int s = 0; s < 4; s++)
        if (4 * q + s < D)
#pragma unroll
            for (int sp = 0; sp < 4; sp++) m = fmaxf(m, fmaxf(fabsf(v[s][sp].x), fabsf(v[s][sp].y)));
    m = rhs_max(m);
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    uint4 *o = (uint4 *)(blk + (size_t)h * blockh_site_bytes(D)) + r;
    double nrm = 0.0;
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const int c = 4 * q + s;
        if (c >= D) continue;
        uint32_t w[4];
#pragma unroll
        for (int sp = 0; sp < 4; sp++) {
            w[sp] = f_to_half2(v[s][sp].x * inv, v[s][sp].y * inv);
            const float2 back = half2_to_f(w[sp]);
            const double br = (double)(back.x * m), bi = (double)(back.y * m);
            nrm += br * br + bi * bi;
        }
        o[c * kNR] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (q == 0) ((float *)(blk + scale_off))[(size_t)h * kNR + r] = m;
    return nrm;
}

// the colours 4q + s (s < 4) of one site and RHS, decoded (slots of colours
// >= D hold a copy of colour D - 1)
template <int D>
__device__ inline void load_site_h(const char *blk, size_t scale_off, uint32_t h, int r, int q, float2 (&v)[4][4]) {
    const uint4 *ip = (const uint4 *)(blk + (size_t)h * blockh_site_bytes(D)) + r;
    const float sc = ((const float *)(blk + scale_off))[(size_t)h * kNR + r];
    // colours >= D load colour D - 1 (unconditional loads; the caller never
    // stores or sums those slots)
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const uint4 w = ip[min(4 * q + s, D - 1) * kNR];
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int sp = 0; sp < 4; sp++) {
            const float2 f = half2_to_f(ws[sp]);
            v[s][sp] = make_float2(f.x * sc, f.y * sc);
        }
    }
}

// Operands of one hop K = 2 mu + (backward ? 1 : 0) of one site: the four
// colours 4q + 0..3 of the neighbour for RHS r (16 bytes each), its scale,
// the link row (8 bytes) and the boundary weight.
struct HopHOps {
    uint4 sv[4];
    u32x2 lk;
    float scl, w;
};

template <int K, int D>
__device__ inline void hoph_load(const Geom &g, const BlockHopHArgs &a, const Coords &c, int p, uint32_t h, int r,
                                 int q, size_t scale_off, HopHOps &o) {
    constexpr int MU = K >> 1;
    constexpr bool back = (K & 1) != 0;
    constexpr int KP = blockh_kpad(D);
    const char *in = a.in[p];
    const uint32_t hn = neighbour<MU>(g, c, back, o.w);
    const uint4 *sp = (const uint4 *)(in + (size_t)hn * blockh_site_bytes(D)) + r;
    // Every load is unconditional, at a clamped index, so that no load sits in
    // a divergent branch (the compiler waits for such a load inside its
    // branch, which serialises the hops).  A colour k >= D loads colour D - 1:
    // its product is zero, as the link columns k >= D are zero (padding, or
    // the operand masked in hoph_apply); a row i >= D loads row D - 1 and
    // gives result rows that are never stored.
    // scale first: loads complete in order, and the scale is the last
    // operand the products need
    o.scl = ((const float *)(in + scale_off))[(size_t)hn * kNR + r];
    const int qm = (back ? 1 - p : p) * 4 + MU;
    const __half *L = a.U + ((size_t)((back ? 8 : 0) + qm) * g.Vh_pad + (back ? hn : h)) * blockh_link_halves(D) +
                      min(r, D - 1) * KP + 4 * min(q, (D - 1) / 4);
    o.lk = __builtin_nontemporal_load((const u32x2 *)L);
#pragma unroll
    for (int s = 0; s < 4; s++) o.sv[s] = sp[min(4 * q + s, D - 1) * kNR];
}

template <int K, int D>
__device__ inline void hoph_apply(const HopHOps &o, int q, float eta, f4 (&acc)[4][2]) {
    constexpr int MU = K >> 1;
    const float sg = (K & 1) ? -eta : eta;
    h4 b0r, b0i, b1r, b1i;
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const float2 s4[4] = {half2_to_f(o.sv[s].x), half2_to_f(o.sv[s].y), half2_to_f(o.sv[s].z),
                              half2_to_f(o.sv[s].w)};
        float2 h0, h1;
        project_c<MU>(s4, sg, h0, h1);
        b0r[s] = (_Float16)h0.x;
        b0i[s] = (_Float16)h0.y;
        b1r[s] = (_Float16)h1.x;
        b1i[s] = (_Float16)h1.y;
    }
    u32x2 lk = o.lk;
    if constexpr (D <= 12) {   // column groups 4q >= D hold no link columns
        lk.x = 4 * q < D ? lk.x : 0u;
        lk.y = 4 * q < D ? lk.y : 0u;
    }
    const h4 A = __builtin_bit_cast(h4, lk);
    const f4 z = {0.f, 0.f, 0.f, 0.f};
    const f4 g0r = __builtin_amdgcn_mfma_f32_16x16x16f16(A, b0r, z, 0, 0, 0);
    const f4 g0i = __builtin_amdgcn_mfma_f32_16x16x16f16(A, b0i, z, 0, 0, 0);
    const f4 g1r = __builtin_amdgcn_mfma_f32_16x16x16f16(A, b1r, z, 0, 0, 0);
    const f4 g1i = __builtin_amdgcn_mfma_f32_16x16x16f16(A, b1i, z, 0, 0, 0);
    reconstruct_c<MU>(acc, sg, o.w * o.scl, g0r, g0i, g1r, g1i);
}

template <int B, int E, class F>
__device__ inline void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// The eight hops of one site in groups of NB: the loads of a whole group
// are issued before its products, so NB neighbour fetches are in flight per
// wavefront (the operands of one hop are 19 registers).  Measured at
// 24^3 x 48, d_R = 15: NB = 2 1144 us, 4 1163 us, 8 1430 us (occupancy 4,
// 3, 2 wavefronts per SIMD).
constexpr int kHopHDepth = 2;

template <int D>
__device__ inline void hoph_site(const Geom &g, const BlockHopHArgs &a, const Coords &c, int p, uint32_t h, int r,
                                 int q, float eta, size_t scale_off, f4 (&acc)[4][2]) {
    constexpr int NB = kHopHDepth;
    static_assert(8 % NB == 0, "hop groups must divide the eight hops");
    static_for<0, 8 / NB>([&](auto gi) {
        constexpr int base = decltype(gi)::value * NB;
        HopHOps o[NB];
        static_for<0, NB>([&](auto j) {
            hoph_load<base + decltype(j)::value, D>(g, a, c, p, h, r, q, scale_off, o[decltype(j)::value]);
        });
        static_for<0, NB>([&](auto j) { hoph_apply<base + decltype(j)::value, D>(o[decltype(j)::value], q, eta, acc); });
        // The group's sums are complete here: the empty statements pin the
        // accumulators to this point (the optimiser would otherwise sink every
        // hop's reconstruction to the end of the site and hold all 32 products
        // at once), and the barrier keeps the next group's loads after this
        // group's products.
#pragma unroll
        for (int sp = 0; sp < 4; sp++) {
            asm volatile("" : "+v"(acc[sp][0]));
            asm volatile("" : "+v"(acc[sp][1]));
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}

// One wavefront per site, WPB = blockDim.x / 64 sites per workgroup.
template <int D>
__global__ __launch_bounds__(256) void k_hop_blockh(Geom g, BlockHopHArgs a, int nblk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const uint32_t lb = xcd_chunk_remap(blockIdx.x, gridDim.x, (uint32_t)a.xchunk);
    const int pi = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t s = (lb - pi * nblk) * (uint32_t)wpb + wave;
    const int p = a.p0 + pi;
    const size_t scale_off = blockh_scale_off(g, D);
    double nrm = 0.0;
    if (s < (uint32_t)g.Vh) {
        const uint32_t h = block_site(g, a.tile, s);
        f4 acc[4][2];
#pragma unroll
        for (int sp = 0; sp < 4; sp++) acc[sp][0] = acc[sp][1] = f4{0.f, 0.f, 0.f, 0.f};
        const Coords c = decode(g, h, p);
        const float eta = a.dagger ? -1.f : 1.f;
        hoph_site<D>(g, a, c, p, h, r, q, eta, scale_off, acc);
        float2 v[4][4];
        if (a.use_x) load_site_h<D>(a.x[p], scale_off, h, r, q, v);
        const float ar = a.use_x ? a.a[r] : 0.f, br = a.b[r];
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                const float re = br * acc[sp][0][k], im = br * acc[sp][1][k];
                v[k][sp] = a.use_x ? make_float2(fmaf(ar, v[k][sp].x, re), fmaf(ar, v[k][sp].y, im))
                                   : make_float2(re, im);
            }
        nrm = store_site_h<D>(a.out[p], scale_off, h, r, q, v);
    }
    if (a.norm_partials) {
        nrm += __shfl_xor(nrm, 16, 64);
        nrm += __shfl_xor(nrm, 32, 64);
        __shared__ double ws[4][kNR];
        if (lane < kNR) ws[wave][lane] = nrm;
        __syncthreads();
        if (threadIdx.x < kNR) {
            double t = ws[0][threadIdx.x];
            for (int k = 1; k < wpb; k++) t += ws[k][threadIdx.x];
            a.norm_partials[(size_t)lb * kNR + threadIdx.x] = t;
        }
    }
}

int hop_blockh_grid(const Geom &g, const BlockHopHArgs &a) { return (g.Vh + a.wpb - 1) / a.wpb * a.np; }

void apply_blockh_plan(const Geom &g, const BlockPlan &p, BlockHopHArgs &a) {
    a.wpb = p.wpb;
    a.tile = p.tiled ? block_tile_for(g) : BlockTile{};
    a.xchunk = p.xchunk;
}

template <int D>
struct BlockHopHByD {
    static bsm_status run(const Geom &g, const BlockHopHArgs &a, hipStream_t st) {
        if constexpr (D == 3 || D == 8 || D == 15) {
            const int grid = hop_blockh_grid(g, a);
            k_hop_blockh<D><<<grid, 64 * a.wpb, 0, st>>>(g, a, grid / a.np);
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        }
        return fail(BSM_ERR_UNSUPPORTED, "block hop: real links exist only for d_R = 3, 8, 15");
    }
};

bsm_status launch_hop_blockh(const Geom &g, int d, const BlockHopHArgs &a, hipStream_t st) {
    if (a.wpb != 1 && a.wpb != 2 && a.wpb != 4) return fail(BSM_ERR_ARG, "block plan: 1, 2 or 4 wavefronts");
    return dispatch_d<BlockHopHByD>(d, g, a, st);
}

bsm_status blockh_autotune(bsm_ctx ctx, int d, const __half *U_blockh, char *scratch_in, char *scratch_out,
                           hipStream_t st) {
    const Geom &g = ctx->g;
    BSM_HIP(hipMemsetAsync(scratch_in, 0, blockh_parity_bytes(g, d), st));
    hipEvent_t e0, e1;
    BSM_HIP(hipEventCreate(&e0));
    BSM_HIP(hipEventCreate(&e1));
    BlockPlan best;
    best.us = 0.f;
    bsm_status status = BSM_OK;
    const BlockTile tile = block_tile_for(g);
    for (int tiled = 0; tiled <= (tile.tt ? 1 : 0) && status == BSM_OK; tiled++)
        for (int xchunk : {0, 1, 16})
            for (int wpb : {1, 2, 4}) {
                if (status != BSM_OK) break;
                BlockHopHArgs a{};
                a.U = U_blockh;
                a.p0 = 0;
                a.np = 1;
                a.in[0] = scratch_in;
                a.out[0] = scratch_out;
                for (int r = 0; r < kNR; r++) { a.a[r] = 0.f; a.b[r] = 1.f; }
                a.wpb = wpb;
                a.xchunk = xchunk;
                if (tiled) a.tile = tile;
                const int reps = 5;
                if ((status = launch_hop_blockh(g, d, a, st)) != BSM_OK) break;   // warm-up
                if (hipEventRecord(e0, st) != hipSuccess) { status = fail(BSM_ERR_HIP, "event"); break; }
                for (int k = 0; k < reps && status == BSM_OK; k++) status = launch_hop_blockh(g, d, a, st);
                if (status != BSM_OK) break;
                float ms = 0.f;
                if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    status = fail(BSM_ERR_HIP, "block autotune timing");
                    break;
                }
                const float us = ms * 1000.f / reps;
                if (best.us == 0.f || us < best.us) {
                    best.spw = 1;
                    best.wpb = wpb;
                    best.tiled = tiled;
                    best.xchunk = xchunk;
                    best.us = us;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == BSM_OK) ctx->block_plans[d][1] = best;
    return status;
}

// --------------------------------------------------------------- layouts
// one thread per (site, parity * 4 + mu): both orientations of the link
// 32 sites per workgroup: link elements read plane by plane into LDS
// ([site][i * d + j]), then both orientations written contiguously two
// halves per thread, the rows padded to kpad columns and the link to dk
// halves with zeros
template <int LP>
__global__ __launch_bounds__(256) void k_gauge_to_blockh(Geom g, int d, const char *src, __half *dst) {
    constexpr int S = 32;
    __shared__ float t[S * 225];
    const uint32_t h0 = blockIdx.x * S;
    const int qm = blockIdx.y;
    const int dd = d * d, ldt = dd | 1;   // odd row stride: no LDS bank conflicts
    const int ns = min(S, (int)((uint32_t)g.Vh_pad - h0));
    const int kp = blockh_kpad(d), dk = blockh_link_halves(d);
    const char *blk = src + (size_t)qm * link_block_bytes(LP, true, d, g.Vh_pad);
    for (int idx = threadIdx.x; idx < S * dd; idx += 256) {
        const int e = idx / S, s = idx - e * S;
        if (s < ns) t[s * ldt + e] = (float)load_link<LP, true, float>(blk, g.Vh_pad, e, h0 + s).re;
    }
    __syncthreads();
    __half2 *o0 = (__half2 *)(dst + ((size_t)qm * g.Vh_pad + h0) * dk);
    __half2 *o1 = (__half2 *)(dst + ((size_t)(8 + qm) * g.Vh_pad + h0) * dk);
    for (int idx = threadIdx.x; idx < ns * dk / 2; idx += 256) {
        const int pos = 2 * idx, s = pos / dk, e = pos - s * dk;
        float u[2], ut[2];
#pragma unroll
        for (int c = 0; c < 2; c++) {
            const int i = (e + c) / kp, k = (e + c) - i * kp;
            const bool in = i < d && k < d;
            u[c] = in ? t[s * ldt + i * d + k] : 0.f;
            ut[c] = in ? t[s * ldt + k * d + i] : 0.f;
        }
        o0[idx] = __floats2half2_rn(u[0], u[1]);
        o1[idx] = __floats2half2_rn(ut[0], ut[1]);
    }
}

bsm_status launch_gauge_to_blockh(const Geom &g, int d, int link_prec, const void *U_rep, __half *U_blockh,
                                  hipStream_t st) {
    if (d > 15) return fail(BSM_ERR_ARG, "block links: d_R above 15");
    dim3 grid((g.Vh_pad + 31) / 32, 8);
    switch (link_prec) {
    case BSM_F64: k_gauge_to_blockh<BSM_F64><<<grid, 256, 0, st>>>(g, d, (const char *)U_rep, U_blockh); break;
    case BSM_F32: k_gauge_to_blockh<BSM_F32><<<grid, 256, 0, st>>>(g, d, (const char *)U_rep, U_blockh); break;
    default: return fail(BSM_ERR_UNSUPPORTED, "FP16 block links from F16 links");
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// one wavefront per site (both parities): lane (r, q) holds RHS r, colours
// 4q + 0..3; the values are first rounded to float32, as the oracle's F16S
// quantisation takes them
template <int D>
__global__ __launch_bounds__(256) void k_pack_blockh(Geom g, int n_rhs, const double2 *canon, char *block,
                                                     int unpack) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const uint32_t sidx = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (sidx >= 2u * (uint32_t)g.Vh_pad) return;   // whole wavefronts leave together
    const int p = sidx >= (uint32_t)g.Vh_pad ? 1 : 0;
    const uint32_t h = sidx - p * g.Vh_pad;
    char *blk = block + (size_t)p * blockh_parity_bytes(g, D);
    const size_t scale_off = blockh_scale_off(g, D);
    const bool live = h < (uint32_t)g.Vh;
    int64_t lex = 0;
    if (live) {
        const Coords co = decode(g, h, p);
        lex = (int64_t)co.row * g.L[1] + co.x;
    }
    const int64_t V = 2 * (int64_t)g.Vh;
    if (!unpack) {
        float2 v[4][4];
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                const int c = 4 * q + s;
                double2 z = make_double2(0.0, 0.0);
                if (live && r < n_rhs && c < D) z = canon[((r * V + lex) * 4 + sp) * D + c];
                v[s][sp] = make_float2((float)z.x, (float)z.y);
            }
        (void)store_site_h<D>(blk, scale_off, h, r, q, v);
    } else if (live && r < n_rhs) {
        float2 v[4][4];
        load_site_h<D>(blk, scale_off, h, r, q, v);
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                const int c = 4 * q + s;
                if (c < D)
                    ((double2 *)canon)[((r * V + lex) * 4 + sp) * D + c] =
                        make_double2((double)v[s][sp].x, (double)v[s][sp].y);
            }
    }
}

template <int D>
struct PackBlockHByD {
    static bsm_status run(const Geom &g, int n_rhs, const double2 *canon, char *block, int unpack,
                          hipStream_t st) {
        if constexpr (D == 3 || D == 8 || D == 15) {
            const unsigned grid = (unsigned)((2 * (size_t)g.Vh_pad + 3) / 4);
            k_pack_blockh<D><<<grid, 256, 0, st>>>(g, n_rhs, canon, block, unpack);
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        }
        return fail(BSM_ERR_UNSUPPORTED, "FP16 block fields exist only for d_R = 3, 8, 15");
    }
};

bsm_status launch_pack_blockh(const Geom &g, int d, int n_rhs, const void *canon, void *block, bool unpack,
                              hipStream_t st) {
    return dispatch_d<PackBlockHByD>(d, g, n_rhs, (const double2 *)canon, (char *)block, unpack ? 1 : 0, st);
}

// ------------------------------------------------------------ vector ops
// One wavefront per site, sites strided over the grid; lanes as in the hop.
int blockh_blas_grid(const Geom &g) {
    const int nb = (g.Vh + 3) / 4;
    return nb < 16384 ? nb : 16384;
}

// r32 element of colour c, spin sp, RHS r at site h (FP32 block layout
// [h][c][spin][rhs] float2)
template <int D>
__device__ inline size_t f32_elem(uint32_t h, int c, int sp, int r) {
    return (((size_t)h * D + c) * 4 + sp) * kNR + r;
}

template <int D>
__global__ __launch_bounds__(256) void k_blockh_xpay(Geom g, char *p, const float2 *r32, const double *beta) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const float b = (float)beta[r];
    const size_t scale_off = blockh_scale_off(g, D);
    for (uint32_t h = blockIdx.x * 4 + (threadIdx.x >> 6); h < (uint32_t)g.Vh; h += gridDim.x * 4) {
        float2 v[4][4];
        load_site_h<D>(p, scale_off, h, r, q, v);
        // unconditional loads at clamped colours (slots >= D are not stored)
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int c = min(4 * q + s, D - 1);
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                const float2 rv = r32[f32_elem<D>(h, c, sp, r)];
                v[s][sp] = make_float2(fmaf(b, v[s][sp].x, rv.x), fmaf(b, v[s][sp].y, rv.y));
            }
        }
        (void)store_site_h<D>(p, scale_off, h, r, q, v);
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_blockh_update(Geom g, float2 *x32, const char *p, float2 *r32,
                                                       const char *qf, const double *alpha, double *partials) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    const float a = (float)alpha[r];
    const size_t scale_off = blockh_scale_off(g, D);
    double nrm = 0.0;
    for (uint32_t h = blockIdx.x * 4 + (threadIdx.x >> 6); h < (uint32_t)g.Vh; h += gridDim.x * 4) {
        float2 pv[4][4], qv[4][4], xv[4][4], rv[4][4];
        load_site_h<D>(p, scale_off, h, r, q, pv);
        load_site_h<D>(qf, scale_off, h, r, q, qv);
        // all loads first, unconditional at clamped colours; stores only for
        // the colours < D
#pragma unroll
        for (int s = 0; s < 4; s++)
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                const size_t e = f32_elem<D>(h, min(4 * q + s, D - 1), sp, r);
                xv[s][sp] = x32[e];
                rv[s][sp] = r32[e];
            }
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int c = 4 * q + s;
            if (c >= D) continue;
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                const size_t e = f32_elem<D>(h, c, sp, r);
                float2 xn = xv[s][sp], rn = rv[s][sp];
                xn.x = fmaf(a, pv[s][sp].x, xn.x);
                xn.y = fmaf(a, pv[s][sp].y, xn.y);
                rn.x = fmaf(-a, qv[s][sp].x, rn.x);
                rn.y = fmaf(-a, qv[s][sp].y, rn.y);
                x32[e] = xn;
                r32[e] = rn;
                nrm += (double)rn.x * rn.x + (double)rn.y * rn.y;
            }
        }
    }
    nrm += __shfl_xor(nrm, 16, 64);
    nrm += __shfl_xor(nrm, 32, 64);
    __shared__ double ws[4][kNR];
    const int wave = threadIdx.x >> 6;
    if (lane < kNR) ws[wave][lane] = nrm;
    __syncthreads();
    if (threadIdx.x < kNR)
        partials[(size_t)blockIdx.x * kNR + threadIdx.x] =
            (ws[0][threadIdx.x] + ws[1][threadIdx.x]) + (ws[2][threadIdx.x] + ws[3][threadIdx.x]);
}

template <int D>
struct BlockHBlasByD {
    static bsm_status run(const Geom &g, int op, char *p, float2 *x, float2 *r, const char *q, const double *coef,
                          double *partials, hipStream_t st) {
        if constexpr (D == 3 || D == 8 || D == 15) {
            if (op == 0) k_blockh_xpay<D><<<blockh_blas_grid(g), 256, 0, st>>>(g, p, r, coef);
            else k_blockh_update<D><<<blockh_blas_grid(g), 256, 0, st>>>(g, x, p, r, q, coef, partials);
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        }
        return fail(BSM_ERR_UNSUPPORTED, "FP16 block fields exist only for d_R = 3, 8, 15");
    }
};

bsm_status blockh_xpay(const Geom &g, int d, char *p, const float2 *r, const double *beta, hipStream_t st) {
    return dispatch_d<BlockHBlasByD>(d, g, 0, p, nullptr, const_cast<float2 *>(r), nullptr, beta, nullptr, st);
}

bsm_status blockh_update(const Geom &g, int d, float2 *x, const char *p, float2 *r, const char *q,
                         const double *alpha, double *partials, hipStream_t st) {
    return dispatch_d<BlockHBlasByD>(d, g, 1, const_cast<char *>(p), x, r, q, alpha, partials, st);
}

}  // namespace bsm
