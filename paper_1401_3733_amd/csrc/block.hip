// Multi-RHS Wilson hop on FP32 matrix cores, and the per-RHS vector kernels of
// the batched solver.
//
// For real (adjoint) links the hop of 16 right-hand sides at one site and
// direction is one dense product: the d x d link times the d x 64 matrix of
// projected half spinors (2 spin components x re/im x 16 RHS).  One wavefront
// owns one site; per K-step of 4 colours it issues four
// v_mfma_f32_16x16x4f32 (one per spin component and re/im part), with
//   A[i][k]  = U_ik (forward) or U_ki (backward, U^dag = U^T),  lane l: i = l%16, k = l/16
//   B[k][j]  = h[colour k][rhs j],                               lane l: k = l/16, j = l%16
//   D[i][j]  -> lane l holds rows 4(l/16)+v, v<4, column j = l%16.
// So lane l owns RHS l%16 and colours l/16 + 4 kb for the operands and rows
// 4(l/16)+v of the result: the per-RHS epilogue coefficients, the spin
// reconstruction and the per-RHS norms never leave the lane.
#include "block.h"
#include "block_dev.h"
#include "dispatch.h"
#include "spinor_io.h"

namespace bsm {

// Both hops along MU for the S sites of this wavefront (S independent MFMA
// chains, so the loads of one site overlap the products of the other).
template <int MU, int D, int S>
__device__ inline void hop_dir_block(const Geom &g, const BlockHopArgs &a, const Coords (&c)[S], int p,
                                     const uint32_t (&h)[S], int r, int q, float eta, f4 (&acc)[S][4][2]) {
    constexpr int KB = (D + 3) / 4;
    constexpr size_t SITE = (size_t)D * 4 * kNR;
    // one direction at a time keeps the operands of a single hop in registers
#pragma unroll 1
    for (int dir = 0; dir < 2; dir++) {
        const bool back = dir == 1;
        float w[S];
        float2 sv[S][KB][4];
        float A[S][KB];
#pragma unroll
        for (int j = 0; j < S; j++) {
            const uint32_t hn = neighbour<MU>(g, c[j], back, w[j]);
            const float2 *sp = a.in[p] + (size_t)hn * SITE;
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                const int cc = q + 4 * kb;
#pragma unroll
                for (int si = 0; si < 4; si++)
                    sv[j][kb][si] = cc < D ? sp[(cc * 4 + si) * kNR + r] : make_float2(0.f, 0.f);
            }
            const float *L =
                a.U + ((size_t)((back ? 1 - p : p) * 4 + MU) * g.Vh_pad + (back ? hn : h[j])) * (D * D);
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                const int k = q + 4 * kb;
                A[j][kb] = (r < D && k < D) ? __builtin_nontemporal_load(L + (back ? k * D + r : r * D + k)) : 0.f;
            }
        }
        const float sg = back ? -eta : eta;
#pragma unroll
        for (int j = 0; j < S; j++) {
            f4 g0r = {0.f, 0.f, 0.f, 0.f}, g0i = g0r, g1r = g0r, g1i = g0r;
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
                float2 h0, h1;
                project_c<MU>(sv[j][kb], sg, h0, h1);
                g0r = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j][kb], h0.x, g0r, 0, 0, 0);
                g0i = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j][kb], h0.y, g0i, 0, 0, 0);
                g1r = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j][kb], h1.x, g1r, 0, 0, 0);
                g1i = __builtin_amdgcn_mfma_f32_16x16x4f32(A[j][kb], h1.y, g1i, 0, 0, 0);
            }
            reconstruct_c<MU>(acc[j], sg, w[j], g0r, g0i, g1r, g1i);
        }
    }
}

// Launch plan (tuned per d_R by bsm_block_autotune):
//   S  = sites per wavefront (1 or 2, interleaved), with a register budget of
//        2 (S = 1) or 1 (S = 2) wavefronts per SIMD;
//   WPB = wavefronts per workgroup (1, 2 or 4), from blockDim.x.
// Workgroup w covers sites [w * WPB * S, (w + 1) * WPB * S); wavefront v owns
// sites base + v + WPB * j, j < S.
template <int D, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S == 1 ? 3 : 1)))
void k_hop_block(Geom g, BlockHopArgs a, int nblk) {
    constexpr size_t SITE = (size_t)D * 4 * kNR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wpb = blockDim.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const uint32_t lb = xcd_chunk_remap(blockIdx.x, gridDim.x, (uint32_t)a.xchunk);
    const int pi = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t base = (lb - pi * nblk) * (uint32_t)(wpb * S);
    const int p = a.p0 + pi;
    uint32_t h[S];
    bool live[S];
#pragma unroll
    for (int j = 0; j < S; j++) {
        const uint32_t hj = base + wave + wpb * j;
        live[j] = hj < (uint32_t)g.Vh;
        h[j] = block_site(g, a.tile, live[j] ? hj : base + wave);   // a dead second site repeats the first (never stored)
    }
    double nrm = 0.0;
    if (live[0]) {
        f4 acc[S][4][2];
        Coords c[S];
#pragma unroll
        for (int j = 0; j < S; j++) {
#pragma unroll
            for (int sp = 0; sp < 4; sp++) acc[j][sp][0] = acc[j][sp][1] = f4{0.f, 0.f, 0.f, 0.f};
            c[j] = decode(g, h[j], p);
        }
        const float eta = a.dagger ? -1.f : 1.f;
        hop_dir_block<0, D, S>(g, a, c, p, h, r, q, eta, acc);
        hop_dir_block<1, D, S>(g, a, c, p, h, r, q, eta, acc);
        hop_dir_block<2, D, S>(g, a, c, p, h, r, q, eta, acc);
        hop_dir_block<3, D, S>(g, a, c, p, h, r, q, eta, acc);
        const float ar = a.a[r], br = a.b[r];
#pragma unroll
        for (int j = 0; j < S; j++) {
            if (!live[j]) continue;
            float2 *o = a.out[p] + (size_t)h[j] * SITE;
            // x first, every load unconditional (rows i >= D read row D - 1
            // and are not stored): a load inside the divergent i < D branch
            // would be waited for there, one memory latency per element
            float2 xv[4][4];
            if (a.use_x) {
                const float2 *x = a.x[p] + (size_t)h[j] * SITE;
#pragma unroll
                for (int v = 0; v < 4; v++)
#pragma unroll
                    for (int sp = 0; sp < 4; sp++) xv[v][sp] = x[(size_t)(min(4 * q + v, D - 1) * 4 + sp) * kNR + r];
            }
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int i = 4 * q + v;
                if (i < D) {
#pragma unroll
                    for (int sp = 0; sp < 4; sp++) {
                        const size_t e = (size_t)(i * 4 + sp) * kNR + r;
                        float re = br * acc[j][sp][0][v], im = br * acc[j][sp][1][v];
                        if (a.use_x) {
                            re = fmaf(ar, xv[v][sp].x, re);
                            im = fmaf(ar, xv[v][sp].y, im);
                        }
                        o[e] = make_float2(re, im);
                        nrm += (double)re * re + (double)im * im;
                    }
                }
            }
        }
    }
    if (a.norm_partials) {
        nrm += __shfl_xor(nrm, 16, 64);
        nrm += __shfl_xor(nrm, 32, 64);
        __shared__ double ws[4][kNR];
        if (lane < kNR) ws[wave][lane] = nrm;
        __syncthreads();
        if (threadIdx.x < kNR) {
            double t = ws[0][threadIdx.x];
            for (int v = 1; v < wpb; v++) t += ws[v][threadIdx.x];
            a.norm_partials[(size_t)lb * kNR + threadIdx.x] = t;
        }
    }
}

BlockTile block_tile_for(const Geom &g) {
    BlockTile b;
    for (int t : {6, 4, 3, 2})
        if (g.L[0] % t == 0) { b.tt = t; break; }
    for (int z : {4, 2})
        if (g.L[3] % z == 0) { b.tz = z; break; }
    for (int y : {4, 2})
        if (g.L[2] % y == 0) { b.ty = y; break; }
    if (b.tt == 0 || b.tz == 0 || b.ty == 0) b = BlockTile{};
    return b;
}

static int block_sites_per_wg(const BlockHopArgs &a) { return a.wpb * a.spw; }

void apply_block_plan(const Geom &g, const BlockPlan &p, BlockHopArgs &a) {
    a.spw = p.spw;
    a.wpb = p.wpb;
    a.tile = p.tiled ? block_tile_for(g) : BlockTile{};
    a.xchunk = p.xchunk;
}

int hop_block_grid(const Geom &g, const BlockHopArgs &a) {
    const int per = block_sites_per_wg(a);
    return (g.Vh + per - 1) / per * a.np;
}

// Only the adjoint representation has real links: d_R = N^2 - 1 in {3, 8, 15}.
template <int D>
struct BlockHopByD {
    static bsm_status run(const Geom &g, const BlockHopArgs &a, hipStream_t st) {
        if constexpr (D == 3 || D == 8 || D == 15) {
            const int grid = hop_block_grid(g, a);
            const dim3 blk(64 * a.wpb);
            if (a.spw == 2) k_hop_block<D, 2><<<grid, blk, 0, st>>>(g, a, grid / a.np);
            else k_hop_block<D, 1><<<grid, blk, 0, st>>>(g, a, grid / a.np);
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        }
        return fail(BSM_ERR_UNSUPPORTED, "block hop: real links exist only for d_R = 3, 8, 15");
    }
};

bsm_status launch_hop_block(const Geom &g, int d, const BlockHopArgs &a, hipStream_t st) {
    if (a.spw != 1 && a.spw != 2) return fail(BSM_ERR_ARG, "block plan: sites per wavefront must be 1 or 2");
    if (a.wpb != 1 && a.wpb != 2 && a.wpb != 4) return fail(BSM_ERR_ARG, "block plan: 1, 2 or 4 wavefronts");
    return dispatch_d<BlockHopByD>(d, g, a, st);
}

bsm_status block_autotune(bsm_ctx ctx, int d, const float *U_block, float2 *scratch_in, float2 *scratch_out,
                          hipStream_t st) {
    const Geom &g = ctx->g;
    BSM_HIP(hipMemsetAsync(scratch_in, 0, block_parity_bytes(g, d), st));
    hipEvent_t e0, e1;
    BSM_HIP(hipEventCreate(&e0));
    BSM_HIP(hipEventCreate(&e1));
    BlockPlan best;
    best.us = 0.f;
    bsm_status status = BSM_OK;
    const BlockTile tile = block_tile_for(g);
    for (int tiled = 0; tiled <= (tile.tt ? 1 : 0) && status == BSM_OK; tiled++)
    for (int xchunk : {0, 1, 16})
    for (int spw = 1; spw <= 2 && status == BSM_OK; spw++) {
        for (int wpb : {1, 2, 4}) {
            BlockHopArgs a{};
            a.U = U_block;
            a.p0 = 0;
            a.np = 1;
            a.in[0] = scratch_in;
            a.out[0] = scratch_out;
            for (int r = 0; r < kNR; r++) { a.a[r] = 0.f; a.b[r] = 1.f; }
            a.spw = spw;
            a.wpb = wpb;
            a.xchunk = xchunk;
            if (tiled) a.tile = tile;
            const int reps = 5;
            if ((status = launch_hop_block(g, d, a, st)) != BSM_OK) break;   // warm-up
            if (hipEventRecord(e0, st) != hipSuccess) { status = fail(BSM_ERR_HIP, "event"); break; }
            for (int k = 0; k < reps && status == BSM_OK; k++) status = launch_hop_block(g, d, a, st);
            if (status != BSM_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                status = fail(BSM_ERR_HIP, "block autotune timing");
                break;
            }
            const float us = ms * 1000.f / reps;
            if (best.us == 0.f || us < best.us) {
                best.spw = spw;
                best.wpb = wpb;
                best.tiled = tiled;
                best.xchunk = xchunk;
                best.us = us;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == BSM_OK) ctx->block_plans[d][0] = best;
    return status;
}

// --------------------------------------------------------------- layouts
// 32 sites per workgroup: the link elements are read plane by plane (lanes
// on consecutive sites) into LDS as [site][i * d + j], which is already the
// block layout of those 32 sites, then written out contiguously (one thread
// per site wrote 225 floats 900 bytes apart from its neighbour's)
constexpr int kLinkTile = 32;

template <int LP>
__global__ __launch_bounds__(256) void k_gauge_to_block(Geom g, int d, const char *src, float *dst) {
    __shared__ float t[kLinkTile * 225];
    const uint32_t h0 = blockIdx.x * kLinkTile;
    const int qm = blockIdx.y;   // parity * 4 + mu
    const int dd = d * d, ldt = dd | 1;   // odd row stride: no LDS bank conflicts
    const int ns = min(kLinkTile, (int)((uint32_t)g.Vh_pad - h0));
    const char *blk = src + (size_t)qm * link_block_bytes(LP, true, d, g.Vh_pad);
    for (int idx = threadIdx.x; idx < kLinkTile * dd; idx += 256) {
        const int e = idx / kLinkTile, s = idx - e * kLinkTile;
        if (s < ns) t[s * ldt + e] = (float)load_link<LP, true, float>(blk, g.Vh_pad, e, h0 + s).re;
    }
    __syncthreads();
    float *o = dst + ((size_t)qm * g.Vh_pad + h0) * dd;
    for (int idx = threadIdx.x; idx < ns * dd; idx += 256) o[idx] = t[(idx / dd) * ldt + idx % dd];
}

bsm_status launch_gauge_to_block(const Geom &g, int d, int link_prec, const void *U_rep, float *U_block,
                                 hipStream_t st) {
    if (d > 15) return fail(BSM_ERR_ARG, "block links: d_R above 15");
    dim3 grid((g.Vh_pad + kLinkTile - 1) / kLinkTile, 8);
    switch (link_prec) {
    case BSM_F64: k_gauge_to_block<BSM_F64><<<grid, 256, 0, st>>>(g, d, (const char *)U_rep, U_block); break;
    case BSM_F32: k_gauge_to_block<BSM_F32><<<grid, 256, 0, st>>>(g, d, (const char *)U_rep, U_block); break;
    default: return fail(BSM_ERR_UNSUPPORTED, "block links from F16 links");
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// one thread per (site, colour-spin component); loops over the 16 RHS slots
__global__ __launch_bounds__(256) void k_pack_block(Geom g, int d, int n_rhs, const double2 *canon,
                                                    float2 *block, int unpack) {
    const uint32_t h = blockIdx.x * 256 + threadIdx.x;
    const int p = blockIdx.y;
    const int cs = blockIdx.z;              // c * 4 + s
    if (h >= (uint32_t)g.Vh_pad) return;
    const int c = cs >> 2, s = cs & 3;
    float2 *o = block + (size_t)p * g.Vh_pad * d * 4 * kNR + ((size_t)h * d * 4 + cs) * kNR;
    const bool real_site = h < (uint32_t)g.Vh;
    int64_t lex = 0;
    if (real_site) {
        Coords co = decode(g, h, p);
        lex = (int64_t)co.row * g.L[1] + co.x;
    }
    const int64_t V = 2 * (int64_t)g.Vh;
    for (int r = 0; r < kNR; r++) {
        const bool use = real_site && r < n_rhs;
        double2 *cp = (double2 *)canon + ((r * V + lex) * 4 + s) * d + c;
        if (!unpack) {
            o[r] = use ? make_float2((float)cp->x, (float)cp->y) : make_float2(0.f, 0.f);
        } else if (use) {
            *cp = make_double2(o[r].x, o[r].y);
        }
    }
}

bsm_status launch_pack_block(const Geom &g, int d, int n_rhs, const void *canon, void *block, bool unpack,
                             hipStream_t st) {
    dim3 grid((g.Vh_pad + 255) / 256, 2, d * 4);
    k_pack_block<<<grid, 256, 0, st>>>(g, d, n_rhs, (const double2 *)canon, (float2 *)block, unpack ? 1 : 0);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// element e of one parity block: r = e % 16, (h, c, s) from e / 16
// Block <-> standard layout through an LDS tile: a workgroup owns one
// (colour, spin) plane of 64 consecutive sites for all 16 RHS, reads one side
// with consecutive lanes on consecutive addresses (16 RHS of a site on the
// block side, 64 sites of one RHS on the standard side), transposes in LDS
// and writes the other side the same way.
//   OP 0: block = std (RHS >= n_rhs zeroed, other unselected RHS untouched)
//   OP 1: std += block  (selected RHS)
//   OP 2: std = block   (selected RHS, sites < Vh only)
__device__ inline float2 blk_from(double2 x, float2) { return make_float2((float)x.x, (float)x.y); }
__device__ inline double2 blk_from(double2 x, double2) { return x; }
__device__ inline double2 blk_to64(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ inline double2 blk_to64(double2 v) { return v; }

template <class BT, int OP>
__global__ __launch_bounds__(256) void k_block_std(Geom g, int d, int n_rhs, unsigned sel, char *std64,
                                                   size_t std_stride, size_t std_off, BT *block) {
    __shared__ BT tile[kNR][65];
    const uint32_t nth = ((uint32_t)g.Vh_pad + 63) / 64;
    const uint32_t hb = blockIdx.x % nth, cs = blockIdx.x / nth;
    const int c = (int)(cs / 4), sp = (int)(cs % 4);
    const uint32_t h0 = hb * 64;
    const int t = threadIdx.x;
    const size_t plane = (size_t)(sp * d + c) * g.Vh_pad;
    auto bidx = [&](int r, uint32_t h) { return (((size_t)h * d + c) * 4 + sp) * kNR + r; };
    auto sptr = [&](int r, uint32_t h) { return (double2 *)(std64 + (size_t)r * std_stride + std_off) + plane + h; };
    if constexpr (OP == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int j = t + 256 * k, hl = j & 63, r = j >> 6;
            const uint32_t h = h0 + hl;
            BT v{};
            if (h < (uint32_t)g.Vh_pad && r < n_rhs) v = blk_from(*sptr(r, h), BT{});
            tile[r][hl] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = t + 256 * k, r = i & 15, hl = i >> 4;
            const uint32_t h = h0 + hl;
            if (h >= (uint32_t)g.Vh_pad) continue;
            if (r < n_rhs && !((sel >> r) & 1u)) continue;
            block[bidx(r, h)] = tile[r][hl];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = t + 256 * k, r = i & 15, hl = i >> 4;
            const uint32_t h = h0 + hl;
            tile[r][hl] = h < (uint32_t)g.Vh_pad ? block[bidx(r, h)] : BT{};
        }
        __syncthreads();
        const uint32_t hmax = OP == 2 ? (uint32_t)g.Vh : (uint32_t)g.Vh_pad;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int j = t + 256 * k, hl = j & 63, r = j >> 6;
            const uint32_t h = h0 + hl;
            if (h >= hmax || r >= n_rhs || !((sel >> r) & 1u)) continue;
            double2 *sv = sptr(r, h);
            const double2 v = blk_to64(tile[r][hl]);
            if constexpr (OP == 1) {
                double2 o = *sv;
                o.x += v.x;
                o.y += v.y;
                *sv = o;
            } else {
                *sv = v;
            }
        }
    }
}

template <class BT, int OP>
static bsm_status run_block_std(const Geom &g, int d, int n_rhs, unsigned sel, char *std64, size_t std_stride,
                                size_t std_off, BT *block, hipStream_t st) {
    const size_t nwg = (size_t)((g.Vh_pad + 63) / 64) * d * 4;
    k_block_std<BT, OP><<<(unsigned)nwg, 256, 0, st>>>(g, d, n_rhs, sel, std64, std_stride, std_off, block);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status launch_std_block(const Geom &g, int d, int n_rhs, unsigned sel, char *std64, size_t std_stride,
                            size_t std_off, float2 *block, int mode, hipStream_t st) {
    if (mode == 0) return run_block_std<float2, 0>(g, d, n_rhs, sel, std64, std_stride, std_off, block, st);
    return run_block_std<float2, 1>(g, d, n_rhs, sel, std64, std_stride, std_off, block, st);
}

bsm_status launch_block64_std(const Geom &g, int d, int n_rhs, unsigned sel, char *std64, size_t std_stride,
                              size_t std_off, double2 *block, int mode, hipStream_t st) {
    if (mode == 0) return run_block_std<double2, 0>(g, d, n_rhs, sel, std64, std_stride, std_off, block, st);
    return run_block_std<double2, 2>(g, d, n_rhs, sel, std64, std_stride, std_off, block, st);
}

// ------------------------------------------------------------ vector ops
constexpr int kBlockBlasMax = 16384;

int block_blas_grid(const Geom &g, int d, int nblk) {
    const size_t n = (size_t)nblk * g.Vh_pad * d * 4 * kNR;
    size_t nb = (n + 255) / 256;
    return (int)(nb < kBlockBlasMax ? nb : kBlockBlasMax);
}

// per-RHS sum over the workgroup: lanes with equal tid % 16 share an RHS
__device__ inline void block_rhs_sum(double v, double *partials) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    __shared__ double ws[4][kNR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < kNR) ws[wave][lane] = v;
    __syncthreads();
    if (threadIdx.x < kNR)
        partials[(size_t)blockIdx.x * kNR + threadIdx.x] =
            (ws[0][threadIdx.x] + ws[1][threadIdx.x]) + (ws[2][threadIdx.x] + ws[3][threadIdx.x]);
}

// Element e of a block field of one or two parity blocks (per elements
// each) lies on a live site when its offset in its block is below live;
// padding sites are skipped (no operator writes them).
__device__ inline bool block_live(size_t e, size_t per, size_t live) {
    return (e >= per ? e - per : e) < live;
}

__global__ __launch_bounds__(256) void k_block_update(size_t n, size_t per, size_t live, float2 *x, const float2 *p,
                                                      float2 *r, const float2 *q, const double *alpha,
                                                      double *partials) {
    const double al = alpha[threadIdx.x % kNR];
    const float a = (float)al;
    double nrm = 0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        if (!block_live(e, per, live)) continue;
        float2 xv = x[e], pv = p[e], rv = r[e], qv = q[e];
        xv.x = fmaf(a, pv.x, xv.x); xv.y = fmaf(a, pv.y, xv.y);
        rv.x = fmaf(-a, qv.x, rv.x); rv.y = fmaf(-a, qv.y, rv.y);
        x[e] = xv;
        r[e] = rv;
        nrm += (double)rv.x * rv.x + (double)rv.y * rv.y;
    }
    block_rhs_sum(nrm, partials);
}

__global__ __launch_bounds__(256) void k_block_xpay(size_t n, size_t per, size_t live, float2 *p, const float2 *r,
                                                    const double *beta) {
    const float b = (float)beta[threadIdx.x % kNR];
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        if (!block_live(e, per, live)) continue;
        float2 pv = p[e], rv = r[e];
        p[e] = make_float2(fmaf(b, pv.x, rv.x), fmaf(b, pv.y, rv.y));
    }
}

__global__ __launch_bounds__(256) void k_block_norm(size_t n, size_t per, size_t live, const float2 *v,
                                                    double *partials) {
    double nrm = 0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        if (!block_live(e, per, live)) continue;
        const float2 t = v[e];
        nrm += (double)t.x * t.x + (double)t.y * t.y;
    }
    block_rhs_sum(nrm, partials);
}

static size_t block_elems(const Geom &g, int d, int nblk) { return (size_t)nblk * g.Vh_pad * d * 4 * kNR; }
static size_t block_per(const Geom &g, int d) { return (size_t)g.Vh_pad * d * 4 * kNR; }
static size_t block_live_elems(const Geom &g, int d) { return (size_t)g.Vh * d * 4 * kNR; }

bsm_status block_update(const Geom &g, int d, int nblk, float2 *x, const float2 *p, float2 *r,
                        const float2 *q, const double *alpha, double *partials, hipStream_t st) {
    if (nblk < 1 || nblk > 2) return fail(BSM_ERR_ARG, "block fields hold one or two parity blocks");
    k_block_update<<<block_blas_grid(g, d, nblk), 256, 0, st>>>(block_elems(g, d, nblk), block_per(g, d),
                                                                 block_live_elems(g, d), x, p, r, q, alpha,
                                                                 partials);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status block_xpay(const Geom &g, int d, int nblk, float2 *p, const float2 *r, const double *beta,
                      hipStream_t st) {
    if (nblk < 1 || nblk > 2) return fail(BSM_ERR_ARG, "block fields hold one or two parity blocks");
    k_block_xpay<<<block_blas_grid(g, d, nblk), 256, 0, st>>>(block_elems(g, d, nblk), block_per(g, d),
                                                               block_live_elems(g, d), p, r, beta);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status block_norm(const Geom &g, int d, int nblk, const float2 *v, double *partials, hipStream_t st) {
    if (nblk < 1 || nblk > 2) return fail(BSM_ERR_ARG, "block fields hold one or two parity blocks");
    k_block_norm<<<block_blas_grid(g, d, nblk), 256, 0, st>>>(block_elems(g, d, nblk), block_per(g, d),
                                                               block_live_elems(g, d), v, partials);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// one workgroup: thread t sums the partials of RHS t % 16 over workgroups
// t / 16, t / 16 + 16, ... (fixed order), then the 16 groups are combined
__global__ __launch_bounds__(256) void k_block_scalars(const double *partials, int nparts, double *scal,
                                                       const int *mask, int op, int slot) {
    const int r = threadIdx.x % kNR, grp = threadIdx.x / kNR;
    double s = 0;
    for (int i = grp; i < nparts; i += 16) s += partials[(size_t)i * kNR + r];
    __shared__ double ws[16][kNR];
    ws[grp][r] = s;
    __syncthreads();
    if (threadIdx.x >= kNR) return;
    double tot = 0;
    for (int k = 0; k < 16; k++) tot += ws[k][r];
    const bool on = mask[r] != 0;
    double *RR = scal + B_RR * kNR, *PAP = scal + B_PAP * kNR, *AL = scal + B_ALPHA * kNR,
           *BE = scal + B_BETA * kNR, *H = scal + (B_HIST + slot) * kNR;
    if (op == 0) {
        PAP[r] = tot;
        const double al = RR[r] / tot;
        AL[r] = (on && tot > 0 && isfinite(al)) ? al : 0.0;
    } else if (op == 1) {
        const double rr = RR[r];
        const double be = tot / rr;
        BE[r] = (on && rr > 0 && isfinite(be)) ? be : 0.0;
        if (on) RR[r] = tot;
        H[r] = tot;
    } else {
        RR[r] = tot;
        H[r] = tot;
    }
}

// first stage of a long per-RHS sum: workgroup b adds the contiguous range
// [b chunk, (b + 1) chunk) of the partials (fixed order) into out[b][r]
__global__ __launch_bounds__(256) void k_block_presum(const double *partials, int nparts, int chunk, double *out) {
    const int r = threadIdx.x % kNR, grp = threadIdx.x / kNR;
    const int i0 = blockIdx.x * chunk, i1 = min(nparts, i0 + chunk);
    double s = 0;
    for (int i = i0 + grp; i < i1; i += 16) s += partials[(size_t)i * kNR + r];
    __shared__ double ws[16][kNR];
    ws[grp][r] = s;
    __syncthreads();
    if (threadIdx.x >= kNR) return;
    double tot = 0;
    for (int k = 0; k < 16; k++) tot += ws[k][r];
    out[(size_t)blockIdx.x * kNR + r] = tot;
}

bsm_status block_scalars(const double *partials, int nparts, double *scal, const int *mask, int op,
                         int hist_slot, double *presum, hipStream_t st) {
    if (nparts > 4 * kBlockPresum && presum) {
        const int chunk = (nparts + kBlockPresum - 1) / kBlockPresum;
        const int nb = (nparts + chunk - 1) / chunk;
        k_block_presum<<<nb, 256, 0, st>>>(partials, nparts, chunk, presum);
        k_block_scalars<<<1, 256, 0, st>>>(presum, nb, scal, mask, op, hist_slot);
    } else {
        k_block_scalars<<<1, 256, 0, st>>>(partials, nparts, scal, mask, op, hist_slot);
    }
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
