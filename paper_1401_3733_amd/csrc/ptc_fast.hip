// The two-layer network applied as one operator.
//
// Both PTC layers are linear and the spin matrices commute with the colour
// transports, so for a 1 -> C -> 1 network
//   M v = sum_p T_p G_p,   G_p(y) = sum_q C_pq (T_q v)(y),
//   C_pq = sum_j W2_p^{0j} W1_q^{j0}          (4 x 4 complex, 81 of them)
// i.e. one transport sweep, a 36 x 36 complex mixing that is the same at
// every site and colour, and a second transport sweep; the C channel fields
// are never formed.
//
// Precision: the transports are FP32 (links FP32, or FP16 where the caller
// passes FP16 links: a further relative 2^-11 on each link element).  The mixing runs on FP16 matrix cores
// with FP32 accumulation: the transported fields are divided by a bound on
// their largest |component| (per site and group of paths) before rounding to
// FP16, C by its largest entry; the nine mixed fields are stored in FP16 with
// a per-site scale.  The scales only keep the values inside the FP16 range
// (its relative precision does not depend on them).  The result agrees with
// the FP32 layers to a relative O(1e-3), which is what a preconditioner of a
// flexible Krylov method needs.
#include "dispatch.h"
#include "ptc.h"
#include "ptc_dev.h"

namespace bsm {

typedef _Float16 h4v __attribute__((ext_vector_type(4)));

constexpr int kFastMaxD = 3;    // colour dimensions of the matrix-core mixing
constexpr int kFastRows = 72;   // (path, spin, re/im) of the real form
constexpr int kFastTiles = 5;   // 16-row tiles covering 72 rows (and 16-deep K steps covering 72)
constexpr int kFastSites = 128; // sites per block of the mixing kernel (4 threads each)
constexpr int kFastSlotsKq = 20;   // groups of 4 K values incl. the zero slot
__host__ __device__ inline int fast_slot_path(int slot);

// C (36 x 36 complex, FP64 sums) -> FP16 real form / cs in the lane order of
// the 16x16x16 matrix-core fragments: frag[(mt * 5 + ks) * 64 + lane] holds
// A[16 mt + lane % 16][16 ks + 4 (lane / 16) + 0..3] with the K index in the
// slot order of k_net_mix16; cs = max |Re|, |Im|.  One workgroup.
__global__ __launch_bounds__(256) void k_net_collapse(const float2 *W1, const float2 *W2, int C, h4v *frag,
                                                      float *cs_out) {
    __shared__ float2 Cm[36 * 36];
    __shared__ float red[256];
    const int tid = threadIdx.x;
    float mx = 0.f;
    for (int e = tid; e < 36 * 36; e += 256) {
        const int row = e / 36, col = e % 36;
        const int p = row / 4, a = row % 4, q = col / 4, b = col % 4;
        double re = 0, im = 0;
        for (int j = 0; j < C; j++)
            for (int c = 0; c < 4; c++) {
                const float2 w2 = W2[((size_t)j * 9 + p) * 16 + a * 4 + c];
                const float2 w1 = W1[((size_t)j * 9 + q) * 16 + c * 4 + b];
                re += (double)w2.x * w1.x - (double)w2.y * w1.y;
                im += (double)w2.x * w1.y + (double)w2.y * w1.x;
            }
        Cm[e] = make_float2((float)re, (float)im);
        mx = fmaxf(mx, fmaxf(fabsf((float)re), fabsf((float)im)));
    }
    red[tid] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
        __syncthreads();
    }
    const float cs = red[0] > 0.f ? red[0] : 1.f;
    const float inv = 1.f / cs;
    for (int e = tid; e < kFastTiles * kFastTiles * 64; e += 256) {
        const int lane = e % 64, mt = e / 64 / kFastTiles, ks = e / 64 % kFastTiles;
        const int m = 16 * mt + lane % 16;
        float v[4];
        for (int j = 0; j < 4; j++) {
            // reordered K index -> (path, spin, re/im) of the transported fields
            const int kq = 4 * ks + lane / 16, path = fast_slot_path(kq / 2);
            const int k = 8 * path + 4 * (kq % 2) + j;
            v[j] = 0.f;
            if (m < kFastRows && path >= 0) {
                const int ro = m & 1, ri = k & 1;
                const float2 z = Cm[(m / 2) * 36 + k / 2];
                v[j] = (ro == ri ? z.x : (ro == 0 ? -z.y : z.y)) * inv;
            }
        }
        frag[e] = h4v{(_Float16)v[0], (_Float16)v[1], (_Float16)v[2], (_Float16)v[3]};
    }
    if (tid == 0) *cs_out = cs;
}

// mixed fields: G[((p * 2 + parity) * 2D + u) * Vh_pad + h] (u = spin pair *
// D + colour; one half4 = the two spins re/im) and S[parity * Vh_pad + h]
template <int D>
__device__ inline size_t g16_index(const Geom &g, int p, int par, int u, uint32_t h) {
    return ((size_t)(p * 2 + par) * (2 * D) + u) * g.Vh_pad + h;
}

template <int D>
__device__ inline void load_g16(const NetFastArgs &a, const Geom &g, int p, int par, uint32_t h,
                                cx<float> (&v)[4 * D]) {
    const float s = a.S[(size_t)par * g.Vh_pad + h];
    const h4v *G = (const h4v *)a.G;
#pragma unroll
    for (int bp = 0; bp < 2; bp++)
#pragma unroll
        for (int cc = 0; cc < D; cc++) {
            const h4v x = __builtin_nontemporal_load(&G[g16_index<D>(g, p, par, bp * D + cc, h)]);
            v[(2 * bp) * D + cc] = mk<float>((float)x[0] * s, (float)x[1] * s);
            v[(2 * bp + 1) * D + cc] = mk<float>((float)x[2] * s, (float)x[3] * s);
        }
}

// t = w U s (forward path) or w U^dag s (backward path); links in LP
template <int D, int LP>
__device__ inline void link_apply(const Geom &g, const PathSite &ps, const cx<float> (&s)[4 * D],
                                  cx<float> (&t)[4 * D]) {
#pragma unroll
    for (int k = 0; k < 4 * D; k++) t[k] = mk<float>(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            const cx<float> u = load_link<LP, false, float>(ps.blk, g.Vh_pad, i * D + j, ps.hl);
#pragma unroll
            for (int a = 0; a < 4; a++) {
                if (!ps.back) t[a * D + i] = cfma(u, s[a * D + j], t[a * D + i]);
                else t[a * D + j] = cfma_conj(u, s[a * D + i], t[a * D + j]);
            }
        }
#pragma unroll
    for (int k = 0; k < 4 * D; k++) t[k] = ps.w * t[k];
}

// workgroup barrier ordering LDS only: the wavefront's outstanding global
// stores (the mixed fields of the previous block) are not waited for
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int D>
__device__ inline float maxabs(const cx<float> (&t)[4 * D], float m) {
#pragma unroll
    for (int k = 0; k < 4 * D; k++) m = fmaxf(m, fmaxf(fabsf(t[k].re), fabsf(t[k].im)));
    return m;
}

// K order of the matrix-core operand: slots of 8 K values (one path's four
// spins, re/im) in the order p0 p4 p8 - p1 p5 p2 p6 p3 p7 ('-' is zero), so
// that each 16-deep K step belongs to one thread of a site's four: steps 0
// and 1 to thread 0 (paths 0, 4, 8), step 1 + g to thread g (paths g, g + 4).
__host__ __device__ inline int fast_slot_path(int slot) {
    constexpr int sp[10] = {0, 4, 8, -1, 1, 5, 2, 6, 3, 7};
    return sp[slot];
}
__device__ inline int fast_path_slot(int p) {
    constexpr int ps[9] = {0, 4, 6, 8, 1, 5, 7, 9, 2};
    return ps[p];
}

// write t * inv as FP16 into the B tile: Bh[(colour * 20 + 2 slot + spin pair) * sites + site]
template <int D>
__device__ inline void stage_path(h4v *Bh, int slot, int s, float inv, const cx<float> (&t)[4 * D]) {
#pragma unroll
    for (int bp = 0; bp < 2; bp++)
#pragma unroll
        for (int cc = 0; cc < D; cc++) {
            const cx<float> x0 = t[(2 * bp) * D + cc], x1 = t[(2 * bp + 1) * D + cc];
            Bh[(cc * kFastSlotsKq + 2 * slot + bp) * kFastSites + s] =
                h4v{(_Float16)(x0.re * inv), (_Float16)(x0.im * inv), (_Float16)(x1.re * inv), (_Float16)(x1.im * inv)};
        }
}

// source site of path p at (px, h): the site itself or its neighbour
template <int D>
__device__ inline float source_maxabs(const Geom &g, const char *v, size_t pblk, int px, uint32_t h,
                                      const PathSite &ps, int p, float m) {
    cx<float> s[4 * D];
    if (p == 0) load_spinor<BSM_F32, D, float>(v + px * pblk, g.Vh_pad, h, s);
    else load_spinor<BSM_F32, D, float>(v + (1 - px) * pblk, g.Vh_pad, ps.hn, s);
    return maxabs<D>(s, m);
}

template <int D, int LP>
__device__ inline void stage_transport(const Geom &g, const char *v, size_t pblk, int px, uint32_t h,
                                       const PathSite &ps, int p, float inv, h4v *Bh, int site) {
    cx<float> s[4 * D];
    if (p == 0) {
        load_spinor<BSM_F32, D, float>(v + px * pblk, g.Vh_pad, h, s);
        stage_path<D>(Bh, fast_path_slot(0), site, inv, s);
    } else {
        load_spinor<BSM_F32, D, float>(v + (1 - px) * pblk, g.Vh_pad, ps.hn, s);
        cx<float> t[4 * D];
        link_apply<D, LP>(g, ps, s, t);
        stage_path<D>(Bh, fast_path_slot(p), site, inv, t);
    }
}

// G'_p(y) = sum_q (C / cs) (T_q v)(y) / S(y) for blocks of 128 sites of one
// parity; a workgroup of 512 threads walks a contiguous range of blocks with
// the matrix fragments in LDS.  Phase 1: thread (site, group g) bounds the
// transports of its paths by sqrt(2 D) max |component| of their sources
// (|U v|_i <= |v|_2 for unitary U), then forms them in FP32, scales them by
// that bound and writes them to LDS in FP16.  Phase 2: wavefront w takes
// sites 16w..16w+15 of the block: each 16-deep K step is one thread's, so its product is
// rescaled by that thread's bound before it is summed; S(y) is the largest
// of the site's four bounds and G' = G / S is stored in FP16 (|G'| <= 72).
template <int D, int LP>
__global__ __launch_bounds__(4 * kFastSites) void k_net_mix16(Geom g, NetFastArgs a, int nblk, int per_wg) {
    __shared__ h4v Bh[D * kFastSlotsKq * kFastSites];
    __shared__ h4v Afs[kFastTiles * kFastTiles * 64];
    __shared__ float sb[4 * kFastSites];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, sl = lane & 15;
    const int pg = tid / kFastSites, site = tid % kFastSites;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(LP, false, D, g.Vh_pad);
    const char *U = (const char *)a.U, *v = (const char *)a.in;
    for (int e = tid; e < kFastTiles * kFastTiles * 64; e += 4 * kFastSites) Afs[e] = ((const h4v *)a.Afrag)[e];
    // the zero slot (thread group 0 owns it)
    if (pg == 0)
#pragma unroll
        for (int cc = 0; cc < D; cc++) {
            Bh[(cc * kFastSlotsKq + 6) * kFastSites + site] = h4v{0, 0, 0, 0};
            Bh[(cc * kFastSlotsKq + 7) * kFastSites + site] = h4v{0, 0, 0, 0};
        }
    const uint32_t wg = xcd_remap(blockIdx.x, gridDim.x);
    const int b0 = wg * per_wg, b1 = min(b0 + per_wg, 2 * nblk);
    h4v *G = (h4v *)a.G;
    for (int blk = b0; blk < b1; blk++) {
        const int px = blk >= nblk ? 1 : 0;
        const uint32_t hb = (blk - px * nblk) * kFastSites;
        {
            const uint32_t h = hb + site;
            const bool live = h < (uint32_t)g.Vh;
            const int pA = pg, pB = pg + 4;
            float bound = 0.f;
            PathSite sA{}, sB{}, sC{};
            if (live) {
                const Coords c = decode(g, h, px);
                if (pA > 0) sA = path_site(g, U, lblk, px, h, c, pA);
                sB = path_site(g, U, lblk, px, h, c, pB);
                if (pg == 0) sC = path_site(g, U, lblk, px, h, c, 8);
                float m = source_maxabs<D>(g, v, pblk, px, h, sA, pA, 0.f);
                m = source_maxabs<D>(g, v, pblk, px, h, sB, pB, m);
                if (pg == 0) m = source_maxabs<D>(g, v, pblk, px, h, sC, 8, m);
                bound = m * sqrtf(2.f * D);
            }
            const float inv = bound > 0.f ? 1.f / bound : 0.f;
            if (live) {
                stage_transport<D, LP>(g, v, pblk, px, h, sA, pA, inv, Bh, site);
                stage_transport<D, LP>(g, v, pblk, px, h, sB, pB, inv, Bh, site);
                if (pg == 0) stage_transport<D, LP>(g, v, pblk, px, h, sC, 8, inv, Bh, site);
            } else {
                cx<float> z[4 * D];
#pragma unroll
                for (int e = 0; e < 4 * D; e++) z[e] = mk<float>(0.f, 0.f);
                stage_path<D>(Bh, fast_path_slot(pA), site, 0.f, z);
                stage_path<D>(Bh, fast_path_slot(pB), site, 0.f, z);
                if (pg == 0) stage_path<D>(Bh, fast_path_slot(8), site, 0.f, z);
            }
            sb[pg * kFastSites + site] = bound;
        }
        lds_barrier();
        const int col = 16 * w + sl;
        const uint32_t h = hb + col;
        const bool live = h < (uint32_t)g.Vh;
        const float S = fmaxf(fmaxf(sb[col], sb[kFastSites + col]), fmaxf(sb[2 * kFastSites + col], sb[3 * kFastSites + col]));
        const float invS = S > 0.f ? 1.f / S : 0.f;
        if (live && q == 0) a.S[(size_t)px * g.Vh_pad + h] = S;
#pragma unroll
        for (int cc = 0; cc < D; cc++) {
            f4v acc[kFastTiles];
#pragma unroll
            for (int mt = 0; mt < kFastTiles; mt++) acc[mt] = f4v{0.f, 0.f, 0.f, 0.f};
            // one K step at a time (its thread's bound rescales the product),
            // fragments read from LDS, so few registers stay live
#pragma unroll 1
            for (int ks = 0; ks < kFastTiles; ks++) {
                const h4v b = Bh[(cc * kFastSlotsKq + 4 * ks + q) * kFastSites + col];
                const float f = sb[(ks < 2 ? 0 : ks - 1) * kFastSites + col] * invS;
#pragma unroll
                for (int mt = 0; mt < kFastTiles; mt++) {
                    const f4v t = __builtin_amdgcn_mfma_f32_16x16x16f16(Afs[(mt * kFastTiles + ks) * 64 + lane], b,
                                                                         f4v{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                    acc[mt] += f * t;
                }
            }
            if (!live) continue;
            // rows 16 mt + 4 q + v: path 2 mt + q / 2, spins 2 (q % 2) and 2 (q % 2) + 1
#pragma unroll
            for (int mt = 0; mt < kFastTiles; mt++) {
                const int p = 2 * mt + q / 2;
                if (p >= 9) continue;
                // streamed: each value is read once, by the transport sum
                __builtin_nontemporal_store(
                    h4v{(_Float16)acc[mt][0], (_Float16)acc[mt][1], (_Float16)acc[mt][2], (_Float16)acc[mt][3]},
                    &G[g16_index<D>(g, p, px, (q & 1) * D + cc, h)]);
            }
        }
        lds_barrier();
    }
}

// z(x) = cs * (S G'_0(x) + sum_{p >= 1} T_p (S G'_p)(x)) with four threads
// per site (thread group q takes the paths q + 1 and q + 5, group 0 also the
// stay path) and the partial sums added in LDS in a fixed order: four times
// the loads in flight of one thread per site (measured 9 % faster on
// 16^3x32, 2 % on 32^3x64)
template <int D, int LP>
__global__ __launch_bounds__(256) void k_net_tsum16(Geom g, NetFastArgs a, int nblk) {
    __shared__ float2 part[4][4 * D][64];
    const int s = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t h = (lb - px * nblk) * 64 + s;
    const bool live = h < (uint32_t)g.Vh;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(LP, false, D, g.Vh_pad);
    cx<float> acc[4 * D];
#pragma unroll
    for (int e = 0; e < 4 * D; e++) acc[e] = mk<float>(0.f, 0.f);
    if (live) {
        const Coords c = decode(g, h, px);
        if (grp == 0) load_g16<D>(a, g, 0, px, h, acc);
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int p = grp + 1 + 4 * k;
            const PathSite ps = path_site(g, (const char *)a.U, lblk, px, h, c, p);
            cx<float> v[4 * D], t[4 * D];
            load_g16<D>(a, g, p, 1 - px, ps.hn, v);
            link_apply<D, LP>(g, ps, v, t);
#pragma unroll
            for (int e = 0; e < 4 * D; e++) acc[e] = acc[e] + t[e];
        }
    }
#pragma unroll
    for (int e = 0; e < 4 * D; e++) part[grp][e][s] = make_float2(acc[e].re, acc[e].im);
    __syncthreads();
    if (grp != 0 || !live) return;
    const float cs = *a.cs;
#pragma unroll
    for (int e = 0; e < 4 * D; e++) {
        const float2 x0 = part[0][e][s], x1 = part[1][e][s], x2 = part[2][e][s], x3 = part[3][e][s];
        acc[e] = mk<float>(cs * ((x0.x + x1.x) + (x2.x + x3.x)), cs * ((x0.y + x1.y) + (x2.y + x3.y)));
    }
    store_spinor<BSM_F32, D, float>((char *)a.out + px * pblk, g.Vh_pad, h, acc);
}

size_t net_fast_bytes(const Geom &g, int d) {
    const size_t G = (size_t)9 * 2 * 2 * d * g.Vh_pad * sizeof(h4v);
    const size_t S = (size_t)2 * g.Vh_pad * sizeof(float);
    const size_t F = (size_t)kFastTiles * kFastTiles * 64 * sizeof(h4v);
    return (G + 255) / 256 * 256 + (S + 255) / 256 * 256 + F + 256;
}

void net_fast_carve(const Geom &g, int d, void *scratch, NetFastArgs &a) {
    char *w = (char *)scratch;
    const size_t G = (size_t)9 * 2 * 2 * d * g.Vh_pad * sizeof(h4v);
    const size_t S = (size_t)2 * g.Vh_pad * sizeof(float);
    const size_t F = (size_t)kFastTiles * kFastTiles * 64 * sizeof(h4v);
    a.G = w;
    w += (G + 255) / 256 * 256;
    a.S = (float *)w;
    w += (S + 255) / 256 * 256;
    a.Afrag = w;
    w += F;
    a.cs = (float *)w;
}

bool net_fast_supported(int d) { return d >= 2 && d <= kFastMaxD; }

bsm_status launch_net_collapse(const void *net, int C, const NetFastArgs &a, hipStream_t st) {
    const float2 *W1 = (const float2 *)net;
    const float2 *W2 = W1 + (size_t)C * 9 * 16;
    k_net_collapse<<<1, 256, 0, st>>>(W1, W2, C, (h4v *)a.Afrag, (float *)a.cs);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

template <int D>
struct NetFastByD {
    static bsm_status run(const Geom &g, const NetFastArgs &a, hipStream_t st) {
        if constexpr (D > kFastMaxD) {
            return fail(BSM_ERR_UNSUPPORTED, "the collapsed network runs for d_R <= 3");
        } else {
            const int nbm = (g.Vh + kFastSites - 1) / kFastSites;
            // up to 4096 workgroups (two fit a CU), each over a contiguous range of blocks
            const int per_wg = std::max(1, (2 * nbm + 4095) / 4096);
            const int grid = (2 * nbm + per_wg - 1) / per_wg;
            const int nb64 = (g.Vh + 63) / 64;
            if (a.link_prec == BSM_F16S) {
                k_net_mix16<D, BSM_F16S><<<grid, 4 * kFastSites, 0, st>>>(g, a, nbm, per_wg);
                k_net_tsum16<D, BSM_F16S><<<2 * nb64, 256, 0, st>>>(g, a, nb64);
            } else {
                k_net_mix16<D, BSM_F32><<<grid, 4 * kFastSites, 0, st>>>(g, a, nbm, per_wg);
                k_net_tsum16<D, BSM_F32><<<2 * nb64, 256, 0, st>>>(g, a, nb64);
            }
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        }
    }
};

bsm_status launch_net_fast(const Geom &g, int d, const NetFastArgs &a, hipStream_t st) {
    if (!net_fast_supported(d)) return fail(BSM_ERR_UNSUPPORTED, "the collapsed network runs for d_R <= 3");
    return dispatch_d<NetFastByD>(d, g, a, st);
}

}  // namespace bsm
