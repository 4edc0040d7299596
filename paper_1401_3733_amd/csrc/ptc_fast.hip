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
// Precision: the transports are FP32.  The mixing runs on FP16 matrix cores
// with FP32 accumulation: each site's nine transported fields are divided by
// their largest |component| before rounding to FP16, C by its largest entry;
// the nine mixed fields are stored in FP16 with that per-site scale.  The
// result agrees with the FP32 layers to a relative O(1e-3), which is what a
// preconditioner of a flexible Krylov method needs.
#include "dispatch.h"
#include "ptc.h"
#include "ptc_dev.h"

namespace bsm {

typedef _Float16 h4v __attribute__((ext_vector_type(4)));

constexpr int kFastMaxD = 3;    // colour dimensions of the matrix-core mixing
constexpr int kFastRows = 72;   // (path, spin, re/im) of the real form
constexpr int kFastTiles = 5;   // 16-row tiles covering 72 rows (and 16-deep K steps covering 72)
constexpr int kFastKq = 18;     // groups of 4 K values per site and colour

// C (36 x 36 complex, FP64 sums) -> FP16 real form / cs in the lane order of
// the 16x16x16 matrix-core fragments: frag[(mt * 5 + ks) * 64 + lane] holds
// A[16 mt + lane % 16][16 ks + 4 (lane / 16) + 0..3]; cs = max |Re|, |Im|.
// One workgroup.
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
            const int k = 16 * ks + 4 * (lane / 16) + j;
            v[j] = 0.f;
            if (m < kFastRows && k < kFastRows) {
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
            const h4v x = G[g16_index<D>(g, p, par, bp * D + cc, h)];
            v[(2 * bp) * D + cc] = mk<float>((float)x[0] * s, (float)x[1] * s);
            v[(2 * bp + 1) * D + cc] = mk<float>((float)x[2] * s, (float)x[3] * s);
        }
}

// t = w U s (forward path) or w U^dag s (backward path)
template <int D>
__device__ inline void link_apply(const Geom &g, const PathSite &ps, const cx<float> (&s)[4 * D],
                                  cx<float> (&t)[4 * D]) {
#pragma unroll
    for (int k = 0; k < 4 * D; k++) t[k] = mk<float>(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            const cx<float> u = load_link<BSM_F32, false, float>(ps.blk, g.Vh_pad, i * D + j, ps.hl);
#pragma unroll
            for (int a = 0; a < 4; a++) {
                if (!ps.back) t[a * D + i] = cfma(u, s[a * D + j], t[a * D + i]);
                else t[a * D + j] = cfma_conj(u, s[a * D + i], t[a * D + j]);
            }
        }
#pragma unroll
    for (int k = 0; k < 4 * D; k++) t[k] = ps.w * t[k];
}

template <int D>
__device__ inline float maxabs(const cx<float> (&t)[4 * D], float m) {
#pragma unroll
    for (int k = 0; k < 4 * D; k++) m = fmaxf(m, fmaxf(fabsf(t[k].re), fabsf(t[k].im)));
    return m;
}

// write t * inv as FP16 into the B tile: Bh[(colour * 18 + 2 p + spin pair) * 64 + site]
template <int D>
__device__ inline void stage_path(h4v *Bh, int p, int s, float inv, const cx<float> (&t)[4 * D]) {
#pragma unroll
    for (int bp = 0; bp < 2; bp++)
#pragma unroll
        for (int cc = 0; cc < D; cc++) {
            const cx<float> x0 = t[(2 * bp) * D + cc], x1 = t[(2 * bp + 1) * D + cc];
            Bh[(cc * kFastKq + 2 * p + bp) * 64 + s] =
                h4v{(_Float16)(x0.re * inv), (_Float16)(x0.im * inv), (_Float16)(x1.re * inv), (_Float16)(x1.im * inv)};
        }
}

// G'_p(y) = sum_q (C / cs) (T_q v)(y) / s(y) for 64 sites of one parity per
// workgroup of 256 threads.  Phase 1: thread (site, path group pg) forms the
// transports of paths pg, pg + 4 (and 8 for pg = 0), the site's scale s(y)
// is their largest |component|, then they go to LDS in FP16.  Phase 2:
// wavefront w multiplies the 72 x 72 real form with the K x 16 tile of its
// sites 16w..16w+15, one colour at a time, and stores G' in FP16.
template <int D>
__global__ __launch_bounds__(256) void k_net_mix16(Geom g, NetFastArgs a, int nblk) {
    __shared__ h4v Bh[D * kFastKq * 64];
    __shared__ float smax[4 * 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, sl = lane & 15;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t hb = (lb - px * nblk) * 64;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(BSM_F32, false, D, g.Vh_pad);
    {
        const int s = tid & 63, pg = tid >> 6;
        const uint32_t h = hb + s;
        const bool live = h < (uint32_t)g.Vh;
        cx<float> t0[4 * D], t1[4 * D], t2[4 * D];
#pragma unroll
        for (int e = 0; e < 4 * D; e++) t0[e] = t1[e] = t2[e] = mk<float>(0.f, 0.f);
        float mx = 0.f;
        if (live) {
            const Coords c = decode(g, h, px);
            const char *U = (const char *)a.U, *v = (const char *)a.in;
            transport<D>(g, U, lblk, v, pblk, px, h, c, pg, t0);
            transport<D>(g, U, lblk, v, pblk, px, h, c, pg + 4, t1);
            if (pg == 0) transport<D>(g, U, lblk, v, pblk, px, h, c, 8, t2);
            mx = maxabs<D>(t2, maxabs<D>(t1, maxabs<D>(t0, 0.f)));
        }
        smax[pg * 64 + s] = mx;
        __syncthreads();
        const float m = fmaxf(fmaxf(smax[s], smax[64 + s]), fmaxf(smax[128 + s], smax[192 + s]));
        const float inv = m > 0.f ? 1.f / m : 0.f;
        stage_path<D>(Bh, pg, s, inv, t0);
        stage_path<D>(Bh, pg + 4, s, inv, t1);
        if (pg == 0) stage_path<D>(Bh, 8, s, inv, t2);
    }
    __syncthreads();
    const uint32_t h = hb + 16 * w + sl;
    const bool live = h < (uint32_t)g.Vh;
    if (live && q == 0) {
        const int s = 16 * w + sl;
        a.S[(size_t)px * g.Vh_pad + h] =
            fmaxf(fmaxf(smax[s], smax[64 + s]), fmaxf(smax[128 + s], smax[192 + s]));
    }
    const h4v *fr = (const h4v *)a.Afrag;
    h4v af[kFastTiles][kFastTiles];
#pragma unroll
    for (int mt = 0; mt < kFastTiles; mt++)
#pragma unroll
        for (int ks = 0; ks < kFastTiles; ks++) af[mt][ks] = fr[(mt * kFastTiles + ks) * 64 + lane];
    h4v *G = (h4v *)a.G;
#pragma unroll
    for (int cc = 0; cc < D; cc++) {
        f4v acc[kFastTiles];
#pragma unroll
        for (int mt = 0; mt < kFastTiles; mt++) acc[mt] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kFastTiles; ks++) {
            const int kq = 4 * ks + q;
            const h4v b = kq < kFastKq ? Bh[(cc * kFastKq + kq) * 64 + 16 * w + sl] : h4v{0, 0, 0, 0};
#pragma unroll
            for (int mt = 0; mt < kFastTiles; mt++)
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x16f16(af[mt][ks], b, acc[mt], 0, 0, 0);
        }
        if (!live) continue;
        // rows 16 mt + 4 q + v: path 2 mt + q / 2, spins 2 (q % 2) and 2 (q % 2) + 1
#pragma unroll
        for (int mt = 0; mt < kFastTiles; mt++) {
            const int p = 2 * mt + q / 2;
            if (p >= 9) continue;
            G[g16_index<D>(g, p, px, (q & 1) * D + cc, h)] =
                h4v{(_Float16)acc[mt][0], (_Float16)acc[mt][1], (_Float16)acc[mt][2], (_Float16)acc[mt][3]};
        }
    }
}

// z(x) = cs * (G_0(x) + sum_{p >= 1} (T_p G_p)(x)), one thread per site
template <int D>
__global__ __launch_bounds__(256) void k_net_tsum16(Geom g, NetFastArgs a, int nblk) {
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t h = (lb - px * nblk) * 256 + threadIdx.x;
    if (h >= (uint32_t)g.Vh) return;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(BSM_F32, false, D, g.Vh_pad);
    const Coords c = decode(g, h, px);
    cx<float> acc[4 * D];
    load_g16<D>(a, g, 0, px, h, acc);
    for (int p = 1; p < 9; p++) {
        const PathSite ps = path_site(g, (const char *)a.U, lblk, px, h, c, p);
        cx<float> v[4 * D], t[4 * D];
        load_g16<D>(a, g, p, 1 - px, ps.hn, v);
        link_apply<D>(g, ps, v, t);
#pragma unroll
        for (int e = 0; e < 4 * D; e++) acc[e] = acc[e] + t[e];
    }
    const float cs = *a.cs;
#pragma unroll
    for (int e = 0; e < 4 * D; e++) acc[e] = cs * acc[e];
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
            const int nb64 = (g.Vh + 63) / 64, nb256 = (g.Vh + 255) / 256;
            k_net_mix16<D><<<2 * nb64, 256, 0, st>>>(g, a, nb64);
            k_net_tsum16<D><<<2 * nb256, 256, 0, st>>>(g, a, nb256);
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
