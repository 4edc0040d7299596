// Parallel-transport convolution (PTC) layers of the learned preconditioner.
//
//   out_i(x) = sum_j sum_p W_p^{ij} (T_p v_j)(x),   p in {stay, +mu, -mu}
//   T_{+mu} v(x) = s+ U_mu(x) v(x+mu),  T_{-mu} v(x) = s- U_mu(x-mu)^dag v(x-mu)
//
// W_p^{ij} is a complex 4 x 4 spin matrix acting on the spin index of the
// transported field; the links act on colour, so the layer commutes with
// gauge transformations.  Channel fields are F32 full internal fields,
// consecutive per channel.  Weights: complex float [cout][cin][9][4][4].
// The adjoint layer is a PTC layer with weights (W_p^{ij})^dag at the
// reversed path and channels swapped (T_{+mu}^dag = T_{-mu}), built by a
// small kernel; the weight gradient is a lattice sum of outer products.
// Arithmetic is FP32; reductions accumulate in FP64.
#include "dispatch.h"
#include "ptc.h"
#include "ptc_dev.h"

namespace bsm {

// acc[q] += W_p^{i0+q, j} t for the output channels of this workgroup
template <int D, int CG>
__device__ inline void mix_spin(const float2 *W, int cin, int cout, int i0, int j, int p, const cx<float> (&t)[4 * D],
                                cx<float> (&acc)[CG][4 * D]) {
#pragma unroll
    for (int q = 0; q < CG; q++) {
        const int i = i0 + q;
        if (i >= cout) break;
        const float2 *w = W + (((size_t)i * cin + j) * 9 + p) * 16;
#pragma unroll
        for (int sa = 0; sa < 4; sa++)
#pragma unroll
            for (int sb = 0; sb < 4; sb++) {
                const float2 wv = w[sa * 4 + sb];
                const cx<float> wc = mk<float>(wv.x, wv.y);
#pragma unroll
                for (int cc = 0; cc < D; cc++) acc[q][sa * D + cc] = cfma(wc, t[sb * D + cc], acc[q][sa * D + cc]);
            }
    }
}

// One thread per site of both parities; blockIdx.y selects a group of CG
// output channels.  Paths outermost: the link of a path is loaded once into
// registers and carries every input channel's neighbour.
template <int D, int CG>
__global__ __launch_bounds__(256) void k_ptc_layer(Geom g, PtcArgs a, int nblk) {
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t h = (lb - px * nblk) * 256 + threadIdx.x;
    if (h >= (uint32_t)g.Vh) return;
    const int i0 = blockIdx.y * CG;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(BSM_F32, false, D, g.Vh_pad);
    const Coords c = decode(g, h, px);
    const float2 *W = (const float2 *)a.W;
    const char *in = (const char *)a.in;
    cx<float> acc[CG][4 * D];
#pragma unroll
    for (int q = 0; q < CG; q++)
#pragma unroll
        for (int k = 0; k < 4 * D; k++) acc[q][k] = mk<float>(0.f, 0.f);
    // stay path
    for (int j = 0; j < a.cin; j++) {
        cx<float> t[4 * D];
        load_spinor<BSM_F32, D, float>(in + (size_t)j * 2 * pblk + px * pblk, g.Vh_pad, h, t);
        mix_spin<D, CG>(W, a.cin, a.cout, i0, j, 0, t, acc);
    }
    for (int p = 1; p < 9; p++) {
        const PathSite ps = path_site(g, (const char *)a.U, lblk, px, h, c, p);
        cx<float> u[D * D];
#pragma unroll
        for (int e = 0; e < D * D; e++) {
            u[e] = load_link<BSM_F32, false, float>(ps.blk, g.Vh_pad, e, ps.hl);
            u[e] = ps.w * u[e];
        }
        for (int j = 0; j < a.cin; j++) {
            cx<float> s[4 * D], t[4 * D];
            load_spinor<BSM_F32, D, float>(in + (size_t)j * 2 * pblk + (1 - px) * pblk, g.Vh_pad, ps.hn, s);
#pragma unroll
            for (int k = 0; k < 4 * D; k++) t[k] = mk<float>(0.f, 0.f);
            if (!ps.back) {
#pragma unroll
                for (int i = 0; i < D; i++)
#pragma unroll
                    for (int jj = 0; jj < D; jj++)
#pragma unroll
                        for (int sa = 0; sa < 4; sa++) t[sa * D + i] = cfma(u[i * D + jj], s[sa * D + jj], t[sa * D + i]);
            } else {
#pragma unroll
                for (int i = 0; i < D; i++)
#pragma unroll
                    for (int jj = 0; jj < D; jj++)
#pragma unroll
                        for (int sa = 0; sa < 4; sa++)
                            t[sa * D + jj] = cfma_conj(u[i * D + jj], s[sa * D + i], t[sa * D + jj]);
            }
            mix_spin<D, CG>(W, a.cin, a.cout, i0, j, p, t, acc);
        }
    }
#pragma unroll
    for (int q = 0; q < CG; q++) {
        const int i = i0 + q;
        if (i >= a.cout) break;
        char *oi = (char *)a.out + (size_t)i * 2 * pblk + px * pblk;
        store_spinor<BSM_F32, D, float>(oi, g.Vh_pad, h, acc[q]);
    }
}

// ------------------------------------------------------ matrix-core layers
// The spin mixing is a dense complex contraction shared by every site, so it
// runs on FP32 matrix cores (v_mfma_f32_16x16x4f32) in its real form
//   [Re o; Im o] = [[Re W, -Im W], [Im W, Re W]] [Re t; Im t],
// with the operand layout  A: lane l -> A[l%16][l/16],  B: lane l ->
// B[l/16][l%16],  D: lane l -> D[4(l/16)+v][l%16], v < 4.  A wavefront owns
// 16 consecutive sites; the N dimension of a tile is those 16 sites at one
// colour, so the colour index never mixes.
//   transport-then-mix (cin <= cout): rows m = (i, a, re/im), columns
//     k = (j, p, b, re/im) of the transported fields, staged in LDS;
//   mix-at-source (cin > cout): rows m = (i, p, a, re/im), columns
//     k = (j, b, re/im) read straight from the input fields, giving
//     G_{i,p} = sum_j W_p^{ij} v_j, then out_i = sum_p T_p G_{i,p}.
__host__ __device__ inline int round16(int x) { return (x + 15) / 16 * 16; }

size_t ptc_areal_floats(int cin, int cout) {
    const size_t t = (size_t)(round16(cout * 8) + 16) * cin * 72, x = (size_t)(round16(cout * 72) + 16) * cin * 8;
    return t > x ? t : x;
}

size_t ptc_gmix_bytes(const Geom &g, int d, int cin, int cout) {
    return (size_t)cout * 9 * 2 * spinor_block_bytes(BSM_F32, d, g.Vh_pad);
}

// row stride of the transposed matrix: the two 16-lane row groups of a half
// wavefront read rows k and k + 1, which then fall in disjoint LDS banks
__host__ __device__ inline int at_stride(int Mp) { return Mp % 32 == 0 ? Mp + 16 : Mp; }

// The real-form matrix, transposed: At[k * at_stride(Mp) + m] (pad entries 0).
// mode 0: transport-then-mix layout; mode 1: mix-at-source layout
__global__ void k_ptc_realform(const float2 *W, float *At, int cin, int cout, int mode) {
    const int M = mode == 0 ? cout * 8 : cout * 72, Mp = round16(M), AS = at_stride(Mp);
    const int K = mode == 0 ? cin * 72 : cin * 8;
    const int n = AS * K;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int k = e / AS, m = e % AS;
        float v = 0.f;
        if (m < M) {
            int i, j, p, aa, bb;
            const int ro = m & 1, ri = k & 1;
            if (mode == 0) {
                i = m / 8; aa = (m % 8) / 2;
                j = k / 72; p = (k % 72) / 8; bb = (k % 8) / 2;
            } else {
                const int ia = m / 2;
                i = ia / 36; p = (ia / 4) % 9; aa = ia % 4;
                j = k / 8; bb = (k % 8) / 2;
            }
            const float2 w = W[(((size_t)i * cin + j) * 9 + p) * 16 + aa * 4 + bb];
            v = ro == ri ? w.x : (ro == 0 ? -w.y : w.y);
        }
        At[e] = v;
    }
}

// F32 full-field element access: complex component comp of site h in the
// parity block starting at blk (float pointer)
__device__ inline size_t f32_elem(int comp, int64_t stride, uint32_t h) {
    return ((size_t)(comp >> 1) * stride + h) * 4 + (comp & 1) * 2;
}

// the real-form matrix, transposed ([k][m], Mp rows), into LDS by the
// whole workgroup
// Matrix-core kernels for the network's shapes (d_R <= 3): a workgroup of
// 256 threads owns 64 consecutive sites of one parity.  Phase 1 stages the
// B operand in LDS with one site per thread (all loads of the 64 sites in
// flight together); phase 2 gives wavefront w the 16 sites 16w..16w+15 at
// every colour, with the A fragments held in registers.
constexpr int kMfmaMaxD = 3;

// this lane's A fragments: a[mt][ks] = At[(4 ks + q) * AS + 16 mt + sl]
template <int MT, int KS>
__device__ inline void load_afrag(const float *At, int AS, int q, int sl, float (&af)[MT][KS]) {
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int ks = 0; ks < KS; ks++) af[mt][ks] = At[(size_t)(4 * ks + q) * AS + 16 * mt + sl];
}

// acc[c][mt] = sum_k A[16 mt + .][k] B[k][colour c, 16 sites]
template <int D, int MT, int KS>
__device__ inline void mfma_block(const float (&af)[MT][KS], const float *Bs, int w, int q, int sl,
                                  f4v (&acc)[D][MT]) {
#pragma unroll
    for (int c = 0; c < D; c++)
#pragma unroll
        for (int mt = 0; mt < MT; mt++) acc[c][mt] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
        const int k = 4 * ks + q;
        float bv[D];
#pragma unroll
        for (int c = 0; c < D; c++) bv[c] = Bs[((size_t)k * D + c) * 64 + 16 * w + sl];
#pragma unroll
        for (int c = 0; c < D; c++)
#pragma unroll
            for (int mt = 0; mt < MT; mt++)
                acc[c][mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mt][ks], bv[c], acc[c][mt], 0, 0, 0);
    }
}

// transport-then-mix for cin = 1: rows m = (i, a, re/im), MT = ceil(8 cout / 16),
// columns k = (p, b, re/im), K = 72
template <int D, int MT>
__global__ __launch_bounds__(256) void k_ptc_l1_mfma(Geom g, PtcArgs a, int nblk) {
    constexpr int K = 72, KS = K / 4, Mp = 16 * MT;
    __shared__ float Bs[K * D * 64];   // [k][colour][site]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, sl = lane & 15;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t hb = (lb - px * nblk) * 64;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(BSM_F32, false, D, g.Vh_pad);
    {
        // phase 1: site hb + (tid & 63), paths pg, pg + 4, pg + 8 with pg = tid >> 6
        const int s = tid & 63, pg = tid >> 6;
        const uint32_t h = hb + s;
        const bool live = h < (uint32_t)g.Vh;
        Coords c{};
        if (live) c = decode(g, h, px);
        for (int p = pg; p < 9; p += 4) {
            cx<float> t[4 * D];
            if (live) {
                transport<D>(g, (const char *)a.U, lblk, (const char *)a.in, pblk, px, h, c, p, t);
            } else {
#pragma unroll
                for (int e = 0; e < 4 * D; e++) t[e] = mk<float>(0.f, 0.f);
            }
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int cc = 0; cc < D; cc++) {
                    const int k = (p * 4 + b) * 2;
                    Bs[((size_t)k * D + cc) * 64 + s] = t[b * D + cc].re;
                    Bs[((size_t)(k + 1) * D + cc) * 64 + s] = t[b * D + cc].im;
                }
        }
    }
    float af[MT][KS];
    load_afrag<MT, KS>(a.Areal, at_stride(Mp), q, sl, af);
    __syncthreads();
    f4v acc[D][MT];
    mfma_block<D, MT, KS>(af, Bs, w, q, sl, acc);
    const uint32_t h = hb + 16 * w + sl;
    if (h >= (uint32_t)g.Vh) return;
#pragma unroll
    for (int cc = 0; cc < D; cc++)
#pragma unroll
        for (int mt = 0; mt < MT; mt++)
#pragma unroll
            for (int v = 0; v < 4; v += 2) {
                const int m = 16 * mt + 4 * q + v;   // (i, a, re); m + 1 is (i, a, im)
                const int i = m / 8, sp = (m % 8) / 2;
                if (i >= a.cout) continue;
                float *oi = (float *)((char *)a.out + (size_t)i * 2 * pblk + px * pblk);
                *(float2 *)(oi + f32_elem(sp * D + cc, g.Vh_pad, h)) = make_float2(acc[cc][mt][v], acc[cc][mt][v + 1]);
            }
}

// mix-at-source for cout = 1: G_p(y) = sum_j W_p^{j} v_j(y); rows m = (p, a,
// re/im) (72, MT = 5), columns k = (j, b, re/im), KS = 2 cin
template <int D, int KS>
__global__ __launch_bounds__(256) void k_ptc_mix1_mfma(Geom g, PtcArgs a, int nblk) {
    constexpr int K = 4 * KS, MT = 5, Mp = 80;
    __shared__ float Bs[K * D * 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, sl = lane & 15;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t hb = (lb - px * nblk) * 64;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    {
        const int s = tid & 63, grp = tid >> 6;
        const uint32_t h = hb + s;
        const bool live = h < (uint32_t)g.Vh;
        for (int j = grp; j < K / 8; j += 4) {
            cx<float> v[4 * D];
            if (live) {
                load_spinor<BSM_F32, D, float>((const char *)a.in + (size_t)j * 2 * pblk + px * pblk, g.Vh_pad, h, v);
            } else {
#pragma unroll
                for (int e = 0; e < 4 * D; e++) v[e] = mk<float>(0.f, 0.f);
            }
#pragma unroll
            for (int b = 0; b < 4; b++)
#pragma unroll
                for (int cc = 0; cc < D; cc++) {
                    const int k = (j * 4 + b) * 2;
                    Bs[((size_t)k * D + cc) * 64 + s] = v[b * D + cc].re;
                    Bs[((size_t)(k + 1) * D + cc) * 64 + s] = v[b * D + cc].im;
                }
        }
    }
    float af[MT][KS];
    load_afrag<MT, KS>(a.Areal, at_stride(Mp), q, sl, af);
    __syncthreads();
    f4v acc[D][MT];
    mfma_block<D, MT, KS>(af, Bs, w, q, sl, acc);
    const uint32_t h = hb + 16 * w + sl;
    if (h >= (uint32_t)g.Vh) return;
#pragma unroll
    for (int cc = 0; cc < D; cc++)
#pragma unroll
        for (int mt = 0; mt < MT; mt++)
#pragma unroll
            for (int v = 0; v < 4; v += 2) {
                const int m = 16 * mt + 4 * q + v;   // (p, a, re)
                if (m >= 72) continue;
                const int p = m / 8, sp = (m % 8) / 2;
                float *gf = (float *)(a.Gmix + (size_t)p * 2 * pblk + px * pblk);
                *(float2 *)(gf + f32_elem(sp * D + cc, g.Vh_pad, h)) = make_float2(acc[cc][mt][v], acc[cc][mt][v + 1]);
            }
}

// out_i(x) = G_{i,0}(x) + sum_{p >= 1} (T_p G_{i,p})(x); blockIdx.y = i
template <int D>
__global__ __launch_bounds__(256) void k_ptc_tsum(Geom g, PtcArgs a, int nblk) {
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t h = (lb - px * nblk) * 256 + threadIdx.x;
    if (h >= (uint32_t)g.Vh) return;
    const int i = blockIdx.y;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(BSM_F32, false, D, g.Vh_pad);
    const Coords c = decode(g, h, px);
    const char *G = a.Gmix + (size_t)i * 9 * 2 * pblk;
    cx<float> acc[4 * D];
    load_spinor<BSM_F32, D, float>(G + px * pblk, g.Vh_pad, h, acc);
    for (int p = 1; p < 9; p++) {
        cx<float> t[4 * D];
        transport<D>(g, (const char *)a.U, lblk, G + (size_t)p * 2 * pblk, pblk, px, h, c, p, t);
#pragma unroll
        for (int e = 0; e < 4 * D; e++) acc[e] = acc[e] + t[e];
    }
    store_spinor<BSM_F32, D, float>((char *)a.out + (size_t)i * 2 * pblk + px * pblk, g.Vh_pad, h, acc);
}

// Wa[j][i][rev p] = W[i][j][p]^dag
__global__ void k_ptc_adjoint_weights(const float2 *W, float2 *Wa, int cin, int cout) {
    const int n = cout * cin * 9 * 16;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int ab = e % 16, rest = e / 16;
        const int p = rest % 9, ij = rest / 9;
        const int j = ij % cin, i = ij / cin;
        const int sa = ab / 4, sb = ab % 4;
        const int pr = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
        const float2 w = W[(((size_t)i * cin + j) * 9 + p) * 16 + sa * 4 + sb];
        Wa[(((size_t)j * cout + i) * 9 + pr) * 16 + sb * 4 + sa] = make_float2(w.x, -w.y);
    }
}

// dW partials: grid.x over sites (both parities), grid.y = cin * 9 (j, p).
// Each thread forms t = T_p v_j at its site and, for every output channel i,
// the 16 spin-matrix entries sum_c G_i[a][c] conj(t[b][c]); the workgroup
// sums them (FP64) into partials[(block * cout + i) * cin * 9 + j * 9 + p][16].
template <int D>
__global__ __launch_bounds__(256) void k_ptc_wgrad(Geom g, PtcArgs a, int nblk, double2 *partials) {
    const uint32_t lb = blockIdx.x;
    const int px = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t h = (lb - px * nblk) * 256 + threadIdx.x;
    const int j = blockIdx.y / 9, p = blockIdx.y % 9;
    const bool active = h < (uint32_t)g.Vh;
    const size_t pblk = spinor_block_bytes(BSM_F32, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(BSM_F32, false, D, g.Vh_pad);
    cx<float> t[4 * D];
    if (active) {
        const Coords c = decode(g, h, px);
        transport<D>(g, (const char *)a.U, lblk, (const char *)a.in + (size_t)j * 2 * pblk, pblk, px, h, c, p, t);
    }
    __shared__ double2 red[4][16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = 0; i < a.cout; i++) {
        cx<float> G[4 * D];
        if (active) load_spinor<BSM_F32, D, float>((const char *)a.G + (size_t)i * 2 * pblk + px * pblk, g.Vh_pad, h, G);
        for (int e = 0; e < 16; e++) {
            const int sa = e / 4, sb = e % 4;
            double re = 0, im = 0;
            if (active) {
                cx<float> s = mk<float>(0.f, 0.f);
#pragma unroll
                for (int cc = 0; cc < D; cc++) s = cfma_conj(t[sb * D + cc], G[sa * D + cc], s);
                re = s.re;
                im = s.im;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                re += __shfl_xor(re, o, 64);
                im += __shfl_xor(im, o, 64);
            }
            if (lane == 0) red[wave][e] = make_double2(re, im);
        }
        __syncthreads();
        if (threadIdx.x < 16) {
            double2 s0 = red[0][threadIdx.x], s1 = red[1][threadIdx.x], s2 = red[2][threadIdx.x],
                    s3 = red[3][threadIdx.x];
            partials[(((size_t)lb * a.cout + i) * a.cin * 9 + j * 9 + p) * 16 + threadIdx.x] =
                make_double2((s0.x + s1.x) + (s2.x + s3.x), (s0.y + s1.y) + (s2.y + s3.y));
        }
        __syncthreads();
    }
}

// dW[e] = sum over workgroups (fixed order), e over cout * cin * 9 * 16
__global__ void k_ptc_wgrad_reduce(const double2 *partials, int nblocks, int nw, float2 *dW, double scale,
                                   int accumulate) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nw; e += gridDim.x * blockDim.x) {
        double re = 0, im = 0;
        for (int b = 0; b < nblocks; b++) {
            const double2 v = partials[(size_t)b * nw + e];
            re += v.x;
            im += v.y;
        }
        float2 o = make_float2((float)(scale * re), (float)(scale * im));
        if (accumulate) {
            o.x += dW[e].x;
            o.y += dW[e].y;
        }
        dW[e] = o;
    }
}

// Adam on the real and imaginary parts (Kingma & Ba 2014)
__global__ void k_adam(float2 *w, const float2 *g, float4 *mv, int n, float lr, float b1, float b2, float eps,
                       int t) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        float4 s = mv[e];   // m.re, m.im, v.re, v.im
        const float2 gv = g[e];
        s.x = b1 * s.x + (1.f - b1) * gv.x;
        s.y = b1 * s.y + (1.f - b1) * gv.y;
        s.z = b2 * s.z + (1.f - b2) * gv.x * gv.x;
        s.w = b2 * s.w + (1.f - b2) * gv.y * gv.y;
        mv[e] = s;
        float2 wv = w[e];
        wv.x -= lr * (s.x / c1) / (sqrtf(s.z / c2) + eps);
        wv.y -= lr * (s.y / c1) / (sqrtf(s.w / c2) + eps);
        w[e] = wv;
    }
}

// ------------------------------------------------------------- launchers
template <int D>
struct PtcByD {
    static bsm_status run(const Geom &g, const PtcArgs &a, int mode, double2 *partials, hipStream_t st) {
        if constexpr (D > kPtcMaxD) {
            return fail(BSM_ERR_UNSUPPORTED, "PTC layers are compiled for d_R <= 6");
        } else {
            const int nblk = (g.Vh + 255) / 256;
            if (mode == 0) {
                // output channels per thread: as many as the registers hold
                // next to a D x D link and two spinors
                constexpr int CG = D <= 3 ? 4 : D <= 4 ? 2 : 1;
                dim3 grid(2 * nblk, (a.cout + CG - 1) / CG);
                const int nb64 = (g.Vh + 63) / 64;
                if (a.Areal && D <= kMfmaMaxD && a.cin == 1 && a.cout <= 8) {
                    const int MT = (8 * a.cout + 15) / 16;
                    const int n = at_stride(16 * MT) * 72;
                    k_ptc_realform<<<(n + 255) / 256, 256, 0, st>>>((const float2 *)a.W, a.Areal, 1, a.cout, 0);
                    if constexpr (D <= kMfmaMaxD) {
                        switch (MT) {
                        case 1: k_ptc_l1_mfma<D, 1><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        case 2: k_ptc_l1_mfma<D, 2><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        case 3: k_ptc_l1_mfma<D, 3><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        default: k_ptc_l1_mfma<D, 4><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        }
                    }
                } else if (a.Areal && a.Gmix && D <= kMfmaMaxD && a.cout == 1 && a.cin >= 2 && a.cin <= 8) {
                    const int n = at_stride(80) * 8 * a.cin;
                    k_ptc_realform<<<(n + 255) / 256, 256, 0, st>>>((const float2 *)a.W, a.Areal, a.cin, 1, 1);
                    if constexpr (D <= kMfmaMaxD) {
                        switch (a.cin) {
                        case 2: k_ptc_mix1_mfma<D, 4><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        case 3: k_ptc_mix1_mfma<D, 6><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        case 4: k_ptc_mix1_mfma<D, 8><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        case 5: k_ptc_mix1_mfma<D, 10><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        case 6: k_ptc_mix1_mfma<D, 12><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        case 7: k_ptc_mix1_mfma<D, 14><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        default: k_ptc_mix1_mfma<D, 16><<<2 * nb64, 256, 0, st>>>(g, a, nb64); break;
                        }
                    }
                    k_ptc_tsum<D><<<dim3(2 * nblk, 1), 256, 0, st>>>(g, a, nblk);
                } else {
                    k_ptc_layer<D, CG><<<grid, 256, 0, st>>>(g, a, nblk);
                }
            } else {
                dim3 grid(2 * nblk, a.cin * 9);
                k_ptc_wgrad<D><<<grid, 256, 0, st>>>(g, a, nblk, partials);
            }
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        }
    }
};

bsm_status launch_ptc_layer(const Geom &g, int d, const PtcArgs &a, hipStream_t st) {
    return dispatch_d<PtcByD>(d, g, a, 0, (double2 *)nullptr, st);
}

int ptc_wgrad_blocks(const Geom &g) { return 2 * ((g.Vh + 255) / 256); }

bsm_status launch_ptc_wgrad(const Geom &g, int d, const PtcArgs &a, double2 *partials, float2 *dW, double scale,
                            bool accumulate, hipStream_t st) {
    bsm_status s = dispatch_d<PtcByD>(d, g, a, 1, partials, st);
    if (s != BSM_OK) return s;
    const int nw = a.cout * a.cin * 9 * 16;
    k_ptc_wgrad_reduce<<<(nw + 255) / 256, 256, 0, st>>>(partials, ptc_wgrad_blocks(g), nw, dW, scale,
                                                          accumulate ? 1 : 0);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status launch_ptc_adjoint_weights(const void *W, void *Wa, int cin, int cout, hipStream_t st) {
    const int n = cout * cin * 9 * 16;
    k_ptc_adjoint_weights<<<(n + 255) / 256, 256, 0, st>>>((const float2 *)W, (float2 *)Wa, cin, cout);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

bsm_status launch_adam(void *w, const void *g, void *mv, int n, float lr, float b1, float b2, float eps, int t,
                       hipStream_t st) {
    k_adam<<<(n + 255) / 256, 256, 0, st>>>((float2 *)w, (const float2 *)g, (float4 *)mv, n, lr, b1, b2, eps, t);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

}  // namespace bsm
