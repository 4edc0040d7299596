// Learned preconditioner: network application, training (Adam on the GPU),
// training pairs from CG, and flexible GCR with the network and a plain-CG
// fall back.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <vector>

#include "ptc.h"
#include "solver.h"
#include "spinor_io.h"

namespace bsm {

static size_t layer_weights(int cin, int cout) { return (size_t)cout * cin * 9 * 16; }   // complex

static bsm_status check_net_desc(bsm_ctx ctx, const bsm_field_desc *desc) {
    if (!ctx || !desc) return fail(BSM_ERR_ARG, "null argument");
    if (bsm_rep_dim(desc->N, desc->rep) != desc->d_R) return fail(BSM_ERR_ARG, "d_R does not match (N, rep)");
    if (desc->prec != BSM_F32 || desc->link_prec != BSM_F32)
        return fail(BSM_ERR_ARG, "the network runs on F32 spinors and F32 links");
    if (desc->rep == BSM_REP_ADJ) return fail(BSM_ERR_UNSUPPORTED, "network kernels use complex links");
    if (desc->d_R > kPtcMaxD) return fail(BSM_ERR_UNSUPPORTED, "network kernels are compiled for d_R <= 6");
    return BSM_OK;
}

// ------------------------------------------------------ FGCR vector kernels
// Flat loops over the complex numbers of F32 full fields (n float2; the
// plane order is the same for every field, so sums over all components do
// not depend on it).  Products are formed in FP32 and summed in FP64.  GCR
// keeps the directions w_j = D z_j unnormalised with nn_j = |w_j|^2, so the
// projections use coefficients <w_j, w> / nn_j.  Orthogonalisation is
// classical Gram-Schmidt in one fused pass (all dots, then all updates),
// equal to modified Gram-Schmidt in exact arithmetic; the residual stays
// consistent either way because r and x are updated with the same (w, z).
constexpr int kGcrMax = 64;   // largest restart length
constexpr int kZdotJ = 8;     // dot products per workgroup row
constexpr int kZblocks = 1024;

struct ZPtrs { const float2 *p[kGcrMax]; };

// Plane geometry of the F32 full fields: complex number e belongs to plane
// index (e / 2) % Vh_pad; indices at or above Vh are padding, which the
// loops skip (no operator writes it, and reused scratch can hold any bytes
// there).
struct ZLive {
    FastDiv pad;
    uint32_t live;
    __device__ inline bool operator()(size_t e) const {
        const uint32_t q = (uint32_t)(e >> 1);
        return q - pad.div(q) * pad.d < live;
    }
};

__device__ inline void block_sum2(double &re, double &im, double2 *ws, int slot, double2 *dst) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) ws[w * kZdotJ + slot] = make_double2(re, im);
    __syncthreads();
    if (threadIdx.x == 0)
        *dst = make_double2((ws[slot].x + ws[kZdotJ + slot].x) + (ws[2 * kZdotJ + slot].x + ws[3 * kZdotJ + slot].x),
                            (ws[slot].y + ws[kZdotJ + slot].y) + (ws[2 * kZdotJ + slot].y + ws[3 * kZdotJ + slot].y));
}

// partials[j][block] = sum conj(W_j) w over this workgroup's elements, for
// j in [blockIdx.y * 8, min(k, +8))
__global__ __launch_bounds__(256) void k_zmultidot(ZPtrs W, int k, const float2 *w, size_t n, ZLive lv, double2 *partials) {
    const int j0 = blockIdx.y * kZdotJ;
    double re[kZdotJ], im[kZdotJ];
#pragma unroll
    for (int q = 0; q < kZdotJ; q++) re[q] = im[q] = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        if (!lv(e)) continue;
        const float2 y = w[e];
#pragma unroll
        for (int q = 0; q < kZdotJ; q++) {
            if (j0 + q >= k) break;
            const float2 x = W.p[j0 + q][e];
            re[q] += (double)(x.x * y.x + x.y * y.y);
            im[q] += (double)(x.x * y.y - x.y * y.x);
        }
    }
    __shared__ double2 ws[4 * kZdotJ];
#pragma unroll
    for (int q = 0; q < kZdotJ; q++) {
        if (j0 + q >= k) break;
        block_sum2(re[q], im[q], ws, q, &partials[(size_t)(j0 + q) * gridDim.x + blockIdx.x]);
    }
}

// one workgroup per column j: coef[j] = (sum of nb partials, fixed order) /
// nn[j] (0 when nn[j] is 0)
__global__ __launch_bounds__(256) void k_zcols(const double2 *partials, int nb, const double *nn, double2 *coef) {
    const int j = blockIdx.x;
    double re = 0, im = 0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        re += partials[(size_t)j * nb + i].x;
        im += partials[(size_t)j * nb + i].y;
    }
    __shared__ double2 ws[4 * kZdotJ];
    __shared__ double2 s;
    block_sum2(re, im, ws, 0, &s);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double d = nn[j];
    coef[j] = d > 0 ? make_double2(s.x / d, s.y / d) : make_double2(0.0, 0.0);
}

// w -= sum_j coef_j W_j ; z -= sum_j coef_j Z_j ; partials of |w|^2 and <w, r>
__global__ __launch_bounds__(256) void k_zorth(ZPtrs W, ZPtrs Z, int k, const double2 *coef, float2 *w, float2 *z,
                                               const float2 *r, size_t n, ZLive lv, double2 *partials) {
    __shared__ float2 cs[kGcrMax];
    if (threadIdx.x < k) cs[threadIdx.x] = make_float2((float)coef[threadIdx.x].x, (float)coef[threadIdx.x].y);
    __syncthreads();
    double nw = 0, dr = 0, di = 0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        if (!lv(e)) continue;
        float2 wv = w[e], zv = z[e];
        for (int j = 0; j < k; j++) {
            const float2 c = cs[j], a = W.p[j][e], b = Z.p[j][e];
            wv.x -= c.x * a.x - c.y * a.y;
            wv.y -= c.x * a.y + c.y * a.x;
            zv.x -= c.x * b.x - c.y * b.y;
            zv.y -= c.x * b.y + c.y * b.x;
        }
        if (k > 0) {
            w[e] = wv;
            z[e] = zv;
        }
        const float2 rv = r[e];
        nw += (double)(wv.x * wv.x + wv.y * wv.y);
        dr += (double)(wv.x * rv.x + wv.y * rv.y);
        di += (double)(wv.x * rv.y - wv.y * rv.x);
    }
    __shared__ double2 ws[4 * kZdotJ];
    double zero = 0;
    block_sum2(nw, zero, ws, 0, &partials[blockIdx.x]);
    block_sum2(dr, di, ws, 1, &partials[(size_t)gridDim.x + blockIdx.x]);
}

// alpha = <w, r> / |w|^2 from the nb workgroup partials of k_zorth (every
// workgroup sums them in the same fixed order, so all get the same alpha and
// no separate reduction launch is needed; workgroup 0 records nn[k] = |w|^2);
// then x += alpha z ; r -= alpha w ; per-workgroup |r|^2 into rr_parts
__global__ __launch_bounds__(256) void k_zupdate(float2 *x, float2 *r, const float2 *z, const float2 *w, size_t n,
                                                 ZLive lv, const double2 *orth, int nb, double *nn, int k, double *rr_parts) {
    __shared__ double2 ws[4 * kZdotJ];
    __shared__ double2 s0, s1;
    {
        double a = 0, b = 0, c = 0;
        for (int i = threadIdx.x; i < nb; i += 256) {
            a += orth[i].x;
            b += orth[nb + i].x;
            c += orth[nb + i].y;
        }
        double zero = 0;
        block_sum2(a, zero, ws, 0, &s0);
        block_sum2(b, c, ws, 1, &s1);
        __syncthreads();
    }
    const double d0 = s0.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) nn[k] = d0;
    const float ar = d0 > 0 ? (float)(s1.x / d0) : 0.f, ai = d0 > 0 ? (float)(s1.y / d0) : 0.f;
    double rr = 0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        if (!lv(e)) continue;
        const float2 zv = z[e], wv = w[e];
        float2 xv = x[e], rv = r[e];
        xv.x += ar * zv.x - ai * zv.y;
        xv.y += ar * zv.y + ai * zv.x;
        rv.x -= ar * wv.x - ai * wv.y;
        rv.y -= ar * wv.y + ai * wv.x;
        x[e] = xv;
        r[e] = rv;
        rr += (double)(rv.x * rv.x + rv.y * rv.y);
    }
    __syncthreads();
    double zero = 0;
    __shared__ double2 t2;
    block_sum2(rr, zero, ws, 2, &t2);
    if (threadIdx.x == 0) rr_parts[blockIdx.x] = t2.x;   // block_sum2's writer is thread 0
}

#define TRY(x)                           \
    do {                                 \
        bsm_status _s = (x);             \
        if (_s != BSM_OK) return _s;     \
    } while (0)

// one PTC layer with the matrix-core scratch (real-form weights, mixed
// fields) from the context's layer buffer
static size_t layer_scratch(const Geom &g, int d, int cin, int cout, size_t *na_out) {
    const size_t na = (ptc_areal_floats(cin, cout) * sizeof(float) + 255) / 256 * 256;
    if (na_out) *na_out = na;
    return na + (cin > cout ? ptc_gmix_bytes(g, d, cin, cout) : 0);
}

static bsm_status layer(bsm_ctx ctx, int d, PtcArgs a, hipStream_t st) {
    size_t na = 0;
    const size_t need = layer_scratch(ctx->g, d, a.cin, a.cout, &na);
    void *w = nullptr;
    TRY(ctx_work_slot(ctx, 2, need, &w));
    a.Areal = (float *)w;
    a.Gmix = a.cin > a.cout ? (char *)w + na : nullptr;
    return launch_ptc_layer(ctx->g, d, a, st);
}

// grow the layer scratch for a 1 -> C -> 1 network before any of its layers
// is queued (the C -> 1 layer needs the most), so it is never reallocated
// while a queued layer still reads it
static bsm_status reserve_net(bsm_ctx ctx, int d, int C) {
    void *w = nullptr;
    return ctx_work_slot(ctx, 2, layer_scratch(ctx->g, d, C, 1, nullptr), &w);
}

// z = M(r) on F32 full fields; h: channels F32 full fields of scratch
static bsm_status net_apply(bsm_ctx ctx, const bsm_field_desc *desc, const void *U, int C, const void *net,
                            const void *r, void *h, void *z, hipStream_t st) {
    const float2 *W1 = (const float2 *)net;
    const float2 *W2 = W1 + layer_weights(1, C);
    TRY(reserve_net(ctx, desc->d_R, C));
    PtcArgs a{};
    a.U = U;
    a.W = W1; a.in = r; a.out = h; a.cin = 1; a.cout = C;
    TRY(layer(ctx, desc->d_R, a, st));
    a.W = W2; a.in = h; a.out = z; a.cin = C; a.cout = 1;
    return layer(ctx, desc->d_R, a, st);
}

// the collapsed network: scratch in the network slot, C from the weights
static bsm_status net_fast_prepare(bsm_ctx ctx, int d, int C, const void *net, const void *U, int link_prec,
                                   NetFastArgs &a, hipStream_t st) {
    void *w = nullptr;
    TRY(ctx_work_slot(ctx, 2, net_fast_bytes(ctx->g, d), &w));
    a = NetFastArgs{};
    a.U = U;
    a.link_prec = link_prec;
    net_fast_carve(ctx->g, d, w, a);
    return launch_net_collapse(net, C, a, st);
}

static uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// ------------------------------------------------ allocation-free network
// Scratch of bsm_precond_apply_collapsed_noalloc: the nine FP16 mixed fields,
// their per-site scales and the collapsed mixing matrix, in a static device
// array (every device the library runs on holds its own copy until the
// process ends).  Host code never passes `scratch` itself to a kernel: its
// device address comes from hipGetSymbolAddress, taken once per device at
// context creation and kept in noalloc_ptr.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
constexpr int kNoallocDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
static std::mutex noalloc_mu;
static void *noalloc_ptr[kNoallocDevices];

bsm_status noalloc_scratch_init(int device) {
    if (device < 0 || device >= kNoallocDevices) return fail(BSM_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (noalloc_ptr[device]) return BSM_OK;
    int cur = -1;
    BSM_HIP(hipGetDevice(&cur));
    if (cur != device) return fail(BSM_ERR_ARG, "static scratch set up with another device current");
    void *ptr = nullptr;
    BSM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(BSM_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
    noalloc_ptr[device] = ptr;
    return BSM_OK;
}

static bsm_status noalloc_scratch(int device, void **out) {
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (device < 0 || device >= kNoallocDevices || !noalloc_ptr[device])
        return fail(BSM_ERR_HIP, "static scratch was not set up for this device");
    *out = noalloc_ptr[device];
    return BSM_OK;
}

}  // namespace bsm

using namespace bsm;

extern "C" {

size_t bsm_net_bytes(int32_t channels) {
    if (channels < 1) return 0;
    return (layer_weights(1, channels) + layer_weights(channels, 1)) * sizeof(float2);
}

bsm_status bsm_ptc_layer(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t cin, int32_t cout,
                         const void *W, const void *in, void *out, void *stream) {
    TRY(check_net_desc(ctx, desc));
    if (!U_rep || !W || !in || !out) return fail(BSM_ERR_ARG, "null pointer");
    if (cin < 1 || cout < 1 || cin > 64 || cout > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    if (in == out) return fail(BSM_ERR_ARG, "in and out must differ");
    PtcArgs a{};
    a.U = U_rep; a.W = W; a.in = in; a.out = out; a.cin = cin; a.cout = cout;
    return layer(ctx, desc->d_R, a, (hipStream_t)stream);
}

bsm_status bsm_ptc_layer_adjoint(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t cin,
                                 int32_t cout, const void *W, const void *in, void *out, void *stream) {
    TRY(check_net_desc(ctx, desc));
    if (!U_rep || !W || !in || !out) return fail(BSM_ERR_ARG, "null pointer");
    if (cin < 1 || cout < 1 || cin > 64 || cout > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    hipStream_t st = (hipStream_t)stream;
    void *Wa = nullptr;
    TRY(ctx_work(ctx, layer_weights(cin, cout) * sizeof(float2), &Wa));
    TRY(launch_ptc_adjoint_weights(W, Wa, cin, cout, st));
    PtcArgs a{};
    a.U = U_rep; a.W = Wa; a.in = in; a.out = out; a.cin = cout; a.cout = cin;
    return layer(ctx, desc->d_R, a, st);
}

bsm_status bsm_ptc_weight_grad(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t cin,
                               int32_t cout, const void *G, const void *v, void *dW, void *stream) {
    TRY(check_net_desc(ctx, desc));
    if (!U_rep || !G || !v || !dW) return fail(BSM_ERR_ARG, "null pointer");
    if (cin < 1 || cout < 1 || cin > 64 || cout > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    void *parts = nullptr;
    TRY(ctx_work(ctx, (size_t)ptc_wgrad_blocks(ctx->g) * layer_weights(cin, cout) * sizeof(double2), &parts));
    PtcArgs a{};
    a.U = U_rep; a.in = v; a.G = G; a.cin = cin; a.cout = cout;
    return launch_ptc_wgrad(ctx->g, desc->d_R, a, (double2 *)parts, (float2 *)dW, 1.0, false, (hipStream_t)stream);
}

bsm_status bsm_precond_apply(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t channels,
                             const void *net, const void *r, void *z, void *stream) {
    TRY(check_net_desc(ctx, desc));
    if (!U_rep || !net || !r || !z) return fail(BSM_ERR_ARG, "null pointer");
    if (channels < 1 || channels > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    const size_t f32 = 2 * spinor_block_bytes(BSM_F32, desc->d_R, ctx->g.Vh_pad);
    void *h = nullptr;
    TRY(ctx_work(ctx, channels * f32, &h));
    return net_apply(ctx, desc, U_rep, channels, net, r, h, z, (hipStream_t)stream);
}

bsm_status bsm_precond_backward(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t channels,
                                const void *net, const void *r, const void *dz, void *dr, void *dweights,
                                void *stream) {
    TRY(check_net_desc(ctx, desc));
    if (!U_rep || !net || !r || !dz || !dweights) return fail(BSM_ERR_ARG, "null pointer");
    if (channels < 1 || channels > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    if (dr && (dr == r || dr == dz)) return fail(BSM_ERR_ARG, "dr must differ from r and dz");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = ctx->g;
    const int d = desc->d_R, C = channels;
    const size_t f32 = 2 * spinor_block_bytes(BSM_F32, d, g.Vh_pad);
    const size_t nw1 = layer_weights(1, C), nw2 = layer_weights(C, 1);
    const size_t parts_bytes = (size_t)ptc_wgrad_blocks(g) * std::max(nw1, nw2) * sizeof(double2);
    // scratch: h = L1 r (C fields), Gh = L2^dag dz (C fields), both adjoint
    // weight sets, the weight-gradient partials
    const size_t need = 2 * C * f32 + (nw1 + nw2) * sizeof(float2) + parts_bytes + 6 * 256;
    TRY(reserve_net(ctx, d, C));
    void *work = nullptr;
    TRY(ctx_work(ctx, need, &work));
    char *w = (char *)work;
    auto take = [&](size_t bytes) { char *q = w; w += (bytes + 255) / 256 * 256; return q; };
    char *h = take(C * f32), *Gh = take(C * f32);
    float2 *W1a = (float2 *)take(nw1 * sizeof(float2)), *W2a = (float2 *)take(nw2 * sizeof(float2));
    double2 *parts = (double2 *)take(parts_bytes);
    const float2 *W1 = (const float2 *)net, *W2 = W1 + nw1;
    float2 *dW1 = (float2 *)dweights, *dW2 = dW1 + nw1;
    PtcArgs a{};
    a.U = U_rep;
    // h = L1 r
    a.W = W1; a.in = r; a.out = h; a.cin = 1; a.cout = C;
    TRY(layer(ctx, d, a, st));
    // dW2 = sum_x dz conj(T_p h_j)
    PtcArgs gw{};
    gw.U = U_rep; gw.in = h; gw.G = dz; gw.cin = C; gw.cout = 1;
    TRY(launch_ptc_wgrad(g, d, gw, parts, dW2, 1.0, false, st));
    // Gh = L2^dag dz
    TRY(launch_ptc_adjoint_weights(W2, W2a, C, 1, st));
    a.W = W2a; a.in = dz; a.out = Gh; a.cin = 1; a.cout = C;
    TRY(layer(ctx, d, a, st));
    // dW1 = sum_x Gh_j conj(T_p r)
    gw.in = r; gw.G = Gh; gw.cin = 1; gw.cout = C;
    TRY(launch_ptc_wgrad(g, d, gw, parts, dW1, 1.0, false, st));
    if (!dr) return BSM_OK;
    // dr = L1^dag Gh
    TRY(launch_ptc_adjoint_weights(W1, W1a, 1, C, st));
    a.W = W1a; a.in = Gh; a.out = dr; a.cin = C; a.cout = 1;
    return layer(ctx, d, a, st);
}

bsm_status bsm_precond_apply_collapsed(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                                       int32_t channels, const void *net, const void *r, void *z, void *stream) {
    if (!desc) return fail(BSM_ERR_ARG, "null argument");
    if (desc->link_prec == BSM_F16S) {
        // FP16 links are accepted here: the same checks with F32 links
        bsm_field_desc d32 = *desc;
        d32.link_prec = BSM_F32;
        TRY(check_net_desc(ctx, &d32));
    } else {
        TRY(check_net_desc(ctx, desc));
    }
    if (!U_rep || !net || !r || !z) return fail(BSM_ERR_ARG, "null pointer");
    if (channels < 1 || channels > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    if (r == z) return fail(BSM_ERR_ARG, "r and z must differ");
    if (!net_fast_supported(desc->d_R)) return fail(BSM_ERR_UNSUPPORTED, "the collapsed network runs for d_R <= 3");
    hipStream_t st = (hipStream_t)stream;
    NetFastArgs a;
    TRY(net_fast_prepare(ctx, desc->d_R, channels, net, U_rep, desc->link_prec, a, st));
    a.in = r;
    a.out = z;
    return launch_net_fast(ctx->g, desc->d_R, a, st);
}

bsm_status bsm_precond_apply_collapsed_noalloc(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                                               int32_t channels, const void *net, const void *r, void *z,
                                               void *stream) {
    if (!desc) return fail(BSM_ERR_ARG, "null argument");
    bsm_field_desc d32 = *desc;
    if (d32.link_prec == BSM_F16S) d32.link_prec = BSM_F32;   // FP16 links accepted, as in the allocating form
    TRY(check_net_desc(ctx, &d32));
    if (!U_rep || !net || !r || !z) return fail(BSM_ERR_ARG, "null pointer");
    if (channels < 1 || channels > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    if (r == z) return fail(BSM_ERR_ARG, "r and z must differ");
    if (!net_fast_supported(desc->d_R)) return fail(BSM_ERR_UNSUPPORTED, "the collapsed network runs for d_R <= 3");
    const size_t need = net_fast_bytes(ctx->g, desc->d_R);
    if (need > kNoallocScratchBytes)
        return fail(BSM_ERR_ARG, "lattice needs " + std::to_string(need) + " bytes of network scratch, more than the " +
                                     std::to_string(kNoallocScratchBytes) + " of the static array");
    int cur = -1;
    BSM_HIP(hipGetDevice(&cur));
    if (cur != ctx->device) return fail(BSM_ERR_ARG, "the context belongs to another device");
    void *ptr = nullptr;
    TRY(noalloc_scratch(ctx->device, &ptr));
    hipStream_t st = (hipStream_t)stream;
    NetFastArgs a{};
    a.U = U_rep;
    a.link_prec = desc->link_prec;
    net_fast_carve(ctx->g, desc->d_R, ptr, a);
    TRY(launch_net_collapse(net, channels, a, st));
    a.in = r;
    a.out = z;
    return launch_net_fast(ctx->g, desc->d_R, a, st);
}

bsm_status bsm_precond_train(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t channels,
                             void *net, void *adam_state, const void *r_pairs, const void *e_pairs, int32_t n_pairs,
                             const bsm_train_params *prm, float *losses, void *stream) {
    TRY(check_net_desc(ctx, desc));
    if (!U_rep || !net || !adam_state || !r_pairs || !e_pairs || !prm) return fail(BSM_ERR_ARG, "null pointer");
    if (channels < 1 || channels > 64 || n_pairs < 1 || prm->batch < 1 || prm->steps < 0)
        return fail(BSM_ERR_ARG, "bad channels, n_pairs, batch or steps");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = ctx->g;
    const int d = desc->d_R, C = channels;
    const size_t f32 = 2 * spinor_block_bytes(BSM_F32, d, g.Vh_pad);
    const size_t nw1 = layer_weights(1, C), nw2 = layer_weights(C, 1), nw = nw1 + nw2;
    const size_t parts_bytes = (size_t)ptc_wgrad_blocks(g) * std::max(nw1, nw2) * sizeof(double2);
    // scratch: h (C fields), y, Gy, Gh (C fields), W2 adjoint, grads, partials
    const size_t need = (2 * C + 2) * f32 + nw2 * sizeof(float2) + nw * sizeof(float2) + parts_bytes + 8 * 256;
    void *work = nullptr;
    TRY(ctx_work(ctx, need, &work));
    char *w = (char *)work;
    auto take = [&](size_t bytes) { char *r = w; w += (bytes + 255) / 256 * 256; return r; };
    char *h = take(C * f32), *y = take(f32), *Gy = take(f32), *Gh = take(C * f32);
    float2 *W2a = (float2 *)take(nw2 * sizeof(float2));
    float2 *grad = (float2 *)take(nw * sizeof(float2));
    double2 *parts = (double2 *)take(parts_bytes);
    float2 *W1 = (float2 *)net, *W2 = W1 + nw1;
    // |e|^2 of every pair, once
    std::vector<double> e2(n_pairs);
    Vec none{nullptr, BSM_F32};
    for (int k = 0; k < n_pairs; k++) {
        TRY(blas_dot(g, d, 2, Vec{(char *)e_pairs + k * f32, BSM_F32}, none, ctx->partials, st));
        e2[k] = reduce_to_host(ctx, ctx->partials, blas_blocks(g, 2), st);
        if (!(e2[k] > 0)) return fail(BSM_ERR_ARG, "a training error field is zero");
    }
    for (int step = 0; step < prm->steps; step++) {
        BSM_HIP(hipMemsetAsync(grad, 0, nw * sizeof(float2), st));
        TRY(launch_ptc_adjoint_weights(W2, W2a, C, 1, st));
        double loss = 0;
        for (int bidx = 0; bidx < prm->batch; bidx++) {
            const uint64_t pick = splitmix64(prm->seed + (uint64_t)step * prm->batch + bidx) % (uint64_t)n_pairs;
            const char *r = (const char *)r_pairs + pick * f32;
            const char *e = (const char *)e_pairs + pick * f32;
            TRY(net_apply(ctx, desc, U_rep, C, net, r, h, y, st));
            // Gy = 2 (y - e) / (|e|^2 B); loss term |Gy|^2 |e|^2 B / 4
            const double c = 2.0 / (e2[pick] * prm->batch);
            TRY(blas_axpby(g, d, 2, Vec{Gy, BSM_F32}, c, Vec{y, BSM_F32}, -c, Vec{(void *)e, BSM_F32}, ctx->partials, st));
            const double g2 = reduce_to_host(ctx, ctx->partials, blas_blocks(g, 2), st);
            loss += g2 * e2[pick] * prm->batch / 4.0;
            PtcArgs a{};
            a.U = U_rep;
            // dW2 += Gy conj(T h)
            a.in = h; a.G = Gy; a.cin = C; a.cout = 1;
            TRY(launch_ptc_wgrad(g, d, a, parts, grad + nw1, 1.0, true, st));
            // Gh = L2^dag Gy
            PtcArgs b{};
            b.U = U_rep; b.W = W2a; b.in = Gy; b.out = Gh; b.cin = 1; b.cout = C;
            TRY(layer(ctx, d, b, st));
            // dW1 += Gh conj(T r)
            a.in = r; a.G = Gh; a.cin = 1; a.cout = C;
            TRY(launch_ptc_wgrad(g, d, a, parts, grad, 1.0, true, st));
        }
        if (losses) losses[step] = (float)loss;
        if (!std::isfinite(loss)) return fail(BSM_ERR_NONFINITE, "non-finite training loss");
        TRY(launch_adam(net, grad, adam_state, (int)nw, prm->lr, prm->beta1, prm->beta2, prm->eps,
                        prm->step0 + step + 1, st));
    }
    BSM_HIP(hipStreamSynchronize(st));
    return BSM_OK;
}

bsm_status bsm_precond_pairs(bsm_ctx ctx, const bsm_field_desc *desc64, const void *U_rep64, double kappa,
                             int32_t n_solves, const void *x_star, int32_t n_snap, const int32_t *iters,
                             void *r_out, void *e_out, void *stream) {
    if (!ctx || !desc64 || !U_rep64 || !x_star || !iters || !r_out || !e_out) return fail(BSM_ERR_ARG, "null pointer");
    if (desc64->prec != BSM_F64 || desc64->link_prec != BSM_F64) return fail(BSM_ERR_ARG, "pairs need F64 desc");
    if (n_solves < 1 || n_snap < 1) return fail(BSM_ERR_ARG, "n_solves and n_snap must be >= 1");
    for (int q = 0; q < n_snap; q++)
        if (iters[q] < 0) return fail(BSM_ERR_ARG, "snapshot iterations must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = ctx->g;
    const int d = desc64->d_R;
    const size_t f64 = 2 * spinor_block_bytes(BSM_F64, d, g.Vh_pad);
    const size_t f32 = 2 * spinor_block_bytes(BSM_F32, d, g.Vh_pad);
    void *bx = nullptr;
    // b, x_k and e in FP64, in the FGCR scratch slot (the CG solves below use
    // the solvers' slot)
    TRY(ctx_work_slot(ctx, 1, 3 * f64, &bx));
    char *b = (char *)bx, *xk = b + f64, *e = xk + f64;
    bsm_status status = BSM_OK;
    for (int s = 0; s < n_solves && status == BSM_OK; s++) {
        const char *xs = (const char *)x_star + s * f64;
        status = bsm_dslash_apply(ctx, desc64, U_rep64, kappa, 0, xs, b, stream);
        for (int q = 0; q < n_snap && status == BSM_OK; q++) {
            if (iters[q] == 0) {
                // the start of the solve: x_0 = 0, e = x*
                if (hipMemsetAsync(xk, 0, f64, st) != hipSuccess) { status = fail(BSM_ERR_HIP, "memset"); break; }
            } else {
                bsm_solver_params p{};
                p.variant = BSM_SOLVER_PLAIN; p.schur = 1; p.kappa = kappa; p.tol = 1e-30;
                p.max_iter = iters[q]; p.check_every = 1 << 20;
                bsm_solver_stats sst{};
                bsm_status cs = bsm_cg_solve(ctx, desc64, U_rep64, U_rep64, &p, b, xk, &sst, stream);
                if (cs != BSM_OK && cs != BSM_ERR_NOT_CONVERGED) { status = cs; break; }
            }
            // e = x* - x_k ; r = D e  (F32 copies)
            Vec E{e, BSM_F64};
            status = blas_axpby(g, d, 2, E, 1.0, Vec{(void *)xs, BSM_F64}, -1.0, Vec{xk, BSM_F64}, nullptr, st);
            if (status != BSM_OK) break;
            const size_t k = (size_t)s * n_snap + q;
            status = blas_axpby(g, d, 2, Vec{(char *)e_out + k * f32, BSM_F32}, 1.0, E, 0.0,
                                Vec{nullptr, BSM_F64}, nullptr, st);
            if (status != BSM_OK) break;
            status = bsm_dslash_apply(ctx, desc64, U_rep64, kappa, 0, e, xk, stream);
            if (status != BSM_OK) break;
            status = blas_axpby(g, d, 2, Vec{(char *)r_out + k * f32, BSM_F32}, 1.0, Vec{xk, BSM_F64}, 0.0,
                                Vec{nullptr, BSM_F64}, nullptr, st);
        }
    }
    (void)hipStreamSynchronize(st);
    return status;
}

bsm_status bsm_fgcr_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, const void *U_rep64,
                          const bsm_solver_params *prm, int32_t channels, const void *net, const void *bin,
                          void *xout, bsm_solver_stats *stats, void *stream) {
    if (stats) *stats = bsm_solver_stats{};
    if (!ctx || !desc || !prm || !bin || !xout || !stats || !U_rep || !U_rep64) return fail(BSM_ERR_ARG, "null argument");
    if (bsm_rep_dim(desc->N, desc->rep) != desc->d_R) return fail(BSM_ERR_ARG, "d_R does not match (N, rep)");
    if (desc->prec != BSM_F32 || desc->link_prec != BSM_F32)
        return fail(BSM_ERR_ARG, "the inner GCR runs on F32 spinors and F32 links");
    if (net) {
        TRY(check_net_desc(ctx, desc));
        if (channels < 1 || channels > 64) return fail(BSM_ERR_ARG, "channels must be in [1, 64]");
    }
    if (!(prm->kappa > 0) || !(prm->tol > 0) || prm->max_iter < 1) return fail(BSM_ERR_ARG, "kappa, tol, max_iter");
    const int m = prm->restart > 0 ? prm->restart : 16;
    if (m > kGcrMax) return fail(BSM_ERR_ARG, "restart must be <= 64");
    if (bin == xout) return fail(BSM_ERR_ARG, "b and x must differ");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = ctx->g;
    const int d = desc->d_R;
    bsm_field_desc d64 = *desc;
    d64.prec = BSM_F64;
    d64.link_prec = BSM_F64;
    const size_t f64 = 2 * spinor_block_bytes(BSM_F64, d, g.Vh_pad);
    const size_t f32 = 2 * spinor_block_bytes(BSM_F32, d, g.Vh_pad);
    const size_t n = f32 / sizeof(float2);
    const ZLive lv{FastDiv((uint32_t)g.Vh_pad), (uint32_t)g.Vh};
    const int nb = (int)std::min<size_t>((n + 255) / 256, kZblocks);
    auto t0 = std::chrono::steady_clock::now();
    // the context's second scratch: the fall back CG uses the first
    const bool fast = net && prm->precond_layers == 0 && net_fast_supported(d);
    // the collapsed network reads FP16 copies of the links (converted once per solve)
    const size_t l16 = fast ? 8 * link_block_bytes(BSM_F16S, false, d, g.Vh_pad) : 0;
    const size_t need = (2 * (size_t)m + 2) * f32 + 2 * f64 + (net && !fast ? (size_t)channels * f32 : 0) + l16 +
                        (size_t)kGcrMax * nb * sizeof(double2) + 4 * kGcrMax * sizeof(double2) +
                        kZblocks * sizeof(double) + 18 * 256;
    void *work = nullptr;
    TRY(ctx_work_slot(ctx, 1, need, &work));
    char *w = (char *)work;
    auto take = [&](size_t bytes) { char *r = w; w += (bytes + 255) / 256 * 256; return r; };
    ZPtrs Zp{}, Wp{};
    std::vector<char *> Z(m), Wv(m);
    for (int k = 0; k < m; k++) {
        Z[k] = take(f32);
        Wv[k] = take(f32);
        Zp.p[k] = (const float2 *)Z[k];
        Wp.p[k] = (const float2 *)Wv[k];
    }
    char *rho = take(f32), *e = take(f32);
    char *h32 = net && !fast ? take((size_t)channels * f32) : nullptr;
    NetFastArgs fa{};
    if (fast) {
        char *U16 = take(l16);
        TRY(launch_convert_links(g, d, false, BSM_F32, BSM_F16S, U_rep, U16, st));
        TRY(net_fast_prepare(ctx, d, channels, net, U16, BSM_F16S, fa, st));
    }
    char *r = take(f64), *t = take(f64);
    double2 *parts = (double2 *)take((size_t)kGcrMax * nb * sizeof(double2));
    double2 *coef = (double2 *)take(4 * kGcrMax * sizeof(double2));
    double *nn = (double *)(coef + kGcrMax);          // kGcrMax doubles
    double *rrp = (double *)take(kZblocks * sizeof(double));   // per-workgroup |rho|^2
    // pinned: two slots of kZblocks partials, the upper half of the context's mirror
    double *host_rr = ctx->host_scal + kScalars / 2;
    static_assert(2 * kZblocks <= kScalars / 2, "host partial slots");
    hipEvent_t ev[2] = {nullptr, nullptr};
    BSM_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    BSM_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    const char *b = (const char *)bin;
    char *x = (char *)xout;
    const Vec none{nullptr, BSM_F64};
    auto norm64 = [&](const void *v, double *out) -> bsm_status {
        TRY(blas_dot(g, d, 2, Vec{(void *)v, BSM_F64}, none, ctx->partials, st));
        *out = reduce_to_host(ctx, ctx->partials, blas_blocks(g, 2), st);
        return BSM_OK;
    };
    // FP64: r = b - D x, |r|^2
    auto residual = [&](double *out) -> bsm_status {
        TRY(bsm_dslash_apply(ctx, &d64, U_rep64, prm->kappa, 0, x, t, stream));
        TRY(blas_axpby(g, d, 2, Vec{r, BSM_F64}, 1.0, Vec{(void *)b, BSM_F64}, -1.0, Vec{t, BSM_F64}, nullptr, st));
        return norm64(r, out);
    };
    // one FP32 GCR step on D e = rho with direction k
    auto step = [&](int k) -> bsm_status {
        if (fast) {
            fa.in = rho;
            fa.out = Z[k];
            TRY(launch_net_fast(g, d, fa, st));
        } else if (net) {
            TRY(net_apply(ctx, desc, U_rep, channels, net, rho, h32, Z[k], st));
        } else {
            BSM_HIP(hipMemcpyAsync(Z[k], rho, f32, hipMemcpyDeviceToDevice, st));
        }
        TRY(bsm_dslash_apply(ctx, desc, U_rep, prm->kappa, 0, Z[k], Wv[k], stream));
        if (k > 0) {
            k_zmultidot<<<dim3(nb, (k + kZdotJ - 1) / kZdotJ), 256, 0, st>>>(Wp, k, (const float2 *)Wv[k], n, lv, parts);
            k_zcols<<<k, 256, 0, st>>>(parts, nb, nn, coef);
        }
        k_zorth<<<nb, 256, 0, st>>>(Wp, Zp, k, coef, (float2 *)Wv[k], (float2 *)Z[k], (const float2 *)rho, n, lv, parts);
        k_zupdate<<<nb, 256, 0, st>>>((float2 *)e, (float2 *)rho, (const float2 *)Z[k], (const float2 *)Wv[k], n, lv,
                                      parts, nb, nn, k, rrp);
        BSM_HIP(hipGetLastError());
        // the workgroup partials of |rho|^2 to a pinned slot; the host sums
        // them one step later, so the next step is already queued meanwhile
        BSM_HIP(hipMemcpyAsync(host_rr + (k & 1) * kZblocks, rrp, nb * sizeof(double), hipMemcpyDeviceToHost, st));
        BSM_HIP(hipEventRecord(ev[k & 1], st));
        return BSM_OK;
    };

    bsm_status status = BSM_OK;
    double bn2 = 0, r2 = 0;
    int it = 0, cycles = 0, applies = 0;
    bool fallback = false;
    hipError_t he = hipMemsetAsync(x, 0, f64, st);
    if (he != hipSuccess) status = hip_check(he, "fgcr init");
    if (status == BSM_OK) status = norm64(b, &bn2);
    if (status == BSM_OK && !std::isfinite(bn2)) status = fail(BSM_ERR_NONFINITE, "non-finite right-hand side");
    const double tol2 = prm->tol * prm->tol * bn2;
    if (status == BSM_OK && bn2 > 0) status = residual(&r2);
    while (status == BSM_OK && bn2 > 0 && it < prm->max_iter) {
        if (!std::isfinite(r2)) { fallback = true; break; }
        if (r2 <= tol2) break;
        const double r2_cycle = r2;
        // inner FP32 cycle on the correction: D e = r, e = 0
        status = blas_axpby(g, d, 2, Vec{rho, BSM_F32}, 1.0, Vec{r, BSM_F64}, 0.0, none, nullptr, st);
        if (status == BSM_OK && hipMemsetAsync(e, 0, f32, st) != hipSuccess) status = fail(BSM_ERR_HIP, "memset");
        for (int k = 0; status == BSM_OK && k < m && it < prm->max_iter; k++) {
            if ((status = step(k)) != BSM_OK) break;
            if (net) applies++;
            it++;
            if (k > 0) {
                // the previous step's residual (this step runs meanwhile and is kept)
                if (hipEventSynchronize(ev[(k - 1) & 1]) != hipSuccess) { status = fail(BSM_ERR_HIP, "event"); break; }
                double rk = 0;
                for (int i = 0; i < nb; i++) rk += host_rr[((k - 1) & 1) * kZblocks + i];
                if (!std::isfinite(rk) || rk <= tol2) break;
            }
        }
        if (status != BSM_OK) break;
        cycles++;
        // x += e in FP64 and the restart residual from scratch
        if ((status = blas_axpby(g, d, 2, Vec{x, BSM_F64}, 1.0, Vec{x, BSM_F64}, 1.0, Vec{e, BSM_F32}, nullptr, st)) !=
            BSM_OK)
            break;
        if ((status = residual(&r2)) != BSM_OK) break;
        if (r2 <= tol2) break;
        if (!std::isfinite(r2) || (it < prm->max_iter && r2 > 0.25 * r2_cycle)) { fallback = true; break; }
    }
    if (status == BSM_OK && fallback) {
        // plain FP64 Schur CG on D c = r from the current x, then x += c
        bsm_solver_params p = *prm;
        p.variant = BSM_SOLVER_PLAIN;
        p.schur = 1;
        if (std::isfinite(r2) && r2 > 0) {
            p.tol = prm->tol * std::sqrt(bn2 / r2);
        } else {
            he = hipMemsetAsync(x, 0, f64, st);
            if (he == hipSuccess) he = hipMemcpyAsync(r, b, f64, hipMemcpyDeviceToDevice, st);
            if (he != hipSuccess) status = hip_check(he, "fgcr fall back");
            p.tol = prm->tol;
        }
        p.max_iter = std::max(1, prm->max_iter - it);
        bsm_solver_stats cs{};
        if (status == BSM_OK) {
            const bsm_status s2 = bsm_cg_solve(ctx, &d64, U_rep64, U_rep64, &p, r, t, &cs, stream);
            it += cs.iters;
            if (s2 == BSM_OK || s2 == BSM_ERR_NOT_CONVERGED) {
                status = blas_axpby(g, d, 2, Vec{x, BSM_F64}, 1.0, Vec{x, BSM_F64}, 1.0, Vec{t, BSM_F64}, nullptr, st);
                if (status == BSM_OK) status = residual(&r2);
            } else {
                status = s2;
            }
        }
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    stats->iters = it;
    stats->restarts = cycles;
    stats->fell_back = fallback ? 1 : 0;
    stats->precond_applies = applies;
    stats->true_rel_res = bn2 > 0 ? std::sqrt(r2 / bn2) : 0.0;
    stats->converged = status == BSM_OK && stats->true_rel_res <= prm->tol;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (status != BSM_OK) return status;
    if (!stats->converged) return fail(BSM_ERR_NOT_CONVERGED, "fgcr: max_iter reached before tol");
    return BSM_OK;
}

}  // extern "C"
