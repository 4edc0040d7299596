// FP64 multi-RHS hop on FP64 matrix cores, for the reliable updates of the
// batched solver: the FP64 normal residual of all 16 right-hand sides shares
// every link load, as the FP32 recurrence does.
//
// Same scheme as the FP32 block hop (one wavefront per site, the d x d real
// link times the d x 64 block of projected half spinors), with
// v_mfma_f64_16x16x4f64, whose operands are laid out like the FP32 ones
// (A: lane l -> A[l%16][l/16], B: lane l -> B[l/16][l%16]) but whose result
// rows are interleaved differently: lane l holds D[l/16 + 4v][l%16], v < 4.
// FP64 block fields: [h][colour][spin][rhs] double2; FP64 block links:
// [q][mu][h][i*d + j] double.
#include "block.h"
#include "dispatch.h"
#include "spinor_io.h"

namespace bsm {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int MU>
__device__ inline void project_d(const double2 (&s)[4], double sg, double2 &h0, double2 &h1) {
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

template <int MU>
__device__ inline void reconstruct_d(d4 (&acc)[4][2], double sg, double w, d4 g0r, d4 g0i, d4 g1r, d4 g1i) {
    const double v = -sg * w;
    acc[0][0] += w * g0r; acc[0][1] += w * g0i;
    acc[1][0] += w * g1r; acc[1][1] += w * g1i;
    if constexpr (MU == 0) {
        acc[2][0] += v * g0r; acc[2][1] += v * g0i;
        acc[3][0] += v * g1r; acc[3][1] += v * g1i;
    } else if constexpr (MU == 1) {
        acc[2][0] -= v * g1i; acc[2][1] += v * g1r;
        acc[3][0] -= v * g0i; acc[3][1] += v * g0r;
    } else if constexpr (MU == 2) {
        acc[2][0] += v * g1r; acc[2][1] += v * g1i;
        acc[3][0] -= v * g0r; acc[3][1] -= v * g0i;
    } else {
        acc[2][0] -= v * g0i; acc[2][1] += v * g0r;
        acc[3][0] += v * g1i; acc[3][1] -= v * g1r;
    }
}

template <int MU, int D>
__device__ inline void hop_dir_block64(const Geom &g, const BlockHop64Args &a, const Coords &c, int p, uint32_t h,
                                       int r, int q, double eta, d4 (&acc)[4][2]) {
    constexpr int KB = (D + 3) / 4;
    constexpr size_t SITE = (size_t)D * 4 * kNR;
    // one direction at a time: its operands alone fill the register budget
#pragma unroll 1
    for (int dir = 0; dir < 2; dir++) {
        const bool back = dir == 1;
        float wf;
        const uint32_t hn = neighbour<MU>(g, c, back, wf);
        const double2 *sp = a.in[p] + (size_t)hn * SITE;
        double2 sv[KB][4];
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            const int cc = q + 4 * kb;
#pragma unroll
            for (int si = 0; si < 4; si++) sv[kb][si] = cc < D ? sp[(cc * 4 + si) * kNR + r] : make_double2(0.0, 0.0);
        }
        const double *L = a.U + ((size_t)((back ? 1 - p : p) * 4 + MU) * g.Vh_pad + (back ? hn : h)) * (D * D);
        double A[KB];
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            const int k = q + 4 * kb;
            A[kb] = (r < D && k < D) ? __builtin_nontemporal_load(L + (back ? k * D + r : r * D + k)) : 0.0;
        }
        const double sg = back ? -eta : eta;
        d4 g0r = {0.0, 0.0, 0.0, 0.0}, g0i = g0r, g1r = g0r, g1i = g0r;
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            double2 h0, h1;
            project_d<MU>(sv[kb], sg, h0, h1);
            g0r = __builtin_amdgcn_mfma_f64_16x16x4f64(A[kb], h0.x, g0r, 0, 0, 0);
            g0i = __builtin_amdgcn_mfma_f64_16x16x4f64(A[kb], h0.y, g0i, 0, 0, 0);
            g1r = __builtin_amdgcn_mfma_f64_16x16x4f64(A[kb], h1.x, g1r, 0, 0, 0);
            g1i = __builtin_amdgcn_mfma_f64_16x16x4f64(A[kb], h1.y, g1i, 0, 0, 0);
        }
        reconstruct_d<MU>(acc, sg, (double)wf, g0r, g0i, g1r, g1i);
    }
}

// 4 sites per 256-thread workgroup, one per wavefront; the register budget
// is capped so that two wavefronts per SIMD overlap their loads
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_hop_block64(Geom g, BlockHop64Args a, int nblk) {
    constexpr size_t SITE = (size_t)D * 4 * kNR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const uint32_t lb = xcd_chunk_remap(blockIdx.x, gridDim.x, (uint32_t)a.xchunk);
    const int pi = lb >= (uint32_t)nblk ? 1 : 0;
    const uint32_t s = (lb - pi * nblk) * 4 + wave;
    const int p = a.p0 + pi;
    if (s >= (uint32_t)g.Vh) return;
    const uint32_t h = block_site(g, a.tile, s);
    d4 acc[4][2];
#pragma unroll
    for (int s = 0; s < 4; s++) acc[s][0] = acc[s][1] = d4{0.0, 0.0, 0.0, 0.0};
    const Coords c = decode(g, h, p);
    const double eta = a.dagger ? -1.0 : 1.0;
    hop_dir_block64<0, D>(g, a, c, p, h, r, q, eta, acc);
    hop_dir_block64<1, D>(g, a, c, p, h, r, q, eta, acc);
    hop_dir_block64<2, D>(g, a, c, p, h, r, q, eta, acc);
    hop_dir_block64<3, D>(g, a, c, p, h, r, q, eta, acc);
    const double ar = a.a[r], br = a.b[r], cr = a.c[r];
    double2 *o = a.out[p] + (size_t)h * SITE;
    // x (and y) first, every load unconditional (rows i >= D read row D - 1
    // and are not stored): a load inside the divergent i < D test is waited
    // for there
    double2 xv[4][4], yv[4][4];
    if (a.use_x) {
        const double2 *x = a.x[p] + (size_t)h * SITE;
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int s = 0; s < 4; s++) xv[v][s] = x[(size_t)(min(q + 4 * v, D - 1) * 4 + s) * kNR + r];
    }
    if (a.use_y) {
        const double2 *y = a.y[p] + (size_t)h * SITE;
#pragma unroll
        for (int v = 0; v < 4; v++)
#pragma unroll
            for (int s = 0; s < 4; s++) yv[v][s] = y[(size_t)(min(q + 4 * v, D - 1) * 4 + s) * kNR + r];
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int i = q + 4 * v;   // the FP64 result interleave
        if (i < D) {
#pragma unroll
            for (int s = 0; s < 4; s++) {
                const size_t e = (size_t)(i * 4 + s) * kNR + r;
                double re = br * acc[s][0][v], im = br * acc[s][1][v];
                if (a.use_x) {
                    re = fma(ar, xv[v][s].x, re);
                    im = fma(ar, xv[v][s].y, im);
                }
                if (a.use_y) {
                    re = fma(cr, yv[v][s].x, re);
                    im = fma(cr, yv[v][s].y, im);
                }
                o[e] = make_double2(re, im);
            }
        }
    }
}

template <int D>
struct BlockHop64ByD {
    static bsm_status run(const Geom &g, const BlockHop64Args &a, hipStream_t st) {
        if constexpr (D == 3 || D == 8 || D == 15) {
            const int nblk = (g.Vh + 3) / 4;
            k_hop_block64<D><<<nblk * a.np, 256, 0, st>>>(g, a, nblk);
            BSM_HIP(hipGetLastError());
            return BSM_OK;
        }
        return fail(BSM_ERR_UNSUPPORTED, "block hop: real links exist only for d_R = 3, 8, 15");
    }
};

bsm_status launch_hop_block64(const Geom &g, int d, const BlockHop64Args &a, hipStream_t st) {
    return dispatch_d<BlockHop64ByD>(d, g, a, st);
}

// --------------------------------------------------------------- layouts
// 32 sites per workgroup, transposed through LDS as for the FP32 block links
template <int LP>
__global__ __launch_bounds__(256) void k_gauge_to_block64(Geom g, int d, const char *src, double *dst) {
    constexpr int S = 32;
    __shared__ double t[S * 225];
    const uint32_t h0 = blockIdx.x * S;
    const int qm = blockIdx.y;
    const int dd = d * d, ldt = dd | 1;   // odd row stride: no LDS bank conflicts
    const int ns = min(S, (int)((uint32_t)g.Vh_pad - h0));
    const char *blk = src + (size_t)qm * link_block_bytes(LP, true, d, g.Vh_pad);
    for (int idx = threadIdx.x; idx < S * dd; idx += 256) {
        const int e = idx / S, s = idx - e * S;
        if (s < ns) t[s * ldt + e] = load_link<LP, true, double>(blk, g.Vh_pad, e, h0 + s).re;
    }
    __syncthreads();
    double *o = dst + ((size_t)qm * g.Vh_pad + h0) * dd;
    for (int idx = threadIdx.x; idx < ns * dd; idx += 256) o[idx] = t[(idx / dd) * ldt + idx % dd];
}

bsm_status launch_gauge_to_block64(const Geom &g, int d, const void *U_rep64, double *U_block, hipStream_t st) {
    if (d > 15) return fail(BSM_ERR_ARG, "block links: d_R above 15");
    dim3 grid((g.Vh_pad + 31) / 32, 8);
    k_gauge_to_block64<BSM_F64><<<grid, 256, 0, st>>>(g, d, (const char *)U_rep64, U_block);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// element e of one FP64 parity block: r = e % 16, (h, c, s) from e / 16
// mode 0: block = std parity block of RHS r (r < n_rhs; zero for r >= n_rhs)
// mode 1: block32[e] = (float) block[e] for the RHS selected in sel
// block32 = (float) block for the RHS selected in sel (same layout)
__global__ __launch_bounds__(256) void k_block64_to32(Geom g, int d, int n_rhs, unsigned sel, const double2 *block,
                                                      float2 *block32) {
    const size_t n = (size_t)g.Vh_pad * d * 4 * kNR;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        const int r = (int)(e % kNR);
        if (r < n_rhs && ((sel >> r) & 1u)) {
            const double2 v = block[e];
            block32[e] = make_float2((float)v.x, (float)v.y);
        }
    }
}

bsm_status launch_block64_io(const Geom &g, int d, int n_rhs, unsigned sel, const char *std64, size_t std_stride,
                             size_t std_off, double2 *block, float2 *block32, int mode, hipStream_t st) {
    if (mode != 1)   // layout changes go through the LDS transpose
        return launch_block64_std(g, d, n_rhs, sel, const_cast<char *>(std64), std_stride, std_off, block,
                                  mode == 0 ? 0 : 2, st);
    const size_t n = (size_t)g.Vh_pad * d * 4 * kNR;
    size_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    k_block64_to32<<<(int)nb, 256, 0, st>>>(g, d, n_rhs, sel, block, block32);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

// padding sites (h >= Vh) are skipped: operator outputs never write them
__global__ __launch_bounds__(256) void k_block64_norm(size_t n, size_t live, const double2 *v, double *partials) {
    double nrm = 0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
        if (e >= live) break;
        const double2 t = v[e];
        nrm += t.x * t.x + t.y * t.y;
    }
    nrm += __shfl_xor(nrm, 16, 64);
    nrm += __shfl_xor(nrm, 32, 64);
    __shared__ double ws[4][kNR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < kNR) ws[wave][lane] = nrm;
    __syncthreads();
    if (threadIdx.x < kNR)
        partials[(size_t)blockIdx.x * kNR + threadIdx.x] =
            (ws[0][threadIdx.x] + ws[1][threadIdx.x]) + (ws[2][threadIdx.x] + ws[3][threadIdx.x]);
}

// dst[r] = sum over nparts workgroups (fixed order), one workgroup
__global__ __launch_bounds__(256) void k_block64_total(const double *partials, int nparts, double *dst) {
    const int r = threadIdx.x % kNR, grp = threadIdx.x / kNR;
    double s = 0;
    for (int i = grp; i < nparts; i += 16) s += partials[(size_t)i * kNR + r];
    __shared__ double ws[16][kNR];
    ws[grp][r] = s;
    __syncthreads();
    if (threadIdx.x >= kNR) return;
    double tot = 0;
    for (int k = 0; k < 16; k++) tot += ws[k][r];
    dst[r] = tot;
}

static int block64_grid(const Geom &g, int d) {
    const size_t n = (size_t)g.Vh_pad * d * 4 * kNR;
    size_t nb = (n + 255) / 256;
    return (int)(nb < 4096 ? nb : 4096);
}

bsm_status block64_norms(const Geom &g, int d, const double2 *v, double *partials, double *dst, hipStream_t st) {
    const int nb = block64_grid(g, d);
    k_block64_norm<<<nb, 256, 0, st>>>((size_t)g.Vh_pad * d * 4 * kNR, (size_t)g.Vh * d * 4 * kNR, v, partials);
    k_block64_total<<<1, 256, 0, st>>>(partials, nb, dst);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}

int block64_norm_parts(const Geom &g, int d) { return block64_grid(g, d); }

}  // namespace bsm
