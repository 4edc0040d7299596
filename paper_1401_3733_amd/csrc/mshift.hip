// One Krylov space for a family of masses (Section II.B's inversion, for many
// kappa at once).  D(kappa) = 1 - kappa H = kappa (sigma - H) with
// sigma = 1/kappa, so the systems (sigma_i - H) y_i = b, x_i = y_i / kappa_i,
// differ only by a multiple of the identity: they share the Krylov space of
// H and b, and one sequence of operator applications serves all of them.
//
// The seed is the hardest member (largest kappa, smallest sigma_0); the
// others are shifted by delta_i = sigma_i - sigma_0 >= 0.  The iteration is
// BiCG with the shadow sequence gamma5 times the primal one, which is valid
// because A = sigma_0 - H satisfies A^dag = gamma5 A gamma5: the shadow
// recurrences then reproduce gamma5 r_n and gamma5 p_n exactly, all
// coefficients are real (r^dag gamma5 r and p^dag gamma5 A p are real), and
// one operator application per iteration suffices.  The residual of shift i
// is zeta_i r_n, with zeta from the three-term recurrence of the residual
// polynomials evaluated at -delta_i:
//   zeta_(n+1) = zeta_n zeta_(n-1) a_(n-1) /
//                (a_(n-1) zeta_(n-1) (1 + delta a_n) + a_n b_(n-1) (zeta_(n-1) - zeta_n)),
//   a_n^i = a_n zeta_(n+1) / zeta_n,  b_n^i = b_n (zeta_(n+1) / zeta_n)^2,
//   x^i += a_n^i p^i,  p^i = zeta_(n+1) r_(n+1) + b_n^i p^i.
// The member vectors are not touched every iteration: x_i and p_i are linear
// combinations of the seed's residuals, so the last L residuals are kept (a
// ring of L + 1 fields) and each member carries, on the host, its
// coefficients on p_i and x_i as they stood at the start of the chunk and on
// those residuals; every L iterations (and at the end) one pass forms
// x_i += cx0 p_i + sum_k cx_k r_k and p_i = cp0 p_i + sum_k cp_k r_k for all
// members.  That reads the L residuals once per chunk instead of reading and
// writing 2 n member fields every iteration; the seed's own direction, which
// the operator needs every iteration, is kept explicitly.
// Shift i retires once |zeta_i| |r| <= (the caller's delta) tol |b|; afterwards every x_i is
// divided by kappa_i and judged by its FP64 true residual ||b - D(kappa_i) x_i||
// / ||b||; a member that misses tol (or a breakdown, a non-finite value) is
// finished by plain FP64 Schur CG.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "blas.h"
#include "block.h"
#include "dispatch.h"
#include "solver.h"
#include "spinor_io.h"

namespace bsm {

constexpr int kMaxShifts = 32;
constexpr int kMsBlocks = 16384;   // reduction workgroups (grid-stride beyond)
constexpr int kMsChunk = 16;       // iterations between member updates (at most)
constexpr int kMsCoefRow = 2 * (kMsChunk + 2);   // per member: cx0, cx[0..L], cp0, cp[0..L]

struct MsGeom {
    size_t n;        // complex elements of a full FP64 field (incl. padding)
    uint32_t Vh, Vh_pad, planes;   // planes = 4 d per parity block
};

__device__ inline bool ms_live(const MsGeom &m, size_t e, double &g5) {
    const uint32_t h = (uint32_t)(e % m.Vh_pad);
    const uint32_t c = (uint32_t)((e / m.Vh_pad) % m.planes);
    g5 = c < m.planes / 2 ? 1.0 : -1.0;   // spins 0, 1 then 2, 3 (chiral basis)
    return h < m.Vh;
}

// partials[block] = sum Re conj(a) gamma5 b over live elements
__global__ __launch_bounds__(256) void k_ms_jdot(MsGeom m, const double2 *a, const double2 *b, double *partials) {
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < m.n; e += (size_t)gridDim.x * 256) {
        double g5;
        if (!ms_live(m, e, g5)) continue;
        const double2 x = a[e], y = b[e];
        s = fma(g5, x.x * y.x + x.y * y.y, s);
    }
    const double t = block_sum_256(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// r_out = r - alpha q; partials of r_out^dag gamma5 r_out (first gridDim.x)
// and |r_out|^2 (next)
__global__ __launch_bounds__(256) void k_ms_residual(MsGeom m, const double2 *r, const double2 *q, double alpha,
                                                     double2 *r_out, double *partials) {
    double sj = 0.0, s2 = 0.0;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < m.n; e += (size_t)gridDim.x * 256) {
        double g5;
        if (!ms_live(m, e, g5)) continue;
        double2 x = r[e];
        const double2 y = q[e];
        x.x = fma(-alpha, y.x, x.x);
        x.y = fma(-alpha, y.y, x.y);
        r_out[e] = x;
        const double n2 = x.x * x.x + x.y * x.y;
        sj = fma(g5, n2, sj);
        s2 += n2;
    }
    const double tj = block_sum_256(sj);
    __syncthreads();   // block_sum_256's LDS slots are read by thread 0 before the second sum reuses them
    const double t2 = block_sum_256(s2);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = tj;
        partials[gridDim.x + blockIdx.x] = t2;
    }
}

// One chunk's member updates.  R holds nring residual fields (stride complex
// numbers apart); chunk residual k is field (ring0 + k) % nring, k < nk.  For
// member i (coefficient row coef + i kMsCoefRow: cx0, cx[0..nk), then at
// kMsChunk + 2: cp0, cp[0..nk)):
//   x_i += cx0 p_i + sum_k cx_k r_k   (members in xmask)
//   p_i  = cp0 p_i + sum_k cp_k r_k   (members in pmask)
// The members to touch come as a list; four are loaded together so their
// loads overlap.  The coefficients are read by every lane alike.
struct MsFlushList {
    int n;
    int idx[kMaxShifts];
    uint32_t xmask, pmask;
};

__global__ __launch_bounds__(256) void k_ms_flush(MsGeom m, const double2 *R, size_t stride, int ring0, int nring,
                                                  int nk, double2 *x, double2 *p, MsFlushList L,
                                                  const double *coef) {
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < m.n; e += (size_t)gridDim.x * 256) {
        double g5;
        if (!ms_live(m, e, g5)) continue;
        double2 rv[kMsChunk + 1];
#pragma unroll
        for (int k = 0; k <= kMsChunk; k++)
            if (k < nk) rv[k] = R[(size_t)((ring0 + k) % nring) * stride + e];
        for (int q0 = 0; q0 < L.n; q0 += 4) {
            double2 pv[4], xv[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (q0 + u >= L.n) continue;
                const int i = L.idx[q0 + u];
                pv[u] = p[i * stride + e];
                if ((L.xmask >> i) & 1u) xv[u] = x[i * stride + e];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (q0 + u >= L.n) continue;
                const int i = L.idx[q0 + u];
                const double *c = coef + (size_t)i * kMsCoefRow;
                if ((L.xmask >> i) & 1u) {
                    double2 a = xv[u];
                    a.x = fma(c[0], pv[u].x, a.x);
                    a.y = fma(c[0], pv[u].y, a.y);
#pragma unroll
                    for (int k = 0; k <= kMsChunk; k++)
                        if (k < nk) {
                            a.x = fma(c[1 + k], rv[k].x, a.x);
                            a.y = fma(c[1 + k], rv[k].y, a.y);
                        }
                    x[i * stride + e] = a;
                }
                if ((L.pmask >> i) & 1u) {
                    const double *cq = c + kMsChunk + 2;
                    double2 np = make_double2(cq[0] * pv[u].x, cq[0] * pv[u].y);
#pragma unroll
                    for (int k = 0; k <= kMsChunk; k++)
                        if (k < nk) {
                            np.x = fma(cq[1 + k], rv[k].x, np.x);
                            np.y = fma(cq[1 + k], rv[k].y, np.y);
                        }
                    p[i * stride + e] = np;
                }
            }
        }
    }
}

static int ms_grid(const MsGeom &m) {
    const size_t nb = (m.n + 255) / 256;
    return (int)std::min<size_t>(nb, kMsBlocks);
}

#define TRY(x)                           \
    do {                                 \
        bsm_status _s = (x);             \
        if (_s != BSM_OK) return _s;     \
    } while (0)

static bsm_status ms_sum(bsm_ctx ctx, const double *partials, int n, double *out, hipStream_t st) {
    *out = reduce_to_host(ctx, partials, n, st);
    return BSM_OK;
}

}  // namespace bsm

using namespace bsm;

extern "C" bsm_status bsm_shifted_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep64,
                                        const bsm_solver_params *prm, int32_t n_kappa, const double *kappas,
                                        const void *b, void *x, bsm_solver_stats *stats, void *stream) {
    if (!ctx || !desc || !prm || !kappas || !b || !x || !stats || !U_rep64) return fail(BSM_ERR_ARG, "null argument");
    if (n_kappa < 1 || n_kappa > kMaxShifts) return fail(BSM_ERR_ARG, "n_kappa must be in [1, 32]");
    for (int i = 0; i < n_kappa; i++) stats[i] = bsm_solver_stats{};
    if (bsm_rep_dim(desc->N, desc->rep) != desc->d_R || desc->d_R < 2 || desc->d_R > 15)
        return fail(BSM_ERR_ARG, "d_R does not match (N, rep) or is outside [2, 15]");
    if (desc->prec != BSM_F64 || link_base(desc->link_prec) != BSM_F64)
        return fail(BSM_ERR_ARG, "the shifted solver runs in FP64: desc prec and link_prec must be F64");
    for (int i = 0; i < n_kappa; i++)
        if (!(kappas[i] > 0) || !std::isfinite(kappas[i])) return fail(BSM_ERR_ARG, "kappas must be finite and > 0");
    if (!(prm->tol > 0) || prm->max_iter < 1) return fail(BSM_ERR_ARG, "tol > 0 and max_iter >= 1 required");
    if (b == x) return fail(BSM_ERR_ARG, "b and x must differ");
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const Geom &g = ctx->g;
    const int d = desc->d_R, n = n_kappa;
    const size_t bb = spinor_block_bytes(BSM_F64, d, g.Vh_pad), full = 2 * bb;
    MsGeom m;
    m.n = full / sizeof(double2);
    m.Vh = (uint32_t)g.Vh;
    m.Vh_pad = (uint32_t)g.Vh_pad;
    m.planes = 4 * d;
    // shifts relative to the seed (the largest kappa)
    int seed = 0;
    for (int i = 1; i < n; i++)
        if (kappas[i] > kappas[seed]) seed = i;
    const double sigma0 = 1.0 / kappas[seed];
    std::vector<double> delta(n);
    for (int i = 0; i < n; i++) delta[i] = 1.0 / kappas[i] - sigma0;
    // scratch: A p, the full-lattice residual field, the seed's explicit
    // direction, a ring of L + 1 residuals, one p per shift and the member
    // coefficients; L shrinks when the device cannot hold the ring
    const size_t coef_bytes = (size_t)n * kMsCoefRow * sizeof(double);
    int L = kMsChunk;
    void *work = nullptr;
    size_t work_bytes = 0;
    for (;;) {
        work_bytes = (3 + (size_t)L + 1 + n) * full + (coef_bytes + 255) / 256 * 256;
        const bsm_status ws = ctx_work(ctx, work_bytes, &work);
        if (ws == BSM_OK) break;
        (void)hipGetLastError();   // the failed allocation's error is not this solve's
        if (L == 1) return ws;
        L /= 2;
    }
    char *Ap = (char *)work, *tfull = Ap + full, *Pd = tfull + full, *R = Pd + full;
    char *P = R + (size_t)(L + 1) * full;
    double *dcoef = (double *)(P + (size_t)n * full);
    char *X = (char *)x;
    const Vec none{nullptr, BSM_F64};
    BSM_HIP(hipMemsetAsync(X, 0, (size_t)n * full, st));
    BSM_HIP(hipMemcpyAsync(R, b, full, hipMemcpyDeviceToDevice, st));
    BSM_HIP(hipMemcpyAsync(Pd, b, full, hipMemcpyDeviceToDevice, st));
    for (int i = 0; i < n; i++) BSM_HIP(hipMemcpyAsync(P + i * full, b, full, hipMemcpyDeviceToDevice, st));
    double *parts = ctx->partials;
    const int grid = ms_grid(m);
    double bnorm2 = 0.0, rrJ = 0.0;
    TRY(blas_dot(g, d, 2, Vec{(void *)b, BSM_F64}, none, parts, st));
    TRY(ms_sum(ctx, parts, blas_blocks(g, 2), &bnorm2, st));
    k_ms_jdot<<<grid, 256, 0, st>>>(m, (const double2 *)R, (const double2 *)R, parts);
    BSM_HIP(hipGetLastError());
    TRY(ms_sum(ctx, parts, grid, &rrJ, st));
    // the operator A = sigma_0 - H on full fields, links as the descriptor says
    bsm_field_desc d64 = *desc;
    const int lc = link_code(&d64);
    const bool real = link_real(&d64);
    auto applyA = [&](const char *in, char *out) -> bsm_status {
        HopArgs a{};
        a.U = U_rep64;
        a.dagger = 0;
        a.p0 = 0;
        a.np = 2;
        a.in[0] = in + bb; a.in[1] = in;
        a.x[0] = in; a.x[1] = in + bb;
        a.out[0] = out; a.out[1] = out + bb;
        a.a = sigma0;
        a.b = -1.0;
        apply_plan(ctx, d, real, BSM_F64, lc, a);
        return launch_hop(g, d, real, BSM_F64, lc, a, st);
    };
    // member coefficients on (p_i at the chunk start, chunk residuals 0..j)
    std::vector<double> coef((size_t)n * kMsCoefRow, 0.0);
    auto cx = [&](int i, int k) -> double & { return coef[(size_t)i * kMsCoefRow + 1 + k]; };   // k = -1: cx0
    auto cp = [&](int i, int k) -> double & { return coef[(size_t)i * kMsCoefRow + kMsChunk + 3 + k]; };
    auto reset = [&]() {
        std::fill(coef.begin(), coef.end(), 0.0);
        for (int i = 0; i < n; i++) cp(i, -1) = 1.0;
    };
    reset();
    int ring0 = 0, j = 0;        // the chunk's first residual field, iterations done in the chunk
    uint32_t xtouched = 0;       // members whose x has a contribution pending
    auto Rk = [&](int k) { return R + (size_t)((ring0 + k) % (L + 1)) * full; };
    auto flush = [&](uint32_t pkeep) -> bsm_status {
        if (j == 0) return BSM_OK;
        MsFlushList fl{};
        fl.xmask = xtouched;
        fl.pmask = pkeep;
        for (int i = 0; i < n; i++)
            if (((xtouched | pkeep) >> i) & 1u) fl.idx[fl.n++] = i;
        BSM_HIP(hipMemcpyAsync(dcoef, coef.data(), coef_bytes, hipMemcpyHostToDevice, st));
        k_ms_flush<<<std::min<int>((int)((m.n + 255) / 256), 65536), 256, 0, st>>>(
            m, (const double2 *)R, full / sizeof(double2), ring0, L + 1, j + 1, (double2 *)X, (double2 *)P, fl,
            dcoef);
        BSM_HIP(hipGetLastError());
        BSM_HIP(hipStreamSynchronize(st));   // coef is rewritten below
        ring0 = (ring0 + j) % (L + 1);
        j = 0;
        xtouched = 0;
        reset();
        return BSM_OK;
    };
    std::vector<double> zeta(n, 1.0), zeta_prev(n, 1.0), zn(n, 1.0), ca(n, 0.0), cb(n, 0.0);
    std::vector<int> iters(n, 0);
    uint32_t active = n == 32 ? 0xffffffffu : ((1u << n) - 1);
    double a_prev = 1.0, b_prev = 0.0;
    const double trig = (prm->delta > 0 ? prm->delta : 0.3) * prm->tol, bnorm = std::sqrt(bnorm2);
    int it = 0;
    bool broke = !(bnorm2 > 0) || !std::isfinite(rrJ);
    while (!broke && active && it < prm->max_iter) {
        TRY(applyA(Pd, Ap));
        double pAp = 0.0;
        k_ms_jdot<<<grid, 256, 0, st>>>(m, (const double2 *)Pd, (const double2 *)Ap, parts);
        BSM_HIP(hipGetLastError());
        TRY(ms_sum(ctx, parts, grid, &pAp, st));
        if (!std::isfinite(pAp) || pAp == 0.0) { broke = true; break; }
        const double alpha = rrJ / pAp;
        // members still iterating (the seed's direction drives the recurrence
        // and is kept while any member runs); retired members keep their zeta
        const uint32_t run = active | (1u << seed);
        for (int i = 0; i < n; i++) {
            if (!((run >> i) & 1u)) continue;
            const double den = a_prev * zeta_prev[i] * (1.0 + delta[i] * alpha) +
                               alpha * b_prev * (zeta_prev[i] - zeta[i]);
            zn[i] = zeta[i] * zeta_prev[i] * a_prev / den;
            ca[i] = alpha * zn[i] / zeta[i];
        }
        k_ms_residual<<<grid, 256, 0, st>>>(m, (const double2 *)Rk(j), (const double2 *)Ap, alpha,
                                            (double2 *)Rk(j + 1), parts);
        BSM_HIP(hipGetLastError());
        double rrJ_new = 0.0, rn2 = 0.0;
        TRY(ms_sum(ctx, parts, grid, &rrJ_new, st));
        TRY(ms_sum(ctx, parts + grid, grid, &rn2, st));
        const double beta = rrJ_new / rrJ;
        bool finite = std::isfinite(alpha) && std::isfinite(beta) && std::isfinite(rn2);
        for (int i = 0; i < n; i++) {
            if (!((run >> i) & 1u)) continue;
            const double q = zn[i] / zeta[i];
            cb[i] = beta * q * q;
            if (!std::isfinite(zn[i]) || !std::isfinite(ca[i]) || !std::isfinite(cb[i])) finite = false;
        }
        if (!finite) { broke = true; break; }
        // x_i += a_i p_i (members still active), p_i = z_i r_(n+1) + b_i p_i
        // (members running), on the coefficients; the seed's direction itself
        for (int i = 0; i < n; i++) {
            if (!((run >> i) & 1u)) continue;
            if ((active >> i) & 1u) {
                for (int k = -1; k <= j; k++) cx(i, k) += ca[i] * cp(i, k);
                xtouched |= 1u << i;
            }
            for (int k = -1; k <= j; k++) cp(i, k) *= cb[i];
            cp(i, j + 1) += zn[i];
        }
        TRY(blas_axpby(g, d, 2, Vec{Pd, BSM_F64}, 1.0, Vec{Rk(j + 1), BSM_F64}, beta, Vec{Pd, BSM_F64}, nullptr,
                       st));
        j++;
        it++;
        for (int i = 0; i < n; i++) {
            if (!((run >> i) & 1u)) continue;
            zeta_prev[i] = zeta[i];
            zeta[i] = zn[i];
        }
        a_prev = alpha;
        b_prev = beta;
        rrJ = rrJ_new;
        const double rn = std::sqrt(rn2);
        for (int i = 0; i < n; i++)
            if (((active >> i) & 1u) && std::fabs(zeta[i]) * rn <= trig * bnorm) {
                active &= ~(1u << i);
                iters[i] = it;
            }
        if (j == L && active) TRY(flush(active | (1u << seed)));
    }
    TRY(flush(0));
    for (int i = 0; i < n; i++)
        if (!iters[i]) iters[i] = it;
    // x_i = y_i / kappa_i (D(kappa) y = kappa b), then each member's FP64 true residual decides
    for (int i = 0; i < n; i++) {
        char *xi = X + i * full;
        TRY(blas_axpby(g, d, 2, Vec{xi, BSM_F64}, 1.0 / kappas[i], Vec{xi, BSM_F64}, 0.0, none, nullptr, st));
    }
    std::vector<double> res(n, INFINITY);
    // With real links (d_R 3, 8, 15) and 6 to 16 members, the 16-RHS FP64
    // block operator forms every member's residual at once in the scratch the
    // iteration no longer needs: the links are read once for all members, not
    // once per member.  r_e = b_e - x_e + kappa H_eo x_o, likewise r_o.
    auto rnd = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t bb64 = block64_parity_bytes(g, d), lk64 = block64_link_bytes(g, d);
    const size_t nparts = (size_t)block64_norm_parts(g, d) * kNR;
    const size_t need_blk = rnd(lk64) + 3 * rnd(bb64) + rnd(nparts * sizeof(double)) + rnd(2 * kNR * sizeof(double));
    const bool by_block = real && !link_is_otf(lc) && (d == 3 || d == 8 || d == 15) && n >= 6 && n <= kNR &&
                          need_blk <= work_bytes;
    if (by_block) {
        char *w = (char *)work;
        auto take = [&](size_t bytes) { char *q = w; w += rnd(bytes); return q; };
        double *Ub = (double *)take(lk64);
        double2 *XE = (double2 *)take(bb64), *XO = (double2 *)take(bb64), *BT = (double2 *)take(bb64);
        double *bparts = (double *)take(nparts * sizeof(double));
        double *dst = (double *)take(2 * kNR * sizeof(double));
        const unsigned all = (1u << n) - 1;
        TRY(launch_gauge_to_block64(g, d, U_rep64, Ub, st));
        TRY(launch_block64_io(g, d, n, all, X, full, 0, XE, nullptr, 0, st));
        TRY(launch_block64_io(g, d, n, all, X, full, bb, XO, nullptr, 0, st));
        auto parity = [&](int p0, const double2 *in, const double2 *xin, size_t b_off, double *nrm) -> bsm_status {
            // b of this parity for every member (stride 0), then the residual over it
            TRY(launch_block64_io(g, d, n, all, (const char *)b, 0, b_off, BT, nullptr, 0, st));
            BlockHop64Args a{};
            a.U = Ub;
            a.np = 1;
            a.p0 = p0;
            a.in[p0] = in;
            a.x[p0] = xin;
            a.y[p0] = BT;    // read before the same site's output is stored
            a.out[p0] = BT;
            a.use_x = 1;
            a.use_y = 1;
            for (int r = 0; r < kNR; r++) {
                a.a[r] = r < n ? -1.0 : 0.0;
                a.b[r] = r < n ? kappas[r] : 0.0;
                a.c[r] = r < n ? 1.0 : 0.0;
            }
            TRY(launch_hop_block64(g, d, a, st));
            return block64_norms(g, d, BT, bparts, nrm, st);
        };
        TRY(parity(0, XO, XE, 0, dst));
        TRY(parity(1, XE, XO, bb, dst + kNR));
        double h2[2 * kNR];
        BSM_HIP(hipMemcpyAsync(h2, dst, sizeof h2, hipMemcpyDeviceToHost, st));
        BSM_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < n; i++) {
            const double rn = h2[i] + h2[kNR + i];
            res[i] = bnorm2 > 0 ? std::sqrt(rn / bnorm2) : std::sqrt(rn);
        }
    } else {
        for (int i = 0; i < n; i++) {
            Op o{};
            o.ctx = ctx; o.g = g; o.d = d; o.real = real; o.schur = false; o.kappa = kappas[i];
            o.U = U_rep64; o.sprec = BSM_F64; o.lprec = lc; o.partials = ctx->partials;
            TRY(true_residual_full(o, (const char *)b, X + i * full, tfull, bnorm2, &res[i], st));
        }
    }
    for (int i = 0; i < n; i++) {
        stats[i].iters = iters[i];
        stats[i].true_rel_res = (!broke || !((active >> i) & 1u)) ? res[i] : INFINITY;
    }
    // members that missed tol: plain CG (it reuses the context scratch this
    // solver's fields were carved from, so only caller memory is used here)
    bsm_status worst = BSM_OK;
    for (int i = 0; i < n; i++) {
        char *xi = X + i * full;
        if (!(stats[i].true_rel_res <= prm->tol)) {
            // finish this member with plain FP64 Schur CG (from x = 0)
            bsm_solver_params p1 = *prm;
            p1.variant = BSM_SOLVER_PLAIN;
            p1.schur = 1;
            p1.kappa = kappas[i];
            bsm_solver_stats s1{};
            bsm_status cs = bsm_cg_solve(ctx, desc, U_rep64, U_rep64, &p1, b, xi, &s1, stream);
            stats[i].fell_back = 1;
            stats[i].iters += s1.iters;
            stats[i].true_rel_res = s1.true_rel_res;
            stats[i].restarts = s1.restarts;
            if (cs != BSM_OK && worst == BSM_OK) worst = cs;
        }
        stats[i].converged = stats[i].true_rel_res <= prm->tol;
    }
    BSM_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < n; i++) stats[i].seconds = secs;
    if (worst == BSM_ERR_NOT_CONVERGED) fail(worst, "max_iter reached before every member met tol");
    if (worst == BSM_ERR_NONFINITE) fail(worst, "non-finite value in a reduction");
    return worst;
}
