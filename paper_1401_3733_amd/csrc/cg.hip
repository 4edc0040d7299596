// Conjugate gradients on the normal equations of the Wilson-Dirac operator
// (full lattice) or of its even-odd Schur complement
//   Dhat = 1 - kappa^2 H_eo H_oe  on even sites,  bhat_e = b_e + kappa H_eo b_o,
//   x_o = b_o + kappa H_oe x_e.
// All CG scalars (alpha, beta, |r|^2) live on the device and are produced by
// fixed-order reductions, so kernels chain without host round trips; the host
// reads the |r|^2 history only to decide when to check convergence.
//
// Stopping rule: the normal-equation residual |r| <= trig |M^dag bhat| only
// triggers a check; the FP64 full-lattice true residual ||b - D x|| / ||b||
// decides.  If it is above tol the solve continues from the current x with
// the trigger tightened by 0.3.
//
// Mixed precision (reliable updates, Sleijpen & van der Vorst 1996; Clark et
// al. 2010): the CG recurrence runs with F32 or F16S vectors and links; when
// |r_lo| falls below delta * max |r_lo| since the last update, the low
// precision solution is folded into the FP64 solution and the residual is
// recomputed in FP64 with FP64 links, then the recurrence continues with the
// same search direction.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "blas.h"
#include "dispatch.h"
#include "solver.h"

namespace bsm {

// BSM_CG_TRACE=1 prints the device CG scalars at every host check
static bool trace_enabled() {
    static int on = -1;
    if (on < 0) {
        const char *e = getenv("BSM_CG_TRACE");
        on = (e && *e && *e != '0') ? 1 : 0;
    }
    return on == 1;
}

size_t blk(const Op &o) { return spinor_block_bytes(o.sprec, o.d, o.g.Vh_pad); }
int nblk_vec(const Op &o) { return o.schur ? 1 : 2; }

// y = M x or M^dag x; norm partials of y when partials != null (count in *np)
bsm_status op_apply(const Op &o, int dagger, const void *x, void *y, bool norm, int *np,
                           hipStream_t st) {
    HopArgs a{};
    a.U = o.U;
    a.dagger = dagger;
    if (o.schur) {
        // tmp_o = H_oe x_e
        a.p0 = 1; a.np = 1;
        a.in[1] = x; a.x[1] = nullptr; a.out[1] = o.tmp;
        a.a = 0.0; a.b = 1.0; a.norm_partials = nullptr;
        apply_plan(o.ctx, o.d, o.real, o.sprec, o.lprec, a);
        bsm_status s = launch_hop(o.g, o.d, o.real, o.sprec, o.lprec, a, st);
        if (s != BSM_OK) return s;
        // y_e = x_e - kappa^2 H_eo tmp_o
        HopArgs b{};
        b.U = o.U; b.dagger = dagger;
        b.p0 = 0; b.np = 1;
        b.in[0] = o.tmp; b.x[0] = x; b.out[0] = y;
        b.a = 1.0; b.b = -o.kappa * o.kappa;
        b.norm_partials = norm ? o.partials : nullptr;
        b.norm_cap = o.ctx->n_partials;
        apply_plan(o.ctx, o.d, o.real, o.sprec, o.lprec, b);
        if (np) *np = hop_grid(o.g, b);
        return launch_hop(o.g, o.d, o.real, o.sprec, o.lprec, b, st);
    }
    size_t bb = blk(o);
    const char *xp = (const char *)x;
    char *yp = (char *)y;
    a.p0 = 0; a.np = 2;
    a.in[0] = xp + bb; a.in[1] = xp;
    a.x[0] = xp; a.x[1] = xp + bb;
    a.out[0] = yp; a.out[1] = yp + bb;
    a.a = 1.0; a.b = -o.kappa;
    a.norm_partials = norm ? o.partials : nullptr;
    a.norm_cap = o.ctx->n_partials;
    apply_plan(o.ctx, o.d, o.real, o.sprec, o.lprec, a);
    if (np) *np = hop_grid(o.g, a);
    return launch_hop(o.g, o.d, o.real, o.sprec, o.lprec, a, st);
}

#define TRY(x)                           \
    do {                                 \
        bsm_status _s = (x);             \
        if (_s != BSM_OK) return _s;     \
    } while (0)

// sum n partials on the device and bring the result to the host (synchronous)
double reduce_to_host(bsm_ctx ctx, const double *partials, int n, hipStream_t st) {
    reduce_into(partials, n, ctx->scal + S_TMP, st);
    (void)hipMemcpyAsync(ctx->host_scal + S_TMP, ctx->scal + S_TMP, sizeof(double), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    return ctx->host_scal[S_TMP];
}

// FP64: out = M^dag (bh - M x), with t as scratch (vectors of o's shape)
bsm_status normal_residual(const Op &o, const char *bh, const char *x, char *t, char *out,
                                  hipStream_t st) {
    Vec T{t, BSM_F64}, BH{(void *)bh, BSM_F64};
    TRY(op_apply(o, 0, x, t, false, nullptr, st));
    TRY(blas_axpby(o.g, o.d, nblk_vec(o), T, -1.0, T, 1.0, BH, nullptr, st));
    return op_apply(o, 1, t, out, false, nullptr, st);
}

// FP64 true relative residual ||b - D x|| / ||b|| of the full system for the
// full fields b, x (Schur: the odd sites of x are first rebuilt from x_e);
// tfull is a full FP64 scratch field
bsm_status true_residual_full(const Op &o, const char *b, char *x, char *tfull, double bnorm2,
                                     double *res, hipStream_t st) {
    const Geom &g = o.g;
    const size_t bb64 = spinor_block_bytes(BSM_F64, o.d, g.Vh_pad);
    if (o.schur) {
        HopArgs a{};
        a.U = o.U; a.dagger = 0; a.p0 = 1; a.np = 1;
        a.in[1] = x; a.x[1] = b + bb64; a.out[1] = x + bb64;
        a.a = 1.0; a.b = o.kappa;
        TRY(launch_hop(g, o.d, o.real, BSM_F64, o.lprec, a, st));
    }
    HopArgs a{};
    a.U = o.U; a.dagger = 0; a.p0 = 0; a.np = 2;
    a.in[0] = x + bb64; a.in[1] = x; a.x[0] = x; a.x[1] = x + bb64;
    a.out[0] = tfull; a.out[1] = tfull + bb64;
    a.a = 1.0; a.b = -o.kappa;
    TRY(launch_hop(g, o.d, o.real, BSM_F64, o.lprec, a, st));
    Vec TF{tfull, BSM_F64}, B{(void *)b, BSM_F64};
    TRY(blas_axpby(g, o.d, 2, TF, -1.0, TF, 1.0, B, o.ctx->partials, st));
    const double rn = reduce_to_host(o.ctx, o.ctx->partials, blas_blocks(g, 2), st);
    *res = bnorm2 > 0 ? std::sqrt(rn / bnorm2) : std::sqrt(rn);
    return BSM_OK;
}

struct Solver {
    bsm_ctx ctx;
    hipStream_t st;
    Geom g;
    int d;
    bool real, schur;
    double kappa;
    const bsm_solver_params *prm;
    const char *b;         // caller b (full F64)
    char *x;               // caller x (full F64)
    Op op64;               // FP64 operator (true residuals, reliable updates)
    size_t bb64;           // FP64 parity block bytes
    char *bh, *r64, *t64, *tfull;   // FP64 work
    double bnorm2;          // |b|^2 (full)
    double rhs_norm2;       // |M^dag bhat|^2

    double host_reduce(const double *partials, int n) { return reduce_to_host(ctx, partials, n, st); }

    // FP64: out = M^dag (bhat - M x64)   (uses t64 as scratch)
    bsm_status normal_residual64(const char *x64, char *out) {
        return normal_residual(op64, bh, x64, t64, out, st);
    }

    // reconstruct odd sites (Schur) and return the FP64 true relative residual
    bsm_status true_residual(double *res) { return true_residual_full(op64, b, x, tfull, bnorm2, res, st); }

    bsm_status setup(void *work_base) {
        char *w = (char *)work_base;
        bb64 = spinor_block_bytes(BSM_F64, d, g.Vh_pad);
        size_t vec64 = (schur ? 1 : 2) * bb64;
        bh = w; w += vec64;
        r64 = w; w += vec64;
        t64 = w; w += vec64;
        tfull = w; w += 2 * bb64;
        op64.tmp = w; w += bb64;
        // bhat
        if (schur) {
            HopArgs a{};
            a.U = op64.U; a.dagger = 0; a.p0 = 0; a.np = 1;
            a.in[0] = b + bb64; a.x[0] = b; a.out[0] = bh;
            a.a = 1.0; a.b = kappa;
            TRY(launch_hop(g, d, real, BSM_F64, op64.lprec, a, st));
        } else {
            BSM_HIP(hipMemcpyAsync(bh, b, vec64, hipMemcpyDeviceToDevice, st));
        }
        Vec B{(void *)b, BSM_F64}, none{nullptr, BSM_F64};
        TRY(blas_dot(g, d, 2, B, none, ctx->partials, st));
        bnorm2 = host_reduce(ctx->partials, blas_blocks(g, 2));
        // rhs = M^dag bhat, its norm
        TRY(op_apply(op64, 1, bh, t64, false, nullptr, st));
        Vec T{t64, BSM_F64};
        TRY(blas_dot(g, d, nblk_vec(op64), T, none, ctx->partials, st));
        rhs_norm2 = host_reduce(ctx->partials, blas_blocks(g, nblk_vec(op64)));
        // x = 0
        BSM_HIP(hipMemsetAsync(x, 0, 2 * bb64, st));
        return BSM_OK;
    }

    static size_t work_bytes64(const Geom &g, int d, bool schur) {
        size_t bb = spinor_block_bytes(BSM_F64, d, g.Vh_pad);
        return (schur ? 3 : 6) * bb + 2 * bb + bb;
    }
};

// --------------------------------------------------------------- plain FP64
static bsm_status solve_plain(Solver &S, bsm_solver_stats *stats) {
    const Geom &g = S.g;
    int d = S.d;
    Op &o = S.op64;
    int nb = nblk_vec(o);
    size_t vec = nb * spinor_block_bytes(BSM_F64, d, g.Vh_pad);
    void *work = nullptr;
    size_t base = Solver::work_bytes64(g, d, S.schur);
    TRY(ctx_work(S.ctx, base + 3 * vec, &work));
    TRY(S.setup(work));
    char *w = (char *)work + base;
    char *p = w, *t = w + vec, *q = w + 2 * vec;
    char *r = S.r64;
    double *scal = S.ctx->scal;
    hipStream_t st = S.st;
    Vec X{S.x, BSM_F64}, P{p, BSM_F64}, R{r, BSM_F64}, Q{q, BSM_F64};
    const int K = S.prm->check_every > 0 ? S.prm->check_every : 8;
    const int hist_cap = kScalars - S_HIST;
    double trig = S.prm->tol;
    int it = 0, restarts = 0;
    double res = INFINITY;
    bsm_status status = BSM_ERR_NOT_CONVERGED;
    for (;;) {
        // r = M^dag (bhat - M x); p = r; rr = |r|^2
        TRY(S.normal_residual64(S.x, r));
        BSM_HIP(hipMemcpyAsync(p, r, vec, hipMemcpyDeviceToDevice, st));
        Vec none{nullptr, BSM_F64};
        TRY(blas_dot(g, d, nb, R, none, S.ctx->partials, st));
        TRY(cg_scalars(S.ctx->partials, blas_blocks(g, nb), scal, 2, it % hist_cap, st));
        const double target = trig * trig * S.rhs_norm2;
        bool triggered = false, bad = false;
        // first check of the current residual
        BSM_HIP(hipMemcpyAsync(S.ctx->host_scal, scal + S_RR, sizeof(double), hipMemcpyDeviceToHost, st));
        BSM_HIP(hipStreamSynchronize(st));
        if (S.ctx->host_scal[0] <= target) triggered = true;
        while (!triggered && it < S.prm->max_iter) {
            int k0 = it;
            int kn = std::min(K, S.prm->max_iter - it);
            for (int k = 0; k < kn; k++) {
                int np = 0;
                TRY(op_apply(o, 0, p, t, true, &np, st));               // t = M p, |t|^2
                TRY(cg_scalars(S.ctx->partials, np, scal, 0, 0, st));  // alpha
                TRY(op_apply(o, 1, t, q, false, nullptr, st));         // q = M^dag t
                TRY(blas_cg_update(g, d, nb, X, P, R, Q, scal, S_ALPHA, S.ctx->partials, st));
                TRY(cg_scalars(S.ctx->partials, blas_blocks(g, nb), scal, 1, (it + 1) % hist_cap, st));
                TRY(blas_cg_xpay(g, d, nb, P, R, scal, S_BETA, st));
                it++;
            }
            // history of |r|^2 for the iterations just run
            for (int k = k0 + 1; k <= it; k++) {
                int s = k % hist_cap;
                BSM_HIP(hipMemcpyAsync(S.ctx->host_scal + S_HIST + s, scal + S_HIST + s, sizeof(double),
                                       hipMemcpyDeviceToHost, st));
            }
            BSM_HIP(hipStreamSynchronize(st));
            if (trace_enabled()) {
                BSM_HIP(hipMemcpyAsync(S.ctx->host_scal + S_TMP2, scal, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
                BSM_HIP(hipStreamSynchronize(st));
                const double *h = S.ctx->host_scal + S_TMP2;
                fprintf(stderr, "[cg] it %d rr %.6e pAp %.6e alpha %.6e beta %.6e target %.3e\n", it,
                        h[S_RR], h[S_PAP], h[S_ALPHA], h[S_BETA], target);
            }
            for (int k = k0 + 1; k <= it; k++) {
                double rr = S.ctx->host_scal[S_HIST + k % hist_cap];
                if (trace_enabled()) fprintf(stderr, "[cg]   hist %d %.6e\n", k, rr);
                if (!std::isfinite(rr)) bad = true;
                if (rr <= target) triggered = true;
            }
            if (bad) break;
        }
        if (bad) { status = BSM_ERR_NONFINITE; S.true_residual(&res); break; }
        TRY(S.true_residual(&res));
        if (trace_enabled()) fprintf(stderr, "[cg] true residual %.6e after %d iterations\n", res, it);
        if (!std::isfinite(res)) { status = BSM_ERR_NONFINITE; break; }
        if (res <= S.prm->tol) { status = BSM_OK; break; }
        if (it >= S.prm->max_iter) break;
        trig *= 0.3;
        restarts++;
    }
    stats->iters = it;
    stats->restarts = restarts;
    stats->reliable_updates = 0;
    stats->true_rel_res = res;
    stats->converged = status == BSM_OK;
    return status;
}

// ------------------------------------------------------- mixed precision RU
static bsm_status solve_mixed(Solver &S, int inner_prec, int link_prec, const void *U_lo,
                              bsm_solver_stats *stats) {
    const Geom &g = S.g;
    int d = S.d;
    Op lo = S.op64;
    lo.sprec = inner_prec;
    lo.lprec = link_prec;
    lo.U = U_lo;
    const int nb = nblk_vec(lo);
    const int acc_prec = BSM_F32;   // x_lo and r_lo
    size_t vlo = nb * spinor_block_bytes(inner_prec, d, g.Vh_pad);
    size_t vacc = nb * spinor_block_bytes(acc_prec, d, g.Vh_pad);
    size_t base = Solver::work_bytes64(g, d, S.schur);
    // K iterations per chunk; the chunk's directions p are kept (a ring of
    // K + 1) and x_lo takes sum_k alpha_k p_k once at the chunk's end rather
    // than alpha p every iteration
    const int hist_cap = kScalars - S_HIST;
    const int K = std::max(1, std::min(S.prm->check_every > 0 ? S.prm->check_every : 8, kAlphaHist));
    const int ring = K + 1;
    void *work = nullptr;
    TRY(ctx_work(S.ctx, base + (ring + 2) * vlo + 2 * vacc + spinor_block_bytes(inner_prec, d, g.Vh_pad), &work));
    TRY(S.setup(work));
    char *w = (char *)work + base;
    char *pring = w; w += ring * vlo;
    char *t = w; w += vlo;
    char *q = w; w += vlo;
    char *xlo = w; w += vacc;
    char *rlo = w; w += vacc;
    lo.tmp = w;
    hipStream_t st = S.st;
    double *scal = S.ctx->scal;
    double *hs = S.ctx->host_scal;
    Vec X64{S.x, BSM_F64}, R64{S.r64, BSM_F64};
    auto Pslot = [&](int i) { return Vec{pring + (size_t)(i % ring) * vlo, inner_prec}; };
    Vec Q{q, inner_prec}, XL{xlo, acc_prec}, RL{rlo, acc_prec};
    Vec none{nullptr, BSM_F64};
    const double delta2 = S.prm->delta > 0 ? S.prm->delta * S.prm->delta : 0.01;

    // r64 = M^dag (bhat - M x64), |r64|^2 ; r_lo = r64 ; p = r_lo ; x_lo = 0
    auto reliable = [&](double *rr_true) -> bsm_status {
        TRY(S.normal_residual64(S.x, S.r64));
        TRY(blas_dot(g, d, nb, R64, none, S.ctx->partials, st));
        *rr_true = S.host_reduce(S.ctx->partials, blas_blocks(g, nb));
        TRY(blas_axpby(g, d, nb, RL, 1.0, R64, 0.0, none, nullptr, st));
        return BSM_OK;
    };

    // K iterations are enqueued between host checks.  An iteration starts
    // with p = r + beta p, so at a chunk boundary a reliable update only
    // replaces r, |r|^2 and beta (the first beta is 0: p = r).  Measured on
    // 32^3 x 64 (K = 1 / 8 / 16): two-index F16+scale with F16 links
    // 0.167 / 0.130 / 0.125 s (fewer reliable updates), fundamental
    // 0.123 / 0.119 / 0.121 s (K = 16 adds iterations).
    double trig = S.prm->tol;
    int it = 0, restarts = 0, updates = 0;
    double res = INFINITY;
    bsm_status status = BSM_ERR_NOT_CONVERGED;
    double rr;
    // restart the recurrence from the FP64 residual: r_lo = r64, beta = 0
    auto restart_from_true = [&](double rr_true) -> bsm_status {
        hs[S_RR] = rr_true;
        hs[S_BETA] = 0.0;
        BSM_HIP(hipMemcpyAsync(scal + S_RR, hs + S_RR, sizeof(double), hipMemcpyHostToDevice, st));
        BSM_HIP(hipMemcpyAsync(scal + S_BETA, hs + S_BETA, sizeof(double), hipMemcpyHostToDevice, st));
        BSM_HIP(hipStreamSynchronize(st));   // hs is rewritten by the next chunk's read-back
        return BSM_OK;
    };
    TRY(reliable(&rr));
    BSM_HIP(hipMemsetAsync(xlo, 0, vacc, st));
    BSM_HIP(hipMemsetAsync(pring, 0, ring * vlo, st));
    TRY(restart_from_true(rr));
    double maxrr = rr;
    for (;;) {
        const double target = trig * trig * S.rhs_norm2;
        bool check = rr <= target;
        while (!check && it < S.prm->max_iter) {
            const int k0 = it, kn = std::min(K, S.prm->max_iter - it);
            for (int k = 0; k < kn; k++) {
                const Vec P = Pslot(it);
                TRY(blas_cg_xpay_to(g, d, nb, P, Pslot(it + ring - 1), RL, scal, S_BETA, st));
                int np = 0;
                TRY(op_apply(lo, 0, P.ptr, t, true, &np, st));
                TRY(cg_scalars(S.ctx->partials, np, scal, 0, k, st));   // alpha_k kept for x
                TRY(op_apply(lo, 1, t, q, false, nullptr, st));
                TRY(blas_cg_update(g, d, nb, Vec{nullptr, acc_prec}, P, RL, Q, scal, S_ALPHA, S.ctx->partials, st));
                TRY(cg_scalars(S.ctx->partials, blas_blocks(g, nb), scal, 1, (it + 1) % hist_cap, st));
                it++;
            }
            // x_lo += sum_k alpha_k p_k over this chunk's directions
            TRY(blas_x_flush(g, d, nb, XL, pring, inner_prec, vlo, ring, k0 % ring, kn, scal + S_AHIST, st));
            for (int k = k0 + 1; k <= it; k++) {
                const int sl = k % hist_cap;
                BSM_HIP(hipMemcpyAsync(hs + S_HIST + sl, scal + S_HIST + sl, sizeof(double), hipMemcpyDeviceToHost,
                                       st));
            }
            BSM_HIP(hipStreamSynchronize(st));
            // |r|^2 of every iteration of the chunk: the last one and the one before it
            double last = rr, before = rr;
            bool trigger = false;
            for (int k = k0 + 1; k <= it; k++) {
                const double v = hs[S_HIST + k % hist_cap];
                if (!std::isfinite(v)) status = BSM_ERR_NONFINITE;
                before = last;
                last = v;
                if (v > maxrr) maxrr = v;
                if (v < delta2 * maxrr || v <= target) trigger = true;
            }
            if (status == BSM_ERR_NONFINITE) break;
            rr = last;
            if (trigger) {
                // fold x_lo into x64, recompute the residual in FP64
                TRY(blas_axpby(g, d, nb, X64, 1.0, X64, 1.0, XL, nullptr, st));
                BSM_HIP(hipMemsetAsync(xlo, 0, vacc, st));
                double rr_true;
                TRY(reliable(&rr_true));
                updates++;
                // beta from the recomputed residual, the search direction kept;
                // a recomputed residual not below the recurrence's value before
                // the last iteration means the recurrence ran ahead of it
                // (FP16): restart from r instead
                hs[S_BETA] = (before > 0 && rr_true < before) ? rr_true / before : 0.0;
                hs[S_RR] = rr_true;
                BSM_HIP(hipMemcpyAsync(scal + S_BETA, hs + S_BETA, sizeof(double), hipMemcpyHostToDevice, st));
                BSM_HIP(hipMemcpyAsync(scal + S_RR, hs + S_RR, sizeof(double), hipMemcpyHostToDevice, st));
                BSM_HIP(hipStreamSynchronize(st));
                rr = rr_true;
                maxrr = rr_true;
                if (rr_true <= target) check = true;
            }
        }
        if (status == BSM_ERR_NONFINITE) break;
        // make sure x64 holds everything
        TRY(blas_axpby(g, d, nb, X64, 1.0, X64, 1.0, XL, nullptr, st));
        BSM_HIP(hipMemsetAsync(xlo, 0, vacc, st));
        TRY(S.true_residual(&res));
        if (!std::isfinite(res)) { status = BSM_ERR_NONFINITE; break; }
        if (res <= S.prm->tol) { status = BSM_OK; break; }
        if (it >= S.prm->max_iter) break;
        trig *= 0.3;
        restarts++;
        TRY(reliable(&rr));
        TRY(restart_from_true(rr));
        maxrr = rr;
    }
    stats->iters = it;
    stats->restarts = restarts;
    stats->reliable_updates = updates;
    stats->true_rel_res = res;
    stats->converged = status == BSM_OK;
    return status;
}

}  // namespace bsm

using namespace bsm;

extern "C" bsm_status bsm_cg_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                                   const void *U_rep64, const bsm_solver_params *prm, const void *b,
                                   void *x, bsm_solver_stats *stats, void *stream) {
    if (prm && prm->variant == BSM_SOLVER_BATCHED)
        return bsm_batched_solve(ctx, desc, U_rep64, prm, prm->n_rhs, prm->kappas, b, x, stats, stream);
    if (prm && prm->variant == BSM_SOLVER_SHIFTED)
        return bsm_shifted_solve(ctx, desc, U_rep64, prm, prm->n_rhs, prm->kappas, b, x, stats, stream);
    if (prm && prm->variant == BSM_SOLVER_FGCR_NET)
        return bsm_fgcr_solve(ctx, desc, U_rep, U_rep64, prm, prm->channels, prm->net, b, x, stats, stream);
    if (!ctx || !desc || !prm || !b || !x || !stats || !U_rep || !U_rep64)
        return fail(BSM_ERR_ARG, "null argument");
    if (bsm_rep_dim(desc->N, desc->rep) != desc->d_R || desc->d_R < 2 || desc->d_R > 15)
        return fail(BSM_ERR_ARG, "d_R does not match (N, rep) or is outside [2, 15]");
    if (!(prm->kappa > 0) || !std::isfinite(prm->kappa)) return fail(BSM_ERR_ARG, "kappa must be > 0");
    if (!(prm->tol > 0)) return fail(BSM_ERR_ARG, "tol must be > 0");
    if (prm->max_iter < 1) return fail(BSM_ERR_ARG, "max_iter must be >= 1");
    if (b == x) return fail(BSM_ERR_ARG, "b and x must differ");
    if ((desc->link_prec & ~BSM_LINKS_FUNDAMENTAL) < 0 || (desc->link_prec & ~BSM_LINKS_FUNDAMENTAL) > 2)
        return fail(BSM_ERR_ARG, "bad link precision");
    if (prm->variant == BSM_SOLVER_PLAIN && (desc->prec != BSM_F64 || link_base(desc->link_prec) != BSM_F64))
        return fail(BSM_ERR_ARG, "plain CG runs in FP64: desc prec and link_prec must be F64");
    if (prm->variant == BSM_SOLVER_MIXED && desc->prec == BSM_F64)
        return fail(BSM_ERR_ARG, "mixed CG needs an F32 or F16S inner precision");
    if (prm->variant != BSM_SOLVER_PLAIN && prm->variant != BSM_SOLVER_MIXED)
        return fail(BSM_ERR_ARG, "unknown solver variant");
    *stats = bsm_solver_stats{};
    auto t0 = std::chrono::steady_clock::now();
    Solver S{};
    S.ctx = ctx;
    S.st = (hipStream_t)stream;
    S.g = ctx->g;
    S.d = desc->d_R;
    S.real = link_real(desc);
    S.schur = prm->schur != 0;
    S.kappa = prm->kappa;
    S.prm = prm;
    S.b = (const char *)b;
    S.x = (char *)x;
    S.op64.ctx = ctx;
    S.op64.g = ctx->g;
    S.op64.d = S.d;
    S.op64.real = link_real(desc);
    S.op64.schur = S.schur;
    S.op64.kappa = prm->kappa;
    S.op64.U = U_rep64;
    S.op64.sprec = BSM_F64;
    // U_rep64 is stored like U_rep: R(U) in FP64, or U in FP64 with the
    // representation formed on the fly
    {
        bsm_field_desc d64 = *desc;
        d64.link_prec = BSM_F64 | (desc->link_prec & BSM_LINKS_FUNDAMENTAL);
        S.op64.lprec = link_code(&d64);
    }
    S.op64.partials = ctx->partials;
    bsm_status s;
    if (prm->variant == BSM_SOLVER_PLAIN) s = solve_plain(S, stats);
    else s = solve_mixed(S, desc->prec, link_code(desc), U_rep, stats);
    hipError_t e = hipStreamSynchronize(S.st);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (e != hipSuccess) return hip_check(e, "bsm_cg_solve");
    if (s == BSM_ERR_NOT_CONVERGED) fail(s, "max_iter reached before the true residual met tol");
    if (s == BSM_ERR_NONFINITE) fail(s, "non-finite value in a reduction");
    return s;
}

// ===================================================================== batched
// Many right-hand sides D(kappa_r) x_r = b_r at once (even-odd Schur CG on
// the normal equations, one kappa per RHS).  For real (adjoint) links the
// recurrence runs on 16-RHS block fields with the matrix-core hop, so every
// link load serves all RHS: FP32 fields and links on FP32 matrix cores, or
// (F16S) FP16 search directions and hop outputs with per-site scales, FP16
// links and FP16 matrix cores, x and r kept in FP32; K iterations are captured once as a HIP
// graph and replayed.  Every RHS keeps its own alpha, beta and |r|^2 on the
// device; between replays the host folds the FP32 solutions into the FP64
// ones, recomputes in FP64 the residual of every RHS whose |r| dropped by
// delta since its last update (reliable update) or reached its trigger, and
// retires an RHS once its FP64 full-lattice true residual is <= tol: its
// alpha and beta are masked to zero from then on.
#include "block.h"

namespace bsm {

struct BlockSolve {
    bsm_ctx ctx;
    Geom g;
    int d, n;
    hipStream_t st;
    const bsm_solver_params *prm;
    const double *kappas;
    const char *b;
    char *x;
    size_t full64, bb64, bbB, bbH;
    bool half;   // F16S inner recurrence (FP16 block fields)
    // FP64 per RHS
    std::vector<Op> ops;
    char *t64, *tfull, *tmp64;
    std::vector<double> bnorm2, rhs_norm2;
    // FP64 block fields for the reliable updates (all RHS share each link load)
    double *Ublk64;
    double2 *X64, *BH64, *T1, *T2, *T3;
    // inner block fields: p, t, q and the odd intermediate tmpB in the inner
    // precision (FP32 or FP16), x and r in FP32; links FP32 or FP16
    float *Ublk;
    __half *Uh;
    char *p, *t, *q, *tmpB;
    float2 *xlo, *rlo;
    double *partials, *scal, *presum;
    int *mask;
    hipGraphExec_t graph = nullptr;
    int K;
    BlockPlan &plan() const { return ctx->block_plans[d][half ? 1 : 0]; }
};

// the two hops of the Schur operator (or its adjoint) on inner block fields:
// tmp_o = H_oe in_e ;  out_e = in_e - kappa_r^2 H_eo tmp_o
template <class Args>
static void block_op_args(BlockSolve &B, int dagger, Args &a, Args &c) {
    a.dagger = dagger;
    a.np = 1;
    a.p0 = 1;
    a.use_x = 0;
    for (int r = 0; r < kNR; r++) { a.a[r] = 0.f; a.b[r] = 1.f; }
    c = a;
    c.p0 = 0;
    c.use_x = 1;
    for (int r = 0; r < kNR; r++) {
        const double k = r < B.n ? B.kappas[r] : 0.0;
        c.a[r] = 1.f;
        c.b[r] = (float)(-k * k);
    }
}

static bsm_status block_op(BlockSolve &B, int dagger, const char *in, char *out, bool norm, int *nparts) {
    if (B.half) {
        BlockHopHArgs a{}, c{};
        a.U = B.Uh;
        apply_blockh_plan(B.g, B.plan(), a);
        block_op_args(B, dagger, a, c);
        a.in[1] = in;
        a.out[1] = B.tmpB;
        TRY(launch_hop_blockh(B.g, B.d, a, B.st));
        c.in[0] = B.tmpB;
        c.x[0] = in;
        c.out[0] = out;
        c.norm_partials = norm ? B.partials : nullptr;
        if (nparts) *nparts = hop_blockh_grid(B.g, c);
        return launch_hop_blockh(B.g, B.d, c, B.st);
    }
    BlockHopArgs a{}, c{};
    a.U = B.Ublk;
    apply_block_plan(B.g, B.plan(), a);
    block_op_args(B, dagger, a, c);
    a.in[1] = (const float2 *)in;
    a.out[1] = (float2 *)B.tmpB;
    TRY(launch_hop_block(B.g, B.d, a, B.st));
    c.in[0] = (const float2 *)B.tmpB;
    c.x[0] = (const float2 *)in;
    c.out[0] = (float2 *)out;
    c.norm_partials = norm ? B.partials : nullptr;
    if (nparts) *nparts = hop_block_grid(B.g, c);
    return launch_hop_block(B.g, B.d, c, B.st);
}

// FP64 Schur operator (or its adjoint) on FP64 block fields, T1 as the odd
// intermediate: out_e = in_e - kappa_r^2 H_eo H_oe in_e
static bsm_status block_op64(BlockSolve &B, int dagger, const double2 *in, double2 *out) {
    BlockHop64Args a{};
    a.U = B.Ublk64;
    a.dagger = dagger;
    // the FP64 blocks follow the site and workgroup orders tuned for the inner ones
    if (B.plan().tiled) a.tile = block_tile_for(B.g);
    a.xchunk = B.plan().xchunk;
    a.np = 1;
    a.p0 = 1;
    a.in[1] = in;
    a.out[1] = B.T1;
    for (int r = 0; r < kNR; r++) { a.a[r] = 0.0; a.b[r] = 1.0; }
    TRY(launch_hop_block64(B.g, B.d, a, B.st));
    BlockHop64Args c = a;
    c.p0 = 0;
    c.in[0] = B.T1;
    c.x[0] = in;
    c.out[0] = out;
    c.use_x = 1;
    for (int r = 0; r < kNR; r++) {
        const double k = r < B.n ? B.kappas[r] : 0.0;
        c.a[r] = 1.0;
        c.b[r] = -k * k;
    }
    return launch_hop_block64(B.g, B.d, c, B.st);
}

// out = y - M in (Schur: M = 1 - kappa_r^2 H_eo H_oe), the subtraction in the
// second hop's epilogue
static bsm_status block_res64(BlockSolve &B, const double2 *in, const double2 *y, double2 *out) {
    BlockHop64Args a{};
    a.U = B.Ublk64;
    a.dagger = 0;
    if (B.plan().tiled) a.tile = block_tile_for(B.g);
    a.xchunk = B.plan().xchunk;
    a.np = 1;
    a.p0 = 1;
    a.in[1] = in;
    a.out[1] = B.T1;
    for (int r = 0; r < kNR; r++) { a.a[r] = 0.0; a.b[r] = 1.0; }
    TRY(launch_hop_block64(B.g, B.d, a, B.st));
    BlockHop64Args c = a;
    c.p0 = 0;
    c.in[0] = B.T1;
    c.x[0] = in;
    c.y[0] = y;
    c.out[0] = out;
    c.use_x = 1;
    c.use_y = 1;
    for (int r = 0; r < kNR; r++) {
        const double k = r < B.n ? B.kappas[r] : 0.0;
        c.a[r] = r < B.n ? -1.0 : 0.0;
        c.b[r] = k * k;
        c.c[r] = r < B.n ? 1.0 : 0.0;
    }
    return launch_hop_block64(B.g, B.d, c, B.st);
}

// one CG iteration on the block fields: p = r + beta p ; t = M p ; alpha ;
// q = M^dag t ; x += alpha p ; r -= alpha q ; beta, |r|^2 -> history slot k
static bsm_status block_iteration(BlockSolve &B, int k) {
    const Geom &g = B.g;
    if (B.half) TRY(blockh_xpay(g, B.d, B.p, B.rlo, B.scal + B_BETA * kNR, B.st));
    else TRY(block_xpay(g, B.d, 1, (float2 *)B.p, B.rlo, B.scal + B_BETA * kNR, B.st));
    int np = 0;
    TRY(block_op(B, 0, B.p, B.t, true, &np));
    TRY(block_scalars(B.partials, np, B.scal, B.mask, 0, 0, B.presum, B.st));
    TRY(block_op(B, 1, B.t, B.q, false, nullptr));
    if (B.half) {
        TRY(blockh_update(g, B.d, B.xlo, B.p, B.rlo, B.q, B.scal + B_ALPHA * kNR, B.partials, B.st));
        TRY(block_scalars(B.partials, blockh_blas_grid(g), B.scal, B.mask, 1, k, B.presum, B.st));
    } else {
        TRY(block_update(g, B.d, 1, B.xlo, (const float2 *)B.p, B.rlo, (const float2 *)B.q,
                         B.scal + B_ALPHA * kNR, B.partials, B.st));
        TRY(block_scalars(B.partials, block_blas_grid(g, B.d, 1), B.scal, B.mask, 1, k, B.presum, B.st));
    }
    return BSM_OK;
}

static bsm_status solve_block(BlockSolve &B, bsm_solver_stats *stats) {
    const Geom &g = B.g;
    const int d = B.d, n = B.n;
    hipStream_t st = B.st;
    // ---- work memory
    const size_t linkB = B.half ? blockh_link_bytes(g, d) : block_link_bytes(g, d);
    const size_t bbI = B.half ? B.bbH : B.bbB;   // inner-precision block fields
    // partials for any plan (the autotuner below may change it)
    const size_t parts = std::max({(size_t)hop_block_grid_max(g), (size_t)block_blas_grid(g, d, 1),
                                   (size_t)blockh_blas_grid(g)}) * kNR;
    // 20 carve-outs below, each rounded up to 256 bytes
    const size_t link64 = block64_link_bytes(g, d), bb64B = block64_parity_bytes(g, d);
    size_t need = linkB + 4 * bbI + 2 * B.bbB + (size_t)4 * B.bb64 + parts * 8 +
                  (size_t)kBlockPresum * kNR * 8 + block_scal_doubles() * 8 + 64 * sizeof(int) + link64 +
                  5 * bb64B + 22 * 256;
    void *work = nullptr;
    TRY(ctx_work(B.ctx, need, &work));
    char *w = (char *)work;
    auto take = [&](size_t bytes) { char *r = w; w += (bytes + 255) / 256 * 256; return r; };
    char *links = take(linkB);
    B.Ublk = B.half ? nullptr : (float *)links;
    B.Uh = B.half ? (__half *)links : nullptr;
    B.p = take(bbI); B.t = take(bbI); B.q = take(bbI); B.tmpB = take(bbI);
    B.xlo = (float2 *)take(B.bbB); B.rlo = (float2 *)take(B.bbB);
    B.t64 = take(B.bb64); B.tmp64 = take(B.bb64); B.tfull = take(2 * B.bb64);
    B.partials = (double *)take(parts * 8);
    B.presum = (double *)take((size_t)kBlockPresum * kNR * 8);
    B.scal = (double *)take(block_scal_doubles() * 8);
    B.mask = (int *)take(64 * sizeof(int));
    B.Ublk64 = (double *)take(link64);
    B.X64 = (double2 *)take(bb64B); B.BH64 = (double2 *)take(bb64B);
    B.T1 = (double2 *)take(bb64B); B.T2 = (double2 *)take(bb64B); B.T3 = (double2 *)take(bb64B);
    // ---- links in block layout, per-RHS FP64 operators and right-hand sides
    if (B.half) TRY(launch_gauge_to_blockh(g, d, BSM_F64, B.ops[0].U, B.Uh, st));
    else TRY(launch_gauge_to_block(g, d, BSM_F64, B.ops[0].U, B.Ublk, st));
    TRY(launch_gauge_to_block64(g, d, B.ops[0].U, B.Ublk64, st));
    // first batched solve for this d_R and precision on the context: tune the
    // block hop plan (t and q are outputs of every iteration, free as scratch)
    if (B.plan().us == 0.f) {
        if (B.half) TRY(blockh_autotune(B.ctx, d, B.Uh, B.t, B.q, st));
        else TRY(block_autotune(B.ctx, d, B.Ublk, (float2 *)B.t, (float2 *)B.q, st));
    }
    BSM_HIP(hipMemsetAsync(B.x, 0, n * B.full64, st));
    B.bnorm2.assign(n, 0.0);
    B.rhs_norm2.assign(n, 0.0);
    for (int r = 0; r < n; r++) B.ops[r].tmp = B.tmp64;
    const unsigned all = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
    auto hop64 = [&](int p0, const double2 *in, const double2 *xin, double sgn, double2 *out) -> bsm_status {
        BlockHop64Args a{};
        a.U = B.Ublk64;
        a.dagger = 0;
        a.np = 1;
        a.p0 = p0;
        a.in[p0] = in;
        a.x[p0] = xin;
        a.out[p0] = out;
        a.use_x = 1;
        if (B.plan().tiled) a.tile = block_tile_for(g);
        a.xchunk = B.plan().xchunk;
        for (int r = 0; r < kNR; r++) {
            a.a[r] = 1.0;
            a.b[r] = r < n ? sgn * B.kappas[r] : 0.0;
        }
        return launch_hop_block64(g, d, a, st);
    };
    // out = y - xin + kappa_r H in on the parity p0 (a residual of D)
    auto res64 = [&](int p0, const double2 *in, const double2 *xin, const double2 *y, double2 *out) -> bsm_status {
        BlockHop64Args a{};
        a.U = B.Ublk64;
        a.dagger = 0;
        a.np = 1;
        a.p0 = p0;
        a.in[p0] = in;
        a.x[p0] = xin;
        a.y[p0] = y;
        a.out[p0] = out;
        a.use_x = 1;
        a.use_y = 1;
        if (B.plan().tiled) a.tile = block_tile_for(g);
        a.xchunk = B.plan().xchunk;
        for (int r = 0; r < kNR; r++) {
            a.a[r] = r < n ? -1.0 : 0.0;
            a.b[r] = r < n ? B.kappas[r] : 0.0;
            a.c[r] = r < n ? 1.0 : 0.0;
        }
        return launch_hop_block64(g, d, a, st);
    };
    // ---- right-hand sides on the FP64 block operator, every RHS at once:
    //      |b_r|^2, bhat_e = b_e + kappa_r H_eo b_o, |M_r^dag bhat_r|^2
    {
        double h48[3 * kNR];
        TRY(launch_block64_io(g, d, n, all, B.b, B.full64, B.bb64, B.T2, nullptr, 0, st));   // b_o
        TRY(launch_block64_io(g, d, n, all, B.b, B.full64, 0, B.T3, nullptr, 0, st));        // b_e
        TRY(block64_norms(g, d, B.T2, B.partials, B.presum, st));
        TRY(block64_norms(g, d, B.T3, B.partials, B.presum + kNR, st));
        TRY(hop64(0, B.T2, B.T3, 1.0, B.BH64));
        TRY(block_op64(B, 1, B.BH64, B.X64));
        TRY(block64_norms(g, d, B.X64, B.partials, B.presum + 2 * kNR, st));
        BSM_HIP(hipMemcpyAsync(h48, B.presum, sizeof h48, hipMemcpyDeviceToHost, st));
        BSM_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < n; r++) {
            B.bnorm2[r] = h48[r] + h48[kNR + r];
            B.rhs_norm2[r] = h48[2 * kNR + r];
        }
    }
    // ---- residuals: r64_r = M_r^dag (bhat_r - M_r x_r) for the selected RHS,
    //      copied into the block residual; returns |r64_r|^2
    std::vector<double> rr(kNR, 0.0), maxrr(kNR, 0.0), trig(n, B.prm->tol), res(n, INFINITY);
    //      (FP64 block operator: every RHS at once, sharing the link loads)
    auto refresh = [&](unsigned sel) -> bsm_status {
        TRY(launch_block64_io(g, d, n, all, B.x, B.full64, 0, B.X64, nullptr, 0, st));
        TRY(block_res64(B, B.X64, B.BH64, B.T2));           // bhat - M x
        TRY(block_op64(B, 1, B.T2, B.X64));                 // M^dag (...)
        TRY(block64_norms(g, d, B.X64, B.partials, B.presum, st));
        double h16[kNR];
        BSM_HIP(hipMemcpyAsync(h16, B.presum, sizeof h16, hipMemcpyDeviceToHost, st));
        BSM_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < n; r++)
            if ((sel >> r) & 1u) rr[r] = h16[r];
        return launch_block64_io(g, d, n, sel, nullptr, 0, 0, B.X64, B.rlo, 1, st);
    };
    // FP64 true residuals |b_r - D_r x_r| / |b_r| of every RHS at once with the
    // block operator (one link load for all): the odd sites are rebuilt,
    // x_o = b_o + kappa_r H_oe x_e, and written back for the RHS in sel; then
    // r_o = b_o - (x_o - kappa_r H_oe x_e) and r_e = b_e - (x_e - kappa_r H_eo x_o)
    auto block_residuals = [&](unsigned sel, std::vector<double> &res_out) -> bsm_status {
        const size_t off_o = B.bb64;
        TRY(launch_block64_io(g, d, n, all, B.x, B.full64, 0, B.X64, nullptr, 0, st));       // x_e
        TRY(launch_block64_io(g, d, n, all, B.b, B.full64, off_o, B.T2, nullptr, 0, st));    // b_o
        TRY(hop64(1, B.X64, B.T2, 1.0, B.T1));                                              // x_o
        TRY(launch_block64_io(g, d, n, sel, B.x, B.full64, off_o, B.T1, nullptr, 2, st));    // x_o -> x
        TRY(res64(1, B.X64, B.T1, B.T2, B.T3));                                             // r_o
        TRY(block64_norms(g, d, B.T3, B.partials, B.presum, st));
        TRY(launch_block64_io(g, d, n, all, B.b, B.full64, 0, B.T2, nullptr, 0, st));        // b_e
        TRY(res64(0, B.T1, B.X64, B.T2, B.T3));                                             // r_e
        TRY(block64_norms(g, d, B.T3, B.partials, B.presum + kNR, st));
        double h32[2 * kNR];
        BSM_HIP(hipMemcpyAsync(h32, B.presum, sizeof h32, hipMemcpyDeviceToHost, st));
        BSM_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < n; r++) {
            if (!((sel >> r) & 1u)) continue;
            const double rn = h32[r] + h32[kNR + r];
            res_out[r] = B.bnorm2[r] > 0 ? std::sqrt(rn / B.bnorm2[r]) : std::sqrt(rn);
        }
        return BSM_OK;
    };
    // per-RHS checks cost about a seventh of the block one (three single-RHS
    // FP64 hops against three block hops and the layout conversions)
    constexpr int kBlockCheckMin = 6;
    auto true_residuals = [&](unsigned sel) -> bsm_status {
        if (__builtin_popcount(sel) >= kBlockCheckMin) return block_residuals(sel, res);
        for (int r = 0; r < n; r++)
            if ((sel >> r) & 1u)
                TRY(true_residual_full(B.ops[r], B.b + r * B.full64, B.x + r * B.full64, B.tfull, B.bnorm2[r],
                                       &res[r], st));
        return BSM_OK;
    };
    TRY(refresh(all));
    BSM_HIP(hipMemsetAsync(B.xlo, 0, B.bbB, st));
    BSM_HIP(hipMemsetAsync(B.p, 0, bbI, st));
    // pinned host mirrors of the device scalars and mask (context scratch)
    void *pin = nullptr;
    const size_t hs_bytes = (block_scal_doubles() * 8 + 255) / 256 * 256;
    TRY(ctx_pinned(B.ctx, hs_bytes + 64 * sizeof(int), &pin));
    double *hs = (double *)pin;
    int *hmask = (int *)((char *)pin + hs_bytes);
    for (size_t i = 0; i < block_scal_doubles(); i++) hs[i] = 0.0;
    for (int i = 0; i < 64; i++) hmask[i] = 0;
    for (int r = 0; r < n; r++) {
        hmask[r] = 1;
        hs[B_RR * kNR + r] = rr[r];
        maxrr[r] = rr[r];
    }
    // beta = 0: the first xpay gives p = r
    BSM_HIP(hipMemcpyAsync(B.scal, hs, block_scal_doubles() * 8, hipMemcpyHostToDevice, st));
    BSM_HIP(hipMemcpyAsync(B.mask, hmask, 64 * sizeof(int), hipMemcpyHostToDevice, st));
    BSM_HIP(hipStreamSynchronize(st));
    // ---- capture K iterations once
    // default replay length: 8 iterations for the FP32 recurrence, 4 for the
    // FP16 one, whose recurrence runs ahead of the true residual sooner
    // (24^3 x 48 SU(4) adjoint, 16 RHS: FP32 K = 8 0.590 s, K = 4 0.719 s;
    // F16S K = 8 0.758 s, K = 4 0.560 s, K = 2 0.62-0.76 s)
    const int K0 = B.half ? 4 : 8;
    B.K = std::max(1, std::min(B.prm->check_every > 0 ? B.prm->check_every : K0, kBlockHist));
    hipGraph_t graph = nullptr;
    BSM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    bsm_status cap = BSM_OK;
    for (int k = 0; k < B.K && cap == BSM_OK; k++) cap = block_iteration(B, k);
    hipError_t ce = hipStreamEndCapture(st, &graph);
    struct GraphGuard {
        hipGraph_t g;
        hipGraphExec_t *e;
        ~GraphGuard() {
            if (g) (void)hipGraphDestroy(g);
            if (*e) (void)hipGraphExecDestroy(*e);
            *e = nullptr;
        }
    } graph_guard{graph, &B.graph};
    if (cap != BSM_OK) return cap;
    BSM_HIP(ce);
    BSM_HIP(hipGraphInstantiate(&B.graph, graph, nullptr, nullptr, 0));

    const double delta2 = B.prm->delta > 0 ? B.prm->delta * B.prm->delta : 0.01;
    int it = 0, active = n;
    std::vector<int> iters(n, 0), updates(n, 0), restarts(n, 0);
    std::vector<bsm_status> status(n, BSM_ERR_NOT_CONVERGED);
    std::vector<double> prev(kNR, 0.0);
    for (int r = 0; r < n; r++) prev[r] = rr[r];
    unsigned waiting = 0;   // RHS whose recomputed residual met the trigger, waiting for the others
    int waited = 0;         // replays since the first of them started waiting
    constexpr int kMaxWait = 4;   // then they are judged alone (their recurrence keeps shrinking)
    while (active > 0 && it < B.prm->max_iter) {
        BSM_HIP(hipGraphLaunch(B.graph, st));
        it += B.K;
        BSM_HIP(hipMemcpyAsync(hs, B.scal, block_scal_doubles() * 8, hipMemcpyDeviceToHost, st));
        BSM_HIP(hipStreamSynchronize(st));
        if (trace_enabled()) {
            double mx = 0;
            for (int r = 0; r < n; r++)
                if (hmask[r]) mx = std::max(mx, hs[B_RR * kNR + r] / B.rhs_norm2[r]);
            fprintf(stderr, "[batched] it %d active %d max rel normal residual^2 %.3e\n", it, active, mx);
        }
        // Every block operation serves all 16 columns, so retiring one RHS
        // early saves nothing.  An RHS whose recomputed residual met its
        // trigger waits (no further reliable updates) for the others; the
        // FP64 true residuals are taken once every RHS still running claims
        // convergence, and when they all claim it on their recurrence
        // residuals, before the FP64 normal residual (four FP64 block hops),
        // which only those that miss tol then need.
        unsigned upd = 0, claim = waiting, running = 0;
        std::vector<double> before(kNR, 0.0);
        for (int r = 0; r < n; r++) {
            if (!hmask[r]) continue;
            iters[r] = it;
            bool bad = false;
            for (int k = 0; k < B.K; k++) {
                const double v = hs[(B_HIST + k) * kNR + r];
                if (!std::isfinite(v)) bad = true;
                maxrr[r] = std::max(maxrr[r], v);
            }
            if (bad) {
                status[r] = BSM_ERR_NONFINITE;
                hmask[r] = 0;
                active--;
                waiting &= ~(1u << r);
                claim &= ~(1u << r);
                continue;
            }
            running |= 1u << r;
            const double rnow = hs[B_RR * kNR + r];
            before[r] = B.K >= 2 ? hs[(B_HIST + B.K - 2) * kNR + r] : prev[r];
            prev[r] = rnow;
            if ((waiting >> r) & 1u) continue;
            const bool reached = rnow <= trig[r] * trig[r] * B.rhs_norm2[r];
            if (reached) claim |= 1u << r;
            if (rnow < delta2 * maxrr[r] || reached) upd |= 1u << r;
        }
        const unsigned early = (running && claim == running) ? running : 0;
        waited = waiting ? waited + 1 : 0;
        const unsigned overdue = (!early && waited > kMaxWait) ? waiting : 0;
        if (upd || early || overdue) {
            // fold every x_lo into x64 (exact bookkeeping for all RHS), then
            // replace the residual of the selected RHS by the FP64 one
            TRY(launch_std_block(g, d, n, all, B.x, B.full64, 0, B.xlo, 1, st));
            BSM_HIP(hipMemsetAsync(B.xlo, 0, B.bbB, st));
            auto judge = [&](unsigned sel) -> bsm_status {
                TRY(true_residuals(sel));
                for (int r = 0; r < n; r++) {
                    if (!((sel >> r) & 1u)) continue;
                    if (trace_enabled())
                        fprintf(stderr, "[batched]   rhs %d check: true residual %.3e (trigger %.1e)\n", r, res[r],
                                trig[r]);
                    if (res[r] <= B.prm->tol) {
                        status[r] = BSM_OK;
                        hmask[r] = 0;
                        active--;
                        upd &= ~(1u << r);
                    } else {
                        trig[r] *= 0.3;
                        restarts[r]++;
                    }
                }
                waiting = 0;
                return BSM_OK;
            };
            if (early || overdue) {
                const unsigned sel = early ? early : overdue;
                TRY(judge(sel));
                for (int r = 0; r < n; r++)   // those that missed tol take the reliable update now
                    if (((sel >> r) & 1u) && hmask[r]) upd |= 1u << r;
            }
            unsigned chk = 0;
            if (upd) TRY(refresh(upd));
            for (int r = 0; r < n; r++) {
                if (!((upd >> r) & 1u)) continue;
                if (trace_enabled())
                    fprintf(stderr, "[batched]   rhs %d update: recurrence %.3e recomputed %.3e (rel^2)\n", r,
                            hs[B_RR * kNR + r] / B.rhs_norm2[r], rr[r] / B.rhs_norm2[r]);
                updates[r]++;
                // beta from the recomputed residual, the search direction
                // kept; but when the recomputed residual is not below the
                // recurrence's value two steps back, the recurrence has run
                // ahead of the true residual (as a fast-converging FP16
                // recurrence does within one replay): restart from r (beta 0)
                hs[B_BETA * kNR + r] = (before[r] > 0 && rr[r] < before[r]) ? rr[r] / before[r] : 0.0;
                hs[B_RR * kNR + r] = rr[r];
                maxrr[r] = rr[r];
                prev[r] = rr[r];
                if (rr[r] <= trig[r] * trig[r] * B.rhs_norm2[r] && !(((early | overdue) >> r) & 1u)) chk |= 1u << r;
            }
            unsigned still = 0;
            for (int r = 0; r < n; r++)
                if (hmask[r]) still |= 1u << r;
            if (chk && (chk | waiting) == still) TRY(judge(still));
            else waiting |= chk;
            // only |r|^2 and beta change on the host (rows of the updated RHS;
            // the others carry the values just read back)
            BSM_HIP(hipMemcpyAsync(B.scal + B_RR * kNR, hs + B_RR * kNR, kNR * 8, hipMemcpyHostToDevice, st));
            BSM_HIP(hipMemcpyAsync(B.scal + B_BETA * kNR, hs + B_BETA * kNR, kNR * 8, hipMemcpyHostToDevice, st));
            BSM_HIP(hipMemcpyAsync(B.mask, hmask, 64 * sizeof(int), hipMemcpyHostToDevice, st));
            BSM_HIP(hipStreamSynchronize(st));
        }
    }
    // RHS still running at max_iter: fold the last FP32 part in and judge
    // them by their true residual (a check deferred for the others may pass)
    if (active > 0) {
        TRY(launch_std_block(g, d, n, all, B.x, B.full64, 0, B.xlo, 1, st));
        unsigned left = 0;
        for (int r = 0; r < n; r++)
            if (hmask[r]) left |= 1u << r;
        TRY(true_residuals(left));
        for (int r = 0; r < n; r++)
            if (((left >> r) & 1u) && status[r] != BSM_ERR_NONFINITE && res[r] <= B.prm->tol) status[r] = BSM_OK;
    }
    bsm_status worst = BSM_OK;
    for (int r = 0; r < n; r++) {
        stats[r].iters = iters[r];
        stats[r].reliable_updates = updates[r];
        stats[r].restarts = restarts[r];
        stats[r].true_rel_res = res[r];
        stats[r].converged = status[r] == BSM_OK;
        if (status[r] != BSM_OK && worst == BSM_OK) worst = status[r];
    }
    return worst;
}

}  // namespace bsm

extern "C" bsm_status bsm_batched_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep64,
                                        const bsm_solver_params *prm, int32_t n_rhs, const double *kappas,
                                        const void *b, void *x, bsm_solver_stats *stats, void *stream) {
    if (!ctx || !desc || !prm || !kappas || !b || !x || !stats || !U_rep64) return fail(BSM_ERR_ARG, "null argument");
    if (bsm_rep_dim(desc->N, desc->rep) != desc->d_R || desc->d_R < 2 || desc->d_R > 15)
        return fail(BSM_ERR_ARG, "d_R does not match (N, rep) or is outside [2, 15]");
    if (n_rhs < 1) return fail(BSM_ERR_ARG, "n_rhs must be >= 1");
    if (desc->link_prec & BSM_LINKS_FUNDAMENTAL)
        return fail(BSM_ERR_ARG, "the batched solver needs links stored in the representation");
    for (int r = 0; r < n_rhs; r++)
        if (!(kappas[r] > 0) || !std::isfinite(kappas[r])) return fail(BSM_ERR_ARG, "kappas must be > 0");
    if (!(prm->tol > 0) || prm->max_iter < 1) return fail(BSM_ERR_ARG, "tol > 0 and max_iter >= 1 required");
    if (b == x) return fail(BSM_ERR_ARG, "b and x must differ");
    const Geom &g = ctx->g;
    const int d = desc->d_R;
    const size_t bb64 = spinor_block_bytes(BSM_F64, d, g.Vh_pad);
    hipStream_t user = (hipStream_t)stream;
    BSM_HIP(hipStreamSynchronize(user));
    auto t0 = std::chrono::steady_clock::now();
    bsm_status worst = BSM_OK;
    if (desc->rep != BSM_REP_ADJ) {
        // complex links: no shared-link block kernel; solve one RHS at a time
        // (plain FP64 for an F64 desc, otherwise reliable-update CG with inner
        // precision desc->prec on links converted to desc->link_prec)
        void *Ulo = nullptr;
        if (desc->prec != BSM_F64) {
            if (desc->link_prec == BSM_F64) return fail(BSM_ERR_ARG, "mixed inner solve needs F32 or F16 links");
            const size_t lb = 8 * link_block_bytes(desc->link_prec, false, d, g.Vh_pad);
            TRY(ctx_work_slot(ctx, 1, lb, &Ulo));
            TRY(launch_convert_links(g, d, false, BSM_F64, desc->link_prec, U_rep64, Ulo, user));
        }
        bsm_field_desc d64 = *desc;
        d64.prec = BSM_F64;
        d64.link_prec = BSM_F64;
        for (int r = 0; r < n_rhs; r++) {
            bsm_solver_params p1 = *prm;
            p1.kappa = kappas[r];
            p1.schur = 1;
            p1.variant = Ulo ? BSM_SOLVER_MIXED : BSM_SOLVER_PLAIN;
            bsm_status s = bsm_cg_solve(ctx, Ulo ? desc : &d64, Ulo ? Ulo : U_rep64, U_rep64, &p1,
                                        (const char *)b + r * 2 * bb64, (char *)x + r * 2 * bb64, &stats[r],
                                        stream);
            if (s != BSM_OK && worst == BSM_OK) worst = s;
        }
        return worst;
    }
    hipStream_t st;
    TRY(ctx_solver_stream(ctx, &st));
    for (int r0 = 0; r0 < n_rhs; r0 += kNR) {
        BlockSolve B{};
        B.ctx = ctx;
        B.g = g;
        B.d = d;
        B.n = std::min(kNR, n_rhs - r0);
        B.st = st;
        B.prm = prm;
        B.kappas = kappas + r0;
        B.b = (const char *)b + (size_t)r0 * 2 * bb64;
        B.x = (char *)x + (size_t)r0 * 2 * bb64;
        B.full64 = 2 * bb64;
        B.bb64 = bb64;
        B.bbB = block_parity_bytes(g, d);
        B.bbH = blockh_parity_bytes(g, d);
        B.half = desc->prec == BSM_F16S;
        for (int r = 0; r < B.n; r++) {
            Op o{};
            o.ctx = ctx; o.g = g; o.d = d; o.real = true; o.schur = true; o.kappa = B.kappas[r];
            o.U = U_rep64; o.sprec = BSM_F64; o.lprec = BSM_F64; o.partials = ctx->partials;
            B.ops.push_back(o);
        }
        bsm_status s = solve_block(B, stats + r0);
        if (s != BSM_OK && worst == BSM_OK) worst = s;
        if (s != BSM_OK && s != BSM_ERR_NOT_CONVERGED && s != BSM_ERR_NONFINITE) break;
    }
    (void)hipStreamSynchronize(st);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < n_rhs; r++) stats[r].seconds = secs;
    if (worst == BSM_ERR_NOT_CONVERGED) fail(worst, "max_iter reached before every RHS met tol");
    if (worst == BSM_ERR_NONFINITE) fail(worst, "non-finite value in a reduction");
    return worst;
}
