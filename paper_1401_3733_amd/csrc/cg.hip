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

struct Op {
    bsm_ctx ctx;
    Geom g;
    int d;
    bool real;
    bool schur;
    double kappa;
    const void *U;
    int sprec, lprec;
    void *tmp;      // one parity block in sprec (Schur intermediate)
    double *partials;
};

static size_t blk(const Op &o) { return spinor_block_bytes(o.sprec, o.d, o.g.Vh_pad); }
static int nblk_vec(const Op &o) { return o.schur ? 1 : 2; }

// y = M x or M^dag x; norm partials of y when partials != null (count in *np)
static bsm_status op_apply(const Op &o, int dagger, const void *x, void *y, bool norm, int *np,
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
    apply_plan(o.ctx, o.d, o.real, o.sprec, o.lprec, a);
    if (np) *np = hop_grid(o.g, a);
    return launch_hop(o.g, o.d, o.real, o.sprec, o.lprec, a, st);
}

#define TRY(x)                           \
    do {                                 \
        bsm_status _s = (x);             \
        if (_s != BSM_OK) return _s;     \
    } while (0)

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

    double host_reduce(const double *partials, int n) {
        reduce_into(partials, n, ctx->scal + S_TMP, st);
        hipMemcpyAsync(ctx->host_scal + S_TMP, ctx->scal + S_TMP, sizeof(double), hipMemcpyDeviceToHost, st);
        hipStreamSynchronize(st);
        return ctx->host_scal[S_TMP];
    }

    // even block (Schur) or the full field of the caller's x / b
    char *xv() { return x; }

    // FP64: out = M^dag (bhat - M x64)   (uses t64 as scratch)
    bsm_status normal_residual64(const char *x64, char *out) {
        Vec T{t64, BSM_F64}, BH{bh, BSM_F64};
        TRY(op_apply(op64, 0, x64, t64, false, nullptr, st));
        TRY(blas_axpby(g, d, nblk_vec(op64), T, -1.0, T, 1.0, BH, nullptr, st));
        return op_apply(op64, 1, t64, out, false, nullptr, st);
    }

    // reconstruct odd sites (Schur) and return the FP64 true relative residual
    bsm_status true_residual(double *res) {
        if (schur) {
            HopArgs a{};
            a.U = op64.U; a.dagger = 0; a.p0 = 1; a.np = 1;
            a.in[1] = x; a.x[1] = b + bb64; a.out[1] = x + bb64;
            a.a = 1.0; a.b = kappa;
            TRY(launch_hop(g, d, real, BSM_F64, BSM_F64, a, st));
        }
        // tfull = D x ; tfull = b - tfull ; |.|^2
        HopArgs a{};
        a.U = op64.U; a.dagger = 0; a.p0 = 0; a.np = 2;
        a.in[0] = x + bb64; a.in[1] = x; a.x[0] = x; a.x[1] = x + bb64;
        a.out[0] = tfull; a.out[1] = tfull + bb64;
        a.a = 1.0; a.b = -kappa;
        TRY(launch_hop(g, d, real, BSM_F64, BSM_F64, a, st));
        Vec TF{tfull, BSM_F64}, B{(void *)b, BSM_F64};
        TRY(blas_axpby(g, d, 2, TF, -1.0, TF, 1.0, B, ctx->partials, st));
        double rn = host_reduce(ctx->partials, blas_blocks(g, 2));
        *res = bnorm2 > 0 ? std::sqrt(rn / bnorm2) : std::sqrt(rn);
        return BSM_OK;
    }

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
            TRY(launch_hop(g, d, real, BSM_F64, BSM_F64, a, st));
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
    void *work = nullptr;
    TRY(ctx_work(S.ctx, base + 3 * vlo + 2 * vacc + spinor_block_bytes(inner_prec, d, g.Vh_pad), &work));
    TRY(S.setup(work));
    char *w = (char *)work + base;
    char *p = w; w += vlo;
    char *t = w; w += vlo;
    char *q = w; w += vlo;
    char *xlo = w; w += vacc;
    char *rlo = w; w += vacc;
    lo.tmp = w;
    hipStream_t st = S.st;
    double *scal = S.ctx->scal;
    double *hs = S.ctx->host_scal;
    Vec X64{S.x, BSM_F64}, R64{S.r64, BSM_F64};
    Vec P{p, inner_prec}, Q{q, inner_prec}, XL{xlo, acc_prec}, RL{rlo, acc_prec};
    Vec none{nullptr, BSM_F64};
    const int hist_cap = kScalars - S_HIST;
    const double delta2 = S.prm->delta > 0 ? S.prm->delta * S.prm->delta : 0.01;

    // r64 = M^dag (bhat - M x64), |r64|^2 ; r_lo = r64 ; p = r_lo ; x_lo = 0
    auto reliable = [&](double *rr_true) -> bsm_status {
        TRY(S.normal_residual64(S.x, S.r64));
        TRY(blas_dot(g, d, nb, R64, none, S.ctx->partials, st));
        *rr_true = S.host_reduce(S.ctx->partials, blas_blocks(g, nb));
        TRY(blas_axpby(g, d, nb, RL, 1.0, R64, 0.0, none, nullptr, st));
        return BSM_OK;
    };

    double trig = S.prm->tol;
    int it = 0, restarts = 0, updates = 0;
    double res = INFINITY;
    bsm_status status = BSM_ERR_NOT_CONVERGED;
    double rr;
    TRY(reliable(&rr));
    BSM_HIP(hipMemsetAsync(xlo, 0, vacc, st));
    TRY(blas_axpby(g, d, nb, P, 1.0, RL, 0.0, none, nullptr, st));
    hs[S_RR] = rr;
    BSM_HIP(hipMemcpyAsync(scal + S_RR, hs + S_RR, sizeof(double), hipMemcpyHostToDevice, st));
    double maxrr = rr;
    for (;;) {
        const double target = trig * trig * S.rhs_norm2;
        bool check = rr <= target;
        while (!check && it < S.prm->max_iter) {
            int np = 0;
            TRY(op_apply(lo, 0, p, t, true, &np, st));
            TRY(cg_scalars(S.ctx->partials, np, scal, 0, 0, st));
            TRY(op_apply(lo, 1, t, q, false, nullptr, st));
            TRY(blas_cg_update(g, d, nb, XL, P, RL, Q, scal, S_ALPHA, S.ctx->partials, st));
            TRY(cg_scalars(S.ctx->partials, blas_blocks(g, nb), scal, 1, (it + 1) % hist_cap, st));
            it++;
            BSM_HIP(hipMemcpyAsync(hs + S_RR, scal + S_RR, sizeof(double), hipMemcpyDeviceToHost, st));
            BSM_HIP(hipStreamSynchronize(st));
            double rr_new = hs[S_RR];
            if (!std::isfinite(rr_new)) { status = BSM_ERR_NONFINITE; break; }
            if (rr_new < delta2 * maxrr || rr_new <= target) {
                // fold x_lo into x64, recompute the residual in FP64
                TRY(blas_axpby(g, d, nb, X64, 1.0, X64, 1.0, XL, nullptr, st));
                BSM_HIP(hipMemsetAsync(xlo, 0, vacc, st));
                double rr_true;
                TRY(reliable(&rr_true));
                updates++;
                // beta from the recomputed residual, search direction kept
                hs[S_BETA] = rr_true / rr;
                hs[S_RR] = rr_true;
                BSM_HIP(hipMemcpyAsync(scal + S_BETA, hs + S_BETA, sizeof(double), hipMemcpyHostToDevice, st));
                BSM_HIP(hipMemcpyAsync(scal + S_RR, hs + S_RR, sizeof(double), hipMemcpyHostToDevice, st));
                rr = rr_true;
                maxrr = rr_true;
                if (rr_true <= target) check = true;
            } else {
                rr = rr_new;
                if (rr > maxrr) maxrr = rr;
            }
            TRY(blas_cg_xpay(g, d, nb, P, RL, scal, S_BETA, st));
            BSM_HIP(hipStreamSynchronize(st));   // host scalars are reused next iteration
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
        // restart the recurrence from the FP64 residual
        TRY(reliable(&rr));
        TRY(blas_axpby(g, d, nb, P, 1.0, RL, 0.0, none, nullptr, st));
        hs[S_RR] = rr;
        BSM_HIP(hipMemcpyAsync(scal + S_RR, hs + S_RR, sizeof(double), hipMemcpyHostToDevice, st));
        BSM_HIP(hipStreamSynchronize(st));
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
    if (!ctx || !desc || !prm || !b || !x || !stats || !U_rep || !U_rep64)
        return fail(BSM_ERR_ARG, "null argument");
    if (bsm_rep_dim(desc->N, desc->rep) != desc->d_R || desc->d_R < 2 || desc->d_R > 15)
        return fail(BSM_ERR_ARG, "d_R does not match (N, rep) or is outside [2, 15]");
    if (!(prm->kappa > 0) || !std::isfinite(prm->kappa)) return fail(BSM_ERR_ARG, "kappa must be > 0");
    if (!(prm->tol > 0)) return fail(BSM_ERR_ARG, "tol must be > 0");
    if (prm->max_iter < 1) return fail(BSM_ERR_ARG, "max_iter must be >= 1");
    if (b == x) return fail(BSM_ERR_ARG, "b and x must differ");
    if (prm->variant == BSM_SOLVER_PLAIN && (desc->prec != BSM_F64 || desc->link_prec != BSM_F64))
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
    S.real = desc->rep == BSM_REP_ADJ;
    S.schur = prm->schur != 0;
    S.kappa = prm->kappa;
    S.prm = prm;
    S.b = (const char *)b;
    S.x = (char *)x;
    S.op64.ctx = ctx;
    S.op64.g = ctx->g;
    S.op64.d = S.d;
    S.op64.real = S.real;
    S.op64.schur = S.schur;
    S.op64.kappa = prm->kappa;
    S.op64.U = U_rep64;
    S.op64.sprec = BSM_F64;
    S.op64.lprec = BSM_F64;
    S.op64.partials = ctx->partials;
    bsm_status s;
    if (prm->variant == BSM_SOLVER_PLAIN) s = solve_plain(S, stats);
    else s = solve_mixed(S, desc->prec, desc->link_prec, U_rep, stats);
    hipError_t e = hipStreamSynchronize(S.st);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (e != hipSuccess) return hip_check(e, "bsm_cg_solve");
    if (s == BSM_ERR_NOT_CONVERGED) fail(s, "max_iter reached before the true residual met tol");
    if (s == BSM_ERR_NONFINITE) fail(s, "non-finite value in a reduction");
    return s;
}
