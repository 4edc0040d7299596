// Shared pieces of the solvers (CG, batched, FGCR): the operator whose
// normal equations are solved and the FP64 residual helpers.
#pragma once
#include "blas.h"
#include "dispatch.h"

namespace bsm {

// D (full lattice) or the even-odd Schur complement Dhat, in one storage
// precision, with its scratch.
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


size_t blk(const Op &o);
int nblk_vec(const Op &o);
// y = M x or M^dag x; |y|^2 partials when norm (count in *np)
bsm_status op_apply(const Op &o, int dagger, const void *x, void *y, bool norm, int *np, hipStream_t st);
// sum n partials on the device, result on the host (synchronous)
double reduce_to_host(bsm_ctx ctx, const double *partials, int n, hipStream_t st);
// FP64: out = M^dag (bh - M x), t scratch
bsm_status normal_residual(const Op &o, const char *bh, const char *x, char *t, char *out, hipStream_t st);
// FP64 ||b - D x|| / ||b|| of the full system (Schur: odd sites of x rebuilt)
bsm_status true_residual_full(const Op &o, const char *b, char *x, char *tfull, double bnorm2, double *res,
                              hipStream_t st);

}  // namespace bsm
