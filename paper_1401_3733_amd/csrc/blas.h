// Site-wise Krylov vector kernels on internal spinor fields.
#pragma once
#include "bsm_internal.h"

namespace bsm {

// A spinor vector: nblk consecutive parity blocks of one precision.
struct Vec {
    void *ptr;
    int prec;
};

// Reductions: every kernel that reduces writes one FP64 partial per
// workgroup (fixed-order wavefront shuffles, then the 4 waves in order);
// reduce_into sums the partials in a fixed order on one workgroup, so every
// result is bitwise reproducible run to run.
int blas_blocks(const Geom &g, int nblk);

// out = a*A + b*B (B may be null); optional |out|^2 partials.
bsm_status blas_axpby(const Geom &g, int d, int nblk, Vec out, double a, Vec A, double b, Vec B,
                      double *partials, hipStream_t st);
// partials of |A|^2, or of Re<A, B> when B.ptr != null
bsm_status blas_dot(const Geom &g, int d, int nblk, Vec A, Vec B, double *partials, hipStream_t st);
// CG update with alpha = scal[ia]:  x += alpha p ; r -= alpha q ; partials of |r|^2
bsm_status blas_cg_update(const Geom &g, int d, int nblk, Vec x, Vec p, Vec r, Vec q,
                          const double *scal, int ia, double *partials, hipStream_t st);
// p = r + scal[ib] * p
bsm_status blas_cg_xpay(const Geom &g, int d, int nblk, Vec p, Vec r, const double *scal, int ib,
                        hipStream_t st);
// p_out = r + scal[ib] * p_in
bsm_status blas_cg_xpay_to(const Geom &g, int d, int nblk, Vec p_out, Vec p_in, Vec r, const double *scal, int ib,
                           hipStream_t st);
// x += sum_k alphas[k] p_k, p_k = ring slot (slot0 + k) % ring of pbase (slots pstride bytes apart)
bsm_status blas_x_flush(const Geom &g, int d, int nblk, Vec x, const char *pbase, int pprec, size_t pstride,
                        int ring, int slot0, int kn, const double *alphas, hipStream_t st);

// dst[0] = sum of n partials (fixed order)
bsm_status reduce_into(const double *partials, int n, double *dst, hipStream_t st);
// CG scalar steps, all on the device:
//   op 0 (alpha): scal[PAP] = sum partials; alpha = rr / pAp (0 if pAp <= 0 or not finite)
//   op 1 (beta) : rr_new = sum partials; beta = rr_new / rr; rr = rr_new; hist[it] = rr_new
//   op 2 (init) : rr = sum partials; hist[it] = rr
bsm_status cg_scalars(const double *partials, int n, double *scal, int op, int it, hipStream_t st);

// device scalar slots
enum { S_RR = 0, S_PAP = 1, S_ALPHA = 2, S_BETA = 3, S_TMP = 4, S_TMP2 = 5, S_AHIST = 16, S_HIST = 64 };
constexpr int kAlphaHist = S_HIST - S_AHIST;   // alpha of each iteration of a chunk (cg_scalars op 0, it >= 0)

}  // namespace bsm
