// One-pass full-lattice Wilson operator (both parities): declarations.
#pragma once
#include "bsm_internal.h"

namespace bsm {

struct DphiArgs {
    const void *U;      // links, internal layout (both parities)
    const void *in;     // full field
    void *out;          // full field (must not overlap in)
    double a, b;        // out = a in + b H in
    int dagger;
    int tc;             // time slices per thread (divides T)
};

// where the kernel is used: FP32 up to d_R = 3 (measured at 32^3 x 64:
// SU(3) 303 -> 228 us, SU(2) 158 -> 128 us; SU(6) FP32 and every FP64 case
// hold more column state than two wavefronts per SIMD fit, and were slower
// than the even-odd hop applied to both parities)
constexpr bool dphi_compiled(int sp, int d) { return sp == BSM_F32 && d <= 3; }
// lattices the kernel covers: LX divides 64 and is at most 32 (two or more
// whole x-rows per wavefront), LY a multiple of 64 / LX
bool dphi_fits(const Geom &g);
int dphi_tchunk(const Geom &g);
bsm_status launch_dphi(const Geom &g, int d, bool real, int prec, int link_prec, const DphiArgs &a,
                       hipStream_t st);

}  // namespace bsm
