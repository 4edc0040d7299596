// Compile-time specialisation over the colour dimension d_R (2..15).
// Every kernel that holds a site's components in registers is a template on
// D, so loops over colour and spin unroll fully and nothing spills to
// scratch memory for the common sizes.
#pragma once
#include "bsm_internal.h"

namespace bsm {

template <template <int> class F, class... A>
bsm_status dispatch_d(int d, A &&...args) {
    switch (d) {
    case 2: return F<2>::run(args...);
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    case 9: return F<9>::run(args...);
    case 10: return F<10>::run(args...);
    case 11: return F<11>::run(args...);
    case 12: return F<12>::run(args...);
    case 13: return F<13>::run(args...);
    case 14: return F<14>::run(args...);
    case 15: return F<15>::run(args...);
    }
    return fail(BSM_ERR_UNSUPPORTED, "no kernel for d_R = " + std::to_string(d));
}

// launchers defined in the .hip sources
bsm_status launch_pack_spinor(const Geom &g, int d, int prec, int n_rhs, const void *canon,
                              void *internal, hipStream_t st, bool unpack);
bsm_status launch_represent(const Geom &g, int N, int rep, int d, int link_prec, const void *Uc,
                            void *out, hipStream_t st);
bsm_status launch_unpack_gauge(const Geom &g, int d, bool real, int link_prec, const void *in,
                               void *canon, hipStream_t st);

// Hopping term on one or both parities:
//   out[p] = a * x[p] + b * H_{p,1-p} in[p]     for p in parities
// in[p] is the block of parity 1-p read to produce parity p.
// norm_partials (nullable): per-block FP64 partial sums of |out|^2, written at
// partials[p * nblk + block], nblk = ceil(Vh / 256).
struct HopArgs {
    const void *U;
    const void *in[2];
    const void *x[2];
    void *out[2];
    double a, b;
    int dagger;
    int p0, np;                 // first output parity, number of parities (1 or 2)
    double *norm_partials;
};
bsm_status launch_hop(const Geom &g, int d, bool real, int prec, int link_prec, const HopArgs &a,
                      hipStream_t st);
// one (spinor precision, link precision, d_R) instance; defined in hop.h and
// explicitly instantiated in the hop_*.hip sources
template <int SP, int LP, int D>
bsm_status hop_run(const Geom &g, bool real, const HopArgs &a, hipStream_t st);
int hop_blocks(const Geom &g);

}  // namespace bsm
