// Compile-time specialisation over the colour dimension d_R (2..15).
// Every kernel that holds a site's components in registers is a template on
// D, so loops over colour and spin unroll fully and nothing spills to
// scratch memory for the common sizes.
#pragma once
#include "bsm_internal.h"
#include "otf.h"

// Bit d of BSM_DMASK selects whether d_R = d is compiled (development
// builds may restrict it to shorten compile times; release builds keep all).
#ifndef BSM_DMASK
#define BSM_DMASK 0xFFFC
#endif

namespace bsm {

template <template <int> class F, class... A>
bsm_status dispatch_d(int d, A &&...args) {
    if (d < 2 || d > 15 || !((BSM_DMASK >> d) & 1))
        return fail(BSM_ERR_UNSUPPORTED, "no kernel compiled for d_R = " + std::to_string(d));
    switch (d) {
    case 2: if constexpr ((BSM_DMASK >> 2) & 1) return F<2>::run(args...); break;
    case 3: if constexpr ((BSM_DMASK >> 3) & 1) return F<3>::run(args...); break;
    case 4: if constexpr ((BSM_DMASK >> 4) & 1) return F<4>::run(args...); break;
    case 5: if constexpr ((BSM_DMASK >> 5) & 1) return F<5>::run(args...); break;
    case 6: if constexpr ((BSM_DMASK >> 6) & 1) return F<6>::run(args...); break;
    case 7: if constexpr ((BSM_DMASK >> 7) & 1) return F<7>::run(args...); break;
    case 8: if constexpr ((BSM_DMASK >> 8) & 1) return F<8>::run(args...); break;
    case 9: if constexpr ((BSM_DMASK >> 9) & 1) return F<9>::run(args...); break;
    case 10: if constexpr ((BSM_DMASK >> 10) & 1) return F<10>::run(args...); break;
    case 11: if constexpr ((BSM_DMASK >> 11) & 1) return F<11>::run(args...); break;
    case 12: if constexpr ((BSM_DMASK >> 12) & 1) return F<12>::run(args...); break;
    case 13: if constexpr ((BSM_DMASK >> 13) & 1) return F<13>::run(args...); break;
    case 14: if constexpr ((BSM_DMASK >> 14) & 1) return F<14>::run(args...); break;
    case 15: if constexpr ((BSM_DMASK >> 15) & 1) return F<15>::run(args...); break;
    }
    return fail(BSM_ERR_UNSUPPORTED, "no kernel for d_R = " + std::to_string(d));
}

// launchers defined in the .hip sources
bsm_status launch_pack_spinor(const Geom &g, int d, int prec, int n_rhs, const void *canon,
                              void *internal, hipStream_t st, bool unpack);
bsm_status launch_represent(const Geom &g, int N, int rep, int d, int link_prec, const void *Uc,
                            void *out, hipStream_t st);
bsm_status launch_convert_links(const Geom &g, int d, bool real, int src_prec, int dst_prec, const void *src,
                                void *dst, hipStream_t st);
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
    int64_t norm_cap;           // slots at norm_partials (checked against the grid)
    // traversal plan (set by launch_hop from the context's tuning):
    //   order 0: workgroup w covers half indices [256 w, 256 w + 256)
    //   order 1: the half lattice is [t][s] with s < S3 = Vh / T split into
    //            256-site tiles; workgroups walk (t-chunk, tile, t in chunk)
    //            with t fastest, so the 8 neighbours of a site are loaded by
    //            workgroups that run at the same time
    //   order 2: as order 0 but workgroups are not regrouped per XCD
    //   order 3: column sweep, one thread per spatial site over tchunk time
    //            slices (time neighbours reused from registers)
    //   order 4: XCD bands: each XCD owns 1/8 of the 256-site tiles of every
    //            time slice and walks them t-major (sites per slice must be a
    //            multiple of 2048)
    // Links are always streamed with non-temporal loads (each link is used
    // once per hop, so it should not displace spinors from L2).
    int order, tchunk;
    // colour split (set by apply_plan from d_R and precision, 0 = off):
    // G threads share one output site, thread g owning colours g, g+G, ...,
    // for the FP64 operators whose one-site-per-thread form spills
    int wide;
};

// colour split used for (d_R, spinor precision): FP64 from d_R = 7 on (measured:
// equal at d_R = 6, 1.4x faster at d_R = 15 than one thread per site)
#ifndef BSM_WIDE_MIN_D
#define BSM_WIDE_MIN_D 7
#endif
inline int hop_wide_of(int d, int prec) {
    return prec == BSM_F64 && d >= BSM_WIDE_MIN_D ? (d <= 8 ? 2 : 4) : 0;
}

// largest d_R compiled with the column sweep (its register ring grows with d_R)
constexpr int kColMaxD = 6;

// workgroups of a hop launch under its plan (= number of norm partials)
inline int hop_grid(const Geom &g, const HopArgs &a) {
    if (a.wide > 0) {
        const int spw = 256 / a.wide;   // sites per workgroup
        return (g.Vh + spw - 1) / spw * a.np;
    }
    int per = (g.Vh + 255) / 256;
    if (a.order == 3) per = (g.Vh / g.L[0] / 256) * (g.L[0] / a.tchunk);
    return per * a.np;
}

// fill a.order / a.tchunk / a.nt from the context's plan for this operator
// (falls back to order 0 where the lattice does not tile)
void apply_plan(bsm_ctx ctx, int d, bool real, int prec, int link_prec, HopArgs &a);
bsm_status launch_hop(const Geom &g, int d, bool real, int prec, int link_prec, const HopArgs &a,
                      hipStream_t st);
// one (spinor precision, link precision, d_R) instance; defined in hop.h and
// explicitly instantiated in the hop_*.hip sources
template <int SP, int LP, int D>
bsm_status hop_run(const Geom &g, bool real, const HopArgs &a, hipStream_t st);
// fundamental links, representation RN = otf_rn(rep, N) formed on the fly;
// defined in hop.h, instantiated in hop_otf.hip
template <int SP, int LP, int RN>
bsm_status hop_run_otf(const Geom &g, const HopArgs &a, hipStream_t st);
int hop_blocks(const Geom &g);

}  // namespace bsm
