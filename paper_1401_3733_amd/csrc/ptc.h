// PTC (parallel-transport convolution) layers: launch interface.
#pragma once
#include "bsm_internal.h"

namespace bsm {

constexpr int kPtcMaxD = 6;   // colour dimensions compiled for the network kernels

struct PtcArgs {
    const void *U;      // F32 links (complex), internal layout
    const void *W;      // complex float [cout][cin][9][4][4]
    const void *in;     // cin F32 full fields (layer input v)
    void *out;          // cout F32 full fields
    const void *G;      // weight gradient: cout F32 full fields (output gradient)
    int cin, cout;
    // matrix-core path (both nullable: then the vector-ALU kernels run)
    float *Areal;       // real form of the mixing matrix, ptc_areal_floats()
    char *Gmix;         // mixed fields for cin > cout: cout * 9 F32 full fields
};

// scratch of the matrix-core path
size_t ptc_areal_floats(int cin, int cout);
size_t ptc_gmix_bytes(const Geom &g, int d, int cin, int cout);
bsm_status launch_ptc_layer(const Geom &g, int d, const PtcArgs &a, hipStream_t st);
// dW (complex float, cout*cin*9*16) = scale * sum_x G (x) conj(T_p v); accumulate adds
int ptc_wgrad_blocks(const Geom &g);
bsm_status launch_ptc_wgrad(const Geom &g, int d, const PtcArgs &a, double2 *partials, float2 *dW, double scale,
                            bool accumulate, hipStream_t st);
bsm_status launch_ptc_adjoint_weights(const void *W, void *Wa, int cin, int cout, hipStream_t st);
// The 1 -> C -> 1 network as one operator (both layers are linear):
// z = cs * sum_p T_p (S * G'_p), with G'_p, S and cs built as described in
// ptc_fast.hip.  Scratch: net_fast_bytes(), carved by net_fast_carve().
struct NetFastArgs {
    const void *U;       // links (complex), internal layout, in link_prec
    int link_prec;       // BSM_F32 or BSM_F16S
    const void *in;      // F32 full field v
    void *out;           // F32 full field z
    void *G;             // nine FP16 mixed fields (both parities)
    float *S;            // per-site scale of the mixed fields
    const void *Afrag;   // FP16 real form of C / cs, matrix-core lane order
    const float *cs;     // largest |entry| of C
};
size_t net_fast_bytes(const Geom &g, int d);
void net_fast_carve(const Geom &g, int d, void *scratch, NetFastArgs &a);
bool net_fast_supported(int d);
// C_pq = sum_j W2_p^{0j} W1_q^{j0} -> a.Afrag, a.cs (net: W1 then W2, complex float)
bsm_status launch_net_collapse(const void *net, int C, const NetFastArgs &a, hipStream_t st);
bsm_status launch_net_fast(const Geom &g, int d, const NetFastArgs &a, hipStream_t st);
bsm_status launch_adam(void *w, const void *g, void *mv, int n, float lr, float b1, float b2, float eps, int t,
                       hipStream_t st);

}  // namespace bsm
