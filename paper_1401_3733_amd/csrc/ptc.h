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
bsm_status launch_adam(void *w, const void *g, void *mv, int n, float lr, float b1, float b2, float eps, int t,
                       hipStream_t st);

}  // namespace bsm
