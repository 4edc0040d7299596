// Hopping-term instances with fundamental links and the representation
// formed on the fly: two-index symmetric N = 2, 3, 4; antisymmetric N = 3, 4;
// adjoint N = 2, 3, 4.  FP32 and FP16+scale spinors (FP32 or FP16 links)
// for all of them, FP64 where d_R <= 6.
#include "hop.h"

namespace bsm {

#define BSM_OTF_INSTANTIATE(SP, LP, RN) \
    template bsm_status hop_run_otf<SP, LP, RN>(const Geom &, const HopArgs &, hipStream_t);

#define BSM_OTF_LOWP(RN)                            \
    BSM_OTF_INSTANTIATE(BSM_F32, BSM_F32, RN)       \
    BSM_OTF_INSTANTIATE(BSM_F16S, BSM_F32, RN)      \
    BSM_OTF_INSTANTIATE(BSM_F16S, BSM_F16S, RN)

BSM_OTF_LOWP(otf_rn(BSM_REP_SYM, 2))
BSM_OTF_LOWP(otf_rn(BSM_REP_SYM, 3))
BSM_OTF_LOWP(otf_rn(BSM_REP_SYM, 4))
BSM_OTF_LOWP(otf_rn(BSM_REP_ASYM, 3))
BSM_OTF_LOWP(otf_rn(BSM_REP_ASYM, 4))
BSM_OTF_LOWP(otf_rn(BSM_REP_ADJ, 2))
BSM_OTF_LOWP(otf_rn(BSM_REP_ADJ, 3))
BSM_OTF_LOWP(otf_rn(BSM_REP_ADJ, 4))

BSM_OTF_INSTANTIATE(BSM_F64, BSM_F64, otf_rn(BSM_REP_SYM, 2))
BSM_OTF_INSTANTIATE(BSM_F64, BSM_F64, otf_rn(BSM_REP_SYM, 3))
BSM_OTF_INSTANTIATE(BSM_F64, BSM_F64, otf_rn(BSM_REP_ASYM, 3))
BSM_OTF_INSTANTIATE(BSM_F64, BSM_F64, otf_rn(BSM_REP_ASYM, 4))
BSM_OTF_INSTANTIATE(BSM_F64, BSM_F64, otf_rn(BSM_REP_ADJ, 2))

}  // namespace bsm
