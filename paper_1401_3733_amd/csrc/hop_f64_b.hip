// Hopping-term instances: spinors BSM_F64, links BSM_F64, d_R 9..15.
#include "hop.h"

namespace bsm {
#if (BSM_DMASK >> 9) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 9)
#endif
#if (BSM_DMASK >> 10) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 10)
#endif
#if (BSM_DMASK >> 11) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 11)
#endif
#if (BSM_DMASK >> 12) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 12)
#endif
#if (BSM_DMASK >> 13) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 13)
#endif
#if (BSM_DMASK >> 14) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 14)
#endif
#if (BSM_DMASK >> 15) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 15)
#endif
}  // namespace bsm
