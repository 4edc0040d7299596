// Hopping-term instances: spinors BSM_F32, links BSM_F32, d_R 9..15.
#include "hop.h"

namespace bsm {
#if (BSM_DMASK >> 9) & 1
BSM_HOP_INSTANTIATE(BSM_F32, BSM_F32, 9)
#endif
#if (BSM_DMASK >> 10) & 1
BSM_HOP_INSTANTIATE(BSM_F32, BSM_F32, 10)
#endif
#if (BSM_DMASK >> 11) & 1
BSM_HOP_INSTANTIATE(BSM_F32, BSM_F32, 11)
#endif
#if (BSM_DMASK >> 12) & 1
BSM_HOP_INSTANTIATE(BSM_F32, BSM_F32, 12)
#endif
#if (BSM_DMASK >> 13) & 1
BSM_HOP_INSTANTIATE(BSM_F32, BSM_F32, 13)
#endif
#if (BSM_DMASK >> 14) & 1
BSM_HOP_INSTANTIATE(BSM_F32, BSM_F32, 14)
#endif
#if (BSM_DMASK >> 15) & 1
BSM_HOP_INSTANTIATE(BSM_F32, BSM_F32, 15)
#endif
}  // namespace bsm
