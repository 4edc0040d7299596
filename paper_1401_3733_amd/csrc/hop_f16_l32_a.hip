// Hopping-term instances: spinors BSM_F16S, links BSM_F32, d_R 2..8.
#include "hop.h"

namespace bsm {
#if (BSM_DMASK >> 2) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F32, 2)
#endif
#if (BSM_DMASK >> 3) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F32, 3)
#endif
#if (BSM_DMASK >> 4) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F32, 4)
#endif
#if (BSM_DMASK >> 5) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F32, 5)
#endif
#if (BSM_DMASK >> 6) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F32, 6)
#endif
#if (BSM_DMASK >> 7) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F32, 7)
#endif
#if (BSM_DMASK >> 8) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F32, 8)
#endif
}  // namespace bsm
