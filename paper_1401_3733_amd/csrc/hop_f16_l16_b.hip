// Hopping-term instances: spinors BSM_F16S, links BSM_F16S, d_R 9..15.
#include "hop.h"

namespace bsm {
#if (BSM_DMASK >> 9) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F16S, 9)
#endif
#if (BSM_DMASK >> 10) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F16S, 10)
#endif
#if (BSM_DMASK >> 11) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F16S, 11)
#endif
#if (BSM_DMASK >> 12) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F16S, 12)
#endif
#if (BSM_DMASK >> 13) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F16S, 13)
#endif
#if (BSM_DMASK >> 14) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F16S, 14)
#endif
#if (BSM_DMASK >> 15) & 1
BSM_HOP_INSTANTIATE(BSM_F16S, BSM_F16S, 15)
#endif
}  // namespace bsm
