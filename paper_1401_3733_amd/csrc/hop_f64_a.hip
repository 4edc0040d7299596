// Hopping-term instances: spinors BSM_F64, links BSM_F64, d_R 2..8.
#include "hop.h"

namespace bsm {
#if (BSM_DMASK >> 2) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 2)
#endif
#if (BSM_DMASK >> 3) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 3)
#endif
#if (BSM_DMASK >> 4) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 4)
#endif
#if (BSM_DMASK >> 5) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 5)
#endif
#if (BSM_DMASK >> 6) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 6)
#endif
#if (BSM_DMASK >> 7) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 7)
#endif
#if (BSM_DMASK >> 8) & 1
BSM_HOP_INSTANTIATE(BSM_F64, BSM_F64, 8)
#endif
}  // namespace bsm
