// Instantiations of the global-table walk kernel k_sfa_global (Algorithm 5,
// Section 5.2) for partial (on-the-fly) D-SFAs, all three id widths.
#include "walk.h"

namespace sfa_rt {
SFA_DISPATCH_PARTIAL(uint8_t);
SFA_DISPATCH_PARTIAL(uint16_t);
SFA_DISPATCH_PARTIAL(uint32_t);
}  // namespace sfa_rt
