// Instantiations of the global-table walk kernel k_sfa_global (Algorithm 5,
// Section 5.2) for partial (on-the-fly) D-SFAs, all three id widths.
#include "walk.h"

namespace sfa_rt {
SFA_DISPATCH_SPECIAL(uint8_t, true, false);
SFA_DISPATCH_SPECIAL(uint16_t, true, false);
SFA_DISPATCH_SPECIAL(uint32_t, true, false);
}  // namespace sfa_rt
