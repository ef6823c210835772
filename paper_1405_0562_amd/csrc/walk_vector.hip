// Instantiations of the global-table walk kernel k_sfa_global (Algorithm 5,
// Section 5.2) for complete D-SFAs whose walk often leaves the hot rows: the
// pieces of a wave that leave them re-walk their word with vector loads.
#include "walk.h"

namespace sfa_rt {
SFA_DISPATCH_SPECIAL(uint8_t, false, true);
SFA_DISPATCH_SPECIAL(uint16_t, false, true);
SFA_DISPATCH_SPECIAL(uint32_t, false, true);
}  // namespace sfa_rt
