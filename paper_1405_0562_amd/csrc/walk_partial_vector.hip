// Instantiations of the global-table walk kernel k_sfa_global (Algorithm 5,
// Section 5.2) for partial (on-the-fly) D-SFAs whose walk often leaves the
// hot rows (vector re-walks of cold words), all three id widths.
#include "walk.h"

namespace sfa_rt {
SFA_DISPATCH_SPECIAL(uint8_t, true, true);
SFA_DISPATCH_SPECIAL(uint16_t, true, true);
SFA_DISPATCH_SPECIAL(uint32_t, true, true);
}  // namespace sfa_rt
