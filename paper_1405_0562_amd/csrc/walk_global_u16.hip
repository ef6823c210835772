// Instantiations of the global-table walk kernel k_sfa_global (Algorithm 5,
// Section 5.2) for u16 D-SFA state ids, one translation unit per id width.
#include "walk.h"

namespace sfa_rt {
SFA_DISPATCH_GLOBAL(uint16_t);
}  // namespace sfa_rt
