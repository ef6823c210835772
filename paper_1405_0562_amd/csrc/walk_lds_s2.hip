// Stride-2 instantiations of the LDS walk kernel k_sfa_lds (Algorithm 5,
// Section 5.2), one translation unit per stride.
#include "walk.h"

namespace sfa_rt {
SFA_DISPATCH_SHAPE(2);
}  // namespace sfa_rt
