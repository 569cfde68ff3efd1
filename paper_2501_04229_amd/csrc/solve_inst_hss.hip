// Solve kernel instantiations of the ModeHSS precision mode.
#include "solve_kernel.h"

namespace gadi {
GADI_INSTANTIATE_MODE(ModeHSS)
}  // namespace gadi
