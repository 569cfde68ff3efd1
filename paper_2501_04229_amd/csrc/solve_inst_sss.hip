// Solve kernel instantiations of the ModeSSS precision mode.
#include "solve_kernel.h"

namespace gadi {
GADI_INSTANTIATE_MODE(ModeSSS)
}  // namespace gadi
