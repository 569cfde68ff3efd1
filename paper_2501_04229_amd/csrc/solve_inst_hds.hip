// Solve kernel instantiations of the ModeHDS precision mode.
#include "solve_kernel.h"

namespace gadi {
GADI_INSTANTIATE_MODE(ModeHDS)
}  // namespace gadi
