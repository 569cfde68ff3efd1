// Solve kernel instantiations of the ModeF8 precision mode.
#include "solve_kernel.h"

namespace gadi {
GADI_INSTANTIATE_MODE(ModeF8)
}  // namespace gadi
