// Solve kernel instantiations of the ModeF32 precision mode.
#include "solve_kernel.h"

namespace gadi {
GADI_INSTANTIATE_MODE(ModeF32)
}  // namespace gadi
