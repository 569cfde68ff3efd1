// Solve kernel instantiations of the ModeF64 precision mode.
#include "solve_kernel.h"

namespace gadi {
GADI_INSTANTIATE_MODE(ModeF64)
}  // namespace gadi
