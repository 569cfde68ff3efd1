// Solve kernel instantiations of the ModeF16 precision mode.
#include "solve_kernel.h"

namespace gadi {
GADI_INSTANTIATE_MODE(ModeF16)
}  // namespace gadi
