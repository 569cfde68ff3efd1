// Batched (alpha, omega) sweep: placeholder entry point until the persistent
// multi-system kernel lands.
#include "internal.h"

extern "C" gadi_status gadi_ir_solve_batched(gadi_handle* const* hs, int32_t nsys, const double* const* b,
                                             double* const* x, const double* alpha, const double* omega,
                                             int32_t ntrial, double tol, const gadi_options* opts,
                                             gadi_solve_info* info) {
  (void)hs; (void)nsys; (void)b; (void)x; (void)alpha; (void)omega; (void)ntrial; (void)tol; (void)opts; (void)info;
  return GADI_EINVAL;
}
