// Vector-Jacobian product kernels (placeholder until the reverse sweep lands).
#include "sgp4mi_common.h"

namespace sgp4mi {

hipError_t launch_vjp(int precision, int64_t n, const double* elem, const void* consts, const double* t, int64_t T,
                      const void* gr, const void* gv, double* gelem, hipStream_t s) {
  (void)precision; (void)n; (void)elem; (void)consts; (void)t; (void)T; (void)gr; (void)gv; (void)gelem; (void)s;
  return hipErrorNotSupported;
}

}  // namespace sgp4mi
