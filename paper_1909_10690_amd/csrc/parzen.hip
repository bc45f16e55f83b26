// Parzen (cubic B-spline) joint histogram and its backward pass.
#include "common.h"

namespace gemi {

hipError_t configure_parzen_kernels() { return hipSuccess; }

}  // namespace gemi
