// Fused Jacobi pass with 3 time levels on chip (kernels in jacobi_impl.h).
#include "jacobi_impl.h"

namespace stk {
template struct JacobiLevels<3>;
}  // namespace stk
