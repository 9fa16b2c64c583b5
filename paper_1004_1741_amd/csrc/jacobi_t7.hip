// Fused Jacobi pass with 7 time levels on chip (kernels in jacobi_impl.h).
#include "jacobi_impl.h"

namespace stk {
template struct JacobiLevels<7>;
}  // namespace stk
