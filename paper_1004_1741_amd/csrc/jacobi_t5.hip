// Fused Jacobi pass with 5 time levels on chip (kernels in jacobi_impl.h).
#include "jacobi_impl.h"

namespace stk {
template struct JacobiLevels<5>;
}  // namespace stk
