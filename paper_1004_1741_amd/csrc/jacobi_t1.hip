// Fused Jacobi pass with 1 time level on chip (kernels in jacobi_impl.h).
#include "jacobi_impl.h"

namespace stk {
template struct JacobiLevels<1>;
}  // namespace stk
