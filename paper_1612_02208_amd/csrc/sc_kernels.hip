// Schur-complement smoother kernels (multicolour Gauss-Seidel, Chebyshev).
#include "internal.hpp"

namespace ibmg {}  // namespace ibmg
