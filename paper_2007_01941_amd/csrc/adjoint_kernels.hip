// Adjoint kernels of the LM step (differentiation form).
#include "kernels.hpp"

namespace bamg {}  // namespace bamg
