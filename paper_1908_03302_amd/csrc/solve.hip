// Solvers on top of the operators (filled in below the apply kernels).
#include "internal.h"
