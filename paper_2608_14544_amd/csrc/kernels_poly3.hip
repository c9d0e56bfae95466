// General-N kernels instantiated for N = 3 states, models with higher
// separable powers of each mode.
#define QCL_GEN_N 3
#define QCL_GEN_POLY 1
#include "kernels_general.inc"
