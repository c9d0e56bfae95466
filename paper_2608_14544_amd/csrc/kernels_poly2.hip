// General-N kernels instantiated for N = 2 states, models with higher
// separable powers of each mode.
#define QCL_GEN_N 2
#define QCL_GEN_POLY 1
#include "kernels_general.inc"
