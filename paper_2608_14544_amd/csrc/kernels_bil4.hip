// General-N kernels instantiated for N = 4 states, models with higher
// separable powers of each mode and cross-mode bilinear terms.
#define QCL_GEN_N 4
#define QCL_GEN_POLY 1
#define QCL_GEN_BIL 1
#include "kernels_general.inc"
