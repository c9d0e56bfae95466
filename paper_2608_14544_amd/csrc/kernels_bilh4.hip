// General-N kernels instantiated for N = 4 states, models with higher
// separable powers of each mode and at most two cross-mode bilinear terms
// (four squared combinations).
#define QCL_GEN_N 4
#define QCL_GEN_POLY 1
#define QCL_GEN_BIL 1
#define QCL_GEN_BIL_SQ 4
#include "kernels_general.inc"
