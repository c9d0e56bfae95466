// General-N kernels instantiated for N = 2 states, models with higher
// separable powers of each mode and five to eight cross-mode bilinear
// terms (sixteen squared combinations, at most 16 modes).
#define QCL_GEN_N 2
#define QCL_GEN_POLY 1
#define QCL_GEN_BIL 1
#define QCL_GEN_BIL_SQ 16
#include "kernels_general.inc"
