// General-N kernels instantiated for N = 3 states.
#define QCL_GEN_N 3
#include "kernels_general.inc"
