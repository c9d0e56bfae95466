// General-N kernels instantiated for N = 8 states.
#define QCL_GEN_N 8
#include "kernels_general.inc"
