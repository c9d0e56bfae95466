// General-N kernels instantiated for N = 2 states.
#define QCL_GEN_N 2
#include "kernels_general.inc"
