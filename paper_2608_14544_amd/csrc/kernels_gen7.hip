// General-N kernels instantiated for N = 7 states.
#define QCL_GEN_N 7
#include "kernels_general.inc"
