// General-N kernels instantiated for N = 4 states.
#define QCL_GEN_N 4
#include "kernels_general.inc"
