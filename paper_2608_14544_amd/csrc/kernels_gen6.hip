// General-N kernels instantiated for N = 6 states.
#define QCL_GEN_N 6
#include "kernels_general.inc"
