// General-N kernels instantiated for N = 5 states.
#define QCL_GEN_N 5
#include "kernels_general.inc"
