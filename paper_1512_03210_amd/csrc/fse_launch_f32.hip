// Complex64 instantiation of the split-step kernels (FP64 reductions).
#define FSE_REAL float
#include "fse_launch.inc"
