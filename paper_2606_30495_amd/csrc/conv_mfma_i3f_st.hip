// Instantiation unit: 3D, float32 operands, restriction and prolongation.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_3f_st, 3, false, st)
