// Instantiation unit: 2D, float32 operands, restriction and prolongation.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_2f_st, 2, false, st)
