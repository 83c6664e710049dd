// Instantiation unit: 3D, bf16 operands, restriction and prolongation.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_3b_st, 3, true, st)
