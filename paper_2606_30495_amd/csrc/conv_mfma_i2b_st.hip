// Instantiation unit: 2D, bf16 operands, restriction and prolongation.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_2b_st, 2, true, st)
