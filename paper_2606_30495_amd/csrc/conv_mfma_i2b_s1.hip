// Instantiation unit: 2D, bf16 operands, stride-1 convolutions.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_2b_s1, 2, true, s1)
