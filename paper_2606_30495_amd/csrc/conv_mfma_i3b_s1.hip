// Instantiation unit: 3D, bf16 operands, stride-1 convolutions.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_3b_s1, 3, true, s1)
