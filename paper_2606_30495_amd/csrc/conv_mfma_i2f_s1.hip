// Instantiation unit: 2D, float32 operands, stride-1 convolutions.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_2f_s1, 2, false, s1)
