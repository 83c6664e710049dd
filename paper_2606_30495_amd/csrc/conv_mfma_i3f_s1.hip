// Instantiation unit: 3D, float32 operands, stride-1 convolutions.
#include "conv_mfma_kern.h"

MCONV_UNIT(mconv_3f_s1, 3, false, s1)
