// Instantiation unit: fused step, bf16 operands.
#include "step_mfma_kern.h"

MSTEP_UNIT(mstep_bf, true)
