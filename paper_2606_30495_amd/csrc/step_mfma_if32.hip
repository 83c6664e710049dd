// Instantiation unit: fused step, float32 operands.
#include "step_mfma_kern.h"

MSTEP_UNIT(mstep_f32, false)
