// Fused matrix-core smoothing step (see step_mfma.hip).
#pragma once
#include "internal.h"

namespace mcmg {

// One fused step of a 2D level with C >= 8 channels: e' = e + Wsm * (s (.)
// (KS * (r - W * e - a (.) (KA * e)))) (var L1_STEP) or e' = Wsm * (s (.)
// (KS * r)) (var L1_FIRST, e = 0), written to eo (eo != e).  Weights are the
// packed matrix-core tensors [4 nsteps][ncols][KV] of the level.
struct StepLaunch {
  int var;                    // L1_STEP or L1_FIRST
  int bf16;                   // operand precision
  int tile;                   // tile id: 0 = 16x4, 1 = 32x4, 2 = 32x8, 3 = 64x8 nodes (x, y)
  int kc1, kc2;               // weight chunk (K-steps) of the W/KA phase and of the KS/Wsm phases
  const float* e;
  float* eo;
  const float *r, *a, *s;
  const void *wW, *wKA, *wKS, *wSM;
  int C, cinp, ncols, nsteps, npairs;
  Dims n;
};

struct SArgs {
  const float* e;
  float* eo;
  const float *r, *a, *s;
  const void *wW, *wKA, *wKS, *wSM;
  int C, cinp, ncols, nsteps, npairs, kc1, kc2;
  Dims n;
  int tiles_x, tiles_y;
};

SArgs step_args(const StepLaunch& l, int* nblk);
size_t mstep_lds_bytes(int tile, int bf16, int nct, int cinp, int kc1, int kc2);
void mstep_tile(int tile, int* TX, int* TY);
hipError_t launch_step(const StepLaunch& l, hipStream_t s);
hipError_t launch_step_batched(const StepLaunch& proto, const BatchLaunch& b, hipStream_t s);
const char* step_kernel_name(const StepLaunch& l);

}  // namespace mcmg
