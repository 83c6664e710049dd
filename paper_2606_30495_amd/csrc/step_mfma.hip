// Fused matrix-core smoothing step of a 2D level with C >= 8 channels
// (Sec. 3.2: e += W^(i) * (s_l (.) (KS * (r_l - W_l * e - a_l (.) (KA * e))))).
//
// Unfused, a step is three launches (residual, modulated smoother, update)
// whose intermediates t and u travel through memory; at the coarse levels a
// launch costs more than its work, so the step is latency-bound.  Here one
// block computes the step for one output tile in three phases, each an
// implicit GEMM on the matrix cores whose rows are the nodes of a region
// linearised in chunks of 16:
//   phase 1: t on the tile grown by 2 (A from e staged with a halo of 3),
//            t = r - acc(W) - a (.) acc(KA), zero outside the grid;
//   phase 2: u = s (.) acc(KS) on the tile grown by 1 (A from t in LDS);
//   phase 3: e' = e + acc(Wsm) on the tile (A from u in LDS), written to a
//            second buffer (neighbouring blocks still read e).
// t and u are rounded to the operand type when they enter LDS, exactly where
// the unfused path rounds them when staging the next convolution, and every
// K-sum runs in the same order, so the fused step gives the unfused step's
// bits.  The extra work is the halo recompute of t and u.  Weights come from
// the level's packed tensors and stream through LDS in chunks when a phase's
// tensors do not fit at once.
#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"
#include "step_mfma.h"

namespace mcmg {

hipError_t mstep_bf(const StepLaunch& l, const BatchLaunch* b, hipStream_t s);
hipError_t mstep_f32(const StepLaunch& l, const BatchLaunch* b, hipStream_t s);

void mstep_tile(int tile, int* TX, int* TY) {
  static const int tx[4] = {16, 32, 32, 64}, ty[4] = {4, 4, 8, 8};
  *TX = tx[tile];
  *TY = ty[tile];
}

size_t mstep_lds_bytes(int tile, int bf16, int nct, int cinp, int kc1, int kc2) {
  int TX, TY;
  mstep_tile(tile, &TX, &TY);
  const size_t es = bf16 ? 2 : 4, kv = bf16 ? 8 : 1;
  const size_t stride = cinp + (bf16 ? 8 : 1);
  auto rb = [&](size_t n) { return ((n * stride * es + 15) / 16) * 16; };
  const size_t n0 = (size_t)(TX + 6) * (TY + 6), n1 = (size_t)(TX + 4) * (TY + 4);
  const size_t n2 = (size_t)(TX + 2) * (TY + 2);
  const size_t brow = (size_t)nct * 16 * kv * es;
  const size_t w1 = 2 * 4 * (size_t)kc1 * brow, w2 = 4 * (size_t)kc2 * brow;
  return (rb(n0) > rb(n2) ? rb(n0) : rb(n2)) + rb(n1) + (w1 > w2 ? w1 : w2);
}

SArgs step_args(const StepLaunch& l, int* nblk) {
  int TX, TY;
  mstep_tile(l.tile, &TX, &TY);
  SArgs A;
  A.e = l.e; A.eo = l.eo; A.r = l.r; A.a = l.a; A.s = l.s;
  A.wW = l.wW; A.wKA = l.wKA; A.wKS = l.wKS; A.wSM = l.wSM;
  A.C = l.C; A.cinp = l.cinp; A.ncols = l.ncols; A.nsteps = l.nsteps; A.npairs = l.npairs;
  A.kc1 = l.kc1; A.kc2 = l.kc2;
  A.n = l.n;
  A.tiles_x = (l.n.n[1] + TX - 1) / TX;
  A.tiles_y = (l.n.n[0] + TY - 1) / TY;
  const int nt = A.tiles_x * A.tiles_y;
  *nblk = ((nt + 7) / 8) * 8;
  return A;
}

hipError_t launch_step(const StepLaunch& l, hipStream_t s) {
  if (l.n.total == 0) return hipSuccess;
  return l.bf16 ? mstep_bf(l, nullptr, s) : mstep_f32(l, nullptr, s);
}

hipError_t launch_step_batched(const StepLaunch& proto, const BatchLaunch& b, hipStream_t s) {
  if (b.np == 0 || b.total == 0) return hipSuccess;
  return proto.bf16 ? mstep_bf(proto, &b, s) : mstep_f32(proto, &b, s);
}

const char* step_kernel_name(const StepLaunch& l) {
  return intern_name(std::string("mstep_kernel<") + std::to_string(l.tile) + ", " +
                     (l.bf16 ? "true" : "false") + ", " + std::to_string(l.ncols / 16) + ", " +
                     std::to_string(l.var) + ">");
}

}  // namespace mcmg
