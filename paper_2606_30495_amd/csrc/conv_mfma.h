// Implicit-GEMM convolutions on the matrix cores (see conv_mfma.hip).
#pragma once
#include "internal.h"

namespace mcmg {

struct MfmaConv {
  int dim;
  int bf16;              // 1: bf16 operands, 0: float32 operands (float32 accumulate)
  int mode;              // CONV_S1 / CONV_S2 (restriction) / CONV_T2 (prolongation)
  int epi;               // EPI_SET / EPI_ADD / EPI_MUL / EPI_RESID
  int mt, ntw;           // tile: 16*mt output nodes per wave row, ntw column tiles per block
  int rpw;               // node rows per wave (block = 4 * rpw rows along y, z)
  int kchunk;            // K-steps per weight chunk staged in LDS
  const float* x;        // input [in nodes][cin] float32
  const void* wA;        // packed [4*nsteps][ncols][KV] (bf16 or float32)
  const void* wB;        // second packed tensor (EPI_RESID)
  float* y;              // output [out nodes][cout]
  const float* r;        // EPI_RESID
  const float* feat;     // EPI_MUL / EPI_RESID
  int cin, cinp, cout, ncols, nsteps, npairs;
  Dims in, out;
};

// Per-problem kernel arguments (also the element of a batch table).
struct MArgs {
  const float* x;
  const void* wA;
  const void* wB;
  float* y;
  const float* r;
  const float* feat;
  int cin, cinp, cout, ncols, nsteps, npairs;
  Dims in, out;
  int tiles_x, tiles_y, tiles_z, kchunk;
  int zc;                // z-marching form: output planes per block
};

// Arguments and block count of one problem's launch.
MArgs mfma_args(const MfmaConv& a, int* nblk);
// One launch over several problems that share every template parameter
// (dim, precision, mode, epilogue, tile) and channel counts: b.tab holds a
// device array of MArgs, b.pre the block prefix (np + 1 ints).
hipError_t launch_conv_mfma_batched(const MfmaConv& proto, const BatchLaunch& b, hipStream_t s);

// Zero K steps stored after every packed weight tensor: the 3D float32
// kernels load B fragments in groups of four steps, up to 2 NB - 1 groups
// past the last group they multiply (NB <= 8 register sets), without a
// bounds clamp.
constexpr int MFMA_PAD_STEPS = 64;

// 3D float32 weights are packed by groups of four K steps, so that a lane
// reads the B values of a whole group as one 16-byte vector: pair q (K step
// q / 4, lane group q % 4) and column col of the GEMM's B sit at this float
// index (the steps are rounded up to a multiple of 4 before the padding).
inline size_t mfma_bg_index(int q, int col, int ncols) {
  const int s = q / 4, lg = q % 4;
  return (((size_t)(s / 4) * 4 + lg) * ncols + col) * 4 + (s % 4);
}

// Padded sizes of the packed operands (see conv_mfma.hip for the layout).
void mfma_pack_dims(int dim, int mode, int cin, int cout, int bf16, int* cinp, int* ncols,
                    int* npairs, int* nsteps);
// LDS of one block: the staged input tile plus the weight chunk, two chunk
// buffers when the nsteps K-steps take more than one chunk.
// Node stride (elements) of the staged input tile in LDS.  3D float32 at
// C = 2 (the restriction from the finest level) stages only the two real
// channels of a node: the K lanes of the padding channels 2 and 3 then read
// the next node's values, which meet zero weights (the tile carries four
// zero floats after its last node for them).
__host__ __device__ inline int mfma_lds_stride(int dim, int bf16, int cin, int cinp) {
  return (!bf16 && dim == 3 && cin == 2) ? 2 : cinp + (bf16 ? 8 : 1);
}
size_t mfma_lds_bytes(int dim, int bf16, int mode, int mt, int ntw, int rpw, int cin, int cinp, int epi,
                      int kchunk, int nsteps);
// Whether a tile (mt, ntw, rpw) is instantiated for this dim / epilogue.
bool mfma_tile_ok(int dim, int epi, int mt, int ntw, int rpw);
hipError_t launch_conv_mfma(const MfmaConv& a, hipStream_t s);

// z-marching form of the 3D float32 stride-1 convolution with 12 input
// channels (conv_mfmaz.hip), selected as the tile (mt, ntw, rpw) = (1, 1,
// MFMAZ_RPW): whether an operation can take it, its LDS bytes, its launch.
constexpr int MFMAZ_RPW = 8;
bool mfmaz_ok(int dim, int bf16, int mode, int cin, int cout);
size_t mfmaz_lds_bytes(int epi);
hipError_t launch_conv_mfmaz(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
const char* mfma_kernel_name(const MfmaConv& a);

}  // namespace mcmg
