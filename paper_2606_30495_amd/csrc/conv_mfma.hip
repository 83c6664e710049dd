// Multi-channel 3^D convolutions of the V-cycle as implicit GEMMs on the
// gfx950 matrix cores (smoother / level-operator convolutions, restriction R
// and prolongation P of Sec. 3.2).
//
// GEMM view: rows = output nodes, columns = output channels, K = (tap,
// input channel).  K is enumerated in "pairs" q = tap * (cinp/KV) + cb, a
// vector of KV consecutive input channels of one tap, so small channel
// counts do not pad K per tap; one MFMA K-step takes 4 pairs (one per group
// of 16 lanes):
//   float32: v_mfma_f32_16x16x4f32     (KV = 1)
//   bf16   : v_mfma_f32_16x16x32_bf16  (KV = 8), float32 accumulation.
// Lane layout of the 16x16 tiles: lane l holds A[row l%16][k-group l/16] and
// B[k-group l/16][col l%16]; the accumulator holds D[4 (l/16) + r][l%16].
//
// Modes (sampling of the A operand):
//   S1: stride 1, zero padding 1 (3^D taps);
//   S2: restriction, coarse node X reads fine nodes 2X + off (3^D taps);
//   T2: prolongation as a depth-to-space convolution on the coarse grid:
//       fine node 2X + a (a in {0,1}^D) only sees coarse nodes X + w,
//       w in {0,1}^D, through tap d = a - 2w + 1 of P; so a 2^D-window
//       convolution producing 2^D * C_fine columns (column = a * C_fine + c)
//       followed by a scatter to the fine grid is exactly the transposed
//       convolution with its output cropped to the fine size.
//
// A workgroup (4 waves) owns 4 output rows (2D) or 2 x 2 rows (3D) of
// 16 * MT nodes and NTW column tiles (blockIdx.y selects the column slice).
// The input tile (with halo) is staged once in LDS (zero outside the grid and
// in padded channels; bf16 with round-to-nearest-even in the bf16 form); the
// weights stream through LDS in chunks of KS K-steps.  Tiles are ordered so
// that each XCD (blockIdx % 8) walks a contiguous band of the grid.
//
// Epilogues (state stays float32): SET y = acc; ADD y += acc; MUL y = feat *
// acc; RESID y = r - acc(W) - feat * acc(KA).
#include <hip/hip_runtime.h>

#include <string>

#include "conv_mfma.h"
#include "internal.h"

namespace mcmg {

// kernels live in the instantiation units conv_mfma_i*.hip
hipError_t mconv_2b_s1(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
hipError_t mconv_2b_st(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
hipError_t mconv_2f_s1(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
hipError_t mconv_2f_st(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
hipError_t mconv_3b_s1(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
hipError_t mconv_3b_st(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
hipError_t mconv_3f_s1(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);
hipError_t mconv_3f_st(const MfmaConv& a, const BatchLaunch* b, hipStream_t s);

namespace {

hipError_t dispatch(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  if (a.rpw == MFMAZ_RPW) return launch_conv_mfmaz(a, b, s);
  const bool st = a.mode != CONV_S1;
  if (a.dim == 2) {
    if (a.bf16) return st ? mconv_2b_st(a, b, s) : mconv_2b_s1(a, b, s);
    return st ? mconv_2f_st(a, b, s) : mconv_2f_s1(a, b, s);
  }
  if (a.dim == 3) {
    if (a.bf16) return st ? mconv_3b_st(a, b, s) : mconv_3b_s1(a, b, s);
    return st ? mconv_3f_st(a, b, s) : mconv_3f_s1(a, b, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

// tile extents (nodes) of a (dim, mt, rpw) tile, as Geo defines them
void mfma_tile(int dim, int mt, int rpw, int* TX, int* TY, int* TZ) {
  *TX = 16 * mt;
  *TY = dim == 2 ? 4 * rpw : (rpw == 1 ? 2 : 4);
  *TZ = dim == 2 ? 1 : 4 * rpw / *TY;
}

bool mfma_tile_ok(int dim, int epi, int mt, int ntw, int rpw) {
  return (epi == EPI_RESID ? 2 : 1) * rpw * mt * ntw <= 16 && rpw <= (dim == 2 ? 2 : 4);
}

// compute units of the current device (for sizing the z-marching forms' chunks)
int device_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}

MArgs mfma_args(const MfmaConv& a, int* nblk) {
  int TX, TY, TZ;
  if (a.rpw == MFMAZ_RPW) {
    // z-marching form: 16 x 8 columns; the z range is cut into as many
    // chunks as keep one wave of resident blocks busy
    MArgs A;
    A.x = a.x; A.wA = a.wA; A.wB = a.wB; A.y = a.y; A.r = a.r; A.feat = a.feat;
    A.cin = a.cin; A.cinp = a.cinp; A.cout = a.cout; A.ncols = a.ncols; A.nsteps = a.nsteps;
    A.npairs = a.npairs; A.in = a.in; A.out = a.out; A.kchunk = a.kchunk;
    A.tiles_x = (a.out.n[2] + 15) / 16;
    A.tiles_y = (a.out.n[1] + 7) / 8;
    const int per_cu = (int)(160 * 1024 / mfmaz_lds_bytes(a.epi));
    const int target = (per_cu > 0 ? per_cu : 1) * device_cus();
    const int txy = A.tiles_x * A.tiles_y;
    const int chunks = target / txy > 1 ? target / txy : 1;
    A.zc = (a.out.n[0] + chunks - 1) / chunks;
    A.tiles_z = (a.out.n[0] + A.zc - 1) / A.zc;
    const int ntiles = A.tiles_x * A.tiles_y * A.tiles_z;
    *nblk = ((ntiles + 7) / 8) * 8;
    return A;
  }
  mfma_tile(a.dim, a.mt, a.rpw, &TX, &TY, &TZ);
  // output tiles are taken over the GEMM row grid: S1 = output grid,
  // S2 = coarse output grid, T2 = coarse (input) grid
  const Dims& rows = (a.mode == CONV_T2) ? a.in : a.out;
  const int RX = (a.dim == 2) ? rows.n[1] : rows.n[2], RY = (a.dim == 2) ? rows.n[0] : rows.n[1];
  const int RZ = (a.dim == 2) ? 1 : rows.n[0];
  MArgs A;
  A.x = a.x; A.wA = a.wA; A.wB = a.wB; A.y = a.y; A.r = a.r; A.feat = a.feat;
  A.cin = a.cin; A.cinp = a.cinp; A.cout = a.cout; A.ncols = a.ncols; A.nsteps = a.nsteps;
  A.npairs = a.npairs; A.in = a.in; A.out = a.out; A.kchunk = a.kchunk; A.zc = 0;
  A.tiles_x = (RX + TX - 1) / TX;
  A.tiles_y = (RY + TY - 1) / TY;
  A.tiles_z = (RZ + TZ - 1) / TZ;
  const int ntiles = A.tiles_x * A.tiles_y * A.tiles_z;
  *nblk = ((ntiles + 7) / 8) * 8;
  return A;
}

hipError_t launch_conv_mfma_batched(const MfmaConv& proto, const BatchLaunch& b, hipStream_t s) {
  if (b.np == 0 || b.total == 0) return hipSuccess;
  return dispatch(proto, &b, s);
}

size_t mfma_lds_bytes(int dim, int bf16, int mode, int mt, int ntw, int rpw, int cin, int cinp, int epi,
                      int kchunk, int nsteps) {
  if (rpw == MFMAZ_RPW) return mfmaz_lds_bytes(epi);
  int TX, TY, TZ;
  mfma_tile(dim, mt, rpw, &TX, &TY, &TZ);
  auto ext = [&](int t) { return mode == CONV_S1 ? t + 2 : (mode == CONV_S2 ? 2 * t + 1 : t + 1); };
  const size_t nodes = (size_t)ext(TX) * ext(TY) * (dim == 2 ? 1 : ext(TZ));
  const int es = bf16 ? 2 : 4, kv = bf16 ? 8 : 1, ks = kchunk;
  const size_t stride = mfma_lds_stride(dim, bf16, cin, cinp);
  const size_t a = ((nodes * stride * es + 15) / 16) * 16 + (stride == 2 && !bf16 ? 16 : 0);
  // 3D float32 reads its B fragments from global memory: no weight chunk
  if (!bf16 && dim == 3) return a;
  const size_t b = (size_t)(epi == EPI_RESID ? 2 : 1) * 4 * ks * ntw * 16 * kv * es;
  return a + (kchunk < nsteps ? 2 : 1) * b;
}

void mfma_pack_dims(int dim, int mode, int cin, int cout, int bf16, int* cinp, int* ncols,
                    int* npairs, int* nsteps) {
  const int KV = bf16 ? 8 : 1;
  const int T = mode == CONV_T2 ? (dim == 2 ? 4 : 8) : (dim == 2 ? 9 : 27);
  *cinp = (cin + KV - 1) / KV * KV;
  if (*cinp % 4) *cinp = (*cinp + 3) / 4 * 4;     // staging works in groups of 4
  const int cols = mode == CONV_T2 ? (1 << dim) * cout : cout;
  *ncols = (cols + 15) / 16 * 16;
  *npairs = T * (*cinp / KV);
  *nsteps = (*npairs + 3) / 4;
}

hipError_t launch_conv_mfma(const MfmaConv& a, hipStream_t s) {
  if (a.out.total == 0 || a.in.total == 0) return hipSuccess;
  return dispatch(a, nullptr, s);
}

const char* mfma_kernel_name(const MfmaConv& a) {
  // the demangled template form profilers print
  if (a.rpw == MFMAZ_RPW) return intern_name(std::string("mconvz_kernel<") + std::to_string(a.epi) + ">");
  return intern_name(std::string("mconv_kernel<") + std::to_string(a.dim) + ", " +
                     (a.bf16 ? "true" : "false") + ", " + std::to_string(a.mode) + ", " +
                     std::to_string(a.epi) + ", " + std::to_string(a.mt) + ", " +
                     std::to_string(a.ntw) + ", " + std::to_string(a.rpw) + ">");
}

}  // namespace mcmg
