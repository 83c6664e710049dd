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
#include <string>
#include <type_traits>

#include "conv_mfma.h"
#include "internal.h"

namespace mcmg {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

__device__ __forceinline__ u16 f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (u16)(u >> 16);
}

// Output tile and staged input tile geometry per (D, MODE, MT).
template <int D, int MODE, int MT>
struct Geo {
  static constexpr int TX = 16 * MT;
  static constexpr int TY = (D == 2) ? 4 : 2;
  static constexpr int TZ = (D == 2) ? 1 : 2;
  // staged tile extent per axis
  static constexpr int ext(int t) { return MODE == CONV_S1 ? t + 2 : (MODE == CONV_S2 ? 2 * t + 1 : t + 1); }
  static constexpr int HX = ext(TX), HY = ext(TY), HZ = (D == 2) ? 1 : ext(TZ);
  static constexpr int NODES = HX * HY * HZ;
  static constexpr int TAPS = (MODE == CONV_T2) ? ((D == 2) ? 4 : 8) : ((D == 2) ? 9 : 27);
  static constexpr int W = (MODE == CONV_T2) ? 2 : 3;   // window per axis
};

template <bool BF> constexpr int KVOF() { return BF ? 8 : 1; }

// One block of the convolution: `vblk` is the block index inside this
// problem's grid (the batched wrapper maps the launch's blocks onto problems).
template <int D, bool BF, int MODE, int EPI, int MT, int NTW>
__device__ __forceinline__ void mconv_body(const MArgs& A, const int vblk) {
  const float* __restrict__ x = A.x;
  const void* __restrict__ wA = A.wA;
  const void* __restrict__ wB = A.wB;
  float* __restrict__ y = A.y;
  const float* __restrict__ r = A.r;
  const float* __restrict__ feat = A.feat;
  const int cin = A.cin, cinp = A.cinp, cout = A.cout, ncols = A.ncols, nsteps = A.nsteps;
  const int npairs = A.npairs, tiles_x = A.tiles_x, tiles_y = A.tiles_y, tiles_z = A.tiles_z;
  const int kchunk = A.kchunk;
  const Dims in = A.in, out = A.out;
  using G = Geo<D, MODE, MT>;
  constexpr int KV = KVOF<BF>();
  constexpr int NACC = (EPI == EPI_RESID) ? 2 : 1;
  constexpr int ES = BF ? 2 : 4;
  extern __shared__ __align__(16) unsigned char smem[];
  const int stride = cinp + (BF ? 8 : 1);  // LDS node stride (elements)
  unsigned char* bsm = smem + (((size_t)G::NODES * stride * ES + 15) / 16) * 16;
  constexpr int BROW = NTW * 16 * KV;      // elements of one pair row in the chunk

  const int ntiles = tiles_x * tiles_y * tiles_z;
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;
  if (tl >= ntiles) return;
  const int tx = tl % tiles_x, ty = (tl / tiles_x) % tiles_y, tz = tl / (tiles_x * tiles_y);
  const int x0 = tx * G::TX, y0 = ty * G::TY, z0 = tz * G::TZ;
  const int col0 = blockIdx.y * NTW * 16;
  // grids: 2D (n[0] rows, n[1] x), 3D (n[0] z, n[1] y, n[2] x)
  const int IX = (D == 2) ? in.n[1] : in.n[2], IY = (D == 2) ? in.n[0] : in.n[1];
  const int IZ = (D == 2) ? 1 : in.n[0];
  const int OX = (D == 2) ? out.n[1] : out.n[2], OY = (D == 2) ? out.n[0] : out.n[1];
  const int OZ = (D == 2) ? 1 : out.n[0];
  // origin of the staged tile in input coordinates
  int sx, sy, sz;
  if (MODE == CONV_S1) { sx = x0 - 1; sy = y0 - 1; sz = z0 - 1; }
  else if (MODE == CONV_S2) { sx = 2 * x0 - 1; sy = 2 * y0 - 1; sz = 2 * z0 - 1; }
  else { sx = x0; sy = y0; sz = z0; }
  if (D == 2) sz = 0;

  // ---- stage the input tile: loads are issued in batches of SB per thread
  // before any LDS store, so a block waits for one memory latency per batch
  {
    constexpr int SB = 8;
    const bool vec4 = (cin % 4) == 0;
    const int ng = cinp / 4;
    const int total = G::NODES * ng;
    for (int base = threadIdx.x; base < total; base += 256 * SB) {
      float4 v[SB];
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int idx = base + k * 256;
        if (idx >= total) continue;
        const int node = idx / ng, c = (idx % ng) * 4;
        const int hx = node % G::HX, hy = (node / G::HX) % G::HY, hz = node / (G::HX * G::HY);
        const int gx = sx + hx, gy = sy + hy, gz = sz + hz;
        if (gx >= 0 && gx < IX && gy >= 0 && gy < IY && gz >= 0 && gz < IZ && c < cin) {
          const long long g = (((long long)gz * IY + gy) * IX + gx) * cin;
          if (vec4) {
            v[k] = *reinterpret_cast<const float4*>(x + g + c);
          } else {
            v[k].x = x[g + c];
            if (c + 1 < cin) v[k].y = x[g + c + 1];
            if (c + 2 < cin) v[k].z = x[g + c + 2];
            if (c + 3 < cin) v[k].w = x[g + c + 3];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        const int idx = base + k * 256;
        if (idx >= total) continue;
        const int node = idx / ng, c = (idx % ng) * 4;
        if constexpr (BF) {
          u16* s = reinterpret_cast<u16*>(smem) + (size_t)node * stride + c;
          s[0] = f2bf(v[k].x); s[1] = f2bf(v[k].y); s[2] = f2bf(v[k].z); s[3] = f2bf(v[k].w);
        } else {
          float* s = reinterpret_cast<float*>(smem) + (size_t)node * stride + c;
          s[0] = v[k].x; s[1] = v[k].y; s[2] = v[k].z; s[3] = v[k].w;
        }
      }
    }
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int wy = (D == 2) ? wave : (wave & 1);
  const int wz = (D == 2) ? 0 : (wave >> 1);

  floatx4 acc[NACC][MT][NTW];
#pragma unroll
  for (int a = 0; a < NACC; ++a)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int t = 0; t < NTW; ++t) acc[a][m][t] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int cpv = cinp / KV;
  const int KS = kchunk;
  for (int s0 = 0; s0 < nsteps; s0 += KS) {
    const int ks = (nsteps - s0) < KS ? (nsteps - s0) : KS;
    __syncthreads();   // previous chunk consumed (and input tile staged)
    {
      // weight chunk rows q in [4 s0, 4 (s0 + ks)), columns [col0, col0 + 16 NTW)
      constexpr int SB = 8;
      const int nrow = 4 * ks;
      constexpr int V16 = BROW * ES / 16;    // 16-byte vectors per row
      const int total = NACC * nrow * V16;
      for (int base = threadIdx.x; base < total; base += 256 * SB) {
        uint4 v[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
          const int idx = base + k * 256;
          if (idx >= total) continue;
          const int a = idx / (nrow * V16), rem = idx % (nrow * V16);
          const int row = rem / V16, vv = rem % V16;
          v[k] = *reinterpret_cast<const uint4*>(reinterpret_cast<const unsigned char*>(a ? wB : wA) +
                                                 (((size_t)(4 * s0 + row) * ncols + col0) * KV) * ES +
                                                 (size_t)vv * 16);
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) {
          const int idx = base + k * 256;
          if (idx >= total) continue;
          const int a = idx / (nrow * V16), rem = idx % (nrow * V16);
          const int row = rem / V16, vv = rem % V16;
          *reinterpret_cast<uint4*>(bsm + (((size_t)a * 4 * KS + row) * BROW) * ES + (size_t)vv * 16) = v[k];
        }
      }
    }
    __syncthreads();
#pragma unroll 2
    for (int ss = 0; ss < ks; ++ss) {
      const int s = s0 + ss;
      int q = 4 * s + lg;
      if (q >= npairs) q = npairs - 1;   // weight rows are zero there
      const int tap = q / cpv, cb = q - tap * cpv;
      int dz = 0, dy, dx;
      if (D == 2) { dy = tap / G::W; dx = tap % G::W; }
      else { dz = tap / (G::W * G::W); dy = (tap / G::W) % G::W; dx = tap % G::W; }
      typename std::conditional<BF, bf16x8, float>::type bf[NACC][NTW];
#pragma unroll
      for (int a = 0; a < NACC; ++a)
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
          const size_t o = ((size_t)a * 4 * KS + 4 * ss + lg) * BROW + (t * 16 + li) * KV;
          if constexpr (BF) bf[a][t] = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const u16*>(bsm) + o);
          else bf[a][t] = reinterpret_cast<const float*>(bsm)[o];
        }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int ox = m * 16 + li;   // output x inside the tile
        int hx, hy, hz;
        if (MODE == CONV_S2) { hx = 2 * ox + dx; hy = 2 * wy + dy; hz = 2 * wz + dz; }
        else { hx = ox + dx; hy = wy + dy; hz = wz + dz; }
        const size_t node = ((size_t)hz * G::HY + hy) * G::HX + hx;
        if constexpr (BF) {
          const bf16x8 af = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const u16*>(smem) +
                                                             node * stride + cb * KV);
#pragma unroll
          for (int t = 0; t < NTW; ++t)
#pragma unroll
            for (int a = 0; a < NACC; ++a)
              acc[a][m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[a][t], acc[a][m][t], 0, 0, 0);
        } else {
          const float af = reinterpret_cast<const float*>(smem)[node * stride + cb];
#pragma unroll
          for (int t = 0; t < NTW; ++t)
#pragma unroll
            for (int a = 0; a < NACC; ++a)
              acc[a][m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf[a][t], acc[a][m][t], 0, 0, 0);
        }
      }
    }
  }

  // ---- epilogue
  const int gy = y0 + wy, gz = z0 + wz;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int col = col0 + t * 16 + li;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int gx = x0 + m * 16 + 4 * lg + rr;
        long long o;
        if (MODE == CONV_T2) {
          // column = class * cout + c; class bits: x fastest
          const int cls = col / cout, c = col - cls * cout;
          if (cls >= (1 << D)) continue;
          const int ax = cls & 1, ay = (cls >> 1) & 1, az = (D == 3) ? ((cls >> 2) & 1) : 0;
          const int fx = 2 * gx + ax, fy = 2 * gy + ay, fz = (D == 3) ? 2 * gz + az : 0;
          if (fx >= OX || fy >= OY || fz >= OZ) continue;
          o = (((long long)fz * OY + fy) * OX + fx) * cout + c;
        } else {
          if (col >= cout || gx >= OX || gy >= OY || gz >= OZ) continue;
          o = (((long long)gz * OY + gy) * OX + gx) * cout + col;
        }
        float v = acc[0][m][t][rr];
        if (EPI == EPI_ADD) v = y[o] + v;
        else if (EPI == EPI_MUL) v = feat[o] * v;
        else if (EPI == EPI_RESID) v = r[o] - v - feat[o] * acc[NACC - 1][m][t][rr];
        y[o] = v;
      }
    }
}

template <int D, bool BF, int MODE, int EPI, int MT, int NTW>
__global__ __launch_bounds__(256) void mconv_kernel(MArgs A) {
  mconv_body<D, BF, MODE, EPI, MT, NTW>(A, blockIdx.x);
}

// Batched form: one launch for several problems; pre[p] is the first block of
// problem p (pre[np] = total blocks), tab[p] its arguments.
template <int D, bool BF, int MODE, int EPI, int MT, int NTW>
__global__ __launch_bounds__(256) void mconv_kernel_batched(const MArgs* __restrict__ tab,
                                                            const int* __restrict__ pre, int np,
                                                            const int* __restrict__ frozen,
    const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const MArgs A = tab[batch_entry(row, np, p)];
  mconv_body<D, BF, MODE, EPI, MT, NTW>(A, blockIdx.x - pre[p]);
}

template <int D, bool BF, int MODE, int EPI, int MT, int NTW>
hipError_t run(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  const int nslices = a.ncols / (16 * NTW);
  const size_t lds = mfma_lds_bytes(a.dim, a.bf16, a.mode, a.mt, a.ntw, a.cinp, a.epi, a.kchunk);
  if (b) {
    hipLaunchKernelGGL((mconv_kernel_batched<D, BF, MODE, EPI, MT, NTW>), dim3(b->total, nslices),
                       dim3(256), lds, s, (const MArgs*)b->tab, b->pre, b->np, b->frozen, b->row);
  } else {
    int nblk;
    const MArgs A = mfma_args(a, &nblk);
    hipLaunchKernelGGL((mconv_kernel<D, BF, MODE, EPI, MT, NTW>), dim3(nblk, nslices), dim3(256),
                       lds, s, A);
  }
  return hipGetLastError();
}

template <int D, bool BF, int MODE, int EPI, int MT>
hipError_t by_ntw(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  switch (a.ntw) {
    case 1: return run<D, BF, MODE, EPI, MT, 1>(a, b, s);
    case 2: return run<D, BF, MODE, EPI, MT, 2>(a, b, s);
    case 4: return run<D, BF, MODE, EPI, MT, 4>(a, b, s);
  }
  return hipErrorInvalidValue;
}

template <int D, bool BF, int MODE, int EPI>
hipError_t by_mt(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  switch (a.mt) {
    case 1: return by_ntw<D, BF, MODE, EPI, 1>(a, b, s);
    case 2: return by_ntw<D, BF, MODE, EPI, 2>(a, b, s);
    case 4: return by_ntw<D, BF, MODE, EPI, 4>(a, b, s);
  }
  return hipErrorInvalidValue;
}

template <int D, bool BF>
hipError_t by_mode(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  if (a.mode == CONV_S1) {
    switch (a.epi) {
      case EPI_SET: return by_mt<D, BF, CONV_S1, EPI_SET>(a, b, s);
      case EPI_ADD: return by_mt<D, BF, CONV_S1, EPI_ADD>(a, b, s);
      case EPI_MUL: return by_mt<D, BF, CONV_S1, EPI_MUL>(a, b, s);
      case EPI_RESID: return by_mt<D, BF, CONV_S1, EPI_RESID>(a, b, s);
    }
  } else if (a.mode == CONV_S2 && a.epi == EPI_SET) {
    return by_mt<D, BF, CONV_S2, EPI_SET>(a, b, s);
  } else if (a.mode == CONV_T2 && a.epi == EPI_ADD) {
    return by_mt<D, BF, CONV_T2, EPI_ADD>(a, b, s);
  }
  return hipErrorInvalidValue;
}

hipError_t dispatch(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  if (a.dim == 2) return a.bf16 ? by_mode<2, true>(a, b, s) : by_mode<2, false>(a, b, s);
  if (a.dim == 3) return a.bf16 ? by_mode<3, true>(a, b, s) : by_mode<3, false>(a, b, s);
  return hipErrorInvalidValue;
}

}  // namespace

MArgs mfma_args(const MfmaConv& a, int* nblk) {
  const int TX = 16 * a.mt, TY = a.dim == 2 ? 4 : 2, TZ = a.dim == 2 ? 1 : 2;
  // output tiles are taken over the GEMM row grid: S1 = output grid,
  // S2 = coarse output grid, T2 = coarse (input) grid
  const Dims& rows = (a.mode == CONV_T2) ? a.in : a.out;
  const int RX = (a.dim == 2) ? rows.n[1] : rows.n[2], RY = (a.dim == 2) ? rows.n[0] : rows.n[1];
  const int RZ = (a.dim == 2) ? 1 : rows.n[0];
  MArgs A;
  A.x = a.x; A.wA = a.wA; A.wB = a.wB; A.y = a.y; A.r = a.r; A.feat = a.feat;
  A.cin = a.cin; A.cinp = a.cinp; A.cout = a.cout; A.ncols = a.ncols; A.nsteps = a.nsteps;
  A.npairs = a.npairs; A.in = a.in; A.out = a.out; A.kchunk = a.kchunk;
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

size_t mfma_lds_bytes(int dim, int bf16, int mode, int mt, int ntw, int cinp, int epi, int kchunk) {
  const int TX = 16 * mt, TY = dim == 2 ? 4 : 2, TZ = dim == 2 ? 1 : 2;
  auto ext = [&](int t) { return mode == CONV_S1 ? t + 2 : (mode == CONV_S2 ? 2 * t + 1 : t + 1); };
  const size_t nodes = (size_t)ext(TX) * ext(TY) * (dim == 2 ? 1 : ext(TZ));
  const int es = bf16 ? 2 : 4, kv = bf16 ? 8 : 1, ks = kchunk;
  const size_t stride = cinp + (bf16 ? 8 : 1);
  const size_t a = ((nodes * stride * es + 15) / 16) * 16;
  const size_t b = (size_t)(epi == EPI_RESID ? 2 : 1) * 4 * ks * ntw * 16 * kv * es;
  return a + b;
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
  return intern_name(std::string("mconv_kernel<") + std::to_string(a.dim) + ", " +
                     (a.bf16 ? "true" : "false") + ", " + std::to_string(a.mode) + ", " +
                     std::to_string(a.epi) + ", " + std::to_string(a.mt) + ", " +
                     std::to_string(a.ntw) + ">");
}

}  // namespace mcmg
