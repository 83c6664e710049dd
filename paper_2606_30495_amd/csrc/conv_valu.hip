// Direct multi-channel 3^D convolutions on the vector ALUs (float32).
//
// One thread computes one output node and a chunk of CT output channels;
// blockIdx.y selects the chunk.  Weights are laid out [tap][cin][cpad] so
// that the CT weights a thread needs for one (tap, cin) pair are contiguous
// and wave-uniform (scalar loads).  Three sampling modes (Sec. 3.2):
//   S1: stride 1, zero padding 1 (lift, projection, setup nets, and solve
//       convolutions on levels without a matrix-core plan);
//   S2: stride 2, pad 1, ceil(n/2) outputs (restriction R, setup f_a);
//   T2: transposed stride-2 (prolongation P), output forced to the fine size:
//       coarse node X feeds fine node 2X + off.
// Epilogues fuse the elementwise work of the V-cycle into the convolution:
//   SET / ADD (e += W * u) / MUL (s (.) (K * t)) / GELU (setup) /
//   RESID (t = r - W * e - a (.) (KA * e), two weight tensors at once).
// The batched form runs the same convolution for several problems (own
// pointers and grids) in one launch.
#include <algorithm>
#include <string>

#include "internal.h"

namespace mcmg {

namespace {

__device__ __forceinline__ float load_as_f32(gptr<const float> p, long long i) { return p[i]; }
__device__ __forceinline__ float load_as_f32(gptr<const double> p, long long i) { return (float)p[i]; }
__device__ __forceinline__ void store_from_f32(gptr<float> p, long long i, float v) { p[i] = v; }
__device__ __forceinline__ void store_from_f32(gptr<double> p, long long i, float v) { p[i] = (double)v; }

__device__ __forceinline__ float gelu_f(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

template <int D, int CT, int MODE, int EPI, typename TIN, typename TOUT>
__device__ __forceinline__ void conv_body(const DArgs& A, const int vblk) {
  const gptr<const TIN> __restrict__ x = to_global<const TIN>(A.x);
  const gptr<const float> __restrict__ w = to_global<const float>(A.w);
  const gptr<const float> __restrict__ w2 = to_global<const float>(A.w2);
  const gptr<TOUT> __restrict__ y = to_global<TOUT>(A.y);
  const gptr<const float> __restrict__ r = to_global<const float>(A.r);
  const gptr<const float> __restrict__ feat = to_global<const float>(A.feat);
  const int cin = A.cin, cout = A.cout, cpad = A.cpad;
  const Dims in = A.in, out = A.out;
  const long long p = (long long)vblk * blockDim.x + threadIdx.x;
  if (p >= out.total) return;
  const int chunk = blockIdx.y;
  int o[3];
  if (out.total < (1LL << 31)) {
    // 32-bit unravel by multiply-high division (no 64-bit divide)
    const uint32_t pp = (uint32_t)p;
    const uint32_t q2 = fdiv(pp, A.fo2);
    const uint32_t q1 = fdiv(q2, A.fo1);
    o[2] = (int)(pp - q2 * (uint32_t)out.n[2]);
    o[1] = (int)(q2 - q1 * (uint32_t)out.n[1]);
    o[0] = (int)q1;
  } else {
    long long q = p;
    o[2] = (int)(q % out.n[2]); q /= out.n[2];
    o[1] = (int)(q % out.n[1]); q /= out.n[1];
    o[0] = (int)q;
  }
  float acc[CT];
  float acc2[CT];
#pragma unroll
  for (int k = 0; k < CT; ++k) { acc[k] = 0.f; acc2[k] = 0.f; }

  constexpr int NT = (D == 2) ? 9 : 27;
  for (int t = 0; t < NT; ++t) {
    int off[3];
    if (D == 2) { off[0] = t / 3 - 1; off[1] = t % 3 - 1; off[2] = 0; }
    else { off[0] = t / 9 - 1; off[1] = (t / 3) % 3 - 1; off[2] = t % 3 - 1; }
    int ii[3];
    bool valid = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= D) { ii[a] = 0; continue; }
      int v;
      if (MODE == CONV_S1) v = o[a] + off[a];
      else if (MODE == CONV_S2) v = 2 * o[a] + off[a];
      else {
        const int tt = o[a] - off[a];
        if (tt & 1) { valid = false; v = 0; }
        else v = tt >> 1;
      }
      if (v < 0 || v >= in.n[a]) valid = false;
      ii[a] = v;
    }
    if (!valid) continue;
    const long long src = (((long long)ii[0] * in.n[1] + ii[1]) * in.n[2] + ii[2]) * cin;
    const gptr<const float> wt = w + (long long)t * cin * cpad + chunk * CT;
    const gptr<const float> wt2 = (EPI == EPI_RESID) ? (w2 + (long long)t * cin * cpad + chunk * CT) : nullptr;
    for (int ci = 0; ci < cin; ++ci) {
      const float xv = load_as_f32(x, src + ci);
#pragma unroll
      for (int k = 0; k < CT; ++k) acc[k] = fmaf(xv, wt[ci * cpad + k], acc[k]);
      if (EPI == EPI_RESID) {
#pragma unroll
        for (int k = 0; k < CT; ++k) acc2[k] = fmaf(xv, wt2[ci * cpad + k], acc2[k]);
      }
    }
  }
  const long long dst = p * cout;
#pragma unroll
  for (int k = 0; k < CT; ++k) {
    const int c = chunk * CT + k;
    if (c >= cout) break;
    float v = acc[k];
    if (EPI == EPI_ADD) v = load_as_f32((gptr<const TOUT>)y, dst + c) + v;
    else if (EPI == EPI_MUL) v = feat[dst + c] * v;
    else if (EPI == EPI_GELU) v = gelu_f(v);
    else if (EPI == EPI_RESID) v = r[dst + c] - v - feat[dst + c] * acc2[k];
    store_from_f32(y, dst + c, v);
  }
}

template <int D, int CT, int MODE, int EPI, typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void conv_direct(DArgs A) {
  conv_body<D, CT, MODE, EPI, TIN, TOUT>(A, blockIdx.x);
}

template <int D, int CT, int MODE, int EPI, typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void conv_direct_batched(const DArgs* __restrict__ tab,
                                                           const int* __restrict__ pre, int np,
                                                           const int* __restrict__ frozen,
    const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const DArgs A = tab[batch_entry(row, np, p)];
  conv_body<D, CT, MODE, EPI, TIN, TOUT>(A, blockIdx.x - pre[p]);
}

// 3D stride-1 2 -> 2 channel convolution (lift and projection) in the
// z-streaming form of the level-1 sweep: a block owns a C3Y x C3X column and a
// chunk of zc planes, keeps three input planes (halo 1 in y and x) in an LDS
// ring and writes one output plane per step, so every input value is read
// once per block instead of once per tap.  Each output sums the same products
// in the same order as conv_body (taps dz-major, then input channel; zero
// outside the grid).
// 9 x 54: 486 outputs in 2 x 256 thread slots, the halo plane 11 x 56 in 3,
// and 54 divides 216, 108 and 54 (a 64-wide tile runs 256 columns for 216).
// The planes per block are chosen at launch (A.zc).
constexpr int C3Y = 9, C3X = 54;
constexpr int C2X = 64;   // 2D tile width

__device__ __forceinline__ int ring3(int pl) { return (pl + 12) % 3; }

bool c22z_ok(const ConvLaunch& a) {
  return a.dim == 3 && a.mode == CONV_S1 && a.epi == EPI_SET && a.cin == 2 && a.cout == 2 &&
         a.cpad == 2;
}

void c22z_tiles(const Dims& out, int zc, int* tx, int* ty, int* tz) {
  *tx = (out.n[2] + C3X - 1) / C3X;
  *ty = (out.n[1] + C3Y - 1) / C3Y;
  *tz = (out.n[0] + zc - 1) / zc;
}

template <typename TIN, typename TOUT>
__device__ __forceinline__ void c22z_body(const DArgs& A, const int vblk) {
  constexpr int EY = C3Y + 2, EX = C3X + 2, NE = EY * EX;
  constexpr int PE = (NE + 255) / 256, NO = C3Y * C3X, PO = (NO + 255) / 256;
  __shared__ float2 se[3 * NE];
  __shared__ float4 sw[27];                 // [tap] (w00, w01, w10, w11)
  const gptr<const TIN> __restrict__ x = to_global<const TIN>(A.x);
  const gptr<TOUT> __restrict__ y = to_global<TOUT>(A.y);
  const gptr<const float> __restrict__ w = to_global<const float>(A.w);
  const int NZ = A.out.n[0], NY = A.out.n[1], NX = A.out.n[2];
  const int zc = A.zc;
  const int tiles_x = (NX + C3X - 1) / C3X, tiles_y = (NY + C3Y - 1) / C3Y;
  const int ntiles = tiles_x * tiles_y * ((NZ + zc - 1) / zc);
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % tiles_x) * C3X, y0 = ((tl / tiles_x) % tiles_y) * C3Y;
  const int zb = (tl / (tiles_x * tiles_y)) * zc;
  const int ze = min(zb + zc, NZ);
  auto inside = [&](int z, int yy, int xx) {
    return xx >= 0 && xx < NX && yy >= 0 && yy < NY && z >= 0 && z < NZ;
  };
  auto gidx = [&](int z, int yy, int xx) { return ((long long)z * NY + yy) * NX + xx; };
  // the 108 weights go to LDS once and are read there with uniform
  // addresses (through the pointer they were vector loads)
  if (threadIdx.x < 27)
    sw[threadIdx.x] = make_float4(w[threadIdx.x * 4 + 0], w[threadIdx.x * 4 + 1],
                                  w[threadIdx.x * 4 + 2], w[threadIdx.x * 4 + 3]);
  // a thread's points are the same in every plane: their in-plane offsets
  // (-1 outside the grid) are computed once, a plane adds a uniform base
  const long long plane = (long long)NY * NX;
  int eoff[PE], ooff[PO];
#pragma unroll
  for (int j = 0; j < PE; ++j) {
    const int i = threadIdx.x + j * 256;
    const int yy = y0 - 1 + i / EX, xx = x0 - 1 + i % EX;
    eoff[j] = (i < NE && inside(0, yy, xx)) ? yy * NX + xx : -1;
  }
#pragma unroll
  for (int j = 0; j < PO; ++j) {
    const int i = threadIdx.x + j * 256;
    const int yy = y0 + i / C3X, xx = x0 + i % C3X;
    ooff[j] = (i < NO && inside(0, yy, xx)) ? yy * NX + xx : -1;
  }
  // input plane k (halo 1), loaded one plane ahead of its store
  float2 v[PE];
  // (unconditional loads from a clamped index, zero selected afterwards, so
  // all of a plane's loads are in flight together)
  auto load_plane = [&](int k) {
    const bool zok = k >= 0 && k < NZ;
    const gptr<const TIN> xk = x + 2 * (zok ? k : 0) * plane;
#pragma unroll
    for (int j = 0; j < PE; ++j) {
      const bool ok = zok && eoff[j] >= 0;
      const unsigned g = ok ? (unsigned)eoff[j] : 0u;
      const float v0 = load_as_f32(xk, 2ll * g), v1 = load_as_f32(xk, 2ll * g + 1);
      v[j] = ok ? make_float2(v0, v1) : make_float2(0.f, 0.f);
    }
  };
  load_plane(zb - 1);
  for (int k = zb - 1; k <= ze; ++k) {
    float2* dst = se + ring3(k) * NE;
#pragma unroll
    for (int j = 0; j < PE; ++j) {
      const int i = threadIdx.x + j * 256;
      if (i < NE) dst[i] = v[j];
    }
    if (k + 1 <= ze) load_plane(k + 1);
    __syncthreads();
    const int z = k - 1;
    if (z >= zb) {
      float a0[PO], a1[PO];
      int eb[PO];
#pragma unroll
      for (int j = 0; j < PO; ++j) {
        const int i = threadIdx.x + j * 256;
        a0[j] = a1[j] = 0.f;
        eb[j] = (i < NO) ? (i / C3X) * EX + (i % C3X) : 0;   // tap (0, 0, 0) of the halo-1 plane
      }
#pragma unroll 1
      for (int dz = 0; dz < 3; ++dz) {
        const float2* P = se + ring3(z - 1 + dz) * NE;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int to = (t / 3) * EX + (t % 3);
          const float4 wt = sw[dz * 9 + t];
#pragma unroll
          for (int j = 0; j < PO; ++j) {
            const float2 e = P[eb[j] + to];
            a0[j] = fmaf(e.x, wt.x, a0[j]);
            a1[j] = fmaf(e.x, wt.y, a1[j]);
            a0[j] = fmaf(e.y, wt.z, a0[j]);
            a1[j] = fmaf(e.y, wt.w, a1[j]);
          }
        }
      }
      const gptr<TOUT> yz = y + 2 * z * plane;
#pragma unroll
      for (int j = 0; j < PO; ++j) {
        if (ooff[j] >= 0) {
          const long long g = (unsigned)ooff[j];
          store_from_f32(yz, 2 * g, a0[j]);
          store_from_f32(yz, 2 * g + 1, a1[j]);
        }
      }
    }
    __syncthreads();
  }
}

template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void c22z_kernel(DArgs A) {
  c22z_body<TIN, TOUT>(A, blockIdx.x);
}

template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void c22z_kernel_batched(const DArgs* __restrict__ tab,
                                                           const int* __restrict__ pre, int np,
                                                           const int* __restrict__ frozen,
                                                           const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const DArgs A = tab[batch_entry(row, np, p)];
  c22z_body<TIN, TOUT>(A, blockIdx.x - pre[p]);
}

// 2D stride-1 2 -> 2 channel convolution (lift and projection): a block
// stages a (C2Y2 + 2) x (C2X + 2) input tile in LDS once and each thread
// writes PO outputs, instead of every output reading its 9 taps through the
// cache.  Each output sums the same products in the same order as conv_body
// (taps row-major, then input channel; zero outside the grid).
constexpr int C2Y2 = 16;

bool c22y_ok(const ConvLaunch& a) {
  return a.dim == 2 && a.mode == CONV_S1 && a.epi == EPI_SET && a.cin == 2 && a.cout == 2 &&
         a.cpad == 2;
}

int c22y_tiles(const Dims& out) {
  return ((out.n[1] + C2X - 1) / C2X) * ((out.n[0] + C2Y2 - 1) / C2Y2);
}

template <typename TIN, typename TOUT>
__device__ __forceinline__ void c22y_body(const DArgs& A, const int vblk) {
  constexpr int EY = C2Y2 + 2, EX = C2X + 2, NE = EY * EX;
  constexpr int PE = (NE + 255) / 256, NO = C2Y2 * C2X, PO = (NO + 255) / 256;
  __shared__ float2 se[NE];
  const gptr<const TIN> __restrict__ x = to_global<const TIN>(A.x);
  const gptr<TOUT> __restrict__ y = to_global<TOUT>(A.y);
  const gptr<const float> __restrict__ w = to_global<const float>(A.w);
  const int NY = A.out.n[0], NX = A.out.n[1];
  const int tiles_x = (NX + C2X - 1) / C2X;
  const int ntiles = tiles_x * ((NY + C2Y2 - 1) / C2Y2);
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % tiles_x) * C2X, y0 = (tl / tiles_x) * C2Y2;
  float2 v[PE];
#pragma unroll
  for (int j = 0; j < PE; ++j) {
    const int i = threadIdx.x + j * 256;
    const int yy = y0 - 1 + i / EX, xx = x0 - 1 + i % EX;
    v[j] = make_float2(0.f, 0.f);
    if (i < NE && yy >= 0 && yy < NY && xx >= 0 && xx < NX) {
      const long long g = (long long)yy * NX + xx;
      v[j] = make_float2(load_as_f32(x, 2 * g), load_as_f32(x, 2 * g + 1));
    }
  }
#pragma unroll
  for (int j = 0; j < PE; ++j) {
    const int i = threadIdx.x + j * 256;
    if (i < NE) se[i] = v[j];
  }
  __syncthreads();
  float a0[PO], a1[PO];
  int eb[PO];
#pragma unroll
  for (int j = 0; j < PO; ++j) {
    const int i = threadIdx.x + j * 256;
    a0[j] = a1[j] = 0.f;
    eb[j] = (i < NO) ? (i / C2X) * EX + (i % C2X) : 0;   // tap (-1, -1) of the halo-1 tile
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int to = (t / 3) * EX + (t % 3);
    const float w00 = w[t * 4 + 0], w01 = w[t * 4 + 1], w10 = w[t * 4 + 2], w11 = w[t * 4 + 3];
#pragma unroll
    for (int j = 0; j < PO; ++j) {
      const float2 e = se[eb[j] + to];
      a0[j] = fmaf(e.x, w00, a0[j]);
      a1[j] = fmaf(e.x, w01, a1[j]);
      a0[j] = fmaf(e.y, w10, a0[j]);
      a1[j] = fmaf(e.y, w11, a1[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < PO; ++j) {
    const int i = threadIdx.x + j * 256;
    const int yy = y0 + i / C2X, xx = x0 + i % C2X;
    if (i < NO && yy < NY && xx < NX) {
      const long long g = (long long)yy * NX + xx;
      store_from_f32(y, 2 * g, a0[j]);
      store_from_f32(y, 2 * g + 1, a1[j]);
    }
  }
}

template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void c22y_kernel(DArgs A) {
  c22y_body<TIN, TOUT>(A, blockIdx.x);
}

template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void c22y_kernel_batched(const DArgs* __restrict__ tab,
                                                           const int* __restrict__ pre, int np,
                                                           const int* __restrict__ frozen,
                                                           const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const DArgs A = tab[batch_entry(row, np, p)];
  c22y_body<TIN, TOUT>(A, blockIdx.x - pre[p]);
}

template <typename TIN, typename TOUT>
hipError_t run_c22y(const ConvLaunch& a, const BatchLaunch* b, hipStream_t s) {
  if (b) {
    hipLaunchKernelGGL((c22y_kernel_batched<TIN, TOUT>), dim3((unsigned)b->total), dim3(256), 0, s,
                       (const DArgs*)b->tab, b->pre, b->np, b->frozen, b->row);
  } else {
    int nblk;
    const DArgs A = conv_args(a, &nblk);
    hipLaunchKernelGGL((c22y_kernel<TIN, TOUT>), dim3((unsigned)nblk), dim3(256), 0, s, A);
  }
  return hipGetLastError();
}

template <typename TIN, typename TOUT>
hipError_t run_c22z(const ConvLaunch& a, const BatchLaunch* b, hipStream_t s) {
  if (b) {
    hipLaunchKernelGGL((c22z_kernel_batched<TIN, TOUT>), dim3((unsigned)b->total), dim3(256), 0, s,
                       (const DArgs*)b->tab, b->pre, b->np, b->frozen, b->row);
  } else {
    int nblk;
    const DArgs A = conv_args(a, &nblk);
    hipLaunchKernelGGL((c22z_kernel<TIN, TOUT>), dim3((unsigned)nblk), dim3(256), 0, s, A);
  }
  return hipGetLastError();
}

template <int D, int CT, int MODE, int EPI, typename TIN, typename TOUT>
hipError_t run(const ConvLaunch& a, const BatchLaunch* b, hipStream_t s) {
  const int nchunk = (a.cout + CT - 1) / CT;
  if (b) {
    hipLaunchKernelGGL((conv_direct_batched<D, CT, MODE, EPI, TIN, TOUT>),
                       dim3((unsigned)b->total, (unsigned)nchunk), dim3(256), 0, s,
                       (const DArgs*)b->tab, b->pre, b->np, b->frozen, b->row);
  } else {
    int nblk;
    const DArgs A = conv_args(a, &nblk);
    hipLaunchKernelGGL((conv_direct<D, CT, MODE, EPI, TIN, TOUT>), dim3((unsigned)nblk, (unsigned)nchunk),
                       dim3(256), 0, s, A);
  }
  return hipGetLastError();
}

template <int D, int CT, int MODE>
hipError_t by_epi(const ConvLaunch& a, const BatchLaunch* b, hipStream_t s) {
  if (a.tin == T_F32 && a.tout == T_F32) {
    switch (a.epi) {
      case EPI_SET: return run<D, CT, MODE, EPI_SET, float, float>(a, b, s);
      case EPI_ADD: return run<D, CT, MODE, EPI_ADD, float, float>(a, b, s);
      case EPI_MUL: return run<D, CT, MODE, EPI_MUL, float, float>(a, b, s);
      case EPI_GELU: return run<D, CT, MODE, EPI_GELU, float, float>(a, b, s);
      case EPI_RESID: return run<D, CT, MODE, EPI_RESID, float, float>(a, b, s);
    }
  }
  if (MODE == CONV_S1 && a.epi == EPI_SET) {
    if (a.tin == T_F64 && a.tout == T_F32) return run<D, CT, MODE, EPI_SET, double, float>(a, b, s);
    if (a.tin == T_F32 && a.tout == T_F64) return run<D, CT, MODE, EPI_SET, float, double>(a, b, s);
  }
  return hipErrorInvalidValue;
}

template <int D, int CT>
hipError_t by_mode(const ConvLaunch& a, const BatchLaunch* b, hipStream_t s) {
  switch (a.mode) {
    case CONV_S1: return by_epi<D, CT, CONV_S1>(a, b, s);
    case CONV_S2: return by_epi<D, CT, CONV_S2>(a, b, s);
    case CONV_T2: return by_epi<D, CT, CONV_T2>(a, b, s);
  }
  return hipErrorInvalidValue;
}

hipError_t dispatch(const ConvLaunch& a, const BatchLaunch* b, hipStream_t s) {
  if (c22y_ok(a)) {
    if (a.tin == T_F64 && a.tout == T_F32) return run_c22y<double, float>(a, b, s);
    if (a.tin == T_F32 && a.tout == T_F32) return run_c22y<float, float>(a, b, s);
    if (a.tin == T_F32 && a.tout == T_F64) return run_c22y<float, double>(a, b, s);
  }
  if (c22z_ok(a)) {
    if (a.tin == T_F64 && a.tout == T_F32) return run_c22z<double, float>(a, b, s);
    if (a.tin == T_F32 && a.tout == T_F32) return run_c22z<float, float>(a, b, s);
    if (a.tin == T_F32 && a.tout == T_F64) return run_c22z<float, double>(a, b, s);
  }
  const int ct = conv_chunk(a.cout);
  if (a.cpad % ct != 0) return hipErrorInvalidValue;
  if (a.dim == 2) return ct == 2 ? by_mode<2, 2>(a, b, s) : by_mode<2, 8>(a, b, s);
  if (a.dim == 3) return ct == 2 ? by_mode<3, 2>(a, b, s) : by_mode<3, 8>(a, b, s);
  return hipErrorInvalidValue;
}

}  // namespace

int conv_chunk(int cout) { return cout <= 2 ? 2 : 8; }

DArgs conv_args(const ConvLaunch& a, int* nblk) {
  DArgs A;
  A.zc = 1;
  A.x = a.x; A.w = a.w; A.w2 = a.w2; A.y = a.y; A.r = a.r; A.feat = a.feat;
  A.cin = a.cin; A.cout = a.cout; A.cpad = a.cpad; A.in = a.in; A.out = a.out;
  A.fo1 = make_fastdiv((uint32_t)a.out.n[1]);
  A.fo2 = make_fastdiv((uint32_t)a.out.n[2]);
  const bool c22_types = (a.tin == T_F64 || a.tin == T_F32) && (a.tout == T_F32 || a.tout == T_F64) &&
                         !(a.tin == T_F64 && a.tout == T_F64);
  if (c22y_ok(a) && c22_types) {
    *nblk = ((c22y_tiles(a.out) + 7) / 8) * 8;
  } else if (c22z_ok(a) && c22_types) {
    // 8-plane chunks: this memory-bound sweep runs faster with more, shorter
    // blocks (2592 at 216^3, about 1.3 rounds of resident blocks) than with
    // chunks sized to one round (1920 blocks: 82 vs 78 us for the lift)
    int tx, ty, tz;
    A.zc = 8;
    c22z_tiles(a.out, A.zc, &tx, &ty, &tz);
    const int nt = tx * ty * tz;
    *nblk = ((nt + 7) / 8) * 8;
  } else {
    *nblk = (int)((a.out.total + 255) / 256);
  }
  return A;
}

hipError_t launch_conv(const ConvLaunch& a, hipStream_t s) {
  if (a.out.total == 0) return hipSuccess;
  return dispatch(a, nullptr, s);
}

hipError_t launch_conv_batched(const ConvLaunch& proto, const BatchLaunch& b, hipStream_t s) {
  if (b.np == 0 || b.total == 0) return hipSuccess;
  return dispatch(proto, &b, s);
}

namespace {
__global__ void zero_f32(float* p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = 0.f;
}
__global__ void zero_f64(double* p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = 0.0;
}
}  // namespace

hipError_t launch_zero_f32(float* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(zero_f32, dim3((unsigned)b), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
hipError_t launch_zero_f64(double* p, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(zero_f64, dim3((unsigned)b), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

const char* conv_kernel_name(const ConvLaunch& a) {
  // the demangled template form profilers print
  static const char* ty_s[3] = {"float", "double", "bf16"};
  const bool c22_types = (a.tin == T_F64 || a.tin == T_F32) && (a.tout == T_F32 || a.tout == T_F64) &&
                         !(a.tin == T_F64 && a.tout == T_F64);
  if (c22y_ok(a) && c22_types)
    return intern_name(std::string("c22y_kernel<") + ty_s[a.tin] + ", " + ty_s[a.tout] + ">");
  if (c22z_ok(a))
    return intern_name(std::string("c22z_kernel<") + ty_s[a.tin] + ", " + ty_s[a.tout] + ">");
  const int ct = conv_chunk(a.cout);
  return intern_name(std::string("conv_direct<") + std::to_string(a.dim) + ", " +
                     std::to_string(ct) + ", " + std::to_string(a.mode) + ", " +
                     std::to_string(a.epi) + ", " + ty_s[a.tin] + ", " + ty_s[a.tout] + ">");
}

void conv_work(const ConvLaunch& a, double* flops, double* bytes) {
  const double T = a.dim == 2 ? 9.0 : 27.0;
  const double pin = (double)a.in.total, pout = (double)a.out.total;
  const double macs = T * a.cin * a.cout * (a.mode == CONV_T2 ? pin : pout);
  *flops = 2.0 * macs * (a.epi == EPI_RESID ? 2.0 : 1.0);
  const double szin = a.tin == T_F64 ? 8.0 : (a.tin == T_BF16 ? 2.0 : 4.0);
  const double szout = a.tout == T_F64 ? 8.0 : (a.tout == T_BF16 ? 2.0 : 4.0);
  double b = pin * a.cin * szin + pout * a.cout * szout;
  if (a.epi == EPI_ADD || a.epi == EPI_MUL) b += pout * a.cout * 4.0;
  if (a.epi == EPI_RESID) b += 2.0 * pout * a.cout * 4.0;
  *bytes = b;
}

}  // namespace mcmg
