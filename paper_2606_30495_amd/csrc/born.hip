// Discrete Green operator and Born-series updates in FP64 (appendix on the
// Born-series variant; appendix on the discrete Green operator,
// Eq. discrete_symbol; CBS relaxation Eq. cbs_gamma).
//
//   G x = F^{-1}[ F[x] / (sum_a d_a[m_a] - k0^2 - i eps) ],
//   d_a[m] = (4/h^2) sin^2(pi m / n_a)
// is the exact inverse of the periodic five-/seven-point background operator
// -Lap_h - k0^2 - i eps on the extended grid.
//
// FFT: one pass per axis, complex FP64, in place.  A block holds TC whole
// lines of the axis in LDS.  For the fastest axis these are TC consecutive
// lines.  For a strided axis they are the lines through TC consecutive
// fastest-axis positions, read row by row in runs of TC elements.  The block
// transforms them with a mixed-radix decimation-in-time FFT.  The input goes
// into LDS in digit-reversed order, and a stage of radix p joins p
// sub-transforms of length m into one of length m p:
//     out[g + k] = sum_t in[g + (k mod m) + t m] w^{t k},   w = exp(-/+ 2 pi i / (m p)),
// one output per element and thread, computed from LDS into registers and
// written back after a barrier.  Twiddles are read from a per-axis table of
// exp(-2 pi i j / n) built on the host.  Any length up to FFT_MAXL works: a
// radix p costs p complex multiply-adds per element.
//
// Passes (2D: x, y with the symbol, x^-1; 3D: x, y, z with the symbol, y^-1,
// x^-1):
//   FWD  forward transform of the axis;
//   SYM  forward, divide by the Green symbol, inverse (the slowest axis: once
//        its forward transform is done every element holds one complete
//        frequency triple);
//   INV  inverse transform;
//   LAST inverse transform of the fastest axis scaled by 1/N, then either
//        stored (y = G x) or applied as the CBS update u += gamma (.) y with
//        gamma = 1 + i V / eps, V = k^2 (1 + i gamma_s) - k0^2.
// Per pass each element is read once and written once (32 B per node).
#include "internal.h"

namespace mcmg {

namespace {

constexpr int FT = 256;              // threads per block
constexpr int FR = FFT_MAXL / FT;    // elements per thread at most

__device__ __forceinline__ double2 cmad(double2 acc, double2 a, double2 w) {
  acc.x = fma(a.x, w.x, fma(-a.y, w.y, acc.x));
  acc.y = fma(a.x, w.y, fma(a.y, w.x, acc.y));
  return acc;
}

// Transform the block's lines held in LDS (digit-reversed order).  reg[r]
// receives the natural-order result for element r of the thread; LDS holds
// it too unless the caller only needs the registers (last stage skipped).
__device__ __forceinline__ void fft_stages(const FftArgs& A, double2* lds, int Lp, const int* cc,
                                           const int* kk, int nr, bool inverse, double2* reg) {
  const int L = A.L;
  for (int s = 0; s < A.nst; ++s) {
    const int p = A.rad[s], m = A.mlen[s], mp = m * p, tstep = L / mp;
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      if (r >= nr || cc[r] < 0) continue;
      const int k = kk[r];
      const int q = k % mp;
      const double2* src = lds + cc[r] * Lp + (k - q) + (q % m);
      double2 acc = make_double2(0.0, 0.0);
      int ti = 0;
      for (int t = 0; t < p; ++t) {
        double2 w = A.tw[ti * tstep];
        if (inverse) w.y = -w.y;
        acc = cmad(acc, src[t * m], w);
        ti += q;
        if (ti >= mp) ti -= mp;
      }
      reg[r] = acc;
    }
    __syncthreads();
    if (s + 1 < A.nst) {
#pragma unroll
      for (int r = 0; r < FR; ++r)
        if (r < nr && cc[r] >= 0) lds[cc[r] * Lp + kk[r]] = reg[r];
      __syncthreads();
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(FT) void fft_kernel(FftArgs A) {
  extern __shared__ __align__(16) double2 lds[];
  const int L = A.L, TC = A.TC, Lp = L + 1;
  const long long S = A.S;
  // this block's lines: contiguous axis -> lines l0 .. l0+TC-1 (each L long);
  // strided axis -> outer o, fastest positions i0 .. i0+TC-1
  long long l0 = 0, o = 0, i0 = 0;
  int ncol;
  if (A.contiguous) {
    l0 = (long long)blockIdx.x * TC;
    const long long nl = A.outer;
    ncol = (int)((nl - l0) < TC ? (nl - l0) : TC);
  } else {
    const long long ntile = (S + TC - 1) / TC;
    o = blockIdx.x / ntile;
    i0 = (blockIdx.x % ntile) * TC;
    ncol = (int)((S - i0) < TC ? (S - i0) : TC);
  }
  const int ne = L * TC;
  const int nr = (ne + FT - 1) / FT;
  int cc[FR], kk[FR];
  long long gi[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int e = threadIdx.x + r * FT;
    int c = -1, k = 0;
    if (r < nr && e < ne) {
      if (A.contiguous) { c = e / L; k = e - c * L; }
      else { k = e / TC; c = e - k * TC; }
      if (c >= ncol) c = -1;
    }
    cc[r] = c;
    kk[r] = k;
    gi[r] = c < 0 ? 0
                  : (A.contiguous ? (l0 + c) * L + k : (o * L + k) * S + i0 + c);
  }
  const double2* __restrict__ src = reinterpret_cast<const double2*>(A.src);
  double2* __restrict__ dst = reinterpret_cast<double2*>(A.dst);
  const bool inv0 = (MODE == FFT_INV || MODE == FFT_LAST);
#pragma unroll
  for (int r = 0; r < FR; ++r)
    if (r < nr && cc[r] >= 0) lds[cc[r] * Lp + A.rev[kk[r]]] = src[gi[r]];
  __syncthreads();
  double2 reg[FR];
  fft_stages(A, lds, Lp, cc, kk, nr, inv0, reg);

  if (MODE == FFT_SYM) {
    // divide by sum_a d_a[m_a] - k0^2 - i eps; the axis is 0, the other
    // frequency indices come from the fastest-axis position i0 + c
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      if (r >= nr || cc[r] < 0) continue;
      const long long i = i0 + cc[r];
      double sr = A.d[0][kk[r]] - A.k0sq;
      if (A.dim == 2) {
        sr += A.d[1][i];
      } else {
        sr += A.d[1][i / A.n[2]] + A.d[2][i % A.n[2]];
      }
      const double si = -A.eps;
      const double den = 1.0 / (sr * sr + si * si);
      const double2 v = reg[r];
      // v / (sr + i si) = v (sr - i si) / |.|^2
      reg[r] = make_double2((v.x * sr + v.y * si) * den, (v.y * sr - v.x * si) * den);
    }
#pragma unroll
    for (int r = 0; r < FR; ++r)
      if (r < nr && cc[r] >= 0) lds[cc[r] * Lp + A.rev[kk[r]]] = reg[r];
    __syncthreads();
    fft_stages(A, lds, Lp, cc, kk, nr, true, reg);
  }

  if (MODE == FFT_LAST) {
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      if (r >= nr || cc[r] < 0) continue;
      const double2 v = make_double2(reg[r].x * A.scale, reg[r].y * A.scale);
      const long long pidx = gi[r];
      if (A.u) {
        // CBS: u += gamma (.) v, gamma = (1 - Im V / eps) + i Re V / eps
        const double kk2 = A.k2[pidx];
        double gs = 0.0;
        if (A.gmax != 0.0) {
          long long t = pidx;
          const int x2 = (int)(t % A.n[2]); t /= A.n[2];
          const int x1 = (int)(t % A.n[1]); t /= A.n[1];
          const int x0 = (int)t;
          double sg = A.g[0][x0] + A.g[1][x1];
          if (A.dim == 3) sg += A.g[2][x2];
          gs = A.gmax * (sg < 1.0 ? sg : 1.0);
        }
        const double vr = kk2 - A.k0sq, vi = kk2 * gs;
        const double gr = 1.0 - vi / A.eps, gim = vr / A.eps;
        double2* u = reinterpret_cast<double2*>(A.u);
        double2 uv = u[pidx];
        uv.x += gr * v.x - gim * v.y;
        uv.y += gr * v.y + gim * v.x;
        u[pidx] = uv;
      } else {
        dst[pidx] = v;
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < FR; ++r)
      if (r < nr && cc[r] >= 0) dst[gi[r]] = reg[r];
  }
}

// Background statistics for the default k0^2 and eps: per-block min/max of
// k^2 (pass 0) and max |k^2 (1 + i gamma_s) - k0^2| (pass 1).
constexpr int SB = 256;

__global__ __launch_bounds__(SB) void born_stats_kernel(BornStatsArgs A, int pass) {
  __shared__ double s0[SB], s1[SB];
  double lo = 1e300, hi = -1e300;
  const long long N = A.N;
  for (long long p = (long long)blockIdx.x * SB + threadIdx.x; p < N;
       p += (long long)gridDim.x * SB) {
    const double kk = A.k2[p];
    if (pass == 0) {
      lo = kk < lo ? kk : lo;
      hi = kk > hi ? kk : hi;
    } else {
      double gs = 0.0;
      if (A.gmax != 0.0) {
        long long t = p;
        const int x2 = (int)(t % A.n[2]); t /= A.n[2];
        const int x1 = (int)(t % A.n[1]); t /= A.n[1];
        const int x0 = (int)t;
        double sg = A.g[0][x0] + A.g[1][x1];
        if (A.dim == 3) sg += A.g[2][x2];
        gs = A.gmax * (sg < 1.0 ? sg : 1.0);
      }
      const double vr = kk - A.k0sq, vi = kk * gs;
      const double m = sqrt(vr * vr + vi * vi);
      hi = m > hi ? m : hi;
    }
  }
  s0[threadIdx.x] = lo;
  s1[threadIdx.x] = hi;
  __syncthreads();
  for (int w = SB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s0[threadIdx.x] = s0[threadIdx.x] < s0[threadIdx.x + w] ? s0[threadIdx.x] : s0[threadIdx.x + w];
      s1[threadIdx.x] = s1[threadIdx.x] > s1[threadIdx.x + w] ? s1[threadIdx.x] : s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    A.out[2 * blockIdx.x] = s0[0];
    A.out[2 * blockIdx.x + 1] = s1[0];
  }
}

}  // namespace

size_t fft_lds_bytes(const FftArgs& a) { return (size_t)a.TC * (a.L + 1) * 16; }

long long fft_blocks(const FftArgs& a) {
  if (a.contiguous) return (a.outer + a.TC - 1) / a.TC;
  return a.outer * ((a.S + a.TC - 1) / a.TC);
}

hipError_t launch_fft(int mode, const FftArgs& a, hipStream_t s) {
  if (a.L < 1 || a.L > FFT_MAXL || a.TC < 1 || (long long)a.L * a.TC > FFT_MAXL || a.nst < 0 ||
      a.nst > FFT_MAXST)
    return hipErrorInvalidValue;
  const long long nb = fft_blocks(a);
  if (nb < 1 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
  const size_t lds = fft_lds_bytes(a);
  switch (mode) {
    case FFT_FWD: hipLaunchKernelGGL((fft_kernel<FFT_FWD>), dim3((unsigned)nb), dim3(FT), lds, s, a); break;
    case FFT_SYM: hipLaunchKernelGGL((fft_kernel<FFT_SYM>), dim3((unsigned)nb), dim3(FT), lds, s, a); break;
    case FFT_INV: hipLaunchKernelGGL((fft_kernel<FFT_INV>), dim3((unsigned)nb), dim3(FT), lds, s, a); break;
    case FFT_LAST: hipLaunchKernelGGL((fft_kernel<FFT_LAST>), dim3((unsigned)nb), dim3(FT), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int born_stats_blocks(long long n) {
  long long b = (n + SB - 1) / SB;
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

hipError_t launch_born_stats(const BornStatsArgs& a, int pass, hipStream_t s) {
  hipLaunchKernelGGL(born_stats_kernel, dim3(born_stats_blocks(a.N)), dim3(SB), 0, s, a, pass);
  return hipGetLastError();
}

}  // namespace mcmg
