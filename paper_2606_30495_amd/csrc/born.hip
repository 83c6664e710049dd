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
//     out[g + q + j m] = sum_t (in[g + q + t m] w_{mp}^{t q}) w_p^{t j},
//     q < m, w_N = exp(-/+ 2 pi i / N).
// For p in {2, 3, 4, 5, 7, 11} a thread takes whole butterflies: it reads
// the p inputs, applies the p - 1 twiddles and the p-point DFT, and writes
// the outputs back to the same slots, so a stage needs one barrier.  Any
// other radix uses a stage with one output per element and thread.  Twiddles
// come from a per-axis table of exp(-2 pi i j / n) built on the host, which
// is staged in LDS when it fits beside the lines.  Any length up to FFT_MAXL
// works.
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

constexpr int FT = 512;              // threads per block
constexpr int FR = FFT_MAXL / FT;    // elements per thread at most

__device__ __forceinline__ double2 cmul(double2 a, double2 w) {
  return make_double2(fma(a.x, w.x, -a.y * w.y), fma(a.x, w.y, a.y * w.x));
}
__device__ __forceinline__ double2 cmad(double2 acc, double2 a, double2 w) {
  acc.x = fma(a.x, w.x, fma(-a.y, w.y, acc.x));
  acc.y = fma(a.x, w.y, fma(a.y, w.x, acc.y));
  return acc;
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conj_if(double2 w, bool c) { return make_double2(w.x, c ? -w.y : w.y); }

// Where this block's lines live: contiguous axis -> lines l0 .. l0+ncol-1;
// strided axis -> outer index o, fastest-axis positions i0 .. i0+ncol-1.
struct Lines {
  long long l0, o, i0;
  int ncol;
};

__device__ __forceinline__ Lines block_lines(const FftArgs& A) {
  Lines b{0, 0, 0, 0};
  if (A.contiguous) {
    b.l0 = (long long)blockIdx.x * A.TC;
    const long long left = A.outer - b.l0;
    b.ncol = (int)(left < A.TC ? left : A.TC);
  } else {
    const long long ntile = (A.S + A.TC - 1) / A.TC;
    b.o = blockIdx.x / ntile;
    b.i0 = (blockIdx.x % ntile) * A.TC;
    const long long left = A.S - b.i0;
    b.ncol = (int)(left < A.TC ? left : A.TC);
  }
  return b;
}

// Element e of the block -> (column c, index j along the axis).  Contiguous
// axis: consecutive threads walk along a line; strided axis: consecutive
// threads walk across the TC columns of one row (TC-element global runs).
struct CJ {
  int c, j;
};
__device__ __forceinline__ CJ elem(const FftArgs& A, int e) {
  const int d = A.contiguous ? A.L : A.TC;
  const int q = e / d, r = e - q * d;
  return A.contiguous ? CJ{q, r} : CJ{r, q};
}

__device__ __forceinline__ long long gaddr(const FftArgs& A, const Lines& b, int c, int j) {
  return A.contiguous ? (b.l0 + c) * A.L + j : (b.o * A.L + j) * A.S + b.i0 + c;
}

// One radix-P stage in place: each butterfly reads its P inputs (stride m),
// applies the twiddles w_{mP}^{t q}, takes the P-point DFT and writes the P
// outputs back to the same slots.  Odd P pairs the inputs, a_t = x_t +
// x_{P-t} and b_t = x_t - x_{P-t}, so that outputs j and P - j share
//     U = x_0 + sum_t a_t cos(2 pi t j / P),  W = sum_t b_t sin(2 pi t j / P),
//     y_j = U -/+ i W,  y_{P-j} = U +/- i W   (forward / inverse).
// The roots are read with block-uniform indices from the global table.
template <int P, class TW>
__device__ __forceinline__ void stage_bfly(const FftArgs& A, double2* lds, int Lp, TW twp, int m,
                                           int ncol, bool inv) {
  const int L = A.L, TC = A.TC, mp = m * P, nbf = L / P, tstep = L / mp;
  // odd P: the (P - 1) / 2 distinct roots (cos, -sin)(2 pi k / P), k <= (P - 1) / 2;
  // cos(2 pi (P - k) / P) = cos(2 pi k / P), sin(2 pi (P - k) / P) = -sin(2 pi k / P)
  constexpr int HR = (P % 2 == 1) ? (P - 1) / 2 : 1;
  double2 rt[HR];
  if constexpr (P % 2 == 1) {
#pragma unroll
    for (int k = 1; k <= HR; ++k) rt[k - 1] = A.tw[k * (L / P)];
  }
  for (int b = threadIdx.x; b < TC * nbf; b += FT) {
    int c, bi;
    if (A.contiguous) { c = b / nbf; bi = b - c * nbf; }
    else { bi = b / TC; c = b - bi * TC; }
    if (c >= ncol) continue;
    const int g = bi / m, q = bi - g * m;
    double2* base = lds + c * Lp + g * mp + q;
    if constexpr (P == 2) {
      const double2 x0 = base[0];
      const double2 x1 = cmul(base[m], conj_if(twp[q * tstep], inv));
      base[0] = cadd(x0, x1);
      base[m] = csub(x0, x1);
    } else if constexpr (P == 4) {
      const double2 x0 = base[0];
      const double2 x1 = cmul(base[m], conj_if(twp[q * tstep], inv));
      const double2 x2 = cmul(base[2 * m], conj_if(twp[2 * q * tstep], inv));
      const double2 x3 = cmul(base[3 * m], conj_if(twp[3 * q * tstep], inv));
      const double2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
      const double2 t2 = cadd(x1, x3), d = csub(x1, x3);
      // forward root w_4 = -i: t3 = -i d; inverse: +i d
      const double2 t3 = inv ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
      base[0] = cadd(t0, t2);
      base[2 * m] = csub(t0, t2);
      base[m] = cadd(t1, t3);
      base[3 * m] = csub(t1, t3);
    } else {
      constexpr int H = (P - 1) / 2;
      const double2 x0 = base[0];
      double2 a[H], d[H];
#pragma unroll
      for (int t = 1; t <= H; ++t) {
        const double2 xp = cmul(base[t * m], conj_if(twp[t * q * tstep], inv));
        const double2 xm = cmul(base[(P - t) * m], conj_if(twp[(P - t) * q * tstep], inv));
        a[t - 1] = cadd(xp, xm);
        d[t - 1] = csub(xp, xm);
      }
      double2 y0 = x0;
#pragma unroll
      for (int t = 0; t < H; ++t) y0 = cadd(y0, a[t]);
      base[0] = y0;
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        double2 U = x0, W = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 1; t <= H; ++t) {
          const int r = (t * j) % P;
          const double cs = r <= H ? rt[r - 1].x : rt[P - r - 1].x;     // cos(2 pi t j / P)
          const double sn = r <= H ? -rt[r - 1].y : rt[P - r - 1].y;    // sin(2 pi t j / P)
          U.x = fma(a[t - 1].x, cs, U.x);
          U.y = fma(a[t - 1].y, cs, U.y);
          W.x = fma(d[t - 1].x, sn, W.x);
          W.y = fma(d[t - 1].y, sn, W.y);
        }
        // -i W = (W.y, -W.x)
        const double2 lo = inv ? make_double2(U.x - W.y, U.y + W.x) : make_double2(U.x + W.y, U.y - W.x);
        const double2 hi = inv ? make_double2(U.x + W.y, U.y - W.x) : make_double2(U.x - W.y, U.y + W.x);
        base[j * m] = lo;
        base[(P - j) * m] = hi;
      }
    }
  }
  __syncthreads();
}

// A stage of any radix p: one output per element, computed from LDS into
// registers, written after a barrier.
template <class TW>
__device__ __forceinline__ void stage_generic(const FftArgs& A, double2* lds, int Lp, TW twp, int p,
                                              int m, int ncol, bool inv) {
  const int L = A.L, mp = m * p, tstep = L / mp, ne = L * A.TC;
  double2 reg[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int e = threadIdx.x + r * FT;
    if (e >= ne) continue;
    const CJ cj = elem(A, e);
    const int c = cj.c, k = cj.j;
    if (c >= ncol) continue;
    const int q = k % mp;
    const double2* src = lds + c * Lp + (k - q) + (q % m);
    double2 acc = make_double2(0.0, 0.0);
    int ti = 0;
    for (int t = 0; t < p; ++t) {
      acc = cmad(acc, src[t * m], conj_if(twp[ti * tstep], inv));
      ti += q;
      if (ti >= mp) ti -= mp;
    }
    reg[r] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int e = threadIdx.x + r * FT;
    if (e >= ne) continue;
    const CJ cj = elem(A, e);
    const int c = cj.c, k = cj.j;
    if (c < ncol) lds[c * Lp + k] = reg[r];
  }
  __syncthreads();
}

// All stages of one transform over the lines in LDS (digit-reversed input,
// natural-order output).  RC is the radix class of the axis (FFT_RC_*): a
// kernel only carries the butterflies its lengths need, which keeps the
// register count of the common lengths low.
template <int RC, class TW>
__device__ __forceinline__ void fft_lines(const FftArgs& A, double2* lds, int Lp, TW twp,
                                          int ncol, bool inv) {
  for (int s = 0; s < A.nst; ++s) {
    const int p = A.plan[2 * s], m = A.plan[2 * s + 1];
    switch (p) {
      case 2: stage_bfly<2>(A, lds, Lp, twp, m, ncol, inv); break;
      case 3: stage_bfly<3>(A, lds, Lp, twp, m, ncol, inv); break;
      case 4: stage_bfly<4>(A, lds, Lp, twp, m, ncol, inv); break;
      case 5: stage_bfly<5>(A, lds, Lp, twp, m, ncol, inv); break;
      case 7: stage_bfly<7>(A, lds, Lp, twp, m, ncol, inv); break;
      default:
        if constexpr (RC >= FFT_RC_11) {
          if (p == 11) { stage_bfly<11>(A, lds, Lp, twp, m, ncol, inv); break; }
        }
        if constexpr (RC == FFT_RC_ANY) stage_generic(A, lds, Lp, twp, p, m, ncol, inv);
        break;
    }
  }
}

template <int MODE, int RC, bool TWL>
__global__ __launch_bounds__(FT) void fft_kernel(FftArgs A) {
  extern __shared__ __align__(16) double2 lds[];
  const int L = A.L, TC = A.TC, Lp = L + 1, ne = L * TC;
  const Lines bl = block_lines(A);
  // twiddle table: staged in LDS after the lines when it fits
  double2* twl = lds + TC * Lp;
  if (TWL)
    for (int j = threadIdx.x; j < L; j += FT) twl[j] = A.tw[j];
  const double2* twp;
  if constexpr (TWL) twp = twl;
  else twp = A.tw;
  const double2* __restrict__ src = reinterpret_cast<const double2*>(A.src);
  double2* __restrict__ dst = reinterpret_cast<double2*>(A.dst);
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int e = threadIdx.x + r * FT;
    if (e >= ne) continue;
    const CJ cj = elem(A, e);
    const int c = cj.c, j = cj.j;
    if (c < bl.ncol) lds[c * Lp + A.rev[j]] = src[gaddr(A, bl, c, j)];
  }
  __syncthreads();
  const bool inv0 = (MODE == FFT_INV || MODE == FFT_LAST);
  fft_lines<RC>(A, lds, Lp, twp, bl.ncol, inv0);

  if (MODE == FFT_SYM) {
    // divide by sum_a d_a[m_a] - k0^2 - i eps (the axis is 0; the other
    // frequency indices come from the fastest-axis position i0 + c), then
    // put the spectrum back in digit-reversed order for the inverse
    double2 reg[FR];
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const int e = threadIdx.x + r * FT;
      if (e >= ne) continue;
      const CJ cj = elem(A, e);
      const int c = cj.c, k = cj.j;
      if (c >= bl.ncol) continue;
      const long long i = bl.i0 + c;
      double sr = A.d[0][k] - A.k0sq;
      if (A.dim == 2) sr += A.d[1][i];
      else sr += A.d[1][i / A.n[2]] + A.d[2][i % A.n[2]];
      const double si = -A.eps;
      const double den = 1.0 / (sr * sr + si * si);
      const double2 v = lds[c * Lp + k];
      // v / (sr + i si) = v (sr - i si) / |.|^2
      reg[r] = make_double2((v.x * sr + v.y * si) * den, (v.y * sr - v.x * si) * den);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const int e = threadIdx.x + r * FT;
      if (e >= ne) continue;
      const CJ cj = elem(A, e);
      const int c = cj.c, k = cj.j;
      if (c < bl.ncol) lds[c * Lp + A.rev[k]] = reg[r];
    }
    __syncthreads();
    fft_lines<RC>(A, lds, Lp, twp, bl.ncol, true);
  }

#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int e = threadIdx.x + r * FT;
    if (e >= ne) continue;
    const CJ cj = elem(A, e);
    const int c = cj.c, k = cj.j;
    if (c >= bl.ncol) continue;
    const long long pidx = gaddr(A, bl, c, k);
    double2 v = lds[c * Lp + k];
    if (MODE == FFT_LAST) {
      v.x *= A.scale;
      v.y *= A.scale;
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
        continue;
      }
    }
    dst[pidx] = v;
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

size_t fft_lds_bytes(const FftArgs& a) {
  return ((size_t)a.TC * (a.L + 1) + (a.tw_lds ? (size_t)a.L : 0)) * 16;
}

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
  if (lds > FFT_MAXLDS) return hipErrorInvalidValue;
#define FFT_LAUNCH(M, R)                                                                  \
  do {                                                                                    \
    if (a.tw_lds) hipLaunchKernelGGL((fft_kernel<M, R, true>), dim3((unsigned)nb), dim3(FT), lds, s, a); \
    else hipLaunchKernelGGL((fft_kernel<M, R, false>), dim3((unsigned)nb), dim3(FT), lds, s, a); \
  } while (0)
#define FFT_BY_RC(M)                                     \
  switch (a.rc) {                                        \
    case FFT_RC_SMALL: FFT_LAUNCH(M, FFT_RC_SMALL); break; \
    case FFT_RC_11: FFT_LAUNCH(M, FFT_RC_11); break;       \
    default: FFT_LAUNCH(M, FFT_RC_ANY); break;             \
  }
  switch (mode) {
    case FFT_FWD: FFT_BY_RC(FFT_FWD); break;
    case FFT_SYM: FFT_BY_RC(FFT_SYM); break;
    case FFT_INV: FFT_BY_RC(FFT_INV); break;
    case FFT_LAST: FFT_BY_RC(FFT_LAST); break;
    default: return hipErrorInvalidValue;
  }
#undef FFT_BY_RC
#undef FFT_LAUNCH
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
