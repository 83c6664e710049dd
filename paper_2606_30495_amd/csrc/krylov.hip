// FP64 Arnoldi / FGMRES kernels (right-preconditioned flexible GMRES).
//
// Classical Gram-Schmidt in "multi-dot" form: one pass reads w once (kept in
// registers) and every basis vector V_i once, producing all inner products
// <V_i, w> plus |w|^2; a second pass updates w -= sum_i h_i V_i and emits
// |w|^2.  The two-pass re-orthogonalisation runs only when the norm dropped
// below 1/sqrt(2) of its value before the pass (the device sets a skip flag
// that the second pass's kernels read, so the host never waits for it).
// All reductions are fixed-order (per-block partials, then one block per
// output), so results are bitwise reproducible run to run and do not depend
// on which other problems share a batched launch.
//
// Every kernel is a device body shared by a single-problem launcher and a
// batched one (one launch for many problems, per-problem arguments from a
// KArgs table; problems flagged in `frozen` return at once).
#include "internal.h"

namespace mcmg {

namespace {

constexpr int RB = 256;   // threads per block
constexpr int RPT = 4;    // complex entries per thread

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block sum, result valid in thread 0.  sh must hold RB/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < RB / 64; ++i) t += sh[i];
  return t;
}

// Block sums of NV values at once, each in block_sum's order (wave tree,
// then the waves in order), with one pair of barriers for all of them;
// results valid in thread 0.  sh must hold NV * RB/64 doubles.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * (RB / 64) + wv] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = 0.0;
      for (int i = 0; i < RB / 64; ++i) t += sh[k * (RB / 64) + i];
      v[k] = t;
    }
  }
}

// Vectors per batch of the multi-dot: the loads of VB basis vectors are in
// flight together and their 2 VB sums share one pair of barriers.
constexpr int VB = 4;

__device__ __forceinline__ void multidot_body(const double* __restrict__ V_, long long ldv, int nvec,
                                              const double* __restrict__ w_, long long n,
                                              double* __restrict__ partial_, int nb, int vblk) {
  const gptr<const double> V = to_global<const double>(V_), w = to_global<const double>(w_);
  const gptr<double> partial = to_global<double>(partial_);
  __shared__ double sh[2 * VB * (RB / 64)];
  const long long base = (long long)vblk * RB * RPT;
  double wr[RPT], wi[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const long long p = base + (long long)q * RB + threadIdx.x;
    if (p < n) { wr[q] = w[2 * p]; wi[q] = w[2 * p + 1]; }
    else { wr[q] = 0.0; wi[q] = 0.0; }
  }
  for (int i0 = 0; i0 < nvec; i0 += VB) {
    // all loads of the batch first (vectors past nvec and points past n
    // read valid entries and are discarded), then the sums
    double vr[VB][RPT], vi[VB][RPT];
#pragma unroll
    for (int k = 0; k < VB; ++k) {
      const gptr<const double> v = V + (long long)(i0 + k < nvec ? i0 + k : 0) * 2 * ldv;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const long long p = base + (long long)q * RB + threadIdx.x;
        const long long pc = p < n ? p : 0;
        vr[k][q] = v[2 * pc];
        vi[k][q] = v[2 * pc + 1];
      }
    }
    double acc[2 * VB];
#pragma unroll
    for (int k = 0; k < VB; ++k) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const long long p = base + (long long)q * RB + threadIdx.x;
        if (p < n) {
          // conj(v) * w
          sr += vr[k][q] * wr[q] + vi[k][q] * wi[q];
          si += vr[k][q] * wi[q] - vi[k][q] * wr[q];
        }
      }
      acc[2 * k] = sr;
      acc[2 * k + 1] = si;
    }
    block_sums<2 * VB>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < VB; ++k) {
        if (i0 + k >= nvec) break;
        partial[2 * ((long long)(i0 + k) * nb + vblk)] = acc[2 * k];
        partial[2 * ((long long)(i0 + k) * nb + vblk) + 1] = acc[2 * k + 1];
      }
    }
  }
  double s2 = 0.0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) s2 += wr[q] * wr[q] + wi[q] * wi[q];
  double t2[1] = {s2};
  block_sums<1>(t2, sh);
  if (threadIdx.x == 0) {
    partial[2 * ((long long)nvec * nb + vblk)] = t2[0];
    partial[2 * ((long long)nvec * nb + vblk) + 1] = 0.0;
  }
}

// Output i of the dot reduction (i == nvec: |w|^2), fixed-order tree.
__device__ __forceinline__ void reduce_dots_body(const double* __restrict__ partial, int nb, int nvec,
                                                 double* __restrict__ coef, double* __restrict__ Hcol,
                                                 double* __restrict__ wnorm2, int i) {
  __shared__ double sh[RB / 64];
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < nb; b += RB) {
    sr += partial[2 * ((long long)i * nb + b)];
    si += partial[2 * ((long long)i * nb + b) + 1];
  }
  const double tr = block_sum(sr, sh);
  const double ti = block_sum(si, sh);
  if (threadIdx.x == 0) {
    if (i < nvec) {
      coef[2 * i] = tr;
      coef[2 * i + 1] = ti;
      Hcol[2 * i] += tr;
      Hcol[2 * i + 1] += ti;
    } else {
      wnorm2[0] = tr;
    }
  }
}

__device__ __forceinline__ void update_body(const double* __restrict__ V_, long long ldv, int nvec,
                                            const double* __restrict__ coef_, double* __restrict__ w_,
                                            long long n, double* __restrict__ partial_, int vblk) {
  const gptr<const double> V = to_global<const double>(V_), coef = to_global<const double>(coef_);
  const gptr<double> w = to_global<double>(w_), partial = to_global<double>(partial_);
  __shared__ double sh[RB / 64];
  const long long base = (long long)vblk * RB * RPT;
  double ar[RPT], ai[RPT];
  bool ok[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const long long p = base + (long long)q * RB + threadIdx.x;
    ok[q] = p < n;
    ar[q] = ok[q] ? w[2 * p] : 0.0;
    ai[q] = ok[q] ? w[2 * p + 1] : 0.0;
  }
  // vector-outer, so the loads of all the thread's points (and, unrolled,
  // of two vectors) are in flight together; each point still sums over i in
  // order
#pragma unroll 2
  for (int i = 0; i < nvec; ++i) {
    const double cr = coef[2 * i], ci = coef[2 * i + 1];
    const gptr<const double> v = V + (long long)i * 2 * ldv;
    // points past n read entry 0 and are never stored (no branch splits
    // the loads); all loads first, then the updates
    double vr[RPT], vi[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const long long p = ok[q] ? base + (long long)q * RB + threadIdx.x : 0;
      vr[q] = v[2 * p];
      vi[q] = v[2 * p + 1];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      ar[q] -= cr * vr[q] - ci * vi[q];
      ai[q] -= cr * vi[q] + ci * vr[q];
    }
  }
  double s2 = 0.0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    if (!ok[q]) continue;
    const long long p = base + (long long)q * RB + threadIdx.x;
    w[2 * p] = ar[q];
    w[2 * p + 1] = ai[q];
    s2 += ar[q] * ar[q] + ai[q] * ai[q];
  }
  const double t = block_sum(s2, sh);
  if (threadIdx.x == 0) partial[vblk] = t;
}

__device__ __forceinline__ void reduce_norm_body(const double* __restrict__ partial, int nb,
                                                 const double* __restrict__ wnorm2,
                                                 double* __restrict__ hn, int* skip, int pass,
                                                 int always_two) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += RB) s += partial[b];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) {
    const double nrm = sqrt(t);
    hn[0] = nrm;
    if (pass == 0) {
      // eta = 1/sqrt(2): re-orthogonalise when cancellation removed more
      // than half of |w|^2 (Daniel-Gragg-Kaufman-Stewart criterion).
      const bool again = always_two || (nrm * nrm < 0.5 * wnorm2[0]);
      skip[0] = again ? 0 : 1;
    }
  }
}

// Largest restart length whose back substitution stages the whole upper
// triangle of H in LDS; the batched engine takes restarts up to this length.
constexpr int KMAX = 64;
// Largest restart length a handle takes (single-problem solves): bounds the
// LDS copies of one Hessenberg column and of the right-hand side of the
// triangular solve.
constexpr int KMAX_LONG = 1024;

// Givens step on column j of H (complex, column-major, ldh rows), by one
// block: the threads copy the column and the stored rotations to LDS, one
// thread applies the rotations there in order (each on the entry the
// previous one produced) and computes the new one, and the threads write
// the column back.  hn[0] may have been written by thread 0 of this block.
// out = (|g_{j+1}|, h_{j+1,j}, |column j| before rotation, |new diagonal|);
// a zero diagonal (a column that is zero after the earlier rotations) makes
// column j unusable for the triangular solve, and the host leaves it out.
__device__ __forceinline__ void givens_block(double* __restrict__ H, int ldh, int j,
                                             const double* hn, double* __restrict__ cs,
                                             double* __restrict__ sn, double* __restrict__ g,
                                             double* out) {
  __shared__ double2 colS[KMAX_LONG + 1];
  __shared__ double2 snS[KMAX_LONG];
  __shared__ double csS[KMAX_LONG];
  double* __restrict__ col = H + 2LL * j * ldh;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i <= j; i += nt) colS[i] = make_double2(col[2 * i], col[2 * i + 1]);
  for (int i = tid; i < j; i += nt) {
    csS[i] = cs[i];
    snS[i] = make_double2(sn[2 * i], sn[2 * i + 1]);
  }
  __syncthreads();
  if (tid == 0) {
    const double b = hn[0];
    // |column j| before rotation, h_{j+1,j} = b (real) in its last entry
    double cn = 0.0;
    for (int i = 0; i <= j; ++i) cn += colS[i].x * colS[i].x + colS[i].y * colS[i].y;
    cn += b * b;
    cn = sqrt(cn);
    // x: entry i after rotations 0..i-1
    double xr = colS[0].x, xi = colS[0].y;
    for (int i = 0; i < j; ++i) {
      const double yr = colS[i + 1].x, yi = colS[i + 1].y;
      const double c = csS[i], sr = snS[i].x, si = snS[i].y;
      // x' = c x + conj(s) y ; y' = -s x + c y
      colS[i] = make_double2(c * xr + (sr * yr + si * yi), c * xi + (sr * yi - si * yr));
      const double nr = -(sr * xr - si * xi) + c * yr;
      const double ni = -(sr * xi + si * xr) + c * yi;
      xr = nr;
      xi = ni;
    }
    const double ar = xr, ai = xi;
    const double aa = hypot(ar, ai);
    const double t = hypot(aa, b);
    double c, sr, si;
    if (aa == 0.0) { c = 0.0; sr = 1.0; si = 0.0; }
    else {
      c = aa / t;
      // s = (conj(a) / |a|) * (b / t)
      sr = (ar / aa) * (b / t);
      si = (-ai / aa) * (b / t);
    }
    cs[j] = c; sn[2 * j] = sr; sn[2 * j + 1] = si;
    // new diagonal = c a + conj(s) b; the rotation zeroes h_{j+1,j}
    colS[j] = make_double2(c * ar + sr * b, c * ai - si * b);
    colS[j + 1] = make_double2(0.0, 0.0);
    const double gr = g[2 * j], gi = g[2 * j + 1];
    // g_{j+1} = -s g_j ; g_j = c g_j
    const double g1r = -(sr * gr - si * gi), g1i = -(sr * gi + si * gr);
    g[2 * (j + 1)] = g1r;
    g[2 * (j + 1) + 1] = g1i;
    g[2 * j] = c * gr;
    g[2 * j + 1] = c * gi;
    out[0] = hypot(g1r, g1i);
    out[1] = b;
    out[2] = cn;
    out[3] = t;
  }
  __syncthreads();
  for (int i = tid; i <= j + 1; i += nt) {
    col[2 * i] = colS[i].x;
    col[2 * i + 1] = colS[i].y;
  }
}

// y = H[0:k,0:k]^{-1} g[0:k] by back substitution, by one block.  Up to
// KMAX columns the threads copy the upper triangle of H (packed by columns)
// and g to LDS, one thread substitutes there (row k-1 first, each row's sum
// in column order), and the threads write y.  Longer systems substitute by
// columns: y_i = s_i / H_ii by one thread, then every thread removes
// H_li y_i from its rows l < i of s (kept in LDS), reading H from global
// memory; each row's sum then runs from column k-1 down.
__device__ __forceinline__ void backsolve_block(const double* __restrict__ H, int ldh, int k,
                                                const double* __restrict__ g,
                                                double* __restrict__ y) {
  __shared__ double2 tri[KMAX * (KMAX + 1) / 2];
  __shared__ double2 ys[KMAX_LONG];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (k > KMAX) {
    for (int i = tid; i < k; i += nt) ys[i] = make_double2(g[2 * i], g[2 * i + 1]);
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
      const double* col = H + 2LL * i * ldh;
      if (tid == 0) {
        const double dr = col[2 * i], di = col[2 * i + 1];
        const double q = dr * dr + di * di;
        const double sr = ys[i].x, si = ys[i].y;
        ys[i] = make_double2((sr * dr + si * di) / q, (si * dr - sr * di) / q);
      }
      __syncthreads();
      const double yr = ys[i].x, yi = ys[i].y;
      for (int l = tid; l < i; l += nt) {
        const double hr = col[2 * l], hi = col[2 * l + 1];
        ys[l] = make_double2(ys[l].x - (hr * yr - hi * yi), ys[l].y - (hr * yi + hi * yr));
      }
      __syncthreads();
    }
    for (int i = tid; i < k; i += nt) {
      y[2 * i] = ys[i].x;
      y[2 * i + 1] = ys[i].y;
    }
    return;
  }
  for (int l = 0; l < k; ++l) {
    const long long c = (long long)l * ldh;
    const int o = l * (l + 1) / 2;
    for (int i = tid; i <= l; i += nt) tri[o + i] = make_double2(H[2 * (c + i)], H[2 * (c + i) + 1]);
  }
  for (int i = tid; i < k; i += nt) ys[i] = make_double2(g[2 * i], g[2 * i + 1]);
  __syncthreads();
  if (tid == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double sr = ys[i].x, si = ys[i].y;
      for (int l = i + 1; l < k; ++l) {
        const double2 h = tri[l * (l + 1) / 2 + i];
        const double hr = h.x, hi = h.y;
        const double yr = ys[l].x, yi = ys[l].y;
        sr -= hr * yr - hi * yi;
        si -= hr * yi + hi * yr;
      }
      const double2 d = tri[i * (i + 1) / 2 + i];
      const double dr = d.x, di = d.y;
      const double q = dr * dr + di * di;
      ys[i] = make_double2((sr * dr + si * di) / q, (si * dr - sr * di) / q);
    }
  }
  __syncthreads();
  for (int i = tid; i < k; i += nt) {
    y[2 * i] = ys[i].x;
    y[2 * i + 1] = ys[i].y;
  }
}

__device__ __forceinline__ void zupdate_body(const float* __restrict__ Z_, long long ldz, int k,
                                             const double* __restrict__ y_, double* __restrict__ u_,
                                             long long n, long long p) {
  const gptr<const float> Z = to_global<const float>(Z_);
  const gptr<const double> y = to_global<const double>(y_);
  const gptr<double> u = to_global<double>(u_);
  if (p >= n) return;
  double ar = u[2 * p], ai = u[2 * p + 1];
  for (int i = 0; i < k; ++i) {
    const gptr<const float> z = Z + (long long)i * 2 * ldz;
    const double zr = z[2 * p], zi = z[2 * p + 1];
    const double yr = y[2 * i], yi = y[2 * i + 1];
    ar += yr * zr - yi * zi;
    ai += yr * zi + yi * zr;
  }
  u[2 * p] = ar;
  u[2 * p + 1] = ai;
}

__device__ __forceinline__ void reduce_sum_body(const double* __restrict__ partial, int nb,
                                                double* __restrict__ out) {
  __shared__ double sh[RB / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += RB) s += partial[b];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) { out[0] = t; out[1] = sqrt(t); }
}

// ---- single-problem kernels -------------------------------------------------

__global__ __launch_bounds__(RB) void multidot_kernel(const double* __restrict__ V, long long ldv,
                                                      int nvec, const double* __restrict__ w,
                                                      long long n, double* __restrict__ partial,
                                                      const int* __restrict__ skip) {
  if (skip && skip[0]) return;
  multidot_body(V, ldv, nvec, w, n, partial, gridDim.x, blockIdx.x);
}

__global__ __launch_bounds__(RB) void reduce_dots_kernel(const double* __restrict__ partial, int nb,
                                                         int nvec, double* __restrict__ coef,
                                                         double* __restrict__ Hcol,
                                                         double* __restrict__ wnorm2,
                                                         const int* __restrict__ skip) {
  if (skip && skip[0]) return;
  reduce_dots_body(partial, nb, nvec, coef, Hcol, wnorm2, blockIdx.x);
}

__global__ __launch_bounds__(RB) void update_kernel(const double* __restrict__ V, long long ldv,
                                                    int nvec, const double* __restrict__ coef,
                                                    double* __restrict__ w, long long n,
                                                    double* __restrict__ partial,
                                                    const int* __restrict__ skip) {
  if (skip && skip[0]) return;
  update_body(V, ldv, nvec, coef, w, n, partial, blockIdx.x);
}

__global__ __launch_bounds__(RB) void reduce_norm_kernel(const double* __restrict__ partial, int nb,
                                                         const double* __restrict__ wnorm2,
                                                         double* __restrict__ hn, int* skip,
                                                         int pass, int always_two) {
  if (pass == 1 && skip[0]) return;
  reduce_norm_body(partial, nb, wnorm2, hn, skip, pass, always_two);
}

__global__ void scale_kernel(const double* __restrict__ w, const double* __restrict__ hn,
                             double* __restrict__ v, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double inv = 1.0 / hn[0];
  v[2 * p] = w[2 * p] * inv;
  v[2 * p + 1] = w[2 * p + 1] * inv;
}

__global__ void init_g_kernel(double* g, int m1, const double* beta) {
  for (int i = threadIdx.x; i < m1; i += blockDim.x) {
    g[2 * i] = (i == 0) ? beta[0] : 0.0;
    g[2 * i + 1] = 0.0;
  }
}

// The norm reduce of the second Gram-Schmidt pass (unless the device skipped
// that pass) and the Givens step on column j, in one launch.
__global__ __launch_bounds__(RB) void norm_givens_kernel(const double* __restrict__ partial, int nb,
                                                         const double* wnorm2, double* hn,
                                                         int* skip, double* H, int ldh, int j,
                                                         double* cs, double* sn, double* g,
                                                         double* out) {
  if (!skip[0]) reduce_norm_body(partial, nb, wnorm2, hn, skip, 1, 0);
  givens_block(H, ldh, j, hn, cs, sn, g, out);
}

__global__ __launch_bounds__(64) void backsolve_kernel(const double* H, int ldh, int k,
                                                       const double* g, double* y) {
  backsolve_block(H, ldh, k, g, y);
}

__global__ __launch_bounds__(RB) void zupdate_kernel(const float* __restrict__ Z, long long ldz,
                                                     int k, const double* __restrict__ y,
                                                     double* __restrict__ u, long long n) {
  zupdate_body(Z, ldz, k, y, u, n, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(RB) void reduce_sum_kernel(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ out) {
  reduce_sum_body(partial, nb, out);
}

__global__ void axpy_f32_kernel(const float* __restrict__ z, double* __restrict__ u, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= 2 * n) return;
  u[p] += (double)z[p];
}

__global__ void cast_kernel(const float* __restrict__ z, double* __restrict__ u, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= 2 * n) return;
  u[p] = (double)z[p];
}

__global__ void copy_kernel(const double* __restrict__ a, double* __restrict__ b, long long n) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= 2 * n) return;
  b[p] = a[p];
}

// ---- batched kernels ---------------------------------------------------------
// pre: per-problem block prefix; frozen: per-problem skip flag (may be null);
// jpos: per-problem Krylov position j (column of H, nvec = j + 1 basis
// vectors); kk: per-problem length of the cycle being closed.

__device__ __forceinline__ bool is_frozen(const int* frozen, int p) { return frozen && frozen[p]; }

__global__ __launch_bounds__(RB) void kb_multidot(const KArgs* __restrict__ tab,
                                                  const int* __restrict__ pre, int np,
                                                  const int* __restrict__ frozen,
                                                  const int* __restrict__ jpos, int pass) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  if (pass == 1 && to_global<const int>(A.skip)[0]) return;
  multidot_body(A.V, A.N, jpos[p] + 1, A.w, A.N, A.partial, red_blocks(A.N), blockIdx.x - pre[p]);
}

// grid (m + 1, np): block x reduces output x of problem y (x == nvec: |w|^2)
__global__ __launch_bounds__(RB) void kb_reduce_dots(const KArgs* __restrict__ tab,
                                                     const int* __restrict__ frozen,
                                                     const int* __restrict__ jpos, int pass) {
  const int p = blockIdx.y;
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  const int j = jpos[p];
  if ((int)blockIdx.x > j + 1) return;
  if (pass == 1 && to_global<const int>(A.skip)[0]) return;
  reduce_dots_body(A.partial, red_blocks(A.N), j + 1, A.coef, A.H + 2LL * j * A.ldh,
                   A.scal + (pass == 0 ? 8 : 10), blockIdx.x);
}

__global__ __launch_bounds__(RB) void kb_update(const KArgs* __restrict__ tab,
                                                const int* __restrict__ pre, int np,
                                                const int* __restrict__ frozen,
                                                const int* __restrict__ jpos, int pass) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  if (pass == 1 && to_global<const int>(A.skip)[0]) return;
  update_body(A.V, A.N, jpos[p] + 1, A.coef, A.w, A.N, A.partial, blockIdx.x - pre[p]);
}

__global__ __launch_bounds__(RB) void kb_reduce_norm(const KArgs* __restrict__ tab,
                                                     const int* __restrict__ frozen, int pass) {
  const int p = blockIdx.x;
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  if (pass == 1 && to_global<const int>(A.skip)[0]) return;
  reduce_norm_body(A.partial, red_blocks(A.N), A.scal + 8, A.scal + 9, A.skip, pass,
                   pass == 0 ? A.always_two : 0);
}

// The second pass's norm reduce (unless skipped) and the Givens step.
__global__ __launch_bounds__(RB) void kb_givens(const KArgs* __restrict__ tab,
                                                const int* __restrict__ frozen,
                                                const int* __restrict__ jpos,
                                                double* __restrict__ gather) {
  const int p = blockIdx.x;
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  if (!to_global<const int>(A.skip)[0])
    reduce_norm_body(A.partial, red_blocks(A.N), A.scal + 8, A.scal + 9, A.skip, 1, 0);
  givens_block(A.H, A.ldh, jpos[p], A.scal + 9, A.cs, A.sn, A.g, A.scal + 16);
  if (threadIdx.x != 0) return;
  gather[4 * p + 0] = A.scal[16];
  gather[4 * p + 1] = A.scal[17];
  gather[4 * p + 2] = A.scal[18];
  gather[4 * p + 3] = A.scal[19];     // |new diagonal| (slot 3 holds |r| after a residual tick)
}

// mode 0: V_0 = r / |r|  (|r| in scal[3]);  mode 1: V_{j+1} = w / h_{j+1,j}
__global__ __launch_bounds__(RB) void kb_scale(const KArgs* __restrict__ tab,
                                               const int* __restrict__ pre, int np,
                                               const int* __restrict__ frozen,
                                               const int* __restrict__ jpos, int mode) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  const long long q = (long long)(blockIdx.x - pre[p]) * RB + threadIdx.x;
  if (q >= A.N) return;
  const gptr<const double> src = to_global<const double>(mode == 0 ? A.r : A.w);
  const gptr<double> dst = to_global<double>(A.V) + (mode == 0 ? 0LL : 2LL * (jpos[p] + 1) * A.N);
  const double inv = 1.0 / (mode == 0 ? to_global<const double>(A.scal)[3] : to_global<const double>(A.scal)[9]);
  dst[2 * q] = src[2 * q] * inv;
  dst[2 * q + 1] = src[2 * q + 1] * inv;
}

// cycle start: H = 0, g = (|r|, 0, ...)
__global__ __launch_bounds__(RB) void kb_cycle_init(const KArgs* __restrict__ tab,
                                                    const int* __restrict__ frozen, int m) {
  const int p = blockIdx.x;
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  const int nh = 2 * A.ldh * m;
  for (int i = threadIdx.x; i < nh; i += RB) A.H[i] = 0.0;
  for (int i = threadIdx.x; i < 2 * (m + 1); i += RB) A.g[i] = (i == 0) ? A.scal[3] : 0.0;
}

__global__ __launch_bounds__(64) void kb_backsolve(const KArgs* __restrict__ tab,
                                                   const int* __restrict__ frozen,
                                                   const int* __restrict__ kk) {
  const int p = blockIdx.x;
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  if (kk[p] > 0) backsolve_block(A.H, A.ldh, kk[p], A.g, A.y);
}

__global__ __launch_bounds__(RB) void kb_zupdate(const KArgs* __restrict__ tab,
                                                 const int* __restrict__ pre, int np,
                                                 const int* __restrict__ frozen,
                                                 const int* __restrict__ kk) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (is_frozen(frozen, p) || kk[p] <= 0) return;
  const KArgs& A = tab[p];
  zupdate_body(A.Z, A.N, kk[p], A.y, A.u, A.N, (long long)(blockIdx.x - pre[p]) * RB + threadIdx.x);
}

// |f - A u| after the batched residual kernel: scal[2] = |r|^2, scal[3] = |r|
__global__ __launch_bounds__(RB) void kb_reduce_sum(const KArgs* __restrict__ tab,
                                                    const int* __restrict__ frozen,
                                                    double* __restrict__ gather) {
  const int p = blockIdx.x;
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  reduce_sum_body(A.partial, red_blocks(A.N), A.scal + 2);
  if (threadIdx.x == 0) gather[4 * p + 3] = A.scal[3];
}

// |f|^2: per-block partials of f (the multi-dot with no basis vectors), then
// the same fixed-order reduction the single-problem solver uses.
__global__ __launch_bounds__(RB) void kb_fnorm_partial(const KArgs* __restrict__ tab,
                                                       const int* __restrict__ pre, int np,
                                                       const int* __restrict__ frozen) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  multidot_body(nullptr, A.N, 0, A.f, A.N, A.partial, red_blocks(A.N), blockIdx.x - pre[p]);
}

__global__ __launch_bounds__(RB) void kb_fnorm_reduce(const KArgs* __restrict__ tab,
                                                      const int* __restrict__ frozen,
                                                      double* __restrict__ gather) {
  const int p = blockIdx.x;
  if (is_frozen(frozen, p)) return;
  const KArgs& A = tab[p];
  reduce_dots_body(A.partial, red_blocks(A.N), 0, A.coef, A.coef, A.scal + 0, 0);
  if (threadIdx.x == 0) gather[4 * p + 0] = A.scal[0];
}

inline unsigned nblk(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

__host__ __device__ int red_blocks(long long n) {
  return (int)((n + (long long)RB * RPT - 1) / ((long long)RB * RPT));
}
int elem_blocks(long long n) { return (int)((n + RB - 1) / RB); }

hipError_t launch_multidot(const double* V, long long ldv, int nvec, const double* w, long long n,
                           double* partial, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(multidot_kernel, dim3(red_blocks(n)), dim3(RB), 0, s, V, ldv, nvec, w, n,
                     partial, skip);
  return hipGetLastError();
}

hipError_t launch_reduce_dots(const double* partial, int nb, int nvec, double* coef, double* Hcol,
                              double* wnorm2, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(reduce_dots_kernel, dim3(nvec + 1), dim3(RB), 0, s, partial, nb, nvec, coef,
                     Hcol, wnorm2, skip);
  return hipGetLastError();
}

hipError_t launch_update(const double* V, long long ldv, int nvec, const double* coef, double* w,
                         long long n, double* partial, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(red_blocks(n)), dim3(RB), 0, s, V, ldv, nvec, coef, w, n,
                     partial, skip);
  return hipGetLastError();
}

hipError_t launch_reduce_norm(const double* partial, int nb, const double* wnorm2, double* hn,
                              int* skip, int pass, int always_two, hipStream_t s) {
  hipLaunchKernelGGL(reduce_norm_kernel, dim3(1), dim3(RB), 0, s, partial, nb, wnorm2, hn, skip,
                     pass, always_two);
  return hipGetLastError();
}

hipError_t launch_scale(const double* w, const double* hn, double* v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, w, hn, v, n);
  return hipGetLastError();
}

hipError_t launch_norm_givens(const double* partial, int nb, const double* wnorm2, double* hn,
                              int* skip, double* H, int ldh, int j, double* cs, double* sn,
                              double* g, double* out, hipStream_t s) {
  if (j < 0 || j >= KMAX_LONG) return hipErrorInvalidValue;
  hipLaunchKernelGGL(norm_givens_kernel, dim3(1), dim3(RB), 0, s, partial, nb, wnorm2, hn, skip, H,
                     ldh, j, cs, sn, g, out);
  return hipGetLastError();
}

hipError_t launch_init_g(double* g, int m1, const double* beta, hipStream_t s) {
  hipLaunchKernelGGL(init_g_kernel, dim3(1), dim3(256), 0, s, g, m1, beta);
  return hipGetLastError();
}

hipError_t launch_backsolve(const double* H, int ldh, int k, const double* g, double* y,
                            hipStream_t s) {
  if (k < 0 || k > KMAX_LONG) return hipErrorInvalidValue;
  hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(64), 0, s, H, ldh, k, g, y);
  return hipGetLastError();
}

hipError_t launch_zupdate(const float* Z, long long ldz, int k, const double* y, double* u,
                          long long n, hipStream_t s) {
  hipLaunchKernelGGL(zupdate_kernel, dim3(nblk(n, RB)), dim3(RB), 0, s, Z, ldz, k, y, u, n);
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* partial, int nb, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(RB), 0, s, partial, nb, out);
  return hipGetLastError();
}

hipError_t launch_axpy_f32(const float* z, double* u, long long n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_f32_kernel, dim3(nblk(2 * n, 256)), dim3(256), 0, s, z, u, n);
  return hipGetLastError();
}

hipError_t launch_cast_f32_f64(const float* z, double* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL(cast_kernel, dim3(nblk(2 * n, 256)), dim3(256), 0, s, z, out, n);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double* a, double* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(nblk(2 * n, 256)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

// ---- batched launchers ------------------------------------------------------

hipError_t kb_launch(int op, const KBatch& b, int pass, int m, hipStream_t s) {
  if (b.np == 0) return hipSuccess;
  if (m < 1 || m > KMAX) return hipErrorInvalidValue;   // LDS copies of H columns
  switch (op) {
    case KB_MULTIDOT:
      hipLaunchKernelGGL(kb_multidot, dim3(b.total_red), dim3(RB), 0, s, b.tab, b.pre_red, b.np,
                         b.frozen, b.jpos, pass);
      break;
    case KB_REDUCE_DOTS:
      hipLaunchKernelGGL(kb_reduce_dots, dim3(m + 1, b.np), dim3(RB), 0, s, b.tab, b.frozen,
                         b.jpos, pass);
      break;
    case KB_UPDATE:
      hipLaunchKernelGGL(kb_update, dim3(b.total_red), dim3(RB), 0, s, b.tab, b.pre_red, b.np,
                         b.frozen, b.jpos, pass);
      break;
    case KB_REDUCE_NORM:
      hipLaunchKernelGGL(kb_reduce_norm, dim3(b.np), dim3(RB), 0, s, b.tab, b.frozen, pass);
      break;
    case KB_GIVENS:
      hipLaunchKernelGGL(kb_givens, dim3(b.np), dim3(RB), 0, s, b.tab, b.frozen, b.jpos, b.gather);
      break;
    case KB_SCALE_R:
      hipLaunchKernelGGL(kb_scale, dim3(b.total_elem), dim3(RB), 0, s, b.tab, b.pre_elem, b.np,
                         b.frozen, b.jpos, 0);
      break;
    case KB_SCALE_W:
      hipLaunchKernelGGL(kb_scale, dim3(b.total_elem), dim3(RB), 0, s, b.tab, b.pre_elem, b.np,
                         b.frozen, b.jpos, 1);
      break;
    case KB_CYCLE_INIT:
      hipLaunchKernelGGL(kb_cycle_init, dim3(b.np), dim3(RB), 0, s, b.tab, b.frozen, m);
      break;
    case KB_BACKSOLVE:
      hipLaunchKernelGGL(kb_backsolve, dim3(b.np), dim3(64), 0, s, b.tab, b.frozen, b.kk);
      break;
    case KB_ZUPDATE:
      hipLaunchKernelGGL(kb_zupdate, dim3(b.total_elem), dim3(RB), 0, s, b.tab, b.pre_elem, b.np,
                         b.frozen, b.kk);
      break;
    case KB_REDUCE_SUM:
      hipLaunchKernelGGL(kb_reduce_sum, dim3(b.np), dim3(RB), 0, s, b.tab, b.frozen, b.gather);
      break;
    case KB_FNORM_PARTIAL:
      hipLaunchKernelGGL(kb_fnorm_partial, dim3(b.total_red), dim3(RB), 0, s, b.tab, b.pre_red,
                         b.np, b.frozen);
      break;
    case KB_FNORM_REDUCE:
      hipLaunchKernelGGL(kb_fnorm_reduce, dim3(b.np), dim3(RB), 0, s, b.tab, b.frozen, b.gather);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mcmg
