// Training kernels: weight gradients, adjoint-weight layouts, GELU and
// elementwise backward pieces, and the Adam update (training section,
// Eq. loss_fun; Sec. llpf freezes tensors by leaving them out of the update).
//
// Parameters live in the canonical layout [d0][d1][3^D] of the weight blob.
// Convolutions read the layout [tap][cin][cpad] (cpad: the output channels
// rounded up to the VALU chunk, zero padded), built by repack_kernel:
//   forward S1 / S2 (d0 = out, d1 = in):  layout[t][b][a] = w[a][b][t];
//   forward T2 (P: d0 = coarse in, d1 = fine out): layout[t][a][b] = w[a][b][t];
//   adjoint of S1: a stride-1 convolution with the taps reversed and the
//     channel roles swapped, layout[T-1-t][a][b] = w[a][b][t];
//   adjoint of S2: the transposed stride-2 convolution with the same tensor;
//   adjoint of T2: the stride-2 convolution with the same tensor.
// The weight gradient of a convolution y = w * x is
//   dw[a][b][t] = sum over output nodes p of dy[p][co] x[q(p, t)][ci],
// with q the sampling map of the mode (S1: p + off_t, S2: 2p + off_t,
// T2: fine node p fed by coarse node (p - off_t) / 2).  wgrad_partial sums
// each entry over one chunk of output nodes; wgrad_reduce adds the chunk
// sums in a fixed order, so the gradient is deterministic.
#include <cmath>

#include "internal.h"

namespace mcmg {

namespace {

constexpr int TB = 256;

__global__ __launch_bounds__(TB) void repack_kernel(const float* __restrict__ w, int d0, int d1,
                                                    int taps, int transposed, int flip, float scale,
                                                    int cin, int cpad, float* __restrict__ out) {
  const long long n = (long long)taps * cin * cpad;
  const int cout = transposed ? d1 : d0;
  for (long long i = (long long)blockIdx.x * TB + threadIdx.x; i < n; i += (long long)gridDim.x * TB) {
    const int co = (int)(i % cpad);
    const long long r = i / cpad;
    const int ci = (int)(r % cin);
    const int t = (int)(r / cin);
    float v = 0.f;
    if (co < cout) {
      const int a = transposed ? ci : co, b = transposed ? co : ci;
      const int ts = flip ? taps - 1 - t : t;
      v = scale * w[((long long)a * d1 + b) * taps + ts];
    }
    out[i] = v;
  }
}

template <typename TX>
__global__ __launch_bounds__(TB) void wgrad_partial(WgArgs A) {
  const TX* __restrict__ x = reinterpret_cast<const TX*>(A.x);
  const float* __restrict__ dy = A.dy;
  const int taps = A.dim == 2 ? 9 : 27;
  const long long E = (long long)taps * A.cin * A.cout;
  const long long e = (long long)blockIdx.x * TB + threadIdx.x;
  if (e >= E) return;
  const int co = (int)(e % A.cout);
  const long long r = e / A.cout;
  const int ci = (int)(r % A.cin);
  const int t = (int)(r / A.cin);
  int off[3];
  if (A.dim == 2) { off[0] = t / 3 - 1; off[1] = t % 3 - 1; off[2] = 0; }
  else { off[0] = t / 9 - 1; off[1] = (t / 3) % 3 - 1; off[2] = t % 3 - 1; }
  const long long p0 = (long long)blockIdx.y * A.chunk;
  const long long p1 = p0 + A.chunk < A.out.total ? p0 + A.chunk : A.out.total;
  float acc = 0.f;
  const bool small = A.out.total < (1LL << 31);
  for (long long p = p0; p < p1; ++p) {
    int o[3];
    if (small) {
      const uint32_t pp = (uint32_t)p;
      const uint32_t q2 = fdiv(pp, A.fo2);
      const uint32_t q1 = fdiv(q2, A.fo1);
      o[2] = (int)(pp - q2 * (uint32_t)A.out.n[2]);
      o[1] = (int)(q2 - q1 * (uint32_t)A.out.n[1]);
      o[0] = (int)q1;
    } else {
      long long q = p;
      o[2] = (int)(q % A.out.n[2]); q /= A.out.n[2];
      o[1] = (int)(q % A.out.n[1]); q /= A.out.n[1];
      o[0] = (int)q;
    }
    int ii[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= A.dim) { ii[a] = 0; continue; }
      int v;
      if (A.mode == CONV_S1) v = o[a] + off[a];
      else if (A.mode == CONV_S2) v = 2 * o[a] + off[a];
      else {
        const int tt = o[a] - off[a];
        if (tt & 1) { ok = false; v = 0; }
        else v = tt >> 1;
      }
      if (v < 0 || v >= A.in.n[a]) ok = false;
      ii[a] = v;
    }
    if (!ok) continue;
    const long long src = ((long long)ii[0] * A.in.n[1] + ii[1]) * A.in.n[2] + ii[2];
    acc = fmaf(dy[p * A.cout + co], (float)x[src * A.cin + ci], acc);
  }
  A.part[(long long)blockIdx.y * E + e] = acc;
}

__global__ __launch_bounds__(TB) void wgrad_reduce(WgArgs A) {
  const int taps = A.dim == 2 ? 9 : 27;
  const long long E = (long long)taps * A.cin * A.cout;
  const long long e = (long long)blockIdx.x * TB + threadIdx.x;
  if (e >= E) return;
  float s = 0.f;
  for (int k = 0; k < A.nchunk; ++k) s += A.part[(long long)k * E + e];
  const int co = (int)(e % A.cout);
  const long long r = e / A.cout;
  const int ci = (int)(r % A.cin);
  const int t = (int)(r / A.cin);
  // canonical [d0][d1][t]: S1/S2 tensors have d0 = out, d1 = in; P (T2) has
  // d0 = coarse in, d1 = fine out
  const int a = A.mode == CONV_T2 ? ci : co, b = A.mode == CONV_T2 ? co : ci;
  const int d1 = A.mode == CONV_T2 ? A.cout : A.cin;
  float* g = A.dw + ((long long)a * d1 + b) * taps + t;
  *g += A.scale * s;
}

__device__ __forceinline__ float gelu_f(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
// d/dx [x Phi(x)] = Phi(x) + x phi(x)
__device__ __forceinline__ float gelu_d(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

__global__ void gelu_fwd_kernel(const float* __restrict__ z, float* __restrict__ a, long long n) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i < n) a[i] = gelu_f(z[i]);
}

__global__ void gelu_bwd_kernel(const float* __restrict__ dy, const float* __restrict__ z,
                                float* __restrict__ dz, long long n) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i < n) dz[i] = dy[i] * gelu_d(z[i]);
}

// out = (acc ? out : 0) + scale x (.) y
__global__ void mul_kernel(float* __restrict__ out, const float* __restrict__ x,
                           const float* __restrict__ y, long long n, float scale, int acc) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const float v = scale * x[i] * y[i];
  out[i] = acc ? out[i] + v : v;
}

__global__ void axpy_kernel(float* __restrict__ out, const float* __restrict__ x, long long n,
                            float scale) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i < n) out[i] += scale * x[i];
}

// complex float64 (interleaved) -> 2-channel float32, scaled
__global__ void c2f_kernel(const double* __restrict__ c, float* __restrict__ out, long long n,
                           double scale) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i < 2 * n) out[i] = (float)(scale * c[i]);
}

__global__ void adam_kernel(float* __restrict__ th, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, long long n, AdamArgs A) {
  const long long i = (long long)blockIdx.x * TB + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = A.b1 * m[i] + (1.f - A.b1) * gi;
  const float vi = A.b2 * v[i] + (1.f - A.b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / A.bc1, vh = vi / A.bc2;
  th[i] -= A.lr * mh / (sqrtf(vh) + A.eps);
}

unsigned blocks(long long n) {
  long long b = (n + TB - 1) / TB;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

hipError_t launch_repack(const float* w, int d0, int d1, int taps, int transposed, int flip,
                         float scale, int cin, int cpad, float* out, hipStream_t s) {
  const long long n = (long long)taps * cin * cpad;
  const unsigned nb = blocks(n) < 4096 ? blocks(n) : 4096;
  hipLaunchKernelGGL(repack_kernel, dim3(nb), dim3(TB), 0, s, w, d0, d1, taps, transposed, flip,
                     scale, cin, cpad, out);
  return hipGetLastError();
}

long long wgrad_part_floats(const WgArgs& a) {
  const int taps = a.dim == 2 ? 9 : 27;
  return (long long)taps * a.cin * a.cout * a.nchunk;
}

hipError_t launch_wgrad(WgArgs a, hipStream_t s) {
  const int taps = a.dim == 2 ? 9 : 27;
  const long long E = (long long)taps * a.cin * a.cout;
  if (a.chunk < 1 || a.nchunk < 1 || (long long)a.nchunk * a.chunk < a.out.total)
    return hipErrorInvalidValue;
  const dim3 g(blocks(E), (unsigned)a.nchunk);
  if (a.tx == T_F64) hipLaunchKernelGGL(wgrad_partial<double>, g, dim3(TB), 0, s, a);
  else hipLaunchKernelGGL(wgrad_partial<float>, g, dim3(TB), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(wgrad_reduce, dim3(blocks(E)), dim3(TB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gelu_fwd(const float* z, float* a, long long n, hipStream_t s) {
  hipLaunchKernelGGL(gelu_fwd_kernel, dim3(blocks(n)), dim3(TB), 0, s, z, a, n);
  return hipGetLastError();
}

hipError_t launch_gelu_bwd(const float* dy, const float* z, float* dz, long long n, hipStream_t s) {
  hipLaunchKernelGGL(gelu_bwd_kernel, dim3(blocks(n)), dim3(TB), 0, s, dy, z, dz, n);
  return hipGetLastError();
}

hipError_t launch_mul(float* out, const float* x, const float* y, long long n, float scale,
                      int acc, hipStream_t s) {
  hipLaunchKernelGGL(mul_kernel, dim3(blocks(n)), dim3(TB), 0, s, out, x, y, n, scale, acc);
  return hipGetLastError();
}

hipError_t launch_axpy(float* out, const float* x, long long n, float scale, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(blocks(n)), dim3(TB), 0, s, out, x, n, scale);
  return hipGetLastError();
}

hipError_t launch_c2f(const double* c, float* out, long long n, double scale, hipStream_t s) {
  hipLaunchKernelGGL(c2f_kernel, dim3(blocks(2 * n)), dim3(TB), 0, s, c, out, n, scale);
  return hipGetLastError();
}

hipError_t launch_adam(float* th, const float* g, float* m, float* v, long long n,
                       const AdamArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks(n)), dim3(TB), 0, s, th, g, m, v, n, a);
  return hipGetLastError();
}

}  // namespace mcmg
