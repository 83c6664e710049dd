// Helmholtz operator with an absorbing layer in FP64 (Sec. 2.1 Eq.
// FDM_stencil and the sponge equation, App. A.1.1 PML) and the setup kernels
// that build its coefficients.
//
// (A u)_I = sum_a [ (cm_a + cp_a) u_I - cm_a u_{I-e_a} - cp_a u_{I+e_a} ]
//           - k_I^2 (1 + i gamma_I) u_I
// with cm_a = 1/(h^2 s_a(I) s_a(I-1/2)), cp_a = 1/(h^2 s_a(I) s_a(I+1/2))
// (divergence form of the stretched Laplacian; Dirichlet zero outside the
// extended grid, or periodic wrap-around for the Born form; the adjoint form
// applies A^H for the training gradient).  PML: gamma = 0;
// sponge: s = 1 and gamma = gmax min(1, sum_a g_a[I_a]) from per-axis tables.
// Per node it streams u (16 B), k^2 (8 B) and the output (16 B); the
// residual form also reads f (16 B) and emits block partial sums of
// |f - A u|^2 for the FP64 norm.
#include "internal.h"

namespace mcmg {

namespace {

struct cplx { double re, im; };
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx ld(const double* p, long long i) { return {p[2 * i], p[2 * i + 1]}; }
__device__ __forceinline__ cplx ld(const float* p, long long i) {
  return {(double)p[2 * i], (double)p[2 * i + 1]};
}

constexpr int HB = 256;          // threads per block
constexpr int HPT = 4;           // nodes per thread (grid-stride within block span)

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  }
  __syncthreads();
  return t;
}

template <int D, typename TIN>
__device__ __forceinline__ void helm_body(const HArgs& A, const int vblk) {
  const TIN* __restrict__ u = reinterpret_cast<const TIN*>(A.u);
  const double* __restrict__ f = A.f;
  double* __restrict__ out = A.out;
  const double* __restrict__ k2 = A.op.k2;
  const double* __restrict__ cm0 = A.op.cm[0];
  const double* __restrict__ cp0 = A.op.cp[0];
  const double* __restrict__ cm1 = A.op.cm[1];
  const double* __restrict__ cp1 = A.op.cp[1];
  const double* __restrict__ cm2 = A.op.cm[2] ? A.op.cm[2] : A.op.cm[0];
  const double* __restrict__ cp2 = A.op.cp[2] ? A.op.cp[2] : A.op.cp[0];
  const Dims n = A.op.ext;
  double* __restrict__ partial = A.partial;
  __shared__ double sh[HB / 64];
  double nrm = 0.0;
  const long long base = (long long)vblk * HB * HPT;
  for (int q = 0; q < HPT; ++q) {
    const long long p = base + (long long)q * HB + threadIdx.x;
    if (p >= n.total) break;
    int i[3];
    {
      long long t = p;
      i[2] = (int)(t % n.n[2]); t /= n.n[2];
      i[1] = (int)(t % n.n[1]); t /= n.n[1];
      i[0] = (int)t;
    }
    cplx uc = ld(u, p);
    if (A.op.adjoint) uc.im = -uc.im;
    const double kk = k2[p];
    cplx acc = {-kk * uc.re, -kk * uc.im};
    if (A.op.gmax != 0.0) {
      double gs = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) gs += A.op.g[a][i[a]];
      const double gk = kk * A.op.gmax * (gs < 1.0 ? gs : 1.0);
      // -k^2 (1 + i gamma) u: the damping part is -i k^2 gamma u
      acc.re += gk * uc.im;
      acc.im -= gk * uc.re;
    }
    const long long stride[3] = {(long long)n.n[1] * n.n[2], (long long)n.n[2], 1};
    const double* cms[3] = {cm0, cm1, cm2};
    const double* cps[3] = {cp0, cp1, cp2};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      // spatial axis a of the D used ones; unused axes have n = 1 and come last
      const int ax = (D == 2) ? a : a;
      const cplx m = ld(cms[ax], i[ax]);
      const cplx pc = ld(cps[ax], i[ax]);
      const cplx d = {m.re + pc.re, m.im + pc.im};
      cplx um = {0.0, 0.0}, up = {0.0, 0.0};
      const long long wrap = (long long)(n.n[ax] - 1) * stride[ax];
      if (i[ax] > 0) um = ld(u, p - stride[ax]);
      else if (A.op.periodic) um = ld(u, p + wrap);
      if (i[ax] < n.n[ax] - 1) up = ld(u, p + stride[ax]);
      else if (A.op.periodic) up = ld(u, p - wrap);
      cplx cmw = m, cpw = pc;
      if (A.op.adjoint) {
        // row I of A^T: the coupling to I - e_a is A[I-e_a][I] = -cp_a(i - 1),
        // to I + e_a it is A[I+e_a][I] = -cm_a(i + 1); input conjugated
        um.im = -um.im;
        up.im = -up.im;
        cmw = i[ax] > 0 ? ld(cps[ax], i[ax] - 1) : cplx{0.0, 0.0};
        cpw = i[ax] < n.n[ax] - 1 ? ld(cms[ax], i[ax] + 1) : cplx{0.0, 0.0};
      }
      const cplx t0 = cmul(d, uc), t1 = cmul(cmw, um), t2 = cmul(cpw, up);
      acc.re += t0.re - t1.re - t2.re;
      acc.im += t0.im - t1.im - t2.im;
    }
    if (A.op.adjoint) acc.im = -acc.im;   // A^H v = conj(A^T conj(v))
    if (f) {
      const cplx fc = ld(f, p);
      acc.re = fc.re - acc.re;
      acc.im = fc.im - acc.im;
    }
    out[2 * p] = acc.re;
    out[2 * p + 1] = acc.im;
    nrm += acc.re * acc.re + acc.im * acc.im;
  }
  if (partial) {
    const double t = block_sum(nrm, sh);
    if (threadIdx.x == 0) partial[vblk] = t;
  }
}

// Logical block t covers nodes [t HB HPT, (t + 1) HB HPT) and writes
// partial[t]; physical blocks take logical ones in XCD-contiguous bands
// (blockIdx % 8 walks one band), so the neighbour planes a block reads sit in
// its own XCD's L2.  The grid is nb rounded up to a multiple of 8.
template <int D, typename TIN>
__global__ __launch_bounds__(HB) void helm_kernel(HArgs A, int nb) {
  const int per = (nb + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= nb) return;
  helm_body<D, TIN>(A, t);
}

template <int D, typename TIN>
__global__ __launch_bounds__(HB) void helm_kernel_batched(const HArgs* __restrict__ tab,
                                                          const int* __restrict__ pre, int np,
                                                          const int* __restrict__ frozen,
    const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const HArgs A = tab[batch_entry(row, np, p)];
  helm_body<D, TIN>(A, blockIdx.x - pre[p]);
}

hipError_t helm_dispatch(int dim, int tin, const HArgs* A, int nb, const BatchLaunch* b,
                         hipStream_t s) {
  // 2D grids use axes 0,1 (axis 2 has n = 1); the kernel indexes axis 2 as
  // the fastest, so 2D data is addressed as n0 x n1 x 1.
  if (b) {
    const HArgs* t = (const HArgs*)b->tab;
    if (dim == 2 && tin == T_F64) hipLaunchKernelGGL((helm_kernel_batched<2, double>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
    else if (dim == 2) hipLaunchKernelGGL((helm_kernel_batched<2, float>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
    else if (tin == T_F64) hipLaunchKernelGGL((helm_kernel_batched<3, double>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
    else hipLaunchKernelGGL((helm_kernel_batched<3, float>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
  } else {
    const unsigned g = (unsigned)((nb + 7) / 8 * 8);
    if (dim == 2 && tin == T_F64) hipLaunchKernelGGL((helm_kernel<2, double>), dim3(g), dim3(HB), 0, s, *A, nb);
    else if (dim == 2) hipLaunchKernelGGL((helm_kernel<2, float>), dim3(g), dim3(HB), 0, s, *A, nb);
    else if (tin == T_F64) hipLaunchKernelGGL((helm_kernel<3, double>), dim3(g), dim3(HB), 0, s, *A, nb);
    else hipLaunchKernelGGL((helm_kernel<3, float>), dim3(g), dim3(HB), 0, s, *A, nb);
  }
  return hipGetLastError();
}

}  // namespace

int helm_blocks(const HelmOp& op) {
  return (int)((op.ext.total + (long long)HB * HPT - 1) / ((long long)HB * HPT));
}

hipError_t launch_helm(const HelmOp& op, int tin, const void* u, const double* f, double* out,
                       double* partial, hipStream_t s) {
  HArgs A{op, u, f, out, partial};
  return helm_dispatch(op.dim, tin, &A, helm_blocks(op), nullptr, s);
}

hipError_t launch_helm_batched(int dim, int tin, const BatchLaunch& b, hipStream_t s) {
  if (b.np == 0 || b.total == 0) return hipSuccess;
  return helm_dispatch(dim, tin, nullptr, 0, &b, s);
}

// ---- setup --------------------------------------------------------------

namespace {

__global__ void setup_medium_kernel(int dim, Dims interior, Dims ext, int npml,
                                    const double* __restrict__ c, double omega, double h,
                                    double* __restrict__ k2, float* __restrict__ m) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ext.total) return;
  long long t = p;
  int I[3];
  I[2] = (int)(t % ext.n[2]); t /= ext.n[2];
  I[1] = (int)(t % ext.n[1]); t /= ext.n[1];
  I[0] = (int)t;
  int i[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= dim) { i[a] = 0; continue; }
    int v = I[a] - npml;                       // edge replication into the layer
    v = v < 0 ? 0 : (v >= interior.n[a] ? interior.n[a] - 1 : v);
    i[a] = v;
  }
  const double cv = c[((long long)i[0] * interior.n[1] + i[1]) * interior.n[2] + i[2]];
  const double k = omega / cv;
  k2[p] = k * k;
  m[p] = (float)(k * h);
}

__device__ __forceinline__ double sigma_at(double x, int npml, int n_int, double smax) {
  const double lo = npml, hi = npml + n_int - 1;
  double d = lo - x;
  if (x - hi > d) d = x - hi;
  if (d < 0.0) d = 0.0;
  if (npml == 0) return 0.0;
  const double r = d / npml;
  return smax * r * r;
}

__device__ __forceinline__ cplx cinv(cplx a) {
  const double q = a.re * a.re + a.im * a.im;
  return {a.re / q, -a.im / q};
}

__global__ void pml_kernel(int n_ext, int npml, double h, double smax, double* cm, double* cp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_ext) return;
  const int n_int = n_ext - 2 * npml;
  const cplx s = {1.0, sigma_at((double)i, npml, n_int, smax)};
  const cplx sl = {1.0, sigma_at(i - 0.5, npml, n_int, smax)};
  const cplx sr = {1.0, sigma_at(i + 0.5, npml, n_int, smax)};
  const double ih2 = 1.0 / (h * h);
  const cplx a = cinv(cmul(s, sl)), b = cinv(cmul(s, sr));
  cm[2 * i] = a.re * ih2; cm[2 * i + 1] = a.im * ih2;
  cp[2 * i] = b.re * ih2; cp[2 * i + 1] = b.im * ih2;
}

}  // namespace

hipError_t launch_setup_medium(int dim, Dims interior, int npml, const double* c_int,
                               double omega, double h, double* k2, float* m, hipStream_t s) {
  int ne[3] = {interior.n[0] + 2 * npml, dim > 1 ? interior.n[1] + 2 * npml : 1,
               dim > 2 ? interior.n[2] + 2 * npml : 1};
  Dims ext = make_dims(dim, ne);
  hipLaunchKernelGGL(setup_medium_kernel, dim3((unsigned)((ext.total + 255) / 256)), dim3(256), 0,
                     s, dim, interior, ext, npml, c_int, omega, h, k2, m);
  return hipGetLastError();
}

hipError_t launch_pml_tables(int n_ext, int npml, double h, double sigma_max, double* cm,
                             double* cp, hipStream_t s) {
  hipLaunchKernelGGL(pml_kernel, dim3((n_ext + 255) / 256), dim3(256), 0, s, n_ext, npml, h,
                     sigma_max, cm, cp);
  return hipGetLastError();
}

}  // namespace mcmg
