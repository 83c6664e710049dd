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

// Complex values as one vector load (16 B for double, 8 B for float).
__device__ __forceinline__ cplx ldv(const double* p, long long i) {
  const double2 v = gld(to_global<const double2>(p), i);
  return {v.x, v.y};
}
__device__ __forceinline__ cplx ldv(const float* p, long long i) {
  const float2 v = gld(to_global<const float2>(p), i);
  return {(double)v.x, (double)v.y};
}

// The operator at one node from its value, the damping sum, the per-axis
// coefficients and the neighbours (axis order 0, 1, 2).  Every kernel that
// applies A calls it, and it rounds every product and sum separately, so the
// block-linear and the z-marching forms give the same bits.
template <int D>
__device__ __forceinline__ cplx node_op(const cplx uc, const double kk, const double gs,
                                        const double gmax, const cplx* m, const cplx* pc,
                                        const cplx* cmw, const cplx* cpw, const cplx* um,
                                        const cplx* up) {
  // no multiply-add contraction: where the compiler would fuse depends on
  // the surrounding kernel, and both kernels must round the same operations
#pragma clang fp contract(off)
  cplx acc = {-kk * uc.re, -kk * uc.im};
  if (gmax != 0.0) {
    const double gk = kk * gmax * (gs < 1.0 ? gs : 1.0);
    // -k^2 (1 + i gamma) u: the damping part is -i k^2 gamma u
    acc.re += gk * uc.im;
    acc.im -= gk * uc.re;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const cplx d = {m[a].re + pc[a].re, m[a].im + pc[a].im};
    // t0 = d uc, t1 = cmw um, t2 = cpw up, written out so that the pragma
    // above covers every operation
    const double t0r = d.re * uc.re - d.im * uc.im, t0i = d.re * uc.im + d.im * uc.re;
    const double t1r = cmw[a].re * um[a].re - cmw[a].im * um[a].im;
    const double t1i = cmw[a].re * um[a].im + cmw[a].im * um[a].re;
    const double t2r = cpw[a].re * up[a].re - cpw[a].im * up[a].im;
    const double t2i = cpw[a].re * up[a].im + cpw[a].im * up[a].re;
    acc.re += t0r - t1r - t2r;
    acc.im += t0i - t1i - t2i;
  }
  return acc;
}

// MODE 0: A u (Dirichlet); 1: periodic (Born form); 2: A^H u (Dirichlet).
// Neighbour loads use clamped addresses and a mask instead of branches.
template <int D, typename TIN, int MODE>
__device__ __forceinline__ void helm_body(const HArgs& A, const int vblk) {
  const TIN* __restrict__ u = reinterpret_cast<const TIN*>(A.u);
  const double* __restrict__ f = A.f;
  const gptr<double> __restrict__ out = to_global<double>(A.out);
  const gptr<const double> __restrict__ k2 = to_global<const double>(A.op.k2);
  const Dims n = A.op.ext;
  const gptr<double> __restrict__ partial = to_global<double>(A.partial);
  __shared__ double sh[HB / 64];
  double nrm = 0.0;
  const long long base = (long long)vblk * HB * HPT;
  const long long stride[3] = {(long long)n.n[1] * n.n[2], (long long)n.n[2], 1};
  const bool small = n.total < (1LL << 31);
  for (int q = 0; q < HPT; ++q) {
    const long long p = base + (long long)q * HB + threadIdx.x;
    if (p >= n.total) break;
    int i[3];
    if (small) {
      // 32-bit unravel by multiply-high division (no 64-bit divide)
      const uint32_t pp = (uint32_t)p;
      const uint32_t q2 = fdiv(pp, A.op.fd2);
      const uint32_t q1 = fdiv(q2, A.op.fd1);
      i[2] = (int)(pp - q2 * (uint32_t)n.n[2]);
      i[1] = (int)(q2 - q1 * (uint32_t)n.n[1]);
      i[0] = (int)q1;
    } else {
      long long t = p;
      i[2] = (int)(t % n.n[2]); t /= n.n[2];
      i[1] = (int)(t % n.n[1]); t /= n.n[1];
      i[0] = (int)t;
    }
    cplx uc = ldv(u, p);
    if (MODE == 2) uc.im = -uc.im;
    const double kk = k2[p];
    double gs = 0.0;
    if (A.op.gmax != 0.0) {
#pragma unroll
      for (int a = 0; a < D; ++a) gs += to_global<const double>(A.op.g[a])[i[a]];
    }
    cplx m[D], pc[D], cmw[D], cpw[D], um[D], up[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int ia = i[a], na = n.n[a];
      const bool hm = ia > 0, hp = ia < na - 1;
      m[a] = ldv(A.op.cm[a], ia);
      pc[a] = ldv(A.op.cp[a], ia);
      const long long wrap = (long long)(na - 1) * stride[a];
      long long pm, pq;
      if (MODE == 1) {
        pm = hm ? p - stride[a] : p + wrap;
        pq = hp ? p + stride[a] : p - wrap;
      } else {
        pm = hm ? p - stride[a] : p;
        pq = hp ? p + stride[a] : p;
      }
      um[a] = ldv(u, pm);
      up[a] = ldv(u, pq);
      cmw[a] = m[a];
      cpw[a] = pc[a];
      if (MODE != 1) {
        if (!hm) um[a] = {0.0, 0.0};
        if (!hp) up[a] = {0.0, 0.0};
      }
      if (MODE == 2) {
        // row I of A^T: the coupling to I - e_a is A[I-e_a][I] = -cp_a(i - 1),
        // to I + e_a it is A[I+e_a][I] = -cm_a(i + 1); input conjugated
        um[a].im = -um[a].im;
        up[a].im = -up[a].im;
        cmw[a] = ldv(A.op.cp[a], hm ? ia - 1 : ia);
        cpw[a] = ldv(A.op.cm[a], hp ? ia + 1 : ia);
      }
    }
    cplx acc = node_op<D>(uc, kk, gs, A.op.gmax, m, pc, cmw, cpw, um, up);
    if (MODE == 2) acc.im = -acc.im;   // A^H v = conj(A^T conj(v))
    if (f) {
      const cplx fc = ldv(f, p);
      acc.re = fc.re - acc.re;
      acc.im = fc.im - acc.im;
    }
    ((gptr<nvd2>)out)[p] = nvd2{acc.re, acc.im};
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
template <int D, typename TIN, int MODE>
__global__ __launch_bounds__(HB) void helm_kernel(HArgs A, int nb) {
  const int per = (nb + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= nb) return;
  helm_body<D, TIN, MODE>(A, t);
}

// 3D plain A u without the residual form: a block owns MC consecutive
// columns of the flattened (y, x) plane (no thread falls outside the grid at
// the x edge: 64 x 4 tiles left 16% idle at 216 nodes per row) and walks MZ
// planes in z.  Each thread keeps u at z - 1, z and z + 1 in registers, so
// the z neighbours and the z coefficients are read once per plane; its x
// and y coefficients are loaded once.  The loads of the next plane (u two
// planes ahead, the four in-plane neighbours, k^2) are issued before the
// current plane is computed, so their latency overlaps the work.  Six loads
// per node instead of fourteen; node_op gives the same bits as the
// block-linear kernel.  8-plane chunks (about 2.5 rounds of resident
// blocks at 216^3) beat 16 (1.25 rounds: 97 vs 100 us) and 4 (104 us).
constexpr int MC = 256, MZ = 8;

int march_tiles(const Dims& n) {
  const long long plane = (long long)n.n[1] * n.n[2];
  return (int)((plane + MC - 1) / MC) * ((n.n[0] + MZ - 1) / MZ);
}

template <typename TIN>
__global__ __launch_bounds__(MC) void helm_march_kernel(HArgs A, int ntiles) {
  const TIN* __restrict__ u = reinterpret_cast<const TIN*>(A.u);
  const gptr<double> __restrict__ out = to_global<double>(A.out);
  const gptr<const double> __restrict__ k2 = to_global<const double>(A.op.k2);
  const int NZ = A.op.ext.n[0], NY = A.op.ext.n[1], NX = A.op.ext.n[2];
  const int per = (ntiles + 7) / 8;
  const int tl = (blockIdx.x % 8) * per + blockIdx.x / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const long long plane = (long long)NY * NX;
  const int tc = (int)((plane + MC - 1) / MC);
  const int z0 = (tl / tc) * MZ;
  const long long col = (long long)(tl % tc) * MC + threadIdx.x;
  if (col >= plane) return;   // no barriers below
  const int gy = (int)(col / NX), gx = (int)(col - (long long)gy * NX);
  const int ze = min(z0 + MZ, NZ);
  const bool hxm = gx > 0, hxp = gx < NX - 1, hym = gy > 0, hyp = gy < NY - 1;
  const long long oxm = hxm ? -1 : 0, oxp = hxp ? 1 : 0;
  const long long oym = hym ? -(long long)NX : 0, oyp = hyp ? (long long)NX : 0;
  const cplx zero = {0.0, 0.0};
  const cplx m1 = ldv(A.op.cm[1], gy), p1 = ldv(A.op.cp[1], gy);
  const cplx m2 = ldv(A.op.cm[2], gx), p2 = ldv(A.op.cp[2], gx);
  const bool sp = A.op.gmax != 0.0;
  const double g1 = sp ? to_global<const double>(A.op.g[1])[gy] : 0.0, g2 = sp ? to_global<const double>(A.op.g[2])[gx] : 0.0;
  // in-plane neighbours of plane z: y-1, y+1, x-1, x+1 (zero outside the grid)
  auto nbrs = [&](int z, cplx* nb) {
    const long long c = (long long)z * plane + col;
    nb[0] = ldv(u, c + oym);
    nb[1] = ldv(u, c + oyp);
    nb[2] = ldv(u, c + oxm);
    nb[3] = ldv(u, c + oxp);
    if (!hym) nb[0] = zero;
    if (!hyp) nb[1] = zero;
    if (!hxm) nb[2] = zero;
    if (!hxp) nb[3] = zero;
  };
  cplx ucm = z0 > 0 ? ldv(u, (long long)(z0 - 1) * plane + col) : zero;
  cplx uc = ldv(u, (long long)z0 * plane + col);
  cplx ucp = z0 + 1 < NZ ? ldv(u, (long long)(z0 + 1) * plane + col) : zero;
  cplx nb[4];
  nbrs(z0, nb);
  double kk = k2[(long long)z0 * plane + col];
  // the z coefficients of the plane (requested with the plane's other
  // operands, one plane ahead)
  const gptr<const double> g0 = sp ? to_global<const double>(A.op.g[0]) : k2;
  cplx mz = ldv(A.op.cm[0], z0), pz = ldv(A.op.cp[0], z0);
  double gz = g0[sp ? z0 : 0];
  for (int z = z0; z < ze; ++z) {
    // next plane's operands, in flight while this plane is computed: the
    // loads are unconditional (plane indices clamped, the last step re-reads
    // its own plane, u beyond the grid replaced by zero afterwards), so no
    // branch makes the compiler wait for them before the products
    const int zn = z + 1 < ze ? z + 1 : z;
    const int z2 = z + 2 < NZ ? z + 2 : NZ - 1;
    cplx ucp2 = ldv(u, (long long)z2 * plane + col);
    if (z + 2 >= NZ) ucp2 = zero;
    cplx nb2[4];
    nbrs(zn, nb2);
    const double kk2 = k2[(long long)zn * plane + col];
    const cplx mz2 = ldv(A.op.cm[0], zn), pz2 = ldv(A.op.cp[0], zn);
    const double gz2 = g0[sp ? zn : 0];
    cplx m[3], pc[3], um[3], up[3];
    m[0] = mz;
    pc[0] = pz;
    m[1] = m1; pc[1] = p1; m[2] = m2; pc[2] = p2;
    um[0] = ucm; up[0] = ucp;
    um[1] = nb[0]; up[1] = nb[1];
    um[2] = nb[2]; up[2] = nb[3];
    double gs = 0.0;
    if (sp) {
      gs += gz;
      gs += g1;
      gs += g2;
    }
    const cplx acc = node_op<3>(uc, kk, gs, A.op.gmax, m, pc, m, pc, um, up);
    ((gptr<nvd2>)out)[(long long)z * plane + col] = nvd2{acc.re, acc.im};
    ucm = uc; uc = ucp; ucp = ucp2;
    nb[0] = nb2[0]; nb[1] = nb2[1]; nb[2] = nb2[2]; nb[3] = nb2[3];
    kk = kk2;
    mz = mz2; pz = pz2; gz = gz2;
  }
}

template <int D, typename TIN>
__global__ __launch_bounds__(HB) void helm_kernel_batched(const HArgs* __restrict__ tab,
                                                          const int* __restrict__ pre, int np,
                                                          const int* __restrict__ frozen,
    const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const HArgs A = tab[batch_entry(row, np, p)];
  helm_body<D, TIN, 0>(A, blockIdx.x - pre[p]);
}

hipError_t helm_dispatch(int dim, int tin, const HArgs* A, int nb, const BatchLaunch* b,
                         hipStream_t s) {
  // 2D grids use axes 0,1 (axis 2 has n = 1); the kernel indexes axis 2 as
  // the fastest, so 2D data is addressed as n0 x n1 x 1.
  if (b) {
    // batched launches apply the plain operator (the FGMRES matvec and residual)
    const HArgs* t = (const HArgs*)b->tab;
    if (dim == 2 && tin == T_F64) hipLaunchKernelGGL((helm_kernel_batched<2, double>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
    else if (dim == 2) hipLaunchKernelGGL((helm_kernel_batched<2, float>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
    else if (tin == T_F64) hipLaunchKernelGGL((helm_kernel_batched<3, double>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
    else hipLaunchKernelGGL((helm_kernel_batched<3, float>), dim3(b->total), dim3(HB), 0, s, t, b->pre, b->np, b->frozen, b->row);
  } else {
    const int mode = A->op.adjoint ? 2 : A->op.periodic ? 1 : 0;
    if (dim == 3 && mode == 0 && !A->f && !A->partial) {
      const int nt = march_tiles(A->op.ext);
      const unsigned gm = (unsigned)((nt + 7) / 8 * 8);
      if (tin == T_F64) hipLaunchKernelGGL((helm_march_kernel<double>), dim3(gm), dim3(MC), 0, s, *A, nt);
      else hipLaunchKernelGGL((helm_march_kernel<float>), dim3(gm), dim3(MC), 0, s, *A, nt);
      return hipGetLastError();
    }
    const unsigned g = (unsigned)((nb + 7) / 8 * 8);
#define HELM_LAUNCH(DD, TT, MM) hipLaunchKernelGGL((helm_kernel<DD, TT, MM>), dim3(g), dim3(HB), 0, s, *A, nb)
#define HELM_BY_MODE(DD, TT)            \
    if (mode == 0) HELM_LAUNCH(DD, TT, 0); \
    else if (mode == 1) HELM_LAUNCH(DD, TT, 1); \
    else HELM_LAUNCH(DD, TT, 2);
    if (dim == 2 && tin == T_F64) { HELM_BY_MODE(2, double) }
    else if (dim == 2) { HELM_BY_MODE(2, float) }
    else if (tin == T_F64) { HELM_BY_MODE(3, double) }
    else { HELM_BY_MODE(3, float) }
#undef HELM_BY_MODE
#undef HELM_LAUNCH
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
