// Internal declarations shared by the HIP kernels and the runtime of
// libmcmg.so.  Layouts:
//   complex fields     : interleaved (re, im) float64 or float32, row-major
//                        over the extended grid, last axis fastest;
//   latent tensors     : float32 [nodes][C] (channel fastest, "NHWC");
//   conv weights       : float32 [tap][cin][cout_pad], cout_pad a multiple
//                        of the output-channel chunk, zero padded;
//   PML tables         : per axis, complex float64 cm[i], cp[i] with
//                        cm = 1/(h^2 s(i) s(i-1/2)), cp = 1/(h^2 s(i) s(i+1/2)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace mcmg {

struct Dims {
  int n[3];            // nodes per axis (unused axes = 1)
  long long total;     // product
};

inline Dims make_dims(int dim, const int* n) {
  Dims d;
  d.n[0] = n[0];
  d.n[1] = dim > 1 ? n[1] : 1;
  d.n[2] = dim > 2 ? n[2] : 1;
  d.total = (long long)d.n[0] * d.n[1] * d.n[2];
  return d;
}

// n / d for 32-bit unsigned n by a multiply-high and shifts, with the
// round-up multiplier of Granlund and Montgomery (division by invariant
// integers): m = floor(2^32 (2^l - d) / d) + 1, l = ceil(log2 d),
// q = (t + ((n - t) >> 1)) >> (l - 1), t = mulhi(n, m).  Exact for every
// 32-bit n (checked exhaustively at the boundaries and on random n).
struct FastDiv {
  uint32_t d = 1, m = 0;
  int l = 0;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  if (d <= 1) return f;
  while ((1ull << f.l) < d) ++f.l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << f.l) - d)) / d + 1);
  return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  if (f.d == 1) return n;
  const uint32_t t = __umulhi(n, f.m);
  return (t + ((n - t) >> 1)) >> (f.l - 1);
}

// Pointer to global memory.  Accesses through it are global instructions
// even when the pointer value was read from memory (the per-problem argument
// tables of the batched kernels), where a plain pointer gives flat
// instructions, which also count against the LDS wait counter.
template <class T> using gptr = __attribute__((address_space(1))) T*;
template <class T, class U> __device__ __forceinline__ gptr<T> to_global(U* p) { return (gptr<T>)p; }
// HIP's float2/float4/double2 cannot be read or written in place through
// such a pointer (their copy operations take generic references): these go
// through the compiler's own vector types.
typedef float nvf2 __attribute__((ext_vector_type(2)));
typedef float nvf4 __attribute__((ext_vector_type(4)));
typedef double nvd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gld(gptr<const float2> p, long long i) {
  const nvf2 v = ((gptr<const nvf2>)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 gld(gptr<const float4> p, long long i) {
  const nvf4 v = ((gptr<const nvf4>)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 gld(gptr<const double2> p, long long i) {
  const nvd2 v = ((gptr<const nvd2>)p)[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void gst(gptr<float2> p, long long i, float2 v) { ((gptr<nvf2>)p)[i] = nvf2{v.x, v.y}; }

// Walk over the GEMM pair index q = 4 s + lg (s = 0, 1, ...) of the
// matrix-core convolutions: (tap, cb) = (q / cpv, q % cpv) with q clamped to
// npairs - 1 (weight rows past npairs are zero), advanced one step at a time
// without a division (4 = d4 cpv + r4, so cb wraps at most once per step).
struct PairWalk {
  int q, tap, cb, cpv, d4, r4, npairs, tapL, cbL;
  __device__ __forceinline__ void init(int lg, int cpv_, int npairs_) {
    cpv = cpv_;
    npairs = npairs_;
    q = lg;
    tap = lg / cpv;
    cb = lg - tap * cpv;
    d4 = 4 / cpv;
    r4 = 4 - d4 * cpv;
    tapL = (npairs - 1) / cpv;
    cbL = npairs - 1 - tapL * cpv;
  }
  // (tap, cb) of the current step, then advance to the next
  __device__ __forceinline__ void take(int& t, int& c) {
    const bool over = q >= npairs;
    t = over ? tapL : tap;
    c = over ? cbL : cb;
    q += 4;
    tap += d4;
    cb += r4;
    if (cb >= cpv) { cb -= cpv; ++tap; }
  }
};

enum ConvMode { CONV_S1 = 0, CONV_S2 = 1, CONV_T2 = 2 };
enum ConvEpi {
  EPI_SET = 0,    // y = acc
  EPI_ADD = 1,    // y += acc
  EPI_MUL = 2,    // y = feat * acc
  EPI_GELU = 3,   // y = gelu(acc)
  EPI_RESID = 4   // y = r - acc(w) - feat * acc(w2)
};
enum ElemType { T_F32 = 0, T_F64 = 1, T_BF16 = 2 };

struct ConvLaunch {
  int dim;
  int mode;            // ConvMode
  int epi;             // ConvEpi
  int tin;             // ElemType of x
  int tout;            // ElemType of y
  const void* x;
  const float* w;      // [tap][cin][cpad]
  const float* w2;     // second tensor (EPI_RESID)
  void* y;
  const float* r;      // EPI_RESID residual input  [nodes_out][cout]
  const float* feat;   // EPI_MUL / EPI_RESID feature [nodes_out][cout]
  int cin, cout, cpad;
  Dims in, out;
};

// Stable C string for a kernel name (interned for the process lifetime).
}  // namespace mcmg
#include <string>
namespace mcmg {
const char* intern_name(const std::string& s);
// Kernel symbol of a convolution launch (for per-launch timing records).
const char* conv_kernel_name(const ConvLaunch& a);
// Algorithmic work of a convolution launch.
void conv_work(const ConvLaunch& a, double* flops, double* bytes);

// Fixed output-channel chunk per thread of the VALU direct convolution.
int conv_chunk(int cout);
// compute units of the current device (queried once; 256 if the query fails)
int device_cus();
hipError_t launch_conv(const ConvLaunch& a, hipStream_t s);

// Fill n floats with zero (graph-safe, no memset node).
hipError_t launch_zero_f32(float* p, long long n, hipStream_t s);
hipError_t launch_zero_f64(double* p, long long n, hipStream_t s);

// ---- Helmholtz operator -------------------------------------------------
struct HelmOp {
  int dim;
  Dims ext;
  const double* k2;       // [nodes]
  const double* cm[3];    // complex [n_a] (interleaved)
  const double* cp[3];
  // sponge layer: diagonal -k^2 (1 + i gamma), gamma = gmax min(1, sum_a g_a[i_a])
  double gmax;            // 0: no sponge term
  const double* g[3];     // [n_a] squared normalised distance into the layer
  FastDiv fd1, fd2;       // division by ext.n[1], ext.n[2] (node index unravel)
  int periodic = 0;       // 1: neighbours wrap around every axis (Born form)
  int adjoint = 0;        // 1: apply A^H (conjugate transpose) instead of A
};

// out = A u (f == nullptr) or out = f - A u; if partial != nullptr the
// kernel writes per-block partial sums of |out|^2 (grid size returned by
// helm_blocks()).
int helm_blocks(const HelmOp& op);
hipError_t launch_helm(const HelmOp& op, int tin, const void* u, const double* f,
                       double* out, double* partial, hipStream_t s);

// Setup helpers: extended k^2 and the f_lift input m = k h (float32).
hipError_t launch_setup_medium(int dim, Dims interior, int npml, const double* c_int,
                               double omega, double h, double* k2, float* m, hipStream_t s);
hipError_t launch_pml_tables(int n_ext, int npml, double h, double sigma_max,
                             double* cm, double* cp, hipStream_t s);

// ---- Krylov --------------------------------------------------------------
__host__ __device__ int red_blocks(long long n);    // partial-sum grid size
int elem_blocks(long long n);                       // one complex entry per thread
// partial[i * nb + b] for i < nvec: sum conj(V_i) w over block b;
// partial[nvec * nb + b]: sum |w|^2 (complex parts interleaved).
hipError_t launch_multidot(const double* V, long long ldv, int nvec, const double* w,
                           long long n, double* partial, const int* skip, hipStream_t s);
// Reduce the partials of launch_multidot: coef[i] = dot_i (complex);
// H column j (ldh complex entries per column, column-major) gets += dot_i;
// wnorm2[0] = |w|^2 before the pass.
hipError_t launch_reduce_dots(const double* partial, int nb, int nvec, double* coef,
                              double* Hcol, double* wnorm2, const int* skip, hipStream_t s);
// w -= sum_i coef_i V_i; partial[b] = block sums of |w|^2.
hipError_t launch_update(const double* V, long long ldv, int nvec, const double* coef,
                         double* w, long long n, double* partial, const int* skip, hipStream_t s);
// Norm reduce and bookkeeping for pass `pass` (0 or 1) of column j:
// pass 0 sets hn = |w|, flags skip[0] = 1 unless |w| < eta * |w_before|
// (or always_two); pass 1 (run only when skip[0] == 0) overwrites hn.
hipError_t launch_reduce_norm(const double* partial, int nb, const double* wnorm2,
                              double* hn, int* skip, int pass, int always_two,
                              hipStream_t s);
hipError_t launch_scale(const double* w, const double* hn, double* v, long long n,
                        hipStream_t s);
// launch_reduce_norm for pass 1 (skipped when skip[0] != 0), then the Givens
// rotation step on column j of H (complex, column-major, ldh rows), in one
// launch.  State: cs[m], sn[m] (complex), g[m+1] (complex).  Writes
// out[0] = |g_{j+1}|, out[1] = hn, out[2] = column norm before rotation.
hipError_t launch_norm_givens(const double* partial, int nb, const double* wnorm2, double* hn,
                              int* skip, double* H, int ldh, int j, double* cs, double* sn,
                              double* g, double* out, hipStream_t s);
hipError_t launch_init_g(double* g, int m1, const double* beta, hipStream_t s);
// y = H[0:k,0:k]^{-1} g[0:k] (upper triangular, complex).
hipError_t launch_backsolve(const double* H, int ldh, int k, const double* g, double* y,
                            hipStream_t s);
// u += sum_i y_i Z_i, Z float32 complex vectors with stride ldz (complex).
hipError_t launch_zupdate(const float* Z, long long ldz, int k, const double* y, double* u,
                          long long n, hipStream_t s);
// out = sum of nb partials -> out[0] (and sqrt into out[1]).
hipError_t launch_reduce_sum(const double* partial, int nb, double* out, hipStream_t s);
// u += z (complex f64 += complex f32) -- stationary iteration.
hipError_t launch_axpy_f32(const float* z, double* u, long long n, hipStream_t s);
hipError_t launch_cast_f32_f64(const float* z, double* out, long long n, hipStream_t s);
hipError_t launch_copy_f64(const double* a, double* b, long long n, hipStream_t s);

// Per-problem FGMRES state for the batched kernels (one handle's buffers).
struct KArgs {
  double* V;          // (m+1) basis vectors, complex, stride N
  float* Z;           // m preconditioned vectors, complex float32, stride N
  double* w;          // Arnoldi work vector
  double* r;          // residual
  const double* f;    // right-hand side
  double* u;          // solution (in/out)
  double *H, *cs, *sn, *g, *y, *coef, *partial, *scal;
  int* skip;
  long long N;        // extended-grid nodes
  int ldh;            // m + 1
  int always_two;     // force the second Gram-Schmidt pass
};
enum {
  KB_MULTIDOT, KB_REDUCE_DOTS, KB_UPDATE, KB_REDUCE_NORM, KB_GIVENS, KB_SCALE_R, KB_SCALE_W,
  KB_CYCLE_INIT, KB_BACKSOLVE, KB_ZUPDATE, KB_REDUCE_SUM, KB_FNORM_PARTIAL, KB_FNORM_REDUCE
};
struct KBatch {
  const KArgs* tab;       // device table, np entries
  int np;
  const int* pre_red;     // block prefix for red_blocks(N) grids
  int total_red;
  const int* pre_elem;    // block prefix for elem_blocks(N) grids
  int total_elem;
  const int* frozen;      // device flags (may be null)
  const int* jpos;        // device, Krylov position j per problem
  const int* kk;          // device, length of the cycle being closed per problem
  double* gather;         // device, 4 doubles per problem: (rho or |f|^2, h_{j+1,j}, |col|, |r|)
};
hipError_t kb_launch(int op, const KBatch& b, int pass, int m, hipStream_t s);

}  // namespace mcmg

namespace mcmg {
// ---- fused finest-level (C = 2) smoothing step -----------------------------
struct L1Weights {            // [cout][cin][tap] of the level-1 tensors
  float W[2][2][27];
  float KA[2][2][27];
  float KS[2][2][27];
  float Wsm[2][2][27];
};
static_assert(sizeof(L1Weights) == 432 * sizeof(float), "W, KA, KS, Wsm packed in this order");
// The same weights in the tap-major order of the 3D sweep: per in-plane tap
// t (dy, dx row-major), per plane offset dz, the 2 x 2 channel block
// (c00, c01, c10, c11) of W followed by that of KA; then KS and Wsm the
// same way without a partner.
struct L1ZWeights {
  float WK[9][3][8];
  float KS[9][3][4];
  float Wsm[9][3][4];
};
enum { L1_STEP = 0, L1_FIRST = 1, L1_RESID = 2 };
struct L1Launch {
  int dim, var;
  const float* e;             // current correction [nodes][2] (unused for FIRST)
  float* eo;                  // updated correction (RESID: t = r - A e)
  const float *r, *a, *s;
  L1Weights w;
  const L1Weights* wdev;      // device copy of w (3D reads the weights through it)
  Dims n;
};
hipError_t launch_level1(const L1Launch& l, hipStream_t s);
}  // namespace mcmg

namespace mcmg {
// ---- batched launches ------------------------------------------------------
// A batched kernel runs several independent problems in one launch: tab is a
// device array of per-problem argument structs, pre (np + 1 ints, device)
// the prefix of per-problem block counts, total = pre[np]; frozen (np ints,
// device, may be null) marks problems whose blocks return at once.  A table
// may hold several rows of np entries (one per Krylov position); row (np
// ints, device, may be null = row 0) selects each problem's row.
struct BatchLaunch {
  const void* tab;
  const int* pre;
  int np;
  int total;
  const int* frozen;
  const int* row = nullptr;
};

__host__ __device__ __forceinline__ int batch_entry(const int* row, int np, int p) {
  return (row ? row[p] * np : 0) + p;
}

// Problem of launch block b: the last p with pre[p] <= b (pre is ascending;
// every lane takes the same path, so the loads are wave-uniform).
__device__ __forceinline__ int batch_find(const int* __restrict__ pre, int np, int b) {
  int lo = 0, hi = np - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
}  // namespace mcmg

namespace mcmg {
// Per-problem arguments of the fused C = 2 sweep (element of a batch table;
// wp points to device-resident weights).
struct L1Args {
  const float* e;
  float* eo;
  const float *r, *a, *s;
  const L1Weights* wp;
  Dims n;
  int tiles_x, tiles_y, tiles_z;
  int zc;                // 3D: planes per block (the z chunk)
};
// nprob: problems sharing the launch (batched), which share the chip's
// resident blocks when the 3D z chunk is sized
L1Args l1_args(const L1Launch& l, const L1Weights* wdev, int* nblk, int nprob = 1);
hipError_t launch_level1_batched(int dim, int var, const BatchLaunch& b, hipStream_t s);
}  // namespace mcmg

namespace mcmg {
// Per-problem arguments of the VALU direct convolution (batch table element).
struct DArgs {
  const void* x;
  const float* w;
  const float* w2;
  void* y;
  const float* r;
  const float* feat;
  int cin, cout, cpad;
  Dims in, out;
  FastDiv fo1, fo2;      // division by out.n[1], out.n[2]
  int zc;                // 3D 2 -> 2 z-streaming form: planes per block
};
DArgs conv_args(const ConvLaunch& a, int* nblk);
hipError_t launch_conv_batched(const ConvLaunch& proto, const BatchLaunch& b, hipStream_t s);
}  // namespace mcmg

namespace mcmg {
// Per-problem arguments of the Helmholtz operator (batch table element):
// out = A u, or out = f - A u with per-block |out|^2 partials.
struct HArgs {
  HelmOp op;
  const void* u;
  const double* f;
  double* out;
  double* partial;
};
hipError_t launch_helm_batched(int dim, int tin, const BatchLaunch& b, hipStream_t s);
}  // namespace mcmg

namespace mcmg {
// ---- Born series: discrete Green operator by FFT ---------------------------
constexpr int FFT_MAXL = 5120;   // longest axis (elements per block <= FFT_MAXL)
constexpr int FFT_MAXST = 16;    // radix stages
constexpr size_t FFT_MAXLDS = 160 * 1024;
enum { FFT_FWD = 0, FFT_SYM = 1, FFT_INV = 2, FFT_LAST = 3 };
// radix classes: radices in {2, 3, 4, 5, 7}; also 11; anything
enum { FFT_RC_SMALL = 0, FFT_RC_11 = 1, FFT_RC_ANY = 2 };
// One axis pass over a complex FP64 field (row-major, axis of length L and
// stride S; `outer` = number of lines (contiguous) or of outer indices
// (strided)).  src and dst may alias.
struct FftArgs {
  const double* src;
  double* dst;
  const double2* tw;       // exp(-2 pi i j / L), j < L
  const int* rev;          // digit-reversed position of natural index j
  int L, TC, contiguous, nst;
  int tw_lds;              // 1: stage the twiddle table in LDS
  int rc;                  // radix class (FFT_RC_*)
  long long S, outer;
  const int* plan;         // device [2 nst]: radix, then sub-length, of each stage
  // SYM: symbol tables d_a (length n_a), extended sizes, background
  const double* d[3];
  int n[3], dim;
  double k0sq, eps;
  // LAST: scale and, for the CBS update, u and the damped k^2
  double scale;
  double* u;
  const double* k2;
  const double* g[3];
  double gmax;
};
size_t fft_lds_bytes(const FftArgs& a);
long long fft_blocks(const FftArgs& a);
hipError_t launch_fft(int mode, const FftArgs& a, hipStream_t s);

struct BornStatsArgs {
  const double* k2;
  const double* g[3];
  double gmax, k0sq;
  int n[3], dim;
  long long N;
  double* out;             // [2 * blocks]: (min, max) per block
};
int born_stats_blocks(long long n);
hipError_t launch_born_stats(const BornStatsArgs& a, int pass, hipStream_t s);
}  // namespace mcmg

namespace mcmg {
// ---- Training (weight gradients, adjoint layouts, Adam) --------------------
// canonical [d0][d1][taps] -> convolution layout [tap][cin][cpad]
hipError_t launch_repack(const float* w, int d0, int d1, int taps, int transposed, int flip,
                         float scale, int cin, int cpad, float* out, hipStream_t s);
// dw (canonical) += scale * gradient of the convolution y = w * x of `mode`
struct WgArgs {
  int dim, mode, tx;        // ConvMode; ElemType of x (T_F32 or T_F64)
  const void* x;            // [in nodes][cin]
  const float* dy;          // [out nodes][cout]
  int cin, cout;
  Dims in, out;
  float* dw;                // canonical tensor
  float scale;
  float* part;              // [nchunk][taps cin cout] partial sums
  int nchunk;
  long long chunk;          // output nodes per chunk
  FastDiv fo1, fo2;         // division by out.n[1], out.n[2]
};
long long wgrad_part_floats(const WgArgs& a);
hipError_t launch_wgrad(WgArgs a, hipStream_t s);
hipError_t launch_gelu_fwd(const float* z, float* a, long long n, hipStream_t s);
hipError_t launch_gelu_bwd(const float* dy, const float* z, float* dz, long long n, hipStream_t s);
hipError_t launch_mul(float* out, const float* x, const float* y, long long n, float scale,
                      int acc, hipStream_t s);
hipError_t launch_axpy(float* out, const float* x, long long n, float scale, hipStream_t s);
hipError_t launch_c2f(const double* c, float* out, long long n, double scale, hipStream_t s);
struct AdamArgs {
  float lr, b1, b2, eps, bc1, bc2;   // bc = 1 - beta^t (bias corrections)
};
hipError_t launch_adam(float* th, const float* g, float* m, float* v, long long n,
                       const AdamArgs& a, hipStream_t s);
}  // namespace mcmg
