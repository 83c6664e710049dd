// Host side of the Born-series path (appendix on the Born-series variant,
// appendix on the discrete Green operator).
//
// The Born solvers act on the periodic operator A_per = -Lap_h^per -
// k^2 (1 + i gamma) of the extended grid, which the FFT diagonalises
// exactly.  They therefore need a sponge layer or no layer at all: a PML
// stretches the Laplacian.
//
// Background (the CBS parameters of the baseline-configuration appendix):
//   k0^2 = (min k^2 + max k^2) / 2,
//   eps  = max |k^2 (1 + i gamma) - k0^2|,
// both found by device reductions; a caller may fix either.  Per axis, the
// host builds the radix list and the digit-reversal, twiddle and symbol
// tables once.  G then runs as one FFT pass per axis on the handle's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.h"
#include "mcmg.h"
#include "runtime.h"

namespace mcmg {

namespace {

// Radices of n in stage order: fours, at most one two, then odd primes.
std::vector<int> radices(int n) {
  std::vector<int> r;
  while (n % 4 == 0) { r.push_back(4); n /= 4; }
  if (n % 2 == 0) { r.push_back(2); n /= 2; }
  for (int p = 3; (long long)p * p <= n; p += 2)
    while (n % p == 0) { r.push_back(p); n /= p; }
  if (n > 1) r.push_back(n);
  return r;
}

// Position in LDS of natural index j for the decimation-in-time stages:
// the last stage's radix p splits j = t + p j' and puts the sub-transform of
// residue t at offset t (n / p); recursively for j'.
std::vector<int> digit_reversal(int n, const std::vector<int>& rad) {
  std::vector<int> rev(n);
  for (int j = 0; j < n; ++j) {
    int jj = j, mm = n, pos = 0;
    for (int s = (int)rad.size() - 1; s >= 0; --s) {
      const int p = rad[s];
      mm /= p;
      pos += (jj % p) * mm;
      jj /= p;
    }
    rev[j] = pos;
  }
  return rev;
}

template <class T>
hipError_t upload(Ctx* c, const std::vector<T>& v, T** dst) {
  *dst = (T*)c->alloc(v.size() * sizeof(T));
  if (!*dst) return hipErrorOutOfMemory;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

mcmg_status Ctx::born_setup(double k0sq_in, double eps_in) {
  if (absorber != MCMG_ABL_SPONGE && npml != 0)
    return fail(MCMG_E_ARG, "the Born form needs the sponge layer or no absorbing layer "
                            "(a PML stretches the Laplacian)");
  for (int a = 0; a < dim; ++a)
    if (next[a] < 2 || next[a] > FFT_MAXL)
      return fail(MCMG_E_ARG, "Born form: extended side %d outside [2, %d]", next[a], FFT_MAXL);
  hipError_t e;
  if (!born.ax[0].tw) {
    for (int a = 0; a < dim; ++a) {
      BornAxis& X = born.ax[a];
      X.n = next[a];
      X.rad = radices(X.n);
      if ((int)X.rad.size() > FFT_MAXST) return fail(MCMG_E_ARG, "Born form: too many FFT stages");
      std::vector<double2> tw(X.n);
      std::vector<double> d(X.n);
      for (int j = 0; j < X.n; ++j) {
        const double ang = 2.0 * M_PI * (double)j / (double)X.n;
        tw[j] = make_double2(std::cos(ang), -std::sin(ang));
        const double sn = std::sin(M_PI * (double)j / (double)X.n);
        d[j] = 4.0 / (h * h) * sn * sn;
      }
      std::vector<int> plan(2 * X.rad.size());
      int ml = 1;
      for (size_t st = 0; st < X.rad.size(); ++st) {
        plan[2 * st] = X.rad[st];
        plan[2 * st + 1] = ml;
        ml *= X.rad[st];
      }
      if ((e = upload(this, tw, &X.tw)) != hipSuccess ||
          (e = upload(this, plan, &X.plan)) != hipSuccess ||
          (e = upload(this, digit_reversal(X.n, X.rad), &X.rev)) != hipSuccess ||
          (e = upload(this, d, &X.d)) != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? MCMG_E_OOM : MCMG_E_HIP, "Born tables: %s",
                    hipGetErrorString(e));
    }
    born.nstats = born_stats_blocks(ext.total);
    born.stats = (double*)alloc((size_t)2 * born.nstats * sizeof(double));
    if (!born.stats) return fail(MCMG_E_OOM, "Born reduction buffer");
  }
  BornStatsArgs sa{};
  sa.k2 = k2;
  for (int a = 0; a < 3; ++a) { sa.g[a] = gtab[a]; sa.n[a] = ext.n[a]; }
  sa.gmax = absorber == MCMG_ABL_SPONGE ? gamma_max : 0.0;
  sa.dim = dim;
  sa.N = ext.total;
  sa.out = born.stats;
  std::vector<double> hs(2 * born.nstats);
  auto reduce = [&](int pass, double* lo, double* hi) -> hipError_t {
    hipError_t r = launch_born_stats(sa, pass, stream);
    if (r != hipSuccess) return r;
    r = hipMemcpyAsync(hs.data(), born.stats, hs.size() * sizeof(double), hipMemcpyDeviceToHost,
                       stream);
    if (r != hipSuccess) return r;
    if ((r = hipStreamSynchronize(stream)) != hipSuccess) return r;
    *lo = hs[0];
    *hi = hs[1];
    for (int b = 1; b < born.nstats; ++b) {
      *lo = std::fmin(*lo, hs[2 * b]);
      *hi = std::fmax(*hi, hs[2 * b + 1]);
    }
    return hipSuccess;
  };
  double k0sq = k0sq_in;
  if (!(k0sq > 0)) {
    double lo, hi;
    if ((e = reduce(0, &lo, &hi)) != hipSuccess)
      return fail(MCMG_E_HIP, "Born background: %s", hipGetErrorString(e));
    k0sq = 0.5 * (lo + hi);
  }
  double eps = eps_in;
  if (!(eps > 0)) {
    sa.k0sq = k0sq;
    double lo, hi;
    if ((e = reduce(1, &lo, &hi)) != hipSuccess)
      return fail(MCMG_E_HIP, "Born background: %s", hipGetErrorString(e));
    eps = hi;
  }
  if (!(eps > 0) || !std::isfinite(eps) || !std::isfinite(k0sq))
    return fail(MCMG_E_ARG, "Born background: eps = %g (a constant medium without a sponge "
                            "has no scattering potential; pass eps > 0)", eps);
  born.k0sq = k0sq;
  born.eps = eps;
  born.ready = true;
  return MCMG_OK;
}

hipError_t Ctx::helm_periodic(const double* u, const double* f, double* out, double* partial) {
  HelmOp op = helm();
  op.periodic = 1;
  const double N = (double)ext.total;
  const double bytes = N * (16.0 + 8.0 + 16.0 + (f ? 16.0 : 0.0));
  const double flops = N * (dim == 2 ? 38.0 : 54.0);
  const char* name = intern_name(std::string("helm_kernel<") + std::to_string(dim) + ", double>");
  return timed(name, flops, bytes,
               [=] { return launch_helm(op, T_F64, u, f, out, partial, stream); });
}

hipError_t Ctx::green(const double* x, double* y, double* u_cbs) {
  const int D = dim;
  long long tot = 1;
  for (int a = 0; a < D; ++a) tot *= next[a];
  auto pass = [&](int mode, int a, const double* src) -> hipError_t {
    const BornAxis& X = born.ax[a];
    FftArgs A{};
    A.src = src;
    A.dst = y;
    A.tw = X.tw;
    A.rev = X.rev;
    A.L = X.n;
    A.nst = (int)X.rad.size();
    A.plan = X.plan;
    double cmacs = 0;
    A.rc = FFT_RC_SMALL;
    for (int s = 0; s < A.nst; ++s) {
      cmacs += X.rad[s];
      if (X.rad[s] == 11) A.rc = std::max(A.rc, (int)FFT_RC_11);
      else if (X.rad[s] > 7) A.rc = FFT_RC_ANY;
    }
    long long S = 1, O = 1;
    for (int b = a + 1; b < D; ++b) S *= next[b];
    for (int b = 0; b < a; ++b) O *= next[b];
    A.S = S;
    A.contiguous = S == 1;
    // about 3072 elements per block: measured best on 1056^2 and 216^3
    // (more lines per block cut the grid below two blocks per CU, fewer
    // leave threads idle in the butterfly stages)
    constexpr int kElems = 3072;
    A.outer = A.contiguous ? tot / X.n : O;
    A.TC = std::max(1, std::min(16, kElems / X.n));
    A.tw_lds = ((size_t)A.TC * (X.n + 1) + X.n) * 16 <= FFT_MAXLDS ? 1 : 0;
    for (int b = 0; b < 3; ++b) {
      A.d[b] = b < D ? born.ax[b].d : nullptr;
      A.n[b] = b < D ? next[b] : 1;
      A.g[b] = gtab[b];
    }
    A.dim = D;
    A.k0sq = born.k0sq;
    A.eps = born.eps;
    A.scale = 1.0 / (double)tot;
    A.u = mode == FFT_LAST ? u_cbs : nullptr;
    A.k2 = k2;
    A.gmax = absorber == MCMG_ABL_SPONGE ? gamma_max : 0.0;
    const double n = (double)tot;
    const double flops = n * 8.0 * cmacs * (mode == FFT_SYM ? 2.0 : 1.0);
    const double bytes = (mode == FFT_LAST && u_cbs) ? n * 56.0 : n * 32.0;
    const char* name = intern_name("fft_kernel<" + std::to_string(mode) + ", " +
                                   std::to_string(A.rc) + ", " + (A.tw_lds ? "true" : "false") +
                                   ">");
    return timed(name, flops, bytes, [=] { return launch_fft(mode, A, stream); });
  };
  hipError_t e;
  if (D == 2) {
    if ((e = pass(FFT_FWD, 1, x)) != hipSuccess) return e;
    if ((e = pass(FFT_SYM, 0, y)) != hipSuccess) return e;
    return pass(FFT_LAST, 1, y);
  }
  if ((e = pass(FFT_FWD, 2, x)) != hipSuccess) return e;
  if ((e = pass(FFT_FWD, 1, y)) != hipSuccess) return e;
  if ((e = pass(FFT_SYM, 0, y)) != hipSuccess) return e;
  if ((e = pass(FFT_INV, 1, y)) != hipSuccess) return e;
  return pass(FFT_LAST, 2, y);
}

}  // namespace mcmg

using namespace mcmg;

extern "C" {

mcmg_status mcmg_born_setup(mcmg_handle h, double k0sq, double eps) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  return ((Ctx*)h)->born_setup(k0sq, eps);
}

mcmg_status mcmg_born_params(mcmg_handle h, double* k0sq, double* eps) {
  if (!h || !k0sq || !eps) return fail(MCMG_E_ARG, "null argument");
  Ctx* c = (Ctx*)h;
  if (!c->born.ready) {
    const mcmg_status st = c->born_setup(0.0, 0.0);
    if (st != MCMG_OK) return st;
  }
  *k0sq = c->born.k0sq;
  *eps = c->born.eps;
  return MCMG_OK;
}

mcmg_status mcmg_born_green(mcmg_handle h, const double* x, double* y) {
  if (!h || !x || !y) return fail(MCMG_E_ARG, "null argument");
  Ctx* c = (Ctx*)h;
  if (!c->born.ready) {
    const mcmg_status st = c->born_setup(0.0, 0.0);
    if (st != MCMG_OK) return st;
  }
  const hipError_t e = c->green(x, y, nullptr);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "green: %s", hipGetErrorString(e));
  return MCMG_OK;
}

mcmg_status mcmg_born_matvec(mcmg_handle h, const double* u, double* Au) {
  if (!h || !u || !Au) return fail(MCMG_E_ARG, "null argument");
  if ((const void*)u == (const void*)Au) return fail(MCMG_E_ARG, "u and Au may not alias");
  Ctx* c = (Ctx*)h;
  if (c->absorber != MCMG_ABL_SPONGE && c->npml != 0)
    return fail(MCMG_E_ARG, "the Born form needs the sponge layer or no absorbing layer");
  const hipError_t e = c->helm_periodic(u, nullptr, Au, nullptr);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "born matvec: %s", hipGetErrorString(e));
  return MCMG_OK;
}

}  // extern "C"
