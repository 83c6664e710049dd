// Outer iterations on the GPU: restarted right-preconditioned FGMRES(m)
// (McMg as the preconditioner, Sec. 3.3 / Sec. 4.1) and the stationary McMg
// iteration u <- u + MG(f - A u) (Eq. mcmg_iteration).
//
// Precision follows the paper's mixed-precision rule (Sec. 4.1): the V-cycle
// runs in float32 (or bf16 operands), while the residual f - A u, the
// Arnoldi process, the Givens least-squares update and the solution update
// run in float64.  z_j = MG(v_j) is stored as float32 complex, which holds
// the projection output exactly.
//
// Host/device traffic per iteration: one 24-byte read of (|g_{j+1}|, h_{j+1,j},
// column norm) for the stopping test; everything else stays on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.h"
#include "mcmg.h"
#include "runtime.h"

using namespace mcmg;

namespace {

struct Finish {
  mcmg_info* info;
  int iters = 0, restarts = 0;
  double relres_true = 0, relres_est = 0;
  std::vector<double> hist;
  mcmg_status done(mcmg_status st) {
    if (info) {
      info->iters = iters;
      info->restarts = restarts;
      info->relres_true = relres_true;
      info->relres_est = relres_est;
      info->status = st;
      const int n = (int)hist.size() < info->hist_cap ? (int)hist.size() : info->hist_cap;
      if (info->hist) for (int i = 0; i < n; ++i) info->hist[i] = hist[i];
      info->hist_len = info->hist ? n : 0;
    }
    return st;
  }
};

#define HCK(x)                                                                  \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) return fin.done(fail(MCMG_E_HIP, "%s: %s", #x, hipGetErrorString(e_))); \
  } while (0)

// |f|: multi-dot with no basis vectors yields |w|^2 only.
hipError_t norm_sq(Ctx* c, const double* x, double* out) {
  const long long N = c->ext.total;
  hipError_t e = launch_multidot(nullptr, N, 0, x, N, c->partial, nullptr, c->stream);
  if (e != hipSuccess) return e;
  return launch_reduce_dots(c->partial, c->nb_red, 0, c->coef, c->coef, out, nullptr, c->stream);
}

// r = f - A u and |r| -> scal[3]
hipError_t true_residual(Ctx* c, const double* f, const double* u) {
  HelmOp op = c->helm();
  hipError_t e = c->helm_timed(T_F64, u, f, c->rv, c->partial);
  if (e != hipSuccess) return e;
  return launch_reduce_sum(c->partial, helm_blocks(op), c->scal + 2, c->stream);
}

hipError_t read_scal(Ctx* c, int off, int n) {
  hipError_t e = hipMemcpyAsync(c->host_scal, c->scal + off, n * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

}  // namespace

namespace mcmg {

mcmg_status fgmres(Ctx* c, const double* f, double* u, double tol, int maxit, mcmg_info* info) {
  Finish fin{info};
  if (!f || !u) return fin.done(fail(MCMG_E_ARG, "null f or u"));
  if (!(tol > 0) || maxit < 0) return fin.done(fail(MCMG_E_ARG, "bad tol/maxit"));
  hipStream_t s = c->stream;
  const long long N = c->ext.total;
  const int m = c->restart;
  const int ldh = m + 1;
  HelmOp op = c->helm();

  HCK(norm_sq(c, f, c->scal + 0));
  HCK(read_scal(c, 0, 1));
  const double fnorm = std::sqrt(c->host_scal[0]);
  if (!std::isfinite(fnorm)) return fin.done(fail(MCMG_E_NONFINITE, "non-finite right-hand side"));
  if (fnorm == 0.0) {
    HCK(launch_zero_f64(u, 2 * N, s));
    HCK(hipStreamSynchronize(s));
    return fin.done(MCMG_OK);
  }
  const double target = tol * fnorm;
  HCK(true_residual(c, f, u));
  HCK(read_scal(c, 3, 1));
  double beta = c->host_scal[0];
  int its = 0;
  while (true) {
    fin.iters = its;
    fin.relres_true = beta / fnorm;
    if (!std::isfinite(beta)) return fin.done(fail(MCMG_E_NONFINITE, "non-finite residual"));
    if (beta <= target) return fin.done(MCMG_OK);
    if (its >= maxit) return fin.done(MCMG_NOT_CONVERGED);
    HCK(launch_scale(c->rv, c->scal + 3, c->V, N, s));
    HCK(launch_zero_f64(c->H, (long long)ldh * m * 2, s));
    HCK(launch_init_g(c->g, m + 1, c->scal + 3, s));
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double* Vj = c->V + 2LL * j * N;
      float* Zj = c->Z + 2LL * j * N;
      HCK(c->vcycle(Vj, T_F64, Zj, T_F32));
      HCK(c->helm_timed(T_F32, Zj, nullptr, c->wv, nullptr));
      ++its;
      double* Hcol = c->H + 2LL * j * ldh;
      const int nv = j + 1;
      const int nb = c->nb_red;
      // pass 0 (always) and pass 1 (device-gated re-orthogonalisation)
      const double vb = 16.0 * (double)N;
      HCK(c->timed("multidot_kernel", 8.0 * N * (nv + 1), vb * (nv + 1),
                   [=] { return launch_multidot(c->V, N, nv, c->wv, N, c->partial, nullptr, s); }));
      HCK(launch_reduce_dots(c->partial, nb, nv, c->coef, Hcol, c->scal + 8, nullptr, s));
      HCK(c->timed("update_kernel", 8.0 * N * (nv + 1), vb * (nv + 2),
                   [=] { return launch_update(c->V, N, nv, c->coef, c->wv, N, c->partial, nullptr, s); }));
      HCK(launch_reduce_norm(c->partial, nb, c->scal + 8, c->scal + 9, c->skip, 0,
                             c->ortho == 1, s));
      // the second pass exits at once unless the device flagged cancellation
      HCK(c->timed("multidot_kernel", 8.0 * N * (nv + 1), vb * (nv + 1),
                   [=] { return launch_multidot(c->V, N, nv, c->wv, N, c->partial, c->skip, s); }));
      HCK(launch_reduce_dots(c->partial, nb, nv, c->coef, Hcol, c->scal + 10, c->skip, s));
      HCK(c->timed("update_kernel", 8.0 * N * (nv + 1), vb * (nv + 2),
                   [=] { return launch_update(c->V, N, nv, c->coef, c->wv, N, c->partial, c->skip, s); }));
      HCK(launch_norm_givens(c->partial, nb, c->scal + 8, c->scal + 9, c->skip, c->H, ldh, j,
                             c->cs, c->sn, c->g, c->scal + 16, s));
      if (j + 1 < m) HCK(launch_scale(c->wv, c->scal + 9, c->V + 2LL * (j + 1) * N, N, s));
      HCK(read_scal(c, 16, 4));
      const double rho = c->host_scal[0], hn = c->host_scal[1], cn = c->host_scal[2];
      const double diag = c->host_scal[3];
      if (c->prof.on && c->prof.recs.size() >= 2) {
        // the second Gram-Schmidt pass did no work when the device skipped it
        int skipped = 0;
        HCK(hipMemcpy(&skipped, c->skip, sizeof(int), hipMemcpyDeviceToHost));
        if (skipped) {
          int fixed = 0;
          for (size_t q = c->prof.recs.size(); q-- > 0 && fixed < 2;) {
            ProfRec& pr = c->prof.recs[q];
            if (pr.name == std::string("multidot_kernel") || pr.name == std::string("update_kernel")) {
              pr.flops = 0.0;
              pr.bytes = 0.0;
              ++fixed;
            }
          }
        }
      }
      fin.hist.push_back(rho / fnorm);
      fin.relres_est = rho / fnorm;
      k = j + 1;
      if (!std::isfinite(rho) || !std::isfinite(hn))
        return fin.done(fail(MCMG_E_NONFINITE, "non-finite value in the Arnoldi process"));
      if (diag == 0.0) {
        // column j is zero after the earlier rotations (e.g. MG(v_j) = 0):
        // the triangular system of the cycle is the j columns before it
        k = j;
        break;
      }
      if (rho <= target || hn <= 1e-14 * cn || its >= maxit) break;
    }
    if (k == 0) {
      // not even the first direction is usable: a restart would repeat this
      // cycle, so stop with u unchanged
      fin.iters = its;
      return fin.done(MCMG_NOT_CONVERGED);
    }
    HCK(launch_backsolve(c->H, ldh, k, c->g, c->y, s));
    HCK(c->timed("zupdate_kernel", 8.0 * N * k, (8.0 * k + 32.0) * N,
                 [=] { return launch_zupdate(c->Z, N, k, c->y, u, N, s); }));
    HCK(true_residual(c, f, u));
    HCK(read_scal(c, 3, 1));
    beta = c->host_scal[0];
    ++fin.restarts;
  }
}

mcmg_status stationary(Ctx* c, const double* f, double* u, double tol, int maxit, mcmg_info* info) {
  Finish fin{info};
  if (!f || !u) return fin.done(fail(MCMG_E_ARG, "null f or u"));
  if (!(tol > 0) || maxit < 0) return fin.done(fail(MCMG_E_ARG, "bad tol/maxit"));
  hipStream_t s = c->stream;
  const long long N = c->ext.total;
  HCK(norm_sq(c, f, c->scal + 0));
  HCK(read_scal(c, 0, 1));
  const double fnorm = std::sqrt(c->host_scal[0]);
  if (!std::isfinite(fnorm)) return fin.done(fail(MCMG_E_NONFINITE, "non-finite right-hand side"));
  if (fnorm == 0.0) {
    HCK(launch_zero_f64(u, 2 * N, s));
    HCK(hipStreamSynchronize(s));
    return fin.done(MCMG_OK);
  }
  int its = 0;
  while (true) {
    HCK(true_residual(c, f, u));
    HCK(read_scal(c, 3, 1));
    const double beta = c->host_scal[0];
    fin.iters = its;
    fin.relres_true = beta / fnorm;
    fin.hist.push_back(beta / fnorm);
    if (!std::isfinite(beta)) return fin.done(fail(MCMG_E_NONFINITE, "non-finite residual"));
    if (beta <= tol * fnorm) return fin.done(MCMG_OK);
    if (its >= maxit) return fin.done(MCMG_NOT_CONVERGED);
    HCK(c->vcycle(c->rv, T_F64, c->zt, T_F32));
    HCK(launch_axpy_f32(c->zt, u, N, s));
    ++its;
  }
}

// Born-series iteration (appendix on the Born-series variant):
//   u <- u + P(G (f - A_per u)),  P = MG (Born+McMg) or gamma (.) (CBS, Eq. cbs_eq),
// with the true periodic residual |f - A_per u| <= tol |f| as the stop test.
// The residual, G and the update run in FP64; MG in the handle's precision.
mcmg_status born_solve(Ctx* c, int method, const double* f, double* u, double tol, int maxit,
                       mcmg_info* info) {
  Finish fin{info};
  if (!f || !u) return fin.done(fail(MCMG_E_ARG, "null f or u"));
  if (!(tol > 0) || maxit < 0) return fin.done(fail(MCMG_E_ARG, "bad tol/maxit"));
  if (method != MCMG_BORN_MCMG && method != MCMG_BORN_CBS)
    return fin.done(fail(MCMG_E_ARG, "unknown Born preconditioner %d", method));
  if (!c->born.ready) {
    const mcmg_status st = c->born_setup(0.0, 0.0);
    if (st != MCMG_OK) return fin.done(st);
  }
  hipStream_t s = c->stream;
  const long long N = c->ext.total;
  HCK(norm_sq(c, f, c->scal + 0));
  HCK(read_scal(c, 0, 1));
  const double fnorm = std::sqrt(c->host_scal[0]);
  if (!std::isfinite(fnorm)) return fin.done(fail(MCMG_E_NONFINITE, "non-finite right-hand side"));
  if (fnorm == 0.0) {
    HCK(launch_zero_f64(u, 2 * N, s));
    HCK(hipStreamSynchronize(s));
    return fin.done(MCMG_OK);
  }
  HelmOp op = c->helm();
  int its = 0;
  while (true) {
    HCK(c->helm_periodic(u, f, c->rv, c->partial));
    HCK(launch_reduce_sum(c->partial, helm_blocks(op), c->scal + 2, s));
    HCK(read_scal(c, 3, 1));
    const double beta = c->host_scal[0];
    fin.iters = its;
    fin.relres_true = beta / fnorm;
    fin.hist.push_back(beta / fnorm);
    if (!std::isfinite(beta)) return fin.done(fail(MCMG_E_NONFINITE, "non-finite residual"));
    if (beta <= tol * fnorm) return fin.done(MCMG_OK);
    if (its >= maxit) return fin.done(MCMG_NOT_CONVERGED);
    if (method == MCMG_BORN_CBS) {
      HCK(c->green(c->rv, c->rv, u));
    } else {
      HCK(c->green(c->rv, c->rv, nullptr));
      HCK(c->vcycle(c->rv, T_F64, c->zt, T_F32));
      HCK(launch_axpy_f32(c->zt, u, N, s));
    }
    ++its;
  }
}

}  // namespace mcmg

extern "C" {

mcmg_status mcmg_born_solve(mcmg_handle h, int method, const double* f, double* u, double tol,
                            int maxit, mcmg_info* info) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  return born_solve((Ctx*)h, method, f, u, tol, maxit, info);
}

mcmg_status mcmg_solve(mcmg_handle h, const double* f, double* u, double tol, int maxit,
                       mcmg_info* info) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  return fgmres((Ctx*)h, f, u, tol, maxit, info);
}

mcmg_status mcmg_stationary(mcmg_handle h, const double* f, double* u, double tol, int maxit,
                            mcmg_info* info) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  return stationary((Ctx*)h, f, u, tol, maxit, info);
}

}  // extern "C"
