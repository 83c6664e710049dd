// Batched FGMRES entry point (many media / right-hand sides).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "mcmg.h"
#include "runtime.h"

using namespace mcmg;

namespace mcmg {
mcmg_status fgmres(Ctx* c, const double* f, double* u, double tol, int maxit, mcmg_info* info);
}

extern "C" mcmg_status mcmg_solve_batch(mcmg_handle* hs, const double* const* f, double* const* u,
                                        int nb, double tol, int maxit, mcmg_info* infos) {
  if (!hs || !f || !u || nb < 0) return fail(MCMG_E_ARG, "null argument");
  mcmg_status worst = MCMG_OK;
  for (int i = 0; i < nb; ++i) {
    if (!hs[i]) return fail(MCMG_E_ARG, "null handle %d", i);
    mcmg_status st = fgmres((Ctx*)hs[i], f[i], u[i], tol, maxit, infos ? &infos[i] : nullptr);
    if (st < 0) return st;
    if (st > worst) worst = st;
  }
  return worst;
}
