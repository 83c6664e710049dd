// Workspace slots (one device chunk per right-hand side in flight) and the
// batched FGMRES entry point, a loop over the batch engine's ticks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "conv_mfma.h"
#include "internal.h"
#include "mcmg.h"
#include "engine.h"
#include "runtime.h"

namespace mcmg {

Slot Ctx::current_slot() const {
  Slot s;
  for (const Level& lv : lev) {
    s.e.push_back(lv.e);
    s.r.push_back(lv.r);
    s.t.push_back(lv.t);
    s.u.push_back(lv.u);
    s.e_alt.push_back(lv.e_alt);
  }
  s.V = V; s.wv = wv; s.rv = rv; s.H = H; s.cs = cs; s.sn = sn; s.g = g; s.y = y;
  s.coef = coef; s.partial = partial; s.scal = scal; s.Z = Z; s.zt = zt; s.skip = skip;
  return s;
}

void Ctx::bind_slot(const Slot& s) {
  for (size_t l = 0; l < lev.size(); ++l) {
    lev[l].e = s.e[l]; lev[l].r = s.r[l]; lev[l].t = s.t[l]; lev[l].u = s.u[l];
    lev[l].e_alt = s.e_alt[l];
  }
  V = s.V; wv = s.wv; rv = s.rv; H = s.H; cs = s.cs; sn = s.sn; g = s.g; y = s.y;
  coef = s.coef; partial = s.partial; scal = s.scal; Z = s.Z; zt = s.zt; skip = s.skip;
}

// A slot is one device allocation carved into its buffers (so that it can be
// released as a whole); `base` null only measures it.
size_t Ctx::slot_layout(Slot* s, unsigned char* base) const {
  const long long N = ext.total;
  const int m = restart;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    const size_t at = off;
    off = (off + bytes + 255) / 256 * 256;
    return base ? (void*)(base + at) : nullptr;
  };
  if (s) { s->e.clear(); s->r.clear(); s->t.clear(); s->u.clear(); s->e_alt.clear(); }
  for (const Level& lv : lev) {
    const size_t nb = (size_t)lv.dims.total * lv.C * sizeof(float);
    float* e = (float*)take(nb);
    float* r = (float*)take(nb);
    float* t = (float*)take(nb);
    float* u = (float*)take(nb);
    float* ea = lv.e_alt ? (float*)take(nb) : nullptr;
    if (s) { s->e.push_back(e); s->r.push_back(r); s->t.push_back(t); s->u.push_back(u); s->e_alt.push_back(ea); }
  }
  const int nbmax = red_blocks(N) > helm_blocks(helm()) ? red_blocks(N) : helm_blocks(helm());
  double* V = (double*)take((size_t)(m + 1) * N * 2 * sizeof(double));
  float* Z = (float*)take((size_t)m * N * 2 * sizeof(float));
  double* wv = (double*)take(N * 2 * sizeof(double));
  double* rv = (double*)take(N * 2 * sizeof(double));
  float* zt = (float*)take(N * 2 * sizeof(float));
  double* H = (double*)take((size_t)(m + 1) * m * 2 * sizeof(double));
  double* cs = (double*)take(m * sizeof(double));
  double* sn = (double*)take(m * 2 * sizeof(double));
  double* g = (double*)take((m + 1) * 2 * sizeof(double));
  double* y = (double*)take(m * 2 * sizeof(double));
  double* coef = (double*)take((m + 2) * 2 * sizeof(double));
  double* partial = (double*)take((size_t)(m + 2) * nbmax * 2 * sizeof(double));
  double* scal = (double*)take(64 * sizeof(double));
  int* skip = (int*)take(64 * sizeof(int));
  if (s) {
    s->V = V; s->Z = Z; s->wv = wv; s->rv = rv; s->zt = zt; s->H = H; s->cs = cs; s->sn = sn;
    s->g = g; s->y = y; s->coef = coef; s->partial = partial; s->scal = scal; s->skip = skip;
  }
  return off;
}

size_t Ctx::slot_bytes() const { return slot_layout(nullptr, nullptr); }

mcmg_status Ctx::alloc_slot(Slot& s) {
  const size_t bytes = slot_bytes();
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MCMG_E_OOM, "slot allocation failed (%zu bytes)", bytes);
  }
  slot_layout(&s, (unsigned char*)p);
  s.chunk = p;
  s.bytes = bytes;
  return MCMG_OK;
}

void Ctx::free_slot(Slot& s) {
  if (s.chunk) (void)hipFree(s.chunk);
  s = Slot();
}

mcmg_status Ctx::ensure_slots(int n) {
  if (slots.empty()) slots.push_back(current_slot());
  while ((int)slots.size() < n) {
    Slot s;
    mcmg_status st = alloc_slot(s);
    if (st != MCMG_OK) return st;
    slots.push_back(s);
  }
  return MCMG_OK;
}

}  // namespace mcmg

using namespace mcmg;

extern "C" mcmg_status mcmg_solve_batch(mcmg_handle* hs, const double* const* f, double* const* u,
                                        int nb, double tol, int maxit, mcmg_info* infos) {
  if (!hs || !f || !u || nb < 0) return fail(MCMG_E_ARG, "null argument");
  if (nb == 0) return MCMG_OK;
  if (!(tol > 0) || maxit < 0) return fail(MCMG_E_ARG, "bad tol/maxit");
  for (int i = 0; i < nb; ++i)
    if (!hs[i] || !f[i] || !u[i]) return fail(MCMG_E_ARG, "null handle/array %d", i);
  Engine eng;
  // MCMG_GRAPHS=0: plain launches instead of the captured tick
  const char* genv = getenv("MCMG_GRAPHS");
  eng.use_graphs = !(genv && genv[0] == '0');
  mcmg_status st = eng.open((Ctx*)hs[0]);
  if (st != MCMG_OK) return st;
  std::string why;
  for (int i = 0; i < nb; ++i)
    if (!eng.compatible((Ctx*)hs[i], &why)) return fail(MCMG_E_ARG, "problem %d: %s", i, why.c_str());
  // workspace slots: a handle that appears k times gets k slots; the
  // handles' own streams are drained first (the batch runs on its own)
  std::map<Ctx*, int> count;
  for (int i = 0; i < nb; ++i) count[(Ctx*)hs[i]]++;
  for (auto& kv : count) {
    if (hipStreamSynchronize(kv.first->stream) != hipSuccess) return fail(MCMG_E_HIP, "stream sync");
    st = kv.first->ensure_slots(kv.second);
    if (st != MCMG_OK) return st;
  }
  std::vector<Work> W(nb);
  std::map<Ctx*, int> next;
  for (int i = 0; i < nb; ++i) {
    Ctx* c = (Ctx*)hs[i];
    W[i].c = c;
    W[i].slot = &c->slots[next[c]++];
    W[i].f = f[i];
    W[i].u = u[i];
    W[i].tol = tol;
    W[i].maxit = maxit;
    W[i].tag = (uint64_t)i;
    st = eng.add(&W[i]);
    if (st != MCMG_OK) return st;
  }
  while (eng.live() > 0) {
    st = eng.issue();
    if (st != MCMG_OK) return st;
    st = eng.complete(nullptr);
    if (st != MCMG_OK) return st;
  }
  mcmg_status worst = MCMG_OK;
  for (int i = 0; i < nb; ++i) {
    const Work& w = W[i];
    if (infos) {
      mcmg_info* in = &infos[i];
      in->iters = w.its;
      in->restarts = w.restarts;
      in->relres_true = w.relres;
      in->relres_est = w.relest;
      in->status = w.status;
      const int n = (int)w.hist.size() < in->hist_cap ? (int)w.hist.size() : in->hist_cap;
      if (in->hist)
        for (int q = 0; q < n; ++q) in->hist[q] = w.hist[q];
      in->hist_len = in->hist ? n : 0;
    }
    if (w.status < 0 && worst >= 0) worst = w.status;
    else if (worst >= 0 && w.status > worst) worst = w.status;
  }
  return worst;
}
