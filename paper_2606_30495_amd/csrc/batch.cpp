// Batched FGMRES: many right-hand sides and media of uneven grid sizes
// advanced together, one launch per operation for the whole batch.
//
// Every problem (handle + workspace slot) records its V-cycle launch
// sequence once per Krylov position j (record mode: launches become RecOp
// descriptors).  Op i of all problems then runs as ONE batched launch whose
// blocks map onto problems through a block prefix; per-problem arguments
// come from device tables built once per solve.  All problems move through
// the restart cycle in lockstep; a problem that has converged (or reached
// maxit, or broken down) inside a cycle is frozen: its blocks return at once
// until the cycle ends, when every problem's solution update and true
// residual run batched.  Only the (rho, h, |col|, |r|) gather (4 doubles per
// problem) travels to the host each iteration, and the frozen flags back.
//
// Problems do not interact: each one's kernels read and write only its own
// buffers, and every reduction is per problem in a fixed order, so a result
// does not depend on what else is in the batch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "conv_mfma.h"
#include "internal.h"
#include "mcmg.h"
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

mcmg_status Ctx::alloc_slot(Slot& s) {
  const long long N = ext.total;
  const int m = restart;
  for (const Level& lv : lev) {
    const size_t nb = (size_t)lv.dims.total * lv.C * sizeof(float);
    float *e = (float*)alloc(nb), *r = (float*)alloc(nb), *t = (float*)alloc(nb), *u = (float*)alloc(nb);
    float* ea = lv.e_alt ? (float*)alloc(nb) : nullptr;
    if (!e || !r || !t || !u || (lv.e_alt && !ea)) return fail(MCMG_E_OOM, "slot allocation failed");
    s.e.push_back(e); s.r.push_back(r); s.t.push_back(t); s.u.push_back(u); s.e_alt.push_back(ea);
  }
  s.V = (double*)alloc((size_t)(m + 1) * N * 2 * sizeof(double));
  s.Z = (float*)alloc((size_t)m * N * 2 * sizeof(float));
  s.wv = (double*)alloc(N * 2 * sizeof(double));
  s.rv = (double*)alloc(N * 2 * sizeof(double));
  s.zt = (float*)alloc(N * 2 * sizeof(float));
  s.H = (double*)alloc((size_t)(m + 1) * m * 2 * sizeof(double));
  s.cs = (double*)alloc(m * sizeof(double));
  s.sn = (double*)alloc(m * 2 * sizeof(double));
  s.g = (double*)alloc((m + 1) * 2 * sizeof(double));
  s.y = (double*)alloc(m * 2 * sizeof(double));
  s.coef = (double*)alloc((m + 2) * 2 * sizeof(double));
  const int nbmax = red_blocks(N) > helm_blocks(helm()) ? red_blocks(N) : helm_blocks(helm());
  s.partial = (double*)alloc((size_t)(m + 2) * nbmax * 2 * sizeof(double));
  s.scal = (double*)alloc(64 * sizeof(double));
  s.skip = (int*)alloc(64 * sizeof(int));
  if (!s.V || !s.Z || !s.wv || !s.rv || !s.zt || !s.H || !s.cs || !s.sn || !s.g || !s.y ||
      !s.coef || !s.partial || !s.scal || !s.skip)
    return fail(MCMG_E_OOM, "slot allocation failed");
  return MCMG_OK;
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

namespace {

struct Prob {
  Ctx* c;
  int slot;
  const double* f;
  double* u;
  mcmg_info* info;
  // host state
  int its = 0, k = 0;
  bool done = false;
  mcmg_status status = MCMG_OK;
  double fnorm = 0, target = 0, relres = 0, relest = 0;
  std::vector<double> hist;
  int restarts = 0;
};

// Device blob holding every table of one batched solve.
struct DevTables {
  std::vector<unsigned char> host;
  void* dev = nullptr;
  size_t add(const void* p, size_t bytes) {
    const size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + bytes);
    memcpy(host.data() + off, p, bytes);
    return off;
  }
  const void* at(size_t off) const { return (const unsigned char*)dev + off; }
};

struct OpTable {
  int kind;
  RecOp proto;
  size_t tab_off, pre_off;
  int total;
};

template <class T>
size_t add_table(DevTables& dt, const std::vector<T>& v) { return dt.add(v.data(), v.size() * sizeof(T)); }

mcmg_status finish_infos(std::vector<Prob>& P) {
  mcmg_status worst = MCMG_OK;
  for (Prob& p : P) {
    if (p.info) {
      p.info->iters = p.its;
      p.info->restarts = p.restarts;
      p.info->relres_true = p.relres;
      p.info->relres_est = p.relest;
      p.info->status = p.status;
      const int n = (int)p.hist.size() < p.info->hist_cap ? (int)p.hist.size() : p.info->hist_cap;
      if (p.info->hist)
        for (int i = 0; i < n; ++i) p.info->hist[i] = p.hist[i];
      p.info->hist_len = p.info->hist ? n : 0;
    }
    if (p.status < 0) return p.status;
    if (p.status > worst) worst = p.status;
  }
  return worst;
}

}  // namespace

extern "C" mcmg_status mcmg_solve_batch(mcmg_handle* hs, const double* const* f, double* const* u,
                                        int nb, double tol, int maxit, mcmg_info* infos) {
  if (!hs || !f || !u || nb < 0) return fail(MCMG_E_ARG, "null argument");
  if (nb == 0) return MCMG_OK;
  if (!(tol > 0) || maxit < 0) return fail(MCMG_E_ARG, "bad tol/maxit");
  Ctx* c0 = (Ctx*)hs[0];
  if (!c0) return fail(MCMG_E_ARG, "null handle 0");
  const int m = c0->restart;
  // ---- compatibility: shared template parameters of every batched launch
  for (int i = 0; i < nb; ++i) {
    Ctx* c = (Ctx*)hs[i];
    if (!c || !f[i] || !u[i]) return fail(MCMG_E_ARG, "null handle/array %d", i);
    if (c->dim != c0->dim || c->L != c0->L || c->precision != c0->precision ||
        c->restart != m || c->ortho != c0->ortho)
      return fail(MCMG_E_ARG, "problem %d: dim, levels, precision and restart must match", i);
    for (int l = 0; l < c->L; ++l) {
      const Level &a = c->lev[l], &b = c0->lev[l];
      if (a.C != b.C || a.nu1 != b.nu1 || a.nu2 != b.nu2 || a.l1w.empty() != b.l1w.empty() ||
          a.op_resid.on != b.op_resid.on || a.op_R.on != b.op_R.on || a.op_P.on != b.op_P.on)
        return fail(MCMG_E_ARG, "problem %d: level %d structure differs", i, l + 1);
      if (a.nu1 == 0) return fail(MCMG_E_ARG, "batched solve needs nu1 > 0 on every level");
    }
  }
  // The batch runs on a stream of its own (graph capture is not possible on
  // the legacy default stream); every handle's stream is drained first, and
  // the call returns only when the batch is done.
  const char* genv = getenv("MCMG_GRAPHS");
  const bool use_graphs = !(genv && genv[0] == '0');
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return fail(MCMG_E_HIP, "stream create failed");
  struct StreamFree { hipStream_t s; ~StreamFree() { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); } } sfree{s};
  // ---- workspace slots: a handle that appears k times gets k slots
  std::map<Ctx*, int> count;
  for (int i = 0; i < nb; ++i) count[(Ctx*)hs[i]]++;
  for (auto& kv : count) {
    if (hipStreamSynchronize(kv.first->stream) != hipSuccess) return fail(MCMG_E_HIP, "stream sync");
    mcmg_status st = kv.first->ensure_slots(kv.second);
    if (st != MCMG_OK) return st;
  }
  std::vector<Prob> P(nb);
  {
    std::map<Ctx*, int> next;
    for (int i = 0; i < nb; ++i) {
      Ctx* c = (Ctx*)hs[i];
      P[i].c = c;
      P[i].slot = next[c]++;
      P[i].f = f[i];
      P[i].u = u[i];
      P[i].info = infos ? &infos[i] : nullptr;
    }
  }
  // ---- record each problem's V-cycle for every Krylov position j
  std::vector<std::vector<std::vector<RecOp>>> ops(nb, std::vector<std::vector<RecOp>>(m));
  for (int i = 0; i < nb; ++i) {
    Ctx* c = P[i].c;
    const Slot base = c->current_slot();
    const Slot& sl = c->slots[P[i].slot];
    const long long N = c->ext.total;
    for (int j = 0; j < m; ++j) {
      c->bind_slot(sl);
      c->rec = &ops[i][j];
      hipError_t e = c->vcycle(sl.V + 2LL * j * N, T_F64, sl.Z + 2LL * j * N, T_F32);
      c->rec = nullptr;
      if (e != hipSuccess) { c->bind_slot(base); return fail(MCMG_E_HIP, "record: %s", hipGetErrorString(e)); }
    }
    c->bind_slot(base);
  }
  const size_t nops = ops[0][0].size();
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < m; ++j) {
      if (ops[i][j].size() != nops) return fail(MCMG_E_ARG, "V-cycle schedules differ");
      for (size_t q = 0; q < nops; ++q)
        if (ops[i][j][q].kind != ops[0][0][q].kind) return fail(MCMG_E_ARG, "V-cycle schedules differ");
    }
  // ---- device tables
  DevTables dt;
  std::vector<std::vector<OpTable>> vt(m, std::vector<OpTable>(nops));
  for (int j = 0; j < m; ++j)
    for (size_t q = 0; q < nops; ++q) {
      OpTable& ot = vt[j][q];
      ot.kind = ops[0][j][q].kind;
      ot.proto = ops[0][j][q];
      std::vector<int> pre(nb + 1, 0);
      if (ot.kind == 0) {
        std::vector<DArgs> tab(nb);
        for (int i = 0; i < nb; ++i) {
          int nblk;
          tab[i] = conv_args(ops[i][j][q].conv, &nblk);
          pre[i + 1] = pre[i] + nblk;
        }
        ot.tab_off = add_table(dt, tab);
      } else if (ot.kind == 1) {
        std::vector<MArgs> tab(nb);
        for (int i = 0; i < nb; ++i) {
          MfmaConv a = ops[i][j][q].mf;
          a.mt = ot.proto.mf.mt;   // one tile shape for the whole launch
          a.ntw = ot.proto.mf.ntw;
          a.kchunk = ot.proto.mf.kchunk;
          int nblk;
          tab[i] = mfma_args(a, &nblk);
          pre[i + 1] = pre[i] + nblk;
        }
        ot.tab_off = add_table(dt, tab);
      } else {
        std::vector<L1Args> tab(nb);
        for (int i = 0; i < nb; ++i) {
          int nblk;
          tab[i] = l1_args(ops[i][j][q].l1, ops[i][j][q].l1w_dev, &nblk);
          pre[i + 1] = pre[i] + nblk;
        }
        ot.tab_off = add_table(dt, tab);
      }
      ot.pre_off = add_table(dt, pre);
      ot.total = pre[nb];
    }
  // Helmholtz tables: matvec w = A Z_j per j, residual r = f - A u
  std::vector<size_t> hmv_off(m);
  std::vector<int> pre_red(nb + 1, 0), pre_elem(nb + 1, 0);
  for (int i = 0; i < nb; ++i) {
    pre_red[i + 1] = pre_red[i] + red_blocks(P[i].c->ext.total);
    pre_elem[i + 1] = pre_elem[i] + elem_blocks(P[i].c->ext.total);
  }
  for (int j = 0; j < m; ++j) {
    std::vector<HArgs> tab(nb);
    for (int i = 0; i < nb; ++i) {
      const Slot& sl = P[i].c->slots[P[i].slot];
      tab[i] = HArgs{P[i].c->helm(), sl.Z + 2LL * j * P[i].c->ext.total, nullptr, sl.wv, nullptr};
    }
    hmv_off[j] = add_table(dt, tab);
  }
  size_t hres_off;
  {
    std::vector<HArgs> tab(nb);
    for (int i = 0; i < nb; ++i) {
      const Slot& sl = P[i].c->slots[P[i].slot];
      tab[i] = HArgs{P[i].c->helm(), P[i].u, P[i].f, sl.rv, sl.partial};
    }
    hres_off = add_table(dt, tab);
  }
  std::vector<KArgs> kargs(nb);
  for (int i = 0; i < nb; ++i) {
    const Slot& sl = P[i].c->slots[P[i].slot];
    KArgs& k = kargs[i];
    k.V = sl.V; k.Z = sl.Z; k.w = sl.wv; k.r = sl.rv; k.f = P[i].f; k.u = P[i].u;
    k.H = sl.H; k.cs = sl.cs; k.sn = sl.sn; k.g = sl.g; k.y = sl.y; k.coef = sl.coef;
    k.partial = sl.partial; k.scal = sl.scal; k.skip = sl.skip;
    k.N = P[i].c->ext.total; k.ldh = m + 1; k.k = 0; k.always_two = P[i].c->ortho == 1;
  }
  const size_t karg_off = add_table(dt, kargs);
  const size_t pre_red_off = add_table(dt, pre_red), pre_elem_off = add_table(dt, pre_elem);
  std::vector<int> zeros_i(nb, 0);
  const size_t frozen_off = add_table(dt, zeros_i);
  std::vector<double> zeros_d(4 * nb, 0.0);
  const size_t gather_off = add_table(dt, zeros_d);

  if (hipMalloc(&dt.dev, dt.host.size()) != hipSuccess) { (void)hipGetLastError(); return fail(MCMG_E_OOM, "batch tables"); }
  struct Free { void* p; int* hf; double* hg; ~Free() { if (p) (void)hipFree(p); if (hf) (void)hipHostFree(hf); if (hg) (void)hipHostFree(hg); } } fr{dt.dev, nullptr, nullptr};
  int* hfrozen = nullptr;
  double* hgather = nullptr;
  if (hipHostMalloc((void**)&hfrozen, nb * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return fail(MCMG_E_OOM, "pinned host buffers");
  fr.hf = hfrozen;
  if (hipHostMalloc((void**)&hgather, 4 * nb * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(MCMG_E_OOM, "pinned host buffers");
  fr.hg = hgather;
  hipError_t e = hipMemcpyAsync(dt.dev, dt.host.data(), dt.host.size(), hipMemcpyHostToDevice, s);
#define BCK(x)                                                                  \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) return fail(MCMG_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)
  BCK(e);
  int* d_frozen = (int*)dt.at(frozen_off);
  double* d_gather = (double*)dt.at(gather_off);
  KBatch kb;
  kb.tab = (const KArgs*)dt.at(karg_off);
  kb.np = nb;
  kb.pre_red = (const int*)dt.at(pre_red_off);
  kb.total_red = pre_red[nb];
  kb.pre_elem = (const int*)dt.at(pre_elem_off);
  kb.total_elem = pre_elem[nb];
  kb.frozen = d_frozen;
  kb.gather = d_gather;
  const int dim = c0->dim;

  auto push_frozen = [&]() -> hipError_t {
    for (int i = 0; i < nb; ++i) hfrozen[i] = P[i].done || P[i].k < 0 ? 1 : 0;
    return hipMemcpyAsync(d_frozen, hfrozen, nb * sizeof(int), hipMemcpyHostToDevice, s);
  };
  auto pull_gather = [&]() -> hipError_t {
    hipError_t ee = hipMemcpyAsync(hgather, d_gather, 4 * nb * sizeof(double), hipMemcpyDeviceToHost, s);
    if (ee != hipSuccess) return ee;
    return hipStreamSynchronize(s);
  };
  auto vcycle_batched = [&](int j) -> hipError_t {
    for (size_t q = 0; q < nops; ++q) {
      const OpTable& ot = vt[j][q];
      BatchLaunch b{dt.at(ot.tab_off), (const int*)dt.at(ot.pre_off), nb, ot.total, d_frozen};
      hipError_t ee;
      if (ot.kind == 0) ee = launch_conv_batched(ot.proto.conv, b, s);
      else if (ot.kind == 1) ee = launch_conv_mfma_batched(ot.proto.mf, b, s);
      else ee = launch_level1_batched(dim, ot.proto.l1.var, b, s);
      if (ee != hipSuccess) return ee;
    }
    return hipSuccess;
  };
  // One FGMRES iteration at Krylov position j for every live problem, ending
  // with the gather copy to the host (no synchronisation inside, so the same
  // sequence can be captured into a graph and replayed).
  auto iteration = [&](int j) -> hipError_t {
    hipError_t ee = vcycle_batched(j);
    if (ee != hipSuccess) return ee;
    {
      BatchLaunch b{dt.at(hmv_off[j]), (const int*)dt.at(pre_red_off), nb, pre_red[nb], d_frozen};
      if ((ee = launch_helm_batched(dim, T_F32, b, s)) != hipSuccess) return ee;
    }
    const int nv = j + 1;
    for (int pass = 0; pass < 2; ++pass) {
      if ((ee = kb_launch(KB_MULTIDOT, kb, nv, j, pass, m, s)) != hipSuccess) return ee;
      if ((ee = kb_launch(KB_REDUCE_DOTS, kb, nv, j, pass, m, s)) != hipSuccess) return ee;
      if ((ee = kb_launch(KB_UPDATE, kb, nv, j, pass, m, s)) != hipSuccess) return ee;
      if ((ee = kb_launch(KB_REDUCE_NORM, kb, nv, j, pass, m, s)) != hipSuccess) return ee;
    }
    if ((ee = kb_launch(KB_GIVENS, kb, nv, j, 0, m, s)) != hipSuccess) return ee;
    if (j + 1 < m && (ee = kb_launch(KB_SCALE_W, kb, nv, j, 0, m, s)) != hipSuccess) return ee;
    return hipMemcpyAsync(hgather, d_gather, 4 * nb * sizeof(double), hipMemcpyDeviceToHost, s);
  };
  // Iterations replay one captured graph per Krylov position (MCMG_GRAPHS=0:
  // plain launches); graph nodes hold only device table pointers, so they
  // stay valid across cycles while the frozen flags and k change.
  std::vector<hipGraphExec_t> gexec(m, nullptr);
  struct GraphFree {
    std::vector<hipGraphExec_t>* g;
    ~GraphFree() { for (auto x : *g) if (x) (void)hipGraphExecDestroy(x); }
  } gfree{&gexec};
  auto residual_batched = [&]() -> hipError_t {
    BatchLaunch b{dt.at(hres_off), (const int*)dt.at(pre_red_off), nb, pre_red[nb], d_frozen};
    hipError_t ee = launch_helm_batched(dim, T_F64, b, s);
    if (ee != hipSuccess) return ee;
    return kb_launch(KB_REDUCE_SUM, kb, 0, 0, 0, m, s);
  };

  // ---- |f| per problem (once per solve)
  for (int i = 0; i < nb; ++i) {
    const Slot& sl = P[i].c->slots[P[i].slot];
    const long long N = P[i].c->ext.total;
    BCK(launch_multidot(nullptr, N, 0, P[i].f, N, sl.partial, nullptr, s));
    BCK(launch_reduce_dots(sl.partial, red_blocks(N), 0, sl.coef, sl.coef, sl.scal + 0, nullptr, s));
    BCK(hipMemcpyAsync(hgather + 4 * i, sl.scal, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  BCK(hipStreamSynchronize(s));
  for (int i = 0; i < nb; ++i) {
    P[i].fnorm = std::sqrt(hgather[4 * i]);
    P[i].target = tol * P[i].fnorm;
    if (!std::isfinite(P[i].fnorm)) {
      P[i].done = true;
      P[i].status = fail(MCMG_E_NONFINITE, "problem %d: non-finite right-hand side", i);
    } else if (P[i].fnorm == 0.0) {
      BCK(launch_zero_f64(P[i].u, 2 * P[i].c->ext.total, s));
      P[i].done = true;
    }
  }
  // ---- initial residuals
  BCK(push_frozen());
  BCK(residual_batched());
  BCK(pull_gather());
  auto settle = [&](int i, double beta) {
    Prob& p = P[i];
    p.relres = beta / p.fnorm;
    if (!std::isfinite(beta)) {
      p.done = true;
      p.status = fail(MCMG_E_NONFINITE, "problem %d: non-finite residual", i);
    } else if (beta <= p.target) {
      p.done = true;
      p.status = MCMG_OK;
    } else if (p.its >= maxit) {
      p.done = true;
      p.status = MCMG_NOT_CONVERGED;
    }
  };
  for (int i = 0; i < nb; ++i)
    if (!P[i].done) settle(i, hgather[4 * i + 3]);

  // ---- restart cycles
  while (true) {
    bool any = false;
    for (Prob& p : P) { p.k = p.done ? -1 : 0; any |= !p.done; }
    if (!any) break;
    BCK(push_frozen());
    BCK(kb_launch(KB_SCALE_R, kb, 0, 0, 0, m, s));
    BCK(kb_launch(KB_CYCLE_INIT, kb, 0, 0, 0, m, s));
    for (int j = 0; j < m; ++j) {
      if (use_graphs) {
        if (!gexec[j]) {
          hipGraph_t g = nullptr;
          BCK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
          hipError_t ce = iteration(j);
          hipError_t ee = hipStreamEndCapture(s, &g);
          if (ce != hipSuccess) { if (g) (void)hipGraphDestroy(g); BCK(ce); }
          BCK(ee);
          ee = hipGraphInstantiate(&gexec[j], g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          BCK(ee);
        }
        BCK(hipGraphLaunch(gexec[j], s));
        BCK(hipStreamSynchronize(s));
      } else {
        BCK(iteration(j));
        BCK(hipStreamSynchronize(s));
      }
      bool live = false;
      for (int i = 0; i < nb; ++i) {
        Prob& p = P[i];
        if (p.done || p.k < 0 || hfrozen[i]) continue;
        const double rho = hgather[4 * i], hn = hgather[4 * i + 1], cn = hgather[4 * i + 2];
        ++p.its;
        p.k = j + 1;
        p.hist.push_back(rho / p.fnorm);
        p.relest = rho / p.fnorm;
        if (!std::isfinite(rho) || !std::isfinite(hn)) {
          p.done = true;
          p.status = fail(MCMG_E_NONFINITE, "problem %d: non-finite value in the Arnoldi process", i);
          continue;
        }
        if (rho <= p.target || hn <= 1e-14 * cn || p.its >= maxit) {
          hfrozen[i] = 1;   // rest of this cycle
        } else {
          live = true;
        }
      }
      if (!live) break;
      BCK(hipMemcpyAsync(d_frozen, hfrozen, nb * sizeof(int), hipMemcpyHostToDevice, s));
    }
    // ---- cycle end: u += Z y and the true residual for every problem that iterated
    for (int i = 0; i < nb; ++i) kargs[i].k = P[i].done ? 0 : (P[i].k > 0 ? P[i].k : 0);
    BCK(hipMemcpyAsync((void*)dt.at(karg_off), kargs.data(), nb * sizeof(KArgs), hipMemcpyHostToDevice, s));
    BCK(kb_launch(KB_BACKSOLVE, kb, 0, 0, 0, m, s));
    BCK(kb_launch(KB_ZUPDATE, kb, 0, 0, 0, m, s));
    for (int i = 0; i < nb; ++i) hfrozen[i] = kargs[i].k > 0 ? 0 : 1;
    BCK(hipMemcpyAsync(d_frozen, hfrozen, nb * sizeof(int), hipMemcpyHostToDevice, s));
    BCK(residual_batched());
    BCK(pull_gather());
    for (int i = 0; i < nb; ++i) {
      if (kargs[i].k <= 0) continue;
      P[i].restarts++;
      settle(i, hgather[4 * i + 3]);
    }
    for (int i = 0; i < nb; ++i) kargs[i].k = 0;
  }
#undef BCK
  return finish_infos(P);
}
