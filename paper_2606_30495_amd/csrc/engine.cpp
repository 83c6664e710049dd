// Batch engine (see engine.h): per-Work FGMRES state machines advanced in
// ticks of one launch per operation for all Works.
#include "engine.h"

#include <cmath>
#include <cstring>

#include "conv_mfma.h"
#include "internal.h"

namespace mcmg {

namespace {

struct Blob {
  std::vector<unsigned char> host;
  size_t add(const void* p, size_t bytes) {
    const size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + bytes);
    if (bytes) memcpy(host.data() + off, p, bytes);
    return off;
  }
  template <class T>
  size_t add(const std::vector<T>& v) { return add(v.data(), v.size() * sizeof(T)); }
};

// Whether two recordings of one V-cycle op use different buffers (the ops
// that read V_j or write Z_j, and nothing else, differ between positions).
bool differs(const RecOp& a, const RecOp& b) {
  switch (a.kind) {
    case 0:
      return a.conv.x != b.conv.x || a.conv.y != b.conv.y || a.conv.r != b.conv.r ||
             a.conv.feat != b.conv.feat;
    case 1:
      return a.mf.x != b.mf.x || a.mf.y != b.mf.y || a.mf.r != b.mf.r || a.mf.feat != b.mf.feat;
    case 2:
      return a.l1.e != b.l1.e || a.l1.eo != b.l1.eo || a.l1.r != b.l1.r;
    default:
      return a.st.e != b.st.e || a.st.eo != b.st.eo || a.st.r != b.st.r || a.st.wSM != b.st.wSM;
  }
}

enum { M_ITER = 0, M_END = 1, M_RES = 2, M_INIT = 3, M_JPOS = 4, M_KK = 5, M_COUNT = 6 };

}  // namespace

Engine::~Engine() {
  if (s_) (void)hipStreamSynchronize(s_);
  free_tables();
  if (ctl_host_) (void)hipHostFree(ctl_host_);
  if (gather_host_) (void)hipHostFree(gather_host_);
  if (s_) (void)hipStreamDestroy(s_);
}

void Engine::free_tables() {
  if (graph_) { (void)hipGraphExecDestroy(graph_); graph_ = nullptr; }
  if (dev_) { (void)hipFree(dev_); dev_ = nullptr; dev_cap_ = 0; }
}

mcmg_status Engine::open(const Ctx* c) {
  if (!c) return fail(MCMG_E_ARG, "null handle");
  if (!s_ && hipStreamCreateWithFlags(&s_, hipStreamNonBlocking) != hipSuccess)
    return fail(MCMG_E_HIP, "engine stream creation failed");
  dim_ = c->dim; L_ = c->L; prec_ = c->precision; m_ = c->restart; ortho_ = c->ortho;
  C_.clear(); nu1_.clear(); nu2_.clear(); l1_.clear(); mf_.clear();
  for (const Level& lv : c->lev) {
    C_.push_back(lv.C); nu1_.push_back(lv.nu1); nu2_.push_back(lv.nu2);
    l1_.push_back(!lv.l1w.empty());
    mf_.push_back(lv.op_resid.on * 4 + lv.op_R.on * 2 + lv.op_P.on + lv.step_on * 8);
  }
  return MCMG_OK;
}

bool Engine::compatible(const Ctx* c, std::string* why) const {
  auto no = [&](const char* w) { if (why) *why = w; return false; };
  if (c->dim != dim_ || c->L != L_) return no("dimension and level count differ");
  if (c->precision != prec_) return no("precision differs");
  if (c->restart != m_ || c->ortho != ortho_) return no("restart length or orthogonalisation differs");
  if (c->restart > 64) return no("batched solves take restart lengths up to 64");
  for (int l = 0; l < L_; ++l) {
    const Level& lv = c->lev[l];
    if (lv.C != C_[l] || lv.nu1 != nu1_[l] || lv.nu2 != nu2_[l]) return no("level structure differs");
    if ((int)!lv.l1w.empty() != l1_[l] ||
        lv.op_resid.on * 4 + lv.op_R.on * 2 + lv.op_P.on + lv.step_on * 8 != mf_[l])
      return no("kernel plan differs");
    if (lv.nu1 == 0) return no("batched solves need nu1 > 0 on every level");
  }
  return true;
}

mcmg_status Engine::add(Work* w) {
  if (!s_) return fail(MCMG_E_ARG, "engine not opened");
  if (!w || !w->c || !w->slot || !w->f || !w->u) return fail(MCMG_E_ARG, "incomplete work");
  if (!(w->tol > 0) || w->maxit < 0) return fail(MCMG_E_ARG, "bad tol/maxit");
  std::string why;
  if (!compatible(w->c, &why)) return fail(MCMG_E_ARG, "batch: %s", why.c_str());
  Ctx* c = w->c;
  const Slot base = c->current_slot();
  const long long N = c->ext.total;
  w->ops.assign(m_, {});
  for (int j = 0; j < m_; ++j) {
    c->bind_slot(*w->slot);
    c->rec = &w->ops[j];
    hipError_t e = c->vcycle(w->slot->V + 2LL * j * N, T_F64, w->slot->Z + 2LL * j * N, T_F32);
    c->rec = nullptr;
    c->bind_slot(base);
    if (e != hipSuccess) return fail(MCMG_E_HIP, "record: %s", hipGetErrorString(e));
  }
  if (kinds_.empty())
    for (const RecOp& r : w->ops[0]) kinds_.push_back(r.kind);
  for (int j = 0; j < m_; ++j) {
    if (w->ops[j].size() != kinds_.size()) return fail(MCMG_E_ARG, "V-cycle schedules differ");
    for (size_t q = 0; q < kinds_.size(); ++q)
      if (w->ops[j][q].kind != kinds_[q]) return fail(MCMG_E_ARG, "V-cycle schedules differ");
  }
  w->st = Work::INIT;
  w->j = w->k = w->its = w->restarts = 0;
  w->hist.clear();
  w->status = MCMG_OK;
  works_.push_back(w);
  dirty_ = true;
  return MCMG_OK;
}

void Engine::drop_done() {
  size_t n = 0;
  for (Work* w : works_)
    if (w->st != Work::DONE) works_[n++] = w;
  if (n != works_.size()) { works_.resize(n); dirty_ = true; }
}

int Engine::live() const {
  int n = 0;
  for (const Work* w : works_) n += w->st != Work::DONE;
  return n;
}

mcmg_status Engine::build() {
  if (hipStreamSynchronize(s_) != hipSuccess) return fail(MCMG_E_HIP, "engine sync");
  if (graph_) { (void)hipGraphExecDestroy(graph_); graph_ = nullptr; }
  ticks_same_ = 0;
  ++rebuilds;
  const int np = (int)works_.size();
  np_ = np;
  vt_.clear();
  dirty_ = false;
  if (np == 0) return MCMG_OK;
  // tile shapes of matrix-core launches come from the largest problem
  int big = 0;
  for (int i = 1; i < np; ++i)
    if (works_[i]->c->ext.total > works_[big]->c->ext.total) big = i;
  Blob b;
  const size_t nops = kinds_.size();
  for (size_t q = 0; q < nops; ++q) {
    OpTable ot;
    ot.kind = kinds_[q];
    ot.proto = works_[big]->ops[0][q];
    ot.jdep = false;
    for (int j = 1; j < m_ && !ot.jdep; ++j) ot.jdep = differs(works_[0]->ops[0][q], works_[0]->ops[j][q]);
    const int rows = ot.jdep ? m_ : 1;
    std::vector<int> pre(np + 1, 0);
    if (ot.kind == 0) {
      std::vector<DArgs> tab((size_t)rows * np);
      for (int r = 0; r < rows; ++r)
        for (int i = 0; i < np; ++i) {
          int nblk;
          tab[(size_t)r * np + i] = conv_args(works_[i]->ops[r][q].conv, &nblk);
          if (r == 0) pre[i + 1] = pre[i] + nblk;
        }
      ot.tab_off = b.add(tab);
    } else if (ot.kind == 1) {
      std::vector<MArgs> tab((size_t)rows * np);
      for (int r = 0; r < rows; ++r)
        for (int i = 0; i < np; ++i) {
          MfmaConv a = works_[i]->ops[r][q].mf;
          a.mt = ot.proto.mf.mt;      // one tile shape for the whole launch
          a.ntw = ot.proto.mf.ntw;
          a.rpw = ot.proto.mf.rpw;
          a.kchunk = ot.proto.mf.kchunk;
          int nblk;
          tab[(size_t)r * np + i] = mfma_args(a, &nblk);
          if (r == 0) pre[i + 1] = pre[i] + nblk;
        }
      ot.tab_off = b.add(tab);
    } else if (ot.kind == 3) {
      std::vector<SArgs> tab((size_t)rows * np);
      for (int r = 0; r < rows; ++r)
        for (int i = 0; i < np; ++i) {
          StepLaunch a = works_[i]->ops[r][q].st;
          a.tile = ot.proto.st.tile;         // one tile shape for the whole launch
          a.kc1 = ot.proto.st.kc1;
          a.kc2 = ot.proto.st.kc2;
          int nblk;
          tab[(size_t)r * np + i] = step_args(a, &nblk);
          if (r == 0) pre[i + 1] = pre[i] + nblk;
        }
      ot.tab_off = b.add(tab);
    } else {
      std::vector<L1Args> tab((size_t)rows * np);
      for (int r = 0; r < rows; ++r)
        for (int i = 0; i < np; ++i) {
          int nblk;
          const RecOp& o = works_[i]->ops[r][q];
          tab[(size_t)r * np + i] = l1_args(o.l1, o.l1w_dev, &nblk, np);
          if (r == 0) pre[i + 1] = pre[i] + nblk;
        }
      ot.tab_off = b.add(tab);
    }
    ot.pre_off = b.add(pre);
    ot.total = pre[np];
    vt_.push_back(ot);
  }
  // Helmholtz tables: w = A Z_j (one row per position), r = f - A u
  {
    std::vector<HArgs> tab((size_t)m_ * np);
    for (int r = 0; r < m_; ++r)
      for (int i = 0; i < np; ++i) {
        const Work* w = works_[i];
        tab[(size_t)r * np + i] =
            HArgs{w->c->helm(), w->slot->Z + 2LL * r * w->c->ext.total, nullptr, w->slot->wv, nullptr};
      }
    hmv_off_ = b.add(tab);
  }
  {
    std::vector<HArgs> tab(np);
    for (int i = 0; i < np; ++i) {
      const Work* w = works_[i];
      tab[i] = HArgs{w->c->helm(), w->u, w->f, w->slot->rv, w->slot->partial};
    }
    hres_off_ = b.add(tab);
  }
  std::vector<int> pre_red(np + 1, 0), pre_elem(np + 1, 0);
  std::vector<KArgs> kargs(np);
  for (int i = 0; i < np; ++i) {
    const Work* w = works_[i];
    const Slot& sl = *w->slot;
    pre_red[i + 1] = pre_red[i] + red_blocks(w->c->ext.total);
    pre_elem[i + 1] = pre_elem[i] + elem_blocks(w->c->ext.total);
    KArgs& k = kargs[i];
    k.V = sl.V; k.Z = sl.Z; k.w = sl.wv; k.r = sl.rv; k.f = w->f; k.u = w->u;
    k.H = sl.H; k.cs = sl.cs; k.sn = sl.sn; k.g = sl.g; k.y = sl.y; k.coef = sl.coef;
    k.partial = sl.partial; k.scal = sl.scal; k.skip = sl.skip;
    k.N = w->c->ext.total; k.ldh = m_ + 1; k.always_two = w->c->ortho == 1;
  }
  karg_off_ = b.add(kargs);
  pre_red_off_ = b.add(pre_red);
  pre_elem_off_ = b.add(pre_elem);
  total_red_ = pre_red[np];
  total_elem_ = pre_elem[np];
  const size_t ctl_off = b.add(std::vector<int>((size_t)M_COUNT * np, 0));
  const size_t gather_off = b.add(std::vector<double>(4 * (size_t)np, 0.0));
  if (b.host.size() > dev_cap_) {
    if (dev_) { (void)hipFree(dev_); dev_ = nullptr; dev_cap_ = 0; }
    const size_t cap = b.host.size() + b.host.size() / 2;
    if (hipMalloc(&dev_, cap) != hipSuccess) {
      (void)hipGetLastError();
      dev_ = nullptr;
      dirty_ = true;
      return fail(MCMG_E_OOM, "batch tables");
    }
    dev_cap_ = cap;
  }
  if (np > host_cap_) {
    if (ctl_host_) (void)hipHostFree(ctl_host_);
    if (gather_host_) (void)hipHostFree(gather_host_);
    ctl_host_ = nullptr; gather_host_ = nullptr; host_cap_ = 0;
    if (hipHostMalloc((void**)&ctl_host_, (size_t)M_COUNT * np * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&gather_host_, 4 * (size_t)np * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      dirty_ = true;
      return fail(MCMG_E_OOM, "pinned host buffers");
    }
    host_cap_ = np;
  }
  ctl_dev_ = (int*)((unsigned char*)dev_ + ctl_off);
  gather_dev_ = (double*)((unsigned char*)dev_ + gather_off);
  if (hipMemcpyAsync(dev_, b.host.data(), b.host.size(), hipMemcpyHostToDevice, s_) != hipSuccess ||
      hipStreamSynchronize(s_) != hipSuccess) {
    dirty_ = true;
    return fail(MCMG_E_HIP, "batch table upload");
  }
  return MCMG_OK;
}

// The launches of one tick.  all_phases: issue every phase even when no Work
// is in it (a captured tick must cover every state mix).
hipError_t Engine::body(bool all_phases) {
  const int np = np_;
  int n_init = 0, n_end = 0, n_iter = 0;
  for (const Work* w : works_) {
    n_init += w->st == Work::INIT;
    n_end += w->st == Work::END;
    n_iter += w->st == Work::ITER;
  }
  auto at = [&](size_t off) { return (const void*)((const unsigned char*)dev_ + off); };
  const int* mask_iter = ctl_dev_ + M_ITER * np;
  const int* mask_end = ctl_dev_ + M_END * np;
  const int* mask_res = ctl_dev_ + M_RES * np;
  const int* mask_init = ctl_dev_ + M_INIT * np;
  const int* jpos = ctl_dev_ + M_JPOS * np;
  KBatch kb;
  kb.tab = (const KArgs*)at(karg_off_);
  kb.np = np;
  kb.pre_red = (const int*)at(pre_red_off_);
  kb.total_red = total_red_;
  kb.pre_elem = (const int*)at(pre_elem_off_);
  kb.total_elem = total_elem_;
  kb.jpos = jpos;
  kb.kk = ctl_dev_ + M_KK * np;
  kb.gather = gather_dev_;
  hipError_t e;
#define ECK(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
  if (all_phases || n_init) {
    kb.frozen = mask_init;
    ECK(kb_launch(KB_FNORM_PARTIAL, kb, 0, m_, s_));
    ECK(kb_launch(KB_FNORM_REDUCE, kb, 0, m_, s_));
  }
  if (all_phases || n_end) {
    kb.frozen = mask_end;
    ECK(kb_launch(KB_BACKSOLVE, kb, 0, m_, s_));
    ECK(kb_launch(KB_ZUPDATE, kb, 0, m_, s_));
  }
  if (all_phases || n_init || n_end) {
    BatchLaunch bl{at(hres_off_), kb.pre_red, np, total_red_, mask_res};
    ECK(launch_helm_batched(dim_, T_F64, bl, s_));
    kb.frozen = mask_res;
    ECK(kb_launch(KB_REDUCE_SUM, kb, 0, m_, s_));
    ECK(kb_launch(KB_SCALE_R, kb, 0, m_, s_));
    ECK(kb_launch(KB_CYCLE_INIT, kb, 0, m_, s_));
  }
  if (all_phases || n_iter) {
    for (const OpTable& ot : vt_) {
      BatchLaunch bl{at(ot.tab_off), (const int*)at(ot.pre_off), np, ot.total, mask_iter,
                     ot.jdep ? jpos : nullptr};
      if (ot.kind == 0) ECK(launch_conv_batched(ot.proto.conv, bl, s_));
      else if (ot.kind == 1) ECK(launch_conv_mfma_batched(ot.proto.mf, bl, s_));
      else if (ot.kind == 3) ECK(launch_step_batched(ot.proto.st, bl, s_));
      else ECK(launch_level1_batched(dim_, ot.proto.l1.var, bl, s_));
    }
    BatchLaunch bl{at(hmv_off_), kb.pre_red, np, total_red_, mask_iter, jpos};
    ECK(launch_helm_batched(dim_, T_F32, bl, s_));
    kb.frozen = mask_iter;
    for (int pass = 0; pass < 2; ++pass) {
      ECK(kb_launch(KB_MULTIDOT, kb, pass, m_, s_));
      ECK(kb_launch(KB_REDUCE_DOTS, kb, pass, m_, s_));
      ECK(kb_launch(KB_UPDATE, kb, pass, m_, s_));
      // the second pass's norm reduce runs inside the Givens launch
      if (pass == 0) ECK(kb_launch(KB_REDUCE_NORM, kb, pass, m_, s_));
    }
    ECK(kb_launch(KB_GIVENS, kb, 0, m_, s_));
    ECK(kb_launch(KB_SCALE_W, kb, 0, m_, s_));
  }
#undef ECK
  return hipMemcpyAsync(gather_host_, gather_dev_, 4 * (size_t)np * sizeof(double),
                        hipMemcpyDeviceToHost, s_);
}

mcmg_status Engine::issue() {
  if (issued_) return fail(MCMG_E_ARG, "engine tick already issued");
  if (dirty_) {
    mcmg_status st = build();
    if (st != MCMG_OK) return st;
  }
  const int np = np_;
  if (np == 0 || live() == 0) return MCMG_OK;
  for (int i = 0; i < np; ++i) {
    const Work* w = works_[i];
    ctl_host_[M_ITER * np + i] = w->st != Work::ITER;
    ctl_host_[M_END * np + i] = w->st != Work::END;
    ctl_host_[M_RES * np + i] = !(w->st == Work::INIT || w->st == Work::END);
    ctl_host_[M_INIT * np + i] = w->st != Work::INIT;
    ctl_host_[M_JPOS * np + i] = w->st == Work::ITER ? w->j : 0;
    ctl_host_[M_KK * np + i] = w->st == Work::END ? w->k : 0;
  }
  if (hipMemcpyAsync(ctl_dev_, ctl_host_, (size_t)M_COUNT * np * sizeof(int), hipMemcpyHostToDevice, s_) != hipSuccess)
    return fail(MCMG_E_HIP, "control upload");
  hipError_t e = hipSuccess;
  if (use_graphs && (graph_ || ticks_same_ >= 1)) {
    if (!graph_) {
      hipGraph_t g = nullptr;
      e = hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return fail(MCMG_E_HIP, "capture: %s", hipGetErrorString(e));
      hipError_t ce = body(true);
      e = hipStreamEndCapture(s_, &g);
      if (ce != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(MCMG_E_HIP, "capture: %s", hipGetErrorString(ce != hipSuccess ? ce : e));
      }
      e = hipGraphInstantiate(&graph_, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) { graph_ = nullptr; return fail(MCMG_E_HIP, "instantiate: %s", hipGetErrorString(e)); }
    }
    e = hipGraphLaunch(graph_, s_);
  } else {
    e = body(false);
  }
  if (e != hipSuccess) return fail(MCMG_E_HIP, "tick: %s", hipGetErrorString(e));
  ++ticks_same_;
  issued_ = true;
  return MCMG_OK;
}

mcmg_status Engine::complete(std::vector<Work*>* finished) {
  if (!issued_) return MCMG_OK;
  issued_ = false;
  if (hipStreamSynchronize(s_) != hipSuccess) return fail(MCMG_E_HIP, "tick sync");
  const double* g = gather_host_;
  bool zeroed = false;
  auto finish = [&](Work* w, mcmg_status st) {
    w->st = Work::DONE;
    w->status = st;
    if (finished) finished->push_back(w);
  };
  auto settle = [&](Work* w, double beta) {
    w->relres = beta / w->fnorm;
    if (!std::isfinite(beta)) finish(w, fail(MCMG_E_NONFINITE, "non-finite residual"));
    else if (beta <= w->target) finish(w, MCMG_OK);
    else if (w->its >= w->maxit) finish(w, MCMG_NOT_CONVERGED);
    else { w->st = Work::ITER; w->j = 0; }
  };
  for (int i = 0; i < np_; ++i) {
    Work* w = works_[i];
    switch (w->st) {
      case Work::INIT: {
        w->fnorm = std::sqrt(g[4 * i]);
        if (!std::isfinite(w->fnorm)) {
          finish(w, fail(MCMG_E_NONFINITE, "non-finite right-hand side"));
        } else if (w->fnorm == 0.0) {
          if (launch_zero_f64(w->u, 2 * w->c->ext.total, s_) != hipSuccess)
            return fail(MCMG_E_HIP, "zero solution");
          zeroed = true;
          finish(w, MCMG_OK);
        } else {
          w->target = w->tol * w->fnorm;
          settle(w, g[4 * i + 3]);
        }
        break;
      }
      case Work::END:
        ++w->restarts;
        settle(w, g[4 * i + 3]);
        break;
      case Work::ITER: {
        const double rho = g[4 * i], hn = g[4 * i + 1], cn = g[4 * i + 2], diag = g[4 * i + 3];
        ++w->its;
        w->hist.push_back(rho / w->fnorm);
        w->relest = rho / w->fnorm;
        w->k = w->j + 1;
        if (!std::isfinite(rho) || !std::isfinite(hn)) {
          finish(w, fail(MCMG_E_NONFINITE, "non-finite value in the Arnoldi process"));
        } else if (diag == 0.0) {
          // column j is zero after the earlier rotations: close the cycle
          // with the columns before it, or stop (u unchanged) when none is left
          w->k = w->j;
          if (w->k == 0) finish(w, MCMG_NOT_CONVERGED);
          else w->st = Work::END;
        } else if (rho <= w->target || hn <= 1e-14 * cn || w->its >= w->maxit || w->j + 1 == m_) {
          w->st = Work::END;
        } else {
          ++w->j;
        }
        break;
      }
      case Work::DONE:
        break;
    }
  }
  if (zeroed && hipStreamSynchronize(s_) != hipSuccess) return fail(MCMG_E_HIP, "tick sync");
  return MCMG_OK;
}

}  // namespace mcmg
