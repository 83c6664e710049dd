// Training of the McMg weights on the GPU: the loss L_H of the training
// section (Eq. loss_fun), its gradient by reverse accumulation through Alg. 1
// and Alg. 2, and the Adam update; LLPF (Sec. llpf) freezes tensors.
//
// Forward: the setup network with its pre-activations kept, then the V-cycle
// of Alg. 2 with the unfused VALU convolutions.  The tape records, per level
// and smoothing step:
//   - e before the step;
//   - t = r - A_l e (the step's operator residual);
//   - u = s (.) (KS * t);
// plus the restriction input and e after the down steps.  The loss of one
// sample is |A z - r| / |r| with A in FP64.  Its gradient with respect to
// the two real channels of z is A^H (A z - r) / (B |A z - r| |r|).
//
// Backward runs the operations in reverse.  Data gradients use the same
// convolution kernels with adjoint weight layouts: S1 is the stride-1
// convolution with reversed taps and swapped channels; S2 and T2 are each
// other's adjoints with the same tensor.  The W and KA adjoints carry the
// minus sign of t = r - W e - a (.) (KA e).  Weight gradients come from
// wgrad (train.hip).  Gradients of a_l, s_l then flow back through the
// setup network's GELUs.
//
// All handles of one training step share the master handle's parameters
// (hs[0]).  Gradients of every sample accumulate in the master's buffer and
// Adam updates the master; the other handles copy its parameters at the
// start of the next step.  The matrix-core packs, the level-1 sweep weights
// and the cached features of inference go stale until mcmg_train_commit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "mcmg.h"
#include "runtime.h"

namespace mcmg {

namespace {

enum { K_FLIFT = 0, K_GLIFT, K_GPROJ, K_FS, K_W, K_KA, K_KS, K_WSM, K_FA, K_R, K_P };

int rup(int v, int m) { return (v + m - 1) / m * m; }

#define TCK(x)                                  \
  do {                                          \
    hipError_t e_ = (x);                        \
    if (e_ != hipSuccess) return e_;            \
  } while (0)

}  // namespace

mcmg_status Ctx::train_init() {
  if (train) return MCMG_OK;
  TrainState* T = new TrainState();
  const int taps = dim == 2 ? 9 : 27;
  size_t off = 0;
  std::vector<int> wsm_seen(L, 0);
  for (const HostTensor& h : host_w) {
    TTensor t;
    t.kind = h.kind; t.level = h.level; t.step = h.step; t.d0 = h.d0; t.d1 = h.d1;
    t.mode = (h.kind == K_FA || h.kind == K_R) ? CONV_S2 : h.kind == K_P ? CONV_T2 : CONV_S1;
    t.off = off;
    t.len = (size_t)h.d0 * h.d1 * taps;
    off += t.len;
    Level* lv = h.level > 0 ? &lev[h.level - 1] : nullptr;
    switch (h.kind) {
      case K_FLIFT: t.fwd = &w_flift; break;
      case K_GLIFT: t.fwd = &w_glift; break;
      case K_GPROJ: t.fwd = &w_gproj; break;
      case K_FS: t.fwd = &lv->w_fs; break;
      case K_W: t.fwd = &lv->w_W; break;
      case K_KA: t.fwd = &lv->w_KA; break;
      case K_KS: t.fwd = &lv->w_KS; break;
      case K_WSM: t.fwd = &lv->w_sm[h.step - 1]; break;
      case K_FA: t.fwd = &lv->w_fa; break;
      case K_R: t.fwd = &lv->w_R; break;
      case K_P: t.fwd = &lv->w_P; break;
    }
    // adjoint convolution (the inputs m and r of f_lift / g_lift need none):
    // S1 and S2 tensors map d0 -> d1, P (T2) maps d1 -> d0
    if (h.kind != K_FLIFT && h.kind != K_GLIFT) {
      t.adj_cin = t.mode == CONV_T2 ? h.d1 : h.d0;
      t.adj_cout = t.mode == CONV_T2 ? h.d0 : h.d1;
      t.adj = (float*)alloc((size_t)taps * t.adj_cin * rup(t.adj_cout, conv_chunk(t.adj_cout)) *
                            sizeof(float));
      if (!t.adj) { delete T; return fail(MCMG_E_OOM, "training allocation failed"); }
    }
    T->ts.push_back(t);
  }
  T->n = off;
  auto fbuf = [&](size_t n) { return (float*)alloc(std::max<size_t>(n, 1) * sizeof(float)); };
  T->theta = fbuf(off); T->grad = fbuf(off); T->m = fbuf(off); T->v = fbuf(off);
  bool ok = T->theta && T->grad && T->m && T->v;
  for (const TTensor& t : T->ts) {
    const HostTensor& h = host_w[&t - &T->ts[0]];
    if (ok && hipMemcpy(T->theta + t.off, h.w.data(), t.len * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
      ok = false;
  }
  if (ok) ok = launch_zero_f32(T->m, off, stream) == hipSuccess && launch_zero_f32(T->v, off, stream) == hipSuccess;
  const long long N1 = lev[0].dims.total;
  T->z_lift = fbuf(N1 * lev[0].C);
  T->z2 = fbuf(2 * N1); T->dz2 = fbuf(2 * N1); T->rin32 = fbuf(2 * N1);
  T->wres = (double*)alloc(2 * N1 * sizeof(double));
  T->ahw = (double*)alloc(2 * N1 * sizeof(double));
  ok = ok && T->z_lift && T->z2 && T->dz2 && T->rin32 && T->wres && T->ahw;
  size_t part = 0;
  for (int l = 0; ok && l < L; ++l) {
    Level& lv = lev[l];
    const size_t n = (size_t)lv.dims.total * lv.C;
    const int ns = (int)lv.w_sm.size();
    T->z_s.push_back(fbuf(n));
    T->z_a.push_back(l < L - 1 ? fbuf((size_t)lev[l + 1].dims.total * lev[l + 1].C) : nullptr);
    T->te.push_back({}); T->tt.push_back({}); T->tu.push_back({});
    for (int i = 0; i < ns; ++i) {
      T->te[l].push_back(fbuf(n)); T->tt[l].push_back(fbuf(n)); T->tu[l].push_back(fbuf(n));
      ok = ok && T->te[l][i] && T->tt[l][i] && T->tu[l][i];
    }
    T->rr.push_back(l < L - 1 ? fbuf(n) : nullptr);
    T->edown.push_back(l < L - 1 ? fbuf(n) : nullptr);
    for (auto* v : {&T->gde, &T->gdr, &T->gda, &T->gds, &T->t1, &T->t2, &T->t3}) {
      v->push_back(fbuf(n));
      ok = ok && v->back();
    }
    ok = ok && T->z_s[l] && (l == L - 1 || (T->z_a[l] && T->rr[l] && T->edown[l]));
    // largest weight-gradient partial buffer: 64 chunks of taps C_in C_out
    const int cmax = std::max(lv.C, l < L - 1 ? lev[l + 1].C : lv.C);
    part = std::max(part, (size_t)64 * taps * cmax * cmax);
  }
  part = std::max(part, (size_t)64 * taps * 2 * lev[0].C);
  T->part = fbuf(part);
  T->part_cap = part;
  if (!ok || !T->part) {
    delete T;
    return fail(MCMG_E_OOM, "training allocation failed");
  }
  train = T;
  if (train_sync_weights() != hipSuccess) return fail(MCMG_E_HIP, "training weight layout");
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(MCMG_E_HIP, "training init");
  return MCMG_OK;
}

hipError_t Ctx::train_sync_weights() {
  TrainState* T = train;
  const int taps = dim == 2 ? 9 : 27;
  for (const TTensor& t : T->ts) {
    const bool tr = t.mode == CONV_T2;
    const int cin = tr ? t.d0 : t.d1, cout = tr ? t.d1 : t.d0;
    TCK(launch_repack(T->theta + t.off, t.d0, t.d1, taps, tr ? 1 : 0, 0, 1.f, cin,
                      rup(cout, conv_chunk(cout)), *t.fwd, stream));
    if (t.adj) {
      const float sc = (t.kind == K_W || t.kind == K_KA) ? -1.f : 1.f;
      TCK(launch_repack(T->theta + t.off, t.d0, t.d1, taps, tr ? 0 : 1, t.mode == CONV_S1 ? 1 : 0,
                        sc, t.adj_cin, rup(t.adj_cout, conv_chunk(t.adj_cout)), t.adj, stream));
    }
  }
  return hipSuccess;
}

hipError_t Ctx::wgrad(int mode, int tx, const void* x, const Dims& in, int cin, const float* dy,
                      const Dims& out, int cout, const TTensor& t, float scale) {
  if (!t.train) return hipSuccess;
  TrainState* T = train;
  WgArgs a{};
  a.dim = dim; a.mode = mode; a.tx = tx; a.x = x; a.dy = dy; a.cin = cin; a.cout = cout;
  a.in = in; a.out = out; a.dw = T->grad + t.off; a.scale = scale; a.part = T->part;
  a.fo1 = make_fastdiv((uint32_t)out.n[1]);
  a.fo2 = make_fastdiv((uint32_t)out.n[2]);
  a.chunk = std::max<long long>(256, (out.total + 63) / 64);
  a.nchunk = (int)((out.total + a.chunk - 1) / a.chunk);
  if ((size_t)wgrad_part_floats(a) > T->part_cap) return hipErrorInvalidValue;
  return launch_wgrad(a, stream);
}

namespace {
const TTensor& find_t(const TrainState* T, int kind, int level, int step) {
  for (const TTensor& t : T->ts)
    if (t.kind == kind && t.level == level && t.step == step) return t;
  return T->ts[0];   // unreachable for a parsed blob
}
}  // namespace

hipError_t Ctx::train_forward(const double* rin) {
  TrainState* T = train;
  hipStream_t s = stream;
  Level& l1 = lev[0];
  const long long N1 = l1.dims.total;
  // Alg. 1 with the pre-activations kept
  TCK(conv(CONV_S1, EPI_SET, T_F32, mfeat, l1.dims, 1, w_flift, nullptr, T_F32, T->z_lift, l1.dims,
           l1.C, nullptr, nullptr));
  TCK(launch_gelu_fwd(T->z_lift, l1.a, N1 * l1.C, s));
  for (int l = 0; l < L; ++l) {
    Level& lv = lev[l];
    const long long n = lv.dims.total * lv.C;
    TCK(conv(CONV_S1, EPI_SET, T_F32, lv.a, lv.dims, lv.C, lv.w_fs, nullptr, T_F32, T->z_s[l],
             lv.dims, lv.C, nullptr, nullptr));
    TCK(launch_gelu_fwd(T->z_s[l], lv.s, n, s));
    if (l < L - 1) {
      Level& nx = lev[l + 1];
      TCK(conv(CONV_S2, EPI_SET, T_F32, lv.a, lv.dims, lv.C, lv.w_fa, nullptr, T_F32, T->z_a[l],
               nx.dims, nx.C, nullptr, nullptr));
      TCK(launch_gelu_fwd(T->z_a[l], nx.a, nx.dims.total * nx.C, s));
    }
  }
  // Alg. 2 with the tape
  TCK(launch_c2f(rin, T->rin32, N1, 1.0, s));
  TCK(conv(CONV_S1, EPI_SET, T_F32, T->rin32, l1.dims, 2, w_glift, nullptr, T_F32, l1.r, l1.dims,
           l1.C, nullptr, nullptr));
  auto step = [&](int l, int i, bool first) -> hipError_t {
    Level& lv = lev[l];
    const size_t nb = (size_t)lv.dims.total * lv.C * sizeof(float);
    if (first) {
      TCK(conv(CONV_S1, EPI_MUL, T_F32, lv.r, lv.dims, lv.C, lv.w_KS, nullptr, T_F32, T->tu[l][i],
               lv.dims, lv.C, nullptr, lv.s));
      return conv(CONV_S1, EPI_SET, T_F32, T->tu[l][i], lv.dims, lv.C, lv.w_sm[i], nullptr, T_F32,
                  lv.e, lv.dims, lv.C, nullptr, nullptr);
    }
    TCK(hipMemcpyAsync(T->te[l][i], lv.e, nb, hipMemcpyDeviceToDevice, s));
    TCK(conv(CONV_S1, EPI_RESID, T_F32, lv.e, lv.dims, lv.C, lv.w_W, lv.w_KA, T_F32, T->tt[l][i],
             lv.dims, lv.C, lv.r, lv.a));
    TCK(conv(CONV_S1, EPI_MUL, T_F32, T->tt[l][i], lv.dims, lv.C, lv.w_KS, nullptr, T_F32,
             T->tu[l][i], lv.dims, lv.C, nullptr, lv.s));
    return conv(CONV_S1, EPI_ADD, T_F32, T->tu[l][i], lv.dims, lv.C, lv.w_sm[i], nullptr, T_F32,
                lv.e, lv.dims, lv.C, nullptr, nullptr);
  };
  for (int l = 0; l < L; ++l) {
    Level& lv = lev[l];
    const long long n = lv.dims.total * lv.C;
    if (lv.nu1 == 0) TCK(launch_zero_f32(lv.e, n, s));
    for (int i = 0; i < lv.nu1; ++i) TCK(step(l, i, i == 0));
    if (l < L - 1) {
      Level& nx = lev[l + 1];
      TCK(hipMemcpyAsync(T->edown[l], lv.e, n * sizeof(float), hipMemcpyDeviceToDevice, s));
      TCK(conv(CONV_S1, EPI_RESID, T_F32, lv.e, lv.dims, lv.C, lv.w_W, lv.w_KA, T_F32, T->rr[l],
               lv.dims, lv.C, lv.r, lv.a));
      TCK(conv(CONV_S2, EPI_SET, T_F32, T->rr[l], lv.dims, lv.C, lv.w_R, nullptr, T_F32, nx.r,
               nx.dims, nx.C, nullptr, nullptr));
    }
  }
  for (int l = L - 2; l >= 0; --l) {
    Level& lv = lev[l];
    Level& nx = lev[l + 1];
    TCK(conv(CONV_T2, EPI_ADD, T_F32, nx.e, nx.dims, nx.C, lv.w_P, nullptr, T_F32, lv.e, lv.dims,
             lv.C, nullptr, nullptr));
    for (int i = lv.nu1; i < lv.nu1 + lv.nu2; ++i) TCK(step(l, i, false));
  }
  return conv(CONV_S1, EPI_SET, T_F32, l1.e, l1.dims, l1.C, w_gproj, nullptr, T_F32, T->z2, l1.dims,
              2, nullptr, nullptr);
}

hipError_t Ctx::train_backward() {
  TrainState* T = train;
  hipStream_t s = stream;
  Level& l1 = lev[0];
  for (int l = 0; l < L; ++l) {
    const long long n = lev[l].dims.total * lev[l].C;
    for (float* p : {T->gde[l], T->gdr[l], T->gda[l], T->gds[l]}) TCK(launch_zero_f32(p, n, s));
  }
  auto adj_conv = [&](int mode, int epi, const float* x, const Dims& in, const TTensor& t, float* y,
                      const Dims& out) {
    return conv(mode, epi, T_F32, x, in, t.adj_cin, t.adj, nullptr, T_F32, y, out, t.adj_cout,
                nullptr, nullptr);
  };
  // one smoothing step in reverse: g = dL/de after the step on entry, dL/de before on exit
  auto step_back = [&](int l, int i, bool first) -> hipError_t {
    Level& lv = lev[l];
    const int lvl = l + 1;
    const long long n = lv.dims.total * lv.C;
    const Dims& d = lv.dims;
    float* g = T->gde[l];
    const float* u = T->tu[l][i];
    const float* t = first ? lv.r : T->tt[l][i];
    const TTensor& tsm = find_t(T, K_WSM, lvl, i + 1);
    const TTensor& tks = find_t(T, K_KS, lvl, 0);
    TCK(wgrad(CONV_S1, T_F32, u, d, lv.C, g, d, lv.C, tsm, 1.f));
    TCK(adj_conv(CONV_S1, EPI_SET, g, d, tsm, T->t1[l], d));          // du
    TCK(conv(CONV_S1, EPI_SET, T_F32, t, d, lv.C, lv.w_KS, nullptr, T_F32, T->t2[l], d, lv.C,
             nullptr, nullptr));                                      // v = KS * t
    TCK(launch_mul(T->gds[l], T->t1[l], T->t2[l], n, 1.f, 1, s));     // ds += du (.) v
    TCK(launch_mul(T->t1[l], lv.s, T->t1[l], n, 1.f, 0, s));          // dv = s (.) du
    TCK(wgrad(CONV_S1, T_F32, t, d, lv.C, T->t1[l], d, lv.C, tks, 1.f));
    TCK(adj_conv(CONV_S1, EPI_SET, T->t1[l], d, tks, T->t2[l], d));   // dt
    TCK(launch_axpy(T->gdr[l], T->t2[l], n, 1.f, s));
    if (first) return hipSuccess;
    const float* e = T->te[l][i];
    const TTensor& tw = find_t(T, K_W, lvl, 0);
    const TTensor& tka = find_t(T, K_KA, lvl, 0);
    TCK(wgrad(CONV_S1, T_F32, e, d, lv.C, T->t2[l], d, lv.C, tw, -1.f));
    TCK(conv(CONV_S1, EPI_SET, T_F32, e, d, lv.C, lv.w_KA, nullptr, T_F32, T->t3[l], d, lv.C,
             nullptr, nullptr));                                      // q = KA * e
    TCK(launch_mul(T->gda[l], T->t2[l], T->t3[l], n, -1.f, 1, s));    // da -= dt (.) q
    TCK(launch_mul(T->t3[l], lv.a, T->t2[l], n, 1.f, 0, s));          // a (.) dt
    TCK(wgrad(CONV_S1, T_F32, e, d, lv.C, T->t3[l], d, lv.C, tka, -1.f));
    TCK(adj_conv(CONV_S1, EPI_ADD, T->t2[l], d, tw, g, d));           // g -= W^T dt
    return adj_conv(CONV_S1, EPI_ADD, T->t3[l], d, tka, g, d);        // g -= KA^T (a (.) dt)
  };
  // projection z = g_proj * e_1
  const TTensor& tproj = find_t(T, K_GPROJ, 0, 0);
  TCK(wgrad(CONV_S1, T_F32, l1.e, l1.dims, l1.C, T->dz2, l1.dims, 2, tproj, 1.f));
  TCK(adj_conv(CONV_S1, EPI_ADD, T->dz2, l1.dims, tproj, T->gde[0], l1.dims));
  // up cycle in reverse: post steps, then the prolongation e_l += P e_{l+1}
  for (int l = 0; l < L - 1; ++l) {
    Level& lv = lev[l];
    Level& nx = lev[l + 1];
    for (int i = lv.nu1 + lv.nu2 - 1; i >= lv.nu1; --i) TCK(step_back(l, i, false));
    const TTensor& tp = find_t(T, K_P, l + 1, 0);
    TCK(wgrad(CONV_T2, T_F32, nx.e, nx.dims, nx.C, T->gde[l], lv.dims, lv.C, tp, 1.f));
    TCK(adj_conv(CONV_S2, EPI_ADD, T->gde[l], lv.dims, tp, T->gde[l + 1], nx.dims));
  }
  {
    Level& lc = lev[L - 1];
    for (int i = lc.nu1 - 1; i >= 0; --i) TCK(step_back(L - 1, i, i == 0));
  }
  // down cycle in reverse: restriction r_{l+1} = R (r_l - A_l e), then the pre steps
  for (int l = L - 2; l >= 0; --l) {
    Level& lv = lev[l];
    Level& nx = lev[l + 1];
    const int lvl = l + 1;
    const long long n = lv.dims.total * lv.C;
    const Dims& d = lv.dims;
    const TTensor& tr = find_t(T, K_R, lvl, 0);
    const TTensor& tw = find_t(T, K_W, lvl, 0);
    const TTensor& tka = find_t(T, K_KA, lvl, 0);
    TCK(wgrad(CONV_S2, T_F32, T->rr[l], d, lv.C, T->gdr[l + 1], nx.dims, nx.C, tr, 1.f));
    TCK(adj_conv(CONV_T2, EPI_SET, T->gdr[l + 1], nx.dims, tr, T->t1[l], d));   // d rr
    TCK(launch_axpy(T->gdr[l], T->t1[l], n, 1.f, s));
    const float* e = T->edown[l];
    TCK(wgrad(CONV_S1, T_F32, e, d, lv.C, T->t1[l], d, lv.C, tw, -1.f));
    TCK(conv(CONV_S1, EPI_SET, T_F32, e, d, lv.C, lv.w_KA, nullptr, T_F32, T->t2[l], d, lv.C,
             nullptr, nullptr));
    TCK(launch_mul(T->gda[l], T->t1[l], T->t2[l], n, -1.f, 1, s));
    TCK(launch_mul(T->t3[l], lv.a, T->t1[l], n, 1.f, 0, s));
    TCK(wgrad(CONV_S1, T_F32, e, d, lv.C, T->t3[l], d, lv.C, tka, -1.f));
    TCK(adj_conv(CONV_S1, EPI_ADD, T->t1[l], d, tw, T->gde[l], d));
    TCK(adj_conv(CONV_S1, EPI_ADD, T->t3[l], d, tka, T->gde[l], d));
    for (int i = lv.nu1 - 1; i >= 0; --i) TCK(step_back(l, i, i == 0));
  }
  // lift r_1 = g_lift * r
  TCK(wgrad(CONV_S1, T_F32, T->rin32, l1.dims, 2, T->gdr[0], l1.dims, l1.C,
            find_t(T, K_GLIFT, 0, 0), 1.f));
  // setup network in reverse (Alg. 1): s_l = GELU(f_s * a_l), a_{l+1} = GELU(f_a *2 a_l)
  for (int l = L - 1; l >= 0; --l) {
    Level& lv = lev[l];
    const int lvl = l + 1;
    const long long n = lv.dims.total * lv.C;
    if (l < L - 1) {
      Level& nx = lev[l + 1];
      const TTensor& tfa = find_t(T, K_FA, lvl, 0);
      TCK(launch_gelu_bwd(T->gda[l + 1], T->z_a[l], T->t1[l + 1], nx.dims.total * nx.C, s));
      TCK(wgrad(CONV_S2, T_F32, lv.a, lv.dims, lv.C, T->t1[l + 1], nx.dims, nx.C, tfa, 1.f));
      TCK(adj_conv(CONV_T2, EPI_ADD, T->t1[l + 1], nx.dims, tfa, T->gda[l], lv.dims));
    }
    const TTensor& tfs = find_t(T, K_FS, lvl, 0);
    TCK(launch_gelu_bwd(T->gds[l], T->z_s[l], T->t2[l], n, s));
    TCK(wgrad(CONV_S1, T_F32, lv.a, lv.dims, lv.C, T->t2[l], lv.dims, lv.C, tfs, 1.f));
    TCK(adj_conv(CONV_S1, EPI_ADD, T->t2[l], lv.dims, tfs, T->gda[l], lv.dims));
  }
  TCK(launch_gelu_bwd(T->gda[0], T->z_lift, T->t3[0], l1.dims.total * l1.C, s));
  return wgrad(CONV_S1, T_F32, mfeat, l1.dims, 1, T->t3[0], l1.dims, l1.C,
               find_t(T, K_FLIFT, 0, 0), 1.f);
}

mcmg_status Ctx::repack_inference() {
  // host copies of the trained parameters, then every derived form
  TrainState* T = train;
  if (!T) return MCMG_OK;
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(MCMG_E_HIP, "commit sync");
  for (size_t k = 0; k < T->ts.size(); ++k) {
    const TTensor& t = T->ts[k];
    if (hipMemcpy(host_w[k].w.data(), T->theta + t.off, t.len * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(MCMG_E_HIP, "commit download");
    for (float v : host_w[k].w)
      if (!std::isfinite(v)) return fail(MCMG_E_NONFINITE, "non-finite trained weight");
  }
  mcmg_status st = refresh_packed();
  if (st != MCMG_OK) return st;
  if (run_setup() != hipSuccess) return fail(MCMG_E_HIP, "commit setup");
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(MCMG_E_HIP, "commit sync");
  return MCMG_OK;
}

}  // namespace mcmg

using namespace mcmg;

namespace {

mcmg_status train_batch(mcmg_handle* hs, int nh, const double* const* r, const mcmg_adam* opt,
                        double* loss, float* grad_out, size_t ngrad) {
  if (!hs || nh < 1 || !r) return fail(MCMG_E_ARG, "null argument");
  Ctx* M = (Ctx*)hs[0];
  for (int i = 0; i < nh; ++i) {
    Ctx* c = (Ctx*)hs[i];
    if (!c || !r[i]) return fail(MCMG_E_ARG, "null handle or residual");
    if (c->dim != M->dim || c->L != M->L || c->host_w.size() != M->host_w.size())
      return fail(MCMG_E_ARG, "training handles must share one model");
    for (int l = 0; l < M->L; ++l)
      if (c->lev[l].C != M->lev[l].C || c->lev[l].nu1 != M->lev[l].nu1 || c->lev[l].nu2 != M->lev[l].nu2)
        return fail(MCMG_E_ARG, "training handles must share one model");
    const mcmg_status st = c->train_init();
    if (st != MCMG_OK) return st;
  }
  TrainState* TM = M->train;
  auto hck = [](hipError_t e, const char* what) {
    return e == hipSuccess ? MCMG_OK : fail(MCMG_E_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  mcmg_status st;
  if ((st = hck(hipStreamSynchronize(M->stream), "train sync")) != MCMG_OK) return st;
  if ((st = hck(launch_zero_f32(TM->grad, TM->n, M->stream), "train zero")) != MCMG_OK) return st;
  double total = 0.0;
  for (int i = 0; i < nh; ++i) {
    Ctx* c = (Ctx*)hs[i];
    TrainState* T = c->train;
    hipStream_t s = c->stream;
    if (c != M) {
      if ((st = hck(hipStreamSynchronize(M->stream), "train sync")) != MCMG_OK) return st;
      if ((st = hck(hipMemcpyAsync(T->theta, TM->theta, TM->n * sizeof(float), hipMemcpyDeviceToDevice, s), "train copy")) != MCMG_OK) return st;
      if ((st = hck(c->train_sync_weights(), "train layout")) != MCMG_OK) return st;
      if ((st = hck(launch_zero_f32(T->grad, T->n, s), "train zero")) != MCMG_OK) return st;
    }
    if ((st = hck(c->train_forward(r[i]), "train forward")) != MCMG_OK) return st;
    // w' = r - A z (FP64) and its norm; |r|
    const long long N = c->ext.total;
    HelmOp op = c->helm();
    if ((st = hck(launch_helm(op, T_F32, T->z2, r[i], T->wres, c->partial, s), "train residual")) != MCMG_OK) return st;
    if ((st = hck(launch_reduce_sum(c->partial, helm_blocks(op), c->scal + 2, s), "train norm")) != MCMG_OK) return st;
    if ((st = hck(launch_multidot(nullptr, N, 0, r[i], N, c->partial, nullptr, s), "train norm")) != MCMG_OK) return st;
    if ((st = hck(launch_reduce_dots(c->partial, c->nb_red, 0, c->coef, c->coef, c->scal + 4, nullptr, s), "train norm")) != MCMG_OK) return st;
    if ((st = hck(hipMemcpyAsync(c->host_scal, c->scal + 2, 3 * sizeof(double), hipMemcpyDeviceToHost, s), "train read")) != MCMG_OK) return st;
    if ((st = hck(hipStreamSynchronize(s), "train sync")) != MCMG_OK) return st;
    const double wn = c->host_scal[1], rn = std::sqrt(c->host_scal[2]);
    if (!(rn > 0) || !std::isfinite(wn)) return fail(MCMG_E_NONFINITE, "training residual is zero or non-finite");
    total += wn / rn;
    // dL/dz = A^H (A z - r) / (B |A z - r| |r|) = -A^H w' / (B |w'| |r|)
    op.adjoint = 1;
    if ((st = hck(launch_helm(op, T_F64, T->wres, nullptr, T->ahw, nullptr, s), "train adjoint")) != MCMG_OK) return st;
    const double sc = wn > 0 ? -1.0 / ((double)nh * wn * rn) : 0.0;
    if ((st = hck(launch_c2f(T->ahw, T->dz2, N, sc, s), "train dz")) != MCMG_OK) return st;
    if ((st = hck(c->train_backward(), "train backward")) != MCMG_OK) return st;
    if (c != M) {
      if ((st = hck(hipStreamSynchronize(s), "train sync")) != MCMG_OK) return st;
      if ((st = hck(launch_axpy(TM->grad, T->grad, TM->n, 1.f, M->stream), "train accumulate")) != MCMG_OK) return st;
    }
  }
  if ((st = hck(hipStreamSynchronize(M->stream), "train sync")) != MCMG_OK) return st;
  if (loss) *loss = total / nh;
  if (grad_out) {
    if (ngrad != TM->n) return fail(MCMG_E_ARG, "gradient buffer holds %zu floats, the model %zu", ngrad, TM->n);
    if ((st = hck(hipMemcpy(grad_out, TM->grad, TM->n * sizeof(float), hipMemcpyDeviceToHost), "grad read")) != MCMG_OK) return st;
  }
  if (!opt) return MCMG_OK;
  if (!(opt->lr > 0) || !(opt->beta1 >= 0 && opt->beta1 < 1) || !(opt->beta2 >= 0 && opt->beta2 < 1) || !(opt->eps > 0))
    return fail(MCMG_E_ARG, "bad Adam parameters");
  TM->t += 1;
  AdamArgs a;
  a.lr = (float)opt->lr; a.b1 = (float)opt->beta1; a.b2 = (float)opt->beta2; a.eps = (float)opt->eps;
  a.bc1 = (float)(1.0 - std::pow(opt->beta1, TM->t));
  a.bc2 = (float)(1.0 - std::pow(opt->beta2, TM->t));
  for (const TTensor& t : TM->ts) {
    if (!t.train) continue;
    if ((st = hck(launch_adam(TM->theta + t.off, TM->grad + t.off, TM->m + t.off, TM->v + t.off,
                              (long long)t.len, a, M->stream), "adam")) != MCMG_OK) return st;
  }
  if ((st = hck(M->train_sync_weights(), "train layout")) != MCMG_OK) return st;
  return hck(hipStreamSynchronize(M->stream), "train sync");
}

}  // namespace

extern "C" {

mcmg_status mcmg_train_step(mcmg_handle* hs, int nh, const double* const* r, const mcmg_adam* opt,
                            double* loss) {
  if (!opt) return fail(MCMG_E_ARG, "null Adam parameters");
  return train_batch(hs, nh, r, opt, loss, nullptr, 0);
}

mcmg_status mcmg_train_loss_grad(mcmg_handle* hs, int nh, const double* const* r, double* loss,
                                 float* grad, size_t ngrad) {
  return train_batch(hs, nh, r, nullptr, loss, grad, ngrad);
}

mcmg_status mcmg_train_set_trainable(mcmg_handle h, const int* mask, int ntensors) {
  if (!h || !mask) return fail(MCMG_E_ARG, "null argument");
  Ctx* c = (Ctx*)h;
  const mcmg_status st = c->train_init();
  if (st != MCMG_OK) return st;
  if (ntensors != (int)c->train->ts.size())
    return fail(MCMG_E_ARG, "mask has %d entries, the model %zu tensors", ntensors, c->train->ts.size());
  for (int i = 0; i < ntensors; ++i) c->train->ts[i].train = mask[i] != 0;
  return MCMG_OK;
}

mcmg_status mcmg_train_commit(mcmg_handle h) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  return ((Ctx*)h)->repack_inference();
}

mcmg_status mcmg_weights_size(mcmg_handle h, int* ntensors, size_t* nfloats) {
  if (!h || !ntensors || !nfloats) return fail(MCMG_E_ARG, "null argument");
  Ctx* c = (Ctx*)h;
  *ntensors = (int)c->host_w.size();
  size_t n = 0;
  for (const HostTensor& t : c->host_w) n += t.w.size();
  *nfloats = n;
  return MCMG_OK;
}

mcmg_status mcmg_get_weights(mcmg_handle h, float* out, size_t nfloats) {
  if (!h || !out) return fail(MCMG_E_ARG, "null argument");
  Ctx* c = (Ctx*)h;
  size_t n = 0;
  for (const HostTensor& t : c->host_w) n += t.w.size();
  if (nfloats != n) return fail(MCMG_E_ARG, "buffer holds %zu floats, the model %zu", nfloats, n);
  if (c->train) {
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemcpy(out, c->train->theta, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(MCMG_E_HIP, "weight download");
    return MCMG_OK;
  }
  size_t off = 0;
  for (const HostTensor& t : c->host_w) {
    std::memcpy(out + off, t.w.data(), t.w.size() * sizeof(float));
    off += t.w.size();
  }
  return MCMG_OK;
}

}  // extern "C"
