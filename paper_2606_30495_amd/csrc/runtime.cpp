// libmcmg.so runtime: handle, weight blob, setup (Alg. 1), V-cycle schedule
// (Alg. 2), FGMRES driver and the C ABI declared in include/mcmg.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "internal.h"
#include "mcmg.h"
#include "runtime.h"
#include "conv_mfma.h"

using namespace mcmg;

namespace {
thread_local std::string g_err;
}

namespace mcmg {

const char* intern_name(const std::string& s) {
  static std::mutex mu;
  static std::set<std::string> names;
  std::lock_guard<std::mutex> lk(mu);
  return names.insert(s).first->c_str();
}

mcmg_status fail(mcmg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

void* Ctx::alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
  allocs.push_back(p);
  device_bytes += bytes;
  return p;
}

Ctx::~Ctx() {
  if (stream) (void)hipStreamSynchronize(stream);
  for (Slot& sl : slots) if (sl.chunk) (void)hipFree(sl.chunk);
  for (void* p : allocs) (void)hipFree(p);
  if (host_scal) (void)hipHostFree(host_scal);
  delete train;
}

}  // namespace mcmg

// ---------------------------------------------------------------------------
// weight blob

namespace {

enum Kind { K_FLIFT = 0, K_GLIFT, K_GPROJ, K_FS, K_W, K_KA, K_KS, K_WSM, K_FA, K_R, K_P };

struct TEntry { uint32_t kind, level, step, d0, d1, taps; uint64_t off; };

struct Expected { int kind, level, step, d0, d1; };

std::vector<Expected> canonical(int dim, int L, const int* C, const int* nu1, const int* nu2) {
  std::vector<Expected> v;
  v.push_back({K_FLIFT, 0, 0, C[0], 1});
  v.push_back({K_GLIFT, 0, 0, C[0], 2});
  v.push_back({K_GPROJ, 0, 0, 2, C[0]});
  for (int l = 1; l <= L; ++l) {
    const int c = C[l - 1];
    v.push_back({K_FS, l, 0, c, c});
    v.push_back({K_W, l, 0, c, c});
    v.push_back({K_KA, l, 0, c, c});
    v.push_back({K_KS, l, 0, c, c});
    const int ns = nu1[l - 1] + (l < L ? nu2[l - 1] : 0);
    for (int i = 1; i <= ns; ++i) v.push_back({K_WSM, l, i, c, c});
    if (l < L) {
      const int cn = C[l];
      v.push_back({K_FA, l, 0, cn, c});
      v.push_back({K_R, l, 0, cn, c});
      v.push_back({K_P, l, 0, cn, c});
    }
  }
  (void)dim;
  return v;
}

// Repack [d0][d1][taps] to [tap][cin][cpad]; `transposed` marks P, whose
// gather input channel is d0 and output channel d1.
std::vector<float> repack(const float* w, int d0, int d1, int taps, bool transposed, int cpad) {
  const int cin = transposed ? d0 : d1;
  const int cout = transposed ? d1 : d0;
  std::vector<float> out((size_t)taps * cin * cpad, 0.f);
  for (int a = 0; a < d0; ++a)
    for (int b = 0; b < d1; ++b)
      for (int t = 0; t < taps; ++t) {
        const int ci = transposed ? a : b;
        const int co = transposed ? b : a;
        out[((size_t)t * cin + ci) * cpad + co] = w[((size_t)a * d1 + b) * taps + t];
      }
  (void)cout;
  return out;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

namespace mcmg {

mcmg_status Ctx::upload_weight(const float* src, int d0, int d1, bool transposed, float** dst) {
  const int taps = dim == 2 ? 9 : 27;
  const int cout = transposed ? d1 : d0;
  const int cpad = round_up(cout, conv_chunk(cout));
  std::vector<float> rp = repack(src, d0, d1, taps, transposed, cpad);
  float* d = (float*)alloc(rp.size() * sizeof(float));
  if (!d) return fail(MCMG_E_OOM, "weight allocation failed");
  hipError_t e = hipMemcpyAsync(d, rp.data(), rp.size() * sizeof(float), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "weight upload: %s", hipGetErrorString(e));
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "weight upload: %s", hipGetErrorString(e));
  *dst = d;
  return MCMG_OK;
}

mcmg_status Ctx::parse_weights(const void* blob, size_t bytes) {
  const uint8_t* b = (const uint8_t*)blob;
  if (!blob || bytes < 256) return fail(MCMG_E_WEIGHTS, "weight blob too small");
  if (memcmp(b, "MCMGWB01", 8) != 0) return fail(MCMG_E_WEIGHTS, "bad weight blob magic");
  uint32_t hdr[4 + 24 + 1];
  memcpy(hdr, b + 8, sizeof(hdr));
  const uint32_t version = hdr[0], bdim = hdr[1], bL = hdr[2], ks = hdr[3];
  if (version != 1 || ks != 3) return fail(MCMG_E_WEIGHTS, "unsupported blob version/ksize");
  if ((int)bdim != dim) return fail(MCMG_E_WEIGHTS, "blob dim %u != grid dim %d", bdim, dim);
  if (bL < 1 || bL > 8) return fail(MCMG_E_WEIGHTS, "blob level count %u out of range", bL);
  L = (int)bL;
  int C[8], n1[8], n2[8];
  for (int i = 0; i < 8; ++i) { C[i] = (int)hdr[4 + i]; n1[i] = (int)hdr[12 + i]; n2[i] = (int)hdr[20 + i]; }
  const uint32_t ntens = hdr[28];
  if (C[0] != 2) return fail(MCMG_E_WEIGHTS, "C_1 must be 2 (Re/Im), got %d", C[0]);
  for (int l = 0; l < L; ++l) {
    if (C[l] < 1 || C[l] > 256) return fail(MCMG_E_WEIGHTS, "channel count out of range");
    if (n1[l] < 0 || n2[l] < 0 || n1[l] > 32 || n2[l] > 32)
      return fail(MCMG_E_WEIGHTS, "smoothing step count out of range");
  }
  std::vector<Expected> ex = canonical(dim, L, C, n1, n2);
  if (ntens != ex.size()) return fail(MCMG_E_WEIGHTS, "blob holds %u tensors, expected %zu", ntens, ex.size());
  if (256 + 32 * (size_t)ntens > bytes) return fail(MCMG_E_WEIGHTS, "blob tensor table truncated");
  const int taps = dim == 2 ? 9 : 27;
  lev.assign(L, Level());
  for (int l = 0; l < L; ++l) {
    lev[l].C = C[l];
    lev[l].nu1 = n1[l];
    lev[l].nu2 = (l < L - 1) ? n2[l] : 0;
  }
  for (size_t k = 0; k < ex.size(); ++k) {
    TEntry te;
    memcpy(&te, b + 256 + 32 * k, sizeof(te));
    const Expected& e = ex[k];
    if ((int)te.kind != e.kind || (int)te.level != e.level || (int)te.step != e.step ||
        (int)te.d0 != e.d0 || (int)te.d1 != e.d1 || (int)te.taps != taps)
      return fail(MCMG_E_WEIGHTS, "tensor %zu does not match the canonical order/shape", k);
    const size_t nbytes = (size_t)te.d0 * te.d1 * te.taps * sizeof(float);
    if (te.off + nbytes > bytes || (te.off & 3)) return fail(MCMG_E_WEIGHTS, "tensor %zu out of blob", k);
    std::vector<float> w((size_t)te.d0 * te.d1 * te.taps);
    memcpy(w.data(), b + te.off, nbytes);
    for (float v : w)
      if (!std::isfinite(v)) return fail(MCMG_E_NONFINITE, "non-finite weight in tensor %zu", k);
    host_w.push_back({e.kind, e.level, e.step, e.d0, e.d1, w});
    float* dst = nullptr;
    mcmg_status st = upload_weight(w.data(), e.d0, e.d1, e.kind == K_P, &dst);
    if (st != MCMG_OK) return st;
    if (e.level == 0) {
      if (e.kind == K_FLIFT) w_flift = dst;
      else if (e.kind == K_GLIFT) w_glift = dst;
      else w_gproj = dst;
    } else {
      Level& lv = lev[e.level - 1];
      switch (e.kind) {
        case K_FS: lv.w_fs = dst; break;
        case K_W: lv.w_W = dst; break;
        case K_KA: lv.w_KA = dst; break;
        case K_KS: lv.w_KS = dst; break;
        case K_WSM: lv.w_sm.push_back(dst); break;
        case K_FA: lv.w_fa = dst; break;
        case K_R: lv.w_R = dst; break;
        case K_P: lv.w_P = dst; break;
      }
    }
  }
  return MCMG_OK;
}

// ---------------------------------------------------------------------------
// convolutions

hipError_t Ctx::conv(int mode, int epi, int tin, const void* x, const Dims& in, int cin,
                     const float* w, const float* w2, int tout, void* y, const Dims& out, int cout,
                     const float* r, const float* feat) {
  ConvLaunch a;
  a.dim = dim; a.mode = mode; a.epi = epi; a.tin = tin; a.tout = tout;
  a.x = x; a.w = w; a.w2 = w2; a.y = y; a.r = r; a.feat = feat;
  a.cin = cin; a.cout = cout; a.cpad = round_up(cout, conv_chunk(cout));
  a.in = in; a.out = out;
  return dispatch_conv(a);
}

hipError_t Ctx::dispatch_conv(const ConvLaunch& a) {
  if (rec) {
    RecOp r{};
    r.kind = 0;
    r.conv = a;
    rec->push_back(r);
    return hipSuccess;
  }
  if (!prof.on) return launch_conv(a, stream);
  double fl, by;
  conv_work(a, &fl, &by);
  return timed(conv_kernel_name(a), fl, by, [=] { return launch_conv(a, stream); });
}

// Alg. 2.  rin: complex field (tin = T_F64 or T_F32); zout: complex (tout).
hipError_t Ctx::vcycle(const void* rin, int tin, void* zout, int tout) {
  hipError_t e;
#define CK(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
  // lift: r_1 = g_lift * (Re, Im)
  Level& l1 = lev[0];
  CK(conv(CONV_S1, EPI_SET, tin, rin, l1.dims, 2, w_glift, nullptr, T_F32, l1.r, l1.dims, l1.C,
          nullptr, nullptr));
  // down cycle
  for (int l = 0; l < L; ++l) {
    Level& lv = lev[l];
    if (lv.nu1 == 0) CK(launch_zero_f32(lv.e, lv.dims.total * lv.C, stream));
    for (int i = 0; i < lv.nu1; ++i) CK(smooth_step(lv, i, i == 0));
    if (l < L - 1) {
      Level& nx = lev[l + 1];
      // t = r - A e ; r_{l+1} = R * t
      if (!lv.l1w.empty())
        CK(level1(lv, L1_RESID, 0));
      else
        CK(conv_level(lv, EPI_RESID, lv.e, lv.w_W, lv.m_W, lv.w_KA, lv.m_KA, lv.t, lv.r, lv.a));
      if (lv.op_R.on)
        CK(run_mop(lv.op_R, lv.t, lv.m_R, nullptr, nx.r, nullptr, nullptr));
      else
        CK(conv(CONV_S2, EPI_SET, T_F32, lv.t, lv.dims, lv.C, lv.w_R, nullptr, T_F32, nx.r, nx.dims,
                nx.C, nullptr, nullptr));
    }
  }
  // up cycle
  for (int l = L - 2; l >= 0; --l) {
    Level& lv = lev[l];
    Level& nx = lev[l + 1];
    if (lv.op_P.on)
      CK(run_mop(lv.op_P, nx.e, lv.m_P, nullptr, lv.e, nullptr, nullptr));
    else
      CK(conv(CONV_T2, EPI_ADD, T_F32, nx.e, nx.dims, nx.C, lv.w_P, nullptr, T_F32, lv.e, lv.dims,
              lv.C, nullptr, nullptr));
    for (int i = 0; i < lv.nu2; ++i) CK(smooth_step(lv, lv.nu1 + i, false));
  }
  // projection
  CK(conv(CONV_S1, EPI_SET, T_F32, l1.e, l1.dims, l1.C, w_gproj, nullptr, tout, zout, l1.dims, 2,
          nullptr, nullptr));
#undef CK
  return hipSuccess;
}

// e <- e + Wsm^(i) * (s (.) (KS * (r - A e))); `first` means e == 0.
hipError_t Ctx::smooth_step(Level& lv, int i, bool first) {
  if (!lv.l1w.empty()) return level1(lv, first ? L1_FIRST : L1_STEP, i);
  hipError_t e;
  if (lv.step_on) {
    // one fused launch: e_alt = step(e), then the buffers swap
    StepLaunch l = lv.step;
    l.var = first ? L1_FIRST : L1_STEP;
    l.e = lv.e; l.eo = lv.e_alt; l.r = lv.r; l.a = lv.a; l.s = lv.s;
    l.wSM = lv.m_sm[i];
    if (rec) {
      RecOp r{};
      r.kind = 3;
      r.st = l;
      rec->push_back(r);
      e = hipSuccess;
    } else if (!prof.on) {
      e = launch_step(l, stream);
    } else {
      const double P = (double)lv.dims.total, C = lv.C;
      const double fl = 2.0 * 9.0 * C * C * P * (first ? 2.0 : 4.0);
      const double by = 4.0 * P * C * (first ? 3.0 : 5.0);
      e = timed(step_kernel_name(l), fl, by, [=] { return launch_step(l, stream); });
    }
    if (e == hipSuccess) std::swap(lv.e, lv.e_alt);
    return e;
  }
  const float* tin = lv.r;
  if (!first) {
    e = conv_level(lv, EPI_RESID, lv.e, lv.w_W, lv.m_W, lv.w_KA, lv.m_KA, lv.t, lv.r, lv.a);
    if (e != hipSuccess) return e;
    tin = lv.t;
  }
  e = conv_level(lv, EPI_MUL, tin, lv.w_KS, lv.m_KS, nullptr, nullptr, lv.u, nullptr, lv.s);
  if (e != hipSuccess) return e;
  return conv_level(lv, first ? EPI_SET : EPI_ADD, lv.u, lv.w_sm[i],
                    lv.m_sm.empty() ? nullptr : lv.m_sm[i], nullptr, nullptr, lv.e, nullptr, nullptr);
}

// Fused C = 2 sweep: STEP / FIRST write the new e into e_alt and swap the
// two buffers; RESID writes t = r - A e into lv.t.
hipError_t Ctx::level1(Level& lv, int var, int step) {
  L1Launch l;
  l.dim = dim;
  l.var = var;
  l.e = lv.e;
  l.eo = var == L1_RESID ? lv.t : lv.e_alt;
  l.r = lv.r; l.a = lv.a; l.s = lv.s;
  l.w = lv.l1w[var == L1_RESID ? 0 : step];
  l.wdev = lv.l1w_dev[var == L1_RESID ? 0 : step];
  l.n = lv.dims;
  hipError_t e;
  if (rec) {
    RecOp r{};
    r.kind = 2;
    r.l1 = l;
    r.l1w_dev = lv.l1w_dev[var == L1_RESID ? 0 : step];
    rec->push_back(r);
    e = hipSuccess;
  } else if (!prof.on) {
    e = launch_level1(l, stream);
  } else {
    const double P = (double)lv.dims.total, T = dim == 2 ? 9.0 : 27.0;
    const double fl = var == L1_RESID ? 2.0 * T * 4 * 2 * P : 2.0 * T * 4 * (var == L1_FIRST ? 2 : 4) * P;
    const double by = var == L1_RESID ? 32.0 * P : (var == L1_FIRST ? 24.0 * P : 40.0 * P);
    const char* name = dim == 3 ? intern_name(std::string("l1z_kernel<") + std::to_string(var) + ">")
                                : intern_name(std::string("l1_kernel<2, ") + std::to_string(var) + ">");
    e = timed(name, fl, by, [=] { return launch_level1(l, stream); });
  }
  if (e == hipSuccess && var != L1_RESID) std::swap(lv.e, lv.e_alt);
  return e;
}

mcmg_status Ctx::refresh_level1() { return plan_level1(true); }

mcmg_status Ctx::plan_level1(bool refresh) {
  for (int l = 0; l < L; ++l) {
    Level& lv = lev[l];
    if (lv.C != 2) continue;
    const int T = dim == 2 ? 9 : 27;
    auto find = [&](int kind, int step) -> const std::vector<float>* {
      for (const HostTensor& t : host_w)
        if (t.kind == kind && t.level == l + 1 && t.step == step) return &t.w;
      return nullptr;
    };
    const std::vector<float>*W = find(4, 0), *KA = find(5, 0), *KS = find(6, 0);
    if (!W || !KA || !KS) return fail(MCMG_E_WEIGHTS, "missing level tensors");
    auto fill = [&](float (*dst)[2][27], const std::vector<float>& src) {
      for (int o = 0; o < 2; ++o)
        for (int c = 0; c < 2; ++c)
          for (int t = 0; t < 27; ++t) dst[o][c][t] = t < T ? src[((size_t)o * 2 + c) * T + t] : 0.f;
    };
    const int nsteps = (int)lv.w_sm.size();
    lv.l1w.assign(nsteps > 0 ? nsteps : 1, L1Weights());
    for (int i = 0; i < (int)lv.l1w.size(); ++i) {
      L1Weights& w = lv.l1w[i];
      fill(w.W, *W);
      fill(w.KA, *KA);
      fill(w.KS, *KS);
      const std::vector<float>* ws = nsteps > 0 ? find(7, i + 1) : KS;
      if (!ws) return fail(MCMG_E_WEIGHTS, "missing smoother tensor");
      fill(w.Wsm, *ws);
    }
    if (!refresh) {
      lv.e_alt = (float*)alloc((size_t)lv.dims.total * 2 * sizeof(float));
      if (!lv.e_alt) return fail(MCMG_E_OOM, "level allocation failed");
      lv.l1w_dev.assign(lv.l1w.size(), nullptr);
    }
    for (size_t i = 0; i < lv.l1w.size(); ++i) {
      if (!refresh) lv.l1w_dev[i] = (L1Weights*)alloc(sizeof(L1Weights));
      if (!lv.l1w_dev[i]) return fail(MCMG_E_OOM, "weight allocation failed");
      if (hipMemcpy(lv.l1w_dev[i], &lv.l1w[i], sizeof(L1Weights), hipMemcpyHostToDevice) != hipSuccess)
        return fail(MCMG_E_HIP, "weight upload failed");
    }
  }
  return MCMG_OK;
}

// Alg. 1: a_1 = f_lift(m), s_l = f_s(a_l), a_{l+1} = f_a(a_l).
hipError_t Ctx::run_setup() {
  hipError_t e;
  Level& l1 = lev[0];
  e = conv(CONV_S1, EPI_GELU, T_F32, mfeat, l1.dims, 1, w_flift, nullptr, T_F32, l1.a, l1.dims,
           l1.C, nullptr, nullptr);
  if (e != hipSuccess) return e;
  for (int l = 0; l < L; ++l) {
    Level& lv = lev[l];
    e = conv(CONV_S1, EPI_GELU, T_F32, lv.a, lv.dims, lv.C, lv.w_fs, nullptr, T_F32, lv.s, lv.dims,
             lv.C, nullptr, nullptr);
    if (e != hipSuccess) return e;
    if (l < L - 1) {
      Level& nx = lev[l + 1];
      e = conv(CONV_S2, EPI_GELU, T_F32, lv.a, lv.dims, lv.C, lv.w_fa, nullptr, T_F32, nx.a,
               nx.dims, nx.C, nullptr, nullptr);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t Ctx::helm_timed(int tin, const void* u, const double* f, double* out, double* partial) {
  const HelmOp op = helm();
  const double N = (double)ext.total;
  // algorithmic traffic: u, k^2 and the output (+ f in residual form)
  const double bytes = N * ((tin == T_F64 ? 16.0 : 8.0) + 8.0 + 16.0 + (f ? 16.0 : 0.0));
  const double flops = N * (dim == 2 ? 38.0 : 54.0);
  const char* name = intern_name(std::string("helm_kernel<") + std::to_string(dim) + ", " +
                                 (tin == T_F64 ? "double" : "float") + ">");
  return timed(name, flops, bytes, [=] { return launch_helm(op, tin, u, f, out, partial, stream); });
}

HelmOp Ctx::helm() const {
  HelmOp op;
  op.dim = dim;
  op.ext = ext;
  op.k2 = k2;
  for (int a = 0; a < 3; ++a) { op.cm[a] = cm[a]; op.cp[a] = cp[a]; op.g[a] = gtab[a]; }
  op.gmax = absorber == MCMG_ABL_SPONGE ? gamma_max : 0.0;
  op.fd1 = make_fastdiv((uint32_t)ext.n[1]);
  op.fd2 = make_fastdiv((uint32_t)ext.n[2]);
  return op;
}

}  // namespace mcmg

// ---------------------------------------------------------------------------
// setup

namespace {

mcmg_status do_setup(const double* c, mcmg_grid grid, double omega, double h, mcmg_pml pml,
                     mcmg_weights w, const mcmg_opts* opt, Ctx* ctx) {
  if (!c) return fail(MCMG_E_ARG, "c is NULL");
  if (grid.dim != 2 && grid.dim != 3) return fail(MCMG_E_ARG, "dim must be 2 or 3");
  if (!(omega > 0) || !std::isfinite(omega)) return fail(MCMG_E_ARG, "omega must be > 0");
  if (!(h > 0) || !std::isfinite(h)) return fail(MCMG_E_ARG, "h must be > 0");
  if (pml.ncells < 0 || pml.ncells > 4096) return fail(MCMG_E_ARG, "bad PML width");
  ctx->dim = grid.dim;
  long long nint = 1;
  for (int a = 0; a < grid.dim; ++a) {
    if (grid.n[a] < 1 || grid.n[a] > (1 << 20)) return fail(MCMG_E_ARG, "bad grid size");
    ctx->nint[a] = grid.n[a];
    ctx->next[a] = grid.n[a] + 2 * pml.ncells;
    nint *= grid.n[a];
  }
  for (int a = grid.dim; a < 3; ++a) { ctx->nint[a] = 1; ctx->next[a] = 1; }
  ctx->npml = pml.ncells;
  ctx->omega = omega;
  ctx->h = h;
  ctx->interior = make_dims(grid.dim, ctx->nint);
  ctx->ext = make_dims(grid.dim, ctx->next);
  if (opt) {
    ctx->precision = opt->precision;
    ctx->restart = opt->restart > 0 ? opt->restart : 30;
    ctx->stream = (hipStream_t)opt->stream;
    ctx->ortho = opt->ortho;
  }
  if (ctx->precision != MCMG_FP32 && ctx->precision != MCMG_BF16)
    return fail(MCMG_E_ARG, "unknown precision %d", ctx->precision);
  if (ctx->restart < 1 || ctx->restart > 1024) return fail(MCMG_E_ARG, "restart must be 1..1024");
  double cmax = 0.0;
  for (long long i = 0; i < nint; ++i) {
    if (!std::isfinite(c[i])) return fail(MCMG_E_NONFINITE, "non-finite wave speed");
    if (!(c[i] > 0)) return fail(MCMG_E_ARG, "wave speed must be > 0");
    if (c[i] > cmax) cmax = c[i];
  }
  if (pml.kind != MCMG_ABL_PML && pml.kind != MCMG_ABL_SPONGE)
    return fail(MCMG_E_ARG, "unknown absorbing layer kind %d", pml.kind);
  ctx->absorber = pml.kind;
  const double kref = omega / cmax;
  if (pml.kind == MCMG_ABL_PML) {
    ctx->sigma_max = pml.sigma_max;
    if (!(pml.sigma_max > 0))
      ctx->sigma_max = pml.ncells == 0 ? 0.0 : 3.0 * std::log(1e6) / (2.0 * kref * pml.ncells * h);
  } else {
    ctx->sigma_max = 0.0;              // no stretching
    ctx->gamma_max = pml.sigma_max;
    if (!(pml.sigma_max > 0))
      ctx->gamma_max = pml.ncells == 0 ? 0.0 : 3.0 * std::log(1e6) / (kref * pml.ncells * h);
  }
  mcmg_status st = ctx->parse_weights(w.blob, w.bytes);
  if (st != MCMG_OK) return st;
  // level geometry: ceil halving per axis
  int side[3] = {ctx->next[0], ctx->next[1], ctx->next[2]};
  for (int l = 0; l < ctx->L; ++l) {
    Level& lv = ctx->lev[l];
    for (int a = 0; a < 3; ++a) lv.n[a] = side[a];
    for (int a = 0; a < ctx->dim; ++a)
      if (side[a] < 2) return fail(MCMG_E_WEIGHTS, "level %d side < 2: too many levels for grid", l + 1);
    lv.dims = make_dims(ctx->dim, lv.n);
    for (int a = 0; a < ctx->dim; ++a) side[a] = (side[a] + 1) / 2;
  }
  // allocations
  const long long N = ctx->ext.total;
  ctx->k2 = (double*)ctx->alloc(N * sizeof(double));
  ctx->mfeat = (float*)ctx->alloc(N * sizeof(float));
  for (int a = 0; a < ctx->dim; ++a) {
    ctx->cm[a] = (double*)ctx->alloc(2 * ctx->next[a] * sizeof(double));
    ctx->cp[a] = (double*)ctx->alloc(2 * ctx->next[a] * sizeof(double));
  }
  double* c_dev = (double*)ctx->alloc(nint * sizeof(double));
  if (!ctx->k2 || !ctx->mfeat || !c_dev) return fail(MCMG_E_OOM, "setup allocation failed");
  for (auto& lv : ctx->lev) {
    const size_t nb = (size_t)lv.dims.total * lv.C * sizeof(float);
    lv.a = (float*)ctx->alloc(nb);
    lv.s = (float*)ctx->alloc(nb);
    lv.e = (float*)ctx->alloc(nb);
    lv.r = (float*)ctx->alloc(nb);
    lv.t = (float*)ctx->alloc(nb);
    lv.u = (float*)ctx->alloc(nb);
    if (!lv.a || !lv.s || !lv.e || !lv.r || !lv.t || !lv.u) return fail(MCMG_E_OOM, "level allocation failed");
  }
  hipStream_t s = ctx->stream;
  hipError_t e = hipMemcpyAsync(c_dev, c, nint * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "copy c: %s", hipGetErrorString(e));
  e = launch_setup_medium(ctx->dim, ctx->interior, ctx->npml, c_dev, omega, h, ctx->k2, ctx->mfeat, s);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "setup_medium: %s", hipGetErrorString(e));
  for (int a = 0; a < ctx->dim; ++a) {
    e = launch_pml_tables(ctx->next[a], ctx->npml, h, ctx->sigma_max, ctx->cm[a], ctx->cp[a], s);
    if (e != hipSuccess) return fail(MCMG_E_HIP, "pml tables: %s", hipGetErrorString(e));
  }
  if (ctx->absorber == MCMG_ABL_SPONGE) {
    // per-axis (d_a / npml)^2, d_a = cells into the layer along axis a
    for (int a = 0; a < ctx->dim; ++a) {
      std::vector<double> g(ctx->next[a], 0.0);
      for (int i = 0; i < ctx->next[a] && ctx->npml > 0; ++i) {
        const int lo = ctx->npml, hi = ctx->npml + ctx->nint[a] - 1;
        const double dd = i < lo ? lo - i : (i > hi ? i - hi : 0);
        g[i] = (dd / ctx->npml) * (dd / ctx->npml);
      }
      ctx->gtab[a] = (double*)ctx->alloc(g.size() * sizeof(double));
      if (!ctx->gtab[a]) return fail(MCMG_E_OOM, "setup allocation failed");
      e = hipMemcpy(ctx->gtab[a], g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) return fail(MCMG_E_HIP, "sponge tables: %s", hipGetErrorString(e));
    }
  }
  e = ctx->run_setup();
  if (e != hipSuccess) return fail(MCMG_E_HIP, "setup convolutions: %s", hipGetErrorString(e));
  st = ctx->plan_mfma();
  if (st != MCMG_OK) return st;
  st = ctx->plan_level1();
  if (st != MCMG_OK) return st;
  st = ctx->alloc_krylov();
  if (st != MCMG_OK) return st;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "setup: %s", hipGetErrorString(e));
  return MCMG_OK;
}

}  // namespace

namespace mcmg {

mcmg_status Ctx::alloc_krylov() {
  const long long N = ext.total;
  const int m = restart;
  V = (double*)alloc((size_t)(m + 1) * N * 2 * sizeof(double));
  Z = (float*)alloc((size_t)m * N * 2 * sizeof(float));
  wv = (double*)alloc(N * 2 * sizeof(double));
  rv = (double*)alloc(N * 2 * sizeof(double));
  zt = (float*)alloc(N * 2 * sizeof(float));
  H = (double*)alloc((size_t)(m + 1) * m * 2 * sizeof(double));
  cs = (double*)alloc(m * sizeof(double));
  sn = (double*)alloc(m * 2 * sizeof(double));
  g = (double*)alloc((m + 1) * 2 * sizeof(double));
  y = (double*)alloc(m * 2 * sizeof(double));
  coef = (double*)alloc((m + 2) * 2 * sizeof(double));
  nb_red = red_blocks(N);
  const int nbh = helm_blocks(helm());
  const int nbmax = nb_red > nbh ? nb_red : nbh;
  partial = (double*)alloc((size_t)(m + 2) * nbmax * 2 * sizeof(double));
  scal = (double*)alloc(64 * sizeof(double));
  skip = (int*)alloc(64 * sizeof(int));
  if (!V || !Z || !wv || !rv || !zt || !H || !cs || !sn || !g || !y || !coef || !partial || !scal || !skip)
    return fail(MCMG_E_OOM, "Krylov workspace allocation failed");
  if (hipHostMalloc((void**)&host_scal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    host_scal = nullptr;
    return fail(MCMG_E_OOM, "pinned host allocation failed");
  }
  return MCMG_OK;
}


}  // namespace mcmg

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* mcmg_last_error(void) { return g_err.c_str(); }

mcmg_status mcmg_setup(const double* c, mcmg_grid grid, double omega, double h, mcmg_pml pml,
                       mcmg_weights w, const mcmg_opts* opt, mcmg_handle* out) {
  if (!out) return fail(MCMG_E_ARG, "out is NULL");
  *out = nullptr;
  Ctx* ctx = new (std::nothrow) Ctx();
  if (!ctx) return fail(MCMG_E_OOM, "host allocation failed");
  mcmg_status st = do_setup(c, grid, omega, h, pml, w, opt, ctx);
  if (st != MCMG_OK) {
    std::string keep = g_err;
    delete ctx;
    g_err = keep;
    return st;
  }
  *out = (mcmg_handle)ctx;
  return MCMG_OK;
}

void mcmg_destroy(mcmg_handle h) { delete (Ctx*)h; }

size_t mcmg_device_bytes(mcmg_handle h) {
  if (!h) return 0;
  const Ctx* c = (const Ctx*)h;
  size_t n = c->device_bytes;
  for (const Slot& s : c->slots) n += s.bytes;
  return n;
}

mcmg_status mcmg_grid_shape(mcmg_handle h, int* dim, int n_ext[3], int* npml) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  Ctx* c = (Ctx*)h;
  if (dim) *dim = c->dim;
  if (n_ext) for (int a = 0; a < 3; ++a) n_ext[a] = c->next[a];
  if (npml) *npml = c->npml;
  return MCMG_OK;
}

mcmg_status mcmg_apply(mcmg_handle h, const double* r, double* z) {
  if (!h || !r || !z) return fail(MCMG_E_ARG, "null argument");
  if ((const void*)r == (const void*)z) return fail(MCMG_E_ARG, "r and z may not alias");
  Ctx* c = (Ctx*)h;
  hipError_t e = c->vcycle(r, T_F64, z, T_F64);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "apply: %s", hipGetErrorString(e));
  return MCMG_OK;
}

mcmg_status mcmg_matvec(mcmg_handle h, const double* u, double* Au) {
  if (!h || !u || !Au) return fail(MCMG_E_ARG, "null argument");
  if ((const void*)u == (const void*)Au) return fail(MCMG_E_ARG, "u and Au may not alias");
  Ctx* c = (Ctx*)h;
  hipError_t e = c->helm_timed(T_F64, u, nullptr, Au, nullptr);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "matvec: %s", hipGetErrorString(e));
  return MCMG_OK;
}

mcmg_status mcmg_prof_enable(mcmg_handle h, int on) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  Ctx* c = (Ctx*)h;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "prof: %s", hipGetErrorString(e));
  c->prof.on = on != 0;
  c->prof.recs.clear();
  c->prof.used = 0;
  return MCMG_OK;
}

mcmg_status mcmg_prof_report(mcmg_handle h, char* buf, size_t cap) {
  if (!h || !buf || cap == 0) return fail(MCMG_E_ARG, "null argument");
  Ctx* c = (Ctx*)h;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "prof: %s", hipGetErrorString(e));
  struct Agg { long long n = 0; double ms = 0, fl = 0, by = 0; };
  std::map<std::string, Agg> agg;
  for (const ProfRec& r : c->prof.recs) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return fail(MCMG_E_HIP, "prof: %s", hipGetErrorString(e));
    Agg& a = agg[r.name];
    a.n += 1; a.ms += ms; a.fl += r.flops; a.by += r.bytes;
  }
  std::string out = "[";
  bool first = true;
  for (auto& kv : agg) {
    char line[512];
    snprintf(line, sizeof(line),
             "%s{\"name\":\"%s\",\"launches\":%lld,\"total_ms\":%.6f,\"avg_ms\":%.6f,"
             "\"flops_per_launch\":%.6e,\"bytes_per_launch\":%.6e}",
             first ? "" : ",", kv.first.c_str(), kv.second.n, kv.second.ms,
             kv.second.ms / kv.second.n, kv.second.fl / kv.second.n, kv.second.by / kv.second.n);
    out += line;
    first = false;
  }
  out += "]";
  if (out.size() + 1 > cap) return fail(MCMG_E_ARG, "report buffer too small (%zu bytes needed)", out.size() + 1);
  memcpy(buf, out.c_str(), out.size() + 1);
  return MCMG_OK;
}

mcmg_status mcmg_prof_replay(mcmg_handle h, const char* name, int reps, double* avg_ms,
                             int* launches) {
  if (!h || !name || !avg_ms || reps < 1) return fail(MCMG_E_ARG, "bad argument");
  Ctx* c = (Ctx*)h;
  std::vector<const ProfRec*> sel;
  for (const ProfRec& r : c->prof.recs)
    if (std::string(r.name) == name) sel.push_back(&r);
  if (sel.empty()) return fail(MCMG_E_ARG, "no recorded launch of %s", name);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(MCMG_E_HIP, "event create");
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(MCMG_E_HIP, "event create"); }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  for (int k = 0; k < reps && e == hipSuccess; ++k)
    for (const ProfRec* r : sel) {
      e = r->replay();
      if (e != hipSuccess) break;
    }
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "replay: %s", hipGetErrorString(e));
  *avg_ms = ms / ((double)sel.size() * reps);
  if (launches) *launches = (int)sel.size() * reps;
  return MCMG_OK;
}

mcmg_status mcmg_debug_level_shape(mcmg_handle h, int level, int n[3], int* channels) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  Ctx* c = (Ctx*)h;
  if (level < 1 || level > c->L) return fail(MCMG_E_ARG, "level out of range");
  const Level& lv = c->lev[level - 1];
  if (n) for (int a = 0; a < 3; ++a) n[a] = lv.n[a];
  if (channels) *channels = lv.C;
  return MCMG_OK;
}

mcmg_status mcmg_debug_set_features(mcmg_handle h, int level, const float* a, const float* s) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  Ctx* c = (Ctx*)h;
  if (level < 1 || level > c->L) return fail(MCMG_E_ARG, "level out of range");
  Level& lv = c->lev[level - 1];
  const size_t nb = (size_t)lv.dims.total * lv.C * sizeof(float);
  hipError_t e = hipSuccess;
  if (a) e = hipMemcpyAsync(lv.a, a, nb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && s) e = hipMemcpyAsync(lv.s, s, nb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = c->on_features_changed();
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "set features: %s", hipGetErrorString(e));
  return MCMG_OK;
}

mcmg_status mcmg_debug_get_features(mcmg_handle h, int level, float* a, float* s) {
  if (!h) return fail(MCMG_E_ARG, "null handle");
  Ctx* c = (Ctx*)h;
  if (level < 1 || level > c->L) return fail(MCMG_E_ARG, "level out of range");
  Level& lv = c->lev[level - 1];
  const size_t nb = (size_t)lv.dims.total * lv.C * sizeof(float);
  hipError_t e = hipSuccess;
  if (a) e = hipMemcpyAsync(a, lv.a, nb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && s) e = hipMemcpyAsync(s, lv.s, nb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "get features: %s", hipGetErrorString(e));
  return MCMG_OK;
}

}  // extern "C"
