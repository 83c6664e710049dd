// Matrix-core plans of the V-cycle convolutions: weight packing for the
// implicit GEMMs (stride-1 solve convolutions, restriction, prolongation) and
// the tile autotuner.
//
// Autotuner: for every convolution instance (mode, epilogue, channels, grid)
// the candidate tiles (16*mt nodes per wave row, mt in {1,2,4}; ntw column
// tiles per block, ntw in {1,2,4}; rpw node rows per wave, rpw in {1,2} in
// 2D and {1,2,4} in 3D) that fit the LDS are each launched on the handle's
// own buffers and timed with HIP events; the fastest is kept.
// Choices are cached per process and, when MCMG_TUNE_CACHE names a file, in
// that JSON file ({"key": [mt, ntw, rpw], ...}; two numbers read as rpw 1), keyed by
// arch|dim|precision|mode|epi|cin|cout|grid.  Without MCMG_TUNE_CACHE the
// table tune_gfx950.json next to libmcmg.so (written by an earlier tuning
// run) is read, so shapes it covers get the same tiles in every process.
// MCMG_AUTOTUNE=0 skips timing and takes the first fitting candidate.
// MCMG_FORCE_TILE=mt,ntw,rpw takes that tile wherever it is a candidate
// (tests use it to run every tile shape against the oracle).
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "conv_mfma.h"
#include "internal.h"
#include "runtime.h"

namespace mcmg {

namespace {

std::mutex g_tune_mu;
struct Tile {
  int mt, ntw, rpw;
  bool operator==(const Tile& o) const { return mt == o.mt && ntw == o.ntw && rpw == o.rpw; }
};
std::map<std::string, Tile> g_tune;
bool g_tune_loaded = false;

const char* cache_path() {
  const char* p = getenv("MCMG_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// The tuning table shipped beside libmcmg.so (read only).
std::string packaged_cache() {
  Dl_info info;
  if (!dladdr((void*)&packaged_cache, &info) || !info.dli_fname) return "";
  std::string so = info.dli_fname;
  const size_t slash = so.rfind('/');
  return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tune_gfx950.json";
}

void load_cache_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* env = cache_path();
  const std::string path = env ? std::string(env) : packaged_cache();
  if (path.empty()) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    int mt = 0, ntw = 0, rpw = 1;
    const size_t b = s.find('[', j);
    if (b == std::string::npos) break;
    const int got = sscanf(s.c_str() + b, "[%d ,%d ,%d", &mt, &ntw, &rpw);
    if (got >= 2) g_tune[key] = {mt, ntw, got == 3 ? rpw : 1};
    i = s.find(']', b);
    if (i == std::string::npos) break;
  }
}

void save_cache_locked() {
  const char* p = cache_path();
  if (!p) return;
  std::ofstream f(p);
  if (!f) return;
  f << "{\n";
  size_t k = 0;
  for (auto& kv : g_tune) {
    f << "  \"" << kv.first << "\": [" << kv.second.mt << ", " << kv.second.ntw << ", "
      << kv.second.rpw << "]" << (++k < g_tune.size() ? ",\n" : "\n");
  }
  f << "}\n";
}

std::string tune_key(int dim, int bf16, const MOp& op) {
  char b[256];
  snprintf(b, sizeof(b), "gfx950|%d|%s|%d|%d|%d|%d|%dx%dx%d", dim, bf16 ? "bf16" : "f32", op.mode,
           op.epi, op.cin, op.cout, op.in.n[0], op.in.n[1], op.in.n[2]);
  return b;
}

// Pack a blob tensor [d0][d1][3^D] into the GEMM layout [4*nsteps][ncols][KV].
std::vector<float> pack_gemm(const std::vector<float>& w, int dim, const MOp& op, int KV) {
  const int T3 = dim == 2 ? 9 : 27;
  const int cpv = op.cinp / KV;
  const bool grouped = dim == 3 && KV == 1;   // 3D float32: see mfma_bg_index
  const int steps = grouped ? (op.nsteps + 3) / 4 * 4 : op.nsteps;
  std::vector<float> out((size_t)4 * (steps + MFMA_PAD_STEPS) * op.ncols * KV, 0.f);
  for (int q = 0; q < op.npairs; ++q) {
    const int tap = q / cpv, cb = q % cpv;
    for (int col = 0; col < op.ncols; ++col)
      for (int v = 0; v < KV; ++v) {
        const int ci = cb * KV + v;
        if (ci >= op.cin) continue;
        float val = 0.f;
        if (op.mode != CONV_T2) {
          if (col >= op.cout) continue;
          val = w[((size_t)col * op.cin + ci) * T3 + tap];
        } else {
          // window tap (w per axis in {0,1}), class a per axis, P tap d = a - 2w + 1
          const int cls = col / op.cout, c = col % op.cout;
          if (cls >= (1 << dim)) continue;
          int wv[3] = {0, 0, 0}, av[3] = {0, 0, 0};
          if (dim == 2) { wv[1] = tap / 2; wv[2] = tap % 2; }
          else { wv[0] = tap / 4; wv[1] = (tap / 2) % 2; wv[2] = tap % 2; }
          av[2] = cls & 1; av[1] = (cls >> 1) & 1; av[0] = dim == 3 ? (cls >> 2) & 1 : 0;
          int d[3];
          bool ok = true;
          for (int a = 0; a < 3; ++a) {
            d[a] = av[a] - 2 * wv[a] + 1;
            if (d[a] < 0 || d[a] > 2) ok = false;
          }
          if (!ok) continue;
          const int t3 = dim == 2 ? d[1] * 3 + d[2] : (d[0] * 3 + d[1]) * 3 + d[2];
          // P is [C_coarse = cin][C_fine = cout][3^D]
          val = w[((size_t)ci * op.cout + c) * T3 + t3];
        }
        out[grouped ? mfma_bg_index(q, col, op.ncols) : ((size_t)q * op.ncols + col) * KV + v] = val;
      }
  }
  return out;
}

}  // namespace

hipError_t Ctx::run_mop(const MOp& op, const float* x, const void* wA, const void* wB, float* y,
                        const float* r, const float* feat) {
  MfmaConv a;
  a.dim = dim;
  a.bf16 = precision == MCMG_BF16 ? 1 : 0;
  a.mode = op.mode; a.epi = op.epi; a.mt = op.mt; a.ntw = op.ntw; a.rpw = op.rpw;
  a.kchunk = op.kchunk;
  a.x = x; a.wA = wA; a.wB = wB; a.y = y; a.r = r; a.feat = feat;
  a.cin = op.cin; a.cinp = op.cinp; a.cout = op.cout; a.ncols = op.ncols;
  a.nsteps = op.nsteps; a.npairs = op.npairs;
  a.in = op.in; a.out = op.out;
  if (rec) {
    RecOp r{};
    r.kind = 1;
    r.mf = a;
    rec->push_back(r);
    return hipSuccess;
  }
  if (!prof.on) return launch_conv_mfma(a, stream);
  const double T = op.mode == CONV_T2 ? 0 : (dim == 2 ? 9.0 : 27.0);
  double fl, by;
  if (op.mode == CONV_T2) {
    // transposed convolution: every coarse input node scatters 3^D taps
    fl = 2.0 * (dim == 2 ? 9.0 : 27.0) * op.cin * op.cout * (double)op.in.total;
    by = 4.0 * ((double)op.in.total * op.cin + 2.0 * (double)op.out.total * op.cout);
  } else {
    fl = 2.0 * T * op.cin * op.cout * (double)op.out.total * (op.epi == EPI_RESID ? 2.0 : 1.0);
    const double pout = (double)op.out.total * op.cout;
    const double extra = op.epi == EPI_RESID ? 2.0 : (op.epi == EPI_SET ? 0.0 : 1.0);
    by = 4.0 * ((double)op.in.total * op.cin + pout * (1.0 + extra));
  }
  return timed(mfma_kernel_name(a), fl, by, [=] { return launch_conv_mfma(a, stream); });
}

hipError_t Ctx::conv_level(Level& lv, int epi, const float* x, const float* w, const void* wm,
                           const float* w2, const void* wm2, float* y, const float* r,
                           const float* feat) {
  const MOp& op = epi == EPI_RESID ? lv.op_resid
                  : epi == EPI_MUL ? lv.op_mul
                  : epi == EPI_SET ? lv.op_set
                                   : lv.op_add;
  if (!op.on)
    return conv(CONV_S1, epi, T_F32, x, lv.dims, lv.C, w, w2, T_F32, y, lv.dims, lv.C, r, feat);
  return run_mop(op, x, wm, wm2, y, r, feat);
}

namespace {
// float32 weights -> the device copy of a matrix-core pack (bf16 with round
// to nearest even when the form is bf16)
hipError_t upload_pack(const std::vector<float>& f, void* dst, bool bf) {
  if (!bf) return hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
  std::vector<uint16_t> b(f.size());
  for (size_t i = 0; i < f.size(); ++i) {
    uint32_t u;
    memcpy(&u, &f[i], 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    b[i] = (uint16_t)(u >> 16);
  }
  return hipMemcpy(dst, b.data(), b.size() * 2, hipMemcpyHostToDevice);
}
}  // namespace

// Re-pack changed weights (host_w) into the existing matrix-core buffers and
// level-1 sweep weights, keeping every plan and tile.
mcmg_status Ctx::refresh_packed() {
  const bool bf = precision == MCMG_BF16;
  const int KV = bf ? 8 : 1;
  auto tensor = [&](int kind, int level, int step) -> const std::vector<float>* {
    for (const HostTensor& t : host_w)
      if (t.kind == kind && t.level == level && t.step == step) return &t.w;
    return nullptr;
  };
  auto put = [&](const std::vector<float>* w, const MOp& op, void* dst) -> mcmg_status {
    if (!dst) return MCMG_OK;
    if (!w) return fail(MCMG_E_WEIGHTS, "missing tensor");
    MOp proto = op;
    if (upload_pack(pack_gemm(*w, dim, proto, KV), dst, bf) != hipSuccess)
      return fail(MCMG_E_HIP, "weight re-pack");
    return MCMG_OK;
  };
  mcmg_status st;
  for (int l = 0; l < L; ++l) {
    Level& lv = lev[l];
    const int lvl = l + 1;
    if (lv.m_W) {
      if ((st = put(tensor(4, lvl, 0), lv.op_resid, lv.m_W)) != MCMG_OK) return st;
      if ((st = put(tensor(5, lvl, 0), lv.op_resid, lv.m_KA)) != MCMG_OK) return st;
      if ((st = put(tensor(6, lvl, 0), lv.op_resid, lv.m_KS)) != MCMG_OK) return st;
      for (size_t i = 0; i < lv.m_sm.size(); ++i)
        if ((st = put(tensor(7, lvl, (int)i + 1), lv.op_resid, lv.m_sm[i])) != MCMG_OK) return st;
    }
    if (lv.m_R && (st = put(tensor(9, lvl, 0), lv.op_R, lv.m_R)) != MCMG_OK) return st;
    if (lv.m_P && (st = put(tensor(10, lvl, 0), lv.op_P, lv.m_P)) != MCMG_OK) return st;
  }
  return refresh_level1();
}

mcmg_status Ctx::plan_mfma() {
  const int bf = precision == MCMG_BF16 ? 1 : 0;
  const int KV = bf ? 8 : 1;
  const char* at = getenv("MCMG_AUTOTUNE");
  const bool tune = !(at && at[0] == '0');
  const size_t lds_max = 160 * 1024;

  auto upload = [&](const std::vector<float>& f, void** dst) -> mcmg_status {
    void* d = alloc(f.size() * (bf ? 2 : 4));
    if (!d) return fail(MCMG_E_OOM, "weight allocation failed");
    hipError_t e;
    if (bf) {
      std::vector<uint16_t> b(f.size());
      for (size_t i = 0; i < f.size(); ++i) {
        uint32_t u;
        memcpy(&u, &f[i], 4);
        u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
        b[i] = (uint16_t)(u >> 16);
      }
      e = hipMemcpy(d, b.data(), b.size() * 2, hipMemcpyHostToDevice);
    } else {
      e = hipMemcpy(d, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return fail(MCMG_E_HIP, "weight upload: %s", hipGetErrorString(e));
    *dst = d;
    return MCMG_OK;
  };
  auto tensor = [&](int kind, int level, int step) -> const std::vector<float>* {
    for (const HostTensor& t : host_w)
      if (t.kind == kind && t.level == level && t.step == step) return &t.w;
    return nullptr;
  };
  auto setup_op = [&](MOp& op, int mode, int epi, int cin, int cout, const Dims& in,
                      const Dims& out) {
    op.mode = mode; op.epi = epi; op.cin = cin; op.cout = cout; op.in = in; op.out = out;
    mfma_pack_dims(dim, mode, cin, cout, bf, &op.cinp, &op.ncols, &op.npairs, &op.nsteps);
    op.on = false;
  };
  // weight chunk: all K-steps at once when the block fits 96 KB of LDS (one
  // load latency per block, two blocks per CU), else halve (the chunks are
  // then double-buffered) until it fits.  A chunk must keep the matrix
  // cores busy for longer than a copy's latency (about 8k cycles of
  // products per wave) for the double buffering to hide it; when the 96 KB
  // budget (a large staged tile) leaves less, the chunk takes the whole LDS.
  auto kchunk_for = [&](const MOp& op, const Tile& t) {
    auto bytes = [&](int kc) {
      return mfma_lds_bytes(dim, bf, op.mode, t.mt, t.ntw, t.rpw, op.cin, op.cinp, op.epi, kc, op.nsteps);
    };
    auto cycles = [&](int kc) {
      return (double)kc * (op.epi == EPI_RESID ? 2 : 1) * t.rpw * t.mt * t.ntw * (bf ? 16.0 : 32.0);
    };
    int kc = op.nsteps;
    if (!bf && dim == 3) return kc;   // 3D float32 streams its weights from global memory
    while (kc > 1 && bytes(kc) > 96 * 1024) kc = (kc + 1) / 2;
    if (bytes(kc) > 96 * 1024 || (kc < op.nsteps && cycles(kc) < 8192.0)) {
      int big = op.nsteps;
      while (big > 1 && bytes(big) > lds_max) big = (big + 1) / 2;
      if (big > kc || bytes(kc) > 96 * 1024) kc = big;
    }
    return kc;
  };
  // candidate tiles that fit, in a fixed preference order
  auto candidates = [&](const MOp& op) {
    std::vector<Tile> c;
    const int nt = op.ncols / 16;
    for (int rpw : {1, 2, 4})
      for (int mt : {2, 4, 1})
        for (int ntw : {1, 2, 4}) {
          if (nt % ntw || !mfma_tile_ok(dim, op.epi, mt, ntw, rpw)) continue;
          const Tile t{mt, ntw, rpw};
          const int kc = kchunk_for(op, t);
          if (mfma_lds_bytes(dim, bf, op.mode, mt, ntw, rpw, op.cin, op.cinp, op.epi, kc, op.nsteps) > lds_max) continue;
          c.push_back(t);
        }
    // the z-marching form (3D float32 stride-1, 12 input channels)
    if (mfmaz_ok(dim, bf, op.mode, op.cin, op.cout) && op.ncols == 16) c.push_back(Tile{1, 1, MFMAZ_RPW});
    return c;
  };
  auto set_tile = [&](MOp& op, const Tile& t) {
    op.mt = t.mt; op.ntw = t.ntw; op.rpw = t.rpw;
    op.kchunk = kchunk_for(op, t);
  };

  // zero the level state so that timing runs read finite data
  for (auto& lv : lev) {
    const long long n = lv.dims.total * lv.C;
    for (float* p : {lv.e, lv.r, lv.t, lv.u}) {
      hipError_t e = launch_zero_f32(p, n, stream);
      if (e != hipSuccess) return fail(MCMG_E_HIP, "zero: %s", hipGetErrorString(e));
    }
  }

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (tune) {
    if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
      return fail(MCMG_E_HIP, "event create failed");
  }
  struct Cleanup {
    hipEvent_t a, b;
    ~Cleanup() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } cleanup{ev0, ev1};

  // choose a tile for op; `launch` runs it once with the chosen tile
  Tile forced{0, 0, 0};
  if (const char* ft = getenv("MCMG_FORCE_TILE"))
    if (sscanf(ft, "%d,%d,%d", &forced.mt, &forced.ntw, &forced.rpw) != 3) forced = Tile{0, 0, 0};
  auto choose = [&](MOp& op, auto&& launch) -> mcmg_status {
    auto cands = candidates(op);
    if (cands.empty()) return MCMG_OK;   // stays on the VALU path
    for (auto& c : cands)
      if (c == forced) {
        set_tile(op, c);
        op.on = true;
        return MCMG_OK;
      }
    const std::string key = tune_key(dim, bf, op);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      load_cache_locked();
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        for (auto& c : cands)
          if (c == it->second) {
            set_tile(op, c);
            op.on = true;
            return MCMG_OK;
          }
      }
    }
    set_tile(op, cands[0]);
    op.on = true;
    if (!tune || cands.size() == 1) return MCMG_OK;
    float best = 1e30f;
    Tile bc = cands[0];
    for (auto& c : cands) {
      set_tile(op, c);
      hipError_t e = launch();                      // warm-up
      if (e != hipSuccess) return fail(MCMG_E_HIP, "tune: %s", hipGetErrorString(e));
      if ((e = hipEventRecord(ev0, stream)) != hipSuccess) return fail(MCMG_E_HIP, "tune event");
      for (int k = 0; k < 3; ++k)
        if ((e = launch()) != hipSuccess) return fail(MCMG_E_HIP, "tune: %s", hipGetErrorString(e));
      if ((e = hipEventRecord(ev1, stream)) != hipSuccess) return fail(MCMG_E_HIP, "tune event");
      if ((e = hipEventSynchronize(ev1)) != hipSuccess) return fail(MCMG_E_HIP, "tune sync");
      float ms = 0.f;
      hipEventElapsedTime(&ms, ev0, ev1);
      if (ms < best) { best = ms; bc = c; }
    }
    set_tile(op, bc);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = bc;
    save_cache_locked();
    return MCMG_OK;
  };

  mcmg_status st;
  for (int l = 0; l < L; ++l) {
    Level& lv = lev[l];
    const int lvl = l + 1;
    // stride-1 solve convolutions (C >= 8: level 1 with C = 2 is an HBM-bound VALU sweep)
    if (lv.C >= 8) {
      const std::vector<float>*W = tensor(4, lvl, 0), *KA = tensor(5, lvl, 0), *KS = tensor(6, lvl, 0);
      if (!W || !KA || !KS) return fail(MCMG_E_WEIGHTS, "missing level tensors");
      MOp proto;
      setup_op(proto, CONV_S1, EPI_SET, lv.C, lv.C, lv.dims, lv.dims);
      if (!candidates(proto).empty()) {
        if ((st = upload(pack_gemm(*W, dim, proto, KV), &lv.m_W)) != MCMG_OK) return st;
        if ((st = upload(pack_gemm(*KA, dim, proto, KV), &lv.m_KA)) != MCMG_OK) return st;
        if ((st = upload(pack_gemm(*KS, dim, proto, KV), &lv.m_KS)) != MCMG_OK) return st;
        lv.m_sm.assign(lv.w_sm.size(), nullptr);
        for (size_t i = 0; i < lv.w_sm.size(); ++i) {
          const std::vector<float>* ws = tensor(7, lvl, (int)i + 1);
          if (!ws) return fail(MCMG_E_WEIGHTS, "missing smoother tensor");
          if ((st = upload(pack_gemm(*ws, dim, proto, KV), &lv.m_sm[i])) != MCMG_OK) return st;
        }
        setup_op(lv.op_resid, CONV_S1, EPI_RESID, lv.C, lv.C, lv.dims, lv.dims);
        setup_op(lv.op_mul, CONV_S1, EPI_MUL, lv.C, lv.C, lv.dims, lv.dims);
        setup_op(lv.op_set, CONV_S1, EPI_SET, lv.C, lv.C, lv.dims, lv.dims);
        setup_op(lv.op_add, CONV_S1, EPI_ADD, lv.C, lv.C, lv.dims, lv.dims);
        if ((st = choose(lv.op_resid, [&] { return run_mop(lv.op_resid, lv.e, lv.m_W, lv.m_KA, lv.t, lv.r, lv.a); })) != MCMG_OK) return st;
        if ((st = choose(lv.op_mul, [&] { return run_mop(lv.op_mul, lv.t, lv.m_KS, nullptr, lv.u, nullptr, lv.s); })) != MCMG_OK) return st;
        if ((st = choose(lv.op_set, [&] { return run_mop(lv.op_set, lv.u, lv.m_sm[0], nullptr, lv.t, nullptr, nullptr); })) != MCMG_OK) return st;
        if ((st = choose(lv.op_add, [&] { return run_mop(lv.op_add, lv.u, lv.m_sm[0], nullptr, lv.t, nullptr, nullptr); })) != MCMG_OK) return st;
      } else if (bf) {
        return fail(MCMG_E_ARG, "bf16 form: no matrix-core tile fits C = %d", lv.C);
      }
    }
    if (l < L - 1) {
      Level& nx = lev[l + 1];
      // restriction R: this level (C_l) -> next (C_{l+1}), stride 2
      setup_op(lv.op_R, CONV_S2, EPI_SET, lv.C, nx.C, lv.dims, nx.dims);
      if (!candidates(lv.op_R).empty()) {
        const std::vector<float>* R = tensor(9, lvl, 0);
        if (!R) return fail(MCMG_E_WEIGHTS, "missing restriction tensor");
        if ((st = upload(pack_gemm(*R, dim, lv.op_R, KV), &lv.m_R)) != MCMG_OK) return st;
        if ((st = choose(lv.op_R, [&] { return run_mop(lv.op_R, lv.t, lv.m_R, nullptr, nx.r, nullptr, nullptr); })) != MCMG_OK) return st;
      }
      // prolongation P: next level (C_{l+1}) -> this level (C_l)
      setup_op(lv.op_P, CONV_T2, EPI_ADD, nx.C, lv.C, nx.dims, lv.dims);
      if (!candidates(lv.op_P).empty()) {
        const std::vector<float>* P = tensor(10, lvl, 0);
        if (!P) return fail(MCMG_E_WEIGHTS, "missing prolongation tensor");
        if ((st = upload(pack_gemm(*P, dim, lv.op_P, KV), &lv.m_P)) != MCMG_OK) return st;
        if ((st = choose(lv.op_P, [&] { return run_mop(lv.op_P, nx.e, lv.m_P, nullptr, lv.e, nullptr, nullptr); })) != MCMG_OK) return st;
      }
    }
  }
  // fused smoothing steps (one launch per step instead of three) on the 2D
  // bf16 levels with 16 <= C <= 32, where one block computing t and u with
  // halos beats three launches at every grid size measured; at C = 8 the
  // halo recompute, at C = 64 the serial weight streaming and with float32
  // operands the heavier MFMA make it slower.  The rule depends on C and the
  // precision only, so all handles of a model share one launch schedule (the
  // tile is autotuned).  MCMG_FUSED_STEP=0 keeps three launches everywhere,
  // =2 fuses every C >= 8 level in both precisions.
  const char* fz = getenv("MCMG_FUSED_STEP");
  const int fuse = fz ? atoi(fz) : 1;
  for (int l = 0; fuse && dim == 2 && l < L; ++l) {
    Level& lv = lev[l];
    if (lv.C < 8 || !lv.op_resid.on || !lv.op_mul.on || !lv.op_add.on || !lv.op_set.on) continue;
    if (fuse == 1 && (lv.C < 16 || lv.C > 32 || !bf)) continue;
    if (lv.m_sm.empty() || !lv.m_W || !lv.m_KA || !lv.m_KS) continue;
    const MOp& ro = lv.op_resid;
    const int nct = ro.ncols / 16;
    if (nct != 1 && nct != 2 && nct != 4) continue;
    const size_t brow = (size_t)ro.ncols * KV * (bf ? 2 : 4);
    std::vector<StepLaunch> cands;
    for (int tile : {1, 0, 2, 3}) {
      // chunks: whole tensors when they fit beside the region buffers
      const size_t regions = mstep_lds_bytes(tile, bf, nct, ro.cinp, 0, 0);
      if (regions + 8 * brow > lds_max) continue;
      const size_t wb = lds_max - regions;
      int kc1 = ro.nsteps, kc2 = ro.nsteps;
      while (kc1 > 1 && 2 * 4 * (size_t)kc1 * brow > wb) kc1 = (kc1 + 1) / 2;
      while (kc2 > 1 && 4 * (size_t)kc2 * brow > wb) kc2 = (kc2 + 1) / 2;
      StepLaunch c{};
      c.var = L1_STEP; c.bf16 = bf; c.tile = tile; c.kc1 = kc1; c.kc2 = kc2;
      c.wW = lv.m_W; c.wKA = lv.m_KA; c.wKS = lv.m_KS; c.wSM = lv.m_sm[0];
      c.C = lv.C; c.cinp = ro.cinp; c.ncols = ro.ncols; c.nsteps = ro.nsteps; c.npairs = ro.npairs;
      c.n = lv.dims;
      if (mstep_lds_bytes(tile, bf, nct, ro.cinp, kc1, kc2) <= lds_max) cands.push_back(c);
    }
    if (cands.empty()) continue;
    if (!lv.e_alt) {
      lv.e_alt = (float*)alloc((size_t)lv.dims.total * lv.C * sizeof(float));
      if (!lv.e_alt) return fail(MCMG_E_OOM, "level allocation failed");
      hipError_t e = launch_zero_f32(lv.e_alt, lv.dims.total * lv.C, stream);
      if (e != hipSuccess) return fail(MCMG_E_HIP, "zero: %s", hipGetErrorString(e));
    }
    for (auto& c : cands) { c.e = lv.e; c.eo = lv.e_alt; c.r = lv.r; c.a = lv.a; c.s = lv.s; }
    char kb[160];
    snprintf(kb, sizeof(kb), "gfx950|%d|%s|step|%d|%dx%dx%d", dim, bf ? "bf16" : "f32", lv.C,
             lv.dims.n[0], lv.dims.n[1], lv.dims.n[2]);
    const std::string key = kb;
    int pick = -1;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      load_cache_locked();
      auto it = g_tune.find(key);
      if (it != g_tune.end())
        for (size_t k = 0; k < cands.size(); ++k)
          if (cands[k].tile == it->second.mt) pick = (int)k;
    }
    if (pick < 0) {
      pick = 0;
      if (tune && cands.size() > 1) {
        float best = 1e30f;
        for (size_t k = 0; k < cands.size(); ++k) {
          hipError_t e = launch_step(cands[k], stream);   // warm-up
          if (e != hipSuccess) return fail(MCMG_E_HIP, "tune: %s", hipGetErrorString(e));
          if ((e = hipEventRecord(ev0, stream)) != hipSuccess) return fail(MCMG_E_HIP, "tune event");
          for (int rep = 0; rep < 3; ++rep)
            if ((e = launch_step(cands[k], stream)) != hipSuccess) return fail(MCMG_E_HIP, "tune: %s", hipGetErrorString(e));
          if ((e = hipEventRecord(ev1, stream)) != hipSuccess) return fail(MCMG_E_HIP, "tune event");
          if ((e = hipEventSynchronize(ev1)) != hipSuccess) return fail(MCMG_E_HIP, "tune sync");
          float ms = 0.f;
          hipEventElapsedTime(&ms, ev0, ev1);
          if (ms < best) { best = ms; pick = (int)k; }
        }
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = Tile{cands[pick].tile, 0, 0};
        save_cache_locked();
      }
    }
    lv.step = cands[pick];
    lv.step_on = true;
  }
  // timing runs wrote into the work buffers; leave them clean
  for (auto& lv : lev) {
    const long long n = lv.dims.total * lv.C;
    if (lv.e_alt) {
      hipError_t e = launch_zero_f32(lv.e_alt, n, stream);
      if (e != hipSuccess) return fail(MCMG_E_HIP, "zero: %s", hipGetErrorString(e));
    }
    for (float* p : {lv.e, lv.r, lv.t, lv.u}) {
      hipError_t e = launch_zero_f32(p, n, stream);
      if (e != hipSuccess) return fail(MCMG_E_HIP, "zero: %s", hipGetErrorString(e));
    }
  }
  return MCMG_OK;
}

}  // namespace mcmg
