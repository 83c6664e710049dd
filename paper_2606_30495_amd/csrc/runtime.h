// Handle state of libmcmg.so (one medium: operator, cached features,
// weights, V-cycle and Krylov workspace).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "conv_mfma.h"
#include "internal.h"
#include "mcmg.h"
#include "step_mfma.h"

namespace mcmg {

mcmg_status fail(mcmg_status s, const char* fmt, ...);

// One matrix-core convolution instance: shapes, packing and tile choice.
struct MOp {
  bool on = false;
  int mode = 0, epi = 0, cin = 0, cout = 0, cinp = 0, ncols = 0, npairs = 0, nsteps = 0;
  int mt = 2, ntw = 1, rpw = 1, kchunk = 1;
  Dims in{}, out{};
};

struct Level {
  int n[3] = {1, 1, 1};
  Dims dims{};
  int C = 0;
  int nu1 = 0, nu2 = 0;
  float *a = nullptr, *s = nullptr;                     // cached features
  float *e = nullptr, *r = nullptr, *t = nullptr, *u = nullptr;   // work
  float *w_fs = nullptr, *w_W = nullptr, *w_KA = nullptr, *w_KS = nullptr;
  std::vector<float*> w_sm;
  float *w_fa = nullptr, *w_R = nullptr, *w_P = nullptr;
  // matrix-core plans and packed weights (op.on == false: VALU path)
  MOp op_resid, op_mul, op_set, op_add;   // stride-1 solve convolutions
  MOp op_R;                                // restriction this level -> next
  MOp op_P;                                // prolongation next level -> this
  void *m_W = nullptr, *m_KA = nullptr, *m_KS = nullptr, *m_R = nullptr, *m_P = nullptr;
  std::vector<void*> m_sm;
  // fused matrix-core smoothing step (2D, C >= 8): tile plan; e ping-pongs
  // with e_alt
  StepLaunch step{};
  bool step_on = false;
  // fused C = 2 sweep: per smoothing step weights; e ping-pongs with e_alt
  std::vector<L1Weights> l1w;
  std::vector<L1Weights*> l1w_dev;          // device copies (batched launches)
  float* e_alt = nullptr;
};

// Optional per-launch timing with HIP events on the handle's stream, with
// the algorithmic work of every launch (flops, bytes) from its shapes.  Each
// record keeps a by-value copy of its launch so that the launches of one
// kernel can be replayed back to back between a single event pair.
struct ProfRec {
  const char* name;
  double flops, bytes;
  hipEvent_t a, b;
  std::function<hipError_t()> replay;
};

struct Prof {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~Prof() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// A recorded launch of the V-cycle (record mode): the batched driver replays
// op i of every problem as one batched launch.
struct RecOp {
  int kind;                   // 0 VALU direct conv, 1 matrix-core conv, 2 fused C = 2 sweep,
                              // 3 fused matrix-core smoothing step
  ConvLaunch conv;
  MfmaConv mf;
  L1Launch l1;
  StepLaunch st;
  const L1Weights* l1w_dev;   // device copy of the sweep's weights
};

// One right-hand side's workspace: V-cycle level state and Krylov buffers.
struct Slot {
  std::vector<float*> e, r, t, u, e_alt;     // per level
  double *V = nullptr, *wv = nullptr, *rv = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr;
  double *g = nullptr, *y = nullptr, *coef = nullptr, *partial = nullptr, *scal = nullptr;
  float *Z = nullptr, *zt = nullptr;
  int* skip = nullptr;
  void* chunk = nullptr;                     // owning allocation (null: the handle's own)
  size_t bytes = 0;
};

struct HostTensor {
  int kind, level, step, d0, d1;
  std::vector<float> w;
};

// Born-series state: background, per-axis FFT plans and symbol tables.
struct BornAxis {
  int n = 1;
  std::vector<int> rad;      // radices in stage order
  int* plan = nullptr;       // device (radix, sub-length) per stage
  double2* tw = nullptr;     // device exp(-2 pi i j / n)
  int* rev = nullptr;        // device digit-reversal table
  double* d = nullptr;       // device (4/h^2) sin^2(pi m / n)
};
struct BornState {
  bool ready = false;
  double k0sq = 0, eps = 0;
  BornAxis ax[3];
  double* stats = nullptr;   // reduction partials
  int nstats = 0;
};

// Training state (train.cpp): parameters, gradients and Adam moments in the
// canonical blob layout, adjoint-layout copies of every tensor, and the tape
// of one forward pass.
struct TTensor {
  int kind = 0, level = 0, step = 0, d0 = 0, d1 = 0, mode = 0;
  size_t off = 0, len = 0;          // in the canonical flat vectors
  bool train = true;                // false: frozen (LLPF)
  float** fwd = nullptr;            // the handle's forward-layout pointer
  float* adj = nullptr;             // adjoint layout (nullptr: not needed)
  int adj_cin = 0, adj_cout = 0;
};
struct TrainState {
  std::vector<TTensor> ts;
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  size_t n = 0;
  int t = 0;                                    // Adam step count
  float* z_lift = nullptr;                      // setup pre-activations
  std::vector<float*> z_s, z_a;
  std::vector<std::vector<float*>> te, tt, tu;  // tape per level and step: e before, t, u
  std::vector<float*> rr, edown;                // restriction input, e after the down steps
  std::vector<float*> gde, gdr, gda, gds, t1, t2, t3;
  float *z2 = nullptr, *dz2 = nullptr, *rin32 = nullptr;
  double *wres = nullptr, *ahw = nullptr;
  float* part = nullptr;
  size_t part_cap = 0;
};

struct Ctx {
  int dim = 2;
  int nint[3] = {1, 1, 1};
  int next[3] = {1, 1, 1};
  int npml = 0;
  Dims interior{}, ext{};
  double omega = 0, h = 0, sigma_max = 0;
  int absorber = MCMG_ABL_PML;
  double gamma_max = 0;                 // sponge damping (absorber == MCMG_ABL_SPONGE)
  double* gtab[3] = {nullptr, nullptr, nullptr};
  int precision = MCMG_FP32, restart = 30, ortho = 0;
  hipStream_t stream = nullptr;

  int L = 0;
  std::vector<Level> lev;
  std::vector<HostTensor> host_w;
  float *w_flift = nullptr, *w_glift = nullptr, *w_gproj = nullptr;

  double* k2 = nullptr;
  double* cm[3] = {nullptr, nullptr, nullptr};
  double* cp[3] = {nullptr, nullptr, nullptr};
  float* mfeat = nullptr;

  // Krylov workspace
  double *V = nullptr, *wv = nullptr, *rv = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr;
  double *g = nullptr, *y = nullptr, *coef = nullptr, *partial = nullptr, *scal = nullptr;
  float *Z = nullptr, *zt = nullptr;
  int* skip = nullptr;
  int nb_red = 0;
  double* host_scal = nullptr;

  std::vector<void*> allocs;
  size_t device_bytes = 0;
  Prof prof;
  // record mode: launches are appended here instead of issued (batching)
  std::vector<RecOp>* rec = nullptr;
  // extra per-RHS workspaces (slot 0 is the handle's own buffers above)
  std::vector<Slot> slots;

  Slot current_slot() const;                // the buffers now bound
  void bind_slot(const Slot& s);            // bind another workspace
  mcmg_status ensure_slots(int n);          // slots 1..n-1 allocated
  mcmg_status alloc_slot(Slot& s);          // one device chunk
  void free_slot(Slot& s);
  size_t slot_bytes() const;                // device bytes of one extra slot
  size_t slot_layout(Slot* s, unsigned char* base) const;

  // `launch` must capture by value: it is kept for replay.
  template <class F>
  hipError_t timed(const char* name, double flops, double bytes, F launch) {
    if (!prof.on) return launch();
    hipEvent_t a = prof.get(), b = prof.get();
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, stream);
    prof.recs.push_back({name, flops, bytes, a, b, std::function<hipError_t()>(launch)});
    return e;
  }

  ~Ctx();
  void* alloc(size_t bytes);
  mcmg_status parse_weights(const void* blob, size_t bytes);
  mcmg_status upload_weight(const float* src, int d0, int d1, bool transposed, float** dst);
  mcmg_status alloc_krylov();
  hipError_t on_features_changed() { return hipSuccess; }

  hipError_t conv(int mode, int epi, int tin, const void* x, const Dims& in, int cin,
                  const float* w, const float* w2, int tout, void* y, const Dims& out, int cout,
                  const float* r, const float* feat);
  // stride-1 solve convolution on level lv: matrix cores when packed, else VALU
  hipError_t conv_level(Level& lv, int epi, const float* x, const float* w, const void* wm,
                        const float* w2, const void* wm2, float* y, const float* r,
                        const float* feat);
  mcmg_status plan_mfma();                 // pack weights, choose tiles (autotune)
  hipError_t run_mop(const MOp& op, const float* x, const void* wA, const void* wB, float* y,
                     const float* r, const float* feat);
  hipError_t dispatch_conv(const ConvLaunch& a);
  hipError_t vcycle(const void* rin, int tin, void* zout, int tout);
  hipError_t smooth_step(Level& lv, int i, bool first);
  hipError_t level1(Level& lv, int var, int step);   // fused C = 2 sweep
  mcmg_status plan_level1(bool refresh = false);
  mcmg_status refresh_level1();                 // re-derive level-1 sweep weights
  mcmg_status refresh_packed();                 // re-pack matrix-core weights (+ level 1)
  hipError_t run_setup();
  HelmOp helm() const;
  hipError_t helm_timed(int tin, const void* u, const double* f, double* out, double* partial);

  // training (train.cpp)
  TrainState* train = nullptr;
  mcmg_status train_init();
  hipError_t train_sync_weights();             // canonical -> forward and adjoint layouts
  hipError_t train_forward(const double* rin);
  hipError_t train_backward();
  hipError_t wgrad(int mode, int tx, const void* x, const Dims& in, int cin, const float* dy,
                   const Dims& out, int cout, const TTensor& t, float scale);
  mcmg_status repack_inference();              // MFMA packs, level-1 sweep weights, features

  // Born series (born.cpp)
  BornState born;
  mcmg_status born_setup(double k0sq, double eps);
  hipError_t green(const double* x, double* y, double* u_cbs);   // y = G x, or u += gamma G x
  hipError_t helm_periodic(const double* u, const double* f, double* out, double* partial);
};

}  // namespace mcmg
