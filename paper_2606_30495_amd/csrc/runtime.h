// Handle state of libmcmg.so (one medium: operator, cached features,
// weights, V-cycle and Krylov workspace).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"
#include "mcmg.h"

namespace mcmg {

mcmg_status fail(mcmg_status s, const char* fmt, ...);

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
};

struct HostTensor {
  int kind, level, step, d0, d1;
  std::vector<float> w;
};

struct Ctx {
  int dim = 2;
  int nint[3] = {1, 1, 1};
  int next[3] = {1, 1, 1};
  int npml = 0;
  Dims interior{}, ext{};
  double omega = 0, h = 0, sigma_max = 0;
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

  ~Ctx();
  void* alloc(size_t bytes);
  mcmg_status parse_weights(const void* blob, size_t bytes);
  mcmg_status upload_weight(const float* src, int d0, int d1, bool transposed, float** dst);
  mcmg_status alloc_krylov();
  bool bf16_supported() const;
  hipError_t on_features_changed() { return hipSuccess; }

  hipError_t conv(int mode, int epi, int tin, const void* x, const Dims& in, int cin,
                  const float* w, const float* w2, int tout, void* y, const Dims& out, int cout,
                  const float* r, const float* feat);
  hipError_t dispatch_conv(const ConvLaunch& a);
  hipError_t vcycle(const void* rin, int tin, void* zout, int tout);
  hipError_t smooth_step(Level& lv, int i, bool first);
  hipError_t run_setup();
  HelmOp helm() const;
};

}  // namespace mcmg
