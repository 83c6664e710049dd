// z = MG(r) without any allocation: the V-cycle's level state (e, r, t, u
// and the ping-pong e of every level) lives in one file-scope device array
// instead of the handle's own buffers, for callers that cannot allocate
// (code under stream capture, serving loops that forbid hipMalloc).
//
// The array holds SCRATCH_BYTES on every GPU the library runs on, until the
// process ends.  Host code never uses the array's name as an address: its
// device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and kept per device.  Every call on a GPU
// shares that GPU's array, so calls that overlap on one GPU (two streams,
// two threads) race; the region a call uses is cleared by a fill kernel
// first, since the array keeps the previous call's contents.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "internal.h"
#include "mcmg.h"
#include "runtime.h"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;   // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, unsigned char*> g_ptr;   // device -> address of `scratch` there

// Device address of this device's array (looked up on first use, with the
// device current).
mcmg_status scratch_ptr(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ptr.find(dev);
  if (it != g_ptr.end()) {
    *out = it->second;
    return MCMG_OK;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return mcmg::fail(MCMG_E_HIP, "hipGetDevice failed");
  if (cur != dev && hipSetDevice(dev) != hipSuccess)
    return mcmg::fail(MCMG_E_HIP, "hipSetDevice(%d) failed", dev);
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p)
    return mcmg::fail(MCMG_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_ptr[dev] = (unsigned char*)p;
  *out = (unsigned char*)p;
  return MCMG_OK;
}

// Level state of the handle carved from `base` (null: only measured), in the
// layout of the handle's own buffers; returns the bytes used.  ptr[l] gets
// level l's (e, r, t, u, e_alt).
constexpr int MAXL = 8;   // levels a weight blob can describe
size_t carve_levels(const mcmg::Ctx* c, float* (*ptr)[5], unsigned char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> float* {
    const size_t at = off;
    off = (off + bytes + 255) / 256 * 256;
    return base ? (float*)(base + at) : nullptr;
  };
  for (int l = 0; l < c->L; ++l) {
    const mcmg::Level& lv = c->lev[l];
    const size_t nb = (size_t)lv.dims.total * lv.C * sizeof(float);
    float* e = take(nb);
    float* r = take(nb);
    float* t = take(nb);
    float* u = take(nb);
    float* ea = lv.e_alt ? take(nb) : nullptr;
    if (ptr) {
      ptr[l][0] = e; ptr[l][1] = r; ptr[l][2] = t; ptr[l][3] = u; ptr[l][4] = ea;
    }
  }
  return off;
}

void bind_levels(mcmg::Ctx* c, float* (*ptr)[5]) {
  for (int l = 0; l < c->L; ++l) {
    mcmg::Level& lv = c->lev[l];
    lv.e = ptr[l][0]; lv.r = ptr[l][1]; lv.t = ptr[l][2]; lv.u = ptr[l][3]; lv.e_alt = ptr[l][4];
  }
}

}  // namespace

using namespace mcmg;

extern "C" mcmg_status mcmg_apply_noalloc(mcmg_handle h, const double* r, double* z) {
  if (!h || !r || !z) return fail(MCMG_E_ARG, "null argument");
  if ((const void*)r == (const void*)z) return fail(MCMG_E_ARG, "r and z may not alias");
  Ctx* c = (Ctx*)h;
  if (c->rec) return fail(MCMG_E_ARG, "handle is recording a batched schedule");
  const size_t need = carve_levels(c, nullptr, nullptr);
  if (need > SCRATCH_BYTES)
    return fail(MCMG_E_ARG,
                "the V-cycle state of this grid needs %zu bytes; the no-allocation entry point "
                "holds %zu", need, SCRATCH_BYTES);
  // the handle's memory tells which device it lives on
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, c->lev[0].a) != hipSuccess)
    return fail(MCMG_E_HIP, "cannot query the handle's device");
  unsigned char* base = nullptr;
  mcmg_status st = scratch_ptr(attr.device, &base);
  if (st != MCMG_OK) return st;
  if (c->L > MAXL) return fail(MCMG_E_ARG, "more than %d levels", MAXL);
  // the handle's own level buffers, and the scratch carved the same way
  // (fixed arrays: no host allocation either)
  float* own[MAXL][5];
  float* tmp[MAXL][5];
  for (int l = 0; l < c->L; ++l) {
    const Level& lv = c->lev[l];
    own[l][0] = lv.e; own[l][1] = lv.r; own[l][2] = lv.t; own[l][3] = lv.u; own[l][4] = lv.e_alt;
  }
  carve_levels(c, tmp, base);
  hipError_t e = launch_zero_f32((float*)base, (long long)(need / sizeof(float)), c->stream);
  if (e != hipSuccess) return fail(MCMG_E_HIP, "scratch clear: %s", hipGetErrorString(e));
  // bind the scratch levels, run the V-cycle on the handle's stream, then
  // give the handle its own buffers back (profiling paused: its per-launch
  // events are created on demand)
  const bool prof_on = c->prof.on;
  c->prof.on = false;
  bind_levels(c, tmp);
  e = c->vcycle(r, T_F64, z, T_F64);
  bind_levels(c, own);
  c->prof.on = prof_on;
  if (e != hipSuccess) return fail(MCMG_E_HIP, "apply: %s", hipGetErrorString(e));
  return MCMG_OK;
}
