// Batch engine: many FGMRES solves (media of uneven grid sizes, several
// right-hand sides per medium) advanced together, one launch per operation.
//
// Every solve is a Work: its handle, a workspace slot, f and u, and a small
// host state machine.  Each tick advances every Work by one step of its own:
//
//   INIT  |f| and the true residual r = f - A u, then V_0 = r / |r|
//   ITER  one FGMRES iteration at the Work's own Krylov position j
//         (V-cycle, matvec, two-pass classical Gram-Schmidt, Givens)
//   END   close the cycle: H y = g, u += Z y, true residual, V_0 = r / |r|
//
// so Works restart independently and a Work admitted mid-flight starts at
// once (continuous batching).  The step of each Work is selected on the
// device by per-Work masks and positions uploaded before the tick (a few
// ints per Work); the launch sequence of a tick depends only on the set of
// Works (the composition), so it is captured once into a HIP graph and
// replayed until the composition changes.  Only 4 doubles per Work come back
// to the host per tick.
//
// Works do not interact: every kernel reads and writes only its own Work's
// buffers, and every reduction is per Work in a fixed order, so a result is
// bitwise the same whatever else shares the tick.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "runtime.h"

namespace mcmg {

struct Work {
  Ctx* c = nullptr;
  Slot* slot = nullptr;
  const double* f = nullptr;
  double* u = nullptr;
  double tol = 1e-6;
  int maxit = 0;
  uint64_t tag = 0;                  // caller's identifier
  enum State { INIT, ITER, END, DONE };
  State st = INIT;
  int j = 0, k = 0, its = 0, restarts = 0;
  double fnorm = 0, target = 0, relres = 0, relest = 0;
  std::vector<double> hist;
  mcmg_status status = MCMG_OK;
  std::vector<std::vector<RecOp>> ops;   // V-cycle launches per Krylov position
};

class Engine {
 public:
  Engine() = default;
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  ~Engine();

  // The first handle fixes the family (dimension, levels, channels,
  // smoothing counts, precision, restart, kernel plan kinds).
  mcmg_status open(const Ctx* model);
  bool compatible(const Ctx* c, std::string* why) const;
  // Records the Work's V-cycle launches; the composition changes.
  mcmg_status add(Work* w);
  // Removes DONE Works (composition changes when any is removed).
  void drop_done();
  // One tick: issue() enqueues it on the engine stream, complete() waits for
  // it and advances the host states; Works that finished are appended.
  mcmg_status issue();
  mcmg_status complete(std::vector<Work*>* finished);
  int live() const;
  int size() const { return (int)works_.size(); }
  hipStream_t stream() const { return s_; }
  bool use_graphs = true;
  long long rebuilds = 0;          // composition changes seen (tables rebuilt)

 private:
  mcmg_status build();
  hipError_t body(bool all_phases);
  void free_tables();

  hipStream_t s_ = nullptr;
  int dim_ = 0, L_ = 0, prec_ = 0, m_ = 0, ortho_ = 0;
  std::vector<int> C_, nu1_, nu2_, l1_, mf_;
  std::vector<int> kinds_;
  std::vector<Work*> works_;
  bool dirty_ = true;

  // device tables of the current composition
  struct OpTable {
    int kind;
    RecOp proto;
    size_t tab_off, pre_off;
    int total;
    bool jdep;
  };
  std::vector<OpTable> vt_;
  size_t hmv_off_ = 0, hres_off_ = 0, karg_off_ = 0, pre_red_off_ = 0, pre_elem_off_ = 0;
  int total_red_ = 0, total_elem_ = 0;
  void* dev_ = nullptr;
  size_t dev_cap_ = 0;
  int* ctl_dev_ = nullptr;        // 6 * n ints: iter, end, res, init masks, jpos, kk
  double* gather_dev_ = nullptr;  // 4 * n doubles
  int* ctl_host_ = nullptr;       // pinned
  double* gather_host_ = nullptr; // pinned
  int host_cap_ = 0;
  int np_ = 0;
  hipGraphExec_t graph_ = nullptr;
  int ticks_same_ = 0;            // ticks since the composition last changed
  bool issued_ = false;
};

}  // namespace mcmg
