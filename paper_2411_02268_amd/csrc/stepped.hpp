// Step-level serving (stepped.hip): the resident requests of a server advance
// together, one local-moving sweep (Section 3.2, the sweep of Louvain / LPA) per
// step, over the disjoint union of their current level graphs; a request whose level
// ended takes its phase transition (Leiden refinement, renumbering, aggregation,
// Section 3.3) on its own before the next step, and new requests join at the next
// step.
#pragma once
#include <string>
#include <vector>

#include "../../include/mgcd.h"
#include "common.hpp"

namespace mgcd {

// The parameters every call checks (mgcd_params as the calls resolve and check them;
// throws Error).
mgcd_params checked_params(const mgcd_params *p);

// One request as the engine sees it.  The caller sets g, out, block and user; the
// engine owns the rest and sets done once the request has finished.
struct StepJob {
  mgcd_csr g{};            // input graph (device arrays, untouched until done)
  int32_t *out = nullptr;  // device int32[g.n]: canonical labels
  char *block = nullptr;   // device, StepEngine::block_bytes(g.n, g.nnz): the job's state
  void *user = nullptr;
  // results, valid once done
  bool done = false;
  int rc = MGCD_OK;
  std::string err;
  mgcd_stats stats{};
  // state: the current level's graph and labels (block memory)
  Graph cur{};
  uint32_t *K[2] = {nullptr, nullptr};
  int kcur = 0;
  int32_t *C = nullptr, *top = nullptr, *D = nullptr, *Dc = nullptr, *R = nullptr;
  uint32_t *Sig = nullptr;
  int64_t *soff[2] = {nullptr, nullptr};
  int32_t *sidx[2] = {nullptr, nullptr};
  uint32_t *sw[2] = {nullptr, nullptr};
  int next_slot = 0;
  uint64_t W = 0;
  int pass = 0;  // level
  int it = 0;    // sweeps made at this level
  double tol = 0;
  double t_admit = 0;  // host seconds
};

class StepEngine {
 public:
  // algo: MGCD_ALGO_*; p: checked (checked_params); a step makes up to
  // sweeps_per_step sweeps (<= 0: max_iterations, every level to its end); the shared
  // region holds the union during steps and the phase work between them; phase work
  // runs on up to phase_lanes streams at once (st and streams of the engine's own), on
  // the device current at construction.
  StepEngine(int algo, const mgcd_params &p, int sweeps_per_step, char *shared, size_t shared_bytes,
             hipStream_t st, int phase_lanes);
  ~StepEngine();
  StepEngine(const StepEngine &) = delete;
  StepEngine &operator=(const StepEngine &) = delete;

  // Bytes of a job's own block, and of the shared region for `count` resident jobs of
  // N vertices and E entries in all, the largest of them max_n / max_nnz.
  static size_t block_bytes(int algo, const mgcd_params &p, int32_t n, int64_t nnz);
  static size_t shared_need(int algo, const mgcd_params &p, int64_t count, int64_t N, int64_t E,
                            int32_t max_n, int64_t max_nnz);
  static size_t phase_bytes(int algo, const mgcd_params &p, int32_t n, int64_t nnz);

  // Takes jobs in (they join the union at the next step).  A job that fails its checks
  // or has nothing to move finishes at once and is appended to `finished`.
  void admit(const std::vector<StepJob *> &js, std::vector<StepJob *> &finished);
  // One step: up to sweeps_per_step sweeps over every resident job (a job whose level
  // ends stays frozen for the rest of the step), then the phase transitions of the jobs
  // whose level ended; jobs that finished are appended to `finished`.
  void step(std::vector<StepJob *> &finished);
  // After an error the engine cannot recover from: every resident job fails.
  void fail_all(int code, const std::string &msg, std::vector<StepJob *> &finished);
  size_t resident() const { return jobs_.size(); }
  const mgcd_step_stats &counters() const { return ctr_; }

 private:
  struct Union;
  struct Lane {  // a stream and its slice of the shared region for phase work
    hipStream_t st;
    char *base;
    size_t cap;
    Arena arena() const {
      Arena a;
      a.base = base;
      a.cap = cap;
      return a;
    }
  };
  void dissolve();
  void repack();
  void batched_end(const std::vector<int32_t> &eg);
  template <typename F>
  void in_lanes(const std::vector<StepJob *> &js, F &&f);
  bool prepare(StepJob *j, const Lane &l);
  void admit_together(const std::vector<StepJob *> &js);
  void enter_level(StepJob *j, bool reset, const Lane &l);
  void end_level(StepJob *j, const Lane &l);
  void finish(StepJob *j, const int32_t *labels, const Lane &l);

  int algo_;
  mgcd_params p_;
  int sweeps_;
  char *shared_;
  size_t shared_bytes_;
  hipStream_t st_;
  int device_ = 0;
  std::vector<hipStream_t> lanes_;  // lanes_[0] = st_
  std::vector<StepJob *> jobs_;  // resident, in admission order
  mgcd_step_stats ctr_{};
  Union *u_;
};

}  // namespace mgcd
