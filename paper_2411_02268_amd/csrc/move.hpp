// Local-moving sweeps (host launchers; kernels in move.hip).
#pragma once
#include "common.hpp"
#include "mgcd.h"

namespace mgcd {

// Everything one synchronous sweep reads and writes.
struct SweepArgs {
  Graph g;
  const int32_t *C;      // membership before the sweep (unused by refinement: keys are j)
  const int32_t *bound;  // refinement only: the local-moving community C_B
  const uint32_t *K;     // weighted degree of every vertex
  const uint32_t *Sig;   // Sigma of every community (refinement: K itself)
  uint64_t W;            // total edge weight 2m
  int32_t dir;           // -1 lower ids only, +1 higher ids only, 0 any
  int32_t *Cnew;         // new membership (refinement: proposed target)
  int64_t *gain;         // optional: gain of each vertex's best move
  unsigned long long *ctr;  // [moved, proposals, sum of gains, candidates] (device)
  // Batched runs (many graphs as one disjoint union): graph of every vertex, its
  // graph's total weight, whether that graph still moves, per-graph counters
  // [3 * graph + {moved, proposals, sum of gains}].  Null for a single graph.
  const int32_t *gid = nullptr;
  const uint32_t *Wg = nullptr;
  const uint8_t *active = nullptr;
  unsigned long long *gctr = nullptr;
  // Batched runs: graphs still moving after the previous sweep (device); at 0 every
  // sweep kernel returns at once.  queue: the QLANES work counters of the persistent
  // main sweep kernel (QSTRIDE apart, zero before the sweep); null launches it with
  // one wave per work item.
  const uint32_t *live = nullptr;
  unsigned long long *queue = nullptr;
  // Graphs at different sweeps of their own levels (serving): each graph's direction
  // (-1, +1 or 0), by graph; null: every vertex takes `dir`.
  const int8_t *gdir = nullptr;
  // Single graph: a device flag; once set, every vertex keeps its community (the
  // sweep only copies C to C_new).  Null: always move.
  const uint32_t *halt = nullptr;
  // LPA, the 1-scan variant (Section 4.3): every row decides from its sketch's values
  // (treated as exact), so no row takes the second pass.
  int32_t one_scan = 0;
  // The small mod-based table of Appendix A.2 (exact kernels only): 0 = the exact
  // table; S > 0 = key c counts in slot c mod S, whose first key (in stream order)
  // stands for every key that lands there.
  int32_t small_slots = 0;
  // C is the identity (every vertex alone, C[j] = j: the first sweep of a level that
  // starts from singletons): the kernels may take a neighbour's community as j without
  // reading C, which must still hold the identity.
  int32_t ident = 0;
};

// The table key of community (or vertex) c: itself, or its slot in the small table.
__device__ inline uint32_t slot_of(const SweepArgs &a, uint32_t c) {
  return a.small_slots > 0 ? c % (uint32_t)a.small_slots : c;
}

// Whether a row whose sketch lost weight still needs the second pass.
__host__ __device__ inline bool second_pass(const SweepArgs &a, int algo) { return !(algo == ALGO_LPA && a.one_scan); }

// A single graph's level, kept on the device so that sweeps need no host round trip:
// set `halt` when the level's stopping rule fires; count sweeps, streamed entries,
// the last sweep's movers and the candidate communities (c != d) whose totals the
// main sweep kernel read (Louvain/Leiden; a measurement figure only).
struct LevelState {
  uint32_t halt;
  uint32_t sweeps;
  unsigned long long edges;
  unsigned long long moved_last;
  unsigned long long cands;
};
// A level's stopping rule: LPA stops when movers <= tol * n, Louvain local moving
// when no vertex has a positive move or 2 * summed gain <= tol * W^2 (WW = W^2).
// The sweep counters ctr [moved, proposals, sum of gains, candidates] are read and
// cleared.
struct LevelRule {
  unsigned long long *ctr = nullptr;
  LevelState *ls = nullptr;
  int64_t nnz = 0;  // entries streamed per sweep
  int32_t n = 0;
  double tol = 0, WW = 0;
  const uint32_t *live = nullptr;  // batched: 0 graphs moving -> no Sigma update
};
// After a sweep: apply the rule to the sweep's counters and update the state.
void launch_level_converge(int algo, const LevelRule &r, hipStream_t st);
void launch_zero_state(LevelState *ls, hipStream_t st);

// The persistent main sweep kernel's work queue: QLANES counters, each on a cache line
// of its own (QSTRIDE u64 apart); counter c hands out work items c, c + QLANES, ...
// (an interleaved share of the heaviest-first order), QGRAB at a time, so that the
// waves' atomics spread over QLANES addresses and a grab serves many items.
constexpr int QLANES = 64, QSTRIDE = 16, QGRAB = 16;

// Row buckets of the main sweep kernel: rows needing 2^b lanes (b = 0..6).
// The grid of the main sweep kernel: first one wave per group of 64 chunks of the
// long rows (more than 64 chunks), then the row buckets.
struct Buckets {
  int64_t wave_begin[7];  // row waves of bucket b: [wave_begin[b], wave_end[b]), counted
  int64_t wave_end[7];    // after the long-row groups; b = 6 first; wave_end[0] = total
  const int32_t *rows[7];
  int64_t nrows[7];
  int64_t ngroups;        // long-row groups (their waves come first)
  const int32_t *multi;   // long rows
  const int32_t *gowner;  // [ngroups] long row of each group
  const int64_t *gstart;  // [nmulti+1] first group of each long row
  const int64_t *cstart;  // [nmulti+1] first chunk of each long row
  Pair *sk;               // [ngroups * k] group roots
  uint32_t *skflag;       // [ngroups] group lost weight
};

// Per-level work lists, built once per level by build_schedule.
struct Schedule {
  // MG mode
  int32_t *single = nullptr;  // vertices whose row fits one chunk (deg <= L), heavy first
  int64_t nsingle = 0;
  int32_t *packed[7] = {};    // [b] long rows of at most 2^b chunks (b = 1..6)
  int64_t npacked[7] = {};
  int32_t *multi = nullptr;   // rows of more than 64 chunks, ascending id
  int64_t nmulti = 0;
  int64_t *cstart = nullptr;  // [nmulti+1] first chunk of each multi vertex
  int32_t *owner = nullptr;   // [nchunks] multi index of each chunk
  int64_t nchunks = 0;
  int64_t maxdeg = 0;          // longest row
  Buckets buckets{};           // bucket table of k_move_rows (passed by value)
  int64_t row_waves = 0;
  uint32_t *keybuf = nullptr; // [nnz] keys C[j] gathered in pass 1, read by pass 2
  int64_t *gstart = nullptr;  // [nmulti+1] first group of 64 chunks of each multi vertex
  int32_t *gowner = nullptr;  // [ngroups] multi index of each group
  int64_t ngroups = 0;
  Pair *sk = nullptr;         // [ngroups * k] merged sketch of each group of 64 chunks
  uint32_t *skflag = nullptr; // [ngroups] some sketch or merge of the group lost weight
  uint32_t *part = nullptr;   // [nchunks * (k+1)] pass-2 counts per chunk of a lossy long row
  Pair *cand = nullptr;       // [nmulti * k] merged candidates of each long row
  uint32_t *cflag = nullptr;  // [nmulti] 0 decided, 1 lossy, 2 frozen
  // MG with K = 32 / 64: multi, cstart and owner list the split rows and their chunks
  Pair *wnode = nullptr;      // [nchunks * k] chunk sketches, merged in place level by level
  uint32_t *wflag = nullptr;  // [nchunks] the node's sketches or merges lost weight
  uint32_t *wcount = nullptr; // [nmulti * (k+1)] pass-2 counts per candidate slot, then K_{i->d}
  // exact mode
  int32_t *tier[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t ntier[4] = {0, 0, 0, 0};
  int64_t *hbase = nullptr;   // [ntier[3]+1] global hash region of each tier-3 vertex
  Pair *htab = nullptr;
  uint32_t *hpos = nullptr;   // small table: first row position of each global slot
  int64_t *sstart = nullptr;  // [ntier[3]+1] first insert segment (GSEG entries) of each row
  int32_t *sowner = nullptr;  // [nseg] tier-3 index of each segment
  int64_t nseg = 0;
  int64_t *tstart = nullptr;  // [ntier[3]+1] first scan segment (TSEG table slots) of each row
  int32_t *towner = nullptr;  // [ntseg] tier-3 index of each scan segment
  int64_t ntseg = 0;
  uint32_t *gkd = nullptr;    // [ntier[3]] K_{i->d} of each row
  int32_t *pbest = nullptr;   // [ntseg] best candidate of each scan segment
  int64_t *pgain = nullptr;   // [ntseg] its gain
};

// What a level's schedule depends on.  mode, k and L change results; the rest only
// changes which kernel and mapping takes a row (results never change):
//   row_lanes_log2: rows of more than 2^row_lanes_log2 chunks (at most 64) take the
//                   long-row path;
//   exact_t0/t1/t2: exact mode, rows of at most t0 entries use one lane each, at most
//                   t1 (<= 512) the 1024-slot LDS table, at most t2 (<= 4096) the
//                   8192-slot LDS table, longer rows a global table.
struct SchedParams {
  int mode = MODE_ALG1;
  int k = 8;
  int64_t L = 128;
  int row_lanes_log2 = 6;
  int64_t exact_t0 = 32, exact_t1 = 512, exact_t2 = 4096;
  bool wave = false;  // K = 32 / 64: rows of at most exact_t0 entries exact, the rest one
                      // wave each
  // K <= 16, Algorithm 1 or the textbook rule: rows of at most mg_short entries hold at
  // most K distinct keys, so no update or merge ever removes weight and the sketch is
  // the row's exact table; they take the exact one-lane kernel (0: none).  short_auto:
  // only when the graph's average row has at most mg_short entries (most rows are
  // short; on skewed graphs the extra launch costs more than the rows it takes over)
  int64_t mg_short = 0;
  bool short_auto = false;
};
constexpr int64_t EXACT_T1_MAX = 512, EXACT_T2_MAX = 4096;
// exact mode, global tables: entries inserted by one workgroup, slots scored by one
constexpr int64_t GSEG = 4096, TSEG = 8192;
// K = 32 / 64: rows of more than max(L, WAVE_SPLIT) entries are split over one wave per
// chunk (schedule only: the merge tree and the results are those of one wave per row)
constexpr int64_t WAVE_SPLIT = 512;

void build_schedule(const Graph &g, const SchedParams &sp, Schedule &s, Arena &a, hipStream_t st);

// The schedule parameters of a call (0 in a schedule field selects its default).
// The small table (MGCD_MODE_SMALL) runs on the exact kernels' schedule: the mode
// that local-moving schedules see.
inline int sched_mode(const mgcd_params *p) {
  return p->mode == MGCD_MODE_SMALL ? MGCD_MODE_EXACT : p->mode;
}
// The mode of aggregation: as the moving mode (the small table aggregates exactly),
// or the exact rows / Algorithm 1 sketch that `aggregation` asks for.
inline int agg_mode(const mgcd_params *p) {
  if (p->aggregation == MGCD_AGG_EXACT) return MGCD_MODE_EXACT;
  if (p->aggregation == MGCD_AGG_SKETCH) return MGCD_MODE_ALG1;
  return sched_mode(p);
}

inline SchedParams sched_params(const mgcd_params *p) {
  SchedParams sp;
  sp.mode = p->mode == MGCD_MODE_SMALL ? MGCD_MODE_EXACT : p->mode;  // small: exact tiers
  sp.k = p->k;
  sp.L = p->chunk_len;
  if (p->row_lanes > 0) {
    int b = 0;
    while ((1 << b) < p->row_lanes) ++b;
    sp.row_lanes_log2 = b;
  }
  if (p->exact_small > 0) sp.exact_t0 = p->exact_small;
  if (p->exact_lds > 0) sp.exact_t1 = p->exact_lds;
  if (p->exact_lds_big > 0) sp.exact_t2 = p->exact_lds_big;
  if (sp.exact_t1 < sp.exact_t0) sp.exact_t1 = sp.exact_t0;
  if (sp.exact_t2 < sp.exact_t1) sp.exact_t2 = sp.exact_t1;
  if ((p->mode == MGCD_MODE_ALG1 || p->mode == MGCD_MODE_STD) && p->k <= 16 && p->short_rows != 1) {
    sp.mg_short = p->k;
    sp.short_auto = p->short_rows == 0;
  }
  if (sp.mode != MGCD_MODE_EXACT && p->k > 16) {
    // a stream of at most 32 items cannot lose weight in a sketch of >= 32 slots under
    // Algorithm 1 or the textbook rule (a free slot is always left); the unconditional
    // rule subtracts on every miss, so it takes the sketch for every row
    sp.wave = true;
    sp.exact_t0 = p->mode == MGCD_MODE_UNCOND ? 0 : 32;
  }
  return sp;
}
size_t schedule_ws_bytes(int32_t n, int64_t nnz, int mode, int k, int64_t L);

// One sweep of `algo` (ALGO_LPA / ALGO_MOVE / ALGO_REFINE) over all vertices.
// ev (optional, 4 events): recorded before the first kernel class and after each
// of the three classes, for per-class timing.
void launch_sweep(const SweepArgs &a, const Schedule &s, int algo, int mode, int k, int64_t L,
                  hipStream_t st, hipEvent_t *ev = nullptr);

// Sigma[c] -= K_i, Sigma[c'] += K_i for every vertex that moved from c to c'.  With
// a rule, the same launch first applies the Louvain stopping rule of that level
// (as launch_level_converge with ALGO_MOVE).
void launch_apply_moves(const int32_t *Cold, const int32_t *Cnew, const uint32_t *K, uint32_t *Sig,
                        int32_t n, hipStream_t st, const LevelRule *rule = nullptr);
// Sigma of a membership from scratch.
void launch_community_totals(const int32_t *C, const uint32_t *K, uint32_t *Sig, int32_t n,
                             hipStream_t st);
// Leiden refinement acceptance: R[i] = prop[i] unless a vertex other than the target
// proposed i, or the target proposed i and has the higher id.
void launch_refine_accept(const int32_t *prop, int32_t *nprop, int32_t *from, int32_t *R, int32_t n,
                          hipStream_t st);
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
void launch_iota(int32_t *p, int64_t n, hipStream_t st);
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st);

}  // namespace mgcd
