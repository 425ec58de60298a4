// Host drivers of LPA, Louvain and Leiden and the C ABI declared in include/mgcd.h.
//
// Louvain pass (Section 3.3, Section 4.1): synchronous local-moving sweeps until no
// vertex has a positive-gain move, the summed gain of those moves is at most the
// tolerance, or max_iterations; sweep t applies only moves to lower community ids
// (t even) or higher ids (t odd), which keeps pairs of vertices from swapping
// forever.  Then communities are renumbered densely (ascending old id) and, unless
// the pass kept more than aggregation_tolerance of its vertices or was the last,
// aggregated into super-vertices whose weighted degree is the exact sum of their
// members' (the total weight W stays the input's).  Leiden (Section 4.2) adds one
// refinement sweep inside each community, aggregates the refined partition
// symmetrically and starts the next pass from the (renumbered) communities.
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/mgcd.h"
#include "aggregate.hpp"
#include "batch.hpp"
#include "move.hpp"
#include "primitives.hpp"
#include "stepped.hpp"

namespace mgcd {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

// Sweeps issued between two host reads of a level's device-side state: the stopping
// rule is applied on the device after every sweep (LevelState), so a segment runs
// without host round trips; sweeps issued after the rule fired leave every vertex
// where it is.
constexpr int SEG = 4;

// Per-kernel-class device time of level-0 sweeps: four events per sweep of a segment.
struct ClassTimer {
  hipEvent_t ev[SEG][4] = {};
  ClassTimer() {
    for (auto &row : ev)
      for (auto &e : row) MGCD_HIP(hipEventCreate(&e));
  }
  ~ClassTimer() {
    for (auto &row : ev)
      for (auto &e : row)
        if (e) (void)hipEventDestroy(e);
  }
  void add(mgcd_stats &s, int j) {  // after sweep j of the segment has completed
    for (int q = 0; q < 3; ++q) {
      float ms = 0;
      MGCD_HIP(hipEventElapsedTime(&ms, ev[j][q], ev[j][q + 1]));
      s.ms_l0_kernel[q] += ms;
    }
    s.l0_sweeps += 1;
  }
};

static void check_params(const mgcd_params *p) {
  if (!p) throw Error(MGCD_E_ARG, "params is null");
  if (p->mode < 0 || (p->mode > 3 && p->mode != MGCD_MODE_SMALL))
    throw Error(MGCD_E_UNSUPPORTED, "unknown sketch mode");
  auto okk = [](int k) {
    return k == 1 || k == 2 || k == 4 || k == 8 || k == 16 || k == 32 || k == 64 || k == 128 || k == 256;
  };
  if (p->mode == MGCD_MODE_SMALL) {
    if (p->k < 1 || p->k > (1 << 30)) throw Error(MGCD_E_UNSUPPORTED, "small-table slots k must be in [1, 2^30]");
  } else if (p->mode != MGCD_MODE_EXACT && !okk(p->k)) {
    throw Error(MGCD_E_UNSUPPORTED, "k must be 1, 2, 4, 8, 16, 32, 64, 128 or 256");
  }
  if (p->aggregation < 0 || p->aggregation > 2) throw Error(MGCD_E_ARG, "aggregation must be 0, 1 or 2");
  if (p->storage_order < 0 || p->storage_order > 2) throw Error(MGCD_E_ARG, "storage_order must be 0, 1 or 2");
  if (p->short_rows < 0 || p->short_rows > 2) throw Error(MGCD_E_ARG, "short_rows must be 0, 1 or 2");
  if (agg_mode(p) != MGCD_MODE_EXACT && !okk(p->k_aggregate))
    throw Error(MGCD_E_UNSUPPORTED, "k_aggregate must be 1, 2, 4, 8, 16, 32, 64, 128 or 256");
  if (p->chunk_len < 1) throw Error(MGCD_E_ARG, "chunk_len must be >= 1");
  if (p->max_iterations < 1 || p->max_passes < 1) throw Error(MGCD_E_ARG, "iteration limits must be >= 1");
  if (!(p->tolerance >= 0.0) || !(p->tolerance_drop > 0.0) || !(p->aggregation_tolerance >= 0.0))
    throw Error(MGCD_E_ARG, "bad tolerance");
  const int rl = p->row_lanes;
  if (rl < 0 || rl > 64 || (rl & (rl - 1)) != 0)
    throw Error(MGCD_E_ARG, "row_lanes must be 0 or a power of two up to 64");
  if (p->direct_launch != 0 && p->direct_launch != 1) throw Error(MGCD_E_ARG, "direct_launch must be 0 or 1");
  if (p->one_scan != 0 && p->one_scan != 1) throw Error(MGCD_E_ARG, "one_scan must be 0 or 1");
  if (p->exact_small < 0 || p->exact_lds < 0 || p->exact_lds_big < 0)
    throw Error(MGCD_E_ARG, "exact tier bounds must be >= 0");
  const SchedParams sp = sched_params(p);
  if (sp.exact_t1 > EXACT_T1_MAX || sp.exact_t2 > EXACT_T2_MAX)
    throw Error(MGCD_E_ARG, "exact tier bounds must be at most 512 (exact_lds) and 4096 (exact_lds_big)");
}

// Level-0 local moving on the degree-ordered storage copy (schedule only): asked for,
// or by default when the input is large enough for the label gathers to miss the
// caches (the copy costs about one sweep's traffic; measured on R-MAT 2^20, 3.1e7
// entries, it saved less than it cost over the four level-0 sweeps, on Chung-Lu
// 2^24, 5.4e8 entries, a third of every sweep).
constexpr int64_t STORAGE_AUTO_NNZ = (int64_t)1 << 26;
static bool use_storage(const mgcd_params *p, int64_t nnz) {
  return p->storage_order == 2 || (p->storage_order == 0 && nnz >= STORAGE_AUTO_NNZ);
}

static Graph view(const mgcd_csr *g) {
  if (!g) throw Error(MGCD_E_ARG, "graph is null");
  if (g->n < 0 || g->nnz < 0) throw Error(MGCD_E_ARG, "negative graph size");
  if (g->n > 0 && (!g->offsets)) throw Error(MGCD_E_ARG, "offsets is null");
  if (g->nnz > 0 && (!g->indices || !g->weights)) throw Error(MGCD_E_ARG, "indices/weights null");
  if ((((uintptr_t)g->indices) | ((uintptr_t)g->weights)) & 15)
    throw Error(MGCD_E_ARG, "indices and weights must be 16-byte aligned");
  return Graph{g->n, g->nnz, g->offsets, g->indices, g->weights};
}

template <typename T>
static T read_dev(const T *p, hipStream_t st) {
  T h{};
  MGCD_HIP(hipMemcpyAsync(&h, p, sizeof(T), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  return h;
}

// Degrees, W, optional validation.  Returns W.
static uint64_t prepare(const Graph &g, const mgcd_params *p, uint32_t *K, Arena &a, hipStream_t st) {
  unsigned long long *scr = a.take<unsigned long long>(2);
  if (p && p->validate) {
    launch_zero_u64(scr, 2, st);
    launch_validate(g, scr, st);
    if (read_dev(scr, st) != 0) throw Error(MGCD_E_GRAPH, "CSR failed validation");
  }
  launch_degrees(g, K, scr + 1, a, st);
  uint64_t W = read_dev(scr + 1, st);
  if (W >= (1ull << 31)) throw Error(MGCD_E_OVERFLOW, "total edge weight must be below 2^31");
  return W;
}

static void require_labels(const int32_t *C, int64_t n, int64_t limit, Arena &a, hipStream_t st,
                           const char *what) {
  unsigned long long *flag = a.take<unsigned long long>(1);
  launch_check_labels(C, n, limit, flag, st);
  if (read_dev(flag, st) != 0) throw Error(MGCD_E_ARG, std::string(what) + " has values out of range");
}

// Runs the local-moving sweeps of one level: sweep(it, slot) issues sweep `it`
// (slot: its place in the segment, for the level-0 events) and returns nothing;
// the sweeps stop once the device-side stopping rule fired or after max_it sweeps.
// Returns the level's state; class timings of the counted sweeps go to `ct` when
// given.
struct Counts {
  unsigned long long moved, prop, sumG;
};

static Counts read_counts(const unsigned long long *ctr, hipStream_t st) {
  unsigned long long h[3];
  MGCD_HIP(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  return Counts{h[0], h[1], h[2]};
}

// grow: a segment that ends with the level still moving is followed by one twice as
// long.  The callers ask for it on aggregated levels of at most GROW_MAX_N vertices:
// such a level tends to run on (often to max_it), and there a sweep issued after the
// rule fired costs a few microseconds of launches and label copies, less than the host
// round trip it saves.
constexpr int32_t GROW_MAX_N = 1 << 21;
template <typename F>
static LevelState run_sweeps(int max_it, LevelState *ls, hipStream_t st, ClassTimer *ct, mgcd_stats &s,
                             bool grow, F &&sweep) {
  LevelState h{};
  int len = SEG;
  for (int it = 0; it < max_it;) {
    const int seg = max_it - it < len ? max_it - it : len;
    for (int j = 0; j < seg; ++j) sweep(it + j, j);
    const uint32_t before = h.sweeps;
    h = read_dev(ls, st);
    if (ct)
      for (uint32_t j = 0; j < h.sweeps - before; ++j) ct->add(s, (int)j);
    it += seg;
    if (h.halt) break;
    if (grow && !ct) len *= 2;
  }
  return h;
}

// ---- LPA ------------------------------------------------------------------------------

static void run_lpa(const mgcd_csr *gin, const mgcd_params *p, int32_t *out, Arena &a, hipStream_t st,
                    mgcd_stats *stats) {
  check_params(p);
  Graph g = view(gin);
  const int32_t n = g.n;
  Timer total(st), lm(st);
  total.start();
  uint32_t *K = a.take<uint32_t>(n);
  prepare(g, p, K, a, st);
  int32_t *Ca = a.take<int32_t>(n), *Cb = a.take<int32_t>(n);
  unsigned long long *ctr = a.take<unsigned long long>(4);
  launch_iota(Ca, n, st);
  // sweeps on the degree-ordered copy (labels by position, values the communities'
  // own ids), or on the input
  const bool sto = use_storage(p, g.nnz);
  StorageCopy sc{};
  Graph gs = g;
  uint32_t *Ks = K;
  int32_t *Ck = Ca;  // the labels the caller sees, by vertex
  if (sto) {
    sc = storage_copy(g, K, a, st);
    gs = sc.g;
    Ks = sc.Kp;
    Ca = a.take<int32_t>(n);
    launch_compose(sc.perm, Ck, Ca, n, st);  // Ca[p] = C[perm[p]]
  }
  if (n > 0) MGCD_HIP(hipMemcpyAsync(Cb, Ca, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  Schedule sch;
  build_schedule(gs, sched_params(p), sch, a, st);
  LevelState *ls = a.take<LevelState>(1);
  mgcd_stats s{};
  ClassTimer ct;
  lm.start();
  launch_zero_u64(ctr, 4, st);
  launch_zero_state(ls, st);
  if (n > 0) {
    LevelState h = run_sweeps(p->max_iterations, ls, st, &ct, s, false, [&](int it, int j) {
      SweepArgs args{gs, Ca, nullptr, Ks, nullptr, 0, 0, Cb, nullptr, ctr};
      args.halt = &ls->halt;
      args.one_scan = p->one_scan;
      args.ident = !sto && it == 0;  // every vertex starts alone (on the copy: C = perm)
      launch_sweep(args, sch, ALGO_LPA, p->mode, p->k, p->chunk_len, st, ct.ev[j]);
      launch_level_converge(ALGO_LPA, LevelRule{ctr, ls, g.nnz, n, p->tolerance, 0.0}, st);
      std::swap(Ca, Cb);  // a halted sweep copies C, so either buffer holds the result
    });
    s.iterations = h.sweeps;
    s.edges_scanned = (int64_t)h.edges;
    s.moved_last = (int64_t)h.moved_last;
  }
  if (sto) {  // back to vertices: C[v] = Ca[pos[v]]
    launch_compose(sc.pos, Ca, Ck, n, st);
    Ca = Ck;
  }
  const float ms_lm = lm.stop();
  s.communities = canonical(Ca, n, out, a, st);
  s.passes = 1;
  s.ms_local_move = ms_lm;
  s.ms_total = total.stop();
  if (stats) *stats = s;
}

// ---- Louvain / Leiden -------------------------------------------------------------------

static void run_levels(bool leiden, const mgcd_csr *gin, const mgcd_params *p, int32_t *out, Arena &a,
                       hipStream_t st, mgcd_stats *stats) {
  check_params(p);
  if (p->one_scan) throw Error(MGCD_E_UNSUPPORTED, "one_scan is defined for LPA only");
  Graph g0 = view(gin);
  const int32_t n = g0.n;
  const int64_t nnz = g0.nnz;
  Timer total(st), tm(st);
  total.start();
  mgcd_stats s{};
  uint32_t *Kbuf[2] = {a.take<uint32_t>(n), a.take<uint32_t>(n)};
  const uint64_t W = prepare(g0, p, Kbuf[0], a, st);
  int32_t *top = a.take<int32_t>(n);
  int32_t *Ca = a.take<int32_t>(n), *Cb = a.take<int32_t>(n);
  int32_t *D = a.take<int32_t>(n), *Dc = a.take<int32_t>(n);
  uint32_t *Sig = a.take<uint32_t>(n);
  int32_t *prop = leiden ? a.take<int32_t>(n) : nullptr;
  int32_t *nprop = leiden ? a.take<int32_t>(n) : nullptr;
  int32_t *from = leiden ? a.take<int32_t>(n) : nullptr;
  unsigned long long *ctr = a.take<unsigned long long>(4);
  LevelState *ls = a.take<LevelState>(1);
  struct Slot {
    int64_t *off;
    int32_t *idx;
    uint32_t *w;
  } slot[2];
  for (int q = 0; q < 2; ++q) {
    slot[q].off = a.take<int64_t>((int64_t)n + 1);
    slot[q].idx = a.take<int32_t>(nnz);
    slot[q].w = a.take<uint32_t>(nnz);
  }
  launch_iota(top, n, st);
  launch_iota(Ca, n, st);
  Graph cur = g0;
  int kcur = 0, next_slot = 0;
  double tol = p->tolerance;
  float ms_lm = 0, ms_ref = 0, ms_agg = 0;
  const double WW = (double)W * (double)W;
  ClassTimer ct;
  for (int pass = 0; pass < p->max_passes && n > 0; ++pass) {
    const int32_t nl = cur.n;
    uint32_t *K = Kbuf[kcur];
    s.passes += 1;
    size_t mark = a.mark();
    Schedule sch;
    tm.start();
    if (!leiden) launch_iota(Ca, nl, st);
    // level 0 may move on the degree-ordered copy: labels by position whose values are
    // the communities' own ids (keys, ties, directions and Sigma unchanged)
    const bool sto = pass == 0 && use_storage(p, cur.nnz);
    StorageCopy sc{};
    Graph gm = cur;
    uint32_t *Km = K;
    int32_t *Cv = Ca, *Cw = Cb;  // the vertex-space buffers
    if (sto) {
      sc = storage_copy(cur, K, a, st);
      gm = sc.g;
      Km = sc.Kp;
      Ca = a.take<int32_t>(nl);
      Cb = a.take<int32_t>(nl);
      launch_compose(sc.perm, Cv, Ca, nl, st);  // Ca[p] = C[perm[p]]
    }
    build_schedule(gm, sched_params(p), sch, a, st);
    // rows without entries are in no sweep: both label buffers start equal
    if (nl > 0) MGCD_HIP(hipMemcpyAsync(Cb, Ca, (size_t)nl * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    launch_community_totals(Ca, Km, Sig, nl, st);
    launch_zero_u64(ctr, 4, st);
    launch_zero_state(ls, st);
    LevelState h = run_sweeps(p->max_iterations, ls, st, pass == 0 ? &ct : nullptr, s,
                              pass > 0 && nl <= GROW_MAX_N, [&](int it, int j) {
      SweepArgs args{gm, Ca, nullptr, Km, Sig, W, (it % 2 == 0) ? -1 : 1, Cb, nullptr, ctr};
      args.halt = &ls->halt;
      // a level starts from singletons (Leiden after its first: from the refined
      // partition's communities); on the copy C holds perm, not positions
      args.ident = !sto && it == 0 && (!leiden || pass == 0);
      launch_sweep(args, sch, ALGO_MOVE, p->mode, p->k, p->chunk_len, st, pass == 0 ? ct.ev[j] : nullptr);
      // a sweep without positive moves, or a halted one, leaves C_new equal to C; the
      // same launch applies the stopping rule to this sweep's counters
      const LevelRule rule{ctr, ls, cur.nnz, nl, tol, WW};
      launch_apply_moves(Ca, Cb, Km, Sig, nl, st, &rule);
      std::swap(Ca, Cb);
    });
    if (sto) {  // back to vertices: C[v] = Ca[pos[v]]; refinement needs the input's schedule
      launch_compose(sc.pos, Ca, Cv, nl, st);
      Ca = Cv;
      Cb = Cw;
      if (leiden) build_schedule(cur, sched_params(p), sch, a, st);
    }
    ms_lm += tm.stop();
    if (pass == 0) s.l0_candidates = (int64_t)h.cands;
    s.iterations += h.sweeps;
    s.edges_scanned += (int64_t)h.edges;
    s.moved_last = (int64_t)h.moved_last;
    int32_t m;
    bool last;
    if (leiden) {
      tm.start();
      SweepArgs r{cur, nullptr, Ca, K, K, W, 0, prop, nullptr, ctr};
      launch_iota(prop, nl, st);  // a row without entries proposes itself
      launch_zero_u64(ctr, 4, st);
      launch_sweep(r, sch, ALGO_REFINE, p->mode, p->k, p->chunk_len, st);
      launch_refine_accept(prop, nprop, from, Cb, nl, st);  // Cb <- refined R
      ms_ref += tm.stop();
      a.release(mark);
      tm.start();
      m = renumber(Cb, nl, D, a, st);
      last = pass == p->max_passes - 1 || (double)m > p->aggregation_tolerance * (double)nl;
      if (last) {
        launch_compose(top, Ca, top, n, st);  // final community of every input vertex
        ms_agg += tm.stop();
        break;
      }
      renumber(Ca, nl, Dc, a, st);
      launch_compose(top, D, top, n, st);
    } else {
      a.release(mark);
      tm.start();
      m = renumber(Ca, nl, D, a, st);
      launch_compose(top, D, top, n, st);
      last = pass == p->max_passes - 1 || (double)m > p->aggregation_tolerance * (double)nl;
      if (last) {
        ms_agg += tm.stop();
        break;
      }
    }
    Slot &sl = slot[next_slot];
    int64_t nnz2 = aggregate(cur, D, m, agg_mode(p), p->k_aggregate, p->chunk_len, leiden ? 1 : 0, sl.off,
                             sl.idx, sl.w, a, st);
    launch_group_sums(D, K, Kbuf[1 - kcur], nl, m, st);
    if (leiden) {
      launch_scatter_labels(D, Dc, Cb, nl, st);  // super-vertex starts in its community
      std::swap(Ca, Cb);
    }
    ms_agg += tm.stop();
    cur = Graph{m, nnz2, sl.off, sl.idx, sl.w};
    next_slot = 1 - next_slot;
    kcur = 1 - kcur;
    tol /= p->tolerance_drop;
  }
  s.communities = canonical(top, n, out, a, st);
  s.ms_local_move = ms_lm;
  s.ms_refine = ms_ref;
  s.ms_aggregate = ms_agg;
  s.ms_total = total.stop();
  if (stats) *stats = s;
}

// ---- workspace ---------------------------------------------------------------------------

static size_t workspace_bytes(int32_t algo, int32_t n, int64_t nnz, const mgcd_params *p) {
  const int64_t L = p->chunk_len > 0 ? p->chunk_len : 1;
  size_t fixed = (size_t)n * 4 * 16 + 64 * 1024;
  if (algo != MGCD_ALGO_LPA) fixed += 2 * ((size_t)(n + 1) * 8 + (size_t)nnz * 8) + 4096;
  size_t sched = schedule_ws_bytes(n, nnz, sched_mode(p), p->k, L);
  // level 0 on the storage copy: the copy and two label buffers by position beside the
  // schedule of the copy (Leiden: and of the input, for the refinement)
  if (use_storage(p, nnz))
    sched = storage_ws_bytes(n, nnz) + (size_t)n * 8 + 8192 + sched * (algo == MGCD_ALGO_LEIDEN ? 2 : 1);
  size_t agg = algo == MGCD_ALGO_LPA ? 0 : aggregate_ws_bytes(n, nnz, agg_mode(p), p->k_aggregate, L, algo == MGCD_ALGO_LEIDEN);
  size_t misc = (size_t)n * (4 + 4 + 8 + 8) + scan_ws_bytes((int64_t)n + 1) + 16 * 1024;
  size_t degrees = degrees_ws_bytes(nnz);
  size_t phase = sched > agg ? sched : agg;
  phase = phase > degrees ? phase : degrees;
  return fixed + phase + misc + (1u << 20);
}

}  // namespace mgcd

// ---- C ABI ---------------------------------------------------------------------------------

using namespace mgcd;

template <typename F>
static int guarded(F &&f) {
  try {
    g_last_error.clear();
    f();
    return MGCD_OK;
  } catch (const Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return MGCD_E_ARG;
  } catch (...) {
    g_last_error = "unknown error";
    return MGCD_E_ARG;
  }
}

static Arena make_arena(void *ws, size_t bytes) {
  if (!ws && bytes) throw Error(MGCD_E_ARG, "workspace is null");
  Arena a;
  a.base = (char *)ws;
  a.cap = bytes;
  return a;
}

// Modularity (Section 3.2, Eq. 1) of membership C with a workspace of ws_bytes >=
// mgcd_modularity_workspace_bytes(g.n, g.nnz) at ws; everything it reads from the
// workspace it first writes there.  Synchronises st.
static void modularity_in(const Graph &g, const int32_t *C, double *q, void *ws, size_t ws_bytes,
                        hipStream_t st) {
  if (g.n == 0) {
    *q = 0.0;
    return;
  }
  Arena a = make_arena(ws, ws_bytes);
  require_labels(C, g.n, g.n, a, st, "communities");
  uint32_t *K = a.take<uint32_t>(g.n);
  unsigned long long *Wd = a.take<unsigned long long>(1);
  unsigned long long *terms = a.take<unsigned long long>(2 * SPREAD);
  launch_degrees(g, K, Wd, a, st);
  modularity_terms(g, C, K, terms, a, st);
  unsigned long long ht[2 * SPREAD], h[2] = {0, 0};
  MGCD_HIP(hipMemcpyAsync(ht, terms, sizeof(ht), hipMemcpyDeviceToHost, st));
  uint64_t W = read_dev(Wd, st);
  for (int c = 0; c < SPREAD; ++c) {
    h[0] += ht[2 * c];
    h[1] += ht[2 * c + 1];
  }
  if (W == 0) {
    *q = 0.0;
    return;
  }
  const double Wd_ = (double)W;
  *q = (double)h[0] / Wd_ - (double)h[1] / (Wd_ * Wd_);
}


// ---- device scratch of modularity_noalloc ---------------------------------------------
//
// One array per device, set aside when the library's code object is loaded there and
// held until the process ends.  Its device address is looked up once per device
// (hipGetSymbolAddress with that device current) and kept; host code uses only that
// address, never the array's name.  Every modularity_noalloc call on a device uses
// the same memory: calls that overlap on one device race.
constexpr size_t NOALLOC_SCRATCH_BYTES = ((size_t)64 << 20) + ((size_t)128 << 10);
static_assert((size_t)MGCD_NOALLOC_MAX_VERTICES * 16 + SPREAD * 8 + 4096 + 64 * 1024 <= NOALLOC_SCRATCH_BYTES,
              "the scratch must hold the modularity workspace of the largest accepted graph");
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_DEVICES] = {};

// The device address of `scratch` on the device of stream st (the current device for
// the null stream).
static void *scratch_of_stream(hipStream_t st) {
  int cur = 0, dev = 0;
  MGCD_HIP(hipGetDevice(&cur));
  dev = cur;
  if (st) MGCD_HIP(hipStreamGetDevice(st, &dev));
  if (dev < 0 || dev >= SCRATCH_DEVICES) throw Error(MGCD_E_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (dev != cur) MGCD_HIP(hipSetDevice(dev));
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (dev != cur) MGCD_HIP(hipSetDevice(cur));
    if (e != hipSuccess || !ptr)
      throw Error(MGCD_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// MGCD_MODE_BM is Algorithm 1 with one slot for local moving and refinement and four
// for aggregation (the weighted Boyer-Moore variant of Section 4.1); every entry
// point works on the resolved copy.
static mgcd_params resolved(const mgcd_params *p) {
  mgcd_params q{};
  if (!p) return q;
  q = *p;
  if (q.mode == MGCD_MODE_BM) {
    q.mode = MGCD_MODE_ALG1;
    q.k = 1;
    q.k_aggregate = 4;
  }
  return q;
}
mgcd_params mgcd::checked_params(const mgcd_params *p) {
  if (!p) throw Error(MGCD_E_ARG, "params is null");
  const mgcd_params q = resolved(p);
  check_params(&q);
  return q;
}

#define MGCD_RESOLVE(p)                 \
  const mgcd_params resolved_ = resolved(p); \
  if (p) p = &resolved_

extern "C" {

void mgcd_default_params(int32_t algo, mgcd_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->mode = MGCD_MODE_ALG1;
  p->k = algo == MGCD_ALGO_LEIDEN ? 16 : 8;
  p->k_aggregate = p->k;
  p->max_iterations = 20;
  p->max_passes = 10;
  p->validate = 0;
  p->chunk_len = 128;
  p->tolerance = algo == MGCD_ALGO_LPA ? 0.05 : 0.01;
  p->tolerance_drop = 10.0;
  p->aggregation_tolerance = 0.8;
}

size_t mgcd_workspace_bytes(int32_t algo, int32_t n, int64_t nnz, const mgcd_params *p) {
  MGCD_RESOLVE(p);
  mgcd_params d;
  if (!p) {
    mgcd_default_params(algo, &d);
    p = &d;
  }
  return workspace_bytes(algo, n < 0 ? 0 : n, nnz < 0 ? 0 : nnz, p);
}

static int run_checked(int32_t algo, const mgcd_csr *g, const mgcd_params *p, int32_t *out, void *ws,
                       size_t ws_bytes, mgcd_stats *stats, void *stream) {
  MGCD_RESOLVE(p);
  return guarded([&] {
    if (!g || !p) throw Error(MGCD_E_ARG, "null argument");
    if (g->n > 0 && !out) throw Error(MGCD_E_ARG, "communities_out is null");
    check_params(p);
    size_t need = workspace_bytes(algo, g->n, g->nnz, p);
    if (ws_bytes < need)
      throw Error(MGCD_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    Arena a = make_arena(ws, ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    if (algo == MGCD_ALGO_LPA)
      run_lpa(g, p, out, a, st, stats);
    else
      run_levels(algo == MGCD_ALGO_LEIDEN, g, p, out, a, st, stats);
  });
}

int lpa_run(const mgcd_csr *g, const mgcd_params *p, int32_t *out, void *ws, size_t ws_bytes,
            mgcd_stats *stats, void *stream) {
  return run_checked(MGCD_ALGO_LPA, g, p, out, ws, ws_bytes, stats, stream);
}

int louvain_run(const mgcd_csr *g, const mgcd_params *p, int32_t *out, void *ws, size_t ws_bytes,
                mgcd_stats *stats, void *stream) {
  return run_checked(MGCD_ALGO_LOUVAIN, g, p, out, ws, ws_bytes, stats, stream);
}

int leiden_run(const mgcd_csr *g, const mgcd_params *p, int32_t *out, void *ws, size_t ws_bytes,
               mgcd_stats *stats, void *stream) {
  return run_checked(MGCD_ALGO_LEIDEN, g, p, out, ws, ws_bytes, stats, stream);
}

size_t mgcd_modularity_workspace_bytes(int32_t n, int64_t nnz) {
  return (size_t)(n > 0 ? n : 0) * 16 + degrees_ws_bytes(nnz > 0 ? nnz : 0) + 64 * 1024;
}

int modularity(const mgcd_csr *gin, const int32_t *C, double *q, void *ws, size_t ws_bytes,
               void *stream) {
  return guarded([&] {
    if (!q) throw Error(MGCD_E_ARG, "q is null");
    Graph g = view(gin);
    if (g.n > 0 && !C) throw Error(MGCD_E_ARG, "communities is null");
    size_t need = mgcd_modularity_workspace_bytes(g.n, g.nnz);
    if (ws_bytes < need) throw Error(MGCD_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    modularity_in(g, C, q, ws, ws_bytes, (hipStream_t)stream);
  });
}

int modularity_noalloc(const mgcd_csr *gin, const int32_t *C, double *q, void *stream) {
  return guarded([&] {
    if (!q) throw Error(MGCD_E_ARG, "q is null");
    Graph g = view(gin);
    if (g.n > 0 && !C) throw Error(MGCD_E_ARG, "communities is null");
    size_t need = mgcd_modularity_workspace_bytes(g.n, g.nnz);
    if (g.n > MGCD_NOALLOC_MAX_VERTICES || need > NOALLOC_SCRATCH_BYTES)
      throw Error(MGCD_E_WORKSPACE, "modularity_noalloc handles at most " +
                                        std::to_string(MGCD_NOALLOC_MAX_VERTICES) + " vertices (this graph needs " +
                                        std::to_string(need) + " bytes of its " +
                                        std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte device scratch)");
    hipStream_t st = (hipStream_t)stream;
    modularity_in(g, C, q, scratch_of_stream(st), NOALLOC_SCRATCH_BYTES, st);
  });
}


int mgcd_move_sweep(const mgcd_csr *gin, const mgcd_params *p, int32_t algo, const int32_t *C,
                    int32_t direction, int32_t *C_new, int64_t *gain, int64_t *counters, void *ws,
                    size_t ws_bytes, void *stream) {
  MGCD_RESOLVE(p);
  return guarded([&] {
    check_params(p);
    Graph g = view(gin);
    if (algo != MGCD_ALGO_LPA && algo != MGCD_ALGO_LOUVAIN) throw Error(MGCD_E_ARG, "algo must be LPA or LOUVAIN");
    if (g.n > 0 && (!C || !C_new)) throw Error(MGCD_E_ARG, "membership is null");
    size_t need = workspace_bytes(MGCD_ALGO_LPA, g.n, g.nnz, p);
    if (ws_bytes < need) throw Error(MGCD_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    Arena a = make_arena(ws, ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    require_labels(C, g.n, g.n, a, st, "C");
    uint32_t *K = a.take<uint32_t>(g.n);
    uint64_t W = prepare(g, p, K, a, st);
    uint32_t *Sig = a.take<uint32_t>(g.n);
    unsigned long long *ctr = a.take<unsigned long long>(4);
    launch_community_totals(C, K, Sig, g.n, st);
    Schedule sch;
    build_schedule(g, sched_params(p), sch, a, st);
    launch_zero_u64(ctr, 4, st);
    // rows without entries are in no sweep: they keep their community and gain 0
    if (g.n > 0) MGCD_HIP(hipMemcpyAsync(C_new, C, (size_t)g.n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (gain) launch_zero_u64(reinterpret_cast<unsigned long long *>(gain), g.n, st);
    SweepArgs args{g, C, nullptr, K, Sig, W, direction < 0 ? -1 : direction > 0 ? 1 : 0, C_new, gain, ctr};
    args.one_scan = algo == MGCD_ALGO_LPA ? p->one_scan : 0;
    launch_sweep(args, sch, algo == MGCD_ALGO_LPA ? ALGO_LPA : ALGO_MOVE, p->mode, p->k, p->chunk_len, st);
    Counts c = read_counts(ctr, st);
    if (counters) {
      counters[0] = (int64_t)c.moved;
      counters[1] = (int64_t)c.prop;
      counters[2] = (int64_t)c.sumG;
    }
  });
}

int mgcd_refine(const mgcd_csr *gin, const mgcd_params *p, const int32_t *bound, int32_t *R, void *ws,
                size_t ws_bytes, void *stream) {
  MGCD_RESOLVE(p);
  return guarded([&] {
    check_params(p);
    Graph g = view(gin);
    if (g.n > 0 && (!bound || !R)) throw Error(MGCD_E_ARG, "bound or R is null");
    size_t need = workspace_bytes(MGCD_ALGO_LPA, g.n, g.nnz, p);
    if (ws_bytes < need) throw Error(MGCD_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    Arena a = make_arena(ws, ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    uint32_t *K = a.take<uint32_t>(g.n);
    uint64_t W = prepare(g, p, K, a, st);
    int32_t *prop = a.take<int32_t>(g.n), *nprop = a.take<int32_t>(g.n), *from = a.take<int32_t>(g.n);
    unsigned long long *ctr = a.take<unsigned long long>(4);
    Schedule sch;
    build_schedule(g, sched_params(p), sch, a, st);
    launch_zero_u64(ctr, 4, st);
    launch_iota(prop, g.n, st);  // a row without entries proposes itself
    SweepArgs r{g, nullptr, bound, K, K, W, 0, prop, nullptr, ctr};
    launch_sweep(r, sch, ALGO_REFINE, p->mode, p->k, p->chunk_len, st);
    launch_refine_accept(prop, nprop, from, R, g.n, st);
    MGCD_HIP(hipStreamSynchronize(st));
  });
}

int mgcd_aggregate(const mgcd_csr *gin, const mgcd_params *p, const int32_t *D, int32_t m,
                   int32_t symmetric, int64_t *out_off, int32_t *out_idx, uint32_t *out_w,
                   int64_t *out_nnz, void *ws, size_t ws_bytes, void *stream) {
  MGCD_RESOLVE(p);
  return guarded([&] {
    check_params(p);
    Graph g = view(gin);
    if (m < 0 || m > g.n) throw Error(MGCD_E_ARG, "m out of range");
    if (!out_off || (g.nnz > 0 && (!out_idx || !out_w)) || !out_nnz) throw Error(MGCD_E_ARG, "null output");
    size_t need = aggregate_ws_bytes(g.n, g.nnz, agg_mode(p), p->k_aggregate, p->chunk_len, symmetric != 0) + 64 * 1024;
    if (ws_bytes < need) throw Error(MGCD_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    Arena a = make_arena(ws, ws_bytes);
    hipStream_t st = (hipStream_t)stream;
    require_labels(D, g.n, m, a, st, "D");
    *out_nnz = aggregate(g, D, m, agg_mode(p), p->k_aggregate, p->chunk_len, symmetric ? 1 : 0, out_off,
                         out_idx, out_w, a, st);
    MGCD_HIP(hipStreamSynchronize(st));
  });
}

size_t mgcd_workspace_bytes_batched(int32_t algo, int32_t count, int64_t total_n, int64_t total_nnz,
                                    const mgcd_params *p) {
  MGCD_RESOLVE(p);
  mgcd_params d;
  if (!p) {
    mgcd_default_params(algo, &d);
    p = &d;
  }
  return batched_workspace_bytes(algo, count < 0 ? 0 : count, total_n < 0 ? 0 : total_n,
                                 total_nnz < 0 ? 0 : total_nnz, p);
}

static int run_batched_checked(int32_t algo, const mgcd_csr *graphs, int32_t count, const mgcd_params *p,
                               int32_t *const *outs, void *ws, size_t ws_bytes, mgcd_graph_stats *gs,
                               mgcd_stats *total, void *stream) {
  MGCD_RESOLVE(p);
  return guarded([&] {
    if (!graphs || !outs || count < 0) throw Error(MGCD_E_ARG, "null argument");
    check_params(p);
    if (p->one_scan && algo != MGCD_ALGO_LPA)
      throw Error(MGCD_E_UNSUPPORTED, "one_scan is defined for LPA only");
    int64_t N = 0, E = 0;
    for (int32_t g = 0; g < count; ++g) {
      N += graphs[g].n;
      E += graphs[g].nnz;
      if ((((uintptr_t)graphs[g].indices) | ((uintptr_t)graphs[g].weights)) & 15)
        throw Error(MGCD_E_ARG, "indices and weights must be 16-byte aligned");
    }
    if (N >= (1ll << 31)) throw Error(MGCD_E_ARG, "batched vertex total must be below 2^31");
    size_t need = batched_workspace_bytes(algo, count, N, E, p);
    if (ws_bytes < need) throw Error(MGCD_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
    Arena a = make_arena(ws, ws_bytes);
    if (count == 0) return;
    run_batched(algo, graphs, count, p, outs, a, (hipStream_t)stream, gs, total);
  });
}

int lpa_run_batched(const mgcd_csr *graphs, int32_t count, const mgcd_params *p, int32_t *const *outs,
                    void *ws, size_t ws_bytes, mgcd_graph_stats *gs, mgcd_stats *total, void *stream) {
  return run_batched_checked(MGCD_ALGO_LPA, graphs, count, p, outs, ws, ws_bytes, gs, total, stream);
}

int louvain_run_batched(const mgcd_csr *graphs, int32_t count, const mgcd_params *p, int32_t *const *outs,
                        void *ws, size_t ws_bytes, mgcd_graph_stats *gs, mgcd_stats *total,
                        void *stream) {
  return run_batched_checked(MGCD_ALGO_LOUVAIN, graphs, count, p, outs, ws, ws_bytes, gs, total, stream);
}

const char *mgcd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
