// Step-level serving: every resident request advances together, sweep by sweep.
//
// While the resident set and their levels stay the same, their current level graphs
// live packed as one disjoint union in the shared region (vertex and entry ids shifted
// by each graph's base), with the union's labels, community totals and schedule.  A
// step is up to S sweeps of Louvain's local moving (or LPA) over the union, each
// followed by the Sigma update and each graph's own stopping rule (Section 3.2, with
// its own W, sweep direction and tolerance) on the device: a graph whose level ended
// is frozen for the rest of the step (its rows copy their labels), and once none moves
// the step's remaining kernels return at once; the host reads the outcome once per
// step.  When some graph's level ended, or requests join, the union is dissolved: labels and community totals go back to each request's
// own block, the graphs whose level ended take their phase transition alone (Leiden
// refinement, renumbering and aggregation, Section 3.3; or their final labels), and
// the next step packs the union anew.  Because a graph's sweeps read only its own
// rows, labels and totals, and every rule is per graph, each request's labels equal
// those of its own call.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <exception>
#include <string>
#include <thread>
#include <vector>

#include "aggregate.hpp"
#include "move.hpp"
#include "primitives.hpp"
#include "stepped.hpp"

namespace mgcd {

namespace {

unsigned grid_of(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, BLOCK); }

double host_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One graph of the union: where its level graph and state live, and its place in the
// union.
struct PackDesc {
  const int64_t *off;
  const int32_t *idx;
  const uint32_t *w;
  int32_t *C;
  uint32_t *Sig;  // null for LPA
  const uint32_t *K;
  int64_t n, nnz, vbase, ebase;
};

// A graph's outcome of one step: movers of its last sweep, sweeps made, whether its
// level ended.
struct StepResult {
  unsigned long long moved;
  uint32_t sweeps;
  uint32_t ended;
};

// Graph y0 + blockIdx.y into the union: its rows (offsets, ids shifted by its bases),
// its vertices' graph, degree, label (both buffers) and community total.
__global__ void k_step_pack(const PackDesc *d, int32_t y0, int64_t *off, int32_t *idx, uint32_t *w,
                            int32_t *gid, int32_t *C0, int32_t *C1, uint32_t *K, uint32_t *Sig) {
  const int32_t gi = y0 + (int32_t)blockIdx.y;
  const PackDesc g = d[gi];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < g.n; v += stride) {
    const int64_t u = g.vbase + v;
    off[u] = g.ebase + g.off[v];
    gid[u] = gi;
    K[u] = g.K[v];
    const int32_t c = (int32_t)(g.vbase + g.C[v]);
    C0[u] = c;
    C1[u] = c;
    if (Sig) Sig[u] = g.Sig[v];
  }
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < g.nnz; e += stride) {
    idx[g.ebase + e] = (int32_t)(g.vbase + g.idx[e]);
    w[g.ebase + e] = g.w[e];
  }
}

__global__ void k_step_last_offset(int64_t *off, int64_t n, int64_t E) { off[n] = E; }

// Labels (back to the graph's own ids) and community totals from the union to each
// graph's block.
__global__ void k_step_unpack(const PackDesc *d, const int32_t *gid, const int32_t *C, const uint32_t *Sig,
                              int64_t N) {
  const int64_t u = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (u >= N) return;
  const PackDesc g = d[gid[u]];
  const int64_t v = u - g.vbase;
  g.C[v] = C[u] - (int32_t)g.vbase;
  if (Sig) g.Sig[v] = Sig[u];
}

// Start of a step: every graph of the union moves (lv = {graphs moving, sweeps in
// which some graph moved}), no outcome yet.
__global__ void k_step_begin(uint32_t *lv, int32_t count, StepResult *res) {
  for (int64_t g = threadIdx.x; g < count; g += BLOCK) res[g] = StepResult{0ull, 0u, 0u};
  if (threadIdx.x == 0) {
    lv[0] = (uint32_t)count;
    lv[1] = 0;
  }
}

// After a sweep, per graph (one workgroup, graphs strided over its threads): its
// counters are read and cleared; a graph still moving counts the sweep and ends its
// level when its stopping rule fires -- LPA: movers <= tol * n_g; Louvain: no positive
// move, or 2 * (summed gain) <= tol * W_g^2, the tests of a call's own level -- or at
// max_it sweeps; its next sweep alternates direction (lower ids first).  A graph whose
// level ended is frozen for the rest of the step.  lv[0] = graphs still moving (0:
// every later sweep kernel of the step returns at once), lv[1] counts the sweeps in
// which some graph moved.
template <int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_step_converge(unsigned long long *gctr, const unsigned long long *Wg64, const int64_t *nvert,
                    const double *gtol, int32_t *git, int8_t *gdir, uint8_t *active, int32_t max_it,
                    int32_t count, StepResult *res, uint32_t *lv) {
  __shared__ uint32_t red[BLOCK / WAVE];
  const uint32_t was = lv[0];
  uint32_t still = 0;
  for (int64_t g = threadIdx.x; g < count; g += BLOCK) {
    unsigned long long *c = gctr + 3 * g;
    // read and clear in one atomic step (a plain load could be served by the scalar
    // cache and be overtaken by the store of 0)
    const unsigned long long moved = atomicExch(&c[0], 0ull), prop = atomicExch(&c[1], 0ull),
                             sumG = atomicExch(&c[2], 0ull);
    if (!active[g]) continue;
    bool stop;
    if (ALGO == ALGO_LPA) {
      stop = (double)moved <= gtol[g] * (double)nvert[g];
    } else {
      const double WW = (double)Wg64[g] * (double)Wg64[g];
      stop = prop == 0 || 2.0 * (double)sumG <= gtol[g] * WW;
    }
    const int32_t it = git[g] + 1;
    git[g] = it;
    if (gdir) gdir[g] = it % 2 == 0 ? (int8_t)-1 : (int8_t)1;
    StepResult r = res[g];
    r.moved = moved;
    r.sweeps += 1;
    if (stop || it >= max_it) {
      r.ended = 1;
      active[g] = 0;
    } else {
      still += 1;
    }
    res[g] = r;
  }
  still = block_sum(still, red);
  if (threadIdx.x == 0) {
    lv[0] = still;
    lv[1] += was > 0 ? 1u : 0u;
  }
}

// ---- phase transitions of many graphs at once (LPA, Louvain) --------------------------

// out[q] = src[pos[q]].
__global__ void k_step_gather(const int64_t *src, const int64_t *pos, int64_t *out, int32_t count) {
  const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (q < count) out[q] = src[pos[q]];
}

// A graph's level map into the union's renumbering: top[v] = D[vbase + top[v]] - db
// (D: dense ids over the graphs renumbered together; the graph's are db, db + 1, ...).
struct ComposeDesc {
  int32_t *top;
  int64_t n, vbase, db;
};
__global__ void k_step_compose(const ComposeDesc *d, int32_t y0, const int32_t *D) {
  const ComposeDesc c = d[y0 + (int32_t)blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < c.n; v += stride)
    c.top[v] = (int32_t)(D[c.vbase + c.top[v]] - c.db);
}

// Canonical labels of many graphs at once: graph f's labels lab[0, n) (values < n)
// and vertices take the global places off .. off + n - 1; a community is numbered by
// the rank of its smallest vertex among the communities of its graph.
struct CanonDesc {
  const int32_t *lab;
  int32_t *out;
  int64_t n, off;
};
__global__ void k_canon_min(const CanonDesc *d, int32_t y0, int32_t *minv) {
  const CanonDesc c = d[y0 + (int32_t)blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < c.n; v += stride)
    atomicMin(&minv[c.off + c.lab[v]], (int32_t)(c.off + v));
}
__global__ void k_canon_first(const CanonDesc *d, int32_t y0, const int32_t *minv, uint32_t *first) {
  const CanonDesc c = d[y0 + (int32_t)blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < c.n; v += stride)
    first[c.off + v] = minv[c.off + c.lab[v]] == (int32_t)(c.off + v) ? 1u : 0u;
}
__global__ void k_canon_write(const CanonDesc *d, int32_t y0, const int32_t *minv, const int64_t *rank) {
  const CanonDesc c = d[y0 + (int32_t)blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < c.n; v += stride)
    c.out[v] = (int32_t)(rank[minv[c.off + c.lab[v]]] - rank[c.off]);
}

// The next level of a graph out of the union's aggregation: its rows are db .. db + m - 1
// and its entries eb .. ee - 1 of (off, idx, w), ids shifted down by db; its degrees K'
// and the start of its next level (every vertex alone: C = iota, Sigma = K').
struct OutDesc {
  int64_t *off;
  int32_t *idx;
  uint32_t *w;
  uint32_t *K, *Sig;
  int32_t *C;
  int64_t db, m, eb, ee;
};
__global__ void k_step_copy_out(const OutDesc *d, int32_t y0, const int64_t *off, const int32_t *idx,
                                const uint32_t *w, const uint32_t *K) {
  const OutDesc o = d[y0 + (int32_t)blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r <= o.m; r += stride) {
    o.off[r] = off[o.db + r] - o.eb;
    if (r < o.m) {
      const uint32_t k = K[o.db + r];
      o.K[r] = k;
      o.Sig[r] = k;
      o.C[r] = (int32_t)r;
    }
  }
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < o.ee - o.eb; e += stride) {
    o.idx[e] = (int32_t)(idx[o.eb + e] - o.db);
    o.w[e] = w[o.eb + e];
  }
}

// Level 0 of admitted graphs: every vertex alone (C = iota, top = iota) and the
// community totals of that membership (Sigma = K).
struct StartDesc {
  int32_t *C, *top;  // top: null for LPA
  uint32_t *Sig;     // null for LPA
  const uint32_t *K;
  int64_t n;
};
__global__ void k_admit_start(const StartDesc *d, int32_t y0) {
  const StartDesc s = d[y0 + (int32_t)blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < s.n; v += stride) {
    s.C[v] = (int32_t)v;
    if (s.top) s.top[v] = (int32_t)v;
    if (s.Sig) s.Sig[v] = s.K[v];
  }
}

size_t up(size_t b) { return (b + 255) & ~(size_t)255; }

// Per-graph table of the union (one upload): its parts at these byte offsets.
struct TableLayout {
  size_t desc, Wg, Wg64, active, nvert, gtol, git, gdir, total;
  explicit TableLayout(int64_t count) {
    size_t o = 0;
    auto put = [&](size_t bytes) {
      const size_t at = o;
      o = up(o + bytes);
      return at;
    };
    desc = put((size_t)count * sizeof(PackDesc));
    Wg = put((size_t)count * 4);
    Wg64 = put((size_t)count * 8);
    active = put((size_t)count);
    nvert = put((size_t)count * 8);
    gtol = put((size_t)count * 8);
    git = put((size_t)count * 4);
    gdir = put((size_t)count);
    total = o;
  }
};

}  // namespace

struct StepEngine::Union {
  bool live = false;
  Arena a;
  Graph g{};
  int32_t count = 0;
  int32_t *gid = nullptr;
  int32_t *C[2] = {nullptr, nullptr};
  uint32_t *K = nullptr, *Sig = nullptr;
  char *table = nullptr;
  PackDesc *desc = nullptr;
  uint32_t *Wg = nullptr;
  unsigned long long *Wg64 = nullptr;
  uint8_t *active = nullptr;
  int64_t *nvert = nullptr;
  double *gtol = nullptr;
  int32_t *git = nullptr;
  int8_t *gdir = nullptr;
  unsigned long long *gctr = nullptr, *ctr = nullptr;
  StepResult *res = nullptr;
  uint32_t *lv = nullptr;
  size_t mark_sched = 0;        // u.a before the schedule (released by batched transitions)
  std::vector<PackDesc> hd;     // host copy of the graphs' places
  Schedule sch;
  std::vector<StepResult> hres;
};

StepEngine::StepEngine(int algo, const mgcd_params &p, int sweeps_per_step, char *shared, size_t shared_bytes,
                       hipStream_t st, int phase_lanes)
    : algo_(algo),
      p_(p),
      sweeps_(sweeps_per_step > 0 ? sweeps_per_step : p.max_iterations),
      shared_(shared),
      shared_bytes_(shared_bytes),
      st_(st),
      u_(new Union) {
  MGCD_HIP(hipGetDevice(&device_));
  lanes_.push_back(st_);
  for (int t = 1; t < phase_lanes; ++t) {
    hipStream_t x = nullptr;
    MGCD_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    lanes_.push_back(x);
  }
}

StepEngine::~StepEngine() {
  for (size_t t = 1; t < lanes_.size(); ++t) (void)hipStreamDestroy(lanes_[t]);
  delete u_;
}

// A job's block: degrees, labels and (Louvain / Leiden) the level maps and the two
// slots of aggregated level graphs, as in a call of its own.
static void block_layout(int algo, StepJob *j, Arena &a) {
  const int32_t n = j->g.n;
  const int64_t nnz = j->g.nnz;
  j->K[0] = a.take<uint32_t>(n);
  j->C = a.take<int32_t>(n);
  if (algo == MGCD_ALGO_LPA) return;
  j->K[1] = a.take<uint32_t>(n);
  j->Sig = a.take<uint32_t>(n);
  j->top = a.take<int32_t>(n);
  j->D = a.take<int32_t>(n);
  if (algo == MGCD_ALGO_LEIDEN) {
    j->Dc = a.take<int32_t>(n);
    j->R = a.take<int32_t>(n);
  }
  for (int q = 0; q < 2; ++q) {
    j->soff[q] = a.take<int64_t>((int64_t)n + 1);
    j->sidx[q] = a.take<int32_t>(nnz);
    j->sw[q] = a.take<uint32_t>(nnz);
  }
}

size_t StepEngine::block_bytes(int algo, const mgcd_params &, int32_t n, int64_t nnz) {
  StepJob j;
  j.g.n = n < 0 ? 0 : n;
  j.g.nnz = nnz < 0 ? 0 : nnz;
  Arena a;
  a.dry = true;
  block_layout(algo, &j, a);
  return up(a.peak) + 4096;
}

// The phase work of one job: admission (degrees, validation), Leiden refinement (its
// schedule and proposal arrays), renumbering, aggregation, final labels.
size_t StepEngine::phase_bytes(int algo, const mgcd_params &p, int32_t n, int64_t nnz) {
  const int64_t L = p.chunk_len > 0 ? p.chunk_len : 1;
  size_t ph = degrees_ws_bytes(nnz);
  if (algo != MGCD_ALGO_LPA) {
    ph = std::max(ph, aggregate_ws_bytes(n, nnz, agg_mode(&p), p.k_aggregate, L, algo == MGCD_ALGO_LEIDEN));
    if (algo == MGCD_ALGO_LEIDEN)
      ph = std::max(ph, schedule_ws_bytes(n, nnz, sched_mode(&p), p.k, L) + (size_t)n * 12 + 8192);
  }
  return ph + (size_t)n * (4 + 4 + 8 + 8) + scan_ws_bytes((int64_t)n + 1) + 64 * 1024 + (1u << 20);
}

size_t StepEngine::shared_need(int algo, const mgcd_params &p, int64_t count, int64_t N, int64_t E,
                               int32_t max_n, int64_t max_nnz) {
  const int64_t L = p.chunk_len > 0 ? p.chunk_len : 1;
  // the union: rows, entries, per-vertex state, per-graph table, counters, schedule
  size_t un = up((size_t)(N + 1) * 8) + up((size_t)E * 4) * 2 + up((size_t)N * 4) * 5;
  un += TableLayout(count).total + up((size_t)count * 24) + up((size_t)count * sizeof(StepResult)) + 4096;
  const int32_t n32 = (int32_t)std::min<int64_t>(N, INT32_MAX);
  // after the arrays: the schedule, or (LPA, Louvain) the transitions made together in
  // its place (two renumberings, canonical labels, the aggregated union and its degrees,
  // small tables)
  size_t after = schedule_ws_bytes(n32, E, sched_mode(&p), p.k, L);
  if (algo != MGCD_ALGO_LEIDEN) {
    size_t b = (size_t)count * 512 + (size_t)N * 96 + (size_t)E * 8 + 2 * scan_ws_bytes(N + 1) + 256 * 1024;
    if (algo == MGCD_ALGO_LOUVAIN) b += aggregate_ws_bytes(n32, E, agg_mode(&p), p.k_aggregate, L, false);
    after = std::max(after, b);
  }
  un += after + 64 * 1024 + (1u << 20);
  return std::max(un, phase_bytes(algo, p, max_n, max_nnz));
}

// Phase work of many jobs over the phase lanes: each lane has its own stream and an
// equal slice of the shared region (as many lanes as slices that hold the largest
// job's phase work), takes the next job until none is left and drains its stream.
// Runs while the union is dissolved, after the main stream's work.
template <typename F>
void StepEngine::in_lanes(const std::vector<StepJob *> &js, F &&f) {
  if (u_->live) throw Error(MGCD_E_ARG, "internal: phase work while the union is packed");
  if (js.empty()) return;
  MGCD_HIP(hipStreamSynchronize(st_));
  size_t need = 0;
  for (StepJob *j : js) need = std::max(need, phase_bytes(algo_, p_, j->g.n, j->g.nnz));  // the input bounds every level
  int T = (int)std::min<size_t>(lanes_.size(), js.size());
  while (T > 1 && shared_bytes_ / (size_t)T / 256 * 256 < need) --T;
  const size_t slice = T > 1 ? shared_bytes_ / (size_t)T / 256 * 256 : shared_bytes_;
  std::atomic<size_t> next{0};
  std::vector<std::exception_ptr> err((size_t)T);
  auto work = [&](int t) {
    try {
      MGCD_HIP(hipSetDevice(device_));
      const Lane l{lanes_[(size_t)t], shared_ + (size_t)t * slice, slice};
      for (size_t q; (q = next.fetch_add(1)) < js.size();) f(js[q], l);
      MGCD_HIP(hipStreamSynchronize(l.st));
    } catch (...) {
      err[(size_t)t] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(work, t);
  work(0);
  for (auto &x : th) x.join();
  for (auto &e : err)
    if (e) std::rethrow_exception(e);
}

// Host checks, degrees and W of a job; false when it finished here (an error, or no
// vertices).
bool StepEngine::prepare(StepJob *j, const Lane &l) {
  const mgcd_csr &c = j->g;
  try {
    if (c.n < 0 || c.nnz < 0) throw Error(MGCD_E_ARG, "negative graph size");
    if (c.n > 0 && (!c.offsets || !j->out)) throw Error(MGCD_E_ARG, "offsets or communities_out is null");
    if (c.nnz > 0 && (!c.indices || !c.weights)) throw Error(MGCD_E_ARG, "indices/weights null");
    if ((((uintptr_t)c.indices) | ((uintptr_t)c.weights)) & 15)
      throw Error(MGCD_E_ARG, "indices and weights must be 16-byte aligned");
    if (c.n == 0) {  // nothing to move: the call's own result
      j->stats.passes = algo_ == MGCD_ALGO_LPA ? 1 : 0;
      j->done = true;
      return false;
    }
    Arena b;
    b.base = j->block;
    b.cap = block_bytes(algo_, p_, c.n, c.nnz);
    block_layout(algo_, j, b);
    const Graph g{c.n, c.nnz, c.offsets, c.indices, c.weights};
    Arena a = l.arena();
    unsigned long long *scr = a.take<unsigned long long>(2);
    unsigned long long h = 0;
    if (p_.validate) {  // before anything reads the rows
      launch_zero_u64(scr, 2, l.st);
      launch_validate(g, scr, l.st);
      MGCD_HIP(hipMemcpyAsync(&h, scr, sizeof(h), hipMemcpyDeviceToHost, l.st));
      MGCD_HIP(hipStreamSynchronize(l.st));
      if (h != 0) throw Error(MGCD_E_GRAPH, "CSR failed validation");
    }
    launch_degrees(g, j->K[0], scr + 1, a, l.st);
    MGCD_HIP(hipMemcpyAsync(&h, scr + 1, sizeof(h), hipMemcpyDeviceToHost, l.st));
    MGCD_HIP(hipStreamSynchronize(l.st));
    if (h >= (1ull << 31)) throw Error(MGCD_E_OVERFLOW, "total edge weight must be below 2^31");
    j->W = h;
    j->cur = g;
    j->kcur = 0;
    j->next_slot = 0;
    j->pass = 0;
    j->tol = p_.tolerance;
    if (algo_ != MGCD_ALGO_LPA) launch_iota(j->top, c.n, l.st);
  } catch (const Error &e) {
    if (e.code == MGCD_E_HIP) throw;
    j->rc = e.code;
    j->err = e.what();
    j->done = true;
    return false;
  }
  enter_level(j, true, l);
  return true;
}

// Host -> device copy of a small table (the stream is synchronised before it returns,
// so the host buffer may go).
template <typename T>
static T *upload(Arena &a, const std::vector<T> &h, hipStream_t st) {
  T *d = a.take<T>((int64_t)h.size());
  if (!h.empty()) {
    MGCD_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
    MGCD_HIP(hipStreamSynchronize(st));
  }
  return d;
}

// src[pos[q]] for the host positions pos, read back to the host.
static std::vector<int64_t> gather(Arena &a, const int64_t *src, const std::vector<int64_t> &pos,
                                   hipStream_t st) {
  std::vector<int64_t> h(pos.size(), 0);
  if (pos.empty()) return h;
  const size_t mk = a.mark();
  const int64_t *pd = upload(a, pos, st);
  int64_t *od = a.take<int64_t>((int64_t)pos.size());
  k_step_gather<<<grid_of((int64_t)pos.size()), BLOCK, 0, st>>>(src, pd, od, (int32_t)pos.size());
  MGCD_LAUNCHED();
  MGCD_HIP(hipMemcpyAsync(h.data(), od, h.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  a.release(mk);
  return h;
}

// Launch `kernel` with grid y over the table's entries (65,535 at a time) and x over the
// longest entry's `len` items.
template <typename D, typename F>
static void per_graph(const D *dd, int32_t count, int64_t len, hipStream_t st, F &&launch) {
  for (int32_t y0 = 0; y0 < count; y0 += 65535) {
    const int32_t ny = std::min<int32_t>(65535, count - y0);
    dim3 grid((unsigned)std::min<int64_t>(ceil_div(len > 0 ? len : 1, BLOCK), 4096), (unsigned)ny);
    launch(grid, y0);
    MGCD_LAUNCHED();
  }
  (void)dd;
}

void StepEngine::admit(const std::vector<StepJob *> &js, std::vector<StepJob *> &finished) {
  if (js.empty()) return;
  dissolve();
  const double t0 = host_seconds();
  for (StepJob *j : js) {
    j->t_admit = t0;
    j->done = false;
    j->rc = MGCD_OK;
    j->stats = mgcd_stats{};
    j->cur = Graph{};
  }
  try {
    if (p_.validate)  // each graph checked before anything reads its rows
      in_lanes(js, [&](StepJob *j, const Lane &l) { prepare(j, l); });
    else
      admit_together(js);
  } catch (...) {
    ctr_.s_admit += host_seconds() - t0;
    throw;
  }
  for (StepJob *j : js) {  // in arrival order
    if (j->done)
      finished.push_back(j);
    else
      jobs_.push_back(j);
  }
  ctr_.s_admit += host_seconds() - t0;
}

// Admission of many graphs without validation: every graph's degrees and W issued on
// the main stream one after the other with no host round trip between them, the W
// read back once, then every level 0 started by one launch.  A graph whose W does not
// fit 32 bits finishes with MGCD_E_OVERFLOW.
void StepEngine::admit_together(const std::vector<StepJob *> &js) {
  hipStream_t st = st_;
  Arena a = Lane{st, shared_, shared_bytes_}.arena();
  std::vector<StepJob *> ok;
  for (StepJob *j : js) {
    const mgcd_csr &c = j->g;
    try {
      if (c.n < 0 || c.nnz < 0) throw Error(MGCD_E_ARG, "negative graph size");
      if (c.n > 0 && (!c.offsets || !j->out)) throw Error(MGCD_E_ARG, "offsets or communities_out is null");
      if (c.nnz > 0 && (!c.indices || !c.weights)) throw Error(MGCD_E_ARG, "indices/weights null");
      if ((((uintptr_t)c.indices) | ((uintptr_t)c.weights)) & 15)
        throw Error(MGCD_E_ARG, "indices and weights must be 16-byte aligned");
    } catch (const Error &e) {
      j->rc = e.code;
      j->err = e.what();
      j->done = true;
      continue;
    }
    if (c.n == 0) {  // nothing to move: the call's own result
      j->stats.passes = algo_ == MGCD_ALGO_LPA ? 1 : 0;
      j->done = true;
      continue;
    }
    Arena b;
    b.base = j->block;
    b.cap = block_bytes(algo_, p_, c.n, c.nnz);
    block_layout(algo_, j, b);
    ok.push_back(j);
  }
  if (ok.empty()) return;
  unsigned long long *Wd = a.take<unsigned long long>((int64_t)ok.size());
  for (size_t q = 0; q < ok.size(); ++q) {
    const mgcd_csr &c = ok[q]->g;
    launch_degrees(Graph{c.n, c.nnz, c.offsets, c.indices, c.weights}, ok[q]->K[0], Wd + q, a, st);
  }
  std::vector<unsigned long long> W(ok.size());
  MGCD_HIP(hipMemcpyAsync(W.data(), Wd, W.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  std::vector<StartDesc> sd;
  int64_t nmax = 1;
  for (size_t q = 0; q < ok.size(); ++q) {
    StepJob *j = ok[q];
    if (W[q] >= (1ull << 31)) {
      j->rc = MGCD_E_OVERFLOW;
      j->err = "total edge weight must be below 2^31";
      j->done = true;
      continue;
    }
    const mgcd_csr &c = j->g;
    j->W = W[q];
    j->cur = Graph{c.n, c.nnz, c.offsets, c.indices, c.weights};
    j->kcur = 0;
    j->next_slot = 0;
    j->pass = 0;
    j->tol = p_.tolerance;
    j->stats.passes += 1;  // level 0
    j->it = 0;
    const bool lpa = algo_ == MGCD_ALGO_LPA;
    sd.push_back(StartDesc{j->C, lpa ? nullptr : j->top, lpa ? nullptr : j->Sig, j->K[0], (int64_t)c.n});
    nmax = std::max<int64_t>(nmax, c.n);
  }
  if (sd.empty()) return;
  const StartDesc *sdd = upload(a, sd, st);
  per_graph(sdd, (int32_t)sd.size(), nmax, st,
            [&](dim3 grid, int32_t y0) { k_admit_start<<<grid, BLOCK, 0, st>>>(sdd, y0); });
  MGCD_HIP(hipStreamSynchronize(st));  // the table's host copy and the blocks are ready
}

// A level starts: labels (every vertex alone, or Leiden's carried-over start) and their
// community totals.
void StepEngine::enter_level(StepJob *j, bool reset, const Lane &l) {
  const int32_t nl = j->cur.n;
  j->stats.passes += 1;
  j->it = 0;
  if (reset) launch_iota(j->C, nl, l.st);
  if (algo_ != MGCD_ALGO_LPA) launch_community_totals(j->C, j->K[j->kcur], j->Sig, nl, l.st);
}

void StepEngine::finish(StepJob *j, const int32_t *labels, const Lane &l) {
  Arena a = l.arena();
  j->stats.communities = canonical(labels, j->g.n, j->out, a, l.st);
  j->stats.ms_total = (float)((host_seconds() - j->t_admit) * 1e3);
  j->done = true;
}

// The phase transition after a level's sweeps, as a call makes it: LPA ends; Louvain
// renumbers, stops or aggregates (Section 3.3); Leiden first refines within the moving
// communities (Section 4.2) and aggregates by the refined ones, each super-vertex
// starting in its moving community.  Sets done when the job finished.
void StepEngine::end_level(StepJob *j, const Lane &l) {
  if (algo_ == MGCD_ALGO_LPA) {
    finish(j, j->C, l);
    return;
  }
  const bool leiden = algo_ == MGCD_ALGO_LEIDEN;
  const int32_t n = j->g.n;
  const int32_t nl = j->cur.n;
  uint32_t *K = j->K[j->kcur];
  hipStream_t st = l.st;
  Arena a = l.arena();
  int32_t m;
  if (leiden) {
    size_t mk = a.mark();
    Schedule sch;
    build_schedule(j->cur, sched_params(&p_), sch, a, st);
    int32_t *prop = a.take<int32_t>(nl), *nprop = a.take<int32_t>(nl), *from = a.take<int32_t>(nl);
    unsigned long long *ctr = a.take<unsigned long long>(4);
    SweepArgs r{j->cur, nullptr, j->C, K, K, j->W, 0, prop, nullptr, ctr};
    launch_iota(prop, nl, st);  // a row without entries proposes itself
    launch_zero_u64(ctr, 4, st);
    launch_sweep(r, sch, ALGO_REFINE, p_.mode, p_.k, p_.chunk_len, st);
    launch_refine_accept(prop, nprop, from, j->R, nl, st);
    a.release(mk);
    m = renumber(j->R, nl, j->D, a, st);
    const bool last = j->pass == p_.max_passes - 1 || (double)m > p_.aggregation_tolerance * (double)nl;
    if (last) {
      launch_compose(j->top, j->C, j->top, n, st);
      finish(j, j->top, l);
      return;
    }
    renumber(j->C, nl, j->Dc, a, st);
    launch_compose(j->top, j->D, j->top, n, st);
  } else {
    m = renumber(j->C, nl, j->D, a, st);
    launch_compose(j->top, j->D, j->top, n, st);
    const bool last = j->pass == p_.max_passes - 1 || (double)m > p_.aggregation_tolerance * (double)nl;
    if (last) {
      finish(j, j->top, l);
      return;
    }
  }
  const int q = j->next_slot;
  const int64_t nnz2 = aggregate(j->cur, j->D, m, agg_mode(&p_), p_.k_aggregate, p_.chunk_len, leiden ? 1 : 0,
                                 j->soff[q], j->sidx[q], j->sw[q], a, st);
  launch_group_sums(j->D, K, j->K[1 - j->kcur], nl, m, st);
  if (leiden) launch_scatter_labels(j->D, j->Dc, j->C, nl, st);  // super-vertex starts in its community
  j->cur = Graph{m, nnz2, j->soff[q], j->sidx[q], j->sw[q]};
  j->next_slot = 1 - q;
  j->kcur = 1 - j->kcur;
  j->tol /= p_.tolerance_drop;
  j->pass += 1;
  enter_level(j, !leiden, l);
}

void StepEngine::dissolve() {
  Union &u = *u_;
  if (!u.live) return;
  if (u.g.n > 0) {
    k_step_unpack<<<grid_of(u.g.n), BLOCK, 0, st_>>>(u.desc, u.gid, u.C[0], u.Sig, u.g.n);
    MGCD_LAUNCHED();
  }
  u.live = false;
}

void StepEngine::repack() {
  Union &u = *u_;
  const double t0 = host_seconds();
  ctr_.packs += 1;
  const int32_t count = (int32_t)jobs_.size();
  std::vector<PackDesc> hd(count);
  int64_t N = 0, E = 0, maxi = 1;
  for (int32_t g = 0; g < count; ++g) {
    StepJob *j = jobs_[g];
    hd[g] = PackDesc{j->cur.off, j->cur.idx, j->cur.w, j->C, j->Sig, j->K[j->kcur], j->cur.n, j->cur.nnz, N, E};
    N += j->cur.n;
    E += j->cur.nnz;
    maxi = std::max<int64_t>(maxi, std::max<int64_t>(j->cur.n, j->cur.nnz));
  }
  if (N >= (1ll << 31)) throw Error(MGCD_E_WORKSPACE, "resident vertices must stay below 2^31");
  u.a = Arena{};
  u.a.base = shared_;
  u.a.cap = shared_bytes_;
  Arena &a = u.a;
  const bool lpa = algo_ == MGCD_ALGO_LPA;
  u.count = count;
  int64_t *off = a.take<int64_t>(N + 1);
  int32_t *idx = a.take<int32_t>(E);
  uint32_t *w = a.take<uint32_t>(E);
  u.g = Graph{(int32_t)N, E, off, idx, w};
  u.gid = a.take<int32_t>(N);
  u.C[0] = a.take<int32_t>(N);
  u.C[1] = a.take<int32_t>(N);
  u.K = a.take<uint32_t>(N);
  u.Sig = lpa ? nullptr : a.take<uint32_t>(N);
  // per-graph table
  const TableLayout tl(count);
  u.table = a.take<char>((int64_t)tl.total);
  std::vector<char> ht(tl.total, 0);
  std::memcpy(ht.data() + tl.desc, hd.data(), hd.size() * sizeof(PackDesc));
  for (int32_t g = 0; g < count; ++g) {
    StepJob *j = jobs_[g];
    const uint32_t w32 = (uint32_t)j->W;
    const unsigned long long w64 = j->W;
    const int64_t nv = j->cur.n;
    const int32_t it = j->it;
    const int8_t dir = it % 2 == 0 ? (int8_t)-1 : (int8_t)1;
    std::memcpy(ht.data() + tl.Wg + 4 * g, &w32, 4);
    std::memcpy(ht.data() + tl.Wg64 + 8 * g, &w64, 8);
    ht[tl.active + g] = 1;
    std::memcpy(ht.data() + tl.nvert + 8 * g, &nv, 8);
    std::memcpy(ht.data() + tl.gtol + 8 * g, &j->tol, 8);
    std::memcpy(ht.data() + tl.git + 4 * g, &it, 4);
    std::memcpy(ht.data() + tl.gdir + g, &dir, 1);
  }
  u.desc = (PackDesc *)(u.table + tl.desc);
  u.Wg = (uint32_t *)(u.table + tl.Wg);
  u.Wg64 = (unsigned long long *)(u.table + tl.Wg64);
  u.active = (uint8_t *)(u.table + tl.active);
  u.nvert = (int64_t *)(u.table + tl.nvert);
  u.gtol = (double *)(u.table + tl.gtol);
  u.git = (int32_t *)(u.table + tl.git);
  u.gdir = (int8_t *)(u.table + tl.gdir);
  u.gctr = a.take<unsigned long long>(3 * (int64_t)count);
  u.ctr = a.take<unsigned long long>(4);
  u.res = a.take<StepResult>(count);
  u.lv = a.take<uint32_t>(2);
  MGCD_HIP(hipMemcpyAsync(u.table, ht.data(), tl.total, hipMemcpyHostToDevice, st_));
  launch_zero_u64(u.gctr, 3 * (int64_t)count, st_);
  launch_zero_u64(u.ctr, 4, st_);
  for (int32_t y0 = 0; y0 < count; y0 += 65535) {
    const int32_t ny = std::min<int32_t>(65535, count - y0);
    dim3 grid((unsigned)std::min<int64_t>(ceil_div(maxi, BLOCK), 4096), (unsigned)ny);
    k_step_pack<<<grid, BLOCK, 0, st_>>>(u.desc, y0, off, idx, w, u.gid, u.C[0], u.C[1], u.K, u.Sig);
    MGCD_LAUNCHED();
  }
  k_step_last_offset<<<1, 1, 0, st_>>>(off, N, E);
  MGCD_LAUNCHED();
  MGCD_HIP(hipStreamSynchronize(st_));  // the host table may go
  u.hd = hd;
  u.sch = Schedule{};
  u.mark_sched = a.mark();
  build_schedule(u.g, sched_params(&p_), u.sch, a, st_);
  u.hres.resize(count);
  u.live = true;
  MGCD_HIP(hipStreamSynchronize(st_));
  ctr_.s_pack += host_seconds() - t0;
}

void StepEngine::step(std::vector<StepJob *> &finished) {
  if (jobs_.empty()) return;
  Union &u = *u_;
  if (!u.live) repack();
  const double t0 = host_seconds();
  ctr_.steps += 1;
  ctr_.sweeps += sweeps_;
  const bool lpa = algo_ == MGCD_ALGO_LPA;
  k_step_begin<<<1, BLOCK, 0, st_>>>(u.lv, u.count, u.res);
  MGCD_LAUNCHED();
  // up to sweeps_ sweeps; once no graph moves, the remaining kernels return at once
  int32_t *C[2] = {u.C[0], u.C[1]};
  for (int s = 0; s < sweeps_; ++s) {
    SweepArgs args{u.g, C[0], nullptr, u.K, u.Sig, 0, 0, C[1], nullptr, u.ctr};
    args.gid = u.gid;
    args.Wg = u.Wg;
    args.active = u.active;
    args.gctr = u.gctr;
    args.live = u.lv;
    args.gdir = lpa ? nullptr : u.gdir;
    args.one_scan = lpa ? p_.one_scan : 0;
    launch_sweep(args, u.sch, lpa ? ALGO_LPA : ALGO_MOVE, p_.mode, p_.k, p_.chunk_len, st_);
    if (!lpa) {
      LevelRule r;
      r.live = u.lv;
      launch_apply_moves(C[0], C[1], u.K, u.Sig, u.g.n, st_, &r);
    }
    if (lpa)
      k_step_converge<ALGO_LPA><<<1, BLOCK, 0, st_>>>(u.gctr, u.Wg64, u.nvert, u.gtol, u.git, nullptr, u.active,
                                                      p_.max_iterations, u.count, u.res, u.lv);
    else
      k_step_converge<ALGO_MOVE><<<1, BLOCK, 0, st_>>>(u.gctr, u.Wg64, u.nvert, u.gtol, u.git, u.gdir, u.active,
                                                       p_.max_iterations, u.count, u.res, u.lv);
    MGCD_LAUNCHED();
    std::swap(C[0], C[1]);
  }
  uint32_t lv[2] = {0, 0};
  MGCD_HIP(hipMemcpyAsync(u.hres.data(), u.res, (size_t)u.count * sizeof(StepResult), hipMemcpyDeviceToHost, st_));
  MGCD_HIP(hipMemcpyAsync(lv, u.lv, sizeof(lv), hipMemcpyDeviceToHost, st_));
  MGCD_HIP(hipStreamSynchronize(st_));
  // the labels are in the buffer the last sweep in which some graph moved wrote
  if (lv[1] % 2 == 1) std::swap(u.C[0], u.C[1]);
  ctr_.sweeps_moving += lv[1];
  ctr_.rows_swept += (int64_t)lv[1] * u.g.n;
  ctr_.s_sweep += host_seconds() - t0;
  const double t1 = host_seconds();
  std::vector<StepJob *> ended;
  for (int32_t g = 0; g < u.count; ++g) {
    StepJob *j = jobs_[g];
    const StepResult &r = u.hres[g];
    ctr_.rows_moving += (int64_t)r.sweeps * j->cur.n;
    if (r.sweeps == 0) continue;
    j->it += (int)r.sweeps;
    j->stats.iterations += (int32_t)r.sweeps;
    j->stats.edges_scanned += (int64_t)r.sweeps * j->cur.nnz;
    j->stats.moved_last = (int64_t)r.moved;
    if (r.ended) ended.push_back(j);
  }
  if (!ended.empty()) {
    ctr_.transitions += (int64_t)ended.size();
    if (algo_ == MGCD_ALGO_LEIDEN) {  // refinement first, graph by graph
      dissolve();
      in_lanes(ended, [&](StepJob *j, const Lane &l) { end_level(j, l); });
    } else {
      std::vector<int32_t> eg;
      for (int32_t g = 0; g < u.count; ++g)
        if (u.hres[(size_t)g].ended) eg.push_back(g);
      batched_end(eg);
    }
    for (StepJob *j : ended)
      if (j->done) {
        jobs_.erase(std::find(jobs_.begin(), jobs_.end(), j));
        finished.push_back(j);
      }
  }
  ctr_.s_phase += host_seconds() - t1;
}

// The phase transitions of the LPA / Louvain graphs eg (places in the union) whose
// level ended in the last step, made together while the union's memory is still
// intact, as run_batched makes them for a batch: every graph's labels and totals go
// back to its block; Louvain renumbers the ended graphs together, composes their level
// maps and decides which stop (Section 3.3); the graphs that stop get their canonical
// labels together; the others are aggregated together, each taking its rows of the
// aggregated union as its next level.  Each graph's result is that of its own call:
// renumbering keeps every graph's ids in order, and a community's stream holds only
// its own graph's rows.
void StepEngine::batched_end(const std::vector<int32_t> &eg) {
  Union &u = *u_;
  const int32_t N = u.g.n;
  hipStream_t st = st_;
  if (N > 0) {
    k_step_unpack<<<grid_of(N), BLOCK, 0, st>>>(u.desc, u.gid, u.C[0], u.Sig, N);
    MGCD_LAUNCHED();
  }
  u.live = false;
  Arena &a = u.a;  // after the union's arrays (the schedule's memory is reused)
  a.release(u.mark_sched);
  const bool lpa = algo_ == MGCD_ALGO_LPA;
  const int32_t q = (int32_t)eg.size();
  std::vector<StepJob *> J((size_t)q);
  for (int32_t i = 0; i < q; ++i) J[(size_t)i] = jobs_[(size_t)eg[(size_t)i]];
  std::vector<uint8_t> last((size_t)q, 1);
  std::vector<int64_t> m((size_t)q, 0);
  if (!lpa) {
    // renumber the ended graphs together; graph g's communities are db[g] .. db[g] + m[g] - 1
    std::vector<uint8_t> keep((size_t)u.count, 0);
    for (int32_t g : eg) keep[(size_t)g] = 1;
    const uint8_t *keep_d = upload(a, keep, st);
    int32_t *D1 = a.take<int32_t>(N);
    int64_t *dense1 = a.take<int64_t>((int64_t)N + 1);
    renumber(u.C[0], N, D1, a, st, u.gid, keep_d, dense1);
    std::vector<int64_t> pos(2 * (size_t)q);
    for (int32_t i = 0; i < q; ++i) {
      const PackDesc &h = u.hd[(size_t)eg[(size_t)i]];
      pos[2 * (size_t)i] = h.vbase;
      pos[2 * (size_t)i + 1] = h.vbase + h.n;
    }
    const std::vector<int64_t> db = gather(a, dense1, pos, st);
    std::vector<ComposeDesc> cd((size_t)q);
    int64_t n0max = 0;
    for (int32_t i = 0; i < q; ++i) {
      StepJob *j = J[(size_t)i];
      m[(size_t)i] = db[2 * (size_t)i + 1] - db[2 * (size_t)i];
      last[(size_t)i] = j->pass == p_.max_passes - 1 ||
                        (double)m[(size_t)i] > p_.aggregation_tolerance * (double)j->cur.n;
      cd[(size_t)i] = ComposeDesc{j->top, j->g.n, u.hd[(size_t)eg[(size_t)i]].vbase, db[2 * (size_t)i]};
      n0max = std::max<int64_t>(n0max, j->g.n);
    }
    const ComposeDesc *cdd = upload(a, cd, st);
    per_graph(cdd, q, n0max, st, [&](dim3 grid, int32_t y0) { k_step_compose<<<grid, BLOCK, 0, st>>>(cdd, y0, D1); });
  }
  // graphs that stop: canonical labels, all together
  {
    std::vector<CanonDesc> fd;
    std::vector<int32_t> fi;
    int64_t X = 0, nmax = 0;
    for (int32_t i = 0; i < q; ++i) {
      if (!last[(size_t)i]) continue;
      StepJob *j = J[(size_t)i];
      fd.push_back(CanonDesc{lpa ? j->C : j->top, j->out, j->g.n, X});
      fi.push_back(i);
      X += j->g.n;
      nmax = std::max<int64_t>(nmax, j->g.n);
    }
    if (!fd.empty()) {
      const size_t mk = a.mark();
      const int32_t nf = (int32_t)fd.size();
      const CanonDesc *fdd = upload(a, fd, st);
      int32_t *minv = a.take<int32_t>(X);
      uint32_t *first = a.take<uint32_t>(X);
      int64_t *rank = a.take<int64_t>(X + 1);
      launch_fill_i32(minv, 0x7FFFFFFF, X, st);
      per_graph(fdd, nf, nmax, st, [&](dim3 grid, int32_t y0) { k_canon_min<<<grid, BLOCK, 0, st>>>(fdd, y0, minv); });
      per_graph(fdd, nf, nmax, st,
                [&](dim3 grid, int32_t y0) { k_canon_first<<<grid, BLOCK, 0, st>>>(fdd, y0, minv, first); });
      scan_u32_i64(first, rank, X, rank + X, a, st);
      per_graph(fdd, nf, nmax, st,
                [&](dim3 grid, int32_t y0) { k_canon_write<<<grid, BLOCK, 0, st>>>(fdd, y0, minv, rank); });
      std::vector<int64_t> pos((size_t)nf + 1);
      for (int32_t f = 0; f < nf; ++f) pos[(size_t)f] = fd[(size_t)f].off;
      pos[(size_t)nf] = X;
      const std::vector<int64_t> rk = gather(a, rank, pos, st);
      const double now = host_seconds();
      for (int32_t f = 0; f < nf; ++f) {
        StepJob *j = J[(size_t)fi[(size_t)f]];
        j->stats.communities = (int32_t)(rk[(size_t)f + 1] - rk[(size_t)f]);
        j->stats.ms_total = (float)((now - j->t_admit) * 1e3);
        j->done = true;
      }
      a.release(mk);
    }
  }
  if (lpa) return;
  // the others: aggregated together, each graph's rows of the result its next level
  std::vector<int32_t> ci;
  for (int32_t i = 0; i < q; ++i)
    if (!last[(size_t)i]) ci.push_back(i);
  if (ci.empty()) return;
  std::vector<uint8_t> keep2((size_t)u.count, 0);
  for (int32_t i : ci) keep2[(size_t)eg[(size_t)i]] = 1;
  const uint8_t *keep2_d = upload(a, keep2, st);
  int32_t *D2 = a.take<int32_t>(N);
  int64_t *dense2 = a.take<int64_t>((int64_t)N + 1);
  const int32_t m2 = renumber(u.C[0], N, D2, a, st, u.gid, keep2_d, dense2);
  std::vector<int64_t> pos(ci.size());
  for (size_t c = 0; c < ci.size(); ++c) pos[c] = u.hd[(size_t)eg[(size_t)ci[c]]].vbase;
  const std::vector<int64_t> db2 = gather(a, dense2, pos, st);
  int64_t *off2 = a.take<int64_t>((int64_t)m2 + 1);
  int32_t *idx2 = a.take<int32_t>(u.g.nnz);
  uint32_t *w2 = a.take<uint32_t>(u.g.nnz);
  aggregate(u.g, D2, m2, agg_mode(&p_), p_.k_aggregate, p_.chunk_len, 0, off2, idx2, w2, a, st);
  uint32_t *Kn = a.take<uint32_t>(m2);
  launch_group_sums(D2, u.K, Kn, N, m2, st);
  std::vector<int64_t> epos(2 * ci.size());
  for (size_t c = 0; c < ci.size(); ++c) {
    epos[2 * c] = db2[c];
    epos[2 * c + 1] = db2[c] + m[(size_t)ci[c]];
  }
  const std::vector<int64_t> eb = gather(a, off2, epos, st);
  std::vector<OutDesc> od(ci.size());
  int64_t len = 1;
  for (size_t c = 0; c < ci.size(); ++c) {
    StepJob *j = J[(size_t)ci[c]];
    const int qs = j->next_slot;
    const int64_t mc = m[(size_t)ci[c]];
    od[c] = OutDesc{j->soff[qs], j->sidx[qs], j->sw[qs], j->K[1 - j->kcur], j->Sig, j->C, db2[c], mc,
                    eb[2 * c], eb[2 * c + 1]};
    len = std::max<int64_t>(len, std::max<int64_t>(mc + 1, eb[2 * c + 1] - eb[2 * c]));
  }
  const OutDesc *odd = upload(a, od, st);
  per_graph(odd, (int32_t)od.size(), len, st, [&](dim3 grid, int32_t y0) {
    k_step_copy_out<<<grid, BLOCK, 0, st>>>(odd, y0, off2, idx2, w2, Kn);
  });
  MGCD_HIP(hipStreamSynchronize(st));
  for (size_t c = 0; c < ci.size(); ++c) {
    StepJob *j = J[(size_t)ci[c]];
    const int qs = j->next_slot;
    j->cur = Graph{(int32_t)m[(size_t)ci[c]], eb[2 * c + 1] - eb[2 * c], j->soff[qs], j->sidx[qs], j->sw[qs]};
    j->next_slot = 1 - qs;
    j->kcur = 1 - j->kcur;
    j->tol /= p_.tolerance_drop;
    j->pass += 1;
    j->stats.passes += 1;  // the next level (its labels and totals are set: C = iota, Sigma = K)
    j->it = 0;
  }
}

void StepEngine::fail_all(int code, const std::string &msg, std::vector<StepJob *> &finished) {
  for (StepJob *j : jobs_) {
    j->rc = code;
    j->err = msg;
    j->done = true;
    finished.push_back(j);
  }
  jobs_.clear();
  u_->live = false;
}

}  // namespace mgcd
