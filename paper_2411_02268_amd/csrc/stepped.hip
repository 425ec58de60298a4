// Step-level serving: one local-moving sweep per step over every resident request.
//
// While the resident set and their levels stay the same, their current level graphs
// live packed as one disjoint union in the shared region (vertex and entry ids shifted
// by each graph's base), with the union's labels, community totals and schedule; a
// step is one sweep of Louvain's local moving (or LPA) over the union, the Sigma
// update, and each graph's own stopping rule (Section 3.2, its own W, sweep direction
// and tolerance), read back in one copy.  When some graph's level ends, or requests
// join, the union is dissolved: labels and community totals go back to each request's
// own block, the graphs whose level ended take their phase transition alone (Leiden
// refinement, renumbering and aggregation, Section 3.3; or their final labels), and
// the next step packs the union anew.  Because a graph's sweeps read only its own
// rows, labels and totals, and every rule is per graph, each request's labels equal
// those of its own call.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
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

// A graph's outcome of one sweep.
struct StepResult {
  unsigned long long moved;
  uint32_t stop;
  uint32_t pad;
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

// After a sweep, per graph: its counters (read and cleared), its stopping rule --
// LPA: movers <= tol * n_g; Louvain: no positive move, or 2 * (summed gain) <= tol *
// W_g^2, the tests of a call's own level -- and the direction of its next sweep
// (lower ids first, then alternating).
template <int ALGO>
__global__ void k_step_converge(unsigned long long *gctr, const unsigned long long *Wg64, const int64_t *nvert,
                                const double *gtol, int32_t *git, int8_t *gdir, int32_t count,
                                StepResult *res) {
  const int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (g >= count) return;
  unsigned long long *c = gctr + 3 * g;
  // read and clear in one atomic step (a plain load could be served by the scalar
  // cache and be overtaken by the store of 0)
  const unsigned long long moved = atomicExch(&c[0], 0ull), prop = atomicExch(&c[1], 0ull),
                           sumG = atomicExch(&c[2], 0ull);
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
  res[g] = StepResult{moved, stop ? 1u : 0u, 0u};
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
  Schedule sch;
  std::vector<StepResult> hres;
};

StepEngine::StepEngine(int algo, const mgcd_params &p, char *shared, size_t shared_bytes, hipStream_t st)
    : algo_(algo), p_(p), shared_(shared), shared_bytes_(shared_bytes), st_(st), u_(new Union) {}

StepEngine::~StepEngine() { delete u_; }

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

size_t StepEngine::shared_need(int algo, const mgcd_params &p, int64_t count, int64_t N, int64_t E,
                               int32_t max_n, int64_t max_nnz) {
  const int64_t L = p.chunk_len > 0 ? p.chunk_len : 1;
  // the union: rows, entries, per-vertex state, per-graph table, counters, schedule
  size_t un = up((size_t)(N + 1) * 8) + up((size_t)E * 4) * 2 + up((size_t)N * 4) * 5;
  un += TableLayout(count).total + up((size_t)count * 24) + up((size_t)count * sizeof(StepResult)) + 4096;
  un += schedule_ws_bytes((int32_t)std::min<int64_t>(N, INT32_MAX), E, sched_mode(&p), p.k, L);
  un += 64 * 1024;
  // the phase work of one job: admission (degrees, validation), Leiden refinement (its
  // schedule and proposal arrays), renumbering, aggregation, final labels
  size_t ph = degrees_ws_bytes(max_nnz);
  if (algo != MGCD_ALGO_LPA) {
    ph = std::max(ph, aggregate_ws_bytes(max_n, max_nnz, agg_mode(&p), p.k_aggregate, L,
                                         algo == MGCD_ALGO_LEIDEN));
    if (algo == MGCD_ALGO_LEIDEN)
      ph = std::max(ph, schedule_ws_bytes(max_n, max_nnz, sched_mode(&p), p.k, L) + (size_t)max_n * 12 + 8192);
  }
  ph += (size_t)max_n * (4 + 4 + 8 + 8) + scan_ws_bytes((int64_t)max_n + 1) + 64 * 1024;
  return std::max(un, ph) + (1u << 20);
}

Arena StepEngine::phase_arena() {
  if (u_->live) throw Error(MGCD_E_ARG, "internal: phase work while the union is packed");
  Arena a;
  a.base = shared_;
  a.cap = shared_bytes_;
  return a;
}

void StepEngine::admit(StepJob *j, std::vector<StepJob *> &finished) {
  dissolve();
  j->t_admit = host_seconds();
  j->done = false;
  j->rc = MGCD_OK;
  j->stats = mgcd_stats{};
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
      finished.push_back(j);
      return;
    }
    Arena b;
    b.base = j->block;
    b.cap = block_bytes(algo_, p_, c.n, c.nnz);
    block_layout(algo_, j, b);
    const Graph g{c.n, c.nnz, c.offsets, c.indices, c.weights};
    Arena a = phase_arena();
    unsigned long long *scr = a.take<unsigned long long>(2);
    unsigned long long h = 0;
    if (p_.validate) {  // before anything reads the rows
      launch_zero_u64(scr, 2, st_);
      launch_validate(g, scr, st_);
      MGCD_HIP(hipMemcpyAsync(&h, scr, sizeof(h), hipMemcpyDeviceToHost, st_));
      MGCD_HIP(hipStreamSynchronize(st_));
      if (h != 0) throw Error(MGCD_E_GRAPH, "CSR failed validation");
    }
    launch_degrees(g, j->K[0], scr + 1, a, st_);
    MGCD_HIP(hipMemcpyAsync(&h, scr + 1, sizeof(h), hipMemcpyDeviceToHost, st_));
    MGCD_HIP(hipStreamSynchronize(st_));
    if (h >= (1ull << 31)) throw Error(MGCD_E_OVERFLOW, "total edge weight must be below 2^31");
    j->W = h;
    j->cur = g;
    j->kcur = 0;
    j->next_slot = 0;
    j->pass = 0;
    j->tol = p_.tolerance;
    if (algo_ != MGCD_ALGO_LPA) launch_iota(j->top, c.n, st_);
  } catch (const Error &e) {
    if (e.code == MGCD_E_HIP) throw;
    j->rc = e.code;
    j->err = e.what();
    j->done = true;
    finished.push_back(j);
    return;
  }
  jobs_.push_back(j);
  enter_level(j, true, finished);
}

// A level starts: labels (every vertex alone, or Leiden's carried-over start) and their
// community totals.
void StepEngine::enter_level(StepJob *j, bool reset, std::vector<StepJob *> &) {
  const int32_t nl = j->cur.n;
  j->stats.passes += 1;
  j->it = 0;
  if (reset) launch_iota(j->C, nl, st_);
  if (algo_ != MGCD_ALGO_LPA) launch_community_totals(j->C, j->K[j->kcur], j->Sig, nl, st_);
}

void StepEngine::finish(StepJob *j, const int32_t *labels, std::vector<StepJob *> &finished) {
  Arena a = phase_arena();
  j->stats.communities = canonical(labels, j->g.n, j->out, a, st_);
  j->stats.ms_total = (float)((host_seconds() - j->t_admit) * 1e3);
  j->done = true;
  jobs_.erase(std::find(jobs_.begin(), jobs_.end(), j));
  finished.push_back(j);
}

// The phase transition after a level's sweeps, as a call makes it: LPA ends; Louvain
// renumbers, stops or aggregates (Section 3.3); Leiden first refines within the moving
// communities (Section 4.2) and aggregates by the refined ones, each super-vertex
// starting in its moving community.
void StepEngine::end_level(StepJob *j, std::vector<StepJob *> &finished) {
  if (algo_ == MGCD_ALGO_LPA) {
    finish(j, j->C, finished);
    return;
  }
  const bool leiden = algo_ == MGCD_ALGO_LEIDEN;
  const int32_t n = j->g.n;
  const int32_t nl = j->cur.n;
  uint32_t *K = j->K[j->kcur];
  Arena a = phase_arena();
  int32_t m;
  if (leiden) {
    size_t mk = a.mark();
    Schedule sch;
    build_schedule(j->cur, sched_params(&p_), sch, a, st_);
    int32_t *prop = a.take<int32_t>(nl), *nprop = a.take<int32_t>(nl), *from = a.take<int32_t>(nl);
    unsigned long long *ctr = a.take<unsigned long long>(4);
    SweepArgs r{j->cur, nullptr, j->C, K, K, j->W, 0, prop, nullptr, ctr};
    launch_iota(prop, nl, st_);  // a row without entries proposes itself
    launch_zero_u64(ctr, 4, st_);
    launch_sweep(r, sch, ALGO_REFINE, p_.mode, p_.k, p_.chunk_len, st_);
    launch_refine_accept(prop, nprop, from, j->R, nl, st_);
    a.release(mk);
    m = renumber(j->R, nl, j->D, a, st_);
    const bool last = j->pass == p_.max_passes - 1 || (double)m > p_.aggregation_tolerance * (double)nl;
    if (last) {
      launch_compose(j->top, j->C, j->top, n, st_);
      finish(j, j->top, finished);
      return;
    }
    renumber(j->C, nl, j->Dc, a, st_);
    launch_compose(j->top, j->D, j->top, n, st_);
  } else {
    m = renumber(j->C, nl, j->D, a, st_);
    launch_compose(j->top, j->D, j->top, n, st_);
    const bool last = j->pass == p_.max_passes - 1 || (double)m > p_.aggregation_tolerance * (double)nl;
    if (last) {
      finish(j, j->top, finished);
      return;
    }
  }
  const int q = j->next_slot;
  const int64_t nnz2 = aggregate(j->cur, j->D, m, agg_mode(&p_), p_.k_aggregate, p_.chunk_len, leiden ? 1 : 0,
                                 j->soff[q], j->sidx[q], j->sw[q], a, st_);
  launch_group_sums(j->D, K, j->K[1 - j->kcur], nl, m, st_);
  if (leiden) launch_scatter_labels(j->D, j->Dc, j->C, nl, st_);  // super-vertex starts in its community
  j->cur = Graph{m, nnz2, j->soff[q], j->sidx[q], j->sw[q]};
  j->next_slot = 1 - q;
  j->kcur = 1 - j->kcur;
  j->tol /= p_.tolerance_drop;
  j->pass += 1;
  enter_level(j, !leiden, finished);
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
  u.a = phase_arena();
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
  u.sch = Schedule{};
  build_schedule(u.g, sched_params(&p_), u.sch, a, st_);
  u.hres.resize(count);
  u.live = true;
}

void StepEngine::step(std::vector<StepJob *> &finished) {
  if (jobs_.empty()) return;
  Union &u = *u_;
  if (!u.live) repack();
  const bool lpa = algo_ == MGCD_ALGO_LPA;
  SweepArgs args{u.g, u.C[0], nullptr, u.K, u.Sig, 0, 0, u.C[1], nullptr, u.ctr};
  args.gid = u.gid;
  args.Wg = u.Wg;
  args.active = u.active;
  args.gctr = u.gctr;
  args.gdir = lpa ? nullptr : u.gdir;
  args.one_scan = lpa ? p_.one_scan : 0;
  launch_sweep(args, u.sch, lpa ? ALGO_LPA : ALGO_MOVE, p_.mode, p_.k, p_.chunk_len, st_);
  if (!lpa) launch_apply_moves(u.C[0], u.C[1], u.K, u.Sig, u.g.n, st_);
  if (lpa)
    k_step_converge<ALGO_LPA><<<grid_of(u.count), BLOCK, 0, st_>>>(u.gctr, u.Wg64, u.nvert, u.gtol, u.git,
                                                                   nullptr, u.count, u.res);
  else
    k_step_converge<ALGO_MOVE><<<grid_of(u.count), BLOCK, 0, st_>>>(u.gctr, u.Wg64, u.nvert, u.gtol, u.git,
                                                                    u.gdir, u.count, u.res);
  MGCD_LAUNCHED();
  MGCD_HIP(hipMemcpyAsync(u.hres.data(), u.res, (size_t)u.count * sizeof(StepResult), hipMemcpyDeviceToHost, st_));
  MGCD_HIP(hipStreamSynchronize(st_));
  std::swap(u.C[0], u.C[1]);
  std::vector<StepJob *> ended;
  for (int32_t g = 0; g < u.count; ++g) {
    StepJob *j = jobs_[g];
    j->it += 1;
    j->stats.iterations += 1;
    j->stats.edges_scanned += j->cur.nnz;
    j->stats.moved_last = (int64_t)u.hres[g].moved;
    if (u.hres[g].stop || j->it >= p_.max_iterations) ended.push_back(j);
  }
  if (ended.empty()) return;
  dissolve();
  for (StepJob *j : ended) end_level(j, finished);
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
