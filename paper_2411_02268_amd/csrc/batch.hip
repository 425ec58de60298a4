// Batched runs: many graphs processed together as one disjoint union.
//
// The graphs are packed into one CSR (vertex ids shifted by each graph's vertex
// base); every sweep is one launch over all of them.  Everything that decides a
// graph's course is kept per graph: its total weight W (Eq. 2), its moved /
// proposal / gain counters, its convergence, its last pass.  A graph that has
// converged stays frozen while the others continue, and a graph that finishes is
// written out and dropped from later levels.  Because communities never cross
// graphs and the union preserves every graph's id order (ties, stream order,
// member order), each graph's labels equal those of its own single run.
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/mgcd.h"
#include "aggregate.hpp"
#include "batch.hpp"
#include "move.hpp"
#include "primitives.hpp"

namespace mgcd {

static unsigned grid_for(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, BLOCK); }

struct DevDesc {
  const int64_t *off;
  const int32_t *idx;
  const uint32_t *w;
  int32_t *out;
  int64_t n, nnz, vbase, ebase;
};

// graph y0 + blockIdx.y; x covers that graph's vertices and entries.
__global__ void k_pack(const DevDesc *d, int32_t y0, int64_t *off, int32_t *idx, uint32_t *w,
                       int32_t *gid) {
  const DevDesc g = d[y0 + blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < g.n; v += stride) {
    off[g.vbase + v] = g.ebase + g.off[v];
    gid[g.vbase + v] = y0 + (int32_t)blockIdx.y;
  }
  for (int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x; e < g.nnz; e += stride) {
    idx[g.ebase + e] = (int32_t)(g.vbase + g.idx[e]);
    w[g.ebase + e] = g.w[e];
  }
}

__global__ void k_set_last_offset(int64_t *off, int64_t n, int64_t E) { off[n] = E; }

// Validation of every graph against its own sizes (validate = 1), before packing:
// offsets[0] = 0, offsets[n_g] = nnz_g, offsets non-decreasing, every index in
// [0, n_g) and every weight >= 1.  *bad receives the smallest failing graph index.
__global__ void k_validate_each(const DevDesc *d, int32_t y0, int32_t *bad) {
  const int32_t gi = y0 + (int32_t)blockIdx.y;
  const DevDesc g = d[gi];
  const int64_t stride = (int64_t)gridDim.x * BLOCK;
  bool ok = true;
  const int64_t t0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (t0 == 0) ok &= g.off[0] == 0 && g.off[g.n] == g.nnz;
  for (int64_t v = t0; v < g.n; v += stride) ok &= g.off[v + 1] >= g.off[v];
  for (int64_t e = t0; e < g.nnz; e += stride) {
    const int32_t j = g.idx[e];
    ok &= j >= 0 && (int64_t)j < g.n && g.w[e] >= 1u;
  }
  if (!ok) atomicMin(bad, gi);
}

// Per-graph sums of K (vertices of one graph are contiguous: a wave whose lanes all
// belong to one graph adds once).
__global__ void k_graph_weights(const uint32_t *K, const int32_t *gid, int64_t n, unsigned long long *Wg) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool in = i < n;
  const int32_t g = in ? gid[i] : -1;
  const unsigned long long k = in ? K[i] : 0;
  const int32_t g0 = __shfl(g, 0);
  if (__ballot(in && g != g0) == 0) {
    unsigned long long s = wave_sum(k);
    if (lane_id() == 0 && g0 >= 0 && s) atomicAdd(&Wg[g0], s);
  } else if (in && k) {
    atomicAdd(&Wg[g], k);
  }
}

__global__ void k_u64_to_u32(const unsigned long long *a, uint32_t *b, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) b[i] = (uint32_t)a[i];
}

// top[v] = D[top[v]] for input vertices whose graph is selected (sel[gid0[v]]).
__global__ void k_compose_sel(int32_t *top, const int32_t *D, const int32_t *gid0, const uint8_t *sel,
                              int64_t n) {
  int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n && sel[gid0[v]]) top[v] = D[top[v]];
}

// Canonical labels of the selected graphs, written to each graph's own output:
// communities numbered in order of their smallest vertex (within the graph).
__global__ void k_min_sel(const int32_t *lab, const int32_t *gid0, const uint8_t *sel, int64_t n,
                          int32_t *minv) {
  int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n && sel[gid0[v]]) atomicMin(&minv[lab[v]], (int32_t)v);
}
__global__ void k_first_sel(const int32_t *lab, const int32_t *gid0, const uint8_t *sel,
                            const int32_t *minv, int64_t n, uint32_t *first) {
  int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) first[v] = (sel[gid0[v]] && minv[lab[v]] == (int32_t)v) ? 1u : 0u;
}
__global__ void k_write_sel(const int32_t *lab, const int32_t *gid0, const uint8_t *sel,
                            const int32_t *minv, const int64_t *rank, const DevDesc *d, int64_t n) {
  int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v >= n) return;
  const int32_t g = gid0[v];
  if (!sel[g]) return;
  const DevDesc dg = d[g];
  dg.out[v - dg.vbase] = (int32_t)(rank[minv[lab[v]]] - rank[dg.vbase]);
}
__global__ void k_fill_i32v(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_gather_i64(const int64_t *src, const int64_t *pos, int64_t *dst, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) dst[i] = src[pos[i]];
}
// graph id of every vertex of the next level: graph g owns [base[g], base[g] + cnt[g]).
__global__ void k_gid_ranges(const int64_t *base, const int64_t *cnt, int32_t y0, int32_t count,
                             int32_t *gid) {
  const int32_t g = y0 + (int32_t)blockIdx.y;
  if (g >= count) return;
  for (int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x; v < cnt[g]; v += (int64_t)gridDim.x * BLOCK)
    gid[base[g] + v] = g;
}

struct Batch {
  int32_t count;
  int64_t N, E;
  std::vector<int64_t> vb, eb, n, nnz;  // host: input bases and sizes
  DevDesc *ddesc;
  int32_t *gid0;
  uint8_t *sel_d;
};

static unsigned long long read_u64(const unsigned long long *p, hipStream_t st) {
  unsigned long long h = 0;
  MGCD_HIP(hipMemcpyAsync(&h, p, sizeof(h), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  return h;
}

static void copy_h2d(void *dst, const void *src, size_t bytes, hipStream_t st) {
  MGCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  MGCD_HIP(hipStreamSynchronize(st));  // the host buffer may go away
}

static void set_sel(Batch &b, const std::vector<uint8_t> &sel, hipStream_t st) {
  copy_h2d(b.sel_d, sel.data(), sel.size(), st);
}

// Write canonical labels for the graphs marked in `sel` from lab (level ids of the
// input vertices).  Returns per-graph community counts through `comms`.
static void write_selected(Batch &b, const int32_t *lab, const std::vector<uint8_t> &sel,
                           std::vector<int64_t> &comms, Arena &a, hipStream_t st) {
  size_t mk = a.mark();
  const int64_t N = b.N;
  int32_t *minv = a.take<int32_t>(N);
  uint32_t *first = a.take<uint32_t>(N);
  int64_t *rank = a.take<int64_t>(N + 1);
  set_sel(b, sel, st);
  k_fill_i32v<<<grid_for(N), BLOCK, 0, st>>>(minv, 0x7FFFFFFF, N);
  MGCD_LAUNCHED();
  k_min_sel<<<grid_for(N), BLOCK, 0, st>>>(lab, b.gid0, b.sel_d, N, minv);
  MGCD_LAUNCHED();
  k_first_sel<<<grid_for(N), BLOCK, 0, st>>>(lab, b.gid0, b.sel_d, minv, N, first);
  MGCD_LAUNCHED();
  scan_u32_i64(first, rank, N, rank + N, a, st);
  k_write_sel<<<grid_for(N), BLOCK, 0, st>>>(lab, b.gid0, b.sel_d, minv, rank, b.ddesc, N);
  MGCD_LAUNCHED();
  // community count of graph g = rank[vb[g+1]] - rank[vb[g]]
  std::vector<int64_t> pos(b.count + 1);
  for (int32_t g = 0; g <= b.count; ++g) pos[g] = b.vb[g];
  int64_t *pos_d = a.take<int64_t>(b.count + 1);
  int64_t *val_d = a.take<int64_t>(b.count + 1);
  copy_h2d(pos_d, pos.data(), pos.size() * sizeof(int64_t), st);
  k_gather_i64<<<grid_for(b.count + 1), BLOCK, 0, st>>>(rank, pos_d, val_d, b.count + 1);
  MGCD_LAUNCHED();
  std::vector<int64_t> val(b.count + 1);
  MGCD_HIP(hipMemcpyAsync(val.data(), val_d, val.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  for (int32_t g = 0; g < b.count; ++g)
    if (sel[g]) comms[g] = val[g + 1] - val[g];
  a.release(mk);
}

// After a sweep, per graph on the device (one workgroup, graphs strided over its
// threads): a graph still moving counts the sweep (stat = {sweeps, entries streamed,
// movers of its last sweep}) and stops when its rule says so -- LPA: movers <=
// tol * n_g; Louvain: no positive move, or 2 * (summed gain) <= tol * W_g^2 -- and
// its counters are cleared for the next sweep (the same double-precision tests the
// single-graph driver makes on the host).  Then lv[0] = graphs still moving (0: every
// later sweep of the level does nothing), lv[1] counts the sweeps in which some graph
// moved, and the persistent sweep kernel's work counter is cleared.
template <int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_batch_converge(unsigned long long *gctr, uint8_t *active, long long *stat, const int64_t *nent,
                     const int64_t *nvert, const unsigned long long *Wg64, double tol, int32_t count,
                     uint32_t *lv, unsigned long long *queue) {
  __shared__ uint32_t red[BLOCK / WAVE];
  const uint32_t was = lv[0];
  uint32_t still = 0;
  for (int64_t g = threadIdx.x; g < count; g += BLOCK) {
    unsigned long long *c = gctr + 3 * g;
    const unsigned long long moved = atomicExch(&c[0], 0ull), prop = atomicExch(&c[1], 0ull),
                             sumG = atomicExch(&c[2], 0ull);
    if (!active[g]) continue;
    stat[3 * g] += 1;
    stat[3 * g + 1] += nent[g];
    stat[3 * g + 2] = (long long)moved;
    bool stop;
    if (ALGO == ALGO_LPA) {
      stop = (double)moved <= tol * (double)nvert[g];
    } else {
      const double WW = (double)Wg64[g] * (double)Wg64[g];
      stop = prop == 0 || 2.0 * (double)sumG <= tol * WW;
    }
    if (stop)
      active[g] = 0;
    else
      still += 1;
  }
  still = block_sum(still, red);
  if (threadIdx.x == 0) {
    lv[0] = still;
    lv[1] += was > 0 ? 1u : 0u;
  }
  if (threadIdx.x < QLANES) queue[threadIdx.x * QSTRIDE] = 0;
}

// Start of a level: lv = {graphs moving, sweeps with moves so far = 0}, queue empty.
__global__ void k_level_start(uint32_t *lv, uint32_t moving, unsigned long long *queue) {
  if (threadIdx.x == 0) {
    lv[0] = moving;
    lv[1] = 0;
  }
  if (threadIdx.x < QLANES) queue[threadIdx.x * QSTRIDE] = 0;
}

// One level's local-moving sweeps for every graph of the batch, as one device-driven
// launch: all max_iterations sweeps (each followed by its Sigma update and the
// per-graph stopping rules of k_batch_converge) are captured as one HIP graph and
// launched once, or issued one by one (direct_launch), and the host waits once, at
// the end.  Within a sweep the main sweep kernel is persistent: its waves take row
// tiles of all graphs from a device work counter.  A graph that has stopped keeps its
// labels (its rows copy C to C_new) while others move; once no graph moves, every
// remaining sweep kernel returns at once, so the labels stay in the buffer the last
// real sweep wrote, found from the device's count of real sweeps.  On return the
// stream is synchronised and C[0] holds the labels.
struct LevelSweeps {
  int algo;             // ALGO_LPA or ALGO_MOVE
  Graph g;
  int32_t *C[2];
  uint32_t *K, *Sig;
  int32_t *gid;
  uint32_t *Wg;
  unsigned long long *Wg64;
  uint8_t *active;
  unsigned long long *gctr;
  long long *stat;
  const int64_t *nent, *nvert;
  int32_t count;
  double tol;
  uint32_t *lv;               // [graphs moving, sweeps with moves]
  unsigned long long *queue;  // work counter of the persistent sweep kernel
  uint32_t moving;            // graphs moving at the start of the level
};

// A stream of the library's own to record graphs on (the caller's stream may be the
// legacy default stream, which cannot be captured); destroyed with the call.
struct CaptureStream {
  hipStream_t s = nullptr;
  hipStream_t get() {
    if (!s) MGCD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
  }
  ~CaptureStream() {
    if (s) (void)hipStreamDestroy(s);
  }
};

static void level_sweeps(LevelSweeps &L, const mgcd_params *p, const Schedule &sch,
                         CaptureStream *capture, hipStream_t st) {
  const int total = p->max_iterations;
  // every sweep of the level on stream s (label buffers swapped after each)
  auto issue = [&](hipStream_t s) {
    int32_t *C[2] = {L.C[0], L.C[1]};
    for (int it = 0; it < total; ++it) {
      const int dir = L.algo == ALGO_LPA ? 0 : (it % 2 == 0 ? -1 : 1);
      SweepArgs args{L.g, C[0], nullptr, L.K, L.Sig, 0, dir, C[1], nullptr, L.gctr};
      args.gid = L.gid;
      args.Wg = L.Wg;
      args.active = L.active;
      args.gctr = L.gctr;
      args.live = L.lv;
      args.queue = L.queue;
      args.one_scan = L.algo == ALGO_LPA ? p->one_scan : 0;
      launch_sweep(args, sch, L.algo, p->mode, p->k, p->chunk_len, s);
      if (L.algo != ALGO_LPA) {
        LevelRule r;
        r.live = L.lv;
        launch_apply_moves(C[0], C[1], L.K, L.Sig, L.g.n, s, &r);
      }
      if (L.algo == ALGO_LPA)
        k_batch_converge<ALGO_LPA><<<1, BLOCK, 0, s>>>(L.gctr, L.active, L.stat, L.nent, L.nvert, L.Wg64,
                                                      L.tol, L.count, L.lv, L.queue);
      else
        k_batch_converge<ALGO_MOVE><<<1, BLOCK, 0, s>>>(L.gctr, L.active, L.stat, L.nent, L.nvert, L.Wg64,
                                                       L.tol, L.count, L.lv, L.queue);
      MGCD_LAUNCHED();
      std::swap(C[0], C[1]);
    }
  };
  k_level_start<<<1, QLANES, 0, st>>>(L.lv, L.moving, L.queue);
  MGCD_LAUNCHED();
  if (capture && total > 0) {
    hipStream_t cs = capture->get();
    hipGraph_t graph = nullptr;
    MGCD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    in_capture = true;
    try {
      issue(cs);
    } catch (...) {
      in_capture = false;
      (void)hipStreamEndCapture(cs, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    in_capture = false;
    MGCD_HIP(hipStreamEndCapture(cs, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, st);  // on the caller's stream, after its work
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    MGCD_HIP(e);
  } else {
    issue(st);
  }
  uint32_t h[2] = {0, 0};
  MGCD_HIP(hipMemcpyAsync(h, L.lv, sizeof(h), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  if (h[1] % 2 == 1) std::swap(L.C[0], L.C[1]);  // an odd count of real sweeps ends in C[1]
}

void run_batched(int algo, const mgcd_csr *graphs, int32_t count, const mgcd_params *p,
                 int32_t *const *outs, Arena &a, hipStream_t st, mgcd_graph_stats *gstats,
                 mgcd_stats *total) {
  Batch b;
  b.count = count;
  b.vb.assign(count + 1, 0);
  b.eb.assign(count + 1, 0);
  b.n.assign(count, 0);
  b.nnz.assign(count, 0);
  for (int32_t g = 0; g < count; ++g) {
    const mgcd_csr &c = graphs[g];
    if (c.n < 0 || c.nnz < 0) throw Error(MGCD_E_ARG, "negative graph size");
    if (c.n > 0 && (!c.offsets || !outs[g])) throw Error(MGCD_E_ARG, "null graph or output");
    if (c.nnz > 0 && (!c.indices || !c.weights)) throw Error(MGCD_E_ARG, "null graph arrays");
    b.n[g] = c.n;
    b.nnz[g] = c.nnz;
    b.vb[g + 1] = b.vb[g] + c.n;
    b.eb[g + 1] = b.eb[g] + c.nnz;
  }
  b.N = b.vb[count];
  b.E = b.eb[count];
  if (b.N >= (1ll << 31)) throw Error(MGCD_E_ARG, "batched vertex total must be below 2^31");
  const int32_t N = (int32_t)b.N;
  const int64_t E = b.E;
  Timer total_t(st), tm(st);
  total_t.start();

  // pack the union
  std::vector<DevDesc> hd(count);
  int64_t max_items = 1;
  for (int32_t g = 0; g < count; ++g) {
    hd[g] = DevDesc{graphs[g].offsets, graphs[g].indices, graphs[g].weights, outs[g], b.n[g], b.nnz[g],
                    b.vb[g], b.eb[g]};
    max_items = std::max<int64_t>(max_items, std::max(b.n[g], b.nnz[g]));
  }
  b.ddesc = a.take<DevDesc>(count);
  copy_h2d(b.ddesc, hd.data(), hd.size() * sizeof(DevDesc), st);
  if (p->validate) {
    int32_t *bad = a.take<int32_t>(1);
    launch_fill_i32(bad, count, 1, st);
    for (int32_t y0 = 0; y0 < count; y0 += 65535) {
      const int32_t ny = std::min<int32_t>(65535, count - y0);
      dim3 grid((unsigned)std::min<int64_t>(ceil_div(max_items + 1, BLOCK), 4096), (unsigned)ny);
      k_validate_each<<<grid, BLOCK, 0, st>>>(b.ddesc, y0, bad);
      MGCD_LAUNCHED();
    }
    int32_t hb = count;
    MGCD_HIP(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, st));
    MGCD_HIP(hipStreamSynchronize(st));
    if (hb < count) throw Error(MGCD_E_GRAPH, "graph " + std::to_string(hb) + " failed validation");
  }
  b.gid0 = a.take<int32_t>(N);
  b.sel_d = a.take<uint8_t>(count);
  uint8_t *active_d = a.take<uint8_t>(count);
  unsigned long long *gctr = a.take<unsigned long long>(3 * (int64_t)count);
  unsigned long long *Wg64 = a.take<unsigned long long>(count);
  uint32_t *Wg = a.take<uint32_t>(count);
  int64_t *uoff = a.take<int64_t>((int64_t)N + 1);
  int32_t *uidx = a.take<int32_t>(E);
  uint32_t *uw = a.take<uint32_t>(E);
  for (int32_t y0 = 0; y0 < count; y0 += 65535) {
    const int32_t ny = std::min<int32_t>(65535, count - y0);
    dim3 grid((unsigned)std::min<int64_t>(ceil_div(max_items, BLOCK), 4096), (unsigned)ny);
    k_pack<<<grid, BLOCK, 0, st>>>(b.ddesc, y0, uoff, uidx, uw, b.gid0);
    MGCD_LAUNCHED();
  }
  k_set_last_offset<<<1, 1, 0, st>>>(uoff, N, E);
  MGCD_LAUNCHED();
  Graph U{N, E, uoff, uidx, uw};
  uint32_t *Kbuf[2] = {a.take<uint32_t>(N), a.take<uint32_t>(N)};
  {
    unsigned long long *Wtot = a.take<unsigned long long>(1);
    launch_degrees(U, Kbuf[0], Wtot, a, st);
    launch_zero_u64(Wg64, count, st);
    if (N > 0) {
      k_graph_weights<<<grid_for(N), BLOCK, 0, st>>>(Kbuf[0], b.gid0, N, Wg64);
      MGCD_LAUNCHED();
    }
    std::vector<unsigned long long> hw(count);
    MGCD_HIP(hipMemcpyAsync(hw.data(), Wg64, count * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    const unsigned long long wall = read_u64(Wtot, st);
    // W_g sums the rows' K, which are 32-bit: a row of 2^32 or more would wrap and
    // drop below its true weight, so the W_g must add up to the exact (64-bit) total
    unsigned long long wsum = 0;
    for (int32_t g = 0; g < count; ++g) {
      if (hw[g] >= (1ull << 31)) throw Error(MGCD_E_OVERFLOW, "graph " + std::to_string(g) + ": total edge weight must be below 2^31");
      wsum += hw[g];
    }
    if (wsum != wall) throw Error(MGCD_E_OVERFLOW, "a graph's total edge weight must be below 2^31");
    k_u64_to_u32<<<grid_for(count), BLOCK, 0, st>>>(Wg64, Wg, count);
    MGCD_LAUNCHED();
  }
  std::vector<uint64_t> W(count);
  {
    std::vector<unsigned long long> hw(count);
    MGCD_HIP(hipMemcpyAsync(hw.data(), Wg64, count * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    MGCD_HIP(hipStreamSynchronize(st));
    for (int32_t g = 0; g < count; ++g) W[g] = hw[g];
  }

  std::vector<mgcd_graph_stats> gs(count);
  for (auto &x : gs) x = mgcd_graph_stats{};
  std::vector<int64_t> comms(count, 0);
  std::vector<uint8_t> finished(count, 0), active(count, 0), sel(count, 0);
  for (int32_t g = 0; g < count; ++g) finished[g] = b.n[g] == 0;
  int32_t *Ca = a.take<int32_t>(N), *Cb = a.take<int32_t>(N);
  mgcd_stats s{};
  float ms_lm = 0, ms_agg = 0;

  CaptureStream cstream;
  CaptureStream *capture = p->direct_launch == 0 ? &cstream : nullptr;
  long long *stat = a.take<long long>(3 * (int64_t)count);
  uint32_t *lvd = a.take<uint32_t>(2);
  unsigned long long *queue = a.take<unsigned long long>((int64_t)QLANES * QSTRIDE);
  auto moving = [&]() {
    uint32_t c = 0;
    for (uint8_t f : active) c += f ? 1u : 0u;
    return c;
  };
  int64_t *nent_d = a.take<int64_t>(count);
  int64_t *nvert_d = a.take<int64_t>(count);
  // per-level stats from the device: sweeps, entries, movers per graph
  auto collect = [&](const std::vector<uint8_t> &was_active) {
    std::vector<long long> h(3 * (size_t)count);
    MGCD_HIP(hipMemcpyAsync(h.data(), stat, h.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
    MGCD_HIP(hipStreamSynchronize(st));
    long long sweeps = 0;
    for (int32_t g = 0; g < count; ++g) {
      if (!was_active[g] || h[3 * g] == 0) continue;
      gs[g].iterations += (int32_t)h[3 * g];
      gs[g].edges_scanned += h[3 * g + 1];
      gs[g].moved_last = h[3 * g + 2];
      s.edges_scanned += h[3 * g + 1];
      sweeps = std::max(sweeps, h[3 * g]);
    }
    s.iterations += (int32_t)sweeps;
  };

  if (algo == MGCD_ALGO_LPA) {
    launch_iota(Ca, N, st);
    launch_iota(Cb, N, st);  // rows without entries are in no sweep: both buffers hold them
    Schedule sch;
    build_schedule(U, sched_params(p), sch, a, st);
    for (int32_t g = 0; g < count; ++g) active[g] = !finished[g];
    copy_h2d(active_d, active.data(), count, st);
    copy_h2d(nent_d, b.nnz.data(), count * sizeof(int64_t), st);
    copy_h2d(nvert_d, b.n.data(), count * sizeof(int64_t), st);
    launch_zero_u64((unsigned long long *)stat, 3 * count, st);
    launch_zero_u64(gctr, 3 * count, st);
    if (N > 0 && p->max_iterations > 0) {
      LevelSweeps lv{ALGO_LPA, U, {Ca, Cb}, Kbuf[0], nullptr, b.gid0, Wg, Wg64,
                     active_d, gctr, stat, nent_d, nvert_d, count, p->tolerance,
                     lvd, queue, moving()};
      tm.start();
      level_sweeps(lv, p, sch, capture, st);
      ms_lm += tm.stop();
      Ca = lv.C[0];
      Cb = lv.C[1];
      collect(active);
    }
    for (int32_t g = 0; g < count; ++g) sel[g] = !finished[g];
    write_selected(b, Ca, sel, comms, a, st);
    for (int32_t g = 0; g < count; ++g) {
      gs[g].passes = b.n[g] > 0 ? 1 : 0;
      gs[g].communities = (int32_t)comms[g];
    }
    s.passes = 1;
  } else {
    // Louvain: all unfinished graphs move through the levels together
    int32_t *top = a.take<int32_t>(N);
    int32_t *D = a.take<int32_t>(N);
    int32_t *gid_cur = a.take<int32_t>(N);
    int32_t *gid_next = a.take<int32_t>(N);
    uint32_t *Sig = a.take<uint32_t>(N);
    int64_t *dense = a.take<int64_t>((int64_t)N + 1);
    int64_t *nb_d = a.take<int64_t>(count + 1);
    int64_t *nc_d = a.take<int64_t>(count + 1);
    int64_t *tmp_d = a.take<int64_t>(count + 1);
    struct Slot {
      int64_t *off;
      int32_t *idx;
      uint32_t *w;
    } slot[2];
    for (int q = 0; q < 2; ++q) {
      slot[q].off = a.take<int64_t>((int64_t)N + 1);
      slot[q].idx = a.take<int32_t>(E);
      slot[q].w = a.take<uint32_t>(E);
    }
    launch_iota(top, N, st);
    MGCD_HIP(hipMemcpyAsync(gid_cur, b.gid0, (size_t)N * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    std::vector<int64_t> vb_cur(b.vb.begin(), b.vb.end() - 1), n_cur(b.n), nnz_cur(b.nnz);
    Graph cur = U;
    int kcur = 0, next_slot = 0;
    double tol = p->tolerance;
    for (int pass = 0; pass < p->max_passes; ++pass) {
      bool any_left = false;
      for (int32_t g = 0; g < count; ++g) any_left |= !finished[g];
      if (!any_left) break;
      const int32_t nl = cur.n;
      uint32_t *K = Kbuf[kcur];
      s.passes += 1;
      size_t mark = a.mark();
      tm.start();
      Schedule sch;
      build_schedule(cur, sched_params(p), sch, a, st);
      launch_iota(Ca, nl, st);
      launch_iota(Cb, nl, st);  // rows without entries are in no sweep
      launch_community_totals(Ca, K, Sig, nl, st);
      ms_lm += tm.stop();
      for (int32_t g = 0; g < count; ++g) {
        active[g] = !finished[g];
        if (!finished[g]) gs[g].passes += 1;
      }
      copy_h2d(active_d, active.data(), count, st);
      copy_h2d(nent_d, nnz_cur.data(), count * sizeof(int64_t), st);
      copy_h2d(nvert_d, n_cur.data(), count * sizeof(int64_t), st);
      launch_zero_u64((unsigned long long *)stat, 3 * count, st);
      launch_zero_u64(gctr, 3 * count, st);
      {
        LevelSweeps lv{ALGO_MOVE, cur, {Ca, Cb}, K, Sig, gid_cur, Wg, Wg64,
                       active_d, gctr, stat, nent_d, nvert_d, count, tol,
                       lvd, queue, moving()};
        tm.start();
        level_sweeps(lv, p, sch, capture, st);
        ms_lm += tm.stop();
        Ca = lv.C[0];
        Cb = lv.C[1];
        collect(active);
      }
      a.release(mark);
      tm.start();
      // renumber over the unfinished graphs and decide who stops here
      for (int32_t g = 0; g < count; ++g) sel[g] = !finished[g];
      set_sel(b, sel, st);
      renumber(Ca, nl, D, a, st, gid_cur, b.sel_d, dense);
      std::vector<int64_t> pos(count + 1);
      for (int32_t g = 0; g < count; ++g) pos[g] = vb_cur[g];
      pos[count] = nl;
      copy_h2d(tmp_d, pos.data(), pos.size() * sizeof(int64_t), st);
      k_gather_i64<<<grid_for(count + 1), BLOCK, 0, st>>>(dense, tmp_d, nb_d, count + 1);
      MGCD_LAUNCHED();
      std::vector<int64_t> db(count + 1);
      MGCD_HIP(hipMemcpyAsync(db.data(), nb_d, db.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
      MGCD_HIP(hipStreamSynchronize(st));
      std::vector<uint8_t> stop(count, 0);
      bool cont = false;
      for (int32_t g = 0; g < count; ++g) {
        if (finished[g]) continue;
        const int64_t m = db[g + 1] - db[g];  // graph g's communities (a contiguous id range)
        stop[g] = pass == p->max_passes - 1 || (double)m > p->aggregation_tolerance * (double)n_cur[g];
        cont |= !stop[g];
      }
      // graphs that stop: compose their labels with this renumbering and write them
      set_sel(b, stop, st);
      k_compose_sel<<<grid_for(N), BLOCK, 0, st>>>(top, D, b.gid0, b.sel_d, N);
      MGCD_LAUNCHED();
      write_selected(b, top, stop, comms, a, st);
      for (int32_t g = 0; g < count; ++g)
        if (stop[g]) {
          finished[g] = 1;
          gs[g].communities = (int32_t)comms[g];
        }
      if (!cont) {
        ms_agg += tm.stop();
        break;
      }
      // renumber again over the graphs that go on, compose, aggregate
      for (int32_t g = 0; g < count; ++g) sel[g] = !finished[g];
      set_sel(b, sel, st);
      const int32_t m = renumber(Ca, nl, D, a, st, gid_cur, b.sel_d, dense);
      k_compose_sel<<<grid_for(N), BLOCK, 0, st>>>(top, D, b.gid0, b.sel_d, N);
      MGCD_LAUNCHED();
      k_gather_i64<<<grid_for(count + 1), BLOCK, 0, st>>>(dense, tmp_d, nb_d, count + 1);
      MGCD_LAUNCHED();
      MGCD_HIP(hipMemcpyAsync(db.data(), nb_d, db.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
      MGCD_HIP(hipStreamSynchronize(st));
      auto &sl = slot[next_slot];
      const int64_t nnz2 = aggregate(cur, D, m, agg_mode(p), p->k_aggregate, p->chunk_len, 0, sl.off, sl.idx,
                                     sl.w, a, st);
      launch_group_sums(D, K, Kbuf[1 - kcur], nl, m, st);
      // next level: graph g owns [db[g], db[g+1]) (empty when finished)
      std::vector<int64_t> cnt(count + 1, 0), base(count + 1, 0);
      for (int32_t g = 0; g < count; ++g) {
        base[g] = db[g];
        cnt[g] = finished[g] ? 0 : db[g + 1] - db[g];
        vb_cur[g] = db[g];
        n_cur[g] = cnt[g];
      }
      copy_h2d(nb_d, base.data(), base.size() * sizeof(int64_t), st);
      copy_h2d(nc_d, cnt.data(), cnt.size() * sizeof(int64_t), st);
      int64_t maxc = 1;
      for (int32_t g = 0; g < count; ++g) maxc = std::max(maxc, cnt[g]);
      for (int32_t y0 = 0; y0 < count; y0 += 65535) {
        const int32_t ny = std::min<int32_t>(65535, count - y0);
        dim3 grid((unsigned)std::min<int64_t>(ceil_div(maxc, BLOCK), 4096), (unsigned)ny);
        k_gid_ranges<<<grid, BLOCK, 0, st>>>(nb_d, nc_d, y0, count, gid_next);
        MGCD_LAUNCHED();
      }
      // entries per graph at the next level
      std::vector<int64_t> pos2(count + 1);
      for (int32_t g = 0; g < count; ++g) pos2[g] = db[g];
      pos2[count] = m;
      copy_h2d(tmp_d, pos2.data(), pos2.size() * sizeof(int64_t), st);
      k_gather_i64<<<grid_for(count + 1), BLOCK, 0, st>>>(sl.off, tmp_d, nb_d, count + 1);
      MGCD_LAUNCHED();
      std::vector<int64_t> eb2(count + 1);
      MGCD_HIP(hipMemcpyAsync(eb2.data(), nb_d, eb2.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
      MGCD_HIP(hipStreamSynchronize(st));
      for (int32_t g = 0; g < count; ++g) nnz_cur[g] = finished[g] ? 0 : eb2[g + 1] - eb2[g];
      std::swap(gid_cur, gid_next);
      ms_agg += tm.stop();
      cur = Graph{m, nnz2, sl.off, sl.idx, sl.w};
      next_slot = 1 - next_slot;
      kcur = 1 - kcur;
      tol /= p->tolerance_drop;
    }
  }
  for (int32_t g = 0; g < count; ++g) {
    if (b.n[g] == 0) gs[g] = mgcd_graph_stats{};
    s.communities += gs[g].communities;
  }
  s.ms_local_move = ms_lm;
  s.ms_aggregate = ms_agg;
  s.ms_total = total_t.stop();
  if (gstats)
    for (int32_t g = 0; g < count; ++g) gstats[g] = gs[g];
  if (total) *total = s;
}

size_t batched_workspace_bytes(int32_t algo, int32_t count, int64_t N, int64_t E, const mgcd_params *p) {
  const int64_t L = p->chunk_len > 0 ? p->chunk_len : 1;
  size_t b = (size_t)count * (sizeof(DevDesc) + 64) + 64 * 1024;
  b += (size_t)(N + 1) * 8 + (size_t)E * 8;                 // union
  b += (size_t)N * 4 * 14 + (size_t)(N + 1) * 8;             // per-vertex state
  if (algo != MGCD_ALGO_LPA) b += 2 * ((size_t)(N + 1) * 8 + (size_t)E * 8);  // level slots
  size_t sched = schedule_ws_bytes((int32_t)N, E, sched_mode(p), p->k, L);
  size_t agg = algo == MGCD_ALGO_LPA ? 0 : aggregate_ws_bytes((int32_t)N, E, agg_mode(p), p->k_aggregate, L, false);
  size_t misc = (size_t)N * (4 + 4 + 8 + 8) + scan_ws_bytes(N + 1) + 64 * 1024;
  size_t phase = sched > agg ? sched : agg;
  phase = phase > degrees_ws_bytes(E) ? phase : degrees_ws_bytes(E);
  return b + phase + misc + (1u << 20);
}

}  // namespace mgcd
