// Renumbering and aggregation (Section 4.1 Fig. 3, Section 4.2), modularity
// (Section 3.2 Eq. 1), canonical labels, weighted degrees and CSR validation.
//
// Aggregation streams community c's members in ascending vertex id, each row in
// CSR order with self-loops, keys D[j].  MG mode sketches that stream with the same
// chunk-then-merge schedule as local moving and keeps the positive slots, sorted by
// key, as the super-vertex row (no second pass).  Exact mode sorts all (D[i], D[j])
// pairs and sums runs.  Leiden adds the reverse of every kept pair and keeps, per
// ordered pair, the larger of the two values.
#include "aggregate.hpp"
#include "move.hpp"
#include "primitives.hpp"
#include "sketch.hpp"
#include "staging.hpp"
#include "wave_sketch.hpp"

namespace mgcd {

static unsigned grid_for(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, BLOCK); }

// ---- small per-vertex kernels ---------------------------------------------------------

__global__ void k_zero_u32(uint32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = 0;
}

static void zero_u32(uint32_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_zero_u32<<<grid_for(n), BLOCK, 0, st>>>(p, n);
  MGCD_LAUNCHED();
}

__global__ void k_flag_used(const int32_t *C, int32_t n, uint32_t *used, const int32_t *gid,
                            const uint8_t *keep) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n && (!gid || keep[gid[i]])) used[C[i]] = 1u;
}

__global__ void k_dense_map(const int32_t *C, const int64_t *dense, int32_t n, int32_t *D,
                            const int32_t *gid, const uint8_t *keep) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) D[i] = (!gid || keep[gid[i]]) ? (int32_t)dense[C[i]] : -1;
}

int32_t renumber(const int32_t *C, int32_t n, int32_t *D, Arena &a, hipStream_t st,
                 const int32_t *gid, const uint8_t *keep, int64_t *dense_out) {
  if (n == 0) return 0;
  size_t mk = a.mark();
  uint32_t *used = a.take<uint32_t>(n);
  int64_t *dense = dense_out ? dense_out : a.take<int64_t>((int64_t)n + 1);
  zero_u32(used, n, st);
  k_flag_used<<<grid_for(n), BLOCK, 0, st>>>(C, n, used, gid, keep);
  MGCD_LAUNCHED();
  scan_u32_i64(used, dense, n, dense + n, a, st);
  k_dense_map<<<grid_for(n), BLOCK, 0, st>>>(C, dense, n, D, gid, keep);
  MGCD_LAUNCHED();
  int64_t m = 0;
  MGCD_HIP(hipMemcpyAsync(&m, dense + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  a.release(mk);
  return (int32_t)m;
}

// Per-workgroup combining of (key, value) updates before the global atomics: an LDS
// open-addressing table of 2 * BLOCK slots (at most BLOCK keys, so probing ends), then
// one global atomic per distinct key of the workgroup.  Without it, a community that
// holds most vertices serialises its updates on one address.  MIN: minimum, else sum.
// Every thread of the workgroup calls it (valid: the thread has an update).
template <bool MIN>
__device__ inline void block_combine(bool valid, uint32_t key, uint32_t val, uint32_t *out) {
  constexpr uint32_t CAP = 2 * BLOCK;
  __shared__ uint32_t tk[CAP], tv[CAP];
  for (uint32_t x = threadIdx.x; x < CAP; x += BLOCK) {
    tk[x] = 0xFFFFFFFFu;
    tv[x] = MIN ? 0xFFFFFFFFu : 0u;
  }
  __syncthreads();
  if (valid) {
    uint32_t h = (key * 2654435761u) & (CAP - 1);
    while (true) {
      const uint32_t prev = atomicCAS(&tk[h], 0xFFFFFFFFu, key);
      if (prev == 0xFFFFFFFFu || prev == key) break;
      h = (h + 1) & (CAP - 1);
    }
    if (MIN)
      atomicMin(&tv[h], val);
    else
      atomicAdd(&tv[h], val);
  }
  __syncthreads();
  for (uint32_t x = threadIdx.x; x < CAP; x += BLOCK) {
    const uint32_t k = tk[x];
    if (k == 0xFFFFFFFFu) continue;
    if (MIN) {
      if (out[k] > tv[x]) atomicMin(&out[k], tv[x]);  // skip once a smaller value won
    } else if (tv[x]) {
      atomicAdd(&out[k], tv[x]);
    }
  }
}

__global__ void __launch_bounds__(BLOCK)
    k_group_sums(const int32_t *D, const uint32_t *K, uint32_t *Kout, int32_t n) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int32_t d = i < n ? D[i] : -1;
  block_combine<false>(d >= 0, d >= 0 ? (uint32_t)d : 0u, d >= 0 ? K[i] : 0u, Kout);
}

void launch_group_sums(const int32_t *D, const uint32_t *K, uint32_t *Kout, int32_t n, int32_t m,
                       hipStream_t st) {
  zero_u32(Kout, m, st);
  if (n <= 0) return;
  k_group_sums<<<grid_for(n), BLOCK, 0, st>>>(D, K, Kout, n);
  MGCD_LAUNCHED();
}

__global__ void k_compose(const int32_t *in, const int32_t *map, int32_t *out, int32_t n) {
  int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) out[v] = map[in[v]];
}

void launch_compose(const int32_t *in, const int32_t *map, int32_t *out, int32_t n, hipStream_t st) {
  if (n <= 0) return;
  k_compose<<<grid_for(n), BLOCK, 0, st>>>(in, map, out, n);
  MGCD_LAUNCHED();
}

__global__ void k_scatter_labels(const int32_t *map, const int32_t *val, int32_t *out, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n && map[i] >= 0) out[map[i]] = val[i];
}

void launch_scatter_labels(const int32_t *map, const int32_t *val, int32_t *out, int32_t n,
                           hipStream_t st) {
  if (n <= 0) return;
  k_scatter_labels<<<grid_for(n), BLOCK, 0, st>>>(map, val, out, n);
  MGCD_LAUNCHED();
}


// K_i = sum of row i's weights (Section 3), W = their total.  A workgroup takes
// DG_TILE consecutive entries: their weights are staged in LDS (coalesced loads) and
// scanned there; every row meeting the tile takes the difference of the scan at its
// bounds within the tile, stored when the row lies inside the tile and added
// atomically (to a zeroed K) when it crosses a tile boundary.  Tile totals go to
// SPREAD copies of W, folded by k_fold_total.
constexpr int DG_ITEMS = 8, DG_TILE = BLOCK * DG_ITEMS;

__device__ inline int32_t row_of_entry(const int64_t *off, int32_t lo, int32_t hi, int64_t e) {
  // the largest r in [lo, hi] with off[r] <= e (the last of equal offsets: a row
  // holding e, not an empty one before it)
  while (lo < hi) {
    const int32_t mid = (int32_t)(((int64_t)lo + hi + 1) >> 1);
    if (off[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

constexpr int SF_ITEMS = 8, SF_TILE = BLOCK * SF_ITEMS;

// The first row of every tile of SF_TILE consecutive CSR entries: first[t] = the row
// holding entry t * SF_TILE (t < ntiles) and first[ntiles] = n - 1, so that a tile's
// rows lie in first[t] .. first[t + 1] (an upper bound: rows after the tile's last
// entry are recognised by their offsets).  One thread per row marks the tile starts
// inside its row; each entry lies in exactly one row, so each slot has one writer.
// This replaces two binary searches over the offsets per workgroup, whose chains of
// dependent loads set the time of the tiled kernels.
__global__ void k_tile_first_rows(const int64_t *off, int32_t n, int64_t ntiles, int32_t *first) {
  const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (r == 0) first[ntiles] = n - 1;
  if (r >= n) return;
  const int64_t lo = off[r], hi = off[r + 1];
  for (int64_t b = (lo + SF_TILE - 1) / SF_TILE; b * SF_TILE < hi; ++b) first[b] = (int32_t)r;
}

size_t tile_table_bytes(int64_t nnz) { return (size_t)(ceil_div(nnz > 0 ? nnz : 0, SF_TILE) + 1) * 4 + 256; }

// The table of a graph with entries (taken from `a`).
static int32_t *tile_first_rows(const Graph &g, Arena &a, hipStream_t st) {
  const int64_t nt = ceil_div(g.nnz, SF_TILE);
  int32_t *first = a.take<int32_t>(nt + 1);
  k_tile_first_rows<<<(unsigned)ceil_div(g.n > 0 ? g.n : 1, BLOCK), BLOCK, 0, st>>>(g.off, g.n, nt, first);
  MGCD_LAUNCHED();
  return first;
}

// Rows of a tile of consecutive CSR entries [e0, e1) (non-empty): the rows meeting it
// lie in r0 .. r1 (from the tile table, or two binary searches when first is null);
// every row r0 < r <= r1 that starts inside the tile marks its first position in an
// LDS count array, whose inclusive prefix sum then gives the entry at tile position x
// the row r0 + starts[x] (no per-entry search).  Whole-workgroup call; returns r0.
__device__ inline int32_t tile_rows(const Graph &g, int64_t e0, int64_t e1, uint32_t *starts,
                                    const int32_t *first) {
  __shared__ uint32_t wsum[BLOCK / WAVE];
  __shared__ int32_t sr[2];
  const int t = threadIdx.x, w = t / WAVE;
  for (int x = t; x < SF_TILE; x += BLOCK) starts[x] = 0;
  if (first) {
    if (t < 2) sr[t] = first[blockIdx.x + t];
  } else {
    if (t == 0) sr[0] = row_of_entry(g.off, 0, g.n - 1, e0);
    if (t == 1) sr[1] = row_of_entry(g.off, 0, g.n - 1, e1 - 1);
  }
  __syncthreads();
  const int32_t r0 = sr[0], r1 = sr[1];
  // rows r0 < r <= r1 starting before e1 start inside the tile (off[r0 + 1] > e0)
  for (int64_t r = (int64_t)r0 + 1 + t; r <= r1; r += BLOCK) {
    const int64_t p = g.off[r] - e0;
    if (p < e1 - e0) atomicAdd(&starts[p], 1u);
  }
  __syncthreads();
  // inclusive prefix sum of the counts: thread t owns positions SF_ITEMS*t ..
  uint32_t v[SF_ITEMS], run = 0;
#pragma unroll
  for (int q = 0; q < SF_ITEMS; ++q) {
    v[q] = starts[t * SF_ITEMS + q];
    run += v[q];
  }
  const uint32_t incl = wave_inclusive_scan(run);
  if (lane_id() == WAVE - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t acc = incl - run;
  for (int q = 0; q < w; ++q) acc += wsum[q];
#pragma unroll
  for (int q = 0; q < SF_ITEMS; ++q) {
    acc += v[q];
    starts[t * SF_ITEMS + q] = acc;
  }
  __syncthreads();
  return r0;
}


__global__ void __launch_bounds__(BLOCK)
    k_row_weight_sums(Graph g, const int32_t *first, uint32_t *K, unsigned long long *Wpart) {
  __shared__ uint32_t ex[DG_TILE + 1];
  __shared__ uint32_t wsum[BLOCK / WAVE];
  __shared__ unsigned long long wtot[BLOCK / WAVE];
  __shared__ int32_t sr[2];
  const int t = threadIdx.x, w = t / WAVE;
  const int64_t e0 = (int64_t)blockIdx.x * DG_TILE;
  const int64_t e1 = e0 + DG_TILE < g.nnz ? e0 + DG_TILE : g.nnz;
  static_assert(DG_TILE == SF_TILE, "one tile table");
  if (first) {  // rows meeting the tile lie in sr[0] .. sr[1]
    if (t < 2) sr[t] = first[blockIdx.x + t];
  } else {
    if (t == 0) sr[0] = row_of_entry(g.off, 0, g.n - 1, e0);
    if (t == 1) sr[1] = row_of_entry(g.off, 0, g.n - 1, e1 - 1);
  }
  unsigned long long tsum = 0;
#pragma unroll
  for (int q = 0; q < DG_ITEMS; ++q) {
    const int x = q * BLOCK + t;
    const uint32_t v = e0 + x < e1 ? __builtin_nontemporal_load(g.w + e0 + x) : 0u;
    ex[x] = v;
    tsum += v;
  }
  __syncthreads();
  // exclusive prefix sums in place: thread t owns positions DG_ITEMS*t ..
  uint32_t v[DG_ITEMS], run = 0;
#pragma unroll
  for (int q = 0; q < DG_ITEMS; ++q) {
    v[q] = ex[t * DG_ITEMS + q];
    run += v[q];
  }
  const uint32_t incl = wave_inclusive_scan(run);
  tsum = wave_sum(tsum);
  if (lane_id() == WAVE - 1) wsum[w] = incl;
  if (lane_id() == 0) wtot[w] = tsum;
  __syncthreads();
  uint32_t acc = incl - run;
  for (int q = 0; q < w; ++q) acc += wsum[q];
#pragma unroll
  for (int q = 0; q < DG_ITEMS; ++q) {
    ex[t * DG_ITEMS + q] = acc;
    acc += v[q];
  }
  if (t == BLOCK - 1) ex[DG_TILE] = acc;
  __syncthreads();
  if (t == 0) {
    unsigned long long total = 0;
    for (int q = 0; q < BLOCK / WAVE; ++q) total += wtot[q];
    if (total) atomicAdd(&Wpart[spread_copy()], total);
  }
  const int32_t r0 = sr[0], r1 = sr[1];
  for (int64_t r = (int64_t)r0 + t; r <= r1; r += BLOCK) {
    const int64_t lo = g.off[r], hi = g.off[r + 1];
    const int64_t a = lo > e0 ? lo : e0, b = hi < e1 ? hi : e1;
    if (b <= a) continue;  // empty row
    const uint32_t part = ex[b - e0] - ex[a - e0];
    if (lo >= e0 && hi <= e1)
      K[r] = part;
    else
      atomicAdd(&K[r], part);
  }
}

__global__ void k_fold_total(const unsigned long long *part, unsigned long long *W) {
  const unsigned long long s = wave_sum(part[lane_id()]);  // one wave, SPREAD == WAVE
  if (lane_id() == 0) *W = s;
}

size_t degrees_ws_bytes(int64_t nnz) { return (size_t)SPREAD * 8 + 4096 + tile_table_bytes(nnz); }

void launch_degrees(const Graph &g, uint32_t *K, unsigned long long *W, Arena &a, hipStream_t st) {
  static_assert(SPREAD == WAVE, "k_fold_total folds one copy per lane");
  size_t mk = a.mark();
  unsigned long long *part = a.take<unsigned long long>(SPREAD);
  launch_zero_u64(part, SPREAD, st);
  if (g.n > 0) zero_u32(K, g.n, st);
  if (g.nnz > 0) {
    // the tile table when the workspace holds it (a fixed scratch may not): else each
    // workgroup finds its rows by binary search
    const size_t tb = (size_t)(ceil_div(g.nnz, SF_TILE) + 1) * 4;
    const int32_t *first = ((a.used + 255) & ~(size_t)255) + tb <= a.cap ? tile_first_rows(g, a, st) : nullptr;
    k_row_weight_sums<<<(unsigned)ceil_div(g.nnz, DG_TILE), BLOCK, 0, st>>>(g, first, K, part);
    MGCD_LAUNCHED();
  }
  k_fold_total<<<1, WAVE, 0, st>>>(part, W);
  MGCD_LAUNCHED();
  a.release(mk);
}

// ---- canonical labels ----------------------------------------------------------------

// Smallest member id of every community (ids are non-negative, so unsigned order).
__global__ void __launch_bounds__(BLOCK) k_min_member(const int32_t *C, int32_t n, int32_t *minv) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool ok = v < n;
  block_combine<true>(ok, ok ? (uint32_t)C[v] : 0u, (uint32_t)v, reinterpret_cast<uint32_t *>(minv));
}
__global__ void k_is_first(const int32_t *C, const int32_t *minv, int32_t n, uint32_t *first) {
  int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) first[v] = minv[C[v]] == (int32_t)v ? 1u : 0u;
}
__global__ void k_canon(const int32_t *C, const int32_t *minv, const int64_t *rank, int32_t n,
                        int32_t *out) {
  int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) out[v] = (int32_t)rank[minv[C[v]]];
}
__global__ void k_fill_max(int32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = 0x7FFFFFFF;
}

int32_t canonical(const int32_t *C, int32_t n, int32_t *out, Arena &a, hipStream_t st) {
  if (n == 0) return 0;
  size_t mk = a.mark();
  int32_t *minv = a.take<int32_t>(n);
  uint32_t *first = a.take<uint32_t>(n);
  int64_t *rank = a.take<int64_t>((int64_t)n + 1);
  k_fill_max<<<grid_for(n), BLOCK, 0, st>>>(minv, n);
  MGCD_LAUNCHED();
  k_min_member<<<grid_for(n), BLOCK, 0, st>>>(C, n, minv);
  MGCD_LAUNCHED();
  k_is_first<<<grid_for(n), BLOCK, 0, st>>>(C, minv, n, first);
  MGCD_LAUNCHED();
  scan_u32_i64(first, rank, n, rank + n, a, st);
  k_canon<<<grid_for(n), BLOCK, 0, st>>>(C, minv, rank, n, out);
  MGCD_LAUNCHED();
  int64_t m = 0;
  MGCD_HIP(hipMemcpyAsync(&m, rank + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  a.release(mk);
  return (int32_t)m;
}

// ---- modularity ------------------------------------------------------------------------

// Weight of the intra-community entries (sigma of Eq. 1 summed over communities):
// SF_TILE consecutive entries per workgroup with their rows from tile_rows, every
// entry's C[row] and C[j] gathered together; the workgroup total goes to one of SPREAD
// copies of terms[0].
__global__ void __launch_bounds__(BLOCK)
    k_intra(Graph g, const int32_t *C, unsigned long long *terms) {
  __shared__ uint32_t starts[SF_TILE];
  __shared__ unsigned long long lw[BLOCK / WAVE];
  const int t = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * SF_TILE;
  const int64_t e1 = e0 + SF_TILE < g.nnz ? e0 + SF_TILE : g.nnz;
  const int32_t r0 = tile_rows(g, e0, e1, starts, nullptr);
  unsigned long long tot = 0;
#pragma unroll
  for (int q = 0; q < SF_ITEMS; ++q) {
    const int64_t x = (int64_t)q * BLOCK + t;
    const bool v = e0 + x < e1;
    const int64_t e = v ? e0 + x : e0;
    const int32_t ci = C[r0 + (int32_t)starts[v ? x : 0]];
    const int32_t cj = C[__builtin_nontemporal_load(g.idx + e)];
    const uint32_t w = __builtin_nontemporal_load(g.w + e);
    tot += (v && ci == cj) ? w : 0u;
  }
  tot = wave_sum(tot);
  if (lane_id() == 0) lw[t / WAVE] = tot;
  __syncthreads();
  if (t == 0) {
    const unsigned long long s = lw[0] + lw[1] + lw[2] + lw[3];
    if (s) atomicAdd(&terms[2 * spread_copy()], s);
  }
}

__global__ void __launch_bounds__(BLOCK)
    k_comm_tot(const int32_t *C, const uint32_t *K, int32_t n, uint32_t *tot) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool ok = i < n;
  block_combine<false>(ok, ok ? (uint32_t)C[i] : 0u, ok ? K[i] : 0u, tot);
}

__global__ void __launch_bounds__(BLOCK)
    k_sum_squares(const uint32_t *tot, int32_t n, unsigned long long *terms) {
  __shared__ unsigned long long lw[4];
  int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  unsigned long long x = c < n ? (unsigned long long)tot[c] : 0ull;
  unsigned long long s = block_sum(x * x, lw);
  if (threadIdx.x == 0 && s) atomicAdd(&terms[2 * spread_copy() + 1], s);
}

void modularity_terms(const Graph &g, const int32_t *C, const uint32_t *K, unsigned long long *terms,
                      Arena &a, hipStream_t st) {
  launch_zero_u64(terms, 2 * SPREAD, st);
  if (g.n == 0) return;
  size_t mk = a.mark();
  uint32_t *tot = a.take<uint32_t>(g.n);
  zero_u32(tot, g.n, st);
  if (g.nnz > 0) {
    k_intra<<<(unsigned)ceil_div(g.nnz, SF_TILE), BLOCK, 0, st>>>(g, C, terms);
    MGCD_LAUNCHED();
  }
  k_comm_tot<<<grid_for(g.n), BLOCK, 0, st>>>(C, K, g.n, tot);
  MGCD_LAUNCHED();
  k_sum_squares<<<grid_for(g.n), BLOCK, 0, st>>>(tot, g.n, terms);
  MGCD_LAUNCHED();
  a.release(mk);
}

// ---- validation --------------------------------------------------------------------------

__global__ void k_check_labels(const int32_t *C, int64_t n, int64_t limit, unsigned long long *flag) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n && (C[i] < 0 || (int64_t)C[i] >= limit)) atomicOr(flag, 1ull);
}

void launch_check_labels(const int32_t *C, int64_t n, int64_t limit, unsigned long long *flag,
                         hipStream_t st) {
  launch_zero_u64(flag, 1, st);
  if (n <= 0) return;
  k_check_labels<<<grid_for(n), BLOCK, 0, st>>>(C, n, limit, flag);
  MGCD_LAUNCHED();
}

__global__ void k_validate_rows(Graph g, unsigned long long *flags) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i > g.n) return;
  bool bad = false;
  if (i == 0) bad |= g.off[0] != 0;
  if (i == g.n) bad |= g.off[g.n] != g.nnz;
  if (i < g.n) bad |= g.off[i + 1] < g.off[i];
  if (bad) atomicOr(&flags[0], 1ull);
}

__global__ void k_validate_entries(Graph g, unsigned long long *flags) {
  int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= g.nnz) return;
  int32_t j = g.idx[e];
  if (j < 0 || j >= g.n || g.w[e] == 0) atomicOr(&flags[0], 2ull);
}

void launch_validate(const Graph &g, unsigned long long *flags, hipStream_t st) {
  k_validate_rows<<<grid_for((int64_t)g.n + 1), BLOCK, 0, st>>>(g, flags);
  MGCD_LAUNCHED();
  if (g.nnz > 0) {
    k_validate_entries<<<grid_for(g.nnz), BLOCK, 0, st>>>(g, flags);
    MGCD_LAUNCHED();
  }
}

// ---- aggregation: member order and community streams ------------------------------------

// Sort keys of the members: their community, or m for a vertex left out (D < 0).
__global__ void k_member_keys(const int32_t *D, int32_t n, int32_t m, uint64_t *key, uint32_t *val) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) {
    key[i] = D[i] >= 0 ? (uint64_t)(uint32_t)D[i] : (uint64_t)m;
    val[i] = (uint32_t)i;
  }
}

// mstart[c] = first position of community c in the sorted member list (every c < m
// has members); mstart[m] = number of members that belong to some community.
__global__ void k_member_bounds(const uint64_t *ks, int32_t n, int32_t m, int32_t *mstart) {
  int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (t >= n) return;
  const uint64_t c = ks[t];
  const bool first = t == 0 || ks[t - 1] != c;
  if (first) mstart[c] = (int32_t)t;  // c <= m; c == m marks the first left-out vertex
  if (t == n - 1 && c < (uint64_t)m) mstart[m] = n;
}

__global__ void k_member_deg(const int64_t *off, const uint32_t *mem, int32_t n, uint32_t *mdeg) {
  int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (t < n) {
    uint32_t i = mem[t];
    mdeg[t] = (uint32_t)(off[i + 1] - off[i]);
  }
}

// Category of every community stream: b = log2 of the lanes it needs (0..6, at
// most 64 chunks; sort key heavy first within b = 0) or 7 = longer.  With split > 0
// (the 32/64-slot sketch): 0 = one wave, 7 = more than max(L, split) positions.
__global__ void __launch_bounds__(BLOCK)
    k_comm_keys(const int32_t *mstart, const int64_t *P, int32_t m, int64_t L, int64_t split,
                uint64_t *key, uint32_t *val, unsigned long long *cnt) {
  __shared__ unsigned long long bc[8];
  if (threadIdx.x < 8) bc[threadIdx.x] = 0;
  __syncthreads();
  int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  int cat = -1;
  int64_t lmax = 0;
  if (c < m) {
    int64_t len = P[mstart[c + 1]] - P[mstart[c]];
    lmax = len;
    if (split != 0) {  // wave sketch: split streams (split < 0: every non-empty one)
      cat = (split < 0 ? len > 0 : (len > L && len > split)) ? 7 : 0;
      int b = 0;
      while (b < 63 && (len >> b) != 0) ++b;
      key[c] = cat == 7 ? 207ull : (uint64_t)(64 - b);
    } else if (len <= L) {
      int b = 0;
      while (b < 63 && (len >> b) != 0) ++b;
      cat = 0;
      key[c] = (uint64_t)(64 - b);
    } else {
      int64_t nc = (len + L - 1) / L;
      int lp = 0;
      while ((1ll << lp) < nc) ++lp;
      cat = lp <= 6 ? lp : 7;
      key[c] = 200ull + (uint64_t)cat;
    }
    val[c] = (uint32_t)c;
  }
  for (int q = 0; q < 8; ++q) {
    uint64_t mk = __ballot(cat == q);
    if (lane_id() == 0 && mk) atomicAdd(&bc[q], (unsigned long long)__popcll(mk));
  }
  __syncthreads();
  cnt += spread_copy() * 9;
  if (threadIdx.x < 8 && bc[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], bc[threadIdx.x]);
  // block maximum, then one atomic per block, skipped when it cannot raise the value
  __shared__ unsigned long long bmax[BLOCK / WAVE];
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int64_t x = __shfl_xor(lmax, o);
    lmax = x > lmax ? x : lmax;
  }
  if (lane_id() == 0) bmax[threadIdx.x / WAVE] = (unsigned long long)lmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mx = bmax[0];
    for (int q = 1; q < BLOCK / WAVE; ++q) mx = bmax[q] > mx ? bmax[q] : mx;
    if (mx > 0 && mx > __hip_atomic_load(&cnt[8], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&cnt[8], mx);
  }  // longest stream
}

__global__ void k_comm_chunks(const int32_t *mstart, const int64_t *P, const int32_t *multi,
                              int64_t nmulti, int64_t L, int64_t *nch) {
  int64_t x = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (x >= nmulti) return;
  int32_t c = multi[x];
  int64_t len = P[mstart[c + 1]] - P[mstart[c]];
  nch[x] = (len + L - 1) / L;
}

__global__ void k_comm_groups(const int64_t *cstart, int64_t nmulti, int64_t *ng) {
  int64_t x = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (x < nmulti) ng[x] = (cstart[x + 1] - cstart[x] + WAVE - 1) / WAVE;
}

__global__ void k_comm_owner(const int64_t *cstart, int64_t nmulti, int32_t *owner) {
  int64_t x = blockIdx.x;
  if (x >= nmulti) return;
  for (int64_t q = cstart[x] + threadIdx.x; q < cstart[x + 1]; q += BLOCK) owner[q] = (int32_t)x;
}

__global__ void k_u32_to_i32(const uint32_t *v, int32_t *out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) out[i] = (int32_t)v[i];
}

struct AggStreams {
  Graph g;
  const int32_t *D;
  const uint32_t *mem;    // members sorted by community, ascending id within one
  const int32_t *mstart;  // [m+1]
  const int64_t *P;       // [n+1] stream position of each member's row
  const int64_t *rs;      // [n] CSR offset of each member's row (off[mem[t]])
  const uint32_t *skey;   // [positions] the streams laid out contiguously: key D[j]
  const uint32_t *sw;     //             and weight of every position
};

// Stream position of every vertex's row (-1: the vertex is in no community); the
// member count *nmem is read on the device (no host round trip).
__global__ void k_row_pos(const uint32_t *mem, const int64_t *P, const int32_t *nmem, int32_t n,
                          int64_t *rowpos) {
  int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (t < n && t < *nmem) rowpos[mem[t]] = P[t];
}

// Lay the community streams out contiguously: entry e of row i goes to position
// rowpos[i] + (e - off[i]) with key D[j] and its weight.  A workgroup takes SF_TILE
// consecutive entries (balanced whatever the row lengths), finds their rows with
// tile_rows and reads and writes the entries in coalesced order.
__global__ void __launch_bounds__(BLOCK)
    k_agg_streamify(Graph g, const int32_t *first, const int32_t *D, const int64_t *rowpos, uint32_t *skey,
                    uint32_t *sw) {
  __shared__ uint32_t starts[SF_TILE];
  const int t = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * SF_TILE;
  const int64_t e1 = e0 + SF_TILE < g.nnz ? e0 + SF_TILE : g.nnz;
  const int32_t r0 = tile_rows(g, e0, e1, starts, first);
  // all loads and gathers are issued first (a position past the end reads entry e0),
  // then the stores, so the gathers of the SF_ITEMS rounds are in flight together
  int64_t pos[SF_ITEMS];
  uint32_t key[SF_ITEMS], wt[SF_ITEMS];
#pragma unroll
  for (int q = 0; q < SF_ITEMS; ++q) {
    const int64_t x = (int64_t)q * BLOCK + t;
    const bool v = e0 + x < e1;
    const int64_t e = v ? e0 + x : e0;
    const int32_t r = r0 + (int32_t)starts[v ? x : 0];
    const int64_t p = rowpos[r];
    // -1 (all ones) for a position past the end or a row in no community; an OR, not
    // a select, so the load of off[r] is not moved into a branch of its own
    pos[q] = (p + (e - g.off[r])) | ((v && p >= 0) ? 0 : -1);
    key[q] = (uint32_t)D[__builtin_nontemporal_load(g.idx + e)];
    wt[q] = __builtin_nontemporal_load(g.w + e);
  }
#pragma unroll
  for (int q = 0; q < SF_ITEMS; ++q) {
    if (pos[q] >= 0) {
      skey[pos[q]] = key[q];
      sw[pos[q]] = wt[q];
    }
  }
}

// ---- storage copy in degree order ---------------------------------------------------

__global__ void k_degree_keys(const int64_t *off, int32_t n, int64_t nnz, uint64_t *key, uint32_t *val) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  key[i] = (uint64_t)(nnz - (off[i + 1] - off[i]));  // descending degree; stable sort: ascending id
  val[i] = (uint32_t)i;
}

__global__ void k_place(const uint32_t *perm, const int64_t *off, const uint32_t *K, int32_t n, int32_t *pos,
                        int64_t *deg, uint32_t *Kp) {
  const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= n) return;
  const uint32_t v = perm[p];
  pos[v] = (int32_t)p;
  deg[p] = off[v + 1] - off[v];
  Kp[p] = K[v];
}

__global__ void k_row_places(const int32_t *pos, const int64_t *offp, int32_t n, int64_t *rowpos) {
  const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (v < n) rowpos[v] = offp[pos[v]];
}

size_t storage_ws_bytes(int32_t n, int64_t nnz) {
  size_t b = (size_t)(n + 1) * 8 + (size_t)nnz * 8 + 4096;       // offsets, indices, weights
  b += (size_t)n * (4 + 4 + 4) + 4096;                            // perm, pos, K
  b += (size_t)n * (8 + 4) * 2 + radix_sort_ws_bytes(n) + 4096;   // degree sort (released)
  b += (size_t)n * 8 * 2 + scan_ws_bytes((int64_t)n + 1) + 8192;  // degrees, row places (released)
  b += tile_table_bytes(nnz);                                     // tile first rows (released)
  return b;
}

StorageCopy storage_copy(const Graph &g, const uint32_t *K, Arena &a, hipStream_t st) {
  const int32_t n = g.n;
  StorageCopy s{};
  int64_t *offp = a.take<int64_t>((int64_t)n + 1);
  int32_t *idxp = a.take<int32_t>(g.nnz);
  uint32_t *wp = a.take<uint32_t>(g.nnz);
  uint32_t *perm = a.take<uint32_t>(n);
  s.pos = a.take<int32_t>(n);
  s.Kp = a.take<uint32_t>(n);
  s.perm = reinterpret_cast<int32_t *>(perm);
  s.g = Graph{n, g.nnz, offp, idxp, wp};
  if (n == 0) {
    launch_zero_u64(reinterpret_cast<unsigned long long *>(offp), 1, st);
    return s;
  }
  const size_t mk = a.mark();
  uint64_t *k0 = a.take<uint64_t>(n), *k1 = a.take<uint64_t>(n);
  uint32_t *v0 = a.take<uint32_t>(n), *v1 = a.take<uint32_t>(n);
  k_degree_keys<<<grid_for(n), BLOCK, 0, st>>>(g.off, n, g.nnz, k0, v0);
  MGCD_LAUNCHED();
  const bool flip = radix_sort_pairs(k0, v0, k1, v1, n, bits_for((uint64_t)g.nnz), a, st);
  MGCD_HIP(hipMemcpyAsync(perm, flip ? v1 : v0, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  int64_t *deg = a.take<int64_t>(n);
  k_place<<<grid_for(n), BLOCK, 0, st>>>(perm, g.off, K, n, s.pos, deg, s.Kp);
  MGCD_LAUNCHED();
  scan_i64(deg, offp, n, offp + n, a, st);
  int64_t *rowpos = a.take<int64_t>(n);
  k_row_places<<<grid_for(n), BLOCK, 0, st>>>(s.pos, offp, n, rowpos);
  MGCD_LAUNCHED();
  if (g.nnz > 0) {  // entries in source order (coalesced reads), written at their new places
    const int32_t *first = tile_first_rows(g, a, st);
    k_agg_streamify<<<(unsigned)ceil_div(g.nnz, SF_TILE), BLOCK, 0, st>>>(
        g, first, s.pos, rowpos, reinterpret_cast<uint32_t *>(idxp), wp);
    MGCD_LAUNCHED();
  }
  a.release(mk);
  return s;
}

__global__ void k_row_starts(const int64_t *off, const uint32_t *mem, int32_t n, int64_t *rs) {
  int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (t < n) rs[t] = off[mem[t]];
}

// Stream positions [p0, p1) of community c into the sketch.
// Communities whose stream has at most 64 chunks: P = 2^b adjacent lanes per
// community (P >= its chunk count), lane q sketches chunk q, the chunk sketches are
// merged by the fixed tree with cross-lane shuffles and lane 0 writes the row.
struct AggBuckets {
  int64_t wave_begin[7];
  int64_t wave_end[7];
  const int32_t *comm[7];
  int64_t ncomm[7];
};

template <int K>
__device__ inline void write_row(uint32_t (&k)[K], uint32_t (&v)[K], int32_t c, Pair *rows,
                                 uint32_t *rcount);

template <int K, int MODE>
__global__ void __launch_bounds__(BLOCK) MGCD_ROWS_OCCUPANCY(K)
    k_agg_rows(AggStreams s, AggBuckets bk, int64_t L, Pair *rows, uint32_t *rcount) {
  __shared__ __attribute__((aligned(16))) uint32_t swin[BLOCK / WAVE][WAVE * WROW];
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE;
  int b = 6;
  while (b > 0 && wave >= bk.wave_end[b]) --b;
  const int logp = b;
  const int q = lane & ((1 << logp) - 1);
  const int64_t r = (wave - bk.wave_begin[b]) * (WAVE >> logp) + (lane >> logp);
  const bool valid = wave < bk.wave_end[0] && r < bk.ncomm[b];
  const int32_t c = valid ? bk.comm[b][r] : 0;
  const int64_t base = valid ? s.P[s.mstart[c]] : 0, end = valid ? s.P[s.mstart[c + 1]] : 0;
  const int64_t nc = (end - base + L - 1) / L;
  RegSketch<K, MODE> sk;
  sk.reset();
  const int64_t p0 = base + q * L;
  const int64_t p1 = q < nc ? (p0 + L < end ? p0 + L : end) : p0;
  staged_fold<K, MODE>(sk, swin[threadIdx.x / WAVE], p0, p1, s.skey, s.sw);
  sk.finalize();
  for (int l = 0; l < logp; ++l) {
    const int stride = 1 << l;
    uint32_t bk_[K], bv_[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      bk_[p] = __shfl_down(sk.key[p], stride);
      bv_[p] = __shfl_down(sk.val[p], stride);
    }
    const int64_t c_l = (nc + stride - 1) >> l;
    const bool left = (q & ((2 << l) - 1)) == 0;
    if (left && (int64_t)(q >> l) + 1 < c_l) merge_sketch<K>(sk.key, sk.val, bk_, bv_);
  }
  if (valid && q == 0) write_row<K>(sk.key, sk.val, c, rows, rcount);
}

template <int K>
__device__ inline void write_row(uint32_t (&k)[K], uint32_t (&v)[K], int32_t c, Pair *rows,
                                 uint32_t *rcount) {
#pragma unroll
  for (int p = 0; p < K; ++p) k[p] = v[p] > 0 ? k[p] : EMPTY;
  sort_by_key<K>(k, v);
  uint32_t x = 0;
#pragma unroll
  for (int p = 0; p < K; ++p)
    if (k[p] != EMPTY) rows[(int64_t)c * K + x++] = Pair{k[p], v[p]};
  rcount[c] = x;
}

// Streams of more than 64 chunks.
struct AggLong {
  const int32_t *multi;   // [nmulti] such communities
  int64_t nmulti;
  const int64_t *cstart;  // [nmulti+1] first chunk of each
  const int64_t *gstart;  // [nmulti+1] first group of 64 chunks of each
  const int32_t *gowner;  // [ngroups] community index (into multi) of each group
  int64_t ngroups;
  Pair *skbuf;            // [ngroups * K] group roots
};

// Wave w takes the aligned group of 64 chunks gstart[x] .. of long stream x (lane =
// chunk within the group): the staged fold of each chunk, then the first six
// levels of the fixed merge tree with shuffles; lane 0 writes the group's root.
template <int K, int MODE>
__global__ void __launch_bounds__(BLOCK) MGCD_ROWS_OCCUPANCY(K)
    k_agg_chunks(AggStreams s, AggLong lg, int64_t L) {
  __shared__ __attribute__((aligned(16))) uint32_t swin[BLOCK / WAVE][WAVE * WROW];
  const int64_t w = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE;  // wave-uniform
  if (w >= lg.ngroups) return;
  const int lane = lane_id();
  const int32_t x = lg.gowner[w];
  const int32_t c = lg.multi[x];
  const int64_t nc = lg.cstart[x + 1] - lg.cstart[x];
  const int64_t q = (w - lg.gstart[x]) * WAVE + lane;  // chunk index within the stream
  const int64_t base = s.P[s.mstart[c]], end = s.P[s.mstart[c + 1]];
  const int64_t p0 = base + q * L;
  const int64_t p1 = q < nc ? (p0 + L < end ? p0 + L : end) : p0;
  RegSketch<K, MODE> sk;
  sk.reset();
  staged_fold<K, MODE>(sk, swin[threadIdx.x / WAVE], p0, p1, s.skey, s.sw);
  sk.finalize();
#pragma unroll 1
  for (int l = 0; l < 6; ++l) {
    const int stride = 1 << l;
    uint32_t bk_[K], bv_[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      bk_[p] = __shfl_down(sk.key[p], stride);
      bv_[p] = __shfl_down(sk.val[p], stride);
    }
    const int64_t c_l = (nc + stride - 1) >> l;  // nodes at level l
    const bool left = (lane & ((2 << l) - 1)) == 0;
    if (left && (q >> l) + 1 < c_l) merge_sketch<K>(sk.key, sk.val, bk_, bv_);
  }
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < K; ++p)
      lg.skbuf[w * K + p] = Pair{sk.val[p] > 0 ? sk.key[p] : EMPTY, sk.val[p]};
  }
}

template <int K>
__global__ void __launch_bounds__(BLOCK) MGCD_SKETCH_OCCUPANCY(K)
    k_agg_multi(AggLong lg, Pair *rows, uint32_t *rcount) {
  __shared__ Pair lds[BLOCK * K];
  const int32_t x = blockIdx.x;
  const int32_t c = lg.multi[x];
  tree_reduce<K>(lg.skbuf, lg.gstart[x], lg.gstart[x + 1] - lg.gstart[x], lds);  // group roots
  if (threadIdx.x == 0) {
    uint32_t k[K], v[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      k[p] = lds[p].key;
      v[p] = lds[p].val;
    }
    write_row<K>(k, v, c, rows, rcount);
  }
}

// rows (K slots per community, rcount used) -> CSR
__global__ void k_compact_rows(const Pair *rows, const uint32_t *rcount, const int64_t *off, int32_t m,
                               int k, int32_t *idx, uint32_t *w) {
  int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= m) return;
  int64_t o = off[c];
  for (uint32_t x = 0; x < rcount[c]; ++x) {
    Pair p = rows[c * k + x];
    idx[o + x] = (int32_t)p.key;
    w[o + x] = p.val;
  }
}

// Leiden: emit every kept pair forward and, off the diagonal, reversed.
__global__ void k_emit_counts(const Pair *rows, const uint32_t *rcount, int32_t m, int k, uint32_t *ec) {
  int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= m) return;
  uint32_t e = 0;
  for (uint32_t x = 0; x < rcount[c]; ++x) e += rows[c * k + x].key == (uint32_t)c ? 1u : 2u;
  ec[c] = e;
}

__global__ void k_emit(const Pair *rows, const uint32_t *rcount, const int64_t *epos, int32_t m, int k,
                       int b, uint64_t *key, uint32_t *val) {
  int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= m) return;
  int64_t o = epos[c];
  for (uint32_t x = 0; x < rcount[c]; ++x) {
    Pair p = rows[c * k + x];
    key[o] = ((uint64_t)c << b) | p.key;
    val[o++] = p.val;
    if (p.key != (uint32_t)c) {
      key[o] = ((uint64_t)p.key << b) | (uint64_t)c;
      val[o++] = p.val;
    }
  }
}

// Sorted (row, col) keys: run heads (first entry of each distinct key).
__global__ void k_heads(const uint64_t *ks, int64_t n, uint32_t *head) {
  int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (e < n) head[e] = (e == 0 || ks[e - 1] != ks[e]) ? 1u : 0u;
}

// Add every row's number of run heads among this wave's lanes to rowcnt.  The keys
// are sorted, so one row's lanes are consecutive: the first head of each row segment
// adds the segment's count (one atomic per row and wave rather than one per head,
// which serialised on the rows of hub communities).  Every lane of the wave calls it.
__device__ inline void count_heads(bool head, uint32_t row, uint32_t *rowcnt) {
  const int lane = lane_id();
  const uint32_t prev = __shfl_up(row, 1);
  const uint64_t seg_start = __ballot(lane == 0 || row != prev);  // bit 0 always set
  const uint64_t heads = __ballot(head);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // lanes 0..lane
  const int s = 63 - __clzll(seg_start & upto);                     // this segment's start
  const uint64_t later = seg_start & ~upto;                          // later segment starts
  const uint64_t seg = (later ? ((1ull << __builtin_ctzll(later)) - 1) : ~0ull) & ~((1ull << s) - 1);
  const uint64_t sh = heads & seg;
  if (head && lane == __builtin_ctzll(sh)) atomicAdd(&rowcnt[row], (uint32_t)__popcll(sh));
}

// Runs have at most two entries (forward and reversed): keep the larger value.
__global__ void k_dedupe_max(const uint64_t *ks, const uint32_t *vs, const uint32_t *head,
                             const int64_t *rid, int64_t n, int b, int32_t *idx, uint32_t *w,
                             uint32_t *rowcnt) {
  const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool h = e < n && head[e];
  const uint64_t key = e < n ? ks[e] : ~0ull;  // every lane's row keeps a row's lanes together
  if (h) {
    uint32_t v = vs[e];
    if (e + 1 < n && ks[e + 1] == key) v = vs[e + 1] > v ? vs[e + 1] : v;
    const int64_t u = rid[e];
    const uint64_t mask = (b >= 64) ? ~0ull : ((1ull << b) - 1);
    idx[u] = (int32_t)(key & mask);
    w[u] = v;
  }
  count_heads(h, (uint32_t)(key >> b), rowcnt);
}

// Exact aggregation: one key (D[i], D[j]) per CSR entry, SF_TILE entries per
// workgroup with their rows from tile_rows.  Entries of left-out rows (D < 0) get
// the key 2^(2b) - 1, sorted past every real key, and are not counted in kept
// (SPREAD copies, by workgroup).
__global__ void __launch_bounds__(BLOCK)
    k_exact_keys(Graph g, const int32_t *first, const int32_t *D, int b, uint64_t *key, uint32_t *val,
                 unsigned long long *kept) {
  __shared__ uint32_t starts[SF_TILE];
  __shared__ unsigned long long bk[BLOCK / WAVE];
  const int t = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * SF_TILE;
  const int64_t e1 = e0 + SF_TILE < g.nnz ? e0 + SF_TILE : g.nnz;
  const int32_t r0 = tile_rows(g, e0, e1, starts, first);
  const uint64_t left_out = (1ull << (2 * b)) - 1;
  uint64_t ks[SF_ITEMS];
  uint32_t vs[SF_ITEMS];
  unsigned long long cnt = 0;
#pragma unroll
  for (int q = 0; q < SF_ITEMS; ++q) {
    const int64_t x = (int64_t)q * BLOCK + t;
    const bool v = e0 + x < e1;
    const int64_t e = v ? e0 + x : e0;
    const int32_t di = D[r0 + (int32_t)starts[v ? x : 0]];
    const int32_t dj = D[__builtin_nontemporal_load(g.idx + e)];
    const bool in = v && di >= 0;
    cnt += in ? 1 : 0;
    ks[q] = in ? ((uint64_t)(uint32_t)di << b) | (uint64_t)(uint32_t)dj : left_out;
    vs[q] = __builtin_nontemporal_load(g.w + e);
  }
#pragma unroll
  for (int q = 0; q < SF_ITEMS; ++q) {
    const int64_t e = e0 + (int64_t)q * BLOCK + t;
    if (e < e1) {
      key[e] = ks[q];
      val[e] = vs[q];
    }
  }
  cnt = wave_sum(cnt);
  if (lane_id() == 0) bk[t / WAVE] = cnt;
  __syncthreads();
  if (t == 0) {
    const unsigned long long s = bk[0] + bk[1] + bk[2] + bk[3];
    if (s) atomicAdd(&kept[2 * spread_copy()], s);
  }
}

// Sum the weights of each run of equal keys: in-wave segmented sums, one atomic
// per run segment of a wave.
__global__ void __launch_bounds__(BLOCK)
    k_run_sums(const uint64_t *ks, const uint32_t *vs, const int64_t *rid, int64_t n, int b,
               int32_t *idx, uint32_t *w, uint32_t *rowcnt) {
  int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool valid = e < n;
  const uint64_t key = valid ? ks[e] : ~0ull;
  const bool head = valid && (e == 0 || ks[e - 1] != key);
  const int lane = lane_id();
  uint64_t incl = wave_inclusive_scan((uint64_t)(valid ? vs[e] : 0u));
  const uint64_t hm = __ballot(head) | 1ull;  // a wave's first lane starts a segment
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  const int start = 63 - __clzll(hm & upto);
  const uint64_t before = __shfl(incl, start > 0 ? start - 1 : 0);
  const bool next_head = lane == 63 || ((hm >> (lane + 1)) & 1ull) || e + 1 >= n;
  if (valid) {
    int64_t u = rid[e] + (head ? 0 : -1);
    if (head) {
      uint64_t mask = (1ull << b) - 1;
      idx[u] = (int32_t)(key & mask);
    }
    if (next_head) atomicAdd(&w[u], (uint32_t)(incl - (start > 0 ? before : 0ull)));
  }
  count_heads(head, (uint32_t)(key >> b), rowcnt);
}

// ---- aggregation driver -----------------------------------------------------------------

// K = 32 or 64: one wave per community holds a WaveSketch (slot p in lane p).  The
// community's stream (members in ascending id, each row in CSR order) is loaded 64
// entries at a time and folded in stream order; every L positions the chunk sketch
// goes into the fixed merge tree.  The row is the positive slots sorted by key: each
// lane's rank is the number of smaller keys, found by scanning the 64 lanes.
template <int K, int MODE, int DEPTH>
__global__ void __launch_bounds__(BLOCK)
    k_agg_wave(AggStreams s, const int32_t *__restrict__ comms, int64_t ncomm, int64_t L,
               Pair *rows, uint32_t *rcount) {
  static_assert(K <= WAVE, "one slot per lane; larger sketches split every stream");
  __shared__ uint32_t sstack[BLOCK / WAVE][DEPTH * 2 * WAVE];
  const int lane = lane_id();
  const int64_t r = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  if (r >= ncomm) return;
  const int32_t c = uniform(comms[r]);
  WaveSketch<K, MODE> sk;
  sk.reset();
  WaveTree<K, DEPTH> tree{sstack[threadIdx.x / WAVE]};
  int64_t left = L;  // positions left in the current chunk
  const int64_t base = uniform(s.P[s.mstart[c]]), end = uniform(s.P[s.mstart[c + 1]]);
  for (int64_t q0 = base; q0 < end; q0 += WAVE) {
    const int64_t q = q0 + lane;
    const bool v = q < end;
    const uint32_t key = v ? __builtin_nontemporal_load(s.skey + q) : EMPTY;
    const uint32_t w = v ? __builtin_nontemporal_load(s.sw + q) : 0u;
    const int nb = end - q0 < WAVE ? (int)(end - q0) : WAVE;
    for (int u = 0; u < nb; ++u) {
      sk.update(lane_value(key, u), lane_value(w, u));
      if (--left == 0) {  // end of a chunk
        sk.finalize();
        tree.push(sk.key[0], sk.val[0]);
        sk.reset();
        left = L;
      }
    }
  }
  if (left != L) {  // the last, partial chunk
    sk.finalize();
    tree.push(sk.key[0], sk.val[0]);
  }
  uint32_t ck, cv;
  tree.result(ck, cv);
  uint32_t rank = 0;
  for (int u = 0; u < WAVE; ++u) rank += lane_value(ck, u) < ck ? 1u : 0u;
  const uint64_t pos = __ballot(cv > 0);
  if (cv > 0) rows[(int64_t)c * K + rank] = Pair{ck, cv};
  if (lane == 0) rcount[c] = (uint32_t)__popcll(pos);
}

// Streams of more than max(L, WAVE_SPLIT) positions at K = 32 / 64 ("split streams"):
// the same chunk sketches, merge tree and row as k_agg_wave, spread over waves.
struct AggSplit {
  const int32_t *multi;   // [nmulti] split communities
  int64_t nmulti;
  const int64_t *cstart;  // [nmulti+1] first chunk of each
  const int32_t *owner;   // [nchunks] index into multi of each chunk
  int64_t nchunks;
  Pair *node;             // [nchunks * K] chunk sketches, merged in place level by level
};

// One wave per chunk of a split stream: its sketch, finalised, into the chunk's node.
template <int K, int MODE>
__global__ void __launch_bounds__(BLOCK) k_aggw_chunks(AggStreams s, AggSplit sp, int64_t L) {
  const int lane = lane_id();
  const int64_t q = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  if (q >= sp.nchunks) return;
  const int32_t x = uniform(sp.owner[q]);
  const int32_t c = uniform(sp.multi[x]);
  const int64_t end = uniform(s.P[s.mstart[c + 1]]);
  const int64_t p0 = uniform(s.P[s.mstart[c]]) + (q - sp.cstart[x]) * L;
  const int64_t p1 = p0 + L < end ? p0 + L : end;
  WaveSketch<K, MODE> sk;
  sk.reset();
  for (int64_t q0 = p0; q0 < p1; q0 += WAVE) {
    const int64_t t = q0 + lane;
    const bool v = t < p1;
    const uint32_t key = v ? __builtin_nontemporal_load(s.skey + t) : EMPTY;
    const uint32_t w = v ? __builtin_nontemporal_load(s.sw + t) : 0u;
    const int nb = p1 - q0 < WAVE ? (int)(p1 - q0) : WAVE;
    for (int u = 0; u < nb; ++u) sk.update(lane_value(key, u), lane_value(w, u));
  }
  sk.finalize();
#pragma unroll
  for (int r = 0; r < WaveSlots<K>::S; ++r)
    if (r * WAVE + lane < K) sp.node[q * K + r * WAVE + lane] = Pair{sk.key[r], sk.val[r]};
}

// Level `level` of the merge tree of every split stream (node x of a stream, x a
// multiple of 2^(level+1), takes in node x + 2^level if that exists; an odd last node
// is carried).
template <int K>
__global__ void __launch_bounds__(BLOCK) k_aggw_level(AggSplit sp, int level) {
  const int lane = lane_id();
  const int64_t q = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  if (q >= sp.nchunks) return;
  const int32_t x = uniform(sp.owner[q]);
  const int64_t half = (int64_t)1 << level;
  if (((q - sp.cstart[x]) & (2 * half - 1)) != 0) return;
  const int64_t r = q + half;
  if (r >= sp.cstart[x + 1]) return;
  constexpr int S = WaveSlots<K>::S;
  uint32_t ak[S], av[S], bk[S], bv[S];
#pragma unroll
  for (int u = 0; u < S; ++u) {
    const int p = u * WAVE + lane;
    ak[u] = EMPTY;
    av[u] = 0;
    bk[u] = EMPTY;
    bv[u] = 0;
    if (p < K) {
      const Pair pa = sp.node[q * K + p], pb = sp.node[r * K + p];
      ak[u] = pa.key;
      av[u] = pa.val;
      bk[u] = pb.key;
      bv[u] = pb.val;
    }
  }
  wave_merge<K>(ak, av, bk, bv);
#pragma unroll
  for (int u = 0; u < S; ++u)
    if (u * WAVE + lane < K) sp.node[q * K + u * WAVE + lane] = Pair{ak[u], av[u]};
}

// The row of every split stream: the root's positive slots sorted by key.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_aggw_rows(AggSplit sp, Pair *rows, uint32_t *rcount) {
  const int lane = lane_id();
  const int64_t x = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  if (x >= sp.nmulti) return;
  const int32_t c = uniform(sp.multi[x]);
  constexpr int S = WaveSlots<K>::S;
  uint32_t ck[S], cv[S];
#pragma unroll
  for (int u = 0; u < S; ++u) {
    ck[u] = EMPTY;
    cv[u] = 0;
    if (u * WAVE + lane < K) {
      const Pair p = sp.node[sp.cstart[x] * K + u * WAVE + lane];
      cv[u] = p.val;
      ck[u] = cv[u] > 0 ? p.key : EMPTY;
    }
  }
  // the row is the positive slots sorted by key: a slot's place is the number of
  // smaller keys among all slots (EMPTY, the largest value, for the others)
  int npos = 0;
#pragma unroll
  for (int u = 0; u < S; ++u) {
    uint32_t rank = 0;
#pragma unroll
    for (int v = 0; v < S; ++v)
      for (int t = 0; t < WAVE; ++t) rank += lane_value(ck[v], t) < ck[u] ? 1u : 0u;
    if (cv[u] > 0) rows[(int64_t)c * K + rank] = Pair{ck[u], cv[u]};
    npos += __popcll(__ballot(cv[u] > 0));
  }
  if (lane == 0) rcount[c] = (uint32_t)npos;
}

// Streams the split path does not take when every non-empty stream is split (K = 128,
// 256): empty ones, whose row is empty.
__global__ void k_empty_rows(const int32_t *comms, int64_t n, uint32_t *rcount) {
  const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (t < n) rcount[comms[t]] = 0;
}

template <int K, int MODE>
static void agg_wave(const AggStreams &s, const int32_t *comms, int64_t ncomm, const AggSplit &sp,
                     int64_t L, Pair *rows, uint32_t *rcount, int64_t max_len, hipStream_t st) {
  if (sp.nmulti > 0) {
    const unsigned cgrid = (unsigned)ceil_div(sp.nchunks, BLOCK / WAVE);
    k_aggw_chunks<K, MODE><<<cgrid, BLOCK, 0, st>>>(s, sp, L);
    MGCD_LAUNCHED();
    const int64_t maxch = (max_len + L - 1) / L;
    for (int l = 0; ((int64_t)1 << l) < maxch; ++l) {
      k_aggw_level<K><<<cgrid, BLOCK, 0, st>>>(sp, l);
      MGCD_LAUNCHED();
    }
    k_aggw_rows<K><<<(unsigned)ceil_div(sp.nmulti, BLOCK / WAVE), BLOCK, 0, st>>>(sp, rows, rcount);
    MGCD_LAUNCHED();
    max_len = L > WAVE_SPLIT ? L : WAVE_SPLIT;  // the longest stream left for one wave
  }
  if (ncomm > 0) {
    if constexpr (K <= WAVE) {
      const unsigned grid = (unsigned)ceil_div(ncomm, BLOCK / WAVE);
      if (wave_depth_for(max_len, L) == WDEPTH_SHALLOW)
        k_agg_wave<K, MODE, WDEPTH_SHALLOW><<<grid, BLOCK, 0, st>>>(s, comms, ncomm, L, rows, rcount);
      else
        k_agg_wave<K, MODE, WDEPTH><<<grid, BLOCK, 0, st>>>(s, comms, ncomm, L, rows, rcount);
    } else {
      k_empty_rows<<<grid_for(ncomm), BLOCK, 0, st>>>(comms, ncomm, rcount);
    }
    MGCD_LAUNCHED();
  }
}

template <int K, int MODE>
static void agg_mg(const AggStreams &s, const AggBuckets &bk, int64_t waves, const AggLong &lg,
                   int64_t L, Pair *rows, uint32_t *rcount, hipStream_t st) {
  if (lg.nmulti > 0) {
    k_agg_chunks<K, MODE><<<(unsigned)ceil_div(lg.ngroups, BLOCK / WAVE), BLOCK, 0, st>>>(s, lg, L);
    MGCD_LAUNCHED();
    k_agg_multi<K><<<(unsigned)lg.nmulti, BLOCK, 0, st>>>(lg, rows, rcount);
    MGCD_LAUNCHED();
  }
  if (waves > 0) {
    k_agg_rows<K, MODE><<<(unsigned)ceil_div(waves, BLOCK / WAVE), BLOCK, 0, st>>>(s, bk, L, rows, rcount);
    MGCD_LAUNCHED();
  }
}

template <int MODE>
static void agg_mg_k(int k, const AggStreams &s, const AggBuckets &bk, int64_t waves, const AggLong &lg,
                     const AggSplit &sp, int64_t L, Pair *rows, uint32_t *rcount, const int32_t *one,
                     int64_t none, int64_t max_len, hipStream_t st) {
  switch (k) {
    case 32: agg_wave<32, MODE>(s, one, none, sp, L, rows, rcount, max_len, st); break;
    case 64: agg_wave<64, MODE>(s, one, none, sp, L, rows, rcount, max_len, st); break;
    case 128: agg_wave<128, MODE>(s, one, none, sp, L, rows, rcount, max_len, st); break;
    case 256: agg_wave<256, MODE>(s, one, none, sp, L, rows, rcount, max_len, st); break;
    case 1: agg_mg<1, MODE>(s, bk, waves, lg, L, rows, rcount, st); break;
    case 2: agg_mg<2, MODE>(s, bk, waves, lg, L, rows, rcount, st); break;
    case 4: agg_mg<4, MODE>(s, bk, waves, lg, L, rows, rcount, st); break;
    case 8: agg_mg<8, MODE>(s, bk, waves, lg, L, rows, rcount, st); break;
    case 16: agg_mg<16, MODE>(s, bk, waves, lg, L, rows, rcount, st); break;
    default: throw Error(-6, "k_aggregate must be 1, 2, 4, 8, 16, 32 or 64");
  }
}

__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = v;
}

static void launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill_i64<<<grid_for(n), BLOCK, 0, st>>>(p, v, n);
  MGCD_LAUNCHED();
}

static int64_t read_i64(const int64_t *p, hipStream_t st) {
  int64_t h = 0;
  MGCD_HIP(hipMemcpyAsync(&h, p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  return h;
}

// CSR offsets from per-row counts.
static void offsets_from_counts(const uint32_t *rowcnt, int32_t m, int64_t *out_off, Arena &a,
                                hipStream_t st) {
  scan_u32_i64(rowcnt, out_off, m, out_off + m, a, st);
}

static int64_t aggregate_exact(const Graph &g, const int32_t *D, int32_t m, int64_t *out_off,
                               int32_t *out_idx, uint32_t *out_w, Arena &a, hipStream_t st) {
  const int64_t E0 = g.nnz;
  const int b = bits_for((uint64_t)m);  // room for the left-out key
  uint32_t *rowcnt = a.take<uint32_t>(m);
  zero_u32(rowcnt, m, st);
  if (E0 == 0) {
    offsets_from_counts(rowcnt, m, out_off, a, st);
    return 0;
  }
  uint64_t *k0 = a.take<uint64_t>(E0), *k1 = a.take<uint64_t>(E0);
  uint32_t *v0 = a.take<uint32_t>(E0), *v1 = a.take<uint32_t>(E0);
  uint32_t *head = a.take<uint32_t>(E0);
  int64_t *rid = a.take<int64_t>(E0 + 1);
  unsigned long long *kept = a.take<unsigned long long>(2 * SPREAD);
  launch_zero_u64(kept, 2 * SPREAD, st);
  const int32_t *first = tile_first_rows(g, a, st);
  k_exact_keys<<<(unsigned)ceil_div(E0, SF_TILE), BLOCK, 0, st>>>(g, first, D, b, k0, v0, kept);
  MGCD_LAUNCHED();
  bool flip = radix_sort_pairs(k0, v0, k1, v1, E0, 2 * b, a, st);
  unsigned long long hk[2];
  read_spread(kept, 1, hk, st);
  const int64_t E = (int64_t)hk[0];
  if (E == 0) {
    offsets_from_counts(rowcnt, m, out_off, a, st);
    return 0;
  }
  const uint64_t *ks = flip ? k1 : k0;
  const uint32_t *vs = flip ? v1 : v0;
  k_heads<<<grid_for(E), BLOCK, 0, st>>>(ks, E, head);
  MGCD_LAUNCHED();
  scan_u32_i64(head, rid, E, rid + E, a, st);
  int64_t R = read_i64(rid + E, st);
  zero_u32(out_w, R, st);
  k_run_sums<<<grid_for(E), BLOCK, 0, st>>>(ks, vs, rid, E, b, out_idx, out_w, rowcnt);
  MGCD_LAUNCHED();
  offsets_from_counts(rowcnt, m, out_off, a, st);
  return R;
}

int64_t aggregate(const Graph &g, const int32_t *D, int32_t m, int mode, int k, int64_t L,
                  int symmetric, int64_t *out_off, int32_t *out_idx, uint32_t *out_w, Arena &a,
                  hipStream_t st) {
  const int32_t n = g.n;
  size_t mk = a.mark();
  if (mode == MODE_EXACT) {
    int64_t r = aggregate_exact(g, D, m, out_off, out_idx, out_w, a, st);
    a.release(mk);
    return r;
  }
  // members in ascending id within each community (stable radix sort by D)
  uint64_t *k0 = a.take<uint64_t>(n), *k1 = a.take<uint64_t>(n);
  uint32_t *v0 = a.take<uint32_t>(n), *v1 = a.take<uint32_t>(n);
  k_member_keys<<<grid_for(n), BLOCK, 0, st>>>(D, n, m, k0, v0);
  MGCD_LAUNCHED();
  bool flip = radix_sort_pairs(k0, v0, k1, v1, n, bits_for((uint64_t)m), a, st);
  const uint64_t *ks = flip ? k1 : k0;
  const uint32_t *mem = flip ? v1 : v0;
  int32_t *mstart = a.take<int32_t>((int64_t)m + 1);
  k_member_bounds<<<grid_for(n), BLOCK, 0, st>>>(ks, n, m, mstart);
  MGCD_LAUNCHED();
  uint32_t *mdeg = a.take<uint32_t>(n);
  int64_t *P = a.take<int64_t>((int64_t)n + 1);
  k_member_deg<<<grid_for(n), BLOCK, 0, st>>>(g.off, mem, n, mdeg);
  MGCD_LAUNCHED();
  scan_u32_i64(mdeg, P, n, P + n, a, st);
  // communities: short streams (one lane each) vs long ones (chunks + merge tree)
  unsigned long long *cnt = a.take<unsigned long long>(SPREAD * 9);
  launch_zero_u64(cnt, SPREAD * 9, st);
  uint64_t *ck0 = a.take<uint64_t>(m), *ck1 = a.take<uint64_t>(m);
  uint32_t *cv0 = a.take<uint32_t>(m), *cv1 = a.take<uint32_t>(m);
  const bool wave = k > 16;  // the 32/64-slot sketch: one wave per stream, long ones split;
                            // 128/256 slots: every non-empty stream split
  k_comm_keys<<<grid_for(m), BLOCK, 0, st>>>(mstart, P, m, L, !wave ? 0 : k > WAVE ? -1 : WAVE_SPLIT, ck0,
                                             cv0, cnt);
  MGCD_LAUNCHED();
  bool cf = radix_sort_pairs(ck0, cv0, ck1, cv1, m, 8, a, st);
  int32_t *corder = a.take<int32_t>(m);
  k_u32_to_i32<<<grid_for(m), BLOCK, 0, st>>>(cf ? cv1 : cv0, corder, m);
  MGCD_LAUNCHED();
  unsigned long long hc[9];
  read_spread(cnt, 8, hc, st);
  MGCD_HIP(hipStreamSynchronize(st));
  AggBuckets bk{};
  int64_t pos = 0, waves = 0;
  const int32_t *bucket_rows[7];
  for (int b = 0; b <= 6; ++b) {
    bucket_rows[b] = corder + pos;
    pos += (int64_t)hc[b];
  }
  for (int b = 6; b >= 0; --b) {  // heaviest bucket first in the grid
    bk.comm[b] = bucket_rows[b];
    bk.ncomm[b] = (int64_t)hc[b];
    bk.wave_begin[b] = waves;
    waves += ceil_div((int64_t)hc[b] << b, WAVE);
    bk.wave_end[b] = waves;
  }
  const int64_t nmulti = (int64_t)hc[7];
  int32_t *multi = corder + pos;
  int64_t *cstart = nullptr;
  AggLong lg{multi, nmulti, nullptr, nullptr, nullptr, 0, nullptr};
  AggSplit sp{multi, 0, nullptr, nullptr, 0, nullptr};
  if (nmulti > 0) {
    int64_t *nch = a.take<int64_t>(nmulti);
    cstart = a.take<int64_t>(nmulti + 1);
    k_comm_chunks<<<grid_for(nmulti), BLOCK, 0, st>>>(mstart, P, multi, nmulti, L, nch);
    MGCD_LAUNCHED();
    scan_i64(nch, cstart, nmulti, cstart + nmulti, a, st);
  }
  if (wave && nmulti > 0) {  // chunks of the split streams
    const int64_t nchunks = read_i64(cstart + nmulti, st);
    int32_t *owner = a.take<int32_t>(nchunks);
    k_comm_owner<<<(unsigned)nmulti, BLOCK, 0, st>>>(cstart, nmulti, owner);
    MGCD_LAUNCHED();
    sp = AggSplit{multi, nmulti, cstart, owner, nchunks, a.take<Pair>(nchunks * k)};
  } else if (nmulti > 0) {
    // groups of 64 chunks per long stream
    int64_t *ng = a.take<int64_t>(nmulti);
    int64_t *gstart = a.take<int64_t>(nmulti + 1);
    k_comm_groups<<<grid_for(nmulti), BLOCK, 0, st>>>(cstart, nmulti, ng);
    MGCD_LAUNCHED();
    scan_i64(ng, gstart, nmulti, gstart + nmulti, a, st);
    const int64_t ngroups = read_i64(gstart + nmulti, st);
    int32_t *gowner = a.take<int32_t>(ngroups);
    k_comm_owner<<<(unsigned)nmulti, BLOCK, 0, st>>>(gstart, nmulti, gowner);
    MGCD_LAUNCHED();
    lg = AggLong{multi, nmulti, cstart, gstart, gowner, ngroups, a.take<Pair>(ngroups * k)};
  }
  Pair *rows = a.take<Pair>((int64_t)m * k);
  uint32_t *rcount = a.take<uint32_t>(m);
  int64_t *rs = a.take<int64_t>(n);
  k_row_starts<<<grid_for(n), BLOCK, 0, st>>>(g.off, mem, n, rs);
  MGCD_LAUNCHED();
  int64_t *rowpos = a.take<int64_t>(n);
  launch_fill_i64(rowpos, -1, n, st);
  if (n > 0) {
    k_row_pos<<<grid_for(n), BLOCK, 0, st>>>(mem, P, mstart + m, n, rowpos);
    MGCD_LAUNCHED();
  }
  // the streams hold the members' rows: at most nnz positions
  uint32_t *skey = a.take<uint32_t>(g.nnz);
  uint32_t *sw = a.take<uint32_t>(g.nnz);
  if (g.nnz > 0) {
    const int32_t *first = tile_first_rows(g, a, st);
    k_agg_streamify<<<(unsigned)ceil_div(g.nnz, SF_TILE), BLOCK, 0, st>>>(g, first, D, rowpos, skey, sw);
    MGCD_LAUNCHED();
  }
  AggStreams s{g, D, mem, mstart, P, rs, skey, sw};
  switch (mode) {
    case MODE_ALG1: agg_mg_k<MODE_ALG1>(k, s, bk, waves, lg, sp, L, rows, rcount, corder, (int64_t)hc[0], (int64_t)hc[8], st); break;
    case MODE_UNCOND: agg_mg_k<MODE_UNCOND>(k, s, bk, waves, lg, sp, L, rows, rcount, corder, (int64_t)hc[0], (int64_t)hc[8], st); break;
    case MODE_STD: agg_mg_k<MODE_STD>(k, s, bk, waves, lg, sp, L, rows, rcount, corder, (int64_t)hc[0], (int64_t)hc[8], st); break;
    default: throw Error(-6, "unknown sketch mode");
  }
  int64_t total = 0;
  if (!symmetric) {
    offsets_from_counts(rcount, m, out_off, a, st);
    k_compact_rows<<<grid_for(m), BLOCK, 0, st>>>(rows, rcount, out_off, m, k, out_idx, out_w);
    MGCD_LAUNCHED();
    total = read_i64(out_off + m, st);
  } else {
    uint32_t *ec = a.take<uint32_t>(m);
    int64_t *epos = a.take<int64_t>((int64_t)m + 1);
    k_emit_counts<<<grid_for(m), BLOCK, 0, st>>>(rows, rcount, m, k, ec);
    MGCD_LAUNCHED();
    scan_u32_i64(ec, epos, m, epos + m, a, st);
    const int64_t E2 = read_i64(epos + m, st);
    const int b = bits_for((uint64_t)(m > 1 ? m - 1 : 1));
    uint64_t *e0 = a.take<uint64_t>(E2), *e1 = a.take<uint64_t>(E2);
    uint32_t *w0 = a.take<uint32_t>(E2), *w1 = a.take<uint32_t>(E2);
    k_emit<<<grid_for(m), BLOCK, 0, st>>>(rows, rcount, epos, m, k, b, e0, w0);
    MGCD_LAUNCHED();
    bool ef = radix_sort_pairs(e0, w0, e1, w1, E2, 2 * b, a, st);
    const uint64_t *sk = ef ? e1 : e0;
    const uint32_t *sv = ef ? w1 : w0;
    uint32_t *head = a.take<uint32_t>(E2);
    int64_t *rid = a.take<int64_t>(E2 + 1);
    uint32_t *rowcnt = a.take<uint32_t>(m);
    zero_u32(rowcnt, m, st);
    if (E2 > 0) {
      k_heads<<<grid_for(E2), BLOCK, 0, st>>>(sk, E2, head);
      MGCD_LAUNCHED();
      scan_u32_i64(head, rid, E2, rid + E2, a, st);
      k_dedupe_max<<<grid_for(E2), BLOCK, 0, st>>>(sk, sv, head, rid, E2, b, out_idx, out_w, rowcnt);
      MGCD_LAUNCHED();
    }
    offsets_from_counts(rowcnt, m, out_off, a, st);
    total = read_i64(out_off + m, st);
  }
  a.release(mk);
  return total;
}

size_t aggregate_ws_bytes(int32_t n, int64_t nnz, int mode, int k, int64_t L, bool symmetric) {
  size_t b = 0;
  if (mode == MODE_EXACT) {
    b += (size_t)nnz * (8 + 8 + 4 + 4 + 4 + 8) + 8192;
    b += radix_sort_ws_bytes(nnz) + scan_ws_bytes(nnz) + (size_t)n * 4 + 4096;
    return b + tile_table_bytes(nnz) + 64 * 1024;
  }
  b += (size_t)n * (8 + 8 + 4 + 4) + 4096;          // member sort buffers
  b += radix_sort_ws_bytes(n) + 4096;
  b += (size_t)(n + 1) * (4 + 4 + 8) + 4096;        // mstart, mdeg, P
  b += scan_ws_bytes(n + 1) + 4096;
  b += (size_t)n * (8 + 8 + 4 + 4 + 4 + 8) + 4096;  // community sort, order, row starts
  // streams of more than 64 chunks: at most nnz / (64 L) of them, at most
  // nnz / L + that many chunks
  const int64_t Lc = L > 0 ? L : 1;
  const int64_t nm = nnz / (64 * Lc) + 1, chunks = nnz / Lc + nm + 1;
  b += (size_t)(nm + 1) * 16 + scan_ws_bytes(nm) + (size_t)chunks * (4 + (size_t)k * sizeof(Pair)) + 8192;
  if (k > 16) {  // split streams of the 32/64-slot sketch: more than max(L, WAVE_SPLIT)
    // positions; of the 128/256-slot sketch: every non-empty stream (at most min(n, nnz))
    const int64_t nw = k > WAVE ? (n < nnz ? (int64_t)n : nnz) + 1 : nnz / (Lc > WAVE_SPLIT ? Lc : WAVE_SPLIT) + 1;
    const int64_t cw = nnz / Lc + nw + 1;
    b += (size_t)(nw + 1) * 16 + scan_ws_bytes(nw) + (size_t)cw * (4 + (size_t)k * sizeof(Pair)) + 8192;
  }
  b += (size_t)n * k * sizeof(Pair) + (size_t)n * 4 + 4096;  // rows, rcount
  b += (size_t)nnz * 8 + (size_t)n * 8 + 4096;               // laid-out streams, row positions
  b += tile_table_bytes(nnz);                                // tile first rows
  if (symmetric) {
    // emit buffers (rows hold at most their stream: <= 2 min(k n, nnz) entries), sort, heads
    int64_t e2 = 2 * ((int64_t)n * k < nnz ? (int64_t)n * k : nnz);
    b += (size_t)n * (4 + 8 + 4) + (size_t)e2 * (8 + 8 + 4 + 4 + 4 + 8) + 16384;
    b += radix_sort_ws_bytes(e2) + scan_ws_bytes(e2);
  }
  return b + 64 * 1024;
}

}  // namespace mgcd
