// Local-moving sweeps: LPA iterations (Section 4.3), Louvain/Leiden local moving
// (Sections 4.1-4.2, Fig. 2) and Leiden refinement, with the weighted Misra-Gries
// sketch (Appendix A.1, Algorithm 1) or an exact table (Section 4, Fig. 1).
//
// Per vertex i with current community d = C[i]:
//   pass 1  stream the row (self excluded; refinement: same bound only), key C[j],
//           into a K-slot sketch; rows longer than L positions are cut into chunks
//           of L, each sketched from empty, then merged pairwise left to right,
//           level by level (odd last moves up);
//   pass 2  exact K_{i->c} of every positive slot and K_{i->d} (skipped when the
//           sketch lost no weight: its values are then exact and complete);
//   decide  LPA: largest K_{i->c}, lowest c on ties.  Louvain/Leiden: largest
//           G = W (K_ic - K_id) - K_i (K_i + Sigma_c - Sigma_d) (Eq. 2 times W^2/2),
//           c != d, G > 0, lowest c on ties; applied only in the sweep's direction.
//
// Mapping on CDNA: every chunk is one lane's stream with the sketch in VGPRs.  A
// row of at most 64 chunks occupies 2^b adjacent lanes of one wave (b = 0 for a
// row of one chunk; rows of one chunk ordered heavy-first so a wave's lanes have
// similar trip counts); its chunk sketches are merged with cross-lane shuffles and
// the same lanes run pass 2.  Rows of more than 64 chunks write chunk sketches to
// scratch and one workgroup per row merges them in LDS and runs pass 2 with
// block-strided (coalesced) reads.
#include "move.hpp"
#include "primitives.hpp"
#include "sketch.hpp"
#include "staging.hpp"
#include "wave_sketch.hpp"

namespace mgcd {

// ---- decision ---------------------------------------------------------------------

struct Counters {
  uint32_t moved = 0, prop = 0, cand = 0;
  int32_t g = 0;  // batched: the graph of the rows counted (one row per lane per flush)
  uint64_t sumG = 0;
};

template <int ALGO>
__device__ inline int32_t community_of_self(const SweepArgs &a, int32_t i) {
  return ALGO == ALGO_REFINE ? i : a.C[i];
}

// Evaluate one candidate community c with exact linking weight kc; keep the best.
// Total weight W of vertex i's graph.
__device__ inline uint64_t weight_of(const SweepArgs &a, int32_t i) {
  return a.gid ? (uint64_t)a.Wg[a.gid[i]] : a.W;
}

// Batched runs: a vertex of a graph that no longer moves keeps its community.
__device__ inline bool frozen(const SweepArgs &a, int32_t i) {
  return (a.halt && *a.halt) || (a.gid && !a.active[a.gid[i]]);
}

// Batched runs: no graph moves any more (set after the previous sweep), so this sweep
// does nothing at all and the labels stay in the buffer the last real sweep wrote.
// Wave-uniform (written before the kernel started).
__device__ inline bool level_over(const SweepArgs &a) { return a.live && *a.live == 0; }

// Evaluate candidate c (present: it exists) with exact linking weight kc and
// community total sc; keep the best.  Branch-free, so gathers feeding sc are issued
// together rather than each inside a branch of its own.
template <int ALGO>
__device__ inline void consider_v(int64_t W, int32_t d, int64_t Ki, int64_t Sd, uint32_t kd, int32_t c,
                                  uint32_t kc, uint32_t sc, bool present, int32_t &best, int64_t &bestG) {
  int64_t G;
  bool ok;
  if (ALGO == ALGO_LPA) {
    G = (int64_t)kc;
    ok = present;
  } else {
    G = W * ((int64_t)kc - (int64_t)kd) - Ki * (Ki + (int64_t)sc - Sd);
    ok = present && c != d && G > 0;
  }
  const bool better = ok && (best < 0 || G > bestG || (G == bestG && c < best));
  best = better ? c : best;
  bestG = better ? G : bestG;
}

template <int ALGO>
__device__ inline void consider(const SweepArgs &a, int64_t W, int32_t d, int64_t Ki, int64_t Sd,
                                uint32_t kd, int32_t c, uint32_t kc, int32_t &best, int64_t &bestG) {
  const uint32_t sc = ALGO == ALGO_LPA ? 0u : a.Sig[c];
  consider_v<ALGO>(W, d, Ki, Sd, kd, c, kc, sc, true, best, bestG);
}

// The best of K candidate slots (EMPTY: no candidate).  LPA scores the linking weights
// alone.  Louvain and Leiden also need each candidate's total Sigma_c, a random read.
// The gain W (k_c - k_d) - K_i (K_i + Sigma_c - Sigma_d) is at most its value at
// Sigma_c = 0, so the heaviest candidate is scored first, and another candidate's total
// is read only when that bound can still beat the best so far (or tie it with a lower
// id); a slot that cannot reads Sigma_d instead (cached; the reads stay branch-free and
// in flight together) and is not scored.  The best gain only grows, so a skipped slot
// could neither win nor tie: the result equals scoring every slot.  Returns the number
// of candidates' totals read.
template <int K, int ALGO>
__device__ inline int consider_slots(const SweepArgs &a, int64_t W, int32_t d, int64_t Ki, int64_t Sd,
                                     uint32_t kd, const uint32_t (&key)[K], const uint32_t (&ex)[K],
                                     int32_t &best, int64_t &bestG) {
  if constexpr (ALGO == ALGO_LPA) {
#pragma unroll
    for (int p = 0; p < K; ++p)
      consider_v<ALGO>(W, d, Ki, Sd, kd, (int32_t)key[p], ex[p], 0u, key[p] != EMPTY, best, bestG);
    return 0;
  } else {
    const uint32_t ud = (uint32_t)d;
    uint32_t c0 = EMPTY, x0 = 0;  // the heaviest candidate other than d (ties: first slot)
#pragma unroll
    for (int p = 0; p < K; ++p) {
      const bool take = key[p] != EMPTY && key[p] != ud && (c0 == EMPTY || ex[p] > x0);
      c0 = take ? key[p] : c0;
      x0 = take ? ex[p] : x0;
    }
    const uint32_t s0 = a.Sig[c0 != EMPTY ? (int32_t)c0 : d];
    consider_v<ALGO>(W, d, Ki, Sd, kd, (int32_t)c0, x0, s0, c0 != EMPTY, best, bestG);
    const int64_t rest = Sd - Ki;  // Sigma_d without i: U(c) = W (k_c - k_d) + K_i (Sigma_d - K_i)
    bool live[K];
    uint32_t sc[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      const int64_t U = W * ((int64_t)ex[p] - (int64_t)kd) + Ki * rest;
      const int32_t c = (int32_t)key[p];
      live[p] = key[p] != EMPTY && key[p] != ud && key[p] != c0 && U > 0 &&
                (best < 0 || U > bestG || (U == bestG && c < best));
      sc[p] = a.Sig[live[p] ? c : d];
    }
    int reads = c0 != EMPTY;
#pragma unroll
    for (int p = 0; p < K; ++p) {
      consider_v<ALGO>(W, d, Ki, Sd, kd, (int32_t)key[p], ex[p], sc[p], live[p], best, bestG);
      reads += live[p];
    }
    return reads;
  }
}

template <int ALGO>
__device__ inline void finish(const SweepArgs &a, int32_t i, int32_t d, int32_t best, int64_t bestG,
                              Counters &ct) {
  int32_t target = d;
  if (ALGO == ALGO_LPA) {
    if (best >= 0) target = best;
  } else if (best >= 0) {
    ct.prop += 1;
    ct.sumG += (uint64_t)bestG;
    const int dir = a.gdir ? (int)a.gdir[a.gid[i]] : a.dir;
    bool ok = dir == 0 || (dir < 0 ? best < d : best > d);
    if (ok) target = best;
  }
  a.Cnew[i] = target;
  if (ALGO != ALGO_LPA && a.gain) a.gain[i] = best >= 0 ? bestG : 0;
  ct.moved += target != d;
  if (a.gctr) ct.g = a.gid[i];  // batched: added to the graph's counters when flushed
}

// Batched runs (all lanes of the wave): the lanes' counts go to their graphs'
// counters, one atomic per graph and counter for the whole wave (lanes grouped by
// graph, each group summed across the wave), then the counts restart.
__device__ inline void flush_graph_counters(const SweepArgs &a, Counters &ct) {
  const int lane = lane_id();
  uint64_t todo = __ballot(ct.moved != 0 || ct.prop != 0);  // a gain comes with a proposal
  while (todo) {  // wave-uniform
    const int leader = __builtin_ctzll(todo);
    const int32_t g = __shfl(ct.g, leader);
    const bool mine = ((todo >> lane) & 1ull) != 0 && ct.g == g;
    const unsigned long long m = wave_sum((unsigned long long)(mine ? ct.moved : 0u));
    const unsigned long long p = wave_sum((unsigned long long)(mine ? ct.prop : 0u));
    const unsigned long long sg = wave_sum((unsigned long long)(mine ? ct.sumG : 0ull));
    if (lane == leader) {
      unsigned long long *c = a.gctr + 3 * (int64_t)g;
      if (m) atomicAdd(&c[0], m);
      if (p) atomicAdd(&c[1], p);
      if (sg) atomicAdd(&c[2], sg);
    }
    todo &= ~__ballot(mine);
  }
  ct = Counters{};
}

// One thread's counts of one row, to its graph's counters (batched) or the sweep's.
__device__ inline void commit_counters(const SweepArgs &a, const Counters &ct) {
  unsigned long long *c = a.gctr ? a.gctr + 3 * (int64_t)ct.g : a.ctr;
  if (ct.moved) atomicAdd(&c[0], (unsigned long long)ct.moved);
  if (ct.prop) atomicAdd(&c[1], (unsigned long long)ct.prop);
  if (ct.sumG) atomicAdd(&c[2], (unsigned long long)ct.sumG);
}

__device__ inline void flush_counters(const SweepArgs &a, Counters ct) {
  if (a.gctr) {  // batched (kernel-uniform): per graph, per wave
    flush_graph_counters(a, ct);
    return;
  }
  __shared__ unsigned long long red[4][4];
  unsigned long long m = wave_sum((unsigned long long)ct.moved);
  unsigned long long p = wave_sum((unsigned long long)ct.prop);
  unsigned long long g = wave_sum((unsigned long long)ct.sumG);
  unsigned long long c = wave_sum((unsigned long long)ct.cand);
  int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    red[0][w] = m;
    red[1][w] = p;
    red[2][w] = g;
    red[3][w] = c;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    unsigned long long s = red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] +
                           red[threadIdx.x][3];
    if (s) atomicAdd(&a.ctr[threadIdx.x], s);
  }
}

// Key of entry (i -> j) in the stream of vertex i, or EMPTY when Algorithm 1's
// early exits skip it (self-loop; refinement across bounds).
template <int ALGO>
__device__ inline uint32_t stream_key(const SweepArgs &a, int32_t i, int32_t j, int32_t bi) {
  if (j == i) return EMPTY;
  if (ALGO == ALGO_REFINE) return a.bound[j] == bi ? (uint32_t)j : EMPTY;
  return a.ident ? (uint32_t)j : (uint32_t)a.C[j];
}

// Keys of U neighbours j (any valid ids): their communities C[j], or j itself when C is
// the identity; refinement keys are j when it shares the row's bound b[u], else EMPTY.
// One wave-uniform branch around all U reads keeps them in flight together.
template <int ALGO, int U>
__device__ inline void neighbour_keys(const SweepArgs &a, const int32_t (&j)[U], const int32_t (&b)[U],
                                      uint32_t (&c)[U]) {
  if (ALGO == ALGO_REFINE) {
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = a.bound[j[u]] == b[u] ? (uint32_t)j[u] : EMPTY;
  } else if (a.ident) {
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = (uint32_t)j[u];
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = (uint32_t)a.C[j[u]];
  }
}

// ---- MG: long rows -----------------------------------------------------------------

// Stage positions s0 .. s0+WIN-1 of every lane's chunk [clo, chi) of row i into the
// wave's LDS window (staging.hpp).  GATHER: the keys are C[j] (with Algorithm 1's
// skips), gathered with the loads of 8 rounds in flight, and are also written to the
// key stream; otherwise they are read from the key stream.  FUSED: each round reads its
// labels in its own step and ignores a.ident (the persistent batched kernel, whose
// graphs never start a sweep from the identity: measured 6 % faster there); otherwise
// the label reads of a group sit behind one branch on a.ident (the single-graph kernel,
// where this form also needs fewer registers: four waves per SIMD at k = 8 instead of
// three).
template <int ALGO, bool GATHER, bool FUSED = false>
__device__ inline void stage_window(const SweepArgs &a, uint32_t *win, int32_t i, int32_t bi,
                                    int64_t clo, int64_t chi, int64_t s0, uint32_t *keybuf) {
  if constexpr (!GATHER) {
    stage_pairs(win, clo, chi, s0, keybuf, a.g.w);
    return;
  }
  constexpr int G = WIN < 8 ? WIN : 8;  // rounds per group of loads in flight
  const int lane = lane_id();
#pragma unroll
  for (int g0 = 0; g0 < WIN; g0 += G) {
    uint32_t kk[G], ww[G];
    uint32_t ok = 0;
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const int src = (g0 + r) * SPR + lane / WIN;
      const int64_t e = __shfl(clo, src) + s0 + lane % WIN;
      const bool v = e < __shfl(chi, src);
      ok |= v ? 1u << r : 0u;
      const int64_t es = v ? e : 0;
      kk[r] = (uint32_t)__builtin_nontemporal_load(a.g.idx + es);
      ww[r] = __builtin_nontemporal_load(a.g.w + es);
    }
    if constexpr (FUSED) {
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int src = (g0 + r) * SPR + lane / WIN;
        const int32_t ii = __shfl(i, src);
        const int32_t bb = __shfl(bi, src);
        const bool v = (ok >> r) & 1u;
        const int32_t j = v ? (int32_t)kk[r] : 0;
        uint32_t c;
        if (ALGO == ALGO_REFINE)
          c = a.bound[j] == bb ? (uint32_t)j : EMPTY;
        else
          c = (uint32_t)a.C[j];
        // self-loops are skipped.  The gathered value is used on every lane (OR with
        // an all-ones mask instead of a select), so the compiler keeps the gathers of
        // all rounds in flight instead of sinking each into a branch of its own.
        kk[r] = c | ((v && j != ii) ? 0u : EMPTY);
      }
    } else {
      int32_t jj[G], bb[G];
      uint32_t c[G];
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int src = (g0 + r) * SPR + lane / WIN;
        jj[r] = ((ok >> r) & 1u) ? (int32_t)kk[r] : 0;
        bb[r] = ALGO == ALGO_REFINE ? __shfl(bi, src) : 0;
      }
      neighbour_keys<ALGO, G>(a, jj, bb, c);
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int src = (g0 + r) * SPR + lane / WIN;
        const int32_t ii = __shfl(i, src);
        const bool v = (ok >> r) & 1u;
        kk[r] = c[r] | ((v && jj[r] != ii) ? 0u : EMPTY);  // self-loops are skipped
      }
    }
    {
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const int src = (g0 + r) * SPR + lane / WIN;
        const int64_t e = __shfl(clo, src) + s0 + lane % WIN;
        if ((ok >> r) & 1u) keybuf[e] = kk[r];
      }
    }
#pragma unroll
    for (int r = 0; r < G; ++r) {
      const bool v = (ok >> r) & 1u;
      put_pair(win, (g0 + r) * SPR + lane / WIN, v ? kk[r] : EMPTY, v ? ww[r] : 0u);
    }
  }
}

// Pass 1 of Algorithm 1 over this lane's chunk [clo, chi) of row i: windows staged
// by stage_window, then every lane folds its own 16 staged entries into its VGPR
// sketch.  Every lane of the wave must call this; an idle lane passes an empty
// chunk.
template <int K, int ALGO, int MODE, bool GATHER = true, bool FUSED = false>
__device__ inline void staged_sketch(const SweepArgs &a, RegSketch<K, MODE> &s, uint32_t *win,
                                     int32_t i, int32_t bi, int64_t clo, int64_t chi,
                                     uint32_t *keybuf) {
  int64_t maxlen = chi - clo;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    int64_t x = __shfl_xor(maxlen, o);
    maxlen = x > maxlen ? x : maxlen;
  }
  for (int64_t s0 = 0; s0 < maxlen; s0 += WIN) {
    stage_window<ALGO, GATHER, FUSED>(a, win, i, bi, clo, chi, s0, keybuf);
    wave_sync();
    uint32_t kk[WIN], ww[WIN];
    read_window(win, kk, ww);
    wave_sync();
#pragma unroll
    for (int t = 0; t < WIN; ++t)
      if (kk[t] != EMPTY) s.update(kk[t], ww[t]);
  }
}

// Rows of more than 64 chunks ("long rows"): the main sweep kernel sketches their
// chunks, one wave per aligned group of 64 chunks (long_group), and merges each
// group with the first six levels of the fixed tree; then
//   k_long_merge   one workgroup per row: the rest of the fixed merge tree over its
//                  group roots; a row whose sketch lost no weight is decided here;
//   k_long_count   one wave per chunk of a lossy row: pass 2 against the row's
//                  candidates, partial counts per chunk;
//   k_long_decide  one workgroup per lossy row: sum the partial counts, decide.

// Chunk q of a long row: its row, its bounds and whether it is active.
struct LongChunk {
  int32_t m, i;
  int64_t lo, hi;
  bool active;
};

__device__ inline LongChunk long_chunk(const SweepArgs &a, const int32_t *multi,
                                       const int32_t *owner, const int64_t *cstart, int64_t q,
                                       int64_t nchunks, int64_t L) {
  LongChunk c{0, 0, 0, 0, false};
  if (q >= nchunks) return c;
  c.m = owner[q];
  c.i = multi[c.m];
  if (frozen(a, c.i)) return c;
  const int64_t rhi = a.g.off[c.i + 1];
  c.lo = a.g.off[c.i] + (q - cstart[c.m]) * L;
  c.hi = c.lo + L < rhi ? c.lo + L : rhi;
  c.active = true;
  return c;
}

// Wave w takes the aligned group of 64 chunks gstart[m] .. of its long row m (lane
// = chunk within the group): Algorithm 1 over the staged entries (keys gathered
// and written to the key stream), then the first six levels of the fixed merge
// tree with cross-lane shuffles; lane 0 writes the group's root.
template <int K, int ALGO, int MODE, bool FUSED = false>
__device__ __attribute__((always_inline)) inline void long_group(const SweepArgs &a, const Buckets &bk, int64_t L,
                                  uint32_t *keybuf, uint32_t *win, int64_t w) {
  const int lane = lane_id();
  const int32_t m = bk.gowner[w];
  const int32_t i = bk.multi[m];
  const int64_t nc = bk.cstart[m + 1] - bk.cstart[m];
  const int64_t q = (w - bk.gstart[m]) * WAVE + lane;  // chunk index within the row
  const bool active = q < nc && !frozen(a, i);
  int64_t lo = 0, hi = 0;
  if (active) {
    const int64_t rhi = a.g.off[i + 1];
    lo = a.g.off[i] + q * L;
    hi = lo + L < rhi ? lo + L : rhi;
  }
  const int32_t bi = (ALGO == ALGO_REFINE && active) ? a.bound[i] : 0;
  RegSketch<K, MODE> s;
  s.reset();
  staged_sketch<K, ALGO, MODE, true, FUSED>(a, s, win, i, bi, lo, hi, keybuf);
  s.finalize();
  bool lossy = s.lossy;
#pragma unroll 1
  for (int l = 0; l < 6; ++l) {
    const int stride = 1 << l;
    uint32_t bk_[K], bv_[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      bk_[p] = __shfl_down(s.key[p], stride);
      bv_[p] = __shfl_down(s.val[p], stride);
    }
    const int64_t c_l = (nc + stride - 1) >> l;  // nodes at level l
    const bool left = (lane & ((2 << l) - 1)) == 0;
    if (left && (q >> l) + 1 < c_l) lossy |= merge_sketch<K>(s.key, s.val, bk_, bv_);
  }
  const bool any = __ballot(lossy) != 0;
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < K; ++p)
      bk.sk[w * K + p] = Pair{s.val[p] > 0 ? s.key[p] : EMPTY, s.val[p]};
    bk.skflag[w] = any ? 1u : 0u;
  }
}

// Choose the best candidate of row i and record the move (one thread).
template <int K, int ALGO>
__device__ inline void decide_long(const SweepArgs &a, int32_t i, int32_t d, const uint32_t (&key)[K],
                                   const uint32_t (&ex)[K], uint32_t kd) {
  Counters ct;
  int32_t best = -1;
  int64_t bestG = 0;
  const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
  const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
  const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
  consider_slots<K, ALGO>(a, W, d, Ki, Sd, kd, key, ex, best, bestG);
  finish<ALGO>(a, i, d, best, bestG, ct);
  commit_counters(a, ct);
}

// cflag[m]: 0 decided here (exact sketch), 1 lossy (candidates in cand), 2 frozen.
template <int K, int ALGO>
__global__ void __launch_bounds__(BLOCK) MGCD_SKETCH_OCCUPANCY(K)
    k_long_merge(SweepArgs a, const int32_t *__restrict__ multi, const int64_t *__restrict__ gstart,
                 Pair *sk, const uint32_t *__restrict__ skflag, Pair *cand, uint32_t *cflag) {
  if (level_over(a)) return;  // batched: every graph has stopped
  __shared__ Pair lds[BLOCK * K];
  __shared__ int flag_any;
  const int t = threadIdx.x;
  const int32_t m = blockIdx.x;
  const int32_t i = multi[m];
  const int64_t cb = gstart[m], nc = gstart[m + 1] - cb;  // group roots of the row
  if (frozen(a, i)) {  // block-uniform
    if (t == 0) {
      a.Cnew[i] = community_of_self<ALGO>(a, i);
      cflag[m] = 2;
    }
    return;
  }
  if (t == 0) flag_any = 0;
  __syncthreads();
  bool f = false;
  for (int64_t q = t; q < nc; q += BLOCK) f |= skflag[cb + q] != 0;
  if (f) flag_any = 1;
  bool lossy = tree_reduce<K>(sk, cb, nc, lds);
  lossy |= flag_any != 0;  // settled by the barriers inside tree_reduce
  if (lossy && second_pass(a, ALGO)) {
    if (t < K) cand[(int64_t)m * K + t] = lds[t];
    if (t == 0) cflag[m] = 1;
    return;
  }
  if (t == 0) {
    cflag[m] = 0;
    uint32_t key[K], ex[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      const Pair x = lds[p];
      key[p] = x.val > 0 ? x.key : EMPTY;
      ex[p] = x.val;
    }
    const int32_t d = community_of_self<ALGO>(a, i);
    uint32_t kd = 0;
#pragma unroll
    for (int p = 0; p < K; ++p) kd += key[p] == (uint32_t)d ? ex[p] : 0u;
    decide_long<K, ALGO>(a, i, d, key, ex, kd);
  }
}

// part[q * (K + 1) + p] = weight of chunk q's entries with key cand[p];
// part[q * (K + 1) + K] = weight of those in the row's own community.
template <int K, int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_long_count(SweepArgs a, const int32_t *__restrict__ multi, const int32_t *__restrict__ owner,
                 const int64_t *__restrict__ cstart, int64_t nchunks, int64_t L,
                 const Pair *__restrict__ cand, const uint32_t *__restrict__ cflag,
                 const uint32_t *__restrict__ keybuf, uint32_t *part) {
  if (level_over(a)) return;  // batched: every graph has stopped
  const int64_t q = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE;  // wave-uniform
  if (q >= nchunks) return;
  const int32_t m = owner[q];
  if (cflag[m] != 1) return;
  const LongChunk c = long_chunk(a, multi, owner, cstart, q, nchunks, L);
  const int32_t d = community_of_self<ALGO>(a, c.i);
  uint32_t key[K], ex[K], kd = 0;
#pragma unroll
  for (int p = 0; p < K; ++p) {
    const Pair x = cand[(int64_t)m * K + p];
    key[p] = x.val > 0 ? x.key : EMPTY;
    ex[p] = 0;
  }
  int64_t e = c.lo + lane_id();
  for (; e + 3 * WAVE < c.hi; e += 4 * WAVE) {
    uint32_t cc[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) cc[u] = __builtin_nontemporal_load(keybuf + e + u * WAVE);
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = __builtin_nontemporal_load(a.g.w + e + u * WAVE);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int p = 0; p < K; ++p) ex[p] += key[p] == cc[u] ? w[u] : 0u;
      kd += cc[u] == (uint32_t)d ? w[u] : 0u;
    }
  }
  for (; e < c.hi; e += WAVE) {
    const uint32_t cc = keybuf[e], w = a.g.w[e];
#pragma unroll
    for (int p = 0; p < K; ++p) ex[p] += key[p] == cc ? w : 0u;
    kd += cc == (uint32_t)d ? w : 0u;
  }
#pragma unroll
  for (int p = 0; p < K; ++p) ex[p] = wave_sum(ex[p]);
  kd = wave_sum(kd);
  const int l = lane_id();
  uint32_t mine = kd;
#pragma unroll
  for (int p = 0; p < K; ++p) mine = l == p ? ex[p] : mine;
  if (l <= K) part[q * (K + 1) + l] = mine;
}

template <int K, int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_long_decide(SweepArgs a, const int32_t *__restrict__ multi, const int64_t *__restrict__ cstart,
                  const Pair *__restrict__ cand, const uint32_t *__restrict__ cflag,
                  const uint32_t *__restrict__ part) {
  if (level_over(a)) return;  // batched: every graph has stopped
  __shared__ uint32_t red[K + 1][BLOCK / WAVE];
  const int32_t m = blockIdx.x;
  if (cflag[m] != 1) return;  // block-uniform
  const int t = threadIdx.x;
  const int64_t cb = cstart[m], ce = cstart[m + 1];
  uint32_t sum[K + 1];
#pragma unroll
  for (int p = 0; p <= K; ++p) sum[p] = 0;
  for (int64_t q = cb + t; q < ce; q += BLOCK) {
#pragma unroll
    for (int p = 0; p <= K; ++p) sum[p] += part[q * (K + 1) + p];
  }
#pragma unroll
  for (int p = 0; p <= K; ++p) {
    const uint32_t v = wave_sum(sum[p]);
    if (lane_id() == 0) red[p][t / WAVE] = v;
  }
  __syncthreads();
  if (t != 0) return;
  const int32_t i = multi[m];
  uint32_t key[K], ex[K];
#pragma unroll
  for (int p = 0; p < K; ++p) {
    const Pair x = cand[(int64_t)m * K + p];
    key[p] = x.val > 0 ? x.key : EMPTY;
    ex[p] = red[p][0] + red[p][1] + red[p][2] + red[p][3];
  }
  const uint32_t kd = red[K][0] + red[K][1] + red[K][2] + red[K][3];
  decide_long<K, ALGO>(a, i, community_of_self<ALGO>(a, i), key, ex, kd);
}

// ---- MG: every row of at most 64 chunks, one launch ---------------------------------

// Rows are grouped in buckets by P = 2^b lanes per row (P >= the row's chunk count;
// b = 0 for rows of one chunk), 64/P rows per wave, heaviest bucket first in the
// grid.  Lane q of a row owns chunk q.
//   pass 1: staged_sketch over the lane's chunk (keys also go to the key stream);
//   merge:  chunk sketches merged by the fixed tree with cross-lane shuffles (node
//           j of level l lives in lane j*2^l, its right partner 2^l lanes up);
//   pass 2: only rows whose sketch lost weight: the same LDS windows over the key
//           stream (no second gather) and the weights, each lane counting its own
//           chunk, then xor-shuffles inside the row's aligned segment;
//   lane 0 of the segment decides.
template <int K, int ALGO, int MODE, bool FUSED = false>
__device__ __attribute__((always_inline)) inline void row_work(const SweepArgs &a, const Buckets &bk, int64_t L, uint32_t *keybuf,
                                uint32_t *win, int64_t wave, Counters &ct) {
  const int lane = lane_id();
  // buckets are laid out in the grid from b = 6 down to b = 0 (wave-uniform)
  int b = 6;
  while (b > 0 && wave >= bk.wave_end[b]) --b;
  const int logp = b;
  const int P = 1 << logp;
  const int q = lane & (P - 1);
  const int base_lane = lane & ~(P - 1);
  const int64_t r = (wave - bk.wave_begin[b]) * (WAVE >> logp) + (lane >> logp);
  const bool listed = wave < bk.wave_end[0] && r < bk.nrows[b];
  const int32_t i = listed ? bk.rows[b][r] : 0;
  const bool valid = listed && !frozen(a, i);
  if (listed && !valid && q == 0) a.Cnew[i] = community_of_self<ALGO>(a, i);
  const int64_t lo = valid ? a.g.off[i] : 0, hi = valid ? a.g.off[i + 1] : 0;
  const int64_t nc = (hi - lo + L - 1) / L;
  const int32_t bi = (ALGO == ALGO_REFINE && valid) ? a.bound[i] : 0;
  // this lane's chunk [clo, chi)
  const int64_t clo = lo + q * L;
  const int64_t chi = q < nc ? (clo + L < hi ? clo + L : hi) : clo;
  RegSketch<K, MODE> s;
  s.reset();
  staged_sketch<K, ALGO, MODE, true, FUSED>(a, s, win, i, bi, clo, chi, keybuf);
  s.finalize();
  bool lossy = s.lossy;
  for (int l = 0; l < logp; ++l) {
    const int stride = 1 << l;
    uint32_t bk_[K], bv_[K];
#pragma unroll
    for (int p = 0; p < K; ++p) {
      bk_[p] = __shfl_down(s.key[p], stride);
      bv_[p] = __shfl_down(s.val[p], stride);
    }
    const int64_t c_l = (nc + stride - 1) >> l;  // nodes at level l
    const bool left = (q & ((2 << l) - 1)) == 0;
    if (left && (int64_t)(q >> l) + 1 < c_l) lossy |= merge_sketch<K>(s.key, s.val, bk_, bv_);
  }
  uint32_t key[K], ex[K];
#pragma unroll
  for (int p = 0; p < K; ++p) {
    uint32_t kk = __shfl(s.key[p], base_lane);
    uint32_t vv = __shfl(s.val[p], base_lane);
    key[p] = vv > 0 ? kk : EMPTY;
    ex[p] = vv;
  }
  const uint64_t lm = __ballot(lossy);
  const uint64_t seg = P == 64 ? lm : (lm >> base_lane) & ((1ull << P) - 1);
  const int32_t d = valid ? community_of_self<ALGO>(a, i) : 0;
  uint32_t kd = 0;
  const bool need2 = seg != 0 && second_pass(a, ALGO);  // same for all lanes of a row
  if (!need2) {
#pragma unroll
    for (int p = 0; p < K; ++p) kd += key[p] == (uint32_t)d ? ex[p] : 0u;
  } else {
#pragma unroll
    for (int p = 0; p < K; ++p) ex[p] = 0;
  }
  // pass 2 over the stashed keys (no second gather), staged like pass 1; rows whose
  // sketch was exact take no part
  const int64_t chi2 = need2 ? chi : clo;
  int64_t maxlen2 = chi2 - clo;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    int64_t x = __shfl_xor(maxlen2, o);
    maxlen2 = x > maxlen2 ? x : maxlen2;
  }
  for (int64_t s0 = 0; s0 < maxlen2; s0 += WIN) {
    stage_window<ALGO, false>(a, win, i, bi, clo, chi2, s0, keybuf);
    wave_sync();
    uint32_t kk[WIN], ww[WIN];
    read_window(win, kk, ww);
    wave_sync();
#pragma unroll
    for (int t = 0; t < WIN; ++t) {
      const uint32_t c = kk[t], w = ww[t];
#pragma unroll
      for (int p = 0; p < K; ++p) ex[p] += key[p] == c ? w : 0u;
      kd += c == (uint32_t)d ? w : 0u;
    }
  }
  if (maxlen2 > 0) {
    for (int o = P / 2; o > 0; o >>= 1) {
#pragma unroll
      for (int p = 0; p < K; ++p) {
        const uint32_t x = __shfl_xor(ex[p], o);
        ex[p] += need2 ? x : 0u;
      }
      const uint32_t x = __shfl_xor(kd, o);
      kd += need2 ? x : 0u;
    }
  }
  if (valid && q == 0) {
    int32_t best = -1;
    int64_t bestG = 0;
    const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
    const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
    const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
    ct.cand += consider_slots<K, ALGO>(a, W, d, Ki, Sd, kd, key, ex, best, bestG);
    finish<ALGO>(a, i, d, best, bestG, ct);
  }
}

// The main sweep kernel: the first bk.ngroups waves sketch the groups of 64 chunks
// of long rows (their merge, pass 2 and decision follow in k_long_*), the rest
// take the row buckets.
template <int K, int ALGO, int MODE, bool PERSIST>
__global__ void __launch_bounds__(BLOCK) MGCD_ROWS_OCCUPANCY(K)
    k_move_rows(SweepArgs a, const Buckets bk, int64_t L, uint32_t *keybuf) {
  __shared__ __attribute__((aligned(16))) uint32_t swin[BLOCK / WAVE][WAVE * WROW];
  uint32_t *const win = swin[threadIdx.x / WAVE];
  if constexpr (!PERSIST) {
    const int64_t wave = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE;  // wave-uniform
    Counters ct;
    if (wave < bk.ngroups)
      long_group<K, ALGO, MODE>(a, bk, L, keybuf, win, wave);
    else
      row_work<K, ALGO, MODE>(a, bk, L, keybuf, win, wave - bk.ngroups, ct);
    flush_counters(a, ct);
  } else {
    // persistent (batched runs): every wave takes work items from its counter of the
    // queue (the items of the grid's order -- long-row groups, then the row buckets
    // heaviest first -- whose index is c mod QLANES), QGRAB at a time, until none is
    // left; nothing at all once every graph has stopped
    if (level_over(a)) return;
    Counters ct;
    const int64_t total = bk.ngroups + bk.wave_end[0];
    const int c = (int)(((int64_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE) % QLANES);
    unsigned long long *q = a.queue + (int64_t)c * QSTRIDE;
    for (;;) {
      unsigned long long j0 = 0;
      if (lane_id() == 0) j0 = atomicAdd(q, (unsigned long long)QGRAB);
      const int64_t j = uniform((int64_t)__shfl(j0, 0));
      if (c + j * QLANES >= total) break;
#pragma unroll 1
      for (int t = 0; t < QGRAB; ++t) {
        const int64_t wave = c + (j + t) * QLANES;  // wave-uniform
        if (wave >= total) break;
        if (wave < bk.ngroups) {
          long_group<K, ALGO, MODE, true>(a, bk, L, keybuf, win, wave);
        } else {
          row_work<K, ALGO, MODE, true>(a, bk, L, keybuf, win, wave - bk.ngroups, ct);
          if (a.gctr) flush_graph_counters(a, ct);  // the next item's rows may be another graph's
        }
      }
    }
    flush_counters(a, ct);
  }
}

// ---- MG with K = 32 or 64: one wave per row -------------------------------------------

// Rows longer than 32 entries when K is 32 or 64 (shorter rows cannot lose weight
// under Algorithm 1 or the textbook rule and take the exact one-lane kernel).  One
// wave per row holds a WaveSketch (slot p in lane p).  Pass 1: the row is loaded 64
// entries at a time (coalesced index and weight loads, 64 label gathers in flight,
// keys written to the key stream) and folded in stream order, one wave-uniform item
// at a time; every L positions the chunk sketch goes into the fixed merge tree
// (WaveTree).  Pass 2 (lossy rows only): the key stream again, each item added to the
// lane whose candidate matches.  Decision: every lane scores its candidate, a
// butterfly keeps the best (lowest id on ties), lane 0 records it.
template <int K, int ALGO, int MODE, int DEPTH>
__global__ void __launch_bounds__(BLOCK)
    k_wave_rows(SweepArgs a, const int32_t *__restrict__ rows, int64_t nrows, int64_t L,
                uint32_t *keybuf) {
  static_assert(K <= WAVE, "one slot per lane; larger sketches take the split rows");
  if (level_over(a)) return;  // batched: every graph has stopped
  __shared__ uint32_t sstack[BLOCK / WAVE][DEPTH * 2 * WAVE];
  const int lane = lane_id();
  const int64_t r = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  Counters ct;
  const bool listed = r < nrows;
  const int32_t i = listed ? uniform(rows[r]) : 0;
  const bool valid = listed && !frozen(a, i);
  if (listed && !valid && lane == 0) a.Cnew[i] = community_of_self<ALGO>(a, i);
  if (valid) {
    const int64_t lo = uniform(a.g.off[i]), hi = uniform(a.g.off[i + 1]);
    const int32_t bi = ALGO == ALGO_REFINE ? uniform(a.bound[i]) : 0;
    const int32_t d = uniform(community_of_self<ALGO>(a, i));
    WaveSketch<K, MODE> s;
    s.reset();
    WaveTree<K, DEPTH> tree{sstack[threadIdx.x / WAVE]};
    bool lossy = false;
    int64_t left = L;  // positions left in the current chunk
    for (int64_t e0 = lo; e0 < hi; e0 += WAVE) {
      const int64_t e = e0 + lane;
      const bool v = e < hi;
      const int32_t j = v ? __builtin_nontemporal_load(a.g.idx + e) : 0;
      const uint32_t w = v ? __builtin_nontemporal_load(a.g.w + e) : 0u;
      uint32_t key = EMPTY;
      if (v) {
        key = stream_key<ALGO>(a, i, j, bi);
        keybuf[e] = key;
      }
      const int nb = hi - e0 < WAVE ? (int)(hi - e0) : WAVE;
      for (int t = 0; t < nb; ++t) {
        const uint32_t c = lane_value(key, t);
        if (c != EMPTY) s.update(c, lane_value(w, t));
        if (--left == 0) {  // end of a chunk
          lossy |= s.lossy;
          s.finalize();
          tree.push(s.key[0], s.val[0]);
          s.reset();
          left = L;
        }
      }
    }
    if (left != L) {  // the last, partial chunk
      lossy |= s.lossy;
      s.finalize();
      tree.push(s.key[0], s.val[0]);
    }
    uint32_t ck, cv;
    tree.result(ck, cv);
    lossy |= tree.lossy;
    uint32_t kd = 0;
    if (!lossy || !second_pass(a, ALGO)) {
      kd = wave_sum(ck == (uint32_t)d ? cv : 0u);
    } else {
      cv = 0;
      for (int64_t e0 = lo; e0 < hi; e0 += WAVE) {
        const int64_t e = e0 + lane;
        const bool v = e < hi;
        const uint32_t key = v ? __builtin_nontemporal_load(keybuf + e) : EMPTY;
        const uint32_t w = v ? __builtin_nontemporal_load(a.g.w + e) : 0u;
        kd += key == (uint32_t)d ? w : 0u;
        const int nb = hi - e0 < WAVE ? (int)(hi - e0) : WAVE;
        for (int t = 0; t < nb; ++t) {
          const uint32_t c = lane_value(key, t);
          if (c != EMPTY && ck == c) cv += lane_value(w, t);
        }
      }
      kd = wave_sum(kd);
    }
    int32_t best = -1;
    int64_t bestG = 0;
    if (ck != EMPTY) {
      const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
      const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
      const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
      consider<ALGO>(a, W, d, Ki, Sd, kd, (int32_t)ck, cv, best, bestG);
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const int32_t b2 = __shfl_xor(best, o);
      const int64_t g2 = __shfl_xor(bestG, o);
      if (b2 >= 0 && (best < 0 || g2 > bestG || (g2 == bestG && b2 < best))) {
        best = b2;
        bestG = g2;
      }
    }
    if (lane == 0) finish<ALGO>(a, i, d, best, bestG, ct);
  }
  flush_counters(a, ct);
}

// Rows of more than max(L, WAVE_SPLIT) entries when K is 32 or 64 ("split rows"): the
// same sketch, merge tree and decision as k_wave_rows, with the work spread over waves
// so that a hub row does not hold one wave for its whole length.
//   k_wave_chunks: one wave per chunk: its Algorithm 1 sketch (keys written to the key
//                  stream), finalised, into the chunk's node;
//   k_wave_level:  one launch per tree level l: node x of a row (x a multiple of
//                  2^(l+1)) takes in node x + 2^l if that exists, left operand first,
//                  an odd last node is carried; after ceil(log2(chunks)) levels node 0
//                  is the root, the same tree as WaveTree;
//   k_wave_count:  pass 2 of lossy rows, one wave per chunk, integer sums added into
//                  the row's counts (order-independent);
//   k_wave_decide: one wave per row: scores and the decision, as in k_wave_rows.
template <int K, int ALGO, int MODE>
__global__ void __launch_bounds__(BLOCK)
    k_wave_chunks(SweepArgs a, const int32_t *__restrict__ rows, const int64_t *__restrict__ cstart,
                  const int32_t *__restrict__ owner, int64_t nchunks, int64_t L, uint32_t *keybuf,
                  Pair *node, uint32_t *nflag, uint32_t *count) {
  if (level_over(a)) return;  // batched: every graph has stopped
  const int lane = lane_id();
  const int64_t q = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  if (q >= nchunks) return;
  const int32_t m = uniform(owner[q]);
  const int32_t i = uniform(rows[m]);
  if (q == cstart[m]) {  // the row's K + 1 pass-2 counts start at zero in every sweep
    uint32_t *cm = count + (int64_t)m * (K + 1);
    for (int p = lane; p <= K; p += WAVE) cm[p] = 0u;
  }
  if (frozen(a, i)) return;
  const int64_t rhi = uniform(a.g.off[i + 1]);
  const int64_t lo = uniform(a.g.off[i]) + (q - cstart[m]) * L;
  const int64_t hi = lo + L < rhi ? lo + L : rhi;
  const int32_t bi = ALGO == ALGO_REFINE ? uniform(a.bound[i]) : 0;
  WaveSketch<K, MODE> s;
  s.reset();
  for (int64_t e0 = lo; e0 < hi; e0 += WAVE) {
    const int64_t e = e0 + lane;
    const bool v = e < hi;
    const int32_t j = v ? __builtin_nontemporal_load(a.g.idx + e) : 0;
    const uint32_t w = v ? __builtin_nontemporal_load(a.g.w + e) : 0u;
    uint32_t key = EMPTY;
    if (v) {
      key = stream_key<ALGO>(a, i, j, bi);
      keybuf[e] = key;
    }
    const int nb = hi - e0 < WAVE ? (int)(hi - e0) : WAVE;
    for (int t = 0; t < nb; ++t) {
      const uint32_t c = lane_value(key, t);
      if (c != EMPTY) s.update(c, lane_value(w, t));
    }
  }
  s.finalize();
#pragma unroll
  for (int r = 0; r < WaveSlots<K>::S; ++r)
    if (r * WAVE + lane < K) node[q * K + r * WAVE + lane] = Pair{s.key[r], s.val[r]};
  if (lane == 0) nflag[q] = s.lossy ? 1u : 0u;
}

template <int K>
__global__ void __launch_bounds__(BLOCK)
    k_wave_level(SweepArgs a, const int32_t *__restrict__ rows, const int64_t *__restrict__ cstart,
                 const int32_t *__restrict__ owner, int64_t nchunks, int level, Pair *node,
                 uint32_t *nflag) {
  if (level_over(a)) return;  // batched: every graph has stopped
  const int lane = lane_id();
  const int64_t q = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  if (q >= nchunks) return;
  const int32_t m = uniform(owner[q]);
  const int64_t x = q - cstart[m], half = (int64_t)1 << level;
  if ((x & (2 * half - 1)) != 0) return;  // not a left node of this level
  const int64_t r = q + half;
  if (r >= cstart[m + 1]) return;  // odd last node: carried up
  if (frozen(a, rows[m])) return;
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
      const Pair pa = node[q * K + p], pb = node[r * K + p];
      ak[u] = pa.key;
      av[u] = pa.val;
      bk[u] = pb.key;
      bv[u] = pb.val;
    }
  }
  const bool lossy = wave_merge<K>(ak, av, bk, bv);
#pragma unroll
  for (int u = 0; u < S; ++u)
    if (u * WAVE + lane < K) node[q * K + u * WAVE + lane] = Pair{ak[u], av[u]};
  if (lane == 0) nflag[q] = nflag[q] | nflag[r] | (lossy ? 1u : 0u);
}

// The root of split row m: keys of positive slots, other slots EMPTY.
template <int K, int S = WaveSlots<K>::S>
__device__ inline void wave_root(const Pair *node, const int64_t *cstart, int32_t m, uint32_t (&ck)[S],
                                 uint32_t (&cv)[S]) {
  const int lane = lane_id();
#pragma unroll
  for (int u = 0; u < S; ++u) {
    ck[u] = EMPTY;
    cv[u] = 0;
    if (u * WAVE + lane < K) {
      const Pair p = node[cstart[m] * K + u * WAVE + lane];
      ck[u] = p.val > 0 ? p.key : EMPTY;
      cv[u] = p.val;
    }
  }
}

template <int K, int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_wave_count(SweepArgs a, const int32_t *__restrict__ rows, const int64_t *__restrict__ cstart,
                 const int32_t *__restrict__ owner, int64_t nchunks, int64_t L,
                 const uint32_t *__restrict__ keybuf, const Pair *__restrict__ node,
                 const uint32_t *__restrict__ nflag, uint32_t *count) {
  if (level_over(a)) return;  // batched: every graph has stopped
  const int lane = lane_id();
  const int64_t q = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  if (q >= nchunks) return;
  const int32_t m = uniform(owner[q]);
  const int32_t i = uniform(rows[m]);
  if (frozen(a, i) || !nflag[cstart[m]]) return;
  const int64_t rhi = uniform(a.g.off[i + 1]);
  const int64_t lo = uniform(a.g.off[i]) + (q - cstart[m]) * L;
  const int64_t hi = lo + L < rhi ? lo + L : rhi;
  const uint32_t d = (uint32_t)uniform(community_of_self<ALGO>(a, i));
  constexpr int S = WaveSlots<K>::S;
  uint32_t ck[S], cv0[S], cv[S];
  wave_root<K>(node, cstart, m, ck, cv0);
#pragma unroll
  for (int u = 0; u < S; ++u) cv[u] = 0;
  uint32_t kd = 0;
  for (int64_t e0 = lo; e0 < hi; e0 += WAVE) {
    const int64_t e = e0 + lane;
    const bool v = e < hi;
    const uint32_t key = v ? __builtin_nontemporal_load(keybuf + e) : EMPTY;
    const uint32_t w = v ? __builtin_nontemporal_load(a.g.w + e) : 0u;
    kd += key == d ? w : 0u;
    const int nb = hi - e0 < WAVE ? (int)(hi - e0) : WAVE;
    for (int t = 0; t < nb; ++t) {
      const uint32_t c = lane_value(key, t);
      const uint32_t wt = lane_value(w, t);
#pragma unroll
      for (int u = 0; u < S; ++u)
        if (c != EMPTY && ck[u] == c) cv[u] += wt;
    }
  }
  kd = wave_sum(kd);
  uint32_t *cm = count + (int64_t)m * (K + 1);
#pragma unroll
  for (int u = 0; u < S; ++u)
    if (u * WAVE + lane < K && cv[u]) atomicAdd(&cm[u * WAVE + lane], cv[u]);
  if (lane == 0 && kd) atomicAdd(&cm[K], kd);
}

template <int K, int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_wave_decide(SweepArgs a, const int32_t *__restrict__ rows, const int64_t *__restrict__ cstart,
                  int64_t nrows, const Pair *__restrict__ node, const uint32_t *__restrict__ nflag,
                  const uint32_t *__restrict__ count) {
  if (level_over(a)) return;  // batched: every graph has stopped
  const int lane = lane_id();
  const int64_t m = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  Counters ct;
  if (m < nrows) {
    const int32_t i = uniform(rows[m]);
    if (frozen(a, i)) {
      if (lane == 0) a.Cnew[i] = community_of_self<ALGO>(a, i);
    } else {
      const int32_t d = uniform(community_of_self<ALGO>(a, i));
      constexpr int S = WaveSlots<K>::S;
      uint32_t ck[S], cv[S];
      wave_root<K>(node, cstart, (int32_t)m, ck, cv);
      uint32_t kd;
      if (!nflag[cstart[m]] || !second_pass(a, ALGO)) {
        uint32_t own = 0;
#pragma unroll
        for (int u = 0; u < S; ++u) own += ck[u] == (uint32_t)d ? cv[u] : 0u;
        kd = wave_sum(own);
      } else {
        const uint32_t *cm = count + m * (K + 1);
#pragma unroll
        for (int u = 0; u < S; ++u) cv[u] = u * WAVE + lane < K ? cm[u * WAVE + lane] : 0u;
        kd = cm[K];
      }
      int32_t best = -1;
      int64_t bestG = 0;
      const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
      const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
      const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
#pragma unroll
      for (int u = 0; u < S; ++u)
        if (ck[u] != EMPTY) consider<ALGO>(a, W, d, Ki, Sd, kd, (int32_t)ck[u], cv[u], best, bestG);
#pragma unroll
      for (int o = WAVE / 2; o > 0; o >>= 1) {
        const int32_t b2 = __shfl_xor(best, o);
        const int64_t g2 = __shfl_xor(bestG, o);
        if (b2 >= 0 && (best < 0 || g2 > bestG || (g2 == bestG && b2 < best))) {
          best = b2;
          bestG = g2;
        }
      }
      if (lane == 0) finish<ALGO>(a, i, d, best, bestG, ct);
    }
  }
  flush_counters(a, ct);
}

// ---- exact mode ----------------------------------------------------------------------

// A row of at most ES entries: keys and weights gathered once into registers, then
// every distinct key summed at its first occurrence (static indices, unrolled).
template <int ALGO, int ES>
__device__ inline void exact_row_regs(const SweepArgs &a, int32_t i, int32_t bi, int64_t lo,
                                      int64_t hi, int32_t d, Counters &ct) {
  // Every load is issued on every lane (an absent position reads a valid entry: the
  // row's first, or entry 0 for an empty row; some row of the wave is non-empty) and
  // its value masked afterwards, so the loads and gathers of all positions are in
  // flight together.
  uint32_t ks[ES], ws[ES];
  const int64_t safe = hi > lo ? lo : 0;
#pragma unroll
  for (int t = 0; t < ES; ++t) {
    const bool v = lo + t < hi;
    const int64_t e = v ? lo + t : safe;
    const int32_t j = a.g.idx[e];
    ws[t] = a.g.w[e] & (v ? ~0u : 0u);
    uint32_t c;
    if (ALGO == ALGO_REFINE)
      c = a.bound[j] == bi ? (uint32_t)j : EMPTY;
    else
      c = (uint32_t)a.C[j];
    ks[t] = c | ((v && j != i) ? 0u : EMPTY);  // self-loops are skipped
  }
  // table keys: the keys themselves, or their slots in the small table (a slot's
  // first key stands for it, K_{i->d} is the sum in d's slot)
  uint32_t ss[ES];
#pragma unroll
  for (int t = 0; t < ES; ++t) ss[t] = ks[t] != EMPTY ? slot_of(a, ks[t]) : EMPTY;
  const uint32_t sd = slot_of(a, (uint32_t)d);
  uint32_t kd = 0;
#pragma unroll
  for (int t = 0; t < ES; ++t) kd += ss[t] == sd ? ws[t] : 0u;
  int32_t best = -1;
  int64_t bestG = 0;
  const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
  const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
  const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
  uint32_t sc[ES];
#pragma unroll
  for (int t = 0; t < ES; ++t) sc[t] = ALGO == ALGO_LPA ? 0u : a.Sig[ks[t] != EMPTY ? (int32_t)ks[t] : d];
#pragma unroll
  for (int t = 0; t < ES; ++t) {
    const uint32_t c = ks[t];
    bool first = c != EMPTY;
#pragma unroll
    for (int u = 0; u < t; ++u) first &= ss[u] != ss[t];
    uint32_t kc = 0;
#pragma unroll
    for (int u = t; u < ES; ++u) kc += ss[u] == ss[t] ? ws[u] : 0u;
    consider_v<ALGO>(W, d, Ki, Sd, kd, (int32_t)c, kc, sc[t], first, best, bestG);
  }
  finish<ALGO>(a, i, d, best, bestG, ct);
}

// Exact mode, the shortest rows (tier 0): one lane per vertex; K_{i->c} of each
// distinct key, summed at its first occurrence in the row.  Rows of at most 32
// entries keep the row in registers (the unroll depth, 2 to 32, follows the longest
// row of the wave); longer tier-0 rows (a raised exact_small) re-read the row.
template <int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_exact_small(SweepArgs a, const int32_t *__restrict__ list, int64_t count) {
  if (level_over(a)) return;  // batched: every graph has stopped
  Counters ct;
  int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool listed = t < count;
  const int32_t i = listed ? list[t] : 0;
  const bool live = listed && !frozen(a, i);
  if (listed && !live) a.Cnew[i] = community_of_self<ALGO>(a, i);
  const int64_t lo = live ? a.g.off[i] : 0, hi = live ? a.g.off[i + 1] : 0;
  int64_t maxdeg = hi - lo;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int64_t x = __shfl_xor(maxdeg, o);
    maxdeg = x > maxdeg ? x : maxdeg;
  }
  maxdeg = uniform(maxdeg);
  const int32_t bi = (ALGO == ALGO_REFINE && live) ? a.bound[i] : 0;
  const int32_t d = live ? community_of_self<ALGO>(a, i) : 0;
  if (maxdeg == 0) {
    if (live) finish<ALGO>(a, i, d, -1, 0, ct);  // no neighbours: stay
  } else if (maxdeg <= 2) {
    if (live) exact_row_regs<ALGO, 2>(a, i, bi, lo, hi, d, ct);
  } else if (maxdeg <= 4) {
    if (live) exact_row_regs<ALGO, 4>(a, i, bi, lo, hi, d, ct);
  } else if (maxdeg <= 8) {
    if (live) exact_row_regs<ALGO, 8>(a, i, bi, lo, hi, d, ct);
  } else if (maxdeg <= 16) {
    if (live) exact_row_regs<ALGO, 16>(a, i, bi, lo, hi, d, ct);
  } else if (maxdeg <= 32) {
    if (live) exact_row_regs<ALGO, 32>(a, i, bi, lo, hi, d, ct);
  } else if (live) {
    // table key of entry f (EMPTY when Algorithm 1's skips drop it)
    auto tkey = [&](int64_t f) {
      const uint32_t c = stream_key<ALGO>(a, i, a.g.idx[f], bi);
      return c != EMPTY ? slot_of(a, c) : EMPTY;
    };
    const uint32_t sd = slot_of(a, (uint32_t)d);
    uint32_t kd = 0;
    for (int64_t e = lo; e < hi; ++e) kd += tkey(e) == sd ? a.g.w[e] : 0u;
    int32_t best = -1;
    int64_t bestG = 0;
    const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
    const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
    const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
    for (int64_t e = lo; e < hi; ++e) {
      const uint32_t c = stream_key<ALGO>(a, i, a.g.idx[e], bi);
      if (c == EMPTY) continue;
      const uint32_t se = slot_of(a, c);
      bool first = true;
      for (int64_t f = lo; f < e && first; ++f) first = tkey(f) != se;
      if (!first) continue;
      uint32_t kc = 0;
      for (int64_t f = e; f < hi; ++f) kc += tkey(f) == se ? a.g.w[f] : 0u;
      consider<ALGO>(a, W, d, Ki, Sd, kd, (int32_t)c, kc, best, bestG);
    }
    finish<ALGO>(a, i, d, best, bestG, ct);
  }
  flush_counters(a, ct);
}

__device__ inline uint32_t hash_slot(uint32_t c, uint32_t mask) {
  return (c * 0x9E3779B1u) & mask;  // Fibonacci hashing, low bits
}

// Exact mode, tier 1 (rows of up to EXACT_T1_MAX entries): one wave per row with an
// LDS open-addressing table of its own, sized to the row (the smallest power of two
// >= 2 * its length, 64 .. 1024 slots), so a block holds four rows instead of one.
// Same table keys, sums, first positions (small table) and decision as k_exact_table.
template <int ALGO, bool SMALL = false>
__global__ void __launch_bounds__(BLOCK)
    k_exact_wave(SweepArgs a, const int32_t *__restrict__ list, int64_t count) {
  if (level_over(a)) return;  // batched: every graph has stopped
  constexpr uint32_t CAPW = 2 * EXACT_T1_MAX;
  __shared__ Pair wtab[BLOCK / WAVE][CAPW];
  __shared__ uint32_t wpos[BLOCK / WAVE][SMALL ? CAPW : 1];
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  const int64_t r = uniform(((int64_t)blockIdx.x * BLOCK + threadIdx.x) / WAVE);
  Counters ct;
  if (r < count) {
    const int32_t i = uniform(list[r]);
    if (frozen(a, i)) {
      if (lane == 0) a.Cnew[i] = community_of_self<ALGO>(a, i);
    } else {
      const int64_t lo = a.g.off[i], hi = a.g.off[i + 1];
      uint32_t cap = 64;
      while (cap < CAPW && (int64_t)cap < 2 * (hi - lo)) cap <<= 1;
      Pair *tab = wtab[w];
      uint32_t *pos = wpos[w];
      for (uint32_t x = lane; x < cap; x += WAVE) {
        tab[x] = Pair{EMPTY, 0u};
        if (SMALL) pos[x] = 0xFFFFFFFFu;
      }
      wave_sync();
      const int32_t bi = ALGO == ALGO_REFINE ? a.bound[i] : 0;
      const uint32_t mask = cap - 1;
      for (int64_t e0 = lo; e0 < hi; e0 += WAVE) {  // wave-uniform rounds
        const int64_t e = e0 + lane;
        const bool v = e < hi;
        uint32_t c = v ? stream_key<ALGO>(a, i, a.g.idx[e], bi) : EMPTY;
        if (c != EMPTY) c = slot_of(a, c);
        uint32_t w = v ? a.g.w[e] : 0u;
        // the lanes holding the first live lane's key add their weights into that lane
        // (one table update instead of one per lane, which serialise on the slot of a
        // community that many neighbours share; the lane is the group's first position)
        const uint64_t lm = __ballot(c != EMPTY);
        if (lm) {
          const int ld = __builtin_ctzll(lm);
          const uint32_t ck = lane_value(c, ld);
          const bool m = c == ck;
          if (__popcll(__ballot(m)) > 1) {
            const uint32_t sum = wave_sum(m ? w : 0u);
            if (lane == ld)
              w = sum;
            else if (m)
              c = EMPTY;
          }
        }
        if (c == EMPTY) continue;
        uint32_t h = hash_slot(c, mask);
        while (true) {
          const uint32_t prev = atomicCAS(&tab[h].key, EMPTY, c);
          if (prev == EMPTY || prev == c) {
            atomicAdd(&tab[h].val, w);
            if (SMALL) atomicMin(&pos[h], (uint32_t)(e - lo));
            break;
          }
          h = (h + 1) & mask;
        }
      }
      wave_sync();
      const int32_t d = community_of_self<ALGO>(a, i);
      const uint32_t sd = slot_of(a, (uint32_t)d);
      uint32_t kd = 0;
      for (uint32_t x = lane; x < cap; x += WAVE) kd += tab[x].key == sd ? tab[x].val : 0u;
      kd = wave_sum(kd);
      int32_t best = -1;
      int64_t bestG = 0;
      const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
      const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
      const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
      for (uint32_t x = lane; x < cap; x += WAVE) {
        Pair p = tab[x];
        const bool present = p.key != EMPTY;
        if (SMALL && present) p.key = stream_key<ALGO>(a, i, a.g.idx[lo + pos[x]], bi);
        const uint32_t sc = ALGO == ALGO_LPA ? 0u : a.Sig[present ? (int32_t)p.key : d];
        consider_v<ALGO>(W, d, Ki, Sd, kd, (int32_t)p.key, p.val, sc, present, best, bestG);
      }
      // wave arg-max: larger gain first, then lower community id
#pragma unroll
      for (int o = WAVE / 2; o > 0; o >>= 1) {
        const int32_t ob = __shfl_xor(best, o);
        const int64_t og = __shfl_xor(bestG, o);
        const bool take = ob >= 0 && (best < 0 || og > bestG || (og == bestG && ob < best));
        best = take ? ob : best;
        bestG = take ? og : bestG;
      }
      if (lane == 0) finish<ALGO>(a, i, d, best, bestG, ct);
    }
  }
  flush_counters(a, ct);
}

// Exact mode, tier 2: a workgroup per vertex with an open-addressing table (linear
// probing) of CAP slots in LDS.
template <int ALGO, int CAP, bool SMALL = false>
__global__ void __launch_bounds__(BLOCK) k_exact_table(SweepArgs a, const int32_t *__restrict__ list) {
  if (level_over(a)) return;  // batched: every graph has stopped
  __shared__ Pair tab[CAP];
  __shared__ uint32_t pos[SMALL ? CAP : 1];  // small table: first row position per slot
  __shared__ uint32_t kd_s;
  __shared__ int32_t bc[4];
  __shared__ int64_t bg[4];
  const int t = threadIdx.x;
  const int32_t i = list[blockIdx.x];
  if (frozen(a, i)) {  // block-uniform
    if (t == 0) a.Cnew[i] = community_of_self<ALGO>(a, i);
    return;
  }
  const int64_t lo = a.g.off[i], hi = a.g.off[i + 1];
  constexpr uint32_t cap = CAP;
  constexpr bool small = SMALL;  // keys are small-table slots (a.small_slots of them)
  for (uint32_t x = t; x < cap; x += BLOCK) {
    tab[x] = Pair{EMPTY, 0u};
    if (small) pos[x] = 0xFFFFFFFFu;
  }
  if (t == 0) kd_s = 0;
  __syncthreads();
  const int32_t bi = ALGO == ALGO_REFINE ? a.bound[i] : 0;
  const uint32_t mask = cap - 1;
  // four entries per thread and round: their loads and gathers are issued together
  // (an absent entry reads the row's first and is masked), then inserted
  constexpr int U = 4;
  for (int64_t e0 = lo + t; e0 < hi; e0 += U * BLOCK) {
    uint32_t cs[U], ws[U];
    int32_t js[U], bs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + (int64_t)u * BLOCK;
      const bool v = e < hi;
      const int64_t es = v ? e : lo;
      js[u] = a.g.idx[es];
      bs[u] = bi;
      ws[u] = a.g.w[es];
    }
    neighbour_keys<ALGO, U>(a, js, bs, cs);
#pragma unroll
    for (int u = 0; u < U; ++u)  // self-loops are skipped
      cs[u] |= ((e0 + (int64_t)u * BLOCK) < hi && js[u] != i) ? 0u : EMPTY;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (cs[u] == EMPTY) continue;
      const uint32_t c = slot_of(a, cs[u]);  // the table key
      uint32_t h = hash_slot(c, mask);
      while (true) {
        uint32_t prev = atomicCAS(&tab[h].key, EMPTY, c);
        if (prev == EMPTY || prev == c) {
          atomicAdd(&tab[h].val, ws[u]);
          if (small) atomicMin(&pos[h], (uint32_t)(e0 + (int64_t)u * BLOCK - lo));
          break;
        }
        h = (h + 1) & mask;
      }
    }
  }
  __syncthreads();
  const int32_t d = community_of_self<ALGO>(a, i);
  const uint32_t sd = slot_of(a, (uint32_t)d);
  for (uint32_t x = t; x < cap; x += BLOCK) {
    Pair p = tab[x];
    if (p.key == sd) kd_s = p.val;
  }
  __syncthreads();
  const uint32_t kd = kd_s;
  int32_t best = -1;
  int64_t bestG = 0;
  const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
  const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
  const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
  for (uint32_t x = t; x < cap; x += BLOCK) {
    Pair p = tab[x];
    const bool present = p.key != EMPTY;
    if (small && present) {
      // the slot stands for its first key: the key of its earliest row entry
      const uint32_t f = pos[x];
      p.key = stream_key<ALGO>(a, i, a.g.idx[lo + f], bi);
    }
    const uint32_t sc = ALGO == ALGO_LPA ? 0u : a.Sig[present ? (int32_t)p.key : d];
    consider_v<ALGO>(W, d, Ki, Sd, kd, (int32_t)p.key, p.val, sc, present, best, bestG);
  }
  // block arg-max: larger gain first, then lower community id
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    int32_t ob = __shfl_xor(best, o);
    int64_t og = __shfl_xor(bestG, o);
    bool take = ob >= 0 && (best < 0 || og > bestG || (og == bestG && ob < best));
    best = take ? ob : best;
    bestG = take ? og : bestG;
  }
  if (lane_id() == 0) {
    bc[t / WAVE] = best;
    bg[t / WAVE] = bestG;
  }
  __syncthreads();
  if (t == 0) {
    for (int q = 1; q < 4; ++q) {
      bool take = bc[q] >= 0 && (best < 0 || bg[q] > bestG || (bg[q] == bestG && bc[q] < best));
      best = take ? bc[q] : best;
      bestG = take ? bg[q] : bestG;
    }
    Counters ct;
    finish<ALGO>(a, i, d, best, bestG, ct);
    commit_counters(a, ct);
  }
}

// Exact mode, rows of more than exact_t2 entries: a global open-addressing table per
// row (hbase), filled by one workgroup per segment of GSEG entries (global atomics,
// so the segments of one row insert concurrently); then K_{i->d} by a probe, one
// workgroup per TSEG table slots scores them and clears them for the next sweep (the
// tables are cleared once when the schedule is built), and one thread per row
// combines the segments' best (the rule is associative) and decides.  Same keys,
// sums, positions and decision as k_exact_table.
template <int ALGO, bool SMALL>
__global__ void __launch_bounds__(BLOCK)
    k_gtab_insert(SweepArgs a, const int32_t *__restrict__ list, const int64_t *__restrict__ hbase,
                  const int64_t *__restrict__ sstart, const int32_t *__restrict__ sowner, Pair *htab,
                  uint32_t *hpos) {
  if (level_over(a)) return;  // batched: every graph has stopped
  // Each round's U * BLOCK entries are first combined in an LDS table (at most U * BLOCK
  // keys in 2 * U * BLOCK slots), then every distinct key goes to the global table
  // once: the entries of a hub row concentrate on a few communities, whose slots
  // would otherwise serialise the global atomics of all the row's workgroups.
  constexpr int U = 4;  // entries per thread and round, loads and gathers issued together
  constexpr uint32_t LCAP = 2 * U * BLOCK;
  __shared__ uint32_t lk[LCAP], lv[LCAP];
  __shared__ uint32_t lp[SMALL ? LCAP : 1];
  const int t = threadIdx.x;
  const int64_t sg = blockIdx.x;
  const int32_t r = sowner[sg];
  const int32_t i = list[r];
  if (frozen(a, i)) return;  // block-uniform
  const int64_t rlo = a.g.off[i], rhi = a.g.off[i + 1];
  const int64_t lo = rlo + (sg - sstart[r]) * GSEG;
  const int64_t hi = lo + GSEG < rhi ? lo + GSEG : rhi;
  Pair *tab = htab + hbase[r];
  uint32_t *pos = hpos + hbase[r];
  const uint32_t mask = (uint32_t)(hbase[r + 1] - hbase[r]) - 1;
  const int32_t bi = ALGO == ALGO_REFINE ? a.bound[i] : 0;
  for (int64_t b0 = lo; b0 < hi; b0 += U * BLOCK) {  // block-uniform rounds
    for (uint32_t x = t; x < LCAP; x += BLOCK) {
      lk[x] = EMPTY;
      lv[x] = 0u;
      if (SMALL) lp[x] = 0xFFFFFFFFu;
    }
    __syncthreads();
    uint32_t cs[U], ws[U];
    int32_t js[U], bs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = b0 + t + (int64_t)u * BLOCK;
      const bool v = e < hi;
      const int64_t es = v ? e : lo;
      js[u] = a.g.idx[es];
      bs[u] = bi;
      ws[u] = a.g.w[es];
    }
    neighbour_keys<ALGO, U>(a, js, bs, cs);
#pragma unroll
    for (int u = 0; u < U; ++u)  // self-loops are skipped
      cs[u] |= ((b0 + t + (int64_t)u * BLOCK) < hi && js[u] != i) ? 0u : EMPTY;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (cs[u] == EMPTY) continue;
      const uint32_t c = slot_of(a, cs[u]);
      uint32_t h = hash_slot(c, LCAP - 1);
      while (true) {
        const uint32_t prev = atomicCAS(&lk[h], EMPTY, c);
        if (prev == EMPTY || prev == c) break;
        h = (h + 1) & (LCAP - 1);
      }
      atomicAdd(&lv[h], ws[u]);
      if (SMALL) atomicMin(&lp[h], (uint32_t)(b0 + t + (int64_t)u * BLOCK - rlo));
    }
    __syncthreads();
    for (uint32_t x = t; x < LCAP; x += BLOCK) {
      const uint32_t c = lk[x];
      if (c == EMPTY) continue;
      uint32_t h = hash_slot(c, mask);
      while (true) {
        const uint32_t prev = atomicCAS(&tab[h].key, EMPTY, c);
        if (prev == EMPTY || prev == c) break;
        h = (h + 1) & mask;
      }
      atomicAdd(&tab[h].val, lv[x]);
      if (SMALL) atomicMin(&pos[h], lp[x]);
    }
    __syncthreads();  // the flush has read the table before the next round clears it
  }
}

// K_{i->d} of every global-table row, by probing its table for d's key (before any
// workgroup of k_gtab_scan clears a segment of the table).
template <int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_gtab_kd(SweepArgs a, const int32_t *__restrict__ list, int64_t count, const int64_t *__restrict__ hbase,
              const Pair *__restrict__ htab, uint32_t *kdout) {
  if (level_over(a)) return;  // batched: every graph has stopped
  const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (r >= count) return;
  const int32_t i = list[r];
  if (frozen(a, i)) return;
  const Pair *tab = htab + hbase[r];
  const uint32_t mask = (uint32_t)(hbase[r + 1] - hbase[r]) - 1;
  const uint32_t sd = slot_of(a, (uint32_t)community_of_self<ALGO>(a, i));
  uint32_t h = hash_slot(sd, mask), kd = 0;
  while (true) {  // the table is at most half full, so an EMPTY slot ends the probe
    const Pair p = tab[h];
    if (p.key == sd) {
      kd = p.val;
      break;
    }
    if (p.key == EMPTY) break;
    h = (h + 1) & mask;
  }
  kdout[r] = kd;
}

// One workgroup per TSEG slots of a row's table: the best candidate among them
// (larger gain, then lower id) into part[], then the slots are cleared for the next
// sweep.
template <int ALGO, bool SMALL>
__global__ void __launch_bounds__(BLOCK)
    k_gtab_scan(SweepArgs a, const int32_t *__restrict__ list, const int64_t *__restrict__ hbase,
                const int64_t *__restrict__ tstart, const int32_t *__restrict__ towner, Pair *htab,
                uint32_t *hpos, const uint32_t *__restrict__ kdin, int32_t *pbest, int64_t *pgain) {
  if (level_over(a)) return;  // batched: every graph has stopped
  __shared__ int32_t bc[BLOCK / WAVE];
  __shared__ int64_t bg[BLOCK / WAVE];
  const int t = threadIdx.x;
  const int64_t sg = blockIdx.x;
  const int32_t r = towner[sg];
  const int32_t i = list[r];
  if (frozen(a, i)) return;  // block-uniform; the table was not filled
  const int64_t lo = a.g.off[i];
  const int64_t x0 = hbase[r] + (sg - tstart[r]) * TSEG;
  const int64_t x1 = x0 + TSEG < hbase[r + 1] ? x0 + TSEG : hbase[r + 1];
  const int32_t bi = ALGO == ALGO_REFINE ? a.bound[i] : 0;
  const int32_t d = community_of_self<ALGO>(a, i);
  const uint32_t kd = kdin[r];
  int32_t best = -1;
  int64_t bestG = 0;
  const int64_t W = ALGO == ALGO_LPA ? 0 : (int64_t)weight_of(a, i);
  const int64_t Ki = ALGO == ALGO_LPA ? 0 : (int64_t)a.K[i];
  const int64_t Sd = ALGO == ALGO_LPA ? 0 : (int64_t)a.Sig[d];
  for (int64_t x = x0 + t; x < x1; x += BLOCK) {
    Pair p = htab[x];
    const bool present = p.key != EMPTY;
    if (SMALL && present) p.key = stream_key<ALGO>(a, i, a.g.idx[lo + hpos[x]], bi);
    const uint32_t sc = ALGO == ALGO_LPA ? 0u : a.Sig[present ? (int32_t)p.key : d];
    consider_v<ALGO>(W, d, Ki, Sd, kd, (int32_t)p.key, p.val, sc, present, best, bestG);
  }
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int32_t ob = __shfl_xor(best, o);
    const int64_t og = __shfl_xor(bestG, o);
    const bool take = ob >= 0 && (best < 0 || og > bestG || (og == bestG && ob < best));
    best = take ? ob : best;
    bestG = take ? og : bestG;
  }
  if (lane_id() == 0) {
    bc[t / WAVE] = best;
    bg[t / WAVE] = bestG;
  }
  __syncthreads();  // every slot of the segment has been read: clear them
  for (int64_t x = x0 + t; x < x1; x += BLOCK) {
    htab[x] = Pair{EMPTY, 0u};
    if (SMALL) hpos[x] = 0xFFFFFFFFu;
  }
  if (t == 0) {
    for (int q = 1; q < BLOCK / WAVE; ++q) {
      const bool take = bc[q] >= 0 && (best < 0 || bg[q] > bestG || (bg[q] == bestG && bc[q] < best));
      best = take ? bc[q] : best;
      bestG = take ? bg[q] : bestG;
    }
    pbest[sg] = best;
    pgain[sg] = bestG;
  }
}

// One thread per global-table row: the best over its segments, then the decision.
template <int ALGO>
__global__ void __launch_bounds__(BLOCK)
    k_gtab_finish(SweepArgs a, const int32_t *__restrict__ list, int64_t count,
                  const int64_t *__restrict__ tstart, const int32_t *__restrict__ pbest,
                  const int64_t *__restrict__ pgain) {
  if (level_over(a)) return;  // batched: every graph has stopped
  const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  Counters ct;
  if (r < count) {
    const int32_t i = list[r];
    const int32_t d = community_of_self<ALGO>(a, i);
    if (frozen(a, i)) {
      a.Cnew[i] = d;
    } else {
      int32_t best = -1;
      int64_t bestG = 0;
      for (int64_t q = tstart[r]; q < tstart[r + 1]; ++q) {
        const bool take = pbest[q] >= 0 && (best < 0 || pgain[q] > bestG || (pgain[q] == bestG && pbest[q] < best));
        best = take ? pbest[q] : best;
        bestG = take ? pgain[q] : bestG;
      }
      finish<ALGO>(a, i, d, best, bestG, ct);
    }
  }
  flush_counters(a, ct);
}

__global__ void k_gtab_clear(Pair *htab, uint32_t *hpos, int64_t n) {
  const int64_t x = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (x < n) {
    htab[x] = Pair{EMPTY, 0u};
    hpos[x] = 0xFFFFFFFFu;
  }
}

// ---- schedule ------------------------------------------------------------------------

// Category of every vertex for this level's schedule, and per-category counts
// (wave ballots, then one atomic per category and workgroup).
//   MG:    0 = row fits one chunk (sort key: heavy first), 1 + b = a long row of at
//          most 2^b <= 64 chunks (b = 1..6), 7 = longer rows;
//   MG with K = 32 / 64: 0 = at most exact_t0 entries, 1 = one wave per row, 2 = split
//          rows (more than max(L, WAVE_SPLIT) entries);
//   exact: tiers 0..3 by degree.
//   every mode: rows without entries (category 8) are sorted last and listed in no
//          kernel's work: their label can never change, so no sweep writes it, and
//          callers keep both label buffers equal for them.
constexpr int NCAT = 10;
constexpr int CAT_EMPTY = 8;
constexpr int CAT_SHORT = 9;  // MG: rows whose sketch cannot lose weight (exact one-lane kernel)

__global__ void __launch_bounds__(BLOCK)
    k_schedule_keys(const int64_t *off, int32_t n, SchedParams sp, uint64_t *key, uint32_t *val,
                    unsigned long long *cnt) {
  const int mode = sp.mode;
  const int64_t L = sp.L;
  __shared__ unsigned long long bc[NCAT];
  if (threadIdx.x < NCAT) bc[threadIdx.x] = 0;
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  int cat = -1;
  int64_t dmax = 0;
  if (i < n) {
    int64_t deg = off[i + 1] - off[i];
    dmax = deg;
    int b = 0;
    while (b < 63 && (deg >> b) != 0) ++b;  // bits of deg
    uint64_t k;
    if (deg == 0) {
      cat = CAT_EMPTY;
      k = 255;  // after every other key of every mode
    } else if (mode == MODE_EXACT) {
      cat = deg <= sp.exact_t0 ? 0 : deg <= sp.exact_t1 ? 1 : deg <= sp.exact_t2 ? 2 : 3;
      k = cat == 0 ? (uint64_t)(64 - b) : (uint64_t)(128 + cat);
    } else if (sp.wave) {  // K >= 32: short rows exact, split rows, the rest one wave each
      // (K = 128 / 256: every other row is a split row, one wave per chunk)
      cat = deg <= sp.exact_t0 ? 0 : (sp.k > WAVE || (deg > L && deg > WAVE_SPLIT)) ? 2 : 1;
      k = (uint64_t)(cat * 64 + 64 - b);  // heavy rows first in each tier
    } else if (deg <= sp.mg_short) {  // after the single-chunk rows, heavy rows first
      cat = CAT_SHORT;
      k = (uint64_t)(128 + 64 - b);
    } else if (deg <= L) {
      cat = 0;
      k = (uint64_t)(64 - b);  // heavy rows first
    } else {
      int64_t nc = (deg + L - 1) / L;
      int lp = 0;
      while ((1ll << lp) < nc) ++lp;
      cat = lp <= sp.row_lanes_log2 ? lp : 7;
      k = 200ull + (uint64_t)cat;
    }
    key[i] = k;
    val[i] = (uint32_t)i;
  }
#pragma unroll
  for (int q = 0; q < NCAT; ++q) {
    uint64_t m = __ballot(cat == q);
    if (lane_id() == 0 && m) atomicAdd(&bc[q], (unsigned long long)__popcll(m));
  }
  __syncthreads();
  cnt += spread_copy() * (NCAT + 1);
  if (threadIdx.x < NCAT && bc[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], bc[threadIdx.x]);
  // block maximum, then one atomic per block, skipped when it cannot raise the value
  __shared__ unsigned long long bmax[BLOCK / WAVE];
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int64_t x = __shfl_xor(dmax, o);
    dmax = x > dmax ? x : dmax;
  }
  if (lane_id() == 0) bmax[threadIdx.x / WAVE] = (unsigned long long)dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mx = bmax[0];
    for (int q = 1; q < BLOCK / WAVE; ++q) mx = bmax[q] > mx ? bmax[q] : mx;
    if (mx > 0 && mx > __hip_atomic_load(&cnt[NCAT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&cnt[NCAT], mx);
  }  // longest row
}

__global__ void k_chunk_counts(const int64_t *off, const int32_t *multi, int64_t nmulti, int64_t L,
                               int64_t *nch) {
  int64_t m = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (m >= nmulti) return;
  int32_t i = multi[m];
  nch[m] = (off[i + 1] - off[i] + L - 1) / L;
}

__global__ void k_group_counts(const int64_t *cstart, int64_t nmulti, int64_t *ng) {
  int64_t m = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (m >= nmulti) return;
  ng[m] = (cstart[m + 1] - cstart[m] + WAVE - 1) / WAVE;
}

__global__ void k_chunk_owner(const int64_t *cstart, int64_t nmulti, int32_t *owner) {
  int64_t m = blockIdx.x;
  if (m >= nmulti) return;
  for (int64_t q = cstart[m] + threadIdx.x; q < cstart[m + 1]; q += BLOCK) owner[q] = (int32_t)m;
}

__global__ void k_table_segs(const int64_t *hbase, int64_t count, int64_t *nt) {
  const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (r < count) nt[r] = (hbase[r + 1] - hbase[r] + TSEG - 1) / TSEG;
}

__global__ void k_hash_caps(const int64_t *off, const int32_t *list, int64_t count, int64_t *cap) {
  int64_t m = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (m >= count) return;
  int32_t i = list[m];
  int64_t need = 2 * (off[i + 1] - off[i]);
  int64_t c = 1;
  while (c < need) c <<= 1;
  cap[m] = c;
}

__global__ void k_u32_from_u64(const uint32_t *v, int32_t *out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) out[i] = (int32_t)v[i];
}

static unsigned grid_for(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, BLOCK); }

size_t schedule_ws_bytes(int32_t n, int64_t nnz, int mode, int k, int64_t L) {
  size_t b = 0;
  b += (size_t)n * (8 + 4) * 2 + 4096;         // sort keys/values, two buffers
  b += radix_sort_ws_bytes(n) + 4096;
  b += (size_t)n * 4 + 1024;                   // ordered list
  if (mode == MODE_EXACT) {
    // rows on global tables: at most min(n, nnz) (each has an entry)
    const int64_t c3 = n < nnz ? n : nnz;
    // per row: table capacity and base, insert-segment count and start, scan-segment
    // count and start (8 B each), K_{i->d} (4 B); three scans
    b += (size_t)(c3 + 2) * (6 * 8 + 4) + 3 * scan_ws_bytes(c3 + 1) + 8192;
    b += (size_t)(4 * nnz + 64) * (sizeof(Pair) + 4) + 2048;  // tables (cap <= 4*deg), positions
    // insert segments (owner) and scan segments (owner, best, gain)
    const int64_t ns = nnz / GSEG + c3 + 2, nt = (4 * nnz + 64) / TSEG + c3 + 2;
    b += (size_t)ns * 4 + (size_t)nt * (4 + 4 + 8) + 4096;
  } else {
    // a long row has more than one chunk, so more than L entries: at most nnz / L
    // long rows, at most 2 nnz / L + 1 of their chunks, and groups of 64 chunks at
    // most chunks / 64 + long rows
    const int64_t Lc = L > 0 ? L : 1;
    const int64_t nl = nnz / Lc + 1, cl = 2 * (nnz / Lc) + 2, gl = cl / 64 + nl + 1;
    b += (size_t)nnz * 4 + 1024;                                     // key stream
    b += (size_t)(nl + 1) * 8 * 2 + scan_ws_bytes(nl) + 2048;        // chunk counts, cstart
    b += (size_t)cl * (4 + (size_t)(k + 1) * 4) + 4096;              // owner, pass-2 counts
    b += (size_t)(nl + 1) * 8 * 2 + scan_ws_bytes(nl) + 2048;        // group counts, gstart
    b += (size_t)gl * (4 + (size_t)k * sizeof(Pair) + 4) + 4096;     // gowner, roots, flags
    b += (size_t)nl * ((size_t)k * sizeof(Pair) + 4) + 2048;         // candidates, flags
    if (k > 16)  // split rows of the 32/64-slot sketch: chunk nodes, flags, pass-2 counts
      b += (size_t)cl * ((size_t)k * sizeof(Pair) + 4) + (size_t)nl * (k + 1) * 4 + 4096;
    if (k > WAVE) {  // 128/256 slots: every row of more than 32 (or, unconditional, 0)
      // entries is split: at most min(n, nnz) rows and nnz / L + that many chunks
      const int64_t rs = (n < nnz ? (int64_t)n : nnz) + 1, cs = nnz / Lc + rs + 1;
      b += (size_t)(rs + 1) * 8 * 2 + scan_ws_bytes(rs) + (size_t)cs * 4 + 4096;  // counts, cstart, owner
      b += (size_t)cs * ((size_t)k * sizeof(Pair) + 4) + (size_t)rs * (k + 1) * 4 + 4096;
    }
  }
  return b + 64 * 1024;
}

void build_schedule(const Graph &g, const SchedParams &sp_in, Schedule &s, Arena &a, hipStream_t st) {
  SchedParams sp = sp_in;
  if (sp.short_auto && g.nnz > sp.mg_short * (int64_t)g.n) sp.mg_short = 0;
  const int mode = sp.mode, k = sp.k;
  const int64_t L = sp.L;
  const int32_t n = g.n;
  s = Schedule{};
  if (n == 0) return;
  unsigned long long *cnt = a.take<unsigned long long>(SPREAD * (NCAT + 1));
  uint64_t *k0 = a.take<uint64_t>(n);
  uint32_t *v0 = a.take<uint32_t>(n);
  uint64_t *k1 = a.take<uint64_t>(n);
  uint32_t *v1 = a.take<uint32_t>(n);
  int32_t *order = a.take<int32_t>(n);
  launch_zero_u64(cnt, SPREAD * (NCAT + 1), st);
  k_schedule_keys<<<grid_for(n), BLOCK, 0, st>>>(g.off, n, sp, k0, v0, cnt);
  MGCD_LAUNCHED();
  bool flip = radix_sort_pairs(k0, v0, k1, v1, n, 8, a, st);
  k_u32_from_u64<<<grid_for(n), BLOCK, 0, st>>>(flip ? v1 : v0, order, n);
  MGCD_LAUNCHED();
  unsigned long long h[NCAT + 1];
  read_spread(cnt, NCAT, h, st);
  s.maxdeg = (int64_t)h[NCAT];
  if (sp.wave) {
    s.tier[0] = order;
    s.ntier[0] = (int64_t)h[0];
    s.tier[1] = order + h[0];
    s.ntier[1] = (int64_t)h[1];
    s.keybuf = a.take<uint32_t>(g.nnz);
    s.multi = order + h[0] + h[1];
    s.nmulti = (int64_t)h[2];
    if (s.nmulti > 0) {
      int64_t *nch = a.take<int64_t>(s.nmulti);
      s.cstart = a.take<int64_t>(s.nmulti + 1);
      k_chunk_counts<<<grid_for(s.nmulti), BLOCK, 0, st>>>(g.off, s.multi, s.nmulti, L, nch);
      MGCD_LAUNCHED();
      scan_i64(nch, s.cstart, s.nmulti, s.cstart + s.nmulti, a, st);
      MGCD_HIP(hipMemcpyAsync(&s.nchunks, s.cstart + s.nmulti, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      MGCD_HIP(hipStreamSynchronize(st));
      s.owner = a.take<int32_t>(s.nchunks);
      k_chunk_owner<<<(unsigned)s.nmulti, BLOCK, 0, st>>>(s.cstart, s.nmulti, s.owner);
      MGCD_LAUNCHED();
      s.wnode = a.take<Pair>(s.nchunks * k);
      s.wflag = a.take<uint32_t>(s.nchunks);
      s.wcount = a.take<uint32_t>(s.nmulti * (k + 1));
    }
    return;
  }
  if (mode == MODE_EXACT) {
    int64_t pos = 0;
    for (int q = 0; q < 4; ++q) {
      s.tier[q] = order + pos;
      s.ntier[q] = (int64_t)h[q];
      pos += (int64_t)h[q];
    }
    if (s.ntier[3] > 0) {
      int64_t c3 = s.ntier[3];
      s.hbase = a.take<int64_t>(c3 + 1);
      int64_t *caps = a.take<int64_t>(c3);
      k_hash_caps<<<grid_for(c3), BLOCK, 0, st>>>(g.off, s.tier[3], c3, caps);
      MGCD_LAUNCHED();
      scan_i64(caps, s.hbase, c3, s.hbase + c3, a, st);
      int64_t *nseg = a.take<int64_t>(c3);
      s.sstart = a.take<int64_t>(c3 + 1);
      k_chunk_counts<<<grid_for(c3), BLOCK, 0, st>>>(g.off, s.tier[3], c3, GSEG, nseg);
      MGCD_LAUNCHED();
      scan_i64(nseg, s.sstart, c3, s.sstart + c3, a, st);
      int64_t *ntab = a.take<int64_t>(c3);
      s.tstart = a.take<int64_t>(c3 + 1);
      k_table_segs<<<grid_for(c3), BLOCK, 0, st>>>(s.hbase, c3, ntab);
      MGCD_LAUNCHED();
      scan_i64(ntab, s.tstart, c3, s.tstart + c3, a, st);
      int64_t tot = 0;  // table slots, insert and scan segments in one host round trip
      MGCD_HIP(hipMemcpyAsync(&tot, s.hbase + c3, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      MGCD_HIP(hipMemcpyAsync(&s.nseg, s.sstart + c3, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      MGCD_HIP(hipMemcpyAsync(&s.ntseg, s.tstart + c3, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      MGCD_HIP(hipStreamSynchronize(st));
      s.sowner = a.take<int32_t>(s.nseg);
      k_chunk_owner<<<(unsigned)c3, BLOCK, 0, st>>>(s.sstart, c3, s.sowner);
      MGCD_LAUNCHED();
      s.towner = a.take<int32_t>(s.ntseg);
      k_chunk_owner<<<(unsigned)c3, BLOCK, 0, st>>>(s.tstart, c3, s.towner);
      MGCD_LAUNCHED();
      s.gkd = a.take<uint32_t>(c3);
      s.pbest = a.take<int32_t>(s.ntseg);
      s.pgain = a.take<int64_t>(s.ntseg);
      s.htab = a.take<Pair>(tot);
      s.hpos = a.take<uint32_t>(tot);
      k_gtab_clear<<<grid_for(tot), BLOCK, 0, st>>>(s.htab, s.hpos, tot);
      MGCD_LAUNCHED();
    }
    return;
  }
  s.keybuf = a.take<uint32_t>(g.nnz);
  int64_t pos = 0;
  s.single = order;
  s.nsingle = (int64_t)h[0];
  pos = s.nsingle;
  s.tier[0] = order + pos;  // short rows
  s.ntier[0] = (int64_t)h[CAT_SHORT];
  pos += s.ntier[0];
  for (int b = 1; b <= 6; ++b) {
    s.packed[b] = order + pos;
    s.npacked[b] = (int64_t)h[b];
    pos += (int64_t)h[b];
  }
  s.multi = order + pos;
  s.nmulti = (int64_t)h[7];
  if (s.nmulti > 0) {
    int64_t *nch = a.take<int64_t>(s.nmulti);
    s.cstart = a.take<int64_t>(s.nmulti + 1);
    k_chunk_counts<<<grid_for(s.nmulti), BLOCK, 0, st>>>(g.off, s.multi, s.nmulti, L, nch);
    MGCD_LAUNCHED();
    scan_i64(nch, s.cstart, s.nmulti, s.cstart + s.nmulti, a, st);
    int64_t *ng = a.take<int64_t>(s.nmulti);
    s.gstart = a.take<int64_t>(s.nmulti + 1);
    k_group_counts<<<grid_for(s.nmulti), BLOCK, 0, st>>>(s.cstart, s.nmulti, ng);
    MGCD_LAUNCHED();
    scan_i64(ng, s.gstart, s.nmulti, s.gstart + s.nmulti, a, st);
    // chunk and group totals in one host round trip
    MGCD_HIP(hipMemcpyAsync(&s.nchunks, s.cstart + s.nmulti, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MGCD_HIP(hipMemcpyAsync(&s.ngroups, s.gstart + s.nmulti, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MGCD_HIP(hipStreamSynchronize(st));
    s.owner = a.take<int32_t>(s.nchunks);
    k_chunk_owner<<<(unsigned)s.nmulti, BLOCK, 0, st>>>(s.cstart, s.nmulti, s.owner);
    MGCD_LAUNCHED();
    s.gowner = a.take<int32_t>(s.ngroups);
    k_chunk_owner<<<(unsigned)s.nmulti, BLOCK, 0, st>>>(s.gstart, s.nmulti, s.gowner);
    MGCD_LAUNCHED();
    s.sk = a.take<Pair>(s.ngroups * k);
    s.skflag = a.take<uint32_t>(s.ngroups);
    s.part = a.take<uint32_t>(s.nchunks * (k + 1));
    s.cand = a.take<Pair>(s.nmulti * k);
    s.cflag = a.take<uint32_t>(s.nmulti);
  }
  {  // bucket table of k_move_rows, heaviest bucket first in the grid
    Buckets bk{};
    int64_t w = 0;
    for (int b = 6; b >= 0; --b) {
      const int64_t rows = b == 0 ? s.nsingle : s.npacked[b];
      bk.rows[b] = b == 0 ? s.single : s.packed[b];
      bk.nrows[b] = rows;
      bk.wave_begin[b] = w;
      w += ceil_div(rows << b, WAVE);
      bk.wave_end[b] = w;
    }
    s.row_waves = w;
    bk.ngroups = s.ngroups;
    bk.multi = s.multi;
    bk.gowner = s.gowner;
    bk.gstart = s.gstart;
    bk.cstart = s.cstart;
    bk.sk = s.sk;
    bk.skflag = s.skflag;
    s.buckets = bk;  // a kernel argument: no upload, no host round trip
  }
}

// ---- launch -------------------------------------------------------------------------

static inline void mark(hipEvent_t *ev, int i, hipStream_t st) {
  if (ev) MGCD_HIP(hipEventRecord(ev[i], st));
}

// Workgroups of the main sweep kernel resident at once on the current device: its LDS
// windows (36 KiB per workgroup) leave room for four per compute unit.
static int64_t resident_blocks() {
  int dev = 0, cus = 0;
  MGCD_HIP(hipGetDevice(&dev));
  MGCD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return 4 * (int64_t)(cus > 0 ? cus : 1);
}

template <int K, int ALGO, int MODE>
static void sweep_mg(const SweepArgs &a, const Schedule &s, int64_t L, hipStream_t st, hipEvent_t *ev) {
  mark(ev, 0, st);
  const int64_t waves = s.ngroups + s.row_waves;
  if (waves > 0) {
    // persistent (a.queue): as many workgroups as stay resident at once, each pulling
    // work until the queue is empty
    const int64_t blocks = ceil_div(waves, BLOCK / WAVE);
    if (a.queue)
      k_move_rows<K, ALGO, MODE, true><<<(unsigned)std::min<int64_t>(blocks, resident_blocks()), BLOCK, 0, st>>>(
          a, s.buckets, L, s.keybuf);
    else
      k_move_rows<K, ALGO, MODE, false><<<(unsigned)blocks, BLOCK, 0, st>>>(a, s.buckets, L, s.keybuf);
    MGCD_LAUNCHED();
  }
  mark(ev, 1, st);
  // long rows: rest of the merge tree, pass 2, decision
  if (s.nmulti > 0) {
    k_long_merge<K, ALGO><<<(unsigned)s.nmulti, BLOCK, 0, st>>>(a, s.multi, s.gstart, s.sk,
                                                                s.skflag, s.cand, s.cflag);
    MGCD_LAUNCHED();
    k_long_count<K, ALGO><<<(unsigned)ceil_div(s.nchunks, BLOCK / WAVE), BLOCK, 0, st>>>(
        a, s.multi, s.owner, s.cstart, s.nchunks, L, s.cand, s.cflag, s.keybuf, s.part);
    MGCD_LAUNCHED();
    k_long_decide<K, ALGO><<<(unsigned)s.nmulti, BLOCK, 0, st>>>(a, s.multi, s.cstart, s.cand,
                                                                 s.cflag, s.part);
    MGCD_LAUNCHED();
  }
  mark(ev, 2, st);
  if (s.ntier[0] > 0) {  // rows whose sketch is their exact table: the exact one-lane kernel
    k_exact_small<ALGO><<<grid_for(s.ntier[0]), BLOCK, 0, st>>>(a, s.tier[0], s.ntier[0]);
    MGCD_LAUNCHED();
  }
  mark(ev, 3, st);
}

template <int ALGO, bool SMALL = false>
static void sweep_exact(const SweepArgs &a, const Schedule &s, hipStream_t st, hipEvent_t *ev) {
  mark(ev, 0, st);
  if (s.ntier[0] > 0) {
    k_exact_small<ALGO><<<grid_for(s.ntier[0]), BLOCK, 0, st>>>(a, s.tier[0], s.ntier[0]);
    MGCD_LAUNCHED();
  }
  mark(ev, 1, st);
  if (s.ntier[1] > 0) {
    k_exact_wave<ALGO, SMALL><<<(unsigned)ceil_div(s.ntier[1], BLOCK / WAVE), BLOCK, 0, st>>>(
        a, s.tier[1], s.ntier[1]);
    MGCD_LAUNCHED();
  }
  if (s.ntier[2] > 0) {
    k_exact_table<ALGO, 8192, SMALL><<<(unsigned)s.ntier[2], BLOCK, 0, st>>>(a, s.tier[2]);
    MGCD_LAUNCHED();
  }
  mark(ev, 2, st);
  if (s.ntier[3] > 0) {
    k_gtab_insert<ALGO, SMALL><<<(unsigned)s.nseg, BLOCK, 0, st>>>(a, s.tier[3], s.hbase, s.sstart, s.sowner,
                                                                  s.htab, s.hpos);
    MGCD_LAUNCHED();
    k_gtab_kd<ALGO><<<grid_for(s.ntier[3]), BLOCK, 0, st>>>(a, s.tier[3], s.ntier[3], s.hbase, s.htab, s.gkd);
    MGCD_LAUNCHED();
    k_gtab_scan<ALGO, SMALL><<<(unsigned)s.ntseg, BLOCK, 0, st>>>(a, s.tier[3], s.hbase, s.tstart, s.towner,
                                                                 s.htab, s.hpos, s.gkd, s.pbest, s.pgain);
    MGCD_LAUNCHED();
    k_gtab_finish<ALGO><<<grid_for(s.ntier[3]), BLOCK, 0, st>>>(a, s.tier[3], s.ntier[3], s.tstart, s.pbest,
                                                                s.pgain);
    MGCD_LAUNCHED();
  }
  mark(ev, 3, st);
}

template <int K, int ALGO, int MODE>
static void sweep_wave(const SweepArgs &a, const Schedule &s, int64_t L, hipStream_t st, hipEvent_t *ev) {
  mark(ev, 0, st);
  if (s.ntier[0] > 0) {  // rows that cannot lose weight: the exact one-lane kernel
    k_exact_small<ALGO><<<grid_for(s.ntier[0]), BLOCK, 0, st>>>(a, s.tier[0], s.ntier[0]);
    MGCD_LAUNCHED();
  }
  mark(ev, 1, st);
  if constexpr (K <= WAVE) {  // K = 128 / 256: every row the sketch takes is a split row
    if (s.ntier[1] > 0) {
      const unsigned grid = (unsigned)ceil_div(s.ntier[1], BLOCK / WAVE);
      if (wave_depth_for(s.nmulti > 0 ? (L > WAVE_SPLIT ? L : WAVE_SPLIT) : s.maxdeg, L) == WDEPTH_SHALLOW)
        k_wave_rows<K, ALGO, MODE, WDEPTH_SHALLOW><<<grid, BLOCK, 0, st>>>(a, s.tier[1], s.ntier[1], L,
                                                                           s.keybuf);
      else
        k_wave_rows<K, ALGO, MODE, WDEPTH><<<grid, BLOCK, 0, st>>>(a, s.tier[1], s.ntier[1], L, s.keybuf);
      MGCD_LAUNCHED();
    }
  }
  mark(ev, 2, st);
  if (s.nmulti > 0) {  // split rows
    const unsigned cgrid = (unsigned)ceil_div(s.nchunks, BLOCK / WAVE);
    k_wave_chunks<K, ALGO, MODE><<<cgrid, BLOCK, 0, st>>>(a, s.multi, s.cstart, s.owner, s.nchunks, L,
                                                          s.keybuf, s.wnode, s.wflag, s.wcount);
    MGCD_LAUNCHED();
    const int64_t maxch = (s.maxdeg + L - 1) / L;
    for (int l = 0; ((int64_t)1 << l) < maxch; ++l) {
      k_wave_level<K><<<cgrid, BLOCK, 0, st>>>(a, s.multi, s.cstart, s.owner, s.nchunks, l, s.wnode,
                                               s.wflag);
      MGCD_LAUNCHED();
    }
    if (second_pass(a, ALGO)) {
      k_wave_count<K, ALGO><<<cgrid, BLOCK, 0, st>>>(a, s.multi, s.cstart, s.owner, s.nchunks, L, s.keybuf,
                                                     s.wnode, s.wflag, s.wcount);
      MGCD_LAUNCHED();
    }
    k_wave_decide<K, ALGO><<<(unsigned)ceil_div(s.nmulti, BLOCK / WAVE), BLOCK, 0, st>>>(
        a, s.multi, s.cstart, s.nmulti, s.wnode, s.wflag, s.wcount);
    MGCD_LAUNCHED();
  }
  mark(ev, 3, st);
}

template <int ALGO, int MODE>
static void sweep_k(const SweepArgs &a, const Schedule &s, int k, int64_t L, hipStream_t st,
                    hipEvent_t *ev) {
  switch (k) {
    case 32: sweep_wave<32, ALGO, MODE>(a, s, L, st, ev); break;
    case 64: sweep_wave<64, ALGO, MODE>(a, s, L, st, ev); break;
    case 128: sweep_wave<128, ALGO, MODE>(a, s, L, st, ev); break;
    case 256: sweep_wave<256, ALGO, MODE>(a, s, L, st, ev); break;
    case 1: sweep_mg<1, ALGO, MODE>(a, s, L, st, ev); break;
    case 2: sweep_mg<2, ALGO, MODE>(a, s, L, st, ev); break;
    case 4: sweep_mg<4, ALGO, MODE>(a, s, L, st, ev); break;
    case 8: sweep_mg<8, ALGO, MODE>(a, s, L, st, ev); break;
    case 16: sweep_mg<16, ALGO, MODE>(a, s, L, st, ev); break;
    default: throw Error(-6, "k must be 1, 2, 4, 8, 16, 32, 64, 128 or 256");
  }
}

template <int ALGO>
static void sweep_algo(const SweepArgs &a, const Schedule &s, int mode, int k, int64_t L,
                       hipStream_t st, hipEvent_t *ev) {
  switch (mode) {
    case MODE_EXACT: sweep_exact<ALGO>(a, s, st, ev); break;
    case MODE_SMALL: {  // the exact kernels keyed by small-table slots (k of them)
      SweepArgs b = a;
      b.small_slots = k;
      sweep_exact<ALGO, true>(b, s, st, ev);
      break;
    }
    case MODE_ALG1: sweep_k<ALGO, MODE_ALG1>(a, s, k, L, st, ev); break;
    case MODE_UNCOND: sweep_k<ALGO, MODE_UNCOND>(a, s, k, L, st, ev); break;
    case MODE_STD: sweep_k<ALGO, MODE_STD>(a, s, k, L, st, ev); break;
    default: throw Error(-6, "unknown sketch mode");
  }
}

void launch_sweep(const SweepArgs &a, const Schedule &s, int algo, int mode, int k, int64_t L,
                  hipStream_t st, hipEvent_t *ev) {
  switch (algo) {
    case ALGO_LPA: sweep_algo<ALGO_LPA>(a, s, mode, k, L, st, ev); break;
    case ALGO_MOVE: sweep_algo<ALGO_MOVE>(a, s, mode, k, L, st, ev); break;
    case ALGO_REFINE: sweep_algo<ALGO_REFINE>(a, s, mode, k, L, st, ev); break;
    default: throw Error(-1, "unknown sweep");
  }
}

// ---- bookkeeping kernels ---------------------------------------------------------------

__device__ inline void level_converge(int algo, const LevelRule &r) {
  // Read and clear in one atomic step: a plain load of these uniform addresses may
  // become a scalar load, which a following vector store of 0 can overtake.
  unsigned long long *ctr = r.ctr;
  const unsigned long long moved = atomicExch(&ctr[0], 0ull), prop = atomicExch(&ctr[1], 0ull),
                           sumG = atomicExch(&ctr[2], 0ull), cands = atomicExch(&ctr[3], 0ull);
  LevelState *ls = r.ls;
  if (ls->halt) return;
  ls->cands += cands;
  ls->sweeps += 1;
  ls->edges += (unsigned long long)r.nnz;
  ls->moved_last = moved;
  const bool stop = algo == ALGO_LPA ? (double)moved <= r.tol * (double)r.n
                                     : prop == 0 || 2.0 * (double)sumG <= r.tol * r.WW;
  if (stop) ls->halt = 1;
}

__global__ void k_apply_moves(const int32_t *Cold, const int32_t *Cnew, const uint32_t *K, uint32_t *Sig,
                              int32_t n, LevelRule rule) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (rule.live && *rule.live == 0) return;  // batched: the sweep did nothing
  if (rule.ls && i == 0) level_converge(ALGO_MOVE, rule);  // the sweep's counters are final
  if (i >= n) return;
  int32_t d = Cold[i], c = Cnew[i];
  if (c == d) return;
  uint32_t k = K[i];
  atomicSub(&Sig[d], k);
  atomicAdd(&Sig[c], k);
}

void launch_apply_moves(const int32_t *Cold, const int32_t *Cnew, const uint32_t *K, uint32_t *Sig,
                        int32_t n, hipStream_t st, const LevelRule *rule) {
  const LevelRule r = rule ? *rule : LevelRule{};
  if (n <= 0 && !rule) return;
  k_apply_moves<<<n > 0 ? grid_for(n) : 1, BLOCK, 0, st>>>(Cold, Cnew, K, Sig, n, r);
  MGCD_LAUNCHED();
}

__global__ void k_zero_totals(uint32_t *Sig, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) Sig[i] = 0;
}

__global__ void k_totals(const int32_t *C, const uint32_t *K, uint32_t *Sig, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) atomicAdd(&Sig[C[i]], K[i]);
}

void launch_community_totals(const int32_t *C, const uint32_t *K, uint32_t *Sig, int32_t n,
                             hipStream_t st) {
  if (n <= 0) return;
  k_zero_totals<<<grid_for(n), BLOCK, 0, st>>>(Sig, n);
  MGCD_LAUNCHED();
  k_totals<<<grid_for(n), BLOCK, 0, st>>>(C, K, Sig, n);
  MGCD_LAUNCHED();
}

__global__ void k_count_proposals(const int32_t *prop, int32_t *nprop, int32_t *from, int32_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  int32_t t = prop[i];
  if (t != (int32_t)i) {
    atomicAdd(&nprop[t], 1);
    from[t] = (int32_t)i;  // read only where exactly one vertex proposed t
  }
}

__global__ void k_accept(const int32_t *prop, const int32_t *nprop, const int32_t *from, int32_t *R,
                         int32_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  int32_t t = prop[i];
  bool ok = t != (int32_t)i &&
            (nprop[i] == 0 || (nprop[i] == 1 && from[i] == t && t < (int32_t)i));
  R[i] = ok ? t : (int32_t)i;
}

void launch_refine_accept(const int32_t *prop, int32_t *nprop, int32_t *from, int32_t *R, int32_t n,
                          hipStream_t st) {
  if (n <= 0) return;
  launch_fill_i32(nprop, 0, n, st);
  k_count_proposals<<<grid_for(n), BLOCK, 0, st>>>(prop, nprop, from, n);
  MGCD_LAUNCHED();
  k_accept<<<grid_for(n), BLOCK, 0, st>>>(prop, nprop, from, R, n);
  MGCD_LAUNCHED();
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_iota(int32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}
__global__ void k_level_converge(int algo, LevelRule r) { level_converge(algo, r); }

void launch_level_converge(int algo, const LevelRule &r, hipStream_t st) {
  k_level_converge<<<1, 1, 0, st>>>(algo, r);
  MGCD_LAUNCHED();
}

__global__ void k_zero_state(LevelState *ls) { *ls = LevelState{0, 0, 0, 0, 0}; }

void launch_zero_state(LevelState *ls, hipStream_t st) {
  k_zero_state<<<1, 1, 0, st>>>(ls);
  MGCD_LAUNCHED();
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = 0;
}

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill_i32<<<grid_for(n), BLOCK, 0, st>>>(p, v, n);
  MGCD_LAUNCHED();
}
void launch_iota(int32_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_iota<<<grid_for(n), BLOCK, 0, st>>>(p, n);
  MGCD_LAUNCHED();
}
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_zero_u64<<<grid_for(n), BLOCK, 0, st>>>(p, n);
  MGCD_LAUNCHED();
}

}  // namespace mgcd
