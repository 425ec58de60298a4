/*
 * mgcd_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU implementation of what the weighted Misra-Gries (MG)
 * community-detection path computes (Sahu, "Memory-Efficient Community Detection
 * on Large Graphs Using Weighted Sketches", arXiv 2411.02268).  It exists to check
 * the HIP implementation; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header or table with the
 * HIP library.
 *
 * Every step follows the paper's text and notation:
 *   - graph, weighted degree K_i, total weight m ........ Section 3 (Preliminaries)
 *   - K_{i->c}, sigma_c, Sigma_c ........................ Section 3.1
 *   - modularity Q ...................................... Section 3.2, Eq. 1
 *   - delta-modularity .................................. Section 3.2, Eq. 2
 *   - LPA ............................................... Sections 3.5 and 4.3
 *   - Louvain local moving and aggregation with MG ...... Section 4.1, Figs. 2-3
 *   - Leiden refinement and symmetric aggregation ....... Section 4.2
 *   - populating the MG sketch .......................... Appendix A.1, Algorithm 1
 *
 * Readings of points the paper leaves open (all also listed in the design notes):
 *   R1  the sketch key of neighbour j is C[j], the neighbour's community (Fig. 2 and
 *       Section 4.1 say the neighbours' memberships populate the sketch; the
 *       "c <- C[i]" of Algorithm 1 is read as a typo);
 *   R2  a fresh sketch has key EMPTY (never a community id) and value 0 in every slot;
 *   R3  candidates after pass 1 are the keys whose value is positive;
 *   R4  pass 2 always accumulates K_{i->d} for the current community d as well;
 *   R5  updates are synchronous (Jacobi): every vertex of a sweep reads the
 *       membership, Sigma and sizes of the previous sweep;
 *   R6  ties go to the lowest community id; Louvain/Leiden move only if the best
 *       gain is strictly positive; the gain is Eq. 2 scaled by W^2/2 (W = 2m), an
 *       exact integer when weights are integers;
 *   R7  synchronous Louvain/Leiden sweeps alternate direction (as in synchronous GPU
 *       Louvain implementations): in sweep t of a pass (t = 0, 1, ...) a vertex's
 *       best move is applied only if it goes to a lower community id (t even) or a
 *       higher one (t odd); otherwise the vertex stays for this sweep.  A pass's
 *       local moving ends when no vertex has a positive-gain move, when the summed
 *       gain of all such moves is at most tol (2*sumG/W^2 <= tol), or after
 *       max_iterations sweeps; this keeps pairs of vertices from swapping forever;
 *   R8  a stream longer than L entries is cut into consecutive chunks of L
 *       positions; each chunk runs Algorithm 1 from an empty sketch; chunk sketches
 *       are merged pairwise, left to right, level by level (an odd last one moves
 *       up unchanged) with the mergeable-summary rule of Agarwal et al. (2012):
 *       add equal keys; if more than k keys remain, subtract the (k+1)-th largest
 *       value and keep the positive ones;
 *   R9  aggregation streams a community's members in ascending vertex id, each
 *       row in CSR order, self-loops included; the new row is the sketch's positive
 *       entries sorted by key; K of a super-vertex is the exact sum of its members'
 *       K and W stays the input's;
 *   R10 Leiden refinement is one greedy Jacobi sweep from singleton sub-communities
 *       inside the local-moving community (the bound); vertex i proposes its best
 *       target t (positive gain); the proposal is accepted unless some vertex other
 *       than t proposed i, or t proposed i with t > i;
 *   R11 Leiden's next pass starts each super-vertex in its bound community; Leiden
 *       aggregation symmetrises the kept pairs, weight max(v_st, v_ts);
 *   R12 modularity sums over CSR entries (a self-loop entry counts once), 2m = W.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

#define EMPTY_KEY 0xFFFFFFFFu
#define KMAX 1024

typedef struct {
  uint32_t key;
  uint32_t val;
} pair_t;

/* ------------------------------------------------------------------------------ */
/* Sketch update rules                                                              */
/* ------------------------------------------------------------------------------ */

/* Algorithm 1 (conditional subtraction, Appendix A.1).  Keys are unique in the
 * sketch, and a key whose value fell to 0 keeps its slot until it is overwritten:
 * an arriving item with that key revives it instead of being inserted.  One scan
 * finds the slot of c, if any, and the highest-index slot of value 0.  A key in
 * the sketch takes w; otherwise c goes into that free slot; with no free slot every
 * value loses w (clamped at 0) and the item is dropped (the conditional rule). */
static void populate_alg1(uint32_t *Sk, uint32_t *Sv, int k, uint32_t c, uint32_t w) {
  int at = -1, free_slot = -1;
  for (int p = 0; p < k; ++p) {
    if (Sk[p] == c) at = p;
    else if (Sv[p] == 0) free_slot = p;
  }
  if (at >= 0) {
    Sv[at] += w;
  } else if (free_slot >= 0) {
    Sk[free_slot] = c;
    Sv[free_slot] = w;
  } else {
    for (int p = 0; p < k; ++p) Sv[p] = Sv[p] > w ? Sv[p] - w : 0;
  }
}

/* Unconditional subtraction (Section 4.1, variant 1): when c is not present (a
 * key counts as present while its value is positive), subtract w from every slot
 * first, then insert (c, w) into the last slot whose value is 0, if there is one. */
static void populate_uncond(uint32_t *Sk, uint32_t *Sv, int k, uint32_t c, uint32_t w) {
  for (int p = 0; p < k; ++p)
    if (Sk[p] == c && Sv[p] > 0) {
      Sv[p] += w;
      return;
    }
  for (int p = 0; p < k; ++p) Sv[p] = Sv[p] > w ? Sv[p] - w : 0;
  int e = -1;
  for (int p = 0; p < k; ++p)
    if (Sv[p] == 0) e = p;
  if (e >= 0) {
    Sk[e] = c;
    Sv[e] = w;
  }
}

/* Textbook weighted Misra-Gries: when c is absent and every slot is full, the
 * amount d = min(w, smallest value) is taken from every slot and from w; a positive
 * remainder of w is then inserted. */
static void populate_std(uint32_t *Sk, uint32_t *Sv, int k, uint32_t c, uint32_t w) {
  for (int p = 0; p < k; ++p)
    if (Sk[p] == c && Sv[p] > 0) {
      Sv[p] += w;
      return;
    }
  int e = -1;
  for (int p = 0; p < k; ++p)
    if (Sv[p] == 0) e = p;
  if (e < 0) {
    uint32_t d = w;
    for (int p = 0; p < k; ++p)
      if (Sv[p] < d) d = Sv[p];
    for (int p = 0; p < k; ++p) Sv[p] -= d;
    w -= d;
    if (w == 0) return;
    for (int p = 0; p < k; ++p)
      if (Sv[p] == 0) e = p;
  }
  Sk[e] = c;
  Sv[e] = w;
}

static void populate(int mode, uint32_t *Sk, uint32_t *Sv, int k, uint32_t c, uint32_t w) {
  if (mode == OR_MODE_UNCOND)
    populate_uncond(Sk, Sv, k, c, w);
  else if (mode == OR_MODE_STD)
    populate_std(Sk, Sv, k, c, w);
  else
    populate_alg1(Sk, Sv, k, c, w);
}

static int cmp_pair_key(const void *a, const void *b) {
  uint32_t x = ((const pair_t *)a)->key, y = ((const pair_t *)b)->key;
  return x < y ? -1 : x > y;
}

static int cmp_u32_desc(const void *a, const void *b) {
  uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
  return x > y ? -1 : x < y;
}

/* One chunk: Algorithm 1 (or a variant) from an empty sketch over stream positions
 * [lo, hi) whose use flag is set.  Returns the positive entries sorted by key. */
static int chunk_sketch(const uint32_t *key, const uint32_t *w, const uint8_t *use, int64_t lo,
                        int64_t hi, int mode, int k, pair_t *out) {
  uint32_t Sk[KMAX], Sv[KMAX];
  for (int p = 0; p < k; ++p) {
    Sk[p] = EMPTY_KEY;
    Sv[p] = 0;
  }
  for (int64_t e = lo; e < hi; ++e)
    if (use[e]) populate(mode, Sk, Sv, k, key[e], w[e]);
  int n = 0;
  for (int p = 0; p < k; ++p)
    if (Sv[p] > 0) {
      out[n].key = Sk[p];
      out[n].val = Sv[p];
      ++n;
    }
  qsort(out, (size_t)n, sizeof(pair_t), cmp_pair_key);
  return n;
}

/* Mergeable MG summaries (Agarwal et al. 2012): add the counters of equal keys; if
 * more than k keys remain, subtract the (k+1)-th largest counter from all of them
 * and keep the positive ones.  Output sorted by key. */
static int mg_merge(const pair_t *a, int na, const pair_t *b, int nb, int k, pair_t *out) {
  pair_t u[2 * KMAX];
  int nu = 0;
  for (int x = 0; x < na; ++x) u[nu++] = a[x];
  for (int y = 0; y < nb; ++y) {
    int found = 0;
    for (int x = 0; x < nu; ++x)
      if (u[x].key == b[y].key) {
        u[x].val += b[y].val;
        found = 1;
        break;
      }
    if (!found) u[nu++] = b[y];
  }
  int n = 0;
  if (nu <= k) {
    for (int x = 0; x < nu; ++x) out[n++] = u[x];
  } else {
    uint32_t vals[2 * KMAX];
    for (int x = 0; x < nu; ++x) vals[x] = u[x].val;
    qsort(vals, (size_t)nu, sizeof(uint32_t), cmp_u32_desc);
    uint32_t t = vals[k];
    for (int x = 0; x < nu; ++x)
      if (u[x].val > t) {
        out[n].key = u[x].key;
        out[n].val = u[x].val - t;
        ++n;
      }
  }
  qsort(out, (size_t)n, sizeof(pair_t), cmp_pair_key);
  return n;
}

/* The sketch of a whole stream of n positions (reading R8).  Returns the positive
 * entries sorted by key; *subtracted is not reported -- the oracle always runs the
 * second pass. */
static int stream_sketch(const uint32_t *key, const uint32_t *w, const uint8_t *use, int64_t n,
                         int mode, int k, int64_t L, pair_t *out) {
  if (n <= 0) return 0;
  if (n <= L) return chunk_sketch(key, w, use, 0, n, mode, k, out);
  int64_t nc = (n + L - 1) / L;
  pair_t *sk = (pair_t *)malloc(sizeof(pair_t) * (size_t)nc * (size_t)k);
  int *cnt = (int *)malloc(sizeof(int) * (size_t)nc);
  for (int64_t q = 0; q < nc; ++q) {
    int64_t lo = q * L, hi = lo + L < n ? lo + L : n;
    cnt[q] = chunk_sketch(key, w, use, lo, hi, mode, k, sk + q * k);
  }
  int64_t len = nc;
  while (len > 1) {
    int64_t next = 0;
    for (int64_t x = 0; x + 1 < len; x += 2) {
      pair_t tmp[KMAX];
      int m = mg_merge(sk + x * k, cnt[x], sk + (x + 1) * k, cnt[x + 1], k, tmp);
      memcpy(sk + next * k, tmp, sizeof(pair_t) * (size_t)m);
      cnt[next] = m;
      ++next;
    }
    if (len & 1) {
      memmove(sk + next * k, sk + (len - 1) * k, sizeof(pair_t) * (size_t)cnt[len - 1]);
      cnt[next] = cnt[len - 1];
      ++next;
    }
    len = next;
  }
  int m = cnt[0];
  memcpy(out, sk, sizeof(pair_t) * (size_t)m);
  free(sk);
  free(cnt);
  return m;
}

/* Exact table: every distinct key of the stream with the sum of its weights
 * (the per-thread hashtable of Section 4 / Fig. 1, written as a plain sort). */
static int exact_table(const uint32_t *key, const uint32_t *w, const uint8_t *use, int64_t n,
                       pair_t *out) {
  int64_t m = 0;
  for (int64_t e = 0; e < n; ++e)
    if (use[e]) {
      out[m].key = key[e];
      out[m].val = w[e];
      ++m;
    }
  qsort(out, (size_t)m, sizeof(pair_t), cmp_pair_key);
  int64_t r = 0;
  for (int64_t e = 0; e < m; ++e) {
    if (r > 0 && out[r - 1].key == out[e].key)
      out[r - 1].val += out[e].val;
    else
      out[r++] = out[e];
  }
  return (int)r;
}

/* The small mod-based table of Appendix A.2 with S slots: an entry with key c lands
 * in slot c mod S; a slot keeps the first key that reached it (in stream order) and
 * accumulates the weights of every key that reaches it, colliding or not.  out:
 * the used slots as (first key, summed weight), ascending slot.  *vd: the sum in
 * the slot of key d (0 if unused), the mod-based lookup of K_{i->d}. */
typedef struct {
  uint64_t slot;
  int64_t pos;
  uint32_t key, w;
} slot_entry_t;

static int cmp_slot_entry(const void *a, const void *b) {
  const slot_entry_t *x = (const slot_entry_t *)a, *y = (const slot_entry_t *)b;
  if (x->slot != y->slot) return x->slot < y->slot ? -1 : 1;
  return x->pos < y->pos ? -1 : x->pos > y->pos;
}

static int small_table(const uint32_t *key, const uint32_t *w, const uint8_t *use, int64_t n,
                       int64_t S, uint32_t d, pair_t *out, int64_t *vd) {
  slot_entry_t *t = (slot_entry_t *)malloc(sizeof(slot_entry_t) * (size_t)(n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t e = 0; e < n; ++e)
    if (use[e]) t[m++] = (slot_entry_t){(uint64_t)key[e] % (uint64_t)S, e, key[e], w[e]};
  qsort(t, (size_t)m, sizeof(slot_entry_t), cmp_slot_entry);
  const uint64_t sd = (uint64_t)d % (uint64_t)S;
  int r = 0;
  *vd = 0;
  for (int64_t e = 0; e < m;) {
    int64_t f = e;
    uint64_t sum = 0;
    while (f < m && t[f].slot == t[e].slot) sum += t[f++].w;
    out[r++] = (pair_t){t[e].key, (uint32_t)sum};  /* t[e]: the slot's first entry */
    if (t[e].slot == sd) *vd = (int64_t)sum;
    e = f;
  }
  free(t);
  return r;
}

/* exported for the sketch tests */
int oracle_sketch_stream(const uint32_t *keys, const uint32_t *weights, int64_t n, int mode, int k,
                         int64_t chunk_len, uint32_t *out_keys, uint32_t *out_vals) {
  if (k < 1 || k > KMAX || chunk_len < 1) return -1;
  uint8_t *use = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  for (int64_t e = 0; e < n; ++e) use[e] = 1;
  pair_t *out = (pair_t *)malloc(sizeof(pair_t) * (size_t)(mode == OR_MODE_EXACT ? (n > 0 ? n : 1) : k));
  int m = mode == OR_MODE_EXACT ? exact_table(keys, weights, use, n, out)
                                : stream_sketch(keys, weights, use, n, mode, k, chunk_len, out);
  for (int x = 0; x < m; ++x) {
    out_keys[x] = out[x].key;
    out_vals[x] = out[x].val;
  }
  free(out);
  free(use);
  return m;
}

int oracle_mg_merge(const uint32_t *ak, const uint32_t *av, int na, const uint32_t *bk,
                    const uint32_t *bv, int nb, int k, uint32_t *ok, uint32_t *ov) {
  if (k < 1 || k > KMAX || na > k || nb > k) return -1;
  pair_t a[KMAX], b[KMAX], o[KMAX];
  for (int x = 0; x < na; ++x) a[x] = (pair_t){ak[x], av[x]};
  for (int x = 0; x < nb; ++x) b[x] = (pair_t){bk[x], bv[x]};
  int m = mg_merge(a, na, b, nb, k, o);
  for (int x = 0; x < m; ++x) {
    ok[x] = o[x].key;
    ov[x] = o[x].val;
  }
  return m;
}

/* ------------------------------------------------------------------------------ */
/* Graph helpers                                                                    */
/* ------------------------------------------------------------------------------ */

typedef struct {
  int32_t n;
  int64_t nnz;
  int64_t *off;
  int32_t *idx;
  uint32_t *w;
  int owned;
} graph_t;

static void graph_free(graph_t *g) {
  if (g->owned) {
    free(g->off);
    free(g->idx);
    free(g->w);
  }
  memset(g, 0, sizeof(*g));
}

/* K_i = sum of the weights in row i (Section 3); a self-loop entry counts once. */
static void weighted_degrees(const graph_t *g, int64_t *K) {
  for (int32_t i = 0; i < g->n; ++i) {
    int64_t s = 0;
    for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) s += g->w[e];
    K[i] = s;
  }
}

/* Dense renumbering in ascending order of the old id; returns the new count. */
static int32_t renumber(int32_t n, const int32_t *C, int32_t *dense_of) {
  for (int32_t c = 0; c < n; ++c) dense_of[c] = -1;
  for (int32_t i = 0; i < n; ++i) dense_of[C[i]] = 0;
  int32_t m = 0;
  for (int32_t c = 0; c < n; ++c)
    if (dense_of[c] == 0) dense_of[c] = m++;
  return m;
}

/* Canonical labels: communities numbered in order of first appearance (ascending
 * smallest member), so equal label arrays mean equal partitions. */
static void canonical(int32_t n, const int32_t *C, int32_t *out) {
  int32_t top = 0;
  for (int32_t i = 0; i < n; ++i)
    if (C[i] + 1 > top) top = C[i] + 1;
  int32_t *map = (int32_t *)malloc(sizeof(int32_t) * (size_t)(top > 0 ? top : 1));
  for (int32_t c = 0; c < top; ++c) map[c] = -1;
  int32_t m = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (map[C[i]] < 0) map[C[i]] = m++;
    out[i] = map[C[i]];
  }
  free(map);
}

void oracle_canonical(int32_t n, const int32_t *C, int32_t *out) { canonical(n, C, out); }

/* ------------------------------------------------------------------------------ */
/* One synchronous local-moving sweep                                               */
/* ------------------------------------------------------------------------------ */

typedef struct {
  const graph_t *g;
  int algo;              /* OR_ALGO_LPA, OR_ALGO_MOVE, OR_ALGO_REFINE */
  int mode, k;
  int64_t L;
  const int32_t *C;      /* keys are C[j] */
  const int32_t *bound;  /* refinement only: C_B */
  const int64_t *K;      /* weighted degree of each vertex */
  const int64_t *Sig;    /* Sigma per community (C's ids) */
  const int32_t *size;   /* members per community */
  int64_t W;             /* total weight = 2m */
  int one_scan;          /* LPA, 1-scan variant: decide from the sketch's values */
} sweep_t;

/* The best move of vertex i.  Returns the target (== C[i] if there is none) and
 * writes the integer gain of that move to *gain (0 when there is none). */
static int32_t decide_vertex(const sweep_t *s, int32_t i, uint32_t *kbuf, uint32_t *wbuf,
                             uint8_t *ubuf, pair_t *cbuf, int64_t *gain) {
  const graph_t *g = s->g;
  int64_t lo = g->off[i], hi = g->off[i + 1], n = hi - lo;
  int32_t d = s->C[i];
  *gain = 0;
  /* the stream: every neighbour j, key C[j] (reading R1); self excluded; in the
   * refinement only neighbours with the same bound (Algorithm 1 early exits) */
  for (int64_t e = 0; e < n; ++e) {
    int32_t j = g->idx[lo + e];
    kbuf[e] = (uint32_t)s->C[j];
    wbuf[e] = g->w[lo + e];
    ubuf[e] = (uint8_t)(j != i);
    if (s->algo == OR_ALGO_REFINE && s->bound[j] != s->bound[i]) ubuf[e] = 0;
  }
  /* pass 1: candidate communities */
  int64_t small_vd = 0;
  int nc = s->mode == OR_MODE_EXACT ? exact_table(kbuf, wbuf, ubuf, n, cbuf)
           : s->mode == OR_MODE_SMALL
               ? small_table(kbuf, wbuf, ubuf, n, s->k, (uint32_t)d, cbuf, &small_vd)
               : stream_sketch(kbuf, wbuf, ubuf, n, s->mode, s->k, s->L, cbuf);
  if (nc == 0) return d;
  if (s->algo == OR_ALGO_LPA && s->one_scan) {
    /* The 1-scan variant of LPA (Section 4.3): no second pass; the label whose
     * accumulated sketch value is largest (ties to the lowest label). */
    int32_t best = -1;
    int64_t bv = -1;
    for (int x = 0; x < nc; ++x) {
      int32_t c = (int32_t)cbuf[x].key;
      int64_t v = (int64_t)cbuf[x].val;
      if (v > bv || (v == bv && c < best)) {
        bv = v;
        best = c;
      }
    }
    return best;
  }
  int64_t Kid = 0;
  int64_t *Kic = (int64_t *)malloc(sizeof(int64_t) * (size_t)nc);
  if (s->mode == OR_MODE_SMALL) {
    /* the small table's values are the linking weights (no second pass), K_{i->d}
     * by mod-based lookup */
    for (int x = 0; x < nc; ++x) Kic[x] = cbuf[x].val;
    Kid = small_vd;
  } else {
    /* pass 2: exact linking weights K_{i->c} of the candidates and K_{i->d} */
    for (int x = 0; x < nc; ++x) cbuf[x].val = 0;
    for (int x = 0; x < nc; ++x) Kic[x] = 0;
    for (int64_t e = 0; e < n; ++e) {
      if (!ubuf[e]) continue;
      for (int x = 0; x < nc; ++x)
        if (cbuf[x].key == kbuf[e]) Kic[x] += wbuf[e];
      if (kbuf[e] == (uint32_t)d) Kid += wbuf[e];
    }
  }
  int32_t best = -1;
  if (s->algo == OR_ALGO_LPA) {
    /* LPA: the label with the largest total weight; ties to the lowest label */
    int64_t bw = -1;
    for (int x = 0; x < nc; ++x) {
      int32_t c = (int32_t)cbuf[x].key;
      if (Kic[x] > bw || (Kic[x] == bw && c < best)) {
        bw = Kic[x];
        best = c;
      }
    }
    free(Kic);
    return best;
  }
  /* Louvain / Leiden: Eq. 2 times W^2/2 (W = 2m):
   *   dQ = (1/m)(K_ic - K_id) - K_i/(2m^2) (K_i + Sigma_c - Sigma_d)
   *   G  = dQ W^2/2 = W (K_ic - K_id) - K_i (K_i + Sigma_c - Sigma_d)        */
  int64_t Ki = s->K[i], bestG = 0;
  for (int x = 0; x < nc; ++x) {
    int32_t c = (int32_t)cbuf[x].key;
    if (c == d) continue;
    int64_t G = s->W * (Kic[x] - Kid) - Ki * (Ki + s->Sig[c] - s->Sig[d]);
    if (G <= 0) continue;
    if (best < 0 || G > bestG || (G == bestG && c < best)) {
      bestG = G;
      best = c;
    }
  }
  free(Kic);
  if (best < 0) return d;
  *gain = bestG;
  return best;
}

static void sweep(const sweep_t *s, int32_t *Cnew, int64_t *gain) {
  const graph_t *g = s->g;
  int64_t maxdeg = 0;
  for (int32_t i = 0; i < g->n; ++i)
    if (g->off[i + 1] - g->off[i] > maxdeg) maxdeg = g->off[i + 1] - g->off[i];
  int64_t cap = maxdeg > 0 ? maxdeg : 1;
#pragma omp parallel
  {
    uint32_t *kb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    uint32_t *wb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    uint8_t *ub = (uint8_t *)malloc((size_t)cap);
    pair_t *cb = (pair_t *)malloc(sizeof(pair_t) * (size_t)(cap > KMAX ? cap : KMAX));
#pragma omp for schedule(dynamic, 256)
    for (int32_t i = 0; i < g->n; ++i) Cnew[i] = decide_vertex(s, i, kb, wb, ub, cb, &gain[i]);
    free(kb);
    free(wb);
    free(ub);
    free(cb);
  }
}

/* Reading R7: keep only the moves that go in this sweep's direction
 * (dir < 0: to a lower id, dir > 0: to a higher id, 0: all). */
static int64_t apply_direction(int32_t n, const int32_t *C, int32_t *Cnew, int dir) {
  int64_t moved = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (Cnew[i] == C[i]) continue;
    if ((dir < 0 && Cnew[i] > C[i]) || (dir > 0 && Cnew[i] < C[i]))
      Cnew[i] = C[i];
    else
      moved += 1;
  }
  return moved;
}

/* exported: one sweep, for iteration-level parity checks.  Cnew receives the
 * applied moves; gain receives the gain of every vertex's best move (also when
 * the direction rule keeps the vertex in place). */
int oracle_move_sweep(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w, int algo,
                      int mode, int k, int64_t chunk_len, const int32_t *C, const int32_t *bound,
                      const int64_t *K, const int64_t *Sigma, const int32_t *size, int64_t W,
                      int direction, int one_scan, int32_t *Cnew, int64_t *gain) {
  if (k < 1 || (k > KMAX && mode != OR_MODE_SMALL) || chunk_len < 1) return -1;
  graph_t g = {n, off[n], (int64_t *)off, (int32_t *)idx, (uint32_t *)w, 0};
  sweep_t s = {&g, algo, mode, k, chunk_len, C, bound, K, Sigma, size, W, one_scan};
  sweep(&s, Cnew, gain);
  if (algo == OR_ALGO_MOVE) apply_direction(n, C, Cnew, direction);
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Leiden refinement (Section 4.2, reading R10)                                     */
/* ------------------------------------------------------------------------------ */

static void refine(const graph_t *g, const int32_t *bound, const int64_t *K, int64_t W, int mode,
                   int k, int64_t L, int32_t *R) {
  int32_t n = g->n;
  int32_t *single = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *ones = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *prop = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int64_t *gain = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int32_t *nprop = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  int32_t *from = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t i = 0; i < n; ++i) {
    single[i] = i; /* every vertex starts in its own sub-community */
    ones[i] = 1;
  }
  /* Sigma of a singleton sub-community is K of its vertex */
  sweep_t s = {g, OR_ALGO_REFINE, mode, k, L, single, bound, K, K, ones, W, 0};
  sweep(&s, prop, gain);
  for (int32_t i = 0; i < n; ++i)
    if (prop[i] != i) {
      nprop[prop[i]] += 1;
      from[prop[i]] = i;
    }
  for (int32_t i = 0; i < n; ++i) {
    int32_t t = prop[i];
    R[i] = i;
    if (t == i) continue;
    int ok = nprop[i] == 0 || (nprop[i] == 1 && from[i] == t && t < i);
    if (ok) R[i] = t;
  }
  free(single);
  free(ones);
  free(prop);
  free(gain);
  free(nprop);
  free(from);
}

int oracle_refine(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                  const int32_t *bound, const int64_t *K, int64_t W, int mode, int k,
                  int64_t chunk_len, int32_t *R) {
  graph_t g = {n, off[n], (int64_t *)off, (int32_t *)idx, (uint32_t *)w, 0};
  refine(&g, bound, K, W, mode, k, chunk_len, R);
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Aggregation (Section 4.1 Fig. 3; Section 4.2; reading R9, R11)                   */
/* ------------------------------------------------------------------------------ */

/* G' of g under the dense membership D (values in [0, m)).  Community c's stream is
 * the rows of its members in ascending vertex id, each in CSR order, with key D[j]. */
static void aggregate(const graph_t *g, const int32_t *D, int32_t m, int mode, int k, int64_t L,
                      int symmetric, graph_t *out) {
  int32_t n = g->n;
  /* members of each community in ascending vertex id (stable counting sort) */
  int64_t *start = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
  int32_t *mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t i = 0; i < n; ++i) start[D[i] + 1] += 1;
  for (int32_t c = 0; c < m; ++c) start[c + 1] += start[c];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  for (int32_t c = 0; c < m; ++c) fill[c] = start[c];
  for (int32_t i = 0; i < n; ++i) mem[fill[D[i]]++] = i;
  free(fill);

  pair_t **rows = (pair_t **)malloc(sizeof(pair_t *) * (size_t)(m > 0 ? m : 1));
  int64_t *rlen = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t c = 0; c < m; ++c) {
    int64_t len = 0;
    for (int64_t t = start[c]; t < start[c + 1]; ++t) len += g->off[mem[t] + 1] - g->off[mem[t]];
    uint32_t *kb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(len > 0 ? len : 1));
    uint32_t *wb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(len > 0 ? len : 1));
    uint8_t *ub = (uint8_t *)malloc((size_t)(len > 0 ? len : 1));
    int64_t pos = 0;
    for (int64_t t = start[c]; t < start[c + 1]; ++t) {
      int32_t i = mem[t];
      for (int64_t e = g->off[i]; e < g->off[i + 1]; ++e) {
        kb[pos] = (uint32_t)D[g->idx[e]];
        wb[pos] = g->w[e];
        ub[pos] = 1;
        ++pos;
      }
    }
    int64_t cap = mode == OR_MODE_EXACT ? (len > 0 ? len : 1) : k;
    pair_t *r = (pair_t *)malloc(sizeof(pair_t) * (size_t)cap);
    int cnt = mode == OR_MODE_EXACT ? exact_table(kb, wb, ub, len, r)
                                    : stream_sketch(kb, wb, ub, len, mode, k, L, r);
    rows[c] = r;
    rlen[c] = cnt;
    free(kb);
    free(wb);
    free(ub);
  }
  free(start);
  free(mem);

  if (symmetric && mode != OR_MODE_EXACT) {
    /* union of the kept pairs in both directions; weight max(v_st, v_ts) */
    int64_t tot = 0;
    for (int32_t c = 0; c < m; ++c) tot += rlen[c];
    int64_t *cnt2 = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    for (int32_t s = 0; s < m; ++s)
      for (int64_t x = 0; x < rlen[s]; ++x) {
        cnt2[s + 1] += 1;
        if ((int32_t)rows[s][x].key != s) cnt2[rows[s][x].key + 1] += 1;
      }
    for (int32_t c = 0; c < m; ++c) cnt2[c + 1] += cnt2[c];
    pair_t *all = (pair_t *)malloc(sizeof(pair_t) * (size_t)(cnt2[m] > 0 ? cnt2[m] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    for (int32_t c = 0; c < m; ++c) fill[c] = cnt2[c];
    for (int32_t s = 0; s < m; ++s)
      for (int64_t x = 0; x < rlen[s]; ++x) {
        uint32_t t = rows[s][x].key, v = rows[s][x].val;
        all[fill[s]++] = (pair_t){t, v};
        if ((int32_t)t != s) all[fill[t]++] = (pair_t){(uint32_t)s, v};
      }
    (void)tot;
    for (int32_t s = 0; s < m; ++s) {
      free(rows[s]);
      int64_t a = cnt2[s], b = cnt2[s + 1];
      qsort(all + a, (size_t)(b - a), sizeof(pair_t), cmp_pair_key);
      int64_t r = 0;
      pair_t *seg = all + a;
      for (int64_t x = 0; x < b - a; ++x) {
        if (r > 0 && seg[r - 1].key == seg[x].key) {
          if (seg[x].val > seg[r - 1].val) seg[r - 1].val = seg[x].val;
        } else {
          seg[r++] = seg[x];
        }
      }
      pair_t *row = (pair_t *)malloc(sizeof(pair_t) * (size_t)(r > 0 ? r : 1));
      memcpy(row, seg, sizeof(pair_t) * (size_t)r);
      rows[s] = row;
      rlen[s] = r;
    }
    free(all);
    free(fill);
    free(cnt2);
  }

  out->n = m;
  out->off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
  out->off[0] = 0;
  for (int32_t c = 0; c < m; ++c) out->off[c + 1] = out->off[c] + rlen[c];
  out->nnz = out->off[m];
  out->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(out->nnz > 0 ? out->nnz : 1));
  out->w = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(out->nnz > 0 ? out->nnz : 1));
  out->owned = 1;
  for (int32_t c = 0; c < m; ++c) {
    for (int64_t x = 0; x < rlen[c]; ++x) {
      out->idx[out->off[c] + x] = (int32_t)rows[c][x].key;
      out->w[out->off[c] + x] = rows[c][x].val;
    }
    free(rows[c]);
  }
  free(rows);
  free(rlen);
}

/* exported: aggregated graph under a dense membership; returns nnz' or -1.  Call
 * once with out arrays NULL to get the size, then again with arrays of that size. */
int64_t oracle_aggregate(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                         const int32_t *D, int32_t m, int mode, int k, int64_t chunk_len,
                         int symmetric, int64_t *out_off, int32_t *out_idx, uint32_t *out_w) {
  graph_t g = {n, off[n], (int64_t *)off, (int32_t *)idx, (uint32_t *)w, 0};
  graph_t a;
  memset(&a, 0, sizeof(a));
  aggregate(&g, D, m, mode, k, chunk_len, symmetric, &a);
  int64_t nnz = a.nnz;
  if (out_off) memcpy(out_off, a.off, sizeof(int64_t) * ((size_t)m + 1));
  if (out_idx) memcpy(out_idx, a.idx, sizeof(int32_t) * (size_t)nnz);
  if (out_w) memcpy(out_w, a.w, sizeof(uint32_t) * (size_t)nnz);
  graph_free(&a);
  return nnz;
}

/* ------------------------------------------------------------------------------ */
/* Modularity, Eq. 1 (reading R12)                                                  */
/* ------------------------------------------------------------------------------ */

double oracle_modularity(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                         const int32_t *C) {
  double W = 0.0;
  double *sig = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));  /* sigma_c */
  double *tot = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));  /* Sigma_c */
  for (int32_t i = 0; i < n; ++i) {
    if (C[i] < 0 || C[i] >= n) {
      free(sig);
      free(tot);
      return NAN;
    }
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
      W += (double)w[e];
      tot[C[i]] += (double)w[e];
      if (C[idx[e]] == C[i]) sig[C[i]] += (double)w[e];
    }
  }
  double Q = 0.0;
  if (W > 0.0)
    for (int32_t c = 0; c < n; ++c) Q += sig[c] / W - (tot[c] / W) * (tot[c] / W);
  free(sig);
  free(tot);
  return Q;
}

/* ------------------------------------------------------------------------------ */
/* Drivers                                                                          */
/* ------------------------------------------------------------------------------ */

static void set_threads(const or_params *p) {
#ifdef _OPENMP
  if (p->threads > 0) omp_set_num_threads(p->threads);
#else
  (void)p;
#endif
}

/* The rows of aggregation: as the moving mode says (Section 4.1: the same sketch;
 * the small table of Appendix A.2 aggregates exactly), or decoupled from it, exact or
 * Algorithm 1 with k_aggregate slots, to measure each phase's share of a sketch's
 * modularity loss. */
static int agg_mode_of(const or_params *p) {
  if (p->aggregation == 1) return OR_MODE_EXACT;
  if (p->aggregation == 2) return OR_MODE_ALG1;
  return p->mode == OR_MODE_SMALL ? OR_MODE_EXACT : p->mode;
}

static int check_params(const or_params *p) {
  if (p->aggregation < 0 || p->aggregation > 2) return -1;
  if (p->chunk_len < 1) return -1;
  if (p->mode == OR_MODE_SMALL) { /* k: slots of the small table */
    if (p->k < 1) return -6;
  } else if (p->k < 1 || p->k > KMAX) {
    return -6;
  }
  if (agg_mode_of(p) != OR_MODE_EXACT && (p->k_aggregate < 1 || p->k_aggregate > KMAX)) return -6;
  return 0;
}

/* LPA (Section 3.5, Section 4.3): synchronous sweeps until at most tau*N labels
 * change or max_iterations sweeps have run. */
int oracle_lpa(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
               const or_params *p, int32_t *labels, or_stats *st) {
  int rc = check_params(p);
  if (rc) return rc;
  set_threads(p);
  graph_t g = {n, off[n], (int64_t *)off, (int32_t *)idx, (uint32_t *)w, 0};
  size_t sz = (size_t)(n > 0 ? n : 1);
  int32_t *C = (int32_t *)malloc(sizeof(int32_t) * sz);
  int32_t *Cn = (int32_t *)malloc(sizeof(int32_t) * sz);
  int64_t *gain = (int64_t *)malloc(sizeof(int64_t) * sz);
  for (int32_t i = 0; i < n; ++i) C[i] = i;
  memset(st, 0, sizeof(*st));
  for (int it = 0; it < p->max_iterations; ++it) {
    sweep_t s = {&g, OR_ALGO_LPA, p->mode, p->k, p->chunk_len, C, NULL, NULL, NULL, NULL, 0,
                 p->one_scan};
    sweep(&s, Cn, gain);
    int64_t moved = 0;
    for (int32_t i = 0; i < n; ++i) moved += Cn[i] != C[i];
    int32_t *t = C;
    C = Cn;
    Cn = t;
    st->iterations += 1;
    st->edges_scanned += g.nnz;
    st->moved_last = moved;
    if ((double)moved <= p->tolerance * (double)n) break;
  }
  canonical(n, C, labels);
  int32_t m = 0;
  for (int32_t i = 0; i < n; ++i)
    if (labels[i] + 1 > m) m = labels[i] + 1;
  st->communities = m;
  st->passes = 1;
  free(C);
  free(Cn);
  free(gain);
  return 0;
}

/* The local-moving phase of one pass (reading R7).  C holds the starting
 * membership and receives the result. */
static void local_moving(const graph_t *g, const or_params *p, int64_t W, const int64_t *K,
                         int32_t *C, double tol, or_stats *st) {
  int32_t n = g->n;
  size_t sz = (size_t)(n > 0 ? n : 1);
  int64_t *Sig = (int64_t *)calloc(sz, sizeof(int64_t));
  int32_t *size = (int32_t *)calloc(sz, sizeof(int32_t));
  int32_t *Cn = (int32_t *)malloc(sizeof(int32_t) * sz);
  int64_t *gain = (int64_t *)malloc(sizeof(int64_t) * sz);
  for (int it = 0; it < p->max_iterations; ++it) {
    /* Sigma_c and sizes of the current membership (Section 3.1) */
    memset(Sig, 0, sizeof(int64_t) * sz);
    memset(size, 0, sizeof(int32_t) * sz);
    for (int32_t i = 0; i < n; ++i) {
      Sig[C[i]] += K[i];
      size[C[i]] += 1;
    }
    sweep_t s = {g, OR_ALGO_MOVE, p->mode, p->k, p->chunk_len, C, NULL, K, Sig, size, W, 0};
    sweep(&s, Cn, gain);
    int64_t proposed = 0;
    uint64_t sumG = 0;
    for (int32_t i = 0; i < n; ++i)
      if (Cn[i] != C[i]) {
        proposed += 1;
        sumG += (uint64_t)gain[i];
      }
    st->iterations += 1;
    st->edges_scanned += g->nnz;
    if (proposed == 0) {
      st->moved_last = 0;
      break;
    }
    st->moved_last = apply_direction(n, C, Cn, (it % 2 == 0) ? -1 : 1);
    memcpy(C, Cn, sizeof(int32_t) * (size_t)n);
    if (2.0 * (double)sumG <= tol * (double)W * (double)W) break;
  }
  free(Sig);
  free(size);
  free(Cn);
  free(gain);
}

/* Louvain (Section 3.3, Section 4.1). */
int oracle_louvain(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                   const or_params *p, int32_t *labels, or_stats *st) {
  int rc = check_params(p);
  if (rc) return rc;
  if (p->one_scan) return -6; /* the 1-scan variant is defined for LPA only */
  set_threads(p);
  memset(st, 0, sizeof(*st));
  graph_t g = {n, off[n], (int64_t *)off, (int32_t *)idx, (uint32_t *)w, 0};
  size_t sz = (size_t)(n > 0 ? n : 1);
  int64_t *K = (int64_t *)malloc(sizeof(int64_t) * sz);
  weighted_degrees(&g, K);
  int64_t W = 0;
  for (int32_t i = 0; i < n; ++i) W += K[i];
  int32_t *top = (int32_t *)malloc(sizeof(int32_t) * sz);
  for (int32_t v = 0; v < n; ++v) top[v] = v;
  double tol = p->tolerance;
  for (int pass = 0; pass < p->max_passes; ++pass) {
    int32_t nl = g.n;
    size_t szl = (size_t)(nl > 0 ? nl : 1);
    int32_t *C = (int32_t *)malloc(sizeof(int32_t) * szl);
    for (int32_t i = 0; i < nl; ++i) C[i] = i;
    local_moving(&g, p, W, K, C, tol, st);
    st->passes += 1;
    int32_t *dense = (int32_t *)malloc(sizeof(int32_t) * szl);
    int32_t m = renumber(nl, C, dense);
    for (int32_t v = 0; v < n; ++v) top[v] = dense[C[top[v]]];
    int last = pass == p->max_passes - 1 || (double)m > p->aggregation_tolerance * (double)nl;
    if (!last) {
      int32_t *D = (int32_t *)malloc(sizeof(int32_t) * szl);
      for (int32_t i = 0; i < nl; ++i) D[i] = dense[C[i]];
      graph_t a;
      aggregate(&g, D, m, agg_mode_of(p), p->k_aggregate, p->chunk_len, 0, &a);
      int64_t *K2 = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
      for (int32_t i = 0; i < nl; ++i) K2[D[i]] += K[i];
      free(K);
      K = K2;
      graph_free(&g);
      g = a;
      free(D);
      tol /= p->tolerance_drop;
    }
    free(C);
    free(dense);
    if (last) break;
  }
  canonical(n, top, labels);
  int32_t m = 0;
  for (int32_t v = 0; v < n; ++v)
    if (labels[v] + 1 > m) m = labels[v] + 1;
  st->communities = m;
  graph_free(&g);
  free(K);
  free(top);
  return 0;
}

/* Leiden (Section 3.4, Section 4.2). */
int oracle_leiden(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                  const or_params *p, int32_t *labels, or_stats *st) {
  int rc = check_params(p);
  if (rc) return rc;
  if (p->one_scan) return -6; /* the 1-scan variant is defined for LPA only */
  set_threads(p);
  memset(st, 0, sizeof(*st));
  graph_t g = {n, off[n], (int64_t *)off, (int32_t *)idx, (uint32_t *)w, 0};
  size_t sz = (size_t)(n > 0 ? n : 1);
  int64_t *K = (int64_t *)malloc(sizeof(int64_t) * sz);
  weighted_degrees(&g, K);
  int64_t W = 0;
  for (int32_t i = 0; i < n; ++i) W += K[i];
  int32_t *top = (int32_t *)malloc(sizeof(int32_t) * sz);
  for (int32_t v = 0; v < n; ++v) top[v] = v;
  int32_t *C = (int32_t *)malloc(sizeof(int32_t) * sz);
  for (int32_t i = 0; i < n; ++i) C[i] = i;
  double tol = p->tolerance;
  for (int pass = 0; pass < p->max_passes; ++pass) {
    int32_t nl = g.n;
    size_t szl = (size_t)(nl > 0 ? nl : 1);
    local_moving(&g, p, W, K, C, tol, st);
    st->passes += 1;
    int32_t *R = (int32_t *)malloc(sizeof(int32_t) * szl);
    refine(&g, C, K, W, p->mode, p->k, p->chunk_len, R);
    int32_t *denseR = (int32_t *)malloc(sizeof(int32_t) * szl);
    int32_t m = renumber(nl, R, denseR);
    int last = pass == p->max_passes - 1 || (double)m > p->aggregation_tolerance * (double)nl;
    if (last) {
      for (int32_t v = 0; v < n; ++v) top[v] = C[top[v]];
      free(R);
      free(denseR);
      break;
    }
    int32_t *denseC = (int32_t *)malloc(sizeof(int32_t) * szl);
    renumber(nl, C, denseC);
    int32_t *D = (int32_t *)malloc(sizeof(int32_t) * szl);
    for (int32_t i = 0; i < nl; ++i) D[i] = denseR[R[i]];
    for (int32_t v = 0; v < n; ++v) top[v] = D[top[v]];
    graph_t a;
    aggregate(&g, D, m, agg_mode_of(p), p->k_aggregate, p->chunk_len, 1, &a);
    int64_t *K2 = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    int32_t *C2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    for (int32_t i = 0; i < nl; ++i) {
      K2[D[i]] += K[i];
      C2[D[i]] = denseC[C[i]]; /* reading R11: start in the bound community */
    }
    free(K);
    K = K2;
    free(C);
    C = C2;
    graph_free(&g);
    g = a;
    free(R);
    free(denseR);
    free(denseC);
    free(D);
    tol /= p->tolerance_drop;
  }
  canonical(n, top, labels);
  int32_t m = 0;
  for (int32_t v = 0; v < n; ++v)
    if (labels[v] + 1 > m) m = labels[v] + 1;
  st->communities = m;
  graph_free(&g);
  free(K);
  free(C);
  free(top);
  return 0;
}
