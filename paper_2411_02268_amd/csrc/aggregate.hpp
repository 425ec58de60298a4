// Renumbering, aggregation, modularity and small per-vertex kernels (aggregate.hip).
#pragma once
#include "common.hpp"

namespace mgcd {

// dense[c] for every used id c of C (ascending old id); D[i] = dense[C[i]]; returns m.
// Batched runs: only vertices whose graph has keep[gid[i]] count; the others get
// D[i] = -1.  dense_out (optional, n+1 entries) receives the exclusive prefix of the
// used flags (dense_out[c] = new id of c; dense_out[n] = m).
int32_t renumber(const int32_t *C, int32_t n, int32_t *D, Arena &a, hipStream_t st,
                 const int32_t *gid = nullptr, const uint8_t *keep = nullptr,
                 int64_t *dense_out = nullptr);

// Aggregated graph of g under the dense membership D (values in [0, m), or -1 for a
// vertex left out, together with its whole row).
// out_off: [m+1]; out_idx/out_w: capacity g.nnz.  Returns the entry count.
// Louvain (symmetric=0): a community's row is the sketch (or exact sums) of the
// stream of its members' rows, members in ascending id.  Leiden (symmetric=1): the
// kept pairs in both directions, weight max(v_st, v_ts).
int64_t aggregate(const Graph &g, const int32_t *D, int32_t m, int mode, int k, int64_t L,
                  int symmetric, int64_t *out_off, int32_t *out_idx, uint32_t *out_w, Arena &a,
                  hipStream_t st);
size_t aggregate_ws_bytes(int32_t n, int64_t nnz, int mode, int k, int64_t L, bool symmetric);

// K'[c] = sum of K[i] over D[i] == c.
void launch_group_sums(const int32_t *D, const uint32_t *K, uint32_t *Kout, int32_t n, int32_t m,
                       hipStream_t st);
// out[v] = map[in[v]] for v < n (in may alias out).
void launch_compose(const int32_t *in, const int32_t *map, int32_t *out, int32_t n, hipStream_t st);
// out[map[i]] = val[i]  (all i with the same map[i] write the same value).
void launch_scatter_labels(const int32_t *map, const int32_t *val, int32_t *out, int32_t n,
                           hipStream_t st);

// K[i] = row sums (uint32) and *W = their total (device uint64).  Uses nnz + 1
// int64 of transient workspace.
void launch_degrees(const Graph &g, uint32_t *K, unsigned long long *W, Arena &a, hipStream_t st);
size_t degrees_ws_bytes(int64_t nnz);

// Storage copy of a graph for local moving: vertices laid out in descending degree
// (ties: ascending id), each row's entries unchanged and in their order, indices
// translated to positions.  perm[p] = vertex at position p, pos[v] = position of v,
// Kp[p] = K[perm[p]].  Arrays are taken from `a` (storage_ws_bytes of them).
struct StorageCopy {
  Graph g;
  int32_t *perm, *pos;
  uint32_t *Kp;
};
StorageCopy storage_copy(const Graph &g, const uint32_t *K, Arena &a, hipStream_t st);
size_t storage_ws_bytes(int32_t n, int64_t nnz);

// Canonical labels: communities numbered in order of their smallest vertex.
// Returns the number of communities (synchronises the stream).
int32_t canonical(const int32_t *C, int32_t n, int32_t *out, Arena &a, hipStream_t st);

// Integers of Eq. 1: I = weight of intra-community entries, S2 = sum of Sigma_c^2,
// accumulated in SPREAD copies: terms[2c] (parts of I) and terms[2c + 1] (parts of S2).
void modularity_terms(const Graph &g, const int32_t *C, const uint32_t *K,
                      unsigned long long *terms /* device [2 * SPREAD] */, Arena &a, hipStream_t st);

// *flag = 1 when some C[i] (i < n) lies outside [0, limit).
void launch_check_labels(const int32_t *C, int64_t n, int64_t limit, unsigned long long *flag,
                         hipStream_t st);

// Validation of a CSR; sets flags[0] when something is wrong.
void launch_validate(const Graph &g, unsigned long long *flags, hipStream_t st);

}  // namespace mgcd
