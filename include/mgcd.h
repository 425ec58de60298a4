/*
 * mgcd.h -- C ABI of the MI355X (gfx950) community-detection library built on
 * weighted Misra-Gries (MG) sketches (Sahu, arXiv 2411.02268).
 *
 * Every entry point works on an undirected graph in CSR form whose arrays live in
 * device memory (the caller's allocation, e.g. PyTorch).  All work is ordered on
 * the caller's HIP stream (passed as `void *`, a hipStream_t).  The library never
 * allocates device memory in these calls: the caller passes one workspace buffer
 * of at least mgcd_workspace_bytes() bytes.  Calls that use different workspaces
 * and streams may run concurrently; calls that share a workspace must not.
 *
 * Return codes: MGCD_OK (0) or a negative error; mgcd_last_error() then returns a
 * message (thread-local).  No C++ exception crosses this boundary.
 */
#ifndef MGCD_H
#define MGCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MGCD_OK = 0,
  MGCD_E_ARG = -1,         /* null pointer, bad size or bad parameter value        */
  MGCD_E_GRAPH = -2,       /* the CSR failed validation (only with validate=1)      */
  MGCD_E_OVERFLOW = -3,    /* total edge weight W >= 2^31                           */
  MGCD_E_WORKSPACE = -4,   /* workspace smaller than mgcd_workspace_bytes()         */
  MGCD_E_HIP = -5,         /* a HIP runtime call failed                             */
  MGCD_E_UNSUPPORTED = -6  /* k, mode or algorithm not built                        */
};

/* Sketch update rule used by local moving, refinement and aggregation. */
enum {
  MGCD_MODE_EXACT = 0,  /* exact per-vertex table (the hashtable of Section 4, Fig. 1) */
  MGCD_MODE_ALG1 = 1,   /* Algorithm 1, conditional subtraction (Appendix A.1)       */
  MGCD_MODE_UNCOND = 2, /* unconditional subtraction (Section 4.1, first variant)    */
  MGCD_MODE_STD = 3,    /* textbook weighted MG (subtract min(w, smallest value))     */
  MGCD_MODE_BM = 4,     /* weighted Boyer-Moore (Section 4.1): Algorithm 1 with k = 1
                           for local moving and refinement and k = 4 for aggregation;
                           the k and k_aggregate fields are ignored                   */
  MGCD_MODE_SMALL = 5   /* small mod-based table (Appendix A.2): k (1 .. 2^30) slots per
                           vertex; key c counts in slot c mod k, a slot stands for the
                           first key (in row order) that reached it with the summed
                           weight of every key that did, and K_{i->d} is the sum in
                           d's slot; no second pass; aggregation is exact (k_aggregate
                           ignored)                                                   */
};

enum { MGCD_ALGO_LPA = 0, MGCD_ALGO_LOUVAIN = 1, MGCD_ALGO_LEIDEN = 2 };

/* How aggregation builds a super-vertex's row (mgcd_params.aggregation). */
enum {
  MGCD_AGG_AS_MODE = 0, /* as `mode` says (the method of Section 4.1: the same sketch as
                           local moving, k_aggregate slots; exact in the exact and
                           small-table modes)                                        */
  MGCD_AGG_EXACT = 1,   /* exact rows (every linked community with its full weight)  */
  MGCD_AGG_SKETCH = 2   /* Algorithm 1 with k_aggregate slots, whatever `mode` is     */
};

/* An undirected graph G = (V, E, w) (Section 3).  Every undirected edge {i, j}
 * appears as the entries i->j and j->i with equal weight; a self-loop appears once.
 * Layout: offsets[n+1] int64 (offsets[0] = 0, non-decreasing, offsets[n] = nnz);
 * indices[nnz] int32 in [0, n); weights[nnz] uint32 >= 1.  Device pointers, read
 * only; indices and weights 16-byte aligned (MGCD_E_ARG otherwise).  The sum W of
 * all weights (= 2m) must be below 2^31. */
typedef struct {
  int32_t n;
  int32_t reserved;
  int64_t nnz;
  const int64_t *offsets;
  const int32_t *indices;
  const uint32_t *weights;
} mgcd_csr;

typedef struct {
  int32_t mode;           /* MGCD_MODE_*                                              */
  int32_t k;              /* sketch slots for moving/refinement: 1, 2, 4, 8, 16, 32,
                             64, 128 or 256 (MGCD_MODE_SMALL: the table's slots,
                             1 .. 2^30)                                               */
  int32_t k_aggregate;    /* sketch slots for aggregation: 1, 2, 4, 8, 16, 32, 64,
                             128 or 256                                               */
  int32_t max_iterations; /* synchronous sweeps per pass (LPA: in total)              */
  int32_t max_passes;     /* Louvain/Leiden passes (levels)                            */
  int32_t validate;       /* 1: check the CSR on the device first (MGCD_E_GRAPH)      */
  int64_t chunk_len;      /* L: streams longer than L are sketched in chunks of L
                             positions, then merged (changes results; >= 1)          */
  double tolerance;       /* LPA: stop when <= tolerance*n labels change; Louvain/
                             Leiden: stop a pass when the summed gain of all
                             positive moves, as a modularity change, is <= tolerance */
  double tolerance_drop;  /* tolerance is divided by this after every pass           */
  double aggregation_tolerance; /* stop when a pass keeps more than this fraction of
                                   its vertices                                    */
  /* Schedule only: these choose which kernel and lane mapping takes a row and never
     change results.  0 selects the default. */
  int32_t row_lanes;      /* most lanes (chunks) a row takes in the row buckets: a
                             power of two up to 64 (default 64); rows of more chunks
                             take the long-row path                                  */
  int32_t exact_small;    /* exact mode: rows of at most this many entries use one
                             lane each (default 32)                                  */
  int32_t exact_lds;      /* exact mode: rows up to this use a 1024-slot LDS table
                             (default and maximum 512)                               */
  int32_t exact_lds_big;  /* exact mode: rows up to this use an 8192-slot LDS table
                             (default and maximum 4096); longer rows a global table  */
  int32_t direct_launch;  /* batched runs: 0 (default) issues each level's sweeps as
                             one captured HIP graph, 1 launches them one by one      */
  /* Changes results: */
  int32_t one_scan;       /* LPA only (Section 4.3, the "1-scan" variant): 1 decides
                             every vertex from its sketch, taking the label with the
                             largest accumulated value (ties: the lowest label) with
                             no second pass; 0 (default) runs the second pass.
                             Louvain/Leiden calls with 1 return MGCD_E_UNSUPPORTED;
                             the exact mode is unaffected (its table is exact).     */
  int32_t aggregation;    /* MGCD_AGG_*: 0 (default) aggregates as `mode` says; 1 and
                             2 decouple aggregation from local moving, to measure
                             how much of a sketch's modularity loss each phase
                             causes                                                 */
  /* Schedule only (never changes results): */
  int32_t storage_order;  /* level-0 local moving on a copy of the input with vertices
                             in descending degree (rows, their order and every
                             community id unchanged; the neighbours' labels that
                             sweeps gather share cache lines): 0 (default) when the
                             input has at least 2^26 entries, 1 never, 2 always      */
  int32_t short_rows;     /* MGCD_MODE_ALG1 / _STD with k <= 16: a row of at most k
                             entries holds at most k distinct keys, so its sketch never
                             loses weight and equals its exact table.  Such rows are
                             decided on the exact one-lane kernel: 0 (default) when the
                             level's average row has at most k entries, 1 never (the
                             sketch kernels take them), 2 always                     */
} mgcd_params;

typedef struct {
  int32_t iterations;     /* local-moving sweeps run, all passes                      */
  int32_t passes;         /* levels run                                               */
  int32_t communities;    /* communities in the output                                */
  int32_t reserved;
  int64_t edges_scanned;  /* CSR entries streamed by local-moving sweeps              */
  int64_t moved_last;     /* vertices that moved in the last sweep                    */
  float ms_local_move;    /* device time in local-moving sweeps                       */
  float ms_refine;        /* device time in Leiden refinement                         */
  float ms_aggregate;     /* device time in renumbering and aggregation               */
  float ms_total;         /* device time of the whole call                            */
  /* Level-0 local-moving sweeps, device time per kernel class (HIP events on the
     call's stream).  MG: [0] the main sweep kernel (every row the sketch takes:
     all rows but those that short_rows sends to the exact kernel, plus the chunk
     sketches of rows longer than 64 chunks), [1] the merge, second pass and
     decision of those long rows, [2] rows of at most k entries on the exact
     one-lane kernel (short_rows).  Exact: [0] rows of at most 32 entries, [1] LDS hash tables,
     [2] global hash tables. */
  int32_t l0_sweeps;
  int32_t reserved2;
  float ms_l0_kernel[3];
  float reserved3;
  /* Louvain/Leiden, level-0 sweeps: candidate communities c != d scored by the main
     sweep kernel (each needs its community total Sigma_c), summed over the sweeps. */
  int64_t l0_candidates;
} mgcd_stats;

/* Defaults for an algorithm: MG Algorithm 1, k = 8 (LPA, Louvain) or 16 (Leiden),
 * L = 128, 20 sweeps, 10 passes, tolerance 0.05 (LPA) or 0.01, drop 10,
 * aggregation tolerance 0.8, validate 0. */
void mgcd_default_params(int32_t algo, mgcd_params *p);

/* Workspace bytes for one run of `algo` on a graph of n vertices and nnz entries. */
size_t mgcd_workspace_bytes(int32_t algo, int32_t n, int64_t nnz, const mgcd_params *p);

/* Label Propagation (Section 3.5) with MG sketches (Section 4.3): every vertex
 * takes the label of largest total edge weight among its neighbours (self
 * excluded; candidates from a k-slot sketch, weights from a second pass; ties to
 * the lowest label); synchronous sweeps until at most tolerance*n labels change or
 * max_iterations sweeps.  communities_out: device int32[n], canonical labels
 * (communities numbered 0.. in order of their smallest vertex).  stats: host, may be
 * NULL.  The call returns after synchronising the stream. */
int lpa_run(const mgcd_csr *g, const mgcd_params *p, int32_t *communities_out, void *ws,
            size_t ws_bytes, mgcd_stats *stats, void *stream);

/* Louvain (Section 3.3) with MG local moving and MG aggregation (Section 4.1,
 * Figs. 2-3); gains by Eq. 2 in exact integer form.  Arguments as lpa_run. */
int louvain_run(const mgcd_csr *g, const mgcd_params *p, int32_t *communities_out, void *ws,
                size_t ws_bytes, mgcd_stats *stats, void *stream);

/* Leiden (Section 3.4) with MG local moving, MG refinement and symmetric MG
 * aggregation (Section 4.2).  Arguments as lpa_run. */
int leiden_run(const mgcd_csr *g, const mgcd_params *p, int32_t *communities_out, void *ws,
               size_t ws_bytes, mgcd_stats *stats, void *stream);

/* Workspace bytes of modularity() for a graph of n vertices and nnz entries. */
size_t mgcd_modularity_workspace_bytes(int32_t n, int64_t nnz);

/* Modularity Q of a membership (Section 3.2, Eq. 1), summing over CSR entries
 * (a self-loop entry counts once; 2m = W).  communities: device int32[n], values
 * in [0, n).  q: host.  Synchronises the stream. */
int modularity(const mgcd_csr *g, const int32_t *communities, double *q, void *ws,
               size_t ws_bytes, void *stream);

/* Largest vertex count modularity_noalloc accepts. */
#define MGCD_NOALLOC_MAX_VERTICES (1 << 22)

/* modularity() for callers that cannot allocate device memory or pass a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, result and synchronisation as modularity(), minus
 * the workspace: the library works in a fixed device scratch array of its own,
 * 64 MiB + 128 KiB per device, set aside when the library is loaded on that device
 * and held until the process ends.  Graphs of more than MGCD_NOALLOC_MAX_VERTICES
 * vertices return MGCD_E_WORKSPACE before any device work.  The call allocates
 * nothing.  All calls on one device share its scratch: calls that overlap on one
 * device (other threads, other streams) race and must not be made; consecutive calls
 * are independent (each writes what it reads first). */
int modularity_noalloc(const mgcd_csr *g, const int32_t *communities, double *q, void *stream);

/* One synchronous local-moving sweep (the hot path on its own, for iteration-level
 * checks).  algo: MGCD_ALGO_LPA or MGCD_ALGO_LOUVAIN.  C: device int32[n], the
 * current membership (values in [0, n)).  C_new: device int32[n] receives the
 * moves allowed by `direction` (-1: to lower ids only, +1: higher only, 0: all).
 * gain: device int64[n] or NULL, the integer gain W(K_ic-K_id)-K_i(K_i+S_c-S_d) of
 * each vertex's best move (Louvain; 0 when none).  counters (host, may be NULL):
 * [moved, proposals, sum of gains].  Sigma/size are derived from C. */
int mgcd_move_sweep(const mgcd_csr *g, const mgcd_params *p, int32_t algo, const int32_t *C,
                    int32_t direction, int32_t *C_new, int64_t *gain, int64_t *counters,
                    void *ws, size_t ws_bytes, void *stream);

/* Leiden refinement on its own (Section 4.2): bound: device int32[n]; R: device
 * int32[n] receives each vertex's sub-community (a vertex id). */
int mgcd_refine(const mgcd_csr *g, const mgcd_params *p, const int32_t *bound, int32_t *R,
                void *ws, size_t ws_bytes, void *stream);

/* Aggregation on its own (Section 4.1 Fig. 3, Section 4.2): D: device int32[n]
 * dense membership in [0, m).  The aggregated CSR is written to out_offsets
 * (device int64[m+1]), out_indices and out_weights (device, capacity nnz entries;
 * the aggregate never has more entries than the input).  *out_nnz (host) receives
 * its entry count.  symmetric: 1 for Leiden's symmetric aggregation. */
int mgcd_aggregate(const mgcd_csr *g, const mgcd_params *p, const int32_t *D, int32_t m,
                   int32_t symmetric, int64_t *out_offsets, int32_t *out_indices,
                   uint32_t *out_weights, int64_t *out_nnz, void *ws, size_t ws_bytes,
                   void *stream);

/* Per-graph statistics of a batched run. */
typedef struct {
  int32_t iterations;     /* local-moving sweeps in which the graph took part         */
  int32_t passes;
  int32_t communities;
  int32_t reserved;
  int64_t edges_scanned;
  int64_t moved_last;
} mgcd_graph_stats;

/* Workspace bytes of a batched run over `count` graphs with total_n vertices and
 * total_nnz entries in all. */
size_t mgcd_workspace_bytes_batched(int32_t algo, int32_t count, int64_t total_n,
                                    int64_t total_nnz, const mgcd_params *p);

/* Batched LPA / Louvain: `count` independent graphs (graphs: host array of
 * descriptors of device CSRs) run together, one launch per sweep for all of them,
 * as one disjoint union with per-graph total weight, counters, convergence and
 * pass control.  Every graph's labels equal those of its own lpa_run/louvain_run
 * with the same parameters.  communities_out: host array of `count` device int32
 * arrays (n_g each).  per_graph: host array of `count` (may be NULL); total: host
 * (may be NULL).  Total vertices must be below 2^31.  Synchronises the stream. */
int lpa_run_batched(const mgcd_csr *graphs, int32_t count, const mgcd_params *p,
                    int32_t *const *communities_out, void *ws, size_t ws_bytes,
                    mgcd_graph_stats *per_graph, mgcd_stats *total, void *stream);
int louvain_run_batched(const mgcd_csr *graphs, int32_t count, const mgcd_params *p,
                        int32_t *const *communities_out, void *ws, size_t ws_bytes,
                        mgcd_graph_stats *per_graph, mgcd_stats *total, void *stream);

/* ---- serving: continuous batching of independent requests ------------------------
 *
 * A server runs whole lpa/louvain/leiden calls for a stream of graphs that arrive
 * over time.  It owns `slots` worker threads, each with its own HIP stream (default
 * priority) on the device that is current at creation, and carves each request's
 * workspace out of one caller-provided device arena (first fit, 256-byte aligned).
 * Requests are admitted in arrival order: the oldest waiting request starts as soon
 * as a slot is free and the arena has a free block of mgcd_workspace_bytes() for it,
 * so requests that arrive while others run are admitted as slots and memory free up,
 * and the work of admitted requests overlaps on the device.  A request's result is
 * identical to the same call made alone (each call is deterministic and shares no
 * state with the others).
 *
 * mgcd_server_create: arena = device pointer, 256-byte aligned, arena_bytes long,
 *   owned by the caller and untouched by anyone else until mgcd_server_destroy
 *   returns; slots in [1, 64]; algo MGCD_ALGO_*; params copied (NULL = defaults).
 *   *out receives the server.  Errors: MGCD_E_ARG, MGCD_E_UNSUPPORTED, MGCD_E_HIP.
 * mgcd_server_submit: g (host struct, copied; its device arrays and
 *   communities_out must stay valid and unmodified until the request is done, and
 *   the arrays must already hold their contents: the server's streams do not wait
 *   on the caller's stream).
 *   *ticket receives the request's id.  MGCD_E_WORKSPACE if the request's
 *   workspace exceeds the whole arena.  Never blocks on the device.
 * mgcd_server_poll: *state = 0 waiting for admission, 1 running, 2 done.
 * mgcd_server_wait: blocks until the request is done and returns its call's return
 *   code (its message through mgcd_last_error on this thread); stats (host, may be
 *   NULL) as the call filled it; times (host, may be NULL) = seconds since server
 *   creation of [submission, admission, completion].  The ticket is then released
 *   (a second wait or poll on it returns MGCD_E_ARG).
 * mgcd_server_info: counts of waiting and running requests, arena bytes in use and
 *   the peak (host pointers, each may be NULL).
 * mgcd_server_destroy: runs every submitted request to completion, joins the
 *   workers and destroys their streams; results not yet collected are dropped. */
typedef struct mgcd_server mgcd_server;
int mgcd_server_create(void *arena, size_t arena_bytes, int32_t slots, int32_t algo,
                       const mgcd_params *p, mgcd_server **out);
int mgcd_server_submit(mgcd_server *s, const mgcd_csr *g, int32_t *communities_out,
                       int64_t *ticket);
int mgcd_server_poll(mgcd_server *s, int64_t ticket, int32_t *state);
int mgcd_server_wait(mgcd_server *s, int64_t ticket, mgcd_stats *stats, double *times);
int mgcd_server_info(mgcd_server *s, int64_t *waiting, int64_t *running, size_t *bytes_in_use,
                     size_t *peak_bytes);
int mgcd_server_destroy(mgcd_server *s);

/* ---- serving by steps (Section 3.2 sweeps as the unit of scheduling) --------------
 *
 * A stepped server keeps every resident request's state on the device and advances
 * all of them together: one step is up to sweeps_per_step local-moving sweeps (LPA:
 * propagation sweeps) over the disjoint union of the resident requests' current level
 * graphs, each graph under its own stopping rule, sweep direction, tolerance and
 * total weight W; a graph whose level ends within the step stays frozen for the rest
 * of it, and the step ends early once no graph moves.  A request whose level ended
 * takes its phase transition on its own between steps (Louvain: renumbering and
 * aggregation, Section 3.3; Leiden: refinement first, Section 4.2; LPA: its final
 * labels), and requests that arrived join at the next step.  Each request's labels and the stats fields iterations, passes, communities,
 * edges_scanned and moved_last are identical to those of the same call made alone;
 * ms_total is the host time from admission to completion and the other times are 0.
 *
 * mgcd_server_create_stepped: arena as for mgcd_server_create.  Its first
 *   shared_bytes (0: 45% of the arena) hold the union during steps and the phase work
 *   between them; the rest holds each resident request's own block (its labels,
 *   degrees and aggregated levels; first fit).  sweeps_per_step >= 1, or 0 for
 *   max_iterations (each step takes every resident level to its end).  A request is
 *   admitted in arrival
 *   order once fewer than max_resident (1..65536) requests are resident, its block
 *   fits and the union of the resident requests with it (sized at their input sizes)
 *   fits its engine's share of the shared region.  Two step engines (one when
 *   max_resident is 1), each with half the resident places and half the shared region,
 *   a scheduler thread and a HIP stream (default priority) of its own on the device
 *   current at creation, so that one engine's sweeps overlap the other's phase work.  params are checked at creation
 *   (MGCD_E_ARG / MGCD_E_UNSUPPORTED as the calls return them).  Submission, poll,
 *   wait, info (bytes_in_use and the peak count the blocks; the shared region is
 *   reserved) and destroy are those of mgcd_server_*.  mgcd_server_submit returns
 *   MGCD_E_WORKSPACE when the request alone exceeds the blocks' part or the shared
 *   region.  Graph errors (validation when params ask for it, MGCD_E_OVERFLOW) fail
 *   that request alone; a device error fails every resident request. */
int mgcd_server_create_stepped(void *arena, size_t arena_bytes, size_t shared_bytes, int32_t max_resident,
                               int32_t sweeps_per_step, int32_t algo, const mgcd_params *p,
                               mgcd_server **out);

/* Where a stepped server's time went (host clock; zero for a whole-call server):
 * steps and sweeps issued, sweeps in which some graph moved, unions packed, phase
 * transitions; rows_swept = union rows summed over the sweeps in which some graph
 * moved and rows_moving = the rows of the graphs that moved in them (their ratio is
 * the share of swept rows that were not frozen); seconds spent packing unions and
 * building their schedules, in sweeps and their read-back, in phase transitions
 * (with final labels) and in admissions.  Counters since creation, summed over the
 * server's engines. */
typedef struct {
  int64_t steps, sweeps, sweeps_moving, packs, transitions;
  int64_t rows_swept, rows_moving;
  double s_pack, s_sweep, s_phase, s_admit;
} mgcd_step_stats;
int mgcd_server_step_stats(mgcd_server *s, mgcd_step_stats *out);

/* Message of the last error on this thread ("" if none). */
const char *mgcd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
