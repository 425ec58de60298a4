/*
 * oracle.h -- declarations of the CPU oracle (test infrastructure only).
 * All pointers are host pointers.  Nothing in the HIP library includes this file.
 */
#ifndef MGCD_ORACLE_H
#define MGCD_ORACLE_H
#include <stdint.h>

#define OR_MODE_EXACT 0  /* exact per-vertex table (the comparison baseline)        */
#define OR_MODE_ALG1 1   /* Algorithm 1, conditional subtraction (the paper's MG)   */
#define OR_MODE_UNCOND 2 /* unconditional subtraction (Section 4.1, variant 1)      */
#define OR_MODE_STD 3    /* textbook weighted MG (min-decrement)                   */
#define OR_MODE_SMALL 5  /* small mod-based table (Appendix A.2): k = its slot count  */

#define OR_ALGO_LPA 0
#define OR_ALGO_MOVE 1
#define OR_ALGO_REFINE 2

typedef struct {
  int32_t mode;
  int32_t k;
  int32_t k_aggregate;
  int32_t max_iterations;
  int32_t max_passes;
  int32_t threads;
  int64_t chunk_len;
  double tolerance;
  double tolerance_drop;
  double aggregation_tolerance;
  int32_t one_scan; /* LPA only: 1 = the 1-scan variant (Section 4.3) */
  int32_t aggregation; /* 0: as mode; 1: exact rows; 2: Algorithm 1, k_aggregate slots */
} or_params;

typedef struct {
  int32_t iterations;
  int32_t passes;
  int32_t communities;
  int32_t reserved;
  int64_t edges_scanned;
  int64_t moved_last;
} or_stats;

int oracle_sketch_stream(const uint32_t *keys, const uint32_t *weights, int64_t n, int mode, int k,
                         int64_t chunk_len, uint32_t *out_keys, uint32_t *out_vals);
int oracle_mg_merge(const uint32_t *ak, const uint32_t *av, int na, const uint32_t *bk,
                    const uint32_t *bv, int nb, int k, uint32_t *ok, uint32_t *ov);
void oracle_canonical(int32_t n, const int32_t *C, int32_t *out);
int oracle_move_sweep(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w, int algo,
                      int mode, int k, int64_t chunk_len, const int32_t *C, const int32_t *bound,
                      const int64_t *K, const int64_t *Sigma, const int32_t *size, int64_t W,
                      int direction, int one_scan, int32_t *Cnew, int64_t *gain);
int oracle_refine(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                  const int32_t *bound, const int64_t *K, int64_t W, int mode, int k,
                  int64_t chunk_len, int32_t *R);
int64_t oracle_aggregate(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                         const int32_t *D, int32_t m, int mode, int k, int64_t chunk_len,
                         int symmetric, int64_t *out_off, int32_t *out_idx, uint32_t *out_w);
double oracle_modularity(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                         const int32_t *C);
int oracle_lpa(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
               const or_params *p, int32_t *labels, or_stats *st);
int oracle_louvain(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                   const or_params *p, int32_t *labels, or_stats *st);
int oracle_leiden(int32_t n, const int64_t *off, const int32_t *idx, const uint32_t *w,
                  const or_params *p, int32_t *labels, or_stats *st);

#endif
