// Batched runs of many graphs as one disjoint union (batch.hip).
#pragma once
#include "../../include/mgcd.h"
#include "common.hpp"

namespace mgcd {

// algo: MGCD_ALGO_LPA or MGCD_ALGO_LOUVAIN.  outs: host array of device label arrays.
void run_batched(int algo, const mgcd_csr *graphs, int32_t count, const mgcd_params *p,
                 int32_t *const *outs, Arena &a, hipStream_t st, mgcd_graph_stats *gstats,
                 mgcd_stats *total);
size_t batched_workspace_bytes(int32_t algo, int32_t count, int64_t N, int64_t E,
                               const mgcd_params *p);

}  // namespace mgcd
