// Exclusive scan and stable LSD radix sort (host launchers; kernels in primitives.hip).
#pragma once
#include "common.hpp"

namespace mgcd {

// out[i] = sum of in[0..i) (exclusive); *total (device, may be null) = sum of all.
// out may alias in.
void scan_u32_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *total, Arena &a,
                  hipStream_t s);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, Arena &a,
              hipStream_t s);

// Stable sort of (key, value) pairs by bits [0, bits) of the key.  Uses k1/v1 as the
// second buffer; returns true when the sorted result ended in (k1, v1).
bool radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                      int bits, Arena &a, hipStream_t s);

// Workspace upper bound of radix_sort_pairs / the scans for n items.
size_t radix_sort_ws_bytes(int64_t n);
size_t scan_ws_bytes(int64_t n);

}  // namespace mgcd
