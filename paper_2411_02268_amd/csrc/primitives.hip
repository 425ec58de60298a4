// Exclusive scan (tile reduce -> recursive scan of tile sums -> tile scan) and a
// stable least-significant-digit radix sort with 8-bit digits.  Both are plain
// data-parallel primitives used by bucketing, renumbering and aggregation.
#include "primitives.hpp"

namespace mgcd {

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;  // 2048 items per workgroup

template <typename Tin>
__global__ void __launch_bounds__(BLOCK) k_tile_sums(const Tin *in, int64_t n, int64_t *sums) {
  __shared__ int64_t lds[4];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t acc = 0;
#pragma unroll
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    int64_t i = base + (int64_t)r * BLOCK + threadIdx.x;
    if (i < n) acc += (int64_t)in[i];
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) sums[blockIdx.x] = acc;
}

// Wave w of the tile scans its SCAN_ITEMS * WAVE consecutive items 64 at a time (one
// coalesced load and store per round, a carry across rounds); the waves' totals give
// their offsets within the tile, tile_off the tile's.
template <typename Tin>
__global__ void __launch_bounds__(BLOCK)
    k_tile_scan(const Tin *in, int64_t *out, int64_t n, const int64_t *tile_off, int64_t *total) {
  __shared__ int64_t wtot[BLOCK / WAVE];
  const int w = threadIdx.x / WAVE, lane = lane_id();
  const int64_t wbase = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)w * (SCAN_ITEMS * WAVE) + lane;
  int64_t ex[SCAN_ITEMS];
  int64_t carry = 0;
#pragma unroll
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    const int64_t i = wbase + (int64_t)r * WAVE;
    const int64_t x = i < n ? (int64_t)in[i] : 0;
    const int64_t incl = wave_inclusive_scan(x);
    ex[r] = carry + incl - x;
    carry += __shfl(incl, WAVE - 1);
  }
  if (lane == 0) wtot[w] = carry;
  __syncthreads();
  int64_t off = tile_off ? tile_off[blockIdx.x] : 0;
  for (int q = 0; q < w; ++q) off += wtot[q];
#pragma unroll
  for (int r = 0; r < SCAN_ITEMS; ++r) {
    const int64_t i = wbase + (int64_t)r * WAVE;
    if (i < n) out[i] = off + ex[r];
  }
  if (total && blockIdx.x == gridDim.x - 1 && w == BLOCK / WAVE - 1 && lane == 0) *total = off + carry;
}

template <typename Tin>
static void scan_impl(const Tin *in, int64_t *out, int64_t n, int64_t *total, Arena &a,
                      hipStream_t s) {
  if (n <= 0) {
    if (total) MGCD_HIP(hipMemsetAsync(total, 0, sizeof(int64_t), s));
    return;
  }
  int64_t tiles = ceil_div(n, SCAN_TILE);
  if (tiles == 1) {
    k_tile_scan<Tin><<<1, BLOCK, 0, s>>>(in, out, n, nullptr, total);
    MGCD_LAUNCHED();
    return;
  }
  size_t m = a.mark();
  int64_t *sums = a.take<int64_t>(tiles);
  k_tile_sums<Tin><<<(unsigned)tiles, BLOCK, 0, s>>>(in, n, sums);
  MGCD_LAUNCHED();
  scan_impl<int64_t>(sums, sums, tiles, nullptr, a, s);
  k_tile_scan<Tin><<<(unsigned)tiles, BLOCK, 0, s>>>(in, out, n, sums, total);
  MGCD_LAUNCHED();
  a.release(m);
}

void scan_u32_i64(const uint32_t *in, int64_t *out, int64_t n, int64_t *total, Arena &a,
                  hipStream_t s) {
  scan_impl<uint32_t>(in, out, n, total, a, s);
}
void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, Arena &a,
              hipStream_t s) {
  scan_impl<int64_t>(in, out, n, total, a, s);
}

size_t scan_ws_bytes(int64_t n) {
  size_t b = 0;
  int64_t t = ceil_div(n > 0 ? n : 1, SCAN_TILE);
  while (t > 1) {
    b += (size_t)t * sizeof(int64_t) + 256;
    t = ceil_div(t, SCAN_TILE);
  }
  return b + 256;
}

// ------------------------------------------------------------------------------------
// radix sort
// ------------------------------------------------------------------------------------
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = BLOCK * RS_ITEMS;  // 4096 items per workgroup
constexpr int RS_BINS = 256;

// hist[d * tiles + t] = items of tile t whose digit is d (digit-major, so one
// exclusive scan yields every (digit, tile) output offset in stable order).
__global__ void __launch_bounds__(BLOCK)
    k_rs_hist(const uint64_t *keys, int64_t n, int shift, uint32_t *hist, int64_t tiles) {
  __shared__ uint32_t h[RS_BINS];
  h[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
#pragma unroll 4
  for (int r = 0; r < RS_ITEMS; ++r) {
    int64_t i = base + (int64_t)r * BLOCK + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Items are visited in tile order (round r covers items base + r*256 + t), ranked
// among equal digits with wave ballots, and written to their stable positions.
__global__ void __launch_bounds__(BLOCK)
    k_rs_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout, uint32_t *vout,
                 int64_t n, int shift, const int64_t *offs, int64_t tiles) {
  __shared__ uint32_t run[RS_BINS];
  __shared__ uint32_t wcnt[4][RS_BINS];
  const int t = threadIdx.x, w = t / WAVE;
  run[t] = 0;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  const int64_t my_off = offs[(int64_t)t * tiles + blockIdx.x];  // thread t owns digit t
  __shared__ int64_t off_lds[RS_BINS];
  off_lds[t] = my_off;
  for (int r = 0; r < RS_ITEMS; ++r) {
    int64_t i = base + (int64_t)r * BLOCK + t;
    bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    uint32_t val = valid ? vin[i] : 0;
    uint32_t d = (uint32_t)(key >> shift) & 255u;
#pragma unroll
    for (int q = 0; q < 4; ++q) wcnt[q][t] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
    __syncthreads();
    wcnt[0][t] = 0;
    wcnt[1][t] = c0;
    wcnt[2][t] = c0 + c1;
    wcnt[3][t] = c0 + c1 + c2;
    uint32_t tot = c0 + c1 + c2 + c3;
    __syncthreads();
    if (valid) {
      int64_t pos = off_lds[d] + run[d] + wcnt[w][d] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    run[t] += tot;
    __syncthreads();
  }
}

bool radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n,
                      int bits, Arena &a, hipStream_t s) {
  if (n <= 1 || bits <= 0) return false;
  int64_t tiles = ceil_div(n, RS_TILE);
  size_t m = a.mark();
  uint32_t *hist = a.take<uint32_t>(tiles * RS_BINS);
  int64_t *offs = a.take<int64_t>(tiles * RS_BINS);
  bool flip = false;
  for (int shift = 0; shift < bits; shift += 8) {
    const uint64_t *ki = flip ? k1 : k0;
    const uint32_t *vi = flip ? v1 : v0;
    uint64_t *ko = flip ? k0 : k1;
    uint32_t *vo = flip ? v0 : v1;
    k_rs_hist<<<(unsigned)tiles, BLOCK, 0, s>>>(ki, n, shift, hist, tiles);
    MGCD_LAUNCHED();
    scan_u32_i64(hist, offs, tiles * RS_BINS, nullptr, a, s);
    k_rs_scatter<<<(unsigned)tiles, BLOCK, 0, s>>>(ki, vi, ko, vo, n, shift, offs, tiles);
    MGCD_LAUNCHED();
    flip = !flip;
  }
  a.release(m);
  return flip;
}

size_t radix_sort_ws_bytes(int64_t n) {
  int64_t tiles = ceil_div(n > 0 ? n : 1, RS_TILE);
  return (size_t)tiles * RS_BINS * (sizeof(uint32_t) + sizeof(int64_t)) + 1024 +
         scan_ws_bytes(tiles * RS_BINS);
}

}  // namespace mgcd
