// Shared device and host helpers of the MI355X (gfx950) community-detection library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace mgcd {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;  // key of a fresh sketch slot; never a community id
constexpr int WAVE = 64;                 // CDNA wavefront width
constexpr int BLOCK = 256;               // four waves per workgroup

enum Algo : int { ALGO_LPA = 0, ALGO_MOVE = 1, ALGO_REFINE = 2 };
enum Mode : int { MODE_EXACT = 0, MODE_ALG1 = 1, MODE_UNCOND = 2, MODE_STD = 3, MODE_SMALL = 5 };

// A CSR graph in device memory (Section 3): rows are the out-entries of a vertex.
struct Graph {
  int32_t n;
  int64_t nnz;
  const int64_t *off;
  const int32_t *idx;
  const uint32_t *w;
};

struct Pair {
  uint32_t key;
  uint32_t val;
};

// ---- errors (host) -------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define MGCD_HIP(x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw ::mgcd::Error(-5, std::string(#x) + ": " + hipGetErrorString(e_));          \
  } while (0)

// Set while this thread records work into a HIP graph: the runtime refuses
// hipGetLastError then, and launch errors surface when the capture ends instead.
inline thread_local bool in_capture = false;

#define MGCD_LAUNCHED()                                      \
  do {                                                       \
    if (!::mgcd::in_capture) MGCD_HIP(hipGetLastError());    \
  } while (0)

// Kernels that hold a K-slot sketch per lane in registers: at K = 16 two waves per
// SIMD leave room for the sketch and its merge partner without spilling.
#define MGCD_SKETCH_OCCUPANCY(K) __attribute__((amdgpu_waves_per_eu(1, (K) >= 16 ? 2 : 8)))
// The row kernels of the sweep and of aggregation (LDS-staged windows) fit 128 VGPRs
// at K = 16 without spilling their sketch: ask for the four waves per SIMD that their
// LDS windows allow, for latency hiding.
#define MGCD_ROWS_OCCUPANCY(K) __attribute__((amdgpu_waves_per_eu((K) >= 16 ? 4 : 1, 8)))

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Sets the calling thread's message returned by mgcd_last_error().
void set_last_error(const std::string &msg);

inline int bits_for(uint64_t maxval) {  // bits needed to hold values <= maxval
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

// ---- bump allocator over the caller's workspace (host) ---------------------------
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0, peak = 0;
  bool dry = false;  // sizing pass: count bytes only
  template <typename T>
  T *take(int64_t count) {
    size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    size_t start = (used + 255) & ~(size_t)255;
    size_t end = start + bytes;
    if (end > peak) peak = end;
    if (!dry && end > cap)
      throw Error(-4, "workspace too small: need more than " + std::to_string(end) + " bytes");
    used = end;
    return dry ? nullptr : reinterpret_cast<T *>(base + start);
  }
  size_t mark() const { return used; }
  void release(size_t m) { used = m; }
};

// ---- device time of a stretch of stream work (host) --------------------------------
struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st;
  explicit Timer(hipStream_t s) : st(s) {
    MGCD_HIP(hipEventCreate(&a));
    MGCD_HIP(hipEventCreate(&b));
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  void start() { MGCD_HIP(hipEventRecord(a, st)); }
  float stop() {  // synchronises
    MGCD_HIP(hipEventRecord(b, st));
    MGCD_HIP(hipEventSynchronize(b));
    float ms = 0;
    MGCD_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
};

// ---- wave helpers (device) -------------------------------------------------------
__device__ inline int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

// A value that is the same in every lane, moved to a scalar register so that the
// compiler treats what depends on it as wave-uniform (scalar branches and loops).
__device__ inline int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)v);
}
__device__ inline int64_t uniform(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : ((~0ull) >> (64 - l));
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <typename T>
__device__ inline T wave_inclusive_scan(T v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T u = __shfl_up(v, o);
    if (l >= o) v += u;
  }
  return v;
}

// Totals that every block adds to one device counter go to one of SPREAD copies (by
// block index), so the atomics of blocks that finish together do not serialise on a
// single address; the reader adds up (or takes the maximum of) the copies.
constexpr int SPREAD = 64;
__device__ inline int spread_copy() { return (int)(blockIdx.x & (SPREAD - 1)); }

// Host: fold SPREAD copies of (nsum counters, then one maximum), each copy nsum + 1
// values, into out[0 .. nsum] (sums, then the maximum).  Synchronises st.
inline void read_spread(const unsigned long long *dev, int nsum, unsigned long long *out,
                        hipStream_t st) {
  std::vector<unsigned long long> h((size_t)SPREAD * (nsum + 1));
  MGCD_HIP(hipMemcpyAsync(h.data(), dev, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  MGCD_HIP(hipStreamSynchronize(st));
  for (int q = 0; q <= nsum; ++q) out[q] = 0;
  for (int c = 0; c < SPREAD; ++c) {
    const unsigned long long *x = h.data() + (size_t)c * (nsum + 1);
    for (int q = 0; q < nsum; ++q) out[q] += x[q];
    out[nsum] = x[nsum] > out[nsum] ? x[nsum] : out[nsum];
  }
}

// Sum over a 256-thread block; every thread gets the total.
template <typename T>
__device__ inline T block_sum(T v, T *lds4) {
  v = wave_sum(v);
  int w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == 0) lds4[w] = v;
  __syncthreads();
  T t = lds4[0] + lds4[1] + lds4[2] + lds4[3];
  __syncthreads();
  return t;
}

}  // namespace mgcd
