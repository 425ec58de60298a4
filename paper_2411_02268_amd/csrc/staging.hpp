// Staging of per-lane streams through LDS: every lane of a wave owns a stream
// segment [lo, hi) of a (key, weight) array pair; the wave loads the segments 16
// positions at a time with 16 lanes per segment (64-byte segments instead of 64
// scattered lines per load) into an LDS window, and each lane then reads back its
// own 16 positions with 128-bit LDS loads.
#pragma once
#include "common.hpp"
#include "sketch.hpp"

namespace mgcd {

constexpr int WIN = 16;            // staged positions per lane and window
constexpr int WROW = 2 * WIN + 4;  // words per lane row: WIN (key, weight) pairs + pad; rows
                                   // are 16-byte aligned and 8 consecutive lanes' rows start
                                   // in distinct 4-bank groups (conflict-free 128-bit reads)
constexpr int SPR = WAVE / WIN;    // segments staged per load round (WIN lanes each); a
                                   // window takes WIN rounds

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void put_pair(uint32_t *win, int src, uint32_t k, uint32_t w) {
  typedef uint32_t v2u __attribute__((ext_vector_type(2)));
  v2u pr;
  pr.x = k;
  pr.y = w;
  *reinterpret_cast<v2u *>(win + src * WROW + 2 * (lane_id() % WIN)) = pr;
}

// Stage positions s0 .. s0+WIN-1 of every lane's segment [lo, hi) of (keys, wts)
// into the wave's window win (WAVE * WROW words): round r serves the segments of
// lanes SPR*r .. SPR*r+SPR-1; all loads of the window are in flight together.  Positions past
// a segment's end stage (EMPTY, 0).
__device__ inline void stage_pairs(uint32_t *win, int64_t lo, int64_t hi, int64_t s0,
                                   const uint32_t *keys, const uint32_t *wts) {
  const int lane = lane_id();
  uint32_t kk[WIN], ww[WIN];
  uint32_t ok = 0;
#pragma unroll
  for (int r = 0; r < WIN; ++r) {
    const int src = r * SPR + lane / WIN;
    const int64_t e = __shfl(lo, src) + s0 + lane % WIN;
    const bool v = e < __shfl(hi, src);
    ok |= v ? 1u << r : 0u;
    const int64_t es = v ? e : 0;
    kk[r] = __builtin_nontemporal_load(keys + es);
    ww[r] = __builtin_nontemporal_load(wts + es);
  }
#pragma unroll
  for (int r = 0; r < WIN; ++r) {
    const bool v = (ok >> r) & 1u;
    put_pair(win, r * SPR + lane / WIN, v ? kk[r] : EMPTY, v ? ww[r] : 0u);
  }
}

// This lane's WIN staged keys and weights, read with 128-bit LDS loads.
__device__ inline void read_window(const uint32_t *win, uint32_t (&kk)[WIN], uint32_t (&ww)[WIN]) {
  typedef uint32_t v4u __attribute__((ext_vector_type(4)));
  const v4u *p = reinterpret_cast<const v4u *>(win + lane_id() * WROW);
#pragma unroll
  for (int q = 0; q < WIN / 2; ++q) {
    const v4u x = p[q];
    kk[2 * q] = x.x;
    ww[2 * q] = x.y;
    kk[2 * q + 1] = x.z;
    ww[2 * q + 1] = x.w;
  }
}

// The longest segment of the wave.
__device__ inline int64_t wave_max_len(int64_t lo, int64_t hi) {
  int64_t m = hi - lo;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const int64_t x = __shfl_xor(m, o);
    m = x > m ? x : m;
  }
  return m;
}

// Algorithm 1 over this lane's segment [lo, hi) of (keys, wts), staged; EMPTY keys
// are skipped.  Every lane of the wave must call this (an idle lane passes lo == hi).
template <int K, int MODE>
__device__ inline void staged_fold(RegSketch<K, MODE> &s, uint32_t *win, int64_t lo, int64_t hi,
                                   const uint32_t *keys, const uint32_t *wts) {
  const int64_t maxlen = wave_max_len(lo, hi);
  for (int64_t s0 = 0; s0 < maxlen; s0 += WIN) {
    stage_pairs(win, lo, hi, s0, keys, wts);
    wave_sync();
    uint32_t kk[WIN], ww[WIN];
    read_window(win, kk, ww);
    wave_sync();
#pragma unroll
    for (int t = 0; t < WIN; ++t)
      if (kk[t] != EMPTY) s.update(kk[t], ww[t]);
  }
}

}  // namespace mgcd
