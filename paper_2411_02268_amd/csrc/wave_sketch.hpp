// The weighted Misra-Gries sketch spread over a wavefront, for K = 32 or 64 slots
// (Appendix A.1, Algorithm 1, and its variants): slot p lives in lane p.  Stream
// items arrive wave-uniform (the same (c, w) in every lane); matching a key is one
// compare per lane plus a ballot, and the free slot that takes a new key is the
// lowest free lane (slot placement does not change the sketch's positive entries).
#pragma once
#include "common.hpp"

namespace mgcd {

__device__ inline int first_lane(uint64_t m) { return __builtin_ctzll(m); }

template <typename T>
__device__ inline T lane_value(T v, int lane) {  // v of `lane` (wave-uniform lane)
  return (T)__builtin_amdgcn_readlane((int)v, lane);
}

template <int K, int MODE>
struct WaveSketch {
  static_assert(K == 32 || K == 64, "one slot per lane");
  static constexpr uint64_t VALID = K == 64 ? ~0ull : ((1ull << K) - 1);
  uint32_t key, val;  // this lane's slot (lanes >= K stay empty)
  bool lossy;         // wave-uniform

  __device__ inline void reset() {
    key = EMPTY;
    val = 0;
    lossy = false;
  }

  // Add (c, w) (wave-uniform, c != EMPTY).
  __device__ inline void update(uint32_t c, uint32_t w) {
    const int lane = lane_id();
    if constexpr (MODE == MODE_ALG1) {
      // accumulate into the slot holding c (a stale key revives); else the first free
      // slot; else subtract w from every slot (clamped at 0) and drop the item
      const bool m = key == c;
      if (__ballot(m) & VALID) {
        if (m) val += w;
        return;
      }
      const uint64_t fr = __ballot(val == 0) & VALID;
      if (fr) {
        if (lane == first_lane(fr)) {
          key = c;
          val = w;
        }
        return;
      }
      lossy = true;
      val = val > w ? val - w : 0u;
    } else if constexpr (MODE == MODE_UNCOND) {
      // present = positive; on a miss subtract w from every slot, then insert
      const bool m = key == c && val > 0;
      if (__ballot(m) & VALID) {
        if (m) val += w;
        return;
      }
      const bool any = (__ballot(val > 0) & VALID) != 0;
      val = val > w ? val - w : 0u;
      const uint64_t fr = __ballot(val == 0) & VALID;
      if (fr && lane == first_lane(fr)) {
        key = c;
        val = w;
      }
      lossy |= any || !fr;
    } else {  // MODE_STD: textbook weighted MG
      const bool m = key == c && val > 0;
      if (__ballot(m) & VALID) {
        if (m) val += w;
        return;
      }
      uint64_t fr = __ballot(val == 0) & VALID;
      if (fr) {
        if (lane == first_lane(fr)) {
          key = c;
          val = w;
        }
        return;
      }
      lossy = true;
      uint32_t d = lane < K ? val : ~0u;
#pragma unroll
      for (int o = WAVE / 2; o > 0; o >>= 1) {
        const uint32_t x = __shfl_xor(d, o);
        d = x < d ? x : d;
      }
      d = d < w ? d : w;
      if (lane < K) val -= d;
      const uint32_t rest = w - d;
      if (rest > 0) {
        fr = __ballot(val == 0) & VALID;
        if (lane == first_lane(fr)) {
          key = c;
          val = rest;
        }
      }
    }
  }

  // Keep only the candidates (positive slots); other keys become EMPTY.
  __device__ inline void finalize() { key = val > 0 ? key : EMPTY; }
};

// Merge sketch (bk, bv) into (ak, av) (mergeable summaries, Agarwal et al. 2012): add
// the values of equal keys; if more than K keys are positive, subtract the (K+1)-th
// largest value from all and keep the positive ones.  Returns true (wave-uniform)
// when the threshold step removed weight.
template <int K>
__device__ inline bool wave_merge(uint32_t &ak, uint32_t &av, uint32_t bk, uint32_t bv) {
  constexpr uint64_t VALID = WaveSketch<K, MODE_ALG1>::VALID;
  const int lane = lane_id();
  uint64_t bpos = __ballot(bv > 0) & VALID;
  while (bpos) {
    const int q = first_lane(bpos);
    bpos &= bpos - 1;
    const uint32_t kq = lane_value(bk, q), vq = lane_value(bv, q);
    const bool m = av > 0 && ak == kq;
    if (__ballot(m) & VALID) {
      if (m) av += vq;
      if (lane == q) bv = 0;
    }
  }
  const int cnt = __popcll(__ballot(av > 0) & VALID) + __popcll(__ballot(bv > 0) & VALID);
  bool lossy = false;
  if (cnt > K) {
    lossy = true;
    // t = the largest value with at least K+1 values >= it (the (K+1)-th largest)
    uint32_t t = 0;
    for (int bit = 31; bit >= 0; --bit) {
      const uint32_t cand = t | (1u << bit);
      const int ge = __popcll(__ballot(av >= cand) & VALID) + __popcll(__ballot(bv >= cand) & VALID);
      if (ge >= K + 1) t = cand;
    }
    av = av > t ? av - t : 0u;
    bv = bv > t ? bv - t : 0u;
  }
  // move the survivors of b into the free slots of a (at most K survive in total)
  bpos = __ballot(bv > 0) & VALID;
  while (bpos) {
    const int q = first_lane(bpos);
    bpos &= bpos - 1;
    const uint32_t kq = lane_value(bk, q), vq = lane_value(bv, q);
    const uint64_t fr = __ballot(av == 0) & VALID;
    if (lane == first_lane(fr)) {
      ak = kq;
      av = vq;
    }
  }
  return lossy;
}

// The fixed merge tree over a stream's chunk sketches, kept as a binary counter:
// level l of `stack` (LDS, DEPTH levels of 2 x 64 words) holds the merged sketch of
// the last complete aligned run of 2^l chunks.  push() merges a finished chunk
// sketch in (left operand = the older run); result() merges the pending runs from
// the right, which is the order of the level-by-level tree with an odd last node
// carried up.  A stream of fewer than 2^DEPTH chunks fits.
constexpr int WDEPTH_SHALLOW = 12, WDEPTH = 31;

// Stack depth for streams of at most max_len positions cut into chunks of L.
inline int wave_depth_for(int64_t max_len, int64_t L) {
  const int64_t chunks = (max_len + L - 1) / L;
  return chunks < ((int64_t)1 << WDEPTH_SHALLOW) ? WDEPTH_SHALLOW : WDEPTH;
}

template <int K, int DEPTH>
struct WaveTree {
  uint32_t *stack;  // this wave's LDS: DEPTH * 2 * WAVE words
  uint32_t mask = 0;  // occupied levels (wave-uniform)
  bool lossy = false;

  __device__ inline void put(int l, uint32_t k, uint32_t v) {
    stack[(2 * l) * WAVE + lane_id()] = k;
    stack[(2 * l + 1) * WAVE + lane_id()] = v;
  }
  __device__ inline void get(int l, uint32_t &k, uint32_t &v) const {
    k = stack[(2 * l) * WAVE + lane_id()];
    v = stack[(2 * l + 1) * WAVE + lane_id()];
  }

  __device__ inline void push(uint32_t k, uint32_t v) {
    int l = 0;
    while ((mask >> l) & 1u) {
      uint32_t lk, lv;
      get(l, lk, lv);
      lossy |= wave_merge<K>(lk, lv, k, v);
      k = lk;
      v = lv;
      mask &= ~(1u << l);
      ++l;
    }
    put(l, k, v);
    mask |= 1u << l;
  }

  // The root (empty if no chunk was pushed).
  __device__ inline void result(uint32_t &k, uint32_t &v) {
    k = EMPTY;
    v = 0;
    bool have = false;
    for (int l = 0; l < DEPTH; ++l) {
      if (!((mask >> l) & 1u)) continue;
      uint32_t lk, lv;
      get(l, lk, lv);
      if (have) lossy |= wave_merge<K>(lk, lv, k, v);
      k = lk;
      v = lv;
      have = true;
    }
    k = v > 0 ? k : EMPTY;
  }
};

}  // namespace mgcd
