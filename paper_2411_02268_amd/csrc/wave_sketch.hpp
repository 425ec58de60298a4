// The weighted Misra-Gries sketch spread over a wavefront, for K = 32, 64, 128 or 256
// slots (Appendix A.1, Algorithm 1, and its variants): slot p lives in lane p mod 64,
// register p / 64.  Stream items arrive wave-uniform (the same (c, w) in every lane);
// matching a key is one compare per slot register plus a ballot, and the free slot
// that takes a new key is the first free one (slot placement does not change the
// sketch's positive entries).
#pragma once
#include "common.hpp"

namespace mgcd {

__device__ inline int first_lane(uint64_t m) { return __builtin_ctzll(m); }

template <typename T>
__device__ inline T lane_value(T v, int lane) {  // v of `lane` (wave-uniform lane)
  return (T)__builtin_amdgcn_readlane((int)v, lane);
}

// Slots per lane of a K-slot wave sketch: one for K <= 64, K / 64 for 128 and 256
// (slot p = s * 64 + lane lives in lane `lane`, register s).
template <int K>
struct WaveSlots {
  static_assert(K == 32 || K == 64 || K == 128 || K == 256, "wave sketch sizes");
  static constexpr int S = K <= WAVE ? 1 : K / WAVE;
  // lanes whose slot s exists (all lanes unless K < 64)
  static constexpr uint64_t VALID = K >= WAVE ? ~0ull : ((1ull << K) - 1);
};

template <int K, int MODE>
struct WaveSketch {
  static constexpr int S = WaveSlots<K>::S;
  static constexpr uint64_t VALID = WaveSlots<K>::VALID;
  uint32_t key[S], val[S];  // this lane's slots (lanes >= K stay empty)
  bool lossy;               // wave-uniform

  __device__ inline void reset() {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      key[s] = EMPTY;
      val[s] = 0;
    }
    lossy = false;
  }

  // The first free slot (value 0; register-major, then lowest lane) takes (c, w);
  // returns false (wave-uniform) when every slot is in use.
  __device__ inline bool insert(uint32_t c, uint32_t w) {
    const int lane = lane_id();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t fr = __ballot(val[s] == 0) & VALID;
      if (fr) {
        if (lane == first_lane(fr)) {
          key[s] = c;
          val[s] = w;
        }
        return true;
      }
    }
    return false;
  }

  // Add w to the slot whose key is c (present: value positive, or any value for
  // Algorithm 1, whose stale keys revive); false (wave-uniform) when c has none.
  __device__ inline bool add(uint32_t c, uint32_t w, bool positive_only) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const bool m = key[s] == c && (!positive_only || val[s] > 0);
      if (__ballot(m) & VALID) {
        if (m) val[s] += w;
        return true;
      }
    }
    return false;
  }

  // Add (c, w) (wave-uniform, c != EMPTY).
  __device__ inline void update(uint32_t c, uint32_t w) {
    const int lane = lane_id();
    if constexpr (MODE == MODE_ALG1) {
      // accumulate into the slot holding c (a stale key revives); else the first free
      // slot; else subtract w from every slot (clamped at 0) and drop the item
      if (add(c, w, false)) return;
      if (insert(c, w)) return;
      lossy = true;
#pragma unroll
      for (int s = 0; s < S; ++s) val[s] = val[s] > w ? val[s] - w : 0u;
    } else if constexpr (MODE == MODE_UNCOND) {
      // present = positive; on a miss subtract w from every slot, then insert
      if (add(c, w, true)) return;
      bool any = false;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        any |= (__ballot(val[s] > 0) & VALID) != 0;
        val[s] = val[s] > w ? val[s] - w : 0u;
      }
      const bool put = insert(c, w);
      lossy |= any || !put;
    } else {  // MODE_STD: textbook weighted MG
      if (add(c, w, true)) return;
      if (insert(c, w)) return;
      lossy = true;
      uint32_t d = ~0u;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const uint32_t x = lane < K ? val[s] : ~0u;
        d = x < d ? x : d;
      }
#pragma unroll
      for (int o = WAVE / 2; o > 0; o >>= 1) {
        const uint32_t x = __shfl_xor(d, o);
        d = x < d ? x : d;
      }
      d = d < w ? d : w;
      if (lane < K) {
#pragma unroll
        for (int s = 0; s < S; ++s) val[s] -= d;
      }
      const uint32_t rest = w - d;
      if (rest > 0) insert(c, rest);
    }
  }

  // Keep only the candidates (positive slots); other keys become EMPTY.
  __device__ inline void finalize() {
#pragma unroll
    for (int s = 0; s < S; ++s) key[s] = val[s] > 0 ? key[s] : EMPTY;
  }
};

// Merge sketch (bk, bv) into (ak, av) (mergeable summaries, Agarwal et al. 2012): add
// the values of equal keys; if more than K keys are positive, subtract the (K+1)-th
// largest value from all and keep the positive ones.  Returns true (wave-uniform)
// when the threshold step removed weight.  S slots per lane as in WaveSketch.
template <int K, int S = WaveSlots<K>::S>
__device__ inline bool wave_merge(uint32_t (&ak)[S], uint32_t (&av)[S], uint32_t (&bk)[S],
                                  uint32_t (&bv)[S]) {
  constexpr uint64_t VALID = WaveSlots<K>::VALID;
  const int lane = lane_id();
#pragma unroll
  for (int sb = 0; sb < S; ++sb) {
    uint64_t bpos = __ballot(bv[sb] > 0) & VALID;
    while (bpos) {
      const int q = first_lane(bpos);
      bpos &= bpos - 1;
      const uint32_t kq = lane_value(bk[sb], q), vq = lane_value(bv[sb], q);
#pragma unroll
      for (int sa = 0; sa < S; ++sa) {
        const bool m = av[sa] > 0 && ak[sa] == kq;
        if (__ballot(m) & VALID) {
          if (m) av[sa] += vq;
          if (lane == q) bv[sb] = 0;
          break;
        }
      }
    }
  }
  int cnt = 0;
#pragma unroll
  for (int s = 0; s < S; ++s)
    cnt += __popcll(__ballot(av[s] > 0) & VALID) + __popcll(__ballot(bv[s] > 0) & VALID);
  bool lossy = false;
  if (cnt > K) {
    lossy = true;
    // t = the largest value with at least K+1 values >= it (the (K+1)-th largest)
    uint32_t t = 0;
    for (int bit = 31; bit >= 0; --bit) {
      const uint32_t cand = t | (1u << bit);
      int ge = 0;
#pragma unroll
      for (int s = 0; s < S; ++s)
        ge += __popcll(__ballot(av[s] >= cand) & VALID) + __popcll(__ballot(bv[s] >= cand) & VALID);
      if (ge >= K + 1) t = cand;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      av[s] = av[s] > t ? av[s] - t : 0u;
      bv[s] = bv[s] > t ? bv[s] - t : 0u;
    }
  }
  // move the survivors of b into the free slots of a (at most K survive in total)
#pragma unroll
  for (int sb = 0; sb < S; ++sb) {
    uint64_t bpos = __ballot(bv[sb] > 0) & VALID;
    while (bpos) {
      const int q = first_lane(bpos);
      bpos &= bpos - 1;
      const uint32_t kq = lane_value(bk[sb], q), vq = lane_value(bv[sb], q);
#pragma unroll
      for (int sa = 0; sa < S; ++sa) {
        const uint64_t fr = __ballot(av[sa] == 0) & VALID;
        if (fr) {
          if (lane == first_lane(fr)) {
            ak[sa] = kq;
            av[sa] = vq;
          }
          break;
        }
      }
    }
  }
  return lossy;
}

// One slot per lane (K = 32, 64): the merge on scalars.
template <int K>
__device__ inline bool wave_merge(uint32_t &ak, uint32_t &av, uint32_t bk, uint32_t bv) {
  uint32_t a1[1] = {ak}, v1[1] = {av}, b1[1] = {bk}, w1[1] = {bv};
  const bool lossy = wave_merge<K, 1>(a1, v1, b1, w1);
  ak = a1[0];
  av = v1[0];
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
