// The weighted Misra-Gries sketch held in registers (Appendix A.1, Algorithm 1).
//
// K slots live in 2K VGPRs of the lane that owns a stream; every loop over the
// slots is unrolled so the compiler keeps the slots in registers (static indices,
// no scratch).  The final sketch is a function of the stream only, not of which
// free slot a new key takes: a slot whose value is 0 is free, and reviving a
// stale key equals inserting it afresh.  So a new key goes to the first free slot
// here, which needs one pass and no slot-index arithmetic.
#pragma once
#include "common.hpp"

namespace mgcd {

template <int K, int MODE>
struct RegSketch {
  uint32_t key[K];
  uint32_t val[K];
  bool lossy;  // some counted weight was removed: values are lower bounds only

  __device__ inline void reset() {
#pragma unroll
    for (int p = 0; p < K; ++p) {
      key[p] = EMPTY;
      val[p] = 0;
    }
    lossy = false;
  }

  // Add (c, w) to the sketch.
  __device__ inline void update(uint32_t c, uint32_t w) {
    if constexpr (MODE == MODE_ALG1) {
      // Algorithm 1: accumulate into the slot holding c; else insert into a free
      // slot; else subtract w from every slot (clamped at 0) and drop the item.
      bool has = false;
#pragma unroll
      for (int p = 0; p < K; ++p) {
        bool m = key[p] == c;
        val[p] += m ? w : 0u;
        has |= m;
      }
      if (!has) {
        bool done = false;
#pragma unroll
        for (int p = 0; p < K; ++p) {
          bool e = !done && val[p] == 0;
          key[p] = e ? c : key[p];
          val[p] = e ? w : val[p];
          done |= e;
        }
        if (!done) {
          lossy = true;
#pragma unroll
          for (int p = 0; p < K; ++p) val[p] = val[p] > w ? val[p] - w : 0u;
        }
      }
    } else if constexpr (MODE == MODE_UNCOND) {
      // Unconditional subtraction: a key is present while its value is positive; on
      // a miss subtract w from every slot first, then insert into a free slot.
      bool has = false;
#pragma unroll
      for (int p = 0; p < K; ++p) {
        bool m = key[p] == c && val[p] > 0;
        val[p] += m ? w : 0u;
        has |= m;
      }
      if (!has) {
        bool any = false;
#pragma unroll
        for (int p = 0; p < K; ++p) {
          any |= val[p] > 0;
          val[p] = val[p] > w ? val[p] - w : 0u;
        }
        bool done = false;
#pragma unroll
        for (int p = 0; p < K; ++p) {
          bool e = !done && val[p] == 0;
          key[p] = e ? c : key[p];
          val[p] = e ? w : val[p];
          done |= e;
        }
        lossy |= any || !done;
      }
    } else {  // MODE_STD: textbook weighted MG
      bool has = false;
#pragma unroll
      for (int p = 0; p < K; ++p) {
        bool m = key[p] == c && val[p] > 0;
        val[p] += m ? w : 0u;
        has |= m;
      }
      if (!has) {
        bool done = false;
#pragma unroll
        for (int p = 0; p < K; ++p) {
          bool e = !done && val[p] == 0;
          key[p] = e ? c : key[p];
          val[p] = e ? w : val[p];
          done |= e;
        }
        if (!done) {
          lossy = true;
          uint32_t d = w;
#pragma unroll
          for (int p = 0; p < K; ++p) d = val[p] < d ? val[p] : d;
          uint32_t rest = w - d;
          bool put = rest == 0;
#pragma unroll
          for (int p = 0; p < K; ++p) {
            val[p] -= d;
            bool e = !put && val[p] == 0;
            key[p] = e ? c : key[p];
            val[p] = e ? rest : val[p];
            put |= e;
          }
        }
      }
    }
  }

  // Keep only the candidates (positive slots); other keys become EMPTY.
  __device__ inline void finalize() {
#pragma unroll
    for (int p = 0; p < K; ++p) key[p] = val[p] > 0 ? key[p] : EMPTY;
  }
};

// Merge sketch b into sketch a (mergeable summaries, Agarwal et al. 2012): add the
// values of equal keys; if more than K keys are positive, subtract the (K+1)-th
// largest value from all and keep the positive ones.  Slots with value 0 are empty.
// Returns true when the threshold step removed weight.  Output in a (K slots).
// Always inlined: as a call its slot arrays would live in scratch memory.
template <int K>
__device__ __attribute__((always_inline)) inline bool merge_sketch(uint32_t (&ak)[K],
                                                                  uint32_t (&av)[K],
                                                                  const uint32_t (&bk)[K],
                                                                  uint32_t (&bv)[K]) {
#pragma unroll
  for (int y = 0; y < K; ++y) {
#pragma unroll
    for (int x = 0; x < K; ++x) {
      bool m = bv[y] > 0 && av[x] > 0 && ak[x] == bk[y];
      av[x] += m ? bv[y] : 0u;
      bv[y] = m ? 0u : bv[y];
    }
  }
  int cnt = 0;
#pragma unroll
  for (int x = 0; x < K; ++x) cnt += (av[x] > 0) + (bv[x] > 0);
  bool lossy = false;
  if (cnt > K) {
    lossy = true;
    // t = the largest value with at least K+1 values >= it (the (K+1)-th largest)
    uint32_t t = 0;
#pragma unroll
    for (int i = 0; i < 2 * K; ++i) {
      uint32_t u = i < K ? av[i] : bv[i - K];
      int ge = 0;
#pragma unroll
      for (int j = 0; j < 2 * K; ++j) {
        uint32_t q = j < K ? av[j] : bv[j - K];
        ge += q >= u;
      }
      t = (ge >= K + 1 && u > t) ? u : t;
    }
#pragma unroll
    for (int x = 0; x < K; ++x) {
      av[x] = av[x] > t ? av[x] - t : 0u;
      bv[x] = bv[x] > t ? bv[x] - t : 0u;
    }
  }
  // move the survivors of b into the free slots of a (at most K survive in total)
#pragma unroll
  for (int y = 0; y < K; ++y) {
    bool put = bv[y] == 0;
#pragma unroll
    for (int x = 0; x < K; ++x) {
      bool e = !put && av[x] == 0;
      ak[x] = e ? bk[y] : ak[x];
      av[x] = e ? bv[y] : av[x];
      put |= e;
    }
  }
  return lossy;
}

// Merge `count` sketches stored at sk[base ..] with the fixed tree (pairs (0,1),
// (2,3), ... per level; an odd last sketch moves up unchanged).  Groups of 256
// consecutive sketches are aligned subtrees, so each is reduced in LDS and its
// root written back to sk[base + group].  The result is left in lds[0 .. K).
// Returns (block-uniform) whether any merge removed weight.
template <int K>
__device__ bool tree_reduce(Pair *sk, int64_t base, int64_t count, Pair *lds) {
  __shared__ int any_lossy;
  const int t = threadIdx.x;
  if (t == 0) any_lossy = 0;
  __syncthreads();
  bool lossy = false;
  int64_t remaining = count;
  while (true) {
    const int64_t groups = (remaining + BLOCK - 1) / BLOCK;
    for (int64_t gi = 0; gi < groups; ++gi) {
      const int64_t left = remaining - gi * BLOCK;
      const int cnt = (int)(left < BLOCK ? left : BLOCK);
      if (t < cnt) {
#pragma unroll
        for (int p = 0; p < K; ++p) lds[t * K + p] = sk[(base + gi * BLOCK + t) * K + p];
      }
      __syncthreads();
      int c = cnt;
      while (c > 1) {
        const int half = c >> 1;
        uint32_t ak[K], av[K], bk[K], bv[K];
        if (t < half) {
#pragma unroll
          for (int p = 0; p < K; ++p) {
            Pair x = lds[(2 * t) * K + p], y = lds[(2 * t + 1) * K + p];
            ak[p] = x.key;
            av[p] = x.val;
            bk[p] = y.key;
            bv[p] = y.val;
          }
        }
        __syncthreads();
        if (t < half) {
          lossy |= merge_sketch<K>(ak, av, bk, bv);
#pragma unroll
          for (int p = 0; p < K; ++p) lds[t * K + p] = Pair{av[p] > 0 ? ak[p] : EMPTY, av[p]};
        }
        if ((c & 1) && t == 0) {
#pragma unroll
          for (int p = 0; p < K; ++p) lds[half * K + p] = lds[(c - 1) * K + p];
        }
        __syncthreads();
        c = half + (c & 1);
      }
      if (groups > 1 && t < K) sk[(base + gi) * K + t] = lds[t];
      __syncthreads();
    }
    if (groups == 1) break;
    remaining = groups;
  }
  if (lossy) any_lossy = 1;
  __syncthreads();
  return any_lossy != 0;
}

// Sort K (key, value) slots by key in registers (odd-even transposition network);
// EMPTY keys sort last.
template <int K>
__device__ inline void sort_by_key(uint32_t (&k)[K], uint32_t (&v)[K]) {
#pragma unroll
  for (int r = 0; r < K; ++r) {
#pragma unroll
    for (int p = (r & 1); p + 1 < K; p += 2) {
      bool sw = k[p] > k[p + 1];
      uint32_t a = k[p], b = k[p + 1], x = v[p], y = v[p + 1];
      k[p] = sw ? b : a;
      k[p + 1] = sw ? a : b;
      v[p] = sw ? y : x;
      v[p + 1] = sw ? x : y;
    }
  }
}

}  // namespace mgcd
