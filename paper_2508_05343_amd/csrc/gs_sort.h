// Sorting helpers shared by the bin sort and the blend: a register bitonic
// sort of one wavefront's keys and merge-path merges of sorted runs.  Keys
// are 64-bit (depth bits << 32 | item); the padding key ~0 sorts last.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
  const int lo = __shfl_xor((int)(uint32_t)x, m, 64), hi = __shfl_xor((int)(uint32_t)(x >> 32), m, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Bitonic sort (ascending) of 64 E keys held in registers, E consecutive
// keys per lane (key i = lane E + r).  Steps whose partner distance j is
// below E pair keys of one lane; the others pair key r of lanes l and
// l ^ (j / E) through a lane shuffle, each side keeping the minimum or the
// maximum.  No LDS, no barrier.
template <int E>
__device__ __forceinline__ void wave_bitonic(uint64_t (&x)[E]) {
  const int lane = __lane_id();
  constexpr int N = 64 * E;
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          if ((r & j) == 0) {
            // ascending where bit k of the key index lane E + r is clear
            const bool up = (((lane * E + r) & k) == 0);
            const uint64_t a = x[r], b = x[r | j];
            const bool sw = (b < a) == up;
            x[r] = sw ? b : a;
            x[r | j] = sw ? a : b;
          }
        }
      } else {
        const int m = j / E;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          // the lower lane of the pair keeps the minimum when ascending
          const bool take_min = ((lane & m) == 0) == (((lane * E + r) & k) == 0);
          const uint64_t y = shfl_xor_u64(x[r], m);
          const bool keep_y = (y < x[r]) == take_min;  // equal keys are equal values
          x[r] = keep_y ? y : x[r];
        }
      }
    }
  }
}

// Merge-path split: the number of elements of run a among the first d
// outputs of merging a = x[a0, a0 + na) and b = x[b0, b0 + nb) (a first on
// equal keys).
__device__ __forceinline__ uint32_t merge_split(const uint64_t* x, uint32_t a0, uint32_t na, uint32_t b0,
                                                uint32_t nb, uint32_t d) {
  uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
  while (lo < hi) {
    const uint32_t m = (lo + hi) >> 1;
    if (x[a0 + m] <= x[b0 + d - 1 - m]) lo = m + 1; else hi = m;
  }
  return lo;
}

// Merge of the sorted runs a = x[a0, a0 + na) and b = x[b0, b0 + nb) by
// `lanes` cooperating threads (this one is `tid`), each writing a contiguous
// slice of the output: as keys to out[o0 + ...] or, with IDS, as the low 32
// bits of the keys to ids[...] for outputs below `limit` only.
template <bool IDS>
__device__ __forceinline__ void merge_runs(const uint64_t* x, uint32_t a0, uint32_t na, uint32_t b0, uint32_t nb,
                                           uint64_t* out, uint32_t* ids, uint32_t o0, uint32_t limit, uint32_t tid,
                                           uint32_t lanes) {
  const uint32_t n = na + nb;
  const uint32_t per = (n + lanes - 1) / lanes;
  const uint32_t d0 = min(n, tid * per), d1 = min(n, d0 + per);
  if (d0 >= d1) return;
  uint32_t ia = merge_split(x, a0, na, b0, nb, d0), ib = d0 - ia;
  for (uint32_t o = d0; o < d1; ++o) {
    const bool takea = ib >= nb || (ia < na && x[a0 + ia] <= x[b0 + ib]);
    const uint64_t v = takea ? x[a0 + ia++] : x[b0 + ib++];
    if (IDS) {
      if (o0 + o < limit) ids[o0 + o] = (uint32_t)v;
    } else {
      out[o0 + o] = v;
    }
  }
}

}  // namespace gs
