// Block-level scan helpers shared by the GPU kernels (256-thread blocks).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gs {

constexpr int kScanThreads = 256;

// inclusive scan of one u32 per lane across a wave64
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int l = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if (l >= d) v += o;
  }
  return v;
}

// block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and the total (all threads).  Contains two barriers.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const uint32_t inc = wave_incl_scan(v);
  if (l == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanThreads / 64; ++i) {
    const uint32_t x = s_wave[i];
    off += (i < w) ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

}  // namespace gs
