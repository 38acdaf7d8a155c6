// K2-K5: visibility compaction, depth sort, tile-key duplication, tile sort,
// tile ranges.
//
// The pairs must end up ordered by the 64-bit key (global tile << 32 | fp32
// depth bits), ties by item index.  An LSD radix sort over that key first
// sorts by the 32 depth bits and then, stably, by the tile bits.  All pairs of
// one primitive share its depth, so the depth passes are run on the visible
// primitives before duplication (V items instead of P pairs); duplication
// then emits pairs in depth order and only ceil(tile_bits / 8) passes run on
// the P pairs, moving 8 bytes per pair instead of 12.
//
// Every pass is one onesweep kernel: partitions of 4096 keys are taken from an
// atomic ticket (so a partition only ever waits on partitions whose blocks are
// already running), ranked in LDS with wave64 ballot matching, and placed
// with a decoupled look-back over per-(partition, digit) status words.
#include <hip/hip_runtime.h>

#include "gs_internal.h"

namespace gs {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kPart = kSortThreads * kSortItems;  // 4096 keys per partition
constexpr int kRadix = 256;
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 1u << 31;
constexpr uint32_t kCountMask = (1u << 30) - 1;
constexpr int kDepthPasses = 4;
constexpr int kMaxTilePasses = 4;

// counters (u32) inside the workspace
enum {
  C_TICKET_COMPACT = 0,
  C_TICKET_SCAN = 1,
  C_TICKET_DEPTH = 2,   // 4 entries
  C_TICKET_TILE = 6,    // 4 entries
  C_NUM_VISIBLE = 16,
  C_NUM_PAIRS = 17,
  C_OVERFLOW = 18,
  C_COUNT = 64
};

__device__ __forceinline__ uint32_t ld_acq(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// inclusive scan of one u32 per lane across a wave64
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if (l >= d) v += o;
  }
  return v;
}

// block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and writes the total to *total (all threads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const uint32_t inc = wave_incl_scan(v);
  if (l == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kSortThreads / 64; ++i) {
    const uint32_t x = s_wave[i];
    off += (i < w) ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// ----------------------------------------------------------------- fill
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// zero the prefix of a look-back array used by `*d_count` keys
__global__ void k_fill_prefix(uint32_t* __restrict__ p, const uint32_t* __restrict__ d_count, uint32_t words_per_part,
                              const int32_t* __restrict__ d_overflow) {
  if (d_overflow && *d_overflow) return;
  const uint32_t cnt = *d_count;
  const size_t words = (size_t)((cnt + kPart - 1) / kPart) * words_per_part;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0u;
}

hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------ decoupled look-back scan
// MODE 0: x_i = (tiles[i] > 0) over all items; emits the compacted depth keys
//         and item ids and writes V to counters[C_NUM_VISIBLE].
// MODE 1: x_j = tiles[ids[j]] over the V depth-sorted visible items; writes the
//         exclusive offsets and P to counters[C_NUM_PAIRS].
template <int MODE>
__global__ __launch_bounds__(kSortThreads) void k_scan(uint32_t n_host, const uint32_t* __restrict__ tiles,
                                                       const uint32_t* __restrict__ depth_bits,
                                                       const uint32_t* __restrict__ ids,
                                                       uint32_t* __restrict__ out_a, uint32_t* __restrict__ out_b,
                                                       uint32_t* __restrict__ counters, uint32_t* __restrict__ look) {
  __shared__ uint32_t s_wave[kSortThreads / 64];
  __shared__ uint32_t s_misc[2];
  const int t = threadIdx.x;
  if (t == 0) s_misc[0] = atomicAdd(&counters[MODE == 0 ? C_TICKET_COMPACT : C_TICKET_SCAN], 1u);
  __syncthreads();
  const uint32_t part = s_misc[0];
  const uint32_t n = (MODE == 0) ? n_host : counters[C_NUM_VISIBLE];
  const uint64_t base = (uint64_t)part * kPart;
  if (base >= n) return;
  const uint64_t first = base + (uint64_t)t * kSortItems;
  uint32_t x[kSortItems];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint64_t i = first + j;
    uint32_t v = 0;
    if (i < n) v = (MODE == 0) ? (tiles[i] > 0 ? 1u : 0u) : tiles[ids[i]];
    x[j] = v;
    sum += v;
  }
  uint32_t block_total;
  const uint32_t tpre = block_excl_scan(sum, s_wave, &block_total);
  if (t == 0) {
    uint32_t excl = 0;
    if (part == 0) {
      st_rel(&look[0], kFlagInc | block_total);
    } else {
      st_rel(&look[part], kFlagAgg | block_total);
      int64_t p = (int64_t)part - 1;
      while (true) {
        const uint32_t v = ld_acq(&look[p]);
        if ((v & (kFlagAgg | kFlagInc)) == 0) {
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += v & kCountMask;
        if (v & kFlagInc) break;
        --p;
      }
      st_rel(&look[part], kFlagInc | (excl + block_total));
    }
    s_misc[1] = excl;
    if (base + kPart >= n) counters[MODE == 0 ? C_NUM_VISIBLE : C_NUM_PAIRS] = excl + block_total;
  }
  __syncthreads();
  uint32_t pos = s_misc[1] + tpre;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint64_t i = first + j;
    if (i < n) {
      if (MODE == 0) {
        if (x[j]) {
          out_a[pos] = depth_bits[i];
          out_b[pos] = (uint32_t)i;
        }
      } else {
        out_a[i] = pos;
      }
    }
    pos += x[j];
  }
}

__global__ void k_finalize_pairs(uint32_t* __restrict__ counters, int64_t capacity, int64_t* __restrict__ d_num_pairs,
                                 int32_t* __restrict__ d_overflow) {
  const uint32_t P = counters[C_NUM_PAIRS];
  *d_num_pairs = (int64_t)P;
  const int32_t ov = ((int64_t)P > capacity) ? 1 : 0;
  *d_overflow = ov;
  counters[C_OVERFLOW] = (uint32_t)ov;
}

// ------------------------------------------------------------ histograms
// Digit histograms of `npass` 8-bit digits starting at bit 0 for keys[0..n).
__global__ __launch_bounds__(kSortThreads) void k_histogram(const uint32_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ d_count, int npass,
                                                            uint32_t* __restrict__ hist,
                                                            const int32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_h[kMaxTilePasses * kRadix];
  if (d_overflow && *d_overflow) return;
  const uint32_t n = *d_count;
  const uint64_t base = (uint64_t)blockIdx.x * kPart;
  if (base >= n) return;
  for (int i = threadIdx.x; i < npass * kRadix; i += kSortThreads) s_h[i] = 0;
  __syncthreads();
#pragma unroll 4
  for (int j = 0; j < kSortItems; ++j) {
    const uint64_t i = base + (uint64_t)j * kSortThreads + threadIdx.x;
    if (i < n) {
      const uint32_t k = keys[i];
      for (int p = 0; p < npass; ++p) atomicAdd(&s_h[p * kRadix + ((k >> (8 * p)) & 255u)], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npass * kRadix; i += kSortThreads) {
    const uint32_t v = s_h[i];
    if (v) atomicAdd(&hist[i], v);
  }
}

// exclusive scan of each pass's 256 bins, in place
__global__ __launch_bounds__(kSortThreads) void k_hist_scan(uint32_t* __restrict__ hist, int npass,
                                                            const int32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_wave[kSortThreads / 64];
  if (d_overflow && *d_overflow) return;
  for (int p = 0; p < npass; ++p) {
    const uint32_t v = hist[p * kRadix + threadIdx.x];
    uint32_t tot;
    const uint32_t ex = block_excl_scan(v, s_wave, &tot);
    hist[p * kRadix + threadIdx.x] = ex;
    __syncthreads();
  }
}

// --------------------------------------------------------------- onesweep
// One LSD pass over digit (key >> shift) & 255.  look is laid out
// [partition][npass][256]; goff holds the exclusive digit offsets of the pass.
__global__ __launch_bounds__(kSortThreads) void k_onesweep(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out,
                                                           const uint32_t* __restrict__ d_count, int shift,
                                                           int pass, int npass, const uint32_t* __restrict__ goff,
                                                           uint32_t* __restrict__ look, uint32_t* __restrict__ ticket,
                                                           const int32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_keys[kPart];
  __shared__ uint32_t s_vals[kPart];
  __shared__ uint32_t s_wh[kSortThreads / 64][kRadix];
  __shared__ uint32_t s_local[kRadix];
  __shared__ uint32_t s_gbase[kRadix];
  __shared__ uint32_t s_wave[kSortThreads / 64];
  __shared__ uint32_t s_part;

  if (d_overflow && *d_overflow) return;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  if (t == 0) s_part = atomicAdd(ticket, 1u);
  for (int i = t; i < (kSortThreads / 64) * kRadix; i += kSortThreads) (&s_wh[0][0])[i] = 0;
  __syncthreads();
  const uint32_t part = s_part;
  const uint32_t n = *d_count;
  const uint64_t base = (uint64_t)part * kPart;
  if (base >= n) return;

  // warp-striped load: wave w owns [w*1024, (w+1)*1024), item j of lane l at j*64 + l
  uint32_t key[kSortItems], val[kSortItems];
  uint16_t rank[kSortItems];
  const uint64_t wbase = base + (uint64_t)w * (64 * kSortItems);
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint64_t i = wbase + (uint64_t)j * 64 + l;
    const bool ok = i < n;
    key[j] = ok ? keys_in[i] : 0xffffffffu;
    val[j] = ok ? vals_in[i] : 0u;
  }
  const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint64_t i = wbase + (uint64_t)j * 64 + l;
    const bool ok = i < n;
    const uint32_t d = (key[j] >> shift) & 255u;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t lower = (uint32_t)__popcll(peers & lt_mask);
    const uint32_t cur = s_wh[w][d];
    rank[j] = (uint16_t)(cur + lower);
    const bool leader = ok && ((peers >> l) == 1ull);
    if (leader) s_wh[w][d] = cur + (uint32_t)__popcll(peers);
  }
  __syncthreads();

  // per digit: wave prefix, block count, publish, look back
  const int d = t;
  uint32_t c[kSortThreads / 64];
  uint32_t tot = 0;
#pragma unroll
  for (int i = 0; i < kSortThreads / 64; ++i) {
    c[i] = s_wh[i][d];
    s_wh[i][d] = tot;
    tot += c[i];
  }
  uint32_t* my_look = look + ((size_t)part * npass + pass) * kRadix + d;
  uint32_t excl = 0;
  if (part == 0) {
    st_rel(my_look, kFlagInc | tot);
  } else {
    st_rel(my_look, kFlagAgg | tot);
    int64_t p = (int64_t)part - 1;
    while (true) {
      const uint32_t v = ld_acq(look + ((size_t)p * npass + pass) * kRadix + d);
      if ((v & (kFlagAgg | kFlagInc)) == 0) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += v & kCountMask;
      if (v & kFlagInc) break;
      --p;
    }
    st_rel(my_look, kFlagInc | (excl + tot));
  }
  s_gbase[d] = goff[d] + excl;
  uint32_t dummy;
  const uint32_t lstart = block_excl_scan(tot, s_wave, &dummy);
  s_local[d] = lstart;
  __syncthreads();

  // scatter into LDS in digit order
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint64_t i = wbase + (uint64_t)j * 64 + l;
    if (i < n) {
      const uint32_t dd = (key[j] >> shift) & 255u;
      const uint32_t lp = s_local[dd] + s_wh[w][dd] + rank[j];
      s_keys[lp] = key[j];
      s_vals[lp] = val[j];
    }
  }
  __syncthreads();
  const uint32_t nvalid = (uint32_t)((n - base) < (uint64_t)kPart ? (n - base) : (uint64_t)kPart);
  for (uint32_t i = t; i < nvalid; i += kSortThreads) {
    const uint32_t k = s_keys[i];
    const uint32_t dd = (k >> shift) & 255u;
    const uint32_t dst = s_gbase[dd] + (i - s_local[dd]);
    keys_out[dst] = k;
    vals_out[dst] = s_vals[i];
  }
}

// ------------------------------------------------------------- duplicate
__global__ __launch_bounds__(256) void k_duplicate(const void* __restrict__ table, const uint32_t* __restrict__ ids,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint32_t* __restrict__ rect,
                                                   const uint32_t* __restrict__ counters,
                                                   uint32_t* __restrict__ tkeys, uint32_t* __restrict__ pvals) {
  if (counters[C_OVERFLOW]) return;
  const uint32_t V = counters[C_NUM_VISIBLE];
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= V) return;
  const uint32_t item = ids[j];
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry* views = table_views(table);
  // view containing this item
  int lo = 0, hi = hdr->num_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].item_offset <= (int64_t)item) lo = mid; else hi = mid - 1;
  }
  const ViewEntry& V_ = views[lo];
  const uint2 r = reinterpret_cast<const uint2*>(rect)[item];
  const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
  uint32_t o = offsets[j];
  for (uint32_t ty = y0; ty < y1; ++ty) {
    const uint32_t rowbase = (uint32_t)V_.tile_offset + ty * (uint32_t)V_.tiles_x;
    for (uint32_t tx = x0; tx < x1; ++tx) {
      tkeys[o] = rowbase + tx;
      pvals[o] = item;
      ++o;
    }
  }
}

// ---------------------------------------------------------------- ranges
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ counters,
                                                uint32_t* __restrict__ ranges) {
  if (counters[C_OVERFLOW]) return;
  const uint32_t P = counters[C_NUM_PAIRS];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const uint32_t tk = tkeys[i];
  if (i == 0 || tkeys[i - 1] != tk) ranges[2 * (size_t)tk] = i;
  if (i == P - 1 || tkeys[i + 1] != tk) ranges[2 * (size_t)tk + 1] = i + 1;
}

__global__ __launch_bounds__(256) void k_keys64(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ vals,
                                                const uint32_t* __restrict__ depth_bits,
                                                const uint32_t* __restrict__ counters, uint64_t* __restrict__ keys) {
  if (counters[C_OVERFLOW]) return;
  const uint32_t P = counters[C_NUM_PAIRS];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  keys[i] = ((uint64_t)tkeys[i] << 32) | (uint64_t)depth_bits[vals[i]];
}

// ------------------------------------------------------------------ plan
static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

BinSortPlan plan_bin_sort(int64_t items, int64_t capacity, int32_t total_tiles) {
  BinSortPlan p{};
  p.items = items;
  p.capacity = capacity;
  p.total_tiles = total_tiles;
  int bits = 1;
  while (bits < 31 && (1ll << bits) < (int64_t)total_tiles) ++bits;
  p.tile_bits = bits;
  p.parts_items = (items + kPart - 1) / kPart;
  p.parts_pairs = (capacity + kPart - 1) / kPart;
  const int tpass = (bits + 7) / 8;
  size_t off = 0;
  p.off_counters = off; off = align_up(off + C_COUNT * 4);
  p.off_hist = off; off = align_up(off + (size_t)(kDepthPasses + kMaxTilePasses) * kRadix * 4);
  p.off_look_scan = off; off = align_up(off + (size_t)2 * (p.parts_items + 1) * 4);
  const size_t head_end = off;  // everything before here is cleared at the start
  (void)head_end;
  p.off_look_sort = off;
  off = align_up(off + ((size_t)p.parts_items * kDepthPasses + (size_t)p.parts_pairs * tpass) * kRadix * 4);
  p.off_dkeys_a = off; off = align_up(off + (size_t)items * 4);
  p.off_dkeys_b = off; off = align_up(off + (size_t)items * 4);
  p.off_dvals_a = off; off = align_up(off + (size_t)items * 4);
  p.off_dvals_b = off; off = align_up(off + (size_t)items * 4);
  p.off_offsets = off; off = align_up(off + (size_t)items * 4);
  p.off_tkeys_a = off; off = align_up(off + (size_t)capacity * 4);
  p.off_tkeys_b = off; off = align_up(off + (size_t)capacity * 4);
  p.off_pvals_b = off; off = align_up(off + (size_t)capacity * 4);
  p.bytes = off;
  return p;
}

hipError_t launch_bin_sort(const gabsplat_geom& g, const BinSortPlan& p, void* ws, uint64_t* keys, uint32_t* vals,
                           uint32_t* ranges, int64_t* d_num_pairs, int32_t* d_overflow, hipStream_t s) {
  char* w = static_cast<char*>(ws);
  uint32_t* counters = reinterpret_cast<uint32_t*>(w + p.off_counters);
  uint32_t* hist = reinterpret_cast<uint32_t*>(w + p.off_hist);
  uint32_t* look_scan = reinterpret_cast<uint32_t*>(w + p.off_look_scan);
  uint32_t* look_depth = reinterpret_cast<uint32_t*>(w + p.off_look_sort);
  uint32_t* look_tile = look_depth + (size_t)p.parts_items * kDepthPasses * kRadix;
  uint32_t* dk[2] = {reinterpret_cast<uint32_t*>(w + p.off_dkeys_a), reinterpret_cast<uint32_t*>(w + p.off_dkeys_b)};
  uint32_t* dv[2] = {reinterpret_cast<uint32_t*>(w + p.off_dvals_a), reinterpret_cast<uint32_t*>(w + p.off_dvals_b)};
  uint32_t* offsets = reinterpret_cast<uint32_t*>(w + p.off_offsets);
  uint32_t* tk[2] = {reinterpret_cast<uint32_t*>(w + p.off_tkeys_a), reinterpret_cast<uint32_t*>(w + p.off_tkeys_b)};
  const int tpass = (p.tile_bits + 7) / 8;
  // pair values: the last tile pass must write into the caller's `vals`
  uint32_t* pv[2];
  if (tpass % 2 == 0) {
    pv[0] = vals;
    pv[1] = reinterpret_cast<uint32_t*>(w + p.off_pvals_b);
  } else {
    pv[0] = reinterpret_cast<uint32_t*>(w + p.off_pvals_b);
    pv[1] = vals;
  }
  const uint32_t* depth_bits = reinterpret_cast<const uint32_t*>(g.depth);
  hipError_t e;

  // clear counters, histograms and the scan look-back, and the tile ranges
  e = fill_u32(counters, 0u, (p.off_look_sort - p.off_counters) / 4, s);
  if (e != hipSuccess) return e;
  e = fill_u32(ranges, 0u, (size_t)p.total_tiles * 2, s);
  if (e != hipSuccess) return e;
  const unsigned parts_i = (unsigned)(p.parts_items > 0 ? p.parts_items : 1);
  const unsigned parts_p = (unsigned)(p.parts_pairs > 0 ? p.parts_pairs : 1);
  uint32_t* look_scan0 = look_scan;
  uint32_t* look_scan1 = look_scan + (p.parts_items + 1);

  // K2a: compaction of visible items (depth keys + ids)
  if (p.items > 0)
    hipLaunchKernelGGL(k_scan<0>, dim3(parts_i), dim3(kSortThreads), 0, s, (uint32_t)p.items, g.tiles, depth_bits,
                       nullptr, dk[0], dv[0], counters, look_scan0);
  // depth sort: 4 passes over V
  hipLaunchKernelGGL(k_fill_prefix, dim3(256), dim3(256), 0, s, look_depth, counters + C_NUM_VISIBLE,
                     (uint32_t)(kDepthPasses * kRadix), nullptr);
  hipLaunchKernelGGL(k_histogram, dim3(parts_i), dim3(kSortThreads), 0, s, dk[0], counters + C_NUM_VISIBLE,
                     kDepthPasses, hist, nullptr);
  hipLaunchKernelGGL(k_hist_scan, dim3(1), dim3(kSortThreads), 0, s, hist, kDepthPasses, nullptr);
  for (int ps = 0; ps < kDepthPasses; ++ps) {
    const int a = ps & 1;
    hipLaunchKernelGGL(k_onesweep, dim3(parts_i), dim3(kSortThreads), 0, s, dk[a], dv[a], dk[a ^ 1], dv[a ^ 1],
                       counters + C_NUM_VISIBLE, 8 * ps, ps, kDepthPasses, hist + ps * kRadix, look_depth,
                       counters + C_TICKET_DEPTH + ps, nullptr);
  }
  // result in dk[0], dv[0] (even number of passes)
  // K2b: tile offsets in depth order, P, overflow
  hipLaunchKernelGGL(k_scan<1>, dim3(parts_i), dim3(kSortThreads), 0, s, 0u, g.tiles, nullptr, dv[0], offsets,
                     nullptr, counters, look_scan1);
  hipLaunchKernelGGL(k_finalize_pairs, dim3(1), dim3(1), 0, s, counters, p.capacity, d_num_pairs, d_overflow);
  // K3: duplicate (pairs in depth order)
  hipLaunchKernelGGL(k_duplicate, dim3(parts_i * (kPart / 256)), dim3(256), 0, s, g.views, dv[0], offsets, g.rect,
                     counters, tk[0], pv[0]);
  // K4: tile passes over P
  uint32_t* thist = hist + kDepthPasses * kRadix;
  hipLaunchKernelGGL(k_fill_prefix, dim3(1024), dim3(256), 0, s, look_tile, counters + C_NUM_PAIRS,
                     (uint32_t)(tpass * kRadix), d_overflow);
  hipLaunchKernelGGL(k_histogram, dim3(parts_p), dim3(kSortThreads), 0, s, tk[0], counters + C_NUM_PAIRS, tpass,
                     thist, d_overflow);
  hipLaunchKernelGGL(k_hist_scan, dim3(1), dim3(kSortThreads), 0, s, thist, tpass, d_overflow);
  for (int ps = 0; ps < tpass; ++ps) {
    const int a = ps & 1;
    hipLaunchKernelGGL(k_onesweep, dim3(parts_p), dim3(kSortThreads), 0, s, tk[a], pv[a], tk[a ^ 1], pv[a ^ 1],
                       counters + C_NUM_PAIRS, 8 * ps, ps, tpass, thist + ps * kRadix, look_tile,
                       counters + C_TICKET_TILE + ps, d_overflow);
  }
  uint32_t* tk_final = tk[tpass & 1];
  // K5: ranges
  const unsigned pblocks = (unsigned)((p.capacity + 255) / 256 > 0 ? (p.capacity + 255) / 256 : 1);
  hipLaunchKernelGGL(k_ranges, dim3(pblocks), dim3(256), 0, s, tk_final, counters, ranges);
  if (keys)
    hipLaunchKernelGGL(k_keys64, dim3(pblocks), dim3(256), 0, s, tk_final, vals, depth_bits, counters, keys);
  return hipGetLastError();
}

}  // namespace gs
