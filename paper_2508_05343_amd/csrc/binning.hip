// K2-K5: binning -- the (tile, item) pairs of every visible item ordered by
// tile, then fp32 depth bits, then item index (the stable sort of the 64-bit
// key tile << 32 | depth bits), and the per-tile ranges.
//
// Frames of at most kTcMaxTiles tiles (one view up to 1920x1080, say) take
// the tile-count path: per-block tile histograms in LDS, per-tile column
// offsets and one scan of the tile totals (which are the ranges), a scatter
// of (depth bits << 32 | item) into each tile's segment through per-block
// LDS cursors, and a sort of every segment by that unique key (one wavefront
// per tile, bitonic in registers; runs of 1024 merged for longer segments).
// Five launches, no global radix passes and no global atomics.  When the
// caller does not ask for the keys, the scatter writes the item ids of each
// segment straight into vals and leaves their order to the forward blend,
// which sorts each list of up to kBlendSortCap pairs in LDS before blending
// it (sorted there, it costs no separate pass over the pairs); only longer
// lists are sorted here.
//
// Larger batches (many views) take the radix path: an LSD radix sort over
// the same key that first sorts by the 32 depth bits and then, stably, by
// the tile bits.  All pairs of one primitive share its depth, so the depth
// passes run on the visible primitives before duplication (V items instead
// of P pairs); duplication then emits pairs in depth order and only
// ceil(tile_bits / 8) passes of equal digit width run on the P pairs.  Every
// pass is reduce-then-scan: per-block digit counts over contiguous ranges of
// partitions of 4096 keys, one scan into (digit, block) output bases, and a
// downsweep that ranks each partition in LDS with wave64 ballot matching and
// places it stably.  Launch sequence: clear the workspace head; compaction of
// the visible items; 4 depth passes; tiles-touched scan; pair emission
// balanced over fixed chunks of pairs; the tile passes; per-tile ranges from
// the boundaries between runs of equal tile keys.
#include <hip/hip_runtime.h>

#include "gs_block.h"
#include "gs_internal.h"
#include "gs_sort.h"

namespace gs {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kPart = kSortThreads * kSortItems;   // 4096 keys per partition
constexpr int kRadix = 256;
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 1u << 31;
constexpr uint32_t kCountMask = (1u << 30) - 1;
constexpr int kDepthPasses = 4;
constexpr int kMaxTilePasses = 4;
constexpr unsigned kLoopBlocks = 512;  // two 256-lane blocks per CU
constexpr int kEmitChunk = 2048;                  // pairs per emission chunk
constexpr int kEmitItems = kEmitChunk / kSortThreads;  // consecutive pairs walked per thread

// counters (u32) at the start of the workspace
enum {
  C_TICKET_EXPAND = 1,
  C_NUM_VISIBLE = 16,
  C_NUM_PAIRS = 17,
  C_OVERFLOW = 18,
  C_LONG_TILES = 19,  // tile-count path without keys: lists longer than the blend sorts
  C_COUNT = 64
};

__device__ __forceinline__ uint32_t ld_flag(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back on a single-value status array, run by one whole wave:
// each step reads the status words of 64 predecessors at once (one load per
// lane), so a walk over p predecessors takes ceil(p / 64) memory round trips
// instead of p.  Returns the exclusive prefix of partition `part` (to every
// lane) after publishing its inclusive value.  Must be called by all 64 lanes.
__device__ __forceinline__ uint32_t lookback_wave(uint32_t* look, uint32_t part, uint32_t aggregate) {
  const int l = __lane_id();
  if (part == 0) {
    if (l == 0) st_flag(&look[0], kFlagInc | aggregate);
    return 0;
  }
  if (l == 0) st_flag(&look[part], kFlagAgg | aggregate);
  uint32_t excl = 0;
  int64_t hi = (int64_t)part - 1;  // newest predecessor not yet accounted for
  while (true) {
    const int64_t p = hi - l;
    uint32_t v = (p >= 0) ? ld_flag(&look[p]) : kFlagInc;  // before partition 0: an inclusive zero
    // wait until every lane's predecessor has published something
    while (__ballot((v & (kFlagAgg | kFlagInc)) == 0) != 0ull) {
      __builtin_amdgcn_s_sleep(1);
      if ((v & (kFlagAgg | kFlagInc)) == 0) v = ld_flag(&look[p]);
    }
    const uint64_t inc = __ballot((v & kFlagInc) != 0);
    // lanes up to (and including) the nearest inclusive predecessor contribute
    const int stop = inc ? __builtin_ctzll(inc) : 64;
    uint32_t c = (l <= stop) ? (v & kCountMask) : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    excl += c;
    if (inc) break;
    hi -= 64;
  }
  if (l == 0) st_flag(&look[part], kFlagInc | (excl + aggregate));
  return excl;
}

// ----------------------------------------------------------------- fill
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// two regions in one launch (the workspace head and the tile ranges)
__global__ void k_fill2_u32(uint32_t* __restrict__ p, size_t n, uint32_t* __restrict__ q, size_t m) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + m; i += stride) {
    if (i < n) p[i] = 0u; else q[i - n] = 0u;
  }
}

hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------- compaction
// The visible items (tiles[i] > 0) with their depth keys, in item order, and
// V, without a single-pass chain: block b owns a contiguous range of items
// (whole steps of kPart); k_cs_count counts its visible items, k_cs_scan turns
// the counts into block offsets and writes V, k_cs_write re-reads the range
// step by step and writes every step in item order.
__device__ __forceinline__ void cs_range(uint64_t n, uint64_t* b0, uint64_t* b1) {
  const uint64_t nparts = (n + kPart - 1) / kPart;
  const uint64_t per = (nparts + gridDim.x - 1) / gridDim.x;
  *b0 = min(n, (uint64_t)blockIdx.x * per * kPart);
  *b1 = min(n, *b0 + per * kPart);
}

__device__ __forceinline__ uint32_t block_total_256(uint32_t v, uint32_t* s_wave) {
  uint32_t total;
  (void)block_excl_scan(v, s_wave, &total);
  return total;
}

__global__ __launch_bounds__(kSortThreads) void k_cs_count(uint64_t n, const uint32_t* __restrict__ tiles,
                                                           uint32_t* __restrict__ bcount) {
  __shared__ uint32_t s_wave[kSortThreads / 64];
  uint64_t b0, b1;
  cs_range(n, &b0, &b1);
  uint32_t c = 0;
  constexpr int kU = 8;  // loads in flight per lane
  for (uint64_t i0 = b0 + threadIdx.x; i0 < b1; i0 += (uint64_t)kU * kSortThreads) {
    uint32_t x[kU];
#pragma unroll
    for (int j = 0; j < kU; ++j) {
      const uint64_t i = i0 + (uint64_t)j * kSortThreads;
      x[j] = i < b1 ? tiles[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kU; ++j) c += x[j] > 0u ? 1u : 0u;
  }
  const uint32_t total = block_total_256(c, s_wave);
  if (threadIdx.x == 0) bcount[blockIdx.x] = total;
}

// One block: bcount[b] := visible items of the blocks before b; V.  nblocks <= 4 * kSortThreads.
__global__ __launch_bounds__(kSortThreads) void k_cs_scan(uint32_t* __restrict__ bcount, int nblocks,
                                                          uint32_t* __restrict__ counters) {
  __shared__ uint32_t s_wave[kSortThreads / 64];
  const int t = threadIdx.x;
  uint32_t c[4], sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int b = 4 * t + j;
    c[j] = b < nblocks ? bcount[b] : 0u;
    sum += c[j];
  }
  uint32_t total;
  uint32_t run = block_excl_scan(sum, s_wave, &total);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int b = 4 * t + j;
    if (b < nblocks) bcount[b] = run;
    run += c[j];
  }
  if (t == 0) counters[C_NUM_VISIBLE] = total;
}

__global__ __launch_bounds__(kSortThreads) void k_cs_write(uint64_t n, const uint32_t* __restrict__ tiles,
                                                           const uint32_t* __restrict__ depth_bits,
                                                           const uint32_t* __restrict__ bcount,
                                                           uint32_t* __restrict__ dkeys, uint32_t* __restrict__ dvals) {
  // A step of kPart items is loaded striped (item base + j * 256 + t:
  // coalesced).  Item order is (j, wave, lane), so an item's output position
  // is the number of visible items in the earlier (j, wave) slots plus its
  // rank in its wave's ballot.
  constexpr int kWaves = kSortThreads / 64;
  constexpr int kSlots = kSortItems * kWaves;
  static_assert(kSlots == 64, "one lane of wave 0 per (j, wave) slot");
  __shared__ uint32_t s_cnt[kSlots];
  __shared__ uint32_t s_total;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
  uint64_t b0, b1;
  cs_range(n, &b0, &b1);
  uint32_t run = bcount[blockIdx.x];
  for (uint64_t base = b0; base < b1; base += kPart) {
    bool vis[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const uint64_t i = base + (uint64_t)j * kSortThreads + t;
      vis[j] = i < b1 && tiles[i] > 0u;
    }
    uint64_t bal[kSortItems];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) bal[j] = __ballot(vis[j]);
    __syncthreads();  // the previous step's readers of s_cnt and s_total are done
    if (l == 0) {
#pragma unroll
      for (int j = 0; j < kSortItems; ++j) s_cnt[j * kWaves + w] = (uint32_t)__popcll(bal[j]);
    }
    __syncthreads();
    if (t < 64) {  // exclusive scan over the slots, in item order
      const uint32_t c = s_cnt[t];
      const uint32_t inc = wave_incl_scan(c);
      s_cnt[t] = inc - c;
      if (t == 63) s_total = inc;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      if (vis[j]) {
        const uint64_t i = base + (uint64_t)j * kSortThreads + t;
        const uint32_t pos = run + s_cnt[j * kWaves + w] + (uint32_t)__popcll(bal[j] & lt_mask);
        dkeys[pos] = depth_bits[i];
        dvals[pos] = (uint32_t)i;
      }
    }
    run += s_total;
  }
}

// -------------------------------------------------------------- expansion
// k_expand_scan: over the V depth-sorted visible items, exclusive scan of
// tiles touched (single pass, wave-parallel decoupled look-back) into
// offsets[]; the last partition writes P and the overflow flag.  Every
// visible item touches at least one tile, so pair index c * kEmitChunk lies in
// exactly one item's range: that item's position is stored as chunk_first[c]
// (c < max_chunks) for the emission kernel.  Blocks take partitions from a
// ticket until they run past V.
__global__ __launch_bounds__(kSortThreads) void k_expand_scan(const uint32_t* __restrict__ tiles,
                                                              const uint32_t* __restrict__ ids, uint32_t capacity,
                                                              uint32_t* __restrict__ counters,
                                                              uint32_t* __restrict__ look,
                                                              uint32_t* __restrict__ offsets,
                                                              uint32_t* __restrict__ chunk_first, uint32_t max_chunks,
                                                              int64_t* __restrict__ d_num_pairs,
                                                              int32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_wave[kSortThreads / 64];
  __shared__ uint32_t s_misc[2];
  const int t = threadIdx.x;
  const uint32_t V = counters[C_NUM_VISIBLE];
  if (V == 0) {
    if (blockIdx.x == 0 && t == 0) {
      counters[C_NUM_PAIRS] = 0;
      counters[C_OVERFLOW] = 0;
      *d_num_pairs = 0;
      *d_overflow = 0;
    }
    return;
  }
  // Only the first ceil(V / kPart) blocks take tickets (one shared counter:
  // every ticket is a same-address atomic).  When the grid has a block per
  // partition each of them takes exactly one; otherwise blocks keep taking
  // tickets until they run past V.  A block only ever waits on partitions
  // that running blocks hold.
  const uint32_t nparts = (V + kPart - 1) / kPart;
  if (blockIdx.x >= nparts) return;
  const bool one_each = gridDim.x >= nparts;
  for (;;) {
    __syncthreads();
    if (t == 0) s_misc[0] = atomicAdd(&counters[C_TICKET_EXPAND], 1u);
    __syncthreads();
    const uint32_t part = s_misc[0];
    const uint64_t base = (uint64_t)part * kPart;
    if (base >= V) return;
    const uint64_t first = base + (uint64_t)t * kSortItems;
    uint32_t x[kSortItems];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const uint64_t jj = first + j;
      x[j] = jj < V ? tiles[ids[jj]] : 0u;
      sum += x[j];
    }
    uint32_t block_total;
    const uint32_t tpre = block_excl_scan(sum, s_wave, &block_total);
    if (t < 64) {
      const uint32_t excl = lookback_wave(look, part, block_total);
      if (t == 0) {
        s_misc[1] = excl;
        if (base + kPart >= V) {
          const uint32_t P = excl + block_total;
          const uint32_t ov = P > capacity ? 1u : 0u;
          counters[C_NUM_PAIRS] = P;
          counters[C_OVERFLOW] = ov;
          *d_num_pairs = (int64_t)P;
          *d_overflow = (int32_t)ov;
        }
      }
    }
    __syncthreads();
    uint32_t pos = s_misc[1] + tpre;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const uint64_t jj = first + j;
      if (jj < V) {
        offsets[jj] = pos;
        for (uint32_t c = (pos + kEmitChunk - 1) / kEmitChunk;
             c < max_chunks && (uint64_t)c * kEmitChunk < (uint64_t)pos + x[j]; ++c)
          chunk_first[c] = (uint32_t)jj;
      }
      pos += x[j];
    }
    if (one_each) return;
  }
}

// Adds 1 to s_h[d] for every active lane with `on`, one LDS atomic per group of
// lanes sharing the digit (ballot matching), so that the common case of a
// whole wave on one digit costs one atomic instead of 64 serialised ones.
template <int RB = 8>
__device__ __forceinline__ void wave_hist_add(uint32_t* s_h, uint32_t d, bool on) {
  uint64_t peers = __ballot(on);
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  const int l = __lane_id();
  if (on && (peers >> l) == 1ull) atomicAdd(&s_h[d], (uint32_t)__popcll(peers));
}

// k_emit: globally load-balanced pair emission.  Chunk c holds pairs
// [c * kEmitChunk, (c + 1) * kEmitChunk) of the depth-ordered pair sequence; blocks
// stride over the chunks.  For one chunk a block first stages, for each item
// from chunk_first[c] to chunk_first[c + 1], its pair offset, id, first tile (view tile offset +
// rect corner) and rect width / tiles per row in LDS (coalesced loads plus
// one gather of the rects, all in parallel); every thread then finds the
// item of its first pair (one binary search) and walks its kEmitItems consecutive
// pairs item by item and tile by tile (row-major inside the rect) in LDS
// alone.  The block writes the (tile, item) pairs coalesced from LDS while
// accumulating the tile-digit histograms of the tile passes.
constexpr int kPad = kEmitChunk + kEmitChunk / kEmitItems;  // LDS index i + i / kEmitItems: conflict-free runs
constexpr int kEmitViews = 1024;  // views whose table columns are cached in LDS (more: searched in memory)

__global__ __launch_bounds__(kSortThreads) void k_emit(const void* __restrict__ table,
                                                       const uint32_t* __restrict__ rect,
                                                       const uint32_t* __restrict__ ids,
                                                       const uint32_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ chunk_first,
                                                       const uint32_t* __restrict__ counters, uint32_t* __restrict__ tkeys,
                                                       uint32_t* __restrict__ pvals) {
  __shared__ uint32_t s_off[kEmitChunk];
  __shared__ uint32_t s_id[kEmitChunk];
  __shared__ uint2 s_geo[kEmitChunk];  // (first tile, width | tiles per row << 16)
  __shared__ uint32_t s_tile[kPad];
  __shared__ uint32_t s_item[kPad];
  // view table columns (first item, first tile, tiles per row) for the item -> view search
  __shared__ uint32_t s_vitem[kEmitViews], s_vtile[kEmitViews], s_vtx[kEmitViews];
  if (counters[C_OVERFLOW]) return;
  const uint32_t P = counters[C_NUM_PAIRS];
  const uint32_t V = counters[C_NUM_VISIBLE];
  if ((uint64_t)blockIdx.x * kEmitChunk >= P) return;
  const int t = threadIdx.x;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry* views = table_views(table);
  const int nv = hdr->num_views;
  const bool cached = nv <= kEmitViews;
  if (cached) {
    for (int v = t; v < nv; v += kSortThreads) {
      s_vitem[v] = (uint32_t)views[v].item_offset;  // items < 2^32
      s_vtile[v] = (uint32_t)views[v].tile_offset;
      s_vtx[v] = (uint32_t)views[v].tiles_x;
    }
  }
  for (uint64_t chunk = blockIdx.x; chunk * kEmitChunk < P; chunk += gridDim.x) {
    const uint64_t p0 = chunk * kEmitChunk;
    __syncthreads();
    // the chunk's pairs belong to items first .. chunk_first[chunk + 1] (the
    // item holding the next chunk's first pair; V - 1 for the last chunk)
    const uint32_t first = chunk_first[chunk];
    const uint64_t nchunks = ((uint64_t)P + kEmitChunk - 1) / kEmitChunk;
    const uint32_t last = chunk + 1 < nchunks ? chunk_first[chunk + 1] : V - 1;
    const uint32_t nitems = min((uint32_t)kEmitChunk, last - first + 1);
    for (uint32_t i = t; i < nitems; i += kSortThreads) {
      const uint32_t item = ids[first + i];
      s_off[i] = offsets[first + i];
      s_id[i] = item;
      const uint2 r = reinterpret_cast<const uint2*>(rect)[item];
      int vlo = 0, vhi = nv - 1;
      uint32_t tx, toff;
      if (cached) {
        while (vlo < vhi) {
          const int mid = (vlo + vhi + 1) >> 1;
          if (s_vitem[mid] <= item) vlo = mid; else vhi = mid - 1;
        }
        tx = s_vtx[vlo];
        toff = s_vtile[vlo];
      } else {
        while (vlo < vhi) {
          const int mid = (vlo + vhi + 1) >> 1;
          if (views[mid].item_offset <= (int64_t)item) vlo = mid; else vhi = mid - 1;
        }
        tx = (uint32_t)views[vlo].tiles_x;
        toff = (uint32_t)views[vlo].tile_offset;
      }
      const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16;
      s_geo[i] = make_uint2(toff + y0 * tx + x0, ((r.y & 0xffffu) - x0) | (tx << 16));
    }
    __syncthreads();
    const uint32_t pend = (uint32_t)min((uint64_t)P, p0 + kEmitChunk);
    const uint32_t mb = (uint32_t)p0 + (uint32_t)t * kEmitItems;
    if (mb < pend) {
      uint32_t lo = 0, hi = nitems - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= mb) lo = mid; else hi = mid - 1;
      }
      uint32_t cur = lo;
      uint2 gg = s_geo[cur];
      uint32_t wdt = gg.y & 0xffffu, tx = gg.y >> 16;
      const uint32_t q = mb - s_off[cur];
      uint32_t row = q / wdt, col = q - row * wdt;
      uint32_t next = cur + 1 < nitems ? s_off[cur + 1] : 0xffffffffu;
#pragma unroll 1
      for (int j = 0; j < kEmitItems; ++j) {
        const uint32_t m = mb + (uint32_t)j;
        if (m >= pend) break;
        if (m >= next) {  // the next item starts exactly here (every item has >= 1 pair)
          ++cur;
          gg = s_geo[cur];
          wdt = gg.y & 0xffffu;
          tx = gg.y >> 16;
          row = 0;
          col = 0;
          next = cur + 1 < nitems ? s_off[cur + 1] : 0xffffffffu;
        }
        const uint32_t li = (uint32_t)t * (kEmitItems + 1) + (uint32_t)j;
        s_tile[li] = gg.x + row * tx + col;
        s_item[li] = s_id[cur];
        if (++col == wdt) {
          col = 0;
          ++row;
        }
      }
    }
    __syncthreads();
    for (uint32_t i = t; i < pend - (uint32_t)p0; i += kSortThreads) {
      const uint32_t li = i + i / kEmitItems;
      tkeys[(uint32_t)p0 + i] = s_tile[li];
      pvals[(uint32_t)p0 + i] = s_item[li];
    }
  }
}

// ------------------------------------------------ reduce-then-scan passes
// Every pass of the radix path (depth passes over the V visible items, tile
// passes over the P pairs) is a reduce-then-scan LSD pass.  With hundreds of
// partitions in flight, a single-pass look-back makes every partition read
// the digit words of each of them, and those loads bound the pass; here
// nothing waits on another block.  Block b owns a contiguous
// range of partitions of kPart keys: (1) k_rs_upsweep counts its digits (and
// adds them into the pass's global histogram), (2) k_rs_scan turns the counts
// into the output base of every (digit, block), (3) k_rs_downsweep re-reads the
// range and places each partition stably (ranks from wave64 ballot matching),
// advancing the block's digit bases partition by partition.
constexpr int kRsBlocks = 768;  // three 256-lane downsweep blocks per CU (141 VGPRs, 39 KB LDS)
static_assert(kRadix == kSortThreads, "one lane per digit");

__device__ __forceinline__ void rs_range(uint32_t n, uint32_t* p0, uint32_t* p1) {
  const uint32_t nparts = (uint32_t)(((uint64_t)n + kPart - 1) / kPart);
  const uint32_t per = (nparts + gridDim.x - 1) / gridDim.x;
  *p0 = min(nparts, blockIdx.x * per);
  *p1 = min(nparts, *p0 + per);
}

// bhist[d * gridDim.x + b] = keys of block b's range with digit d; ghist[d] += the same.
constexpr int kRsUpThreads = 512;
template <int RB>
__global__ __launch_bounds__(kRsUpThreads) void k_rs_upsweep(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ d_count, int shift,
                                                             uint32_t* __restrict__ bhist,
                                                             uint32_t* __restrict__ ghist,
                                                             const uint32_t* __restrict__ d_overflow) {
  constexpr int D = 1 << RB;
  __shared__ uint32_t s_h[D];
  if (d_overflow != nullptr && *d_overflow != 0) return;
  const uint32_t n = *d_count;
  const int t = threadIdx.x;
  if (t < D) s_h[t] = 0;
  __syncthreads();
  uint32_t p0, p1;
  rs_range(n, &p0, &p1);
  const uint64_t b0 = (uint64_t)p0 * kPart, b1 = min((uint64_t)n, (uint64_t)p1 * kPart);
  constexpr int kU = 8;  // loads in flight per lane
  for (uint64_t i0 = b0; i0 < b1; i0 += (uint64_t)kU * kRsUpThreads) {  // uniform trip count
    uint32_t k[kU];
#pragma unroll
    for (int j = 0; j < kU; ++j) {
      const uint64_t i = i0 + (uint64_t)j * kRsUpThreads + t;
      k[j] = i < b1 ? keys[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kU; ++j)
      wave_hist_add<RB>(s_h, (k[j] >> shift) & (uint32_t)(D - 1), i0 + (uint64_t)j * kRsUpThreads + t < b1);
  }
  __syncthreads();
  if (t < D) {
    const uint32_t c = s_h[t];
    bhist[(size_t)t * gridDim.x + blockIdx.x] = c;
    if (c) atomicAdd(&ghist[t], c);
  }
}

// Block d: bhist[d][b] := (keys with a digit below d) + (keys with digit d in
// the ranges of blocks before b).  nblocks <= 4 * kSortThreads.
static_assert(kRsBlocks <= 4 * kSortThreads, "k_rs_scan covers four blocks per lane");
template <int RB>
__global__ __launch_bounds__(kSortThreads) void k_rs_scan(uint32_t* __restrict__ bhist, int nblocks,
                                                          const uint32_t* __restrict__ ghist,
                                                          const uint32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_wave[kSortThreads / 64];
  __shared__ uint32_t s_base;
  if (d_overflow != nullptr && *d_overflow != 0) return;
  const int t = threadIdx.x, d = blockIdx.x;
  uint32_t dummy;
  const uint32_t below = block_excl_scan(t < (1 << RB) ? ghist[t] : 0u, s_wave, &dummy);
  if (t == d) s_base = below;
  uint32_t* row = bhist + (size_t)d * nblocks;
  uint32_t c[4], sum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int b = 4 * t + j;
    c[j] = b < nblocks ? row[b] : 0u;
    sum += c[j];
  }
  uint32_t run = block_excl_scan(sum, s_wave, &dummy);  // its barriers also publish s_base
  run += s_base;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int b = 4 * t + j;
    if (b < nblocks) row[b] = run;
    run += c[j];
  }
}

// keys per lane in the downsweep: 4096-key steps (about 16 keys per digit, so
// the scattered writes fill whole 64-byte sectors); 2048-key steps, with more
// blocks resident, measured slower
constexpr int kDsItems = 16;
constexpr int kDsPart = kSortThreads * kDsItems;
static_assert(kPart % kDsPart == 0, "block ranges split into whole sub-partitions");

template <int RB>
__global__ __launch_bounds__(kSortThreads) void k_rs_downsweep(const uint32_t* __restrict__ keys_in,
                                                               const uint32_t* __restrict__ vals_in,
                                                               uint32_t* __restrict__ keys_out,
                                                               uint32_t* __restrict__ vals_out,
                                                               const uint32_t* __restrict__ d_count, int shift,
                                                               const uint32_t* __restrict__ bbase,
                                                               const uint32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_keys[kDsPart];
  __shared__ uint32_t s_vals[kDsPart];
  constexpr int D = 1 << RB;
  constexpr uint32_t kMask = (uint32_t)(D - 1);
  __shared__ uint32_t s_wh[kSortThreads / 64][D];
  __shared__ uint32_t s_local[D];
  __shared__ uint32_t s_run[D];
  __shared__ uint32_t s_wave[kSortThreads / 64];
  if (d_overflow != nullptr && *d_overflow != 0) return;
  const uint32_t n = *d_count;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  uint32_t p0, p1;
  rs_range(n, &p0, &p1);
  const uint64_t b0 = (uint64_t)p0 * kPart, b1 = min((uint64_t)n, (uint64_t)p1 * kPart);
  if (t < D) s_run[t] = bbase[(size_t)t * gridDim.x + blockIdx.x];
  const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (64 - l));
  for (uint64_t base = b0; base < b1; base += kDsPart) {
    __syncthreads();
    for (int i = t; i < (kSortThreads / 64) * D; i += kSortThreads) (&s_wh[0][0])[i] = 0;
    __syncthreads();
    // wave-striped load: wave w owns [w*64*kDsItems, (w+1)*64*kDsItems), item j of lane l at j*64 + l
    uint32_t key[kDsItems], val[kDsItems];
    uint16_t rank[kDsItems];
    const uint64_t wbase = base + (uint64_t)w * (64 * kDsItems);
#pragma unroll
    for (int j = 0; j < kDsItems; ++j) {
      const uint64_t i = wbase + (uint64_t)j * 64 + l;
      key[j] = i < b1 ? keys_in[i] : 0xffffffffu;
      val[j] = i < b1 ? vals_in[i] : 0u;
    }
    // stable rank within the wave's digit (ballot matching), in index order
#pragma unroll
    for (int j = 0; j < kDsItems; ++j) {
      const uint64_t i = wbase + (uint64_t)j * 64 + l;
      const bool ok = i < b1;
      const uint32_t d = (key[j] >> shift) & kMask;
      uint64_t peers = __ballot(ok);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
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
    // per digit (lane t = digit): wave prefixes, sub-partition count, local start
    uint32_t tot = 0;
    if (t < D) {
#pragma unroll
      for (int i = 0; i < kSortThreads / 64; ++i) {
        const uint32_t c = s_wh[i][t];
        s_wh[i][t] = tot;
        tot += c;
      }
    }
    uint32_t dummy;
    const uint32_t lstart = block_excl_scan(tot, s_wave, &dummy);
    if (t < D) s_local[t] = lstart;
    __syncthreads();
    // scatter into LDS in digit order
#pragma unroll
    for (int j = 0; j < kDsItems; ++j) {
      const uint64_t i = wbase + (uint64_t)j * 64 + l;
      if (i < b1) {
        const uint32_t dd = (key[j] >> shift) & kMask;
        const uint32_t lp = s_local[dd] + s_wh[w][dd] + rank[j];
        s_keys[lp] = key[j];
        s_vals[lp] = val[j];
      }
    }
    __syncthreads();
    const uint32_t nvalid = (uint32_t)((b1 - base) < (uint64_t)kDsPart ? (b1 - base) : (uint64_t)kDsPart);
    for (uint32_t i = t; i < nvalid; i += kSortThreads) {
      const uint32_t k = s_keys[i];
      const uint32_t dd = (k >> shift) & kMask;
      const uint32_t dst = s_run[dd] + (i - s_local[dd]);
      keys_out[dst] = k;
      vals_out[dst] = s_vals[i];
    }
    __syncthreads();
    if (t < D) s_run[t] += tot;
  }
}

// Tile ranges from the sorted tile keys: every lane takes 8 consecutive keys
// (two 16-byte loads) and their two neighbours, and writes the start / end of
// every tile that begins / ends among them.
constexpr int kRangeKeys = 8;
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tkeys,
                                                const uint32_t* __restrict__ counters,
                                                uint32_t* __restrict__ ranges) {
  if (counters[C_OVERFLOW]) return;
  const uint32_t P = counters[C_NUM_PAIRS];
  constexpr uint32_t kNone = 0xffffffffu;  // no tile (ids are below 2^31)
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kRangeKeys;
  for (uint64_t i0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeKeys; i0 < P; i0 += stride) {
    uint32_t k[kRangeKeys + 2];
    k[0] = i0 > 0 ? tkeys[i0 - 1] : kNone;
    if (i0 + kRangeKeys <= P) {
      const uint4 a = *reinterpret_cast<const uint4*>(tkeys + i0);
      const uint4 b = *reinterpret_cast<const uint4*>(tkeys + i0 + 4);
      k[1] = a.x; k[2] = a.y; k[3] = a.z; k[4] = a.w;
      k[5] = b.x; k[6] = b.y; k[7] = b.z; k[8] = b.w;
    } else {
#pragma unroll
      for (int j = 0; j < kRangeKeys; ++j) k[1 + j] = i0 + j < P ? tkeys[i0 + j] : kNone;
    }
    k[kRangeKeys + 1] = i0 + kRangeKeys < P ? tkeys[i0 + kRangeKeys] : kNone;
#pragma unroll
    for (int j = 0; j < kRangeKeys; ++j) {
      const uint32_t i = (uint32_t)(i0 + j), tk = k[1 + j];
      if (tk == kNone) break;
      if (k[j] != tk) ranges[2 * (size_t)tk] = i;
      if (k[j + 2] != tk) ranges[2 * (size_t)tk + 1] = i + 1;
    }
  }
}

__global__ __launch_bounds__(256) void k_keys64(const uint32_t* __restrict__ tkeys, const uint32_t* __restrict__ vals,
                                                const uint32_t* __restrict__ depth_bits,
                                                const uint32_t* __restrict__ counters, uint64_t* __restrict__ keys) {
  if (counters[C_OVERFLOW]) return;
  const uint32_t P = counters[C_NUM_PAIRS];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x)
    keys[i] = ((uint64_t)tkeys[i] << 32) | (uint64_t)depth_bits[vals[i]];
}

// ------------------------------------------------------ blend dispatch order
// The blend kernels give workgroup b the tile order[b], with the tiles in
// decreasing order of their list length (geometric buckets 2^(1/8) apart,
// arbitrary order inside a bucket; empty tiles last).  The hardware starts
// workgroups in index order as slots free up, so the longest tiles start
// first and the last workgroups to start are short ones: dispatched in image
// order, the densest tiles could start last and run with most of the GPU idle
// around them.  One workgroup; order lives after the ranges in tile_ranges.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 160;

__device__ __forceinline__ int order_bucket(uint32_t len) {
  if (len == 0u) return 0;
  // 1 + floor(8 log2 len), from the bit length and the next three mantissa bits
  const int lz = 31 - __builtin_clz(len);
  const uint32_t frac = lz >= 3 ? (len >> (lz - 3)) & 7u : (len << (3 - lz)) & 7u;
  const int b = 1 + 8 * lz + (int)frac;
  return b < kOrderBuckets ? b : kOrderBuckets - 1;
}

// Bucket counts -> bucket starts, longest bucket first: an exclusive scan of
// s_cnt in decreasing bucket order by the first wavefront (three buckets per
// lane, one shuffle scan).  The caller brackets it with barriers.
__device__ __forceinline__ void order_bucket_starts(uint32_t* s_cnt) {
  static_assert(kOrderBuckets <= 3 * 64, "three buckets per lane");
  if (threadIdx.x >= 64) return;
  const int l = threadIdx.x;
  uint32_t c[3], sum = 0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int b = kOrderBuckets - 1 - (3 * l + r);
    c[r] = b >= 0 ? s_cnt[b] : 0u;
    sum += c[r];
  }
  uint32_t inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, 64);
    if (l >= d) inc += o;
  }
  uint32_t run = inc - sum;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int b = kOrderBuckets - 1 - (3 * l + r);
    if (b >= 0) s_cnt[b] = run;
    run += c[r];
  }
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint32_t* __restrict__ ranges, int ntiles,
                                                              const uint32_t* __restrict__ counters,
                                                              uint32_t* __restrict__ order) {
  __shared__ uint32_t s_cnt[kOrderBuckets];
  if (counters[C_OVERFLOW]) return;
  const int t = threadIdx.x;
  for (int b = t; b < kOrderBuckets; b += kOrderThreads) s_cnt[b] = 0;
  __syncthreads();
  for (int i = t; i < ntiles; i += kOrderThreads)
    atomicAdd(&s_cnt[order_bucket(ranges[2 * (size_t)i + 1] - ranges[2 * (size_t)i])], 1u);
  __syncthreads();
  order_bucket_starts(s_cnt);
  __syncthreads();
  for (int i = t; i < ntiles; i += kOrderThreads) {
    const int b = order_bucket(ranges[2 * (size_t)i + 1] - ranges[2 * (size_t)i]);
    order[atomicAdd(&s_cnt[b], 1u)] = (uint32_t)i;
  }
}

// ---------------------------------------------------------- tile-count path
// For frames with at most kTcMaxTiles tiles the pairs are binned without a
// global radix sort: per-block tile histograms (LDS), per-tile column offsets
// and one scan of the tile totals into the tile ranges, a scatter of (depth
// bits, item) into each tile's segment through per-block LDS cursors
// (arbitrary order inside the segment), and a sort of every segment by the
// unique key (depth bits, item).  The result is the same order as the stable
// (tile, depth) sort of the radix path.
constexpr int kTcMaxTiles = 8192;   // per-block tile histograms in LDS (32 KB)
constexpr int kTcBig = 64;        // items with more tiles are walked by a whole wavefront
constexpr int kSegCap = 1024;     // segment sorted in registers in one piece (16 u64 keys per lane): one wavefront per tile

struct ItemTiles {
  uint32_t base;  // global tile id of the rect's top-left tile
  uint32_t w, h;  // rect width and height in tiles
  uint32_t tx;    // tiles per row of the item's view
};

__device__ __forceinline__ ItemTiles item_tiles(const ViewEntry* views, int nv, uint32_t item, uint2 r) {
  int vlo = 0, vhi = nv - 1;
  while (vlo < vhi) {
    const int mid = (vlo + vhi + 1) >> 1;
    if (views[mid].item_offset <= (int64_t)item) vlo = mid; else vhi = mid - 1;
  }
  const uint32_t x0 = r.x & 0xffffu, y0 = r.x >> 16, x1 = r.y & 0xffffu, y1 = r.y >> 16;
  ItemTiles it;
  it.tx = (uint32_t)views[vlo].tiles_x;
  it.base = (uint32_t)views[vlo].tile_offset + y0 * it.tx + x0;
  it.w = x1 - x0;
  it.h = y1 - y0;
  return it;
}

__device__ __forceinline__ uint32_t tile_of(const ItemTiles& it, uint32_t q) {
  const uint32_t row = q / it.w;
  return it.base + row * it.tx + (q - row * it.w);
}

// Calls f(item, tile) for every (visible item, tile) pair of the items
// i0 + k * blockDim + lane (k < kTcItems, below i1) of a wavefront: the tile
// counts and rectangles of all of them are loaded first.  The pairs of small
// rectangles are dealt out evenly: a wave prefix sum of the 64 items' pair
// counts numbers them, and lane l takes pairs l, l + 64, ..., finding the
// owning item by a binary search over the prefix sums (most items touch no
// tile or a few, so walking each item in its own lane would leave most
// lanes idle for as long as the largest item of the wave).  Large rectangles
// are walked by the whole wavefront.  Must be called by full wavefronts.
constexpr int kTcItems = 4;

template <typename F>
__device__ __forceinline__ void for_each_pair(const ViewEntry* views, int nv, const uint32_t* __restrict__ tiles,
                                              const uint32_t* __restrict__ rect, int64_t i0, int64_t i1, F f) {
  uint32_t nt[kTcItems];
  uint2 rc[kTcItems];
#pragma unroll
  for (int k = 0; k < kTcItems; ++k) {
    const int64_t i = i0 + (int64_t)k * blockDim.x + threadIdx.x;
    nt[k] = i < i1 ? tiles[i] : 0u;
    rc[k] = i < i1 ? reinterpret_cast<const uint2*>(rect)[i] : make_uint2(0u, 0u);
  }
  const int l = __lane_id();
#pragma unroll
  for (int k = 0; k < kTcItems; ++k) {
    const uint32_t item = (uint32_t)(i0 + (int64_t)k * blockDim.x + threadIdx.x);
    ItemTiles it{};
    uint32_t n = nt[k];
    if (n) {
      it = item_tiles(views, nv, item, rc[k]);
      n = min(n, it.w * it.h);  // never past the rectangle (and no division by a zero width)
    }
    // small rectangles: pairs numbered by a wave prefix sum, dealt to lanes
    const uint32_t ns = n <= (uint32_t)kTcBig ? n : 0u;
    uint32_t inc = ns;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = (uint32_t)__shfl_up((int)inc, d, 64);
      if (l >= d) inc += o;
    }
    const uint32_t total = (uint32_t)__shfl((int)inc, 63, 64);
    for (uint32_t p0 = 0; p0 < total; p0 += 64) {  // uniform trip count, every lane active
      const uint32_t p = min(p0 + (uint32_t)l, total - 1u);
      int src = 0;  // the first lane whose inclusive count exceeds p
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1)
        if ((uint32_t)__shfl((int)inc, src + step - 1, 64) <= p) src += step;
      const uint32_t s_inc = (uint32_t)__shfl((int)inc, src, 64), s_n = (uint32_t)__shfl((int)ns, src, 64);
      ItemTiles st;
      st.base = (uint32_t)__shfl((int)it.base, src, 64);
      st.w = (uint32_t)__shfl((int)it.w, src, 64);
      st.tx = (uint32_t)__shfl((int)it.tx, src, 64);
      const uint32_t s_item = (uint32_t)__shfl((int)item, src, 64);
      if (p0 + (uint32_t)l < total) f(s_item, tile_of(st, p - (s_inc - s_n)));
    }
    uint64_t big = __ballot(n > (uint32_t)kTcBig);
    while (big) {
      const int src = __builtin_ctzll(big);
      big &= big - 1;
      const uint32_t bi = (uint32_t)__shfl((int)item, src, 64);
      const uint32_t bn = (uint32_t)__shfl((int)n, src, 64);
      ItemTiles bt;
      bt.base = (uint32_t)__shfl((int)it.base, src, 64);
      bt.w = (uint32_t)__shfl((int)it.w, src, 64);
      bt.h = (uint32_t)__shfl((int)it.h, src, 64);
      bt.tx = (uint32_t)__shfl((int)it.tx, src, 64);
      for (uint32_t q = (uint32_t)l; q < bn; q += 64) f(bi, tile_of(bt, q));
    }
  }
}

// The items are split into kTcBlocks contiguous ranges, one per block of the
// histogram and scatter kernels (the same ranges in both).  The number of
// blocks sets the size of the count matrix (kTcBlocks x tiles); wide blocks
// keep enough wavefronts in flight to cover the load latency of their items.
constexpr int kTcBlocks = 512;
constexpr int kTcThreads = 1024;

__device__ __forceinline__ void tc_item_range(int64_t items, int64_t* i0, int64_t* i1) {
  const int64_t per = (items + kTcBlocks - 1) / kTcBlocks;
  *i0 = min(items, (int64_t)blockIdx.x * per);
  *i1 = min(items, *i0 + per);
}

// Per-block tile histograms in LDS, written as row blockIdx.x of cnt[kTcBlocks][T].
__global__ __launch_bounds__(kTcThreads) void k_tc_hist(const void* __restrict__ table, int64_t items,
                                                 const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ rect,
                                                 int ntiles, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_h[kTcMaxTiles];
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry* views = table_views(table);
  const int nv = hdr->num_views;
  for (int i = threadIdx.x; i < ntiles; i += blockDim.x) s_h[i] = 0;
  __syncthreads();
  int64_t i0, i1;
  tc_item_range(items, &i0, &i1);
  for (int64_t b = i0; b < i1; b += (int64_t)kTcItems * blockDim.x)  // uniform trip count
    for_each_pair(views, nv, tiles, rect, b, i1, [&](uint32_t, uint32_t t) { atomicAdd(&s_h[t], 1u); });
  __syncthreads();
  uint32_t* row = cnt + (size_t)blockIdx.x * ntiles;
  for (int i = threadIdx.x; i < ntiles; i += blockDim.x) row[i] = s_h[i];
}

// Column offsets: lane (tile j of the block's 32, group g of 8) sums 64
// rows; the 8 group sums of a tile are scanned in LDS; the per-block counts
// become exclusive offsets in place and the tile totals go to tot[].  32
// consecutive tiles make every row access one 128-byte line (8 tiles, 32-byte
// pieces, measured 6 us slower over the whole bin sort).
constexpr int kColTiles = 32, kColGroups = 8, kColRows = kTcBlocks / kColGroups;
__global__ __launch_bounds__(256) void k_tc_colscan(uint32_t* __restrict__ cnt, int ntiles,
                                                    uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_g[kColTiles][kColGroups + 1];
  const int j = threadIdx.x % kColTiles, g = threadIdx.x / kColTiles;
  const int tile = blockIdx.x * kColTiles + j;
  uint32_t c[kColRows];
  uint32_t sum = 0;
  if (tile < ntiles) {
#pragma unroll
    for (int r = 0; r < kColRows; ++r) c[r] = cnt[(size_t)(g * kColRows + r) * ntiles + tile];
#pragma unroll
    for (int r = 0; r < kColRows; ++r) sum += c[r];
  }
  s_g[j][g] = sum;
  __syncthreads();
  if (g == 0) {  // exclusive scan of the 32 group sums of tile j
    uint32_t run = 0;
    for (int q = 0; q < kColGroups; ++q) {
      const uint32_t v = s_g[j][q];
      s_g[j][q] = run;
      run += v;
    }
    if (tile < ntiles) tot[tile] = run;
  }
  __syncthreads();
  if (tile < ntiles) {
    uint32_t run = s_g[j][g];
#pragma unroll
    for (int r = 0; r < kColRows; ++r) {
      cnt[(size_t)(g * kColRows + r) * ntiles + tile] = run;
      run += c[r];
    }
  }
}

// One block: exclusive scan of the tile totals -> tile starts, ranges ((0, 0)
// for empty tiles), pair count and overflow flag; then the dispatch order of
// the segment sort and the blend (as k_tile_order) after the ranges.  The
// totals are staged in LDS with coalesced loads; each thread then scans
// kTileScanPer consecutive tiles held in registers (no dependent global loads)
// and the starts and ranges go out coalesced from LDS again.  With `direct`
// (no keys: the scatter writes ids and the blend orders the lists) every
// list of two or more pairs is marked unsorted (kUnsortedBit on its end) and
// the lists longer than kBlendSortCap are listed, into `tot` (whose totals are
// in LDS by then), for k_tc_sort_long.
constexpr int kTileScanThreads = 1024;
constexpr int kTileScanPer = kTcMaxTiles / kTileScanThreads;
__global__ __launch_bounds__(kTileScanThreads) void k_tc_tilescan(uint32_t* __restrict__ tot, int ntiles,
                                                             uint32_t capacity, int direct,
                                                             uint32_t* __restrict__ tstart,
                                                             uint32_t* __restrict__ ranges,
                                                             uint32_t* __restrict__ counters,
                                                             int64_t* __restrict__ d_num_pairs,
                                                             int32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_v[kTcMaxTiles];
  __shared__ uint32_t s_wave[kTileScanThreads / 64];
  __shared__ uint32_t s_cnt[kOrderBuckets];
  __shared__ uint32_t s_long;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
#pragma unroll
  for (int r = 0; r < kTileScanPer; ++r) {
    const int i = r * kTileScanThreads + t;
    if (i < ntiles) s_v[i] = tot[i];
  }
  if (t == 0) s_long = 0;
  for (int b = t; b < kOrderBuckets; b += kTileScanThreads) s_cnt[b] = 0;
  __syncthreads();
  const int i0 = t * kTileScanPer;
  uint32_t c[kTileScanPer], sum = 0;
#pragma unroll
  for (int r = 0; r < kTileScanPer; ++r) {
    c[r] = i0 + r < ntiles ? s_v[i0 + r] : 0u;
    sum += c[r];
  }
  // tiles per length bucket (dispatch order, longest bucket first)
#pragma unroll
  for (int r = 0; r < kTileScanPer; ++r)
    if (i0 + r < ntiles) atomicAdd(&s_cnt[order_bucket(c[r])], 1u);
  uint32_t inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, 64);
    if (l >= d) inc += o;
  }
  if (l == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t run = inc - sum, total = 0;
#pragma unroll
  for (int q = 0; q < kTileScanThreads / 64; ++q) {
    const uint32_t x = s_wave[q];
    run += q < w ? x : 0u;
    total += x;
  }
  order_bucket_starts(s_cnt);
  // every read of the totals in s_v is done: the starts replace them
#pragma unroll
  for (int r = 0; r < kTileScanPer; ++r) {
    if (i0 + r < ntiles) s_v[i0 + r] = run;
    run += c[r];
  }
  __syncthreads();
  uint32_t* order = ranges + 2 * (size_t)ntiles;
#pragma unroll
  for (int r = 0; r < kTileScanPer; ++r)
    if (i0 + r < ntiles) order[atomicAdd(&s_cnt[order_bucket(c[r])], 1u)] = (uint32_t)(i0 + r);
#pragma unroll
  for (int r = 0; r < kTileScanPer; ++r) {
    const int i = r * kTileScanThreads + t;
    if (i < ntiles) {
      const uint32_t st = s_v[i], nx = i + 1 < ntiles ? s_v[i + 1] : total;
      tstart[i] = st;
      ranges[2 * (size_t)i] = nx > st ? st : 0u;
      ranges[2 * (size_t)i + 1] = nx > st ? (nx | (direct && nx - st > 1u ? kUnsortedBit : 0u)) : 0u;
    }
  }
  if (direct) {
#pragma unroll
    for (int r = 0; r < kTileScanPer; ++r)
      if (i0 + r < ntiles && c[r] > (uint32_t)kBlendSortCap) tot[atomicAdd(&s_long, 1u)] = (uint32_t)(i0 + r);
  }
  __syncthreads();
  if (t == 0) {
    const uint32_t ov = total > capacity ? 1u : 0u;
    counters[C_NUM_PAIRS] = total;
    counters[C_OVERFLOW] = ov;
    counters[C_LONG_TILES] = s_long;
    *d_num_pairs = (int64_t)total;
    *d_overflow = (int32_t)ov;
  }
}

// Scatter of every (item, tile) pair into its tile's segment, as the 64-bit
// key (depth bits << 32 | item) into spair, or (ids given) as the item id
// straight into ids: block b owns the positions tstart[t] + cnt[b][t]
// onwards of each tile (LDS cursors, so the order inside a segment is
// arbitrary; the segment sort, or the blend, fixes it).
__global__ __launch_bounds__(kTcThreads) void k_tc_scatter(const void* __restrict__ table, int64_t items,
                                                    const uint32_t* __restrict__ tiles,
                                                    const uint32_t* __restrict__ rect,
                                                    const uint32_t* __restrict__ depth_bits, int ntiles,
                                                    const uint32_t* __restrict__ cnt,
                                                    const uint32_t* __restrict__ tstart,
                                                    const uint32_t* __restrict__ counters,
                                                    uint64_t* __restrict__ spair,
                                                    uint32_t* __restrict__ ids) {
  __shared__ uint32_t s_cur[kTcMaxTiles];
  if (counters[C_OVERFLOW]) return;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry* views = table_views(table);
  const int nv = hdr->num_views;
  const uint32_t* row = cnt + (size_t)blockIdx.x * ntiles;
  for (int i = threadIdx.x; i < ntiles; i += blockDim.x) s_cur[i] = tstart[i] + row[i];
  __syncthreads();
  int64_t i0, i1;
  tc_item_range(items, &i0, &i1);
  for (int64_t b = i0; b < i1; b += (int64_t)kTcItems * blockDim.x)
    for_each_pair(views, nv, tiles, rect, b, i1, [&](uint32_t item, uint32_t t) {
      const uint32_t pos = atomicAdd(&s_cur[t], 1u);
      if (ids) ids[pos] = item;  // ordered later by (depth bits, item)
      else spair[pos] = ((uint64_t)depth_bits[item] << 32) | item;  // the sort key (depth bits, item)
    });
}


// Sorts the n <= 64 E keys at pa[start ..) and writes them either as item ids
// (+ 64-bit tile keys) to vals / keys, or (TO_VALS = false) back to pa.
template <int E, bool TO_VALS>
__device__ __forceinline__ void tile_sort_regs(uint64_t* __restrict__ pa, uint32_t start, uint32_t n,
                                               uint32_t tile, uint32_t* __restrict__ vals,
                                               uint64_t* __restrict__ keys) {
  const int lane = __lane_id();
  uint64_t x[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const uint32_t i = (uint32_t)(lane * E + r);
    x[r] = i < n ? pa[start + i] : ~0ull;
  }
  wave_bitonic<E>(x);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const uint32_t i = (uint32_t)(lane * E + r);
    if (i < n) {
      if (TO_VALS) {
        vals[start + i] = (uint32_t)x[r];
        if (keys) keys[start + i] = ((uint64_t)tile << 32) | (x[r] >> 32);
      } else {
        pa[start + i] = x[r];
      }
    }
  }
}

// Global-memory writes of one wavefront made visible to its own later reads
// from other lanes (a workgroup-scope release and acquire around the point
// where the lanes trade data).
__device__ __forceinline__ void wave_memory_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Sorts the long segment pa[start, start + n) (n > kSegCap) of tile `tile` as
// register-sorted runs of kSegCap merged pairwise through the ping-pong
// buffer pb, by one wavefront, and writes the item ids to vals (and the
// 64-bit keys when asked for).
__device__ void sort_long_segment(uint64_t* __restrict__ pa, uint64_t* __restrict__ pb, uint32_t start, uint32_t n,
                                  uint32_t tile, uint32_t* __restrict__ vals, uint64_t* __restrict__ keys) {
  for (uint32_t r0 = 0; r0 < n; r0 += kSegCap)
    tile_sort_regs<16, false>(pa, start + r0, min((uint32_t)kSegCap, n - r0), tile, vals, keys);
  wave_memory_sync();
  uint64_t *src = pa, *dst = pb;
  for (uint32_t width = kSegCap; width < n; width <<= 1) {
    for (uint32_t lo = 0; lo < n; lo += 2 * width) {
      const uint32_t na = min(width, n - lo);
      const uint32_t nb = n - lo > width ? min(width, n - lo - width) : 0u;
      merge_runs<false>(src, start + lo, na, start + lo + na, nb, dst, nullptr, start + lo, 0u,
                        (uint32_t)__lane_id(), 64u);
    }
    wave_memory_sync();
    uint64_t* tmp = src; src = dst; dst = tmp;
  }
  for (uint32_t i = __lane_id(); i < n; i += 64) {
    const uint64_t x = src[start + i];
    vals[start + i] = (uint32_t)x;
    if (keys) keys[start + i] = ((uint64_t)tile << 32) | (x >> 32);
  }
}

// One wavefront per tile, kSortWaves tiles per workgroup (independent
// wavefronts, no barrier), tiles in the blend's dispatch order (longest
// first): sorts the tile's segment of (depth bits, item) keys and writes the
// item ids to vals (and the 64-bit keys when asked for).  Segments of up to
// kSegCap pairs are sorted in registers, longer ones by sort_long_segment.
constexpr int kSortWaves = 4;
__global__ __launch_bounds__(64 * kSortWaves) void k_tc_sort(const uint32_t* __restrict__ ranges, int ntiles,
                                                            const uint32_t* __restrict__ counters,
                                                            uint64_t* __restrict__ pa, uint64_t* __restrict__ pb,
                                                            uint32_t* __restrict__ vals,
                                                            uint64_t* __restrict__ keys) {
  const int slot = (int)blockIdx.x * kSortWaves + (int)(threadIdx.x >> 6);
  if (slot >= ntiles) return;
  // the order is written whether or not the pairs overflowed: read it
  // alongside the overflow flag
  const int tile = (int)ranges[2 * (size_t)ntiles + slot];
  if (counters[C_OVERFLOW]) return;
  const uint32_t start = ranges[2 * (size_t)tile], end = ranges[2 * (size_t)tile + 1];
  const uint32_t n = end - start;
  if (n == 0) return;
  static_assert(kSegCap == 1024, "register sort sizes");
  if (n <= 64) return tile_sort_regs<1, true>(pa, start, n, tile, vals, keys);
  if (n <= 128) return tile_sort_regs<2, true>(pa, start, n, tile, vals, keys);
  if (n <= 256) return tile_sort_regs<4, true>(pa, start, n, tile, vals, keys);
  if (n <= 512) return tile_sort_regs<8, true>(pa, start, n, tile, vals, keys);
  if (n <= 1024) return tile_sort_regs<16, true>(pa, start, n, tile, vals, keys);
  sort_long_segment(pa, pb, start, n, tile, vals, keys);
}

// Without keys the scatter writes item ids straight into vals and the blend
// orders every list of up to kBlendSortCap pairs itself; this kernel orders
// the longer ones, listed by the tile scan (counters[C_LONG_TILES] of them in
// `long_tiles`): each wavefront takes listed tiles in turn, builds the keys
// (depth bits, item) in pa, sorts them and writes the ids back, then clears
// the tile's unsorted bit.  A small fixed grid: with no long tile every
// wavefront reads the count and ends.
constexpr int kLongSortBlocks = 64;
__global__ __launch_bounds__(64 * kSortWaves) void k_tc_sort_long(uint32_t* __restrict__ ranges,
                                                                 const uint32_t* __restrict__ long_tiles,
                                                                 const uint32_t* __restrict__ counters,
                                                                 const uint32_t* __restrict__ depth_bits,
                                                                 uint64_t* __restrict__ pa,
                                                                 uint64_t* __restrict__ pb,
                                                                 uint32_t* __restrict__ vals) {
  if (counters[C_OVERFLOW]) return;
  const uint32_t count = counters[C_LONG_TILES];
  const uint32_t waves = gridDim.x * kSortWaves;
  for (uint32_t li = blockIdx.x * kSortWaves + (threadIdx.x >> 6); li < count; li += waves) {
    const uint32_t tile = long_tiles[li];
    const uint32_t start = ranges[2 * (size_t)tile], end = ranges[2 * (size_t)tile + 1] & ~kUnsortedBit;
    const uint32_t n = end - start;
    for (uint32_t i = __lane_id(); i < n; i += 64) {
      const uint32_t id = vals[start + i];
      pa[start + i] = ((uint64_t)depth_bits[id] << 32) | id;
    }
    wave_memory_sync();
    if (n <= kSegCap) tile_sort_regs<16, true>(pa, start, n, tile, vals, nullptr);
    else sort_long_segment(pa, pb, start, n, tile, vals, nullptr);
    if (__lane_id() == 0) ranges[2 * (size_t)tile + 1] = end;
  }
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
  const int64_t parts_exp = (items + kPart - 1) / kPart;
  size_t off = 0;
  // --- head: cleared at the start of every call
  p.off_counters = off; off += C_COUNT * 4;
  p.off_tcount = off; off += (size_t)total_tiles * 4;  // tile totals
  p.off_hist = off; off += (size_t)(kDepthPasses + kMaxTilePasses) * kRadix * 4;
  p.off_look_scan = off; off += (size_t)(parts_exp + 1) * 4;
  off = align_up(off);
  p.off_dkeys_a = off; off = align_up(off + (size_t)items * 4);
  // --- body
  p.off_dkeys_b = off; off = align_up(off + (size_t)items * 4);
  p.off_dvals_a = off; off = align_up(off + (size_t)items * 4);
  p.off_dvals_b = off; off = align_up(off + (size_t)items * 4);
  p.off_offsets = off; off = align_up(off + (size_t)items * 4);
  p.off_chunks = off; off = align_up(off + (size_t)((capacity + kEmitChunk - 1) / kEmitChunk + 1) * 4);
  p.off_tkeys_a = off; off = align_up(off + (size_t)capacity * 4);
  p.off_tkeys_b = off; off = align_up(off + (size_t)capacity * 4);
  p.off_pvals_b = off; off = align_up(off + (size_t)capacity * 4);
  p.off_tcursor = off; off = align_up(off + (size_t)total_tiles * 4);
  p.off_rs_hist = off; off = align_up(off + (size_t)kRadix * kRsBlocks * 4);
  const bool tc = total_tiles <= kTcMaxTiles;
  p.off_tcmat = off; off = align_up(off + (tc ? (size_t)kTcBlocks * total_tiles * 4 : 0));
  p.off_tcpair_a = off; off = align_up(off + (tc ? (size_t)capacity * 8 : 0));
  p.off_tcpair_b = off; off = align_up(off + (tc ? (size_t)capacity * 8 : 0));
  p.bytes = off;
  return p;
}

// One reduce-then-scan pass: the RB-bit digit at `shift` of the *d_count
// keys (with their values) from kin / vin to kout / vout; ghist (zeroed)
// receives the pass's digit histogram.
template <int RB>
static hipError_t rs_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                          const uint32_t* d_count, int shift, uint32_t* bhist, uint32_t* ghist, unsigned grid,
                          const uint32_t* ov, hipStream_t s) {
  hipLaunchKernelGGL((k_rs_upsweep<RB>), dim3(grid), dim3(kRsUpThreads), 0, s, kin, d_count, shift, bhist, ghist, ov);
  hipLaunchKernelGGL((k_rs_scan<RB>), dim3(1u << RB), dim3(kSortThreads), 0, s, bhist, (int)grid, ghist, ov);
  hipLaunchKernelGGL((k_rs_downsweep<RB>), dim3(grid), dim3(kSortThreads), 0, s, kin, vin, kout, vout, d_count, shift,
                     bhist, ov);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const gabsplat_geom& g, const BinSortPlan& p, void* ws, uint64_t* keys, uint32_t* vals,
                           uint32_t* ranges, int64_t* d_num_pairs, int32_t* d_overflow, hipStream_t s) {
  char* w = static_cast<char*>(ws);
  uint32_t* counters = reinterpret_cast<uint32_t*>(w + p.off_counters);
  uint32_t* hist = reinterpret_cast<uint32_t*>(w + p.off_hist);
  uint32_t* look_expand = reinterpret_cast<uint32_t*>(w + p.off_look_scan);
  uint32_t* dk[2] = {reinterpret_cast<uint32_t*>(w + p.off_dkeys_a), reinterpret_cast<uint32_t*>(w + p.off_dkeys_b)};
  uint32_t* dv[2] = {reinterpret_cast<uint32_t*>(w + p.off_dvals_a), reinterpret_cast<uint32_t*>(w + p.off_dvals_b)};
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
  const uint32_t* ov = counters + C_OVERFLOW;

  if (p.total_tiles <= kTcMaxTiles) {
    uint32_t* tot = reinterpret_cast<uint32_t*>(w + p.off_tcount);
    uint32_t* tstart = reinterpret_cast<uint32_t*>(w + p.off_tcursor);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(w + p.off_tcmat);
    uint64_t* pa = reinterpret_cast<uint64_t*>(w + p.off_tcpair_a);
    uint64_t* pb = reinterpret_cast<uint64_t*>(w + p.off_tcpair_b);
    const int nt = p.total_tiles;
    // no counter clear: the tile scan writes the only counters this path reads.
    // Without keys (and with pair positions below the unsorted bit) the
    // lists are left for the blend to order.
    const int direct = (keys == nullptr && p.capacity < (int64_t)kUnsortedBit) ? 1 : 0;
    if (nt > 0) {
      hipLaunchKernelGGL(k_tc_hist, dim3(kTcBlocks), dim3(kTcThreads), 0, s, g.views, p.items, g.tiles, g.rect, nt, cnt);
      hipLaunchKernelGGL(k_tc_colscan, dim3((unsigned)((nt + kColTiles - 1) / kColTiles)), dim3(256), 0, s, cnt, nt,
                         tot);
    }
    hipLaunchKernelGGL(k_tc_tilescan, dim3(1), dim3(kTileScanThreads), 0, s, tot, nt, (uint32_t)p.capacity, direct,
                       tstart, ranges, counters, d_num_pairs, d_overflow);
    if (nt > 0) {
      hipLaunchKernelGGL(k_tc_scatter, dim3(kTcBlocks), dim3(kTcThreads), 0, s, g.views, p.items, g.tiles, g.rect,
                         depth_bits, nt, cnt, tstart, counters, pa, direct ? vals : nullptr);
      if (direct)
        hipLaunchKernelGGL(k_tc_sort_long, dim3(kLongSortBlocks), dim3(64 * kSortWaves), 0, s, ranges, tot, counters,
                           depth_bits, pa, pb, vals);
      else
        hipLaunchKernelGGL(k_tc_sort, dim3((unsigned)((nt + kSortWaves - 1) / kSortWaves)), dim3(64 * kSortWaves), 0,
                           s, ranges, nt, counters, pa, pb, vals, keys);
    }
    return hipGetLastError();
  }

  {
    const size_t nh = (p.off_dkeys_a - p.off_counters) / 4, nr = (size_t)p.total_tiles * 2;
    size_t blocks = (nh + nr + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill2_u32, dim3((unsigned)blocks), dim3(256), 0, s, counters, nh, ranges, nr);
  }
  const unsigned parts_i = (unsigned)(p.parts_items > 0 ? p.parts_items : 1);
  const unsigned parts_p = (unsigned)(p.parts_pairs > 0 ? p.parts_pairs : 1);
  // grids of the ticket / stride loops: bounded, independent of the capacity
  const unsigned grid_i = parts_i < kLoopBlocks ? parts_i : kLoopBlocks;
  const int64_t pe = (p.capacity + kEmitChunk - 1) / kEmitChunk;
  const unsigned parts_e = (unsigned)(pe > 0 ? pe : 1);
  const unsigned grid_e = parts_e < kLoopBlocks ? parts_e : kLoopBlocks;  // two 54 KB-LDS blocks per CU
  uint32_t* offsets = reinterpret_cast<uint32_t*>(w + p.off_offsets);
  uint32_t* chunk_first = reinterpret_cast<uint32_t*>(w + p.off_chunks);

  uint32_t* bhist = reinterpret_cast<uint32_t*>(w + p.off_rs_hist);
  // K2a: compaction of the visible items (depth keys, item ids, V); the block
  // counts live in bhist until the depth passes take it over
  const unsigned grid_c = parts_i < (unsigned)kRsBlocks ? parts_i : (unsigned)kRsBlocks;
  if (p.items > 0) {
    hipLaunchKernelGGL(k_cs_count, dim3(grid_c), dim3(kSortThreads), 0, s, (uint64_t)p.items, g.tiles, bhist);
    hipLaunchKernelGGL(k_cs_scan, dim3(1), dim3(kSortThreads), 0, s, bhist, (int)grid_c, counters);
    hipLaunchKernelGGL(k_cs_write, dim3(grid_c), dim3(kSortThreads), 0, s, (uint64_t)p.items, g.tiles, depth_bits,
                       bhist, dk[0], dv[0]);
  }
  // K4a: depth passes over the V visible items (even count: result in dk[0], dv[0])
  const unsigned grid_d = parts_i < (unsigned)kRsBlocks ? parts_i : (unsigned)kRsBlocks;
  for (int ps = 0; ps < kDepthPasses; ++ps) {
    const int a = ps & 1;
    const hipError_t e = rs_pass<8>(dk[a], dv[a], dk[a ^ 1], dv[a ^ 1], counters + C_NUM_VISIBLE, 8 * ps, bhist,
                                    hist + ps * kRadix, grid_d, nullptr, s);
    if (e != hipSuccess) return e;
  }
  // K2b: tiles-touched scan in depth order, P, overflow
  uint32_t* thist = hist + kDepthPasses * kRadix;
  hipLaunchKernelGGL(k_expand_scan, dim3(grid_i), dim3(kSortThreads), 0, s, g.tiles, dv[0], (uint32_t)p.capacity,
                     counters, look_expand, offsets, chunk_first, parts_e, d_num_pairs, d_overflow);
  // K3: load-balanced pair emission in depth order
  hipLaunchKernelGGL(k_emit, dim3(grid_e), dim3(kSortThreads), 0, s, g.views, g.rect, dv[0], offsets, chunk_first,
                     counters, tk[0], pv[0]);
  // K4b: tile passes over the P pairs (reduce-then-scan), tpass passes of rb
  // bits each: the fewest passes, then the narrowest digits (fewer, longer
  // output runs per digit)
  const unsigned grid_rs = parts_p < (unsigned)kRsBlocks ? parts_p : (unsigned)kRsBlocks;
  int rb = (p.tile_bits + tpass - 1) / tpass;
  if (rb < 4) rb = 4;
  for (int ps = 0; ps < tpass; ++ps) {
    const int a = ps & 1;
    hipError_t e;
    switch (rb) {
      case 4: e = rs_pass<4>(tk[a], pv[a], tk[a ^ 1], pv[a ^ 1], counters + C_NUM_PAIRS, 4 * ps, bhist,
                                  thist + ps * kRadix, grid_rs, ov, s); break;
      case 5: e = rs_pass<5>(tk[a], pv[a], tk[a ^ 1], pv[a ^ 1], counters + C_NUM_PAIRS, 5 * ps, bhist,
                                  thist + ps * kRadix, grid_rs, ov, s); break;
      case 6: e = rs_pass<6>(tk[a], pv[a], tk[a ^ 1], pv[a ^ 1], counters + C_NUM_PAIRS, 6 * ps, bhist,
                                  thist + ps * kRadix, grid_rs, ov, s); break;
      case 7: e = rs_pass<7>(tk[a], pv[a], tk[a ^ 1], pv[a ^ 1], counters + C_NUM_PAIRS, 7 * ps, bhist,
                                  thist + ps * kRadix, grid_rs, ov, s); break;
      default: e = rs_pass<8>(tk[a], pv[a], tk[a ^ 1], pv[a ^ 1], counters + C_NUM_PAIRS, 8 * ps, bhist,
                              thist + ps * kRadix, grid_rs, ov, s); break;
    }
    if (e != hipSuccess) return e;
  }
  uint32_t* tk_final = tk[tpass & 1];
  // K5: ranges
  const int64_t pb = (p.capacity + 255) / 256;
  const unsigned pblocks = (unsigned)(pb < 1 ? 1 : (pb > 2048 ? 2048 : pb));
  const int64_t rbk = (p.capacity + 256 * kRangeKeys - 1) / (256 * kRangeKeys);
  const unsigned rblocks = (unsigned)(rbk < 1 ? 1 : (rbk > 65536 ? 65536 : rbk));
  hipLaunchKernelGGL(k_ranges, dim3(rblocks), dim3(256), 0, s, tk_final, counters, ranges);
  if (p.total_tiles > 0)
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, s, ranges, p.total_tiles, counters,
                       ranges + 2 * (size_t)p.total_tiles);
  if (keys)
    hipLaunchKernelGGL(k_keys64, dim3(pblocks), dim3(256), 0, s, tk_final, vals, depth_bits, counters, keys);
  return hipGetLastError();
}

}  // namespace gs
