// K6 (front-to-back Gabor alpha blending) and K7 (its backward).
//
// One 256-lane workgroup per 16x16 tile; wave w covers the 8x8 quadrant
// (w & 1, w >> 1) of the tile so that a wave's pixels are spatially compact.
// Batches of render records are staged in LDS (one record per lane) and
// every lane walks them in order.  Workgroup b renders the tile the binning
// put at position b of its dispatch order (longest tile lists first), so that
// the GPU never ends with a few long tiles running on an otherwise idle chip.
//
// The forward and the backward evaluate alpha with the same sequence of
// operations and only explicit fused multiply-adds (the library is built
// without FP contraction), so the backward takes exactly the forward's skip
// decisions; it recovers T_i = T_{i+1} / (1 - alpha_i) up to rounding.
#include <hip/hip_runtime.h>

#include "gs_internal.h"
#include "gs_sort.h"

namespace gs {

// records staged in LDS per batch (<= kBlock): the forward's smaller batch
// lowers its LDS use so that more wavefronts fit on a CU (measured faster);
// the backward is not LDS-limited in the same way
constexpr int kBatchFwd = 192;
constexpr int kBatchBwd = 256;

__device__ __forceinline__ int find_view_by_tile(const ViewEntry* views, int nv, int tile) {
  int lo = 0, hi = nv - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (views[mid].tile_offset <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// cos(2 pi x) of any x; the hardware unit takes revolutions
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(x)); }
// 2^x on the hardware unit.  Every result that is used has x >= log2(1/255);
// lanes with smaller x (whose results are discarded) get 0 or a denormal.
__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }

// Bit q (q = 0..3, quadrant (q & 1, q >> 1) of 8x8 pixels of the tile whose
// top-left pixel is (ox, oy)) is set when the record's support o G >= 1/255
// can reach a pixel centre of that quadrant.  With Q(d) = -(a dx^2 + b dx dy +
// c dy^2) (positive definite) the support is {Q(d) <= R}, R = log2 o -
// log2(1/255); the quadrant is reached iff the minimum of Q over its rectangle
// of pixel centres is <= R.  A convex quadratic attains that minimum at the
// origin when the origin is inside, else on an edge, where it is the clamped
// one-dimensional minimiser.  A small relative margin keeps the per-pixel test
// the only decision.
__device__ __forceinline__ float edge_min_x(float a, float b, float c, float X, float y0, float y1) {
  const float y = fminf(fmaxf(-b * X / (2.0f * c), y0), y1);
  return fmaf(fmaf(a, X, b * y), X, c * y * y);
}
__device__ __forceinline__ float edge_min_y(float a, float b, float c, float Y, float x0, float x1) {
  const float x = fminf(fmaxf(-b * Y / (2.0f * a), x0), x1);
  return fmaf(fmaf(a, x, b * Y), x, c * Y * Y);
}

__device__ __forceinline__ uint32_t quadrant_mask(float4 r0, float4 r1, float ox, float oy) {
  const float a = -r0.z, b = -r0.w, c = -r1.x;
  const float R = r1.y - kLog2AlphaMin;
  if (!(R > 0.f) || !(a > 0.f) || !(c > 0.f)) return 0u;
  const float lim = R * 1.002f + 1e-4f;
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float x0 = ox + 8.0f * (q & 1) + 0.5f - r0.x, x1 = x0 + 7.0f;
    const float y0 = oy + 8.0f * (q >> 1) + 0.5f - r0.y, y1 = y0 + 7.0f;
    float mn;
    if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) {
      mn = 0.f;
    } else {
      mn = fminf(fminf(edge_min_x(a, b, c, x0, y0, y1), edge_min_x(a, b, c, x1, y0, y1)),
                 fminf(edge_min_y(a, b, c, y0, x0, x1), edge_min_y(a, b, c, y1, x0, x1)));
    }
    m |= (mn <= lim) ? (1u << q) : 0u;
  }
  return m;
}

// A record as staged in LDS for one tile, relative to the tile origin (ox, oy):
// m = (mu_x - ox, mu_y - oy) is the mean in the tile's frame, and a pixel with
// in-tile centre (u, v) = (px - ox + 0.5, py - oy + 0.5) sits at the offset
// d = (u, v) - m from it.  The envelope exponent q(d) + log2 o is evaluated as
// dx (A dx + B dy) + C dy^2 + log2 o at the offset itself: expanded around the
// tile origin instead, the constant term A |m|^2 of a sharp footprint centred
// far from the origin cancels against the pixel terms and leaves errors of
// ~1e-5 of the result.
//
// The phase f_k . d of component k (cycles) is evaluated as
// f_k . (p - c) + phi_k, with p - c = (u - 8, v - 8) the pixel centre's offset
// from the tile centre (at most 7.5 per axis) and phi_k = f_k . (c - m)
// reduced to [-1/2, 1/2]: equal to f_k . d up to a whole number of cycles,
// and to the same rounding (phi_k carries the large part, rounded once).  The
// hardware cosine and sine take revolutions and reduce them exactly, so these
// small phases need no fract() per pixel; a record whose
// 7.5 (|fx| + |fy|) + 1/2 could leave kPhaseRaw ("wide") has its phases
// reduced per pixel all the same.  Floats (3 + K float4s):
//   [A B C log2o] [m_x m_y 0 0] [r g b w0] then per component [fx fy w' phi].
template <int K>
struct Staged {
  static constexpr int S4 = 3 + K;
};

constexpr float kTileHalf = 0.5f * kTile;
constexpr float kPhaseRaw = 250.0f;
// bit of the staged quadrant mask that flags a wide record
constexpr uint32_t kWideBit = 16u;

// Stages record q for the tile at (ox, oy) into dst; returns whether it is wide.
template <int K>
__device__ __forceinline__ bool stage_record(const float4* q, float ox, float oy, float4* dst) {
  // record fields (gabsplat_geom.rec): mu 0-1, conic terms 2-4, log2 o 5,
  // rgb 6-8, w0 9, component k at 10 + 3k (fx, fy, w'), then the residuals
  // of the mean's float32 rounding
  constexpr int R4 = record_stride(K) / 4;
  float f[4 * R4];
#pragma unroll
  for (int j = 0; j < R4; ++j) {
    f[4 * j] = q[j].x; f[4 * j + 1] = q[j].y; f[4 * j + 2] = q[j].z; f[4 * j + 3] = q[j].w;
  }
  // tile-relative mean: f[0] - ox is exact whenever the offset is no larger
  // in magnitude than f[0] (both are multiples of the ulp of f[0]), so the
  // residual restores the precision the absolute coordinate could not hold;
  // a larger offset (a wide footprint centred far from the tile) is rounded
  // at its own ulp
  const float mx = (f[0] - ox) + f[record_mean_lo(K)], my = (f[1] - oy) + f[record_mean_lo(K) + 1];
  dst[0] = make_float4(f[2], f[3], f[4], f[5]);
  dst[1] = make_float4(mx, my, 0.f, 0.f);
  dst[2] = make_float4(f[6], f[7], f[8], f[9]);
  bool wide = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float fx = f[10 + 3 * k], fy = f[11 + 3 * k];
    const float c = fmaf(fx, kTileHalf - mx, fy * (kTileHalf - my));
    wide = wide || !(fmaf(kTileHalf - 0.5f, fabsf(fx) + fabsf(fy), 0.5f) <= kPhaseRaw);
    dst[3 + k] = make_float4(fx, fy, f[12 + 3 * k], c - rintf(c));
  }
  return wide;
}

// Envelope exponent q(d) + log2 o of a staged record at the offset d = (dx, dy)
// of a pixel centre from its mean (the forward and the backward evaluate it
// with these operations in this order, so their alphas agree bit for bit).
__device__ __forceinline__ float staged_power(float4 s0, float dx, float dy) {
  return fmaf(dx, fmaf(s0.x, dx, s0.y * dy), fmaf(s0.z * dy, dy, s0.w));
}

// Phase (cycles, up to whole cycles) of a staged component (fx, fy, w', phi)
// at the pixel whose centre is (pu, pv) from the tile centre.
__device__ __forceinline__ float staged_phase(float4 c, float pu, float pv) { return fmaf(c.x, pu, fmaf(c.y, pv, c.w)); }

// ------------------------------------------------- list order in the blend
// A tile list the bin sort left unsorted (kUnsortedBit on its end) is put in
// depth order by the tile's own workgroup before blending: the ids
// vals[start, start + n), 2 <= n <= kBlendSortCap, are sorted in place by the
// unique key (depth bits << 32 | id).  Up to 256 ids: the first wavefront
// sorts them in registers.  More: each wavefront sorts a quarter (64 E keys,
// E = 2 or 4) in registers and two rounds of merge-path merges in LDS (2
// kBlendSortCap keys in `lds`) join the quarters.  Called by the whole
// workgroup; ends with a barrier, after which the sorted ids are visible to
// every wavefront of it.
template <int E>
__device__ __forceinline__ void load_list_keys(const uint32_t* vals, const uint32_t* depth_bits, uint32_t start,
                                               uint32_t base, uint32_t n, uint64_t (&x)[E]) {
  const int lane = __lane_id();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const uint32_t i = base + (uint32_t)(lane * E + r);
    uint64_t key = ~0ull;
    if (i < n) {
      const uint32_t id = vals[start + i];
      key = ((uint64_t)depth_bits[id] << 32) | id;
    }
    x[r] = key;
  }
}

template <int E>
__device__ __forceinline__ void wave_sort_list(uint32_t* vals, const uint32_t* depth_bits, uint32_t start,
                                               uint32_t n) {
  uint64_t x[E];
  load_list_keys<E>(vals, depth_bits, start, 0u, n, x);
  wave_bitonic<E>(x);
  const int lane = __lane_id();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const uint32_t i = (uint32_t)(lane * E + r);
    if (i < n) vals[start + i] = (uint32_t)x[r];
  }
}

template <int E>
__device__ __forceinline__ void block_sort_quarters(uint32_t* vals, const uint32_t* depth_bits, uint32_t start,
                                                    uint32_t n, uint64_t* lds) {
  constexpr uint32_t C = 64 * E;
  static_assert(4 * C <= (uint32_t)kBlendSortCap, "quarters fit the sort buffer");
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  uint64_t x[E];
  load_list_keys<E>(vals, depth_bits, start, (uint32_t)w * C, n, x);
  wave_bitonic<E>(x);
#pragma unroll
  for (int r = 0; r < E; ++r) lds[(uint32_t)w * C + (uint32_t)(lane * E + r)] = x[r];
  __syncthreads();
  // quarters (0, 1) and (2, 3), 128 threads each, into the second half
  uint64_t* b = lds + kBlendSortCap;
  const uint32_t h = (uint32_t)t >> 7;
  merge_runs<false>(lds, 2 * C * h, C, 2 * C * h + C, C, b, nullptr, 2 * C * h, 0u, (uint32_t)t & 127u, 128u);
  __syncthreads();
  merge_runs<true>(b, 0u, 2 * C, 2 * C, 2 * C, nullptr, vals + start, 0u, n, (uint32_t)t, (uint32_t)kBlock);
}

__device__ __forceinline__ void block_sort_list(uint32_t* vals, const uint32_t* depth_bits, uint32_t start,
                                                uint32_t n, uint64_t* lds) {
  static_assert(kBlock == 256 && kBlendSortCap == 1024, "four wavefronts, quarters of up to 256 keys");
  if (n <= 256) {
    if (threadIdx.x < 64) {
      if (n <= 64) wave_sort_list<1>(vals, depth_bits, start, n);
      else if (n <= 128) wave_sort_list<2>(vals, depth_bits, start, n);
      else wave_sort_list<4>(vals, depth_bits, start, n);
    }
  } else if (n <= 512) {
    block_sort_quarters<2>(vals, depth_bits, start, n, lds);
  } else {
    block_sort_quarters<4>(vals, depth_bits, start, n, lds);
  }
  __syncthreads();
}

// --------------------------------------------------------------------- K6
// The ANALYSIS variant (never the timed one) can also report, per pixel, how
// far down its tile list the blend had to go (the stopping position, or the
// list length) and how many of those pairs passed the envelope test (full
// Gabor evaluations) -- the algorithmic work of the blend -- and a frequency
// map: each primitive's weighted image-plane frequency sum_k w_k |f2d_k|
// (cycles per pixel) blended with the same weights alpha_i T_i as its colour.
template <int K, bool ANALYSIS>
__global__ __launch_bounds__(kBlock) void k_render_fwd(const void* __restrict__ table,
                                                       const float* __restrict__ rec,
                                                       const uint32_t* __restrict__ depth_bits,
                                                       uint32_t* __restrict__ vals,
                                                       uint32_t* __restrict__ ranges,
                                                       float* __restrict__ image, float* __restrict__ final_T,
                                                       uint32_t* __restrict__ n_contrib,
                                                       uint32_t* __restrict__ eval_counts,
                                                       float* __restrict__ freq_map,
                                                       const int32_t* __restrict__ d_overflow) {
  constexpr int RF = record_stride(K);
  constexpr int R4 = RF / 4;
  constexpr int S4 = Staged<K>::S4;
  // the staged records; before the first batch, the list sort's keys
  constexpr int kRecF4 = kBatchFwd * S4, kSortF4 = kBlendSortCap;  // 2 u64 keys per float4
  __shared__ float4 s_rec[kRecF4 > kSortF4 ? kRecF4 : kSortF4];
  __shared__ uint32_t s_mask[kBatchFwd];
  if (d_overflow != nullptr && *d_overflow != 0) return;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry* views = table_views(table);
  // longest tile lists first (the order gabsplat_bin_sort writes after the ranges)
  const int tile = (int)ranges[2 * (size_t)gridDim.x + blockIdx.x];
  const ViewEntry& V = views[find_view_by_tile(views, hdr->num_views, tile)];
  const int lt = tile - V.tile_offset;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int px = tx * kTile + (w & 1) * 8 + (l & 7);
  const int py = ty * kTile + (w >> 1) * 8 + (l >> 3);
  const bool inside = px < V.width && py < V.height;
  const float u = (float)((w & 1) * 8 + (l & 7)) + 0.5f, v = (float)((w >> 1) * 8 + (l >> 3)) + 0.5f;
  const float pu = u - kTileHalf, pv = v - kTileHalf;
  const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
  const uint32_t start = ranges[2 * (size_t)tile], end_word = ranges[2 * (size_t)tile + 1];
  const uint32_t end = end_word & ~kUnsortedBit;
  if (end_word & kUnsortedBit) {  // the same for the whole workgroup
    block_sort_list(vals, depth_bits, start, end - start, reinterpret_cast<uint64_t*>(s_rec));
    if (t == 0) ranges[2 * (size_t)tile + 1] = end;
  }

  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t last = 0, stop_pos = end - start, n_full = 0;
  float Fm = 0.f;
  bool done = !inside;
  for (uint32_t b = start; b < end; b += kBatchFwd) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t idx = b + t;
    uint32_t m = 0;
    if (t < kBatchFwd && idx < end) {
      const float4* src = reinterpret_cast<const float4*>(rec + (size_t)vals[idx] * RF);
      float4 q[R4];
#pragma unroll
      for (int j = 0; j < R4; ++j) q[j] = src[j];
      const bool wide = stage_record<K>(q, ox, oy, &s_rec[t * S4]);
      m = quadrant_mask(q[0], q[1], ox, oy) | (wide ? kWideBit : 0u);
    }
    if (t < kBatchFwd) s_mask[t] = m;
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBatchFwd, end - b);
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      // lanes still blending when the chunk starts (a lane that stops inside
      // the chunk only makes the skip test below less strict)
      const uint64_t act = __builtin_amdgcn_ballot_w64(!done);
      if (act == 0ull) break;
      const uint32_t ml = c0 + l < cnt ? s_mask[c0 + l] : 0u;
      uint64_t bits = __ballot((ml >> w) & 1u);
      const uint64_t wide_bits = __ballot((ml & kWideBit) != 0u);
      while (bits) {
        const int jj = __builtin_ctzll(bits);
        const int j = c0 + jj;
        const bool wide = (wide_bits >> jj) & 1ull;
        bits &= bits - 1;
        const float4 s0 = s_rec[j * S4], s1 = s_rec[j * S4 + 1];
        const float dx = u - s1.x, dy = v - s1.y;
        const float pw = staged_power(s0, dx, dy);
        // o G < 1/255 with B <= 1 means alpha < 1/255: no full evaluation
        const bool env = !(pw < kLog2AlphaMin);
        if ((__builtin_amdgcn_ballot_w64(env) & act) == 0ull) continue;
        bool live = !done && env;
        if (ANALYSIS) n_full += live ? 1u : 0u;
        const float4 col = s_rec[j * S4 + 2];
        // straight-line update: lanes that do not take the record keep their state
        const float E = exp2_hw(pw);
        float Bv = col.w;
        if (wide) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float4 c = s_rec[j * S4 + 3 + k];
            Bv = fmaf(c.z, cos_rev(staged_phase(c, pu, pv)), Bv);
          }
        } else {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float4 c = s_rec[j * S4 + 3 + k];
            Bv = fmaf(c.z, __builtin_amdgcn_cosf(staged_phase(c, pu, pv)), Bv);
          }
        }
        const float alpha = fminf(kAlphaMax, E * Bv);
        live = live && !(alpha < kAlphaMin);
        const float Tn = fmaf(-alpha, T, T);  // T (1 - alpha), rounded once
        const bool stop = live && Tn < kTMin;
        const bool take = live && !stop;
        if (ANALYSIS && stop) stop_pos = b - start + (uint32_t)j + 1;
        done = done || stop;
        const float wt = take ? alpha * T : 0.f;
        C0 = fmaf(col.x, wt, C0);
        C1 = fmaf(col.y, wt, C1);
        C2 = fmaf(col.z, wt, C2);
        if (ANALYSIS) {
          float phi = 0.f;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float4 c = s_rec[j * S4 + 3 + k];
            phi = fmaf(c.z, sqrtf(c.x * c.x + c.y * c.y), phi);
          }
          Fm = fmaf(phi, wt, Fm);
        }
        T = take ? Tn : T;
        last = take ? b - start + (uint32_t)j + 1 : last;
      }
    }
  }
  if (inside) {
    const size_t hw = (size_t)V.width * V.height;
    const size_t pix = (size_t)py * V.width + px;
    float* img = image + 3 * (size_t)V.pixel_offset;
    img[pix] = fmaf(T, V.bg[0], C0);
    img[hw + pix] = fmaf(T, V.bg[1], C1);
    img[2 * hw + pix] = fmaf(T, V.bg[2], C2);
    final_T[V.pixel_offset + pix] = T;
    n_contrib[V.pixel_offset + pix] = last;
    if (ANALYSIS && eval_counts) {
      eval_counts[2 * (V.pixel_offset + pix)] = stop_pos;
      eval_counts[2 * (V.pixel_offset + pix) + 1] = n_full;
    }
    if (ANALYSIS && freq_map) freq_map[V.pixel_offset + pix] = Fm;
  }
}

// ------------------------------------------------- wave reduce-scatter-add
// Sums v[0..G) over the 64 lanes of a wavefront by recursive halving: at each
// of six stages a lane holding L partial sums pairs them as (j, j + ceil(L/2))
// and keeps one of each pair (the first on the lower side of the stage's lane
// bit, the second on the upper side), adding the partner lane's partial sum
// of that component; an unpaired last component (L odd) is summed with the
// partner and kept on both sides.  After the stages every lane holds the
// wavefront total of one component (which, and whether the lane is the one
// that writes it, depends only on the lane: halving_slot) and a single vector
// atomic writes all G components.  Partners, stage by stage: lane l ^ 32 and
// l ^ 16 through the lane-swap instructions of gfx950 -- swapping the upper
// 32 (odd 16-lane) lanes of x with the lower 32 (even) lanes of y leaves x's
// pair sums in the lower and y's in the upper lanes of x + y, one add per
// pair -- then the DPP patterns 15 - i within a row of 16, 7 - i within its
// halves, 3 - i and i ^ 1 within quads.  Each stage pairs lanes that differ
// in the stage's bit and agree in the bits above it, and the six partner
// masks 32, 16, 15, 7, 3, 1 together span all six lane bits.  Every lane of
// the wavefront must be active.
constexpr int halving_len(int g, int stage) {
  for (int i = 0; i < stage; ++i) g = (g + 1) / 2;
  return g;
}

// Component held by `lane` after the six stages; *writer is set for exactly
// one lane per component.
template <int G>
__device__ __forceinline__ int halving_slot(int lane, bool* writer) {
  int j = 0;
  bool w = true;
#pragma unroll
  for (int st = 5; st >= 0; --st) {
    const int L = halving_len(G, st), h = (L + 1) / 2;
    const bool upper = (lane >> (5 - st)) & 1;
    if (upper) {
      if (j + h < L) j += h;
      else w = false;  // duplicate of the lower side's component
    }
  }
  *writer = w;
  return j;
}

template <int CTRL>
__device__ __forceinline__ float dpp_get(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

template <int G, int ST, bool SWAP32>
__device__ __forceinline__ void stage_swap(float (&v)[G]) {
  constexpr int L = halving_len(G, ST), h = (L + 1) / 2;
#pragma unroll
  for (int j = 0; j < h; ++j) {
    const uint32_t x = __float_as_uint(v[j]);
    const uint32_t y = (j + h < L) ? __float_as_uint(v[j + h]) : x;
    const auto r = SWAP32 ? __builtin_amdgcn_permlane32_swap(x, y, false, false)
                          : __builtin_amdgcn_permlane16_swap(x, y, false, false);
    v[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

// a where the lane's bit of `upper` is clear, b where it is set.  Written as
// the instruction itself: as a plain ?: the optimizer merges the selects of a
// stage into one run-time index into v[] and lowers that as a compare chain
// over every element.
__device__ __forceinline__ float lane_select(float a, float b, uint64_t upper) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(upper));
  return r;
}

template <int G, int ST, int CTRL>
__device__ __forceinline__ void stage_dpp(float (&v)[G], uint64_t upper) {
  constexpr int L = halving_len(G, ST), h = (L + 1) / 2;
#pragma unroll
  for (int j = 0; j < h; ++j) {
    if (j + h < L) {
      const float keep = lane_select(v[j], v[j + h], upper);
      const float send = lane_select(v[j + h], v[j], upper);
      v[j] = keep + dpp_get<CTRL>(send);
    } else {
      v[j] += dpp_get<CTRL>(v[j]);
    }
  }
}

template <int G>
__device__ __forceinline__ void wave_reduce_add(float (&v)[G], float* dst, int slot, bool writer) {
  static_assert(G >= 1 && G <= 64, "component count");
  stage_swap<G, 0, true>(v);
  stage_swap<G, 1, false>(v);
  // lane masks of the stage bits 3, 2, 1, 0
  stage_dpp<G, 2, 0x140>(v, 0xFF00FF00FF00FF00ull);   // row mirror
  stage_dpp<G, 3, 0x141>(v, 0xF0F0F0F0F0F0F0F0ull);   // half-row mirror
  stage_dpp<G, 4, 0x1B>(v, 0xCCCCCCCCCCCCCCCCull);    // quad (3, 2, 1, 0)
  stage_dpp<G, 5, 0xB1>(v, 0xAAAAAAAAAAAAAAAAull);    // quad (1, 0, 3, 2)
  if (writer) atomicAdd(dst + slot, v[0]);
}

// --------------------------------------------------------------------- K7
// ABS adds two components per pair: |dL_p/d mu2d_x| and |dL_p/d mu2d_y| of the
// pixel, whose wave sums build the homodirectional (AbsGS) statistic.
template <int K, bool ABS>
__global__ __launch_bounds__(kBlock) void k_render_bwd(const void* __restrict__ table,
                                                       const float* __restrict__ rec,
                                                       const uint32_t* __restrict__ vals,
                                                       const uint32_t* __restrict__ ranges,
                                                       const float* __restrict__ final_T,
                                                       const uint32_t* __restrict__ n_contrib,
                                                       const float* __restrict__ dl_dimage,
                                                       float* __restrict__ grad2d,
                                                       const int32_t* __restrict__ d_overflow) {
  constexpr int RF = record_stride(K);
  constexpr int R4 = RF / 4;
  constexpr int S4 = Staged<K>::S4;
  constexpr int GS = 10 + 3 * K + (ABS ? 2 : 0);  // gradient components per pair (record fields [+ 2])
  constexpr int GF = (GS + 3) & ~3;               // grad2d row stride
  __shared__ float4 s_rec[kBatchBwd * S4];
  __shared__ uint32_t s_id[kBatchBwd];
  __shared__ uint32_t s_mask[kBatchBwd];
  __shared__ uint32_t s_max;
  if (d_overflow != nullptr && *d_overflow != 0) return;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry* views = table_views(table);
  // longest tile lists first (the order gabsplat_bin_sort writes after the ranges)
  const int tile = (int)ranges[2 * (size_t)gridDim.x + blockIdx.x];
  const ViewEntry& V = views[find_view_by_tile(views, hdr->num_views, tile)];
  const int lt = tile - V.tile_offset;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int px = tx * kTile + (w & 1) * 8 + (l & 7);
  const int py = ty * kTile + (w >> 1) * 8 + (l >> 3);
  const bool inside = px < V.width && py < V.height;
  const float u = (float)((w & 1) * 8 + (l & 7)) + 0.5f, v = (float)((w >> 1) * 8 + (l >> 3)) + 0.5f;
  const float pu = u - kTileHalf, pv = v - kTileHalf;
  const float ox = (float)(tx * kTile), oy = (float)(ty * kTile);
  const uint32_t start = ranges[2 * (size_t)tile];
  bool red_writer;
  const int red_slot = halving_slot<GS>(l, &red_writer);

  float T = 1.0f, Tf = 1.0f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f;
  uint32_t last = 0;
  if (inside) {
    const size_t hw = (size_t)V.width * V.height;
    const size_t pix = (size_t)py * V.width + px;
    Tf = final_T[V.pixel_offset + pix];
    last = n_contrib[V.pixel_offset + pix];
    const float* g = dl_dimage + 3 * (size_t)V.pixel_offset;
    dC0 = g[pix];
    dC1 = g[hw + pix];
    dC2 = g[2 * hw + pix];
  }
  T = Tf;
  const float Tbg = Tf * (V.bg[0] * dC0 + V.bg[1] * dC1 + V.bg[2] * dC2);
  if (t == 0) s_max = 0;
  __syncthreads();
  if (last) atomicMax(&s_max, last);
  __syncthreads();
  const uint32_t maxlast = s_max;
  // the wave's own furthest contributor (positions beyond it are skipped)
  uint32_t wlast = last;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, d, 64));

  // colour blended from the contributors behind the current record (back to front)
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  for (uint32_t hi = maxlast; hi > 0;) {
    const uint32_t lo = hi > (uint32_t)kBatchBwd ? hi - kBatchBwd : 0u;
    const uint32_t cnt = hi - lo;
    __syncthreads();
    uint32_t m = 0;
    if ((uint32_t)t < cnt) {
      const uint32_t gid = vals[start + lo + t];
      s_id[t] = gid;
      const float4* src = reinterpret_cast<const float4*>(rec + (size_t)gid * RF);
      float4 q[R4];
#pragma unroll
      for (int j = 0; j < R4; ++j) q[j] = src[j];
      const bool wide = stage_record<K>(q, ox, oy, &s_rec[t * S4]);
      m = quadrant_mask(q[0], q[1], ox, oy) | (wide ? kWideBit : 0u);
    }
    if (t < kBatchBwd) s_mask[t] = m;
    __syncthreads();
    // chunks of 64 records, newest first; records past the wave's last contributor are skipped
    for (int c0 = ((int)cnt - 1) & ~63; c0 >= 0; c0 -= 64) {
      const uint32_t pos_l = lo + (uint32_t)(c0 + l) + 1;
      const uint32_t ml = c0 + l < (int)cnt && pos_l <= wlast ? s_mask[c0 + l] : 0u;
      uint64_t bits = __ballot((ml >> w) & 1u);
      const uint64_t wide_bits = __ballot((ml & kWideBit) != 0u);
      while (bits) {
        const int hb = 63 - __builtin_clzll(bits);
        const bool wide = (wide_bits >> hb) & 1ull;
        bits &= ~(1ull << hb);
        const int j = __builtin_amdgcn_readfirstlane(c0 + hb);  // wave-uniform: scalar addressing
        const uint32_t pos = lo + (uint32_t)j + 1;
        const float4 s0 = s_rec[j * S4], s1 = s_rec[j * S4 + 1];
        const float dx = u - s1.x, dy = v - s1.y;
        const float pw = staged_power(s0, dx, dy);
        bool contrib = pos <= last && !(pw < kLog2AlphaMin);
        const uint64_t cb = __builtin_amdgcn_ballot_w64(contrib);
        if (cb == 0ull) continue;
        const float4 col = s_rec[j * S4 + 2];
        float4 cc[K > 0 ? K : 1];
#pragma unroll
        for (int k = 0; k < K; ++k) cc[k] = s_rec[j * S4 + 3 + k];
        // alpha exactly as the forward evaluates it (same operations, same order)
        const float E = exp2_hw(pw);
        float cs[K > 0 ? K : 1], sn[K > 0 ? K : 1];
        float Bv = col.w;
        if (wide) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float fr = __builtin_amdgcn_fractf(staged_phase(cc[k], pu, pv));
            cs[k] = __builtin_amdgcn_cosf(fr);
            sn[k] = __builtin_amdgcn_sinf(fr);
          }
        } else {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float ph = staged_phase(cc[k], pu, pv);
            cs[k] = __builtin_amdgcn_cosf(ph);
            sn[k] = __builtin_amdgcn_sinf(ph);
          }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) Bv = fmaf(cc[k].z, cs[k], Bv);
        const float EB = E * Bv;
        const float alpha = fminf(kAlphaMax, EB);
        // the ballot of the alpha compare alone, masked in scalar registers
        const bool a_ok = !(alpha < kAlphaMin);
        if ((__builtin_amdgcn_ballot_w64(a_ok) & cb) == 0ull) continue;
        contrib = contrib && a_ok;
        // lanes without a contribution keep their state and produce zero gradients
        const float inv = __builtin_amdgcn_rcpf(1.0f - alpha);
        T = contrib ? T * inv : T;  // T_i = T_(i+1) / (1 - alpha_i)
        const float ac = contrib ? alpha : 0.f;
        const float wt = ac * T;
        const float e0 = col.x - acc0, e1 = col.y - acc1, e2 = col.z - acc2;
        float da = fmaf(e2, dC2, fmaf(e1, dC1, e0 * dC0));
        da = da * T - Tbg * inv;
        da = (contrib && !(EB > kAlphaMax)) ? da : 0.f;  // a binding clamp has zero derivative
        // this record joins the colour behind the next (nearer) one
        acc0 = fmaf(ac, e0, acc0);
        acc1 = fmaf(ac, e1, acc1);
        acc2 = fmaf(ac, e2, acc2);
        const float dB = da * E;
        const float dp = dB * Bv * kLn2;
        float gv[GS];
        gv[5] = dp;
        gv[6] = wt * dC0;
        gv[7] = wt * dC1;
        gv[8] = wt * dC2;
        gv[9] = dB;  // DC weight
        // with (ex, ey) = mean - pixel centre the mean gradient -(dL/d pixel
        // offset) is dp (2A ex + B ey, B ex + 2C ey) - sum_k dph_k f_k, where
        // dph_k = dL/d phase_k; nph = -dph_k
        const float ex = -dx, ey = -dy;
        const float px_ = dp * ex, py_ = dp * ey;
        gv[2] = px_ * ex;
        gv[3] = px_ * ey;
        gv[4] = py_ * ey;
        float g0 = fmaf(s0.x, px_ + px_, s0.y * py_);
        float g1 = fmaf(s0.z, py_ + py_, s0.y * px_);
        const float dB2pi = dB * 6.283185307179586f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float nph = dB2pi * cc[k].z * sn[k];
          gv[10 + 3 * k] = nph * ex;  // = dph_k (u - mean_x)
          gv[11 + 3 * k] = nph * ey;
          gv[12 + 3 * k] = dB * cs[k];
          g0 = fmaf(nph, cc[k].x, g0);
          g1 = fmaf(nph, cc[k].y, g1);
        }
        gv[0] = g0;
        gv[1] = g1;
        if (ABS) {
          gv[GS - 2] = fabsf(g0);
          gv[GS - 1] = fabsf(g1);
        }
        wave_reduce_add<GS>(gv, grad2d + (size_t)s_id[j] * GF, red_slot, red_writer);
      }
    }
    hi = lo;
  }
}

// ------------------------------------------------------ grad2d row clear
// Zeroes the grad2d rows of the items that touch a tile: the only rows the
// backward adds into and the only rows read afterwards.  A wavefront takes 64
// consecutive items, whose rows are one contiguous run of 64 * gf4 float4s,
// and writes the run with consecutive lanes on consecutive float4s, skipping
// the rows of items that touch no tile.
__global__ void k_clear_visible_rows(const uint32_t* __restrict__ tiles, float* __restrict__ grad2d, int64_t items,
                                     int gf4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t vmask = __ballot(i < items ? tiles[i] != 0 : false);
  if (vmask == 0) return;
  const int l = threadIdx.x & 63;
  float4* run = reinterpret_cast<float4*>(grad2d) + (i - l) * gf4;
  // row p = floor(q / gf4) through a float reciprocal: q < 64 * 9 and q + 0.5
  // sits at least 0.5 / gf4 from a multiple of gf4, far beyond the rounding
  const float inv = 1.0f / (float)gf4;
  for (int j = 0; j < gf4; ++j) {
    const int q = j * 64 + l;
    const int p = (int)(((float)q + 0.5f) * inv);
    if ((vmask >> p) & 1ull) run[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

hipError_t launch_clear_grad2d(const uint32_t* tiles, float* grad2d, int64_t items, int gf, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const int64_t blocks = (items + 255) / 256;  // items < 2^32: fewer than 2^24 blocks
  hipLaunchKernelGGL(k_clear_visible_rows, dim3((unsigned)blocks), dim3(256), 0, s, tiles, grad2d, items, gf / 4);
  return hipGetLastError();
}

// --------------------------------------------------------------- launchers
template <int K>
static hipError_t fwd_k(const void* d_table, const HostTable& h, const gabsplat_geom& g, uint32_t* vals,
                        uint32_t* ranges, float* image, float* final_T, uint32_t* n_contrib,
                        uint32_t* eval_counts, float* freq_map, const int32_t* ov, hipStream_t s) {
  if (h.hdr.total_tiles == 0) return hipSuccess;
  const uint32_t* depth_bits = reinterpret_cast<const uint32_t*>(g.depth);
  if (eval_counts || freq_map)
    hipLaunchKernelGGL((k_render_fwd<K, true>), dim3((unsigned)h.hdr.total_tiles), dim3(kBlock), 0, s, d_table, g.rec,
                       depth_bits, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov);
  else
    hipLaunchKernelGGL((k_render_fwd<K, false>), dim3((unsigned)h.hdr.total_tiles), dim3(kBlock), 0, s, d_table,
                       g.rec, depth_bits, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov);
  return hipGetLastError();
}

hipError_t launch_render_fwd(const void* d_table, const HostTable& h, const gabsplat_geom& g, int k,
                             uint32_t* vals, uint32_t* ranges, float* image, float* final_T,
                             uint32_t* n_contrib, uint32_t* eval_counts, float* freq_map, const int32_t* ov,
                             hipStream_t s) {
  switch (k) {
    case 0: return fwd_k<0>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 1: return fwd_k<1>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 2: return fwd_k<2>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 3: return fwd_k<3>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 4: return fwd_k<4>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 5: return fwd_k<5>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 6: return fwd_k<6>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 7: return fwd_k<7>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
    case 8: return fwd_k<8>(d_table, h, g, vals, ranges, image, final_T, n_contrib, eval_counts, freq_map, ov, s);
  }
  return hipErrorInvalidValue;
}

template <int K>
static hipError_t bwd_k(const void* d_table, const HostTable& h, const gabsplat_geom& g, const uint32_t* vals,
                        const uint32_t* ranges, const float* final_T, const uint32_t* n_contrib,
                        const float* dl, float* grad2d, bool abs_mean2d, const int32_t* ov, hipStream_t s) {
  if (h.hdr.total_tiles == 0) return hipSuccess;
  if (abs_mean2d)
    hipLaunchKernelGGL((k_render_bwd<K, true>), dim3((unsigned)h.hdr.total_tiles), dim3(kBlock), 0, s, d_table,
                       g.rec, vals, ranges, final_T, n_contrib, dl, grad2d, ov);
  else
    hipLaunchKernelGGL((k_render_bwd<K, false>), dim3((unsigned)h.hdr.total_tiles), dim3(kBlock), 0, s, d_table,
                       g.rec, vals, ranges, final_T, n_contrib, dl, grad2d, ov);
  return hipGetLastError();
}

hipError_t launch_render_bwd(const void* d_table, const HostTable& h, const gabsplat_geom& g, int k,
                             const uint32_t* vals, const uint32_t* ranges, const float* final_T,
                             const uint32_t* n_contrib, const float* dl, float* grad2d, bool abs_mean2d,
                             const int32_t* ov, hipStream_t s) {
  switch (k) {
    case 0: return bwd_k<0>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 1: return bwd_k<1>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 2: return bwd_k<2>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 3: return bwd_k<3>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 4: return bwd_k<4>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 5: return bwd_k<5>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 6: return bwd_k<6>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 7: return bwd_k<7>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
    case 8: return bwd_k<8>(d_table, h, g, vals, ranges, final_T, n_contrib, dl, grad2d, abs_mean2d, ov, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gs
