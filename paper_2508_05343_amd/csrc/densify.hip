// Frequency-adaptive density control (Sec. 3.4.2): view-space gradient
// statistics, clone / split / prune with the frequencies and frequency weights
// of every new child reset to small values, and the periodic reset of all
// frequency weights together with the opacity reset.  With the AbsGS variant
// (the densification the paper combines with its primitive, Sec. 4.1) a second
// statistic, the norm of the per-axis sums of absolute per-pixel mean
// gradients, can also trigger splits.
//
// Densification keeps a stable output order (kept primitives, then clone
// copies, then split children, each by ascending source index) with three
// launches: per-block category counts, one block scanning the block counts,
// and a write pass that recomputes the same decisions.
#include <hip/hip_runtime.h>

#include "gs_block.h"
#include "gs_internal.h"

namespace gs {

constexpr int kDenItems = 4;
constexpr int kDenBlock = 256 * kDenItems;

// --------------------------------------------------------------- statistics
// accum[i] += |dL/d mu2d| in normalised device coordinates (pixel gradient
// times (W/2, H/2)), denom[i] += 1, for every view in which i is visible; with
// abs_col >= 0 also accum_abs[i] += the norm of grad2d columns abs_col and
// abs_col + 1 (the per-axis absolute sums) in the same units.
__global__ __launch_bounds__(256) void k_densify_stats(const void* __restrict__ table, int64_t n,
                                                       const uint32_t* __restrict__ tiles,
                                                       const float* __restrict__ grad2d, int gf, int abs_col,
                                                       float* __restrict__ accum, float* __restrict__ accum_abs,
                                                       float* __restrict__ denom) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry* views = table_views(table);
  float a = 0.f, aa = 0.f, d = 0.f;
  for (int v = 0; v < hdr->num_views; ++v) {
    const int64_t item = views[v].item_offset + i;
    if (tiles[item] == 0) continue;
    const float hw = 0.5f * (float)views[v].width, hh = 0.5f * (float)views[v].height;
    const float gx = grad2d[item * gf] * hw;
    const float gy = grad2d[item * gf + 1] * hh;
    a += sqrtf(gx * gx + gy * gy);
    if (abs_col >= 0) {
      const float ax = grad2d[item * gf + abs_col] * hw;
      const float ay = grad2d[item * gf + abs_col + 1] * hh;
      aa += sqrtf(ax * ax + ay * ay);
    }
    d += 1.f;
  }
  accum[i] += a;
  if (abs_col >= 0) accum_abs[i] += aa;
  denom[i] += d;
}

// ----------------------------------------------------------------- decisions
enum { KIND_KEEP = 0, KIND_CLONE = 1, KIND_SPLIT = 2, KIND_PRUNE = 3 };

__device__ __forceinline__ int densify_kind(const gabsplat_scene& in, const float* accum, const float* denom,
                                            const float* accum_abs, const gabsplat_densify_params& p, int64_t i) {
  const int64_t n = in.n;
  const float dn = denom[i];
  const float avg = dn > 0.f ? accum[i] / dn : 0.f;
  const float smax = fmaxf(fmaxf(in.scales[i], in.scales[n + i]), in.scales[2 * n + i]);
  const float o = in.opacities[i];
  bool prune = o < p.min_opacity;
  if (p.prune_big) prune = prune || smax > p.max_world_frac * p.scene_extent;
  if (prune) return KIND_PRUNE;
  const bool big = smax > p.percent_dense * p.scene_extent;
  bool sel = avg >= p.grad_threshold;
  if (big && !sel && p.abs_grad_threshold > 0.f) sel = (dn > 0.f ? accum_abs[i] / dn : 0.f) >= p.abs_grad_threshold;
  if (sel) return big ? KIND_SPLIT : KIND_CLONE;
  return KIND_KEEP;
}

// counts[b][3]: kept (keep + clone), clone, split of block b
__global__ __launch_bounds__(256) void k_densify_count(gabsplat_scene in, const float* __restrict__ accum,
                                                       const float* __restrict__ denom,
                                                       const float* __restrict__ accum_abs, gabsplat_densify_params p,
                                                       uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_c[3];
  if (threadIdx.x < 3) s_c[threadIdx.x] = 0;
  __syncthreads();
  uint32_t kept = 0, clone = 0, split = 0;
#pragma unroll
  for (int j = 0; j < kDenItems; ++j) {
    const int64_t i = (int64_t)blockIdx.x * kDenBlock + j * 256 + threadIdx.x;
    if (i >= in.n) continue;
    const int k = densify_kind(in, accum, denom, accum_abs, p, i);
    kept += (k == KIND_KEEP || k == KIND_CLONE);
    clone += (k == KIND_CLONE);
    split += (k == KIND_SPLIT);
  }
  atomicAdd(&s_c[0], kept);
  atomicAdd(&s_c[1], clone);
  atomicAdd(&s_c[2], split);
  __syncthreads();
  if (threadIdx.x < 3) counts[3 * (size_t)blockIdx.x + threadIdx.x] = s_c[threadIdx.x];
}

// One block: exclusive scan of each category over the blocks (in place), the
// totals, the output count and the overflow flag.  totals[0..2] = category
// totals, totals[3] = output count, totals[4] = overflow.
__global__ __launch_bounds__(256) void k_densify_scan(uint32_t* __restrict__ counts, int nblocks, int split_count,
                                                      int64_t capacity, uint32_t* __restrict__ totals,
                                                      int64_t* __restrict__ d_n_out, int32_t* __restrict__ d_overflow) {
  __shared__ uint32_t s_wave[4];
  for (int c = 0; c < 3; ++c) {
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += 256) {
      const int b = b0 + threadIdx.x;
      const uint32_t v = b < nblocks ? counts[3 * (size_t)b + c] : 0u;
      uint32_t tot;
      const uint32_t ex = block_excl_scan(v, s_wave, &tot);
      if (b < nblocks) counts[3 * (size_t)b + c] = carry + ex;
      carry += tot;
    }
    if (threadIdx.x == 0) totals[c] = carry;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint64_t n_out = (uint64_t)totals[0] + totals[1] + (uint64_t)split_count * totals[2];
    const int32_t ov = (int64_t)n_out > capacity ? 1 : 0;
    totals[3] = (uint32_t)n_out;
    totals[4] = (uint32_t)ov;
    *d_n_out = (int64_t)n_out;
    *d_overflow = ov;
  }
}

__device__ __forceinline__ void copy_attrs(const gabsplat_scene& in, const gabsplat_scene_out& out, int64_t i,
                                           int64_t o, int64_t no, bool child, const gabsplat_densify_params& p) {
  const int64_t n = in.n;
  for (int a = 0; a < 3; ++a) out.means[a * no + o] = in.means[a * n + i];
  for (int a = 0; a < 3; ++a) out.scales[a * no + o] = in.scales[a * n + i];
  for (int a = 0; a < 4; ++a) out.quats[a * no + o] = in.quats[a * n + i];
  out.opacities[o] = in.opacities[i];
  // colour arrays are stored row by row
  if (in.sh) {
    const int nd = (in.sh_degree + 1) * (in.sh_degree + 1) * 3;
    for (int a = 0; a < nd; ++a) out.sh[o * nd + a] = in.sh[i * nd + a];
  } else {
    for (int a = 0; a < 3; ++a) out.colors[o * 3 + a] = in.colors[i * 3 + a];
  }
  for (int a = 0; a < 3 * in.k; ++a) out.freqs[(int64_t)a * no + o] = child ? p.freq_reset : in.freqs[(int64_t)a * n + i];
  for (int a = 0; a < in.k; ++a) out.weights[(int64_t)a * no + o] = child ? p.weight_reset : in.weights[(int64_t)a * n + i];
}

__global__ __launch_bounds__(256) void k_densify_write(gabsplat_scene in, const float* __restrict__ accum,
                                                       const float* __restrict__ denom,
                                                       const float* __restrict__ accum_abs,
                                                       const float* __restrict__ normals, gabsplat_densify_params p,
                                                       const uint32_t* __restrict__ counts,
                                                       const uint32_t* __restrict__ totals, gabsplat_scene_out out,
                                                       uint32_t* __restrict__ src_index, uint32_t* __restrict__ tag) {
  __shared__ uint32_t s_wave[4];
  if (totals[4]) return;
  const int64_t n = in.n;
  const int64_t no = totals[3];
  const uint32_t base_clone = totals[0], base_split = totals[0] + totals[1];
  const int t = threadIdx.x;
  int kind[kDenItems];
  uint32_t ck = 0, cc = 0, cs = 0;
#pragma unroll
  for (int j = 0; j < kDenItems; ++j) {
    // blocked within the block so that a thread's items are consecutive
    const int64_t i = (int64_t)blockIdx.x * kDenBlock + t * kDenItems + j;
    kind[j] = i < n ? densify_kind(in, accum, denom, accum_abs, p, i) : KIND_PRUNE;
    ck += (kind[j] == KIND_KEEP || kind[j] == KIND_CLONE);
    cc += (kind[j] == KIND_CLONE);
    cs += (kind[j] == KIND_SPLIT);
  }
  uint32_t tot;
  uint32_t pk = counts[3 * (size_t)blockIdx.x + 0] + block_excl_scan(ck, s_wave, &tot);
  uint32_t pc = counts[3 * (size_t)blockIdx.x + 1] + block_excl_scan(cc, s_wave, &tot);
  uint32_t ps = counts[3 * (size_t)blockIdx.x + 2] + block_excl_scan(cs, s_wave, &tot);
#pragma unroll
  for (int j = 0; j < kDenItems; ++j) {
    const int64_t i = (int64_t)blockIdx.x * kDenBlock + t * kDenItems + j;
    const int k = kind[j];
    if (k == KIND_KEEP || k == KIND_CLONE) {
      copy_attrs(in, out, i, pk, no, false, p);
      src_index[pk] = (uint32_t)i;
      tag[pk] = 0;
      ++pk;
    }
    if (k == KIND_CLONE) {
      const int64_t o = base_clone + pc;
      copy_attrs(in, out, i, o, no, true, p);
      src_index[o] = (uint32_t)i;
      tag[o] = 1;
      ++pc;
    }
    if (k == KIND_SPLIT) {
      // R(q) of the normalised quaternion
      const float qw = in.quats[i], qx = in.quats[n + i], qy = in.quats[2 * n + i], qz = in.quats[3 * n + i];
      const float il = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
      const float w = qw * il, x = qx * il, y = qy * il, z = qz * il;
      const float R[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                             {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                             {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
      const float s[3] = {in.scales[i], in.scales[n + i], in.scales[2 * n + i]};
      for (int c = 0; c < p.split_count; ++c) {
        const int64_t o = base_split + (int64_t)ps * p.split_count + c;
        copy_attrs(in, out, i, o, no, true, p);
        float zs[3];
        for (int a = 0; a < 3; ++a) zs[a] = s[a] * normals[((int64_t)c * 3 + a) * n + i];
        for (int a = 0; a < 3; ++a) {
          out.means[a * no + o] = in.means[a * n + i] + (R[a][0] * zs[0] + R[a][1] * zs[1] + R[a][2] * zs[2]);
          out.scales[a * no + o] = s[a] * p.split_shrink;
        }
        src_index[o] = (uint32_t)i;
        tag[o] = 2 + c;
      }
      ++ps;
    }
  }
}

__global__ __launch_bounds__(256) void k_reset_weights(gabsplat_scene_out sc, float wv, float ocap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sc.n) return;
  for (int a = 0; a < sc.k; ++a) sc.weights[(int64_t)a * sc.n + i] = wv;
  sc.opacities[i] = fminf(sc.opacities[i], ocap);
}

}  // namespace gs

using namespace gs;

extern "C" {

gabsplat_status gabsplat_densify_stats(const gabsplat_geom* geom, const gabsplat_camera* cams, int32_t num_views,
                                       int64_t n, const float* grad2d, int32_t grad_flags, float* accum,
                                       float* accum_abs, float* denom, void* stream) {
  try {
    const bool abs_stat = (grad_flags & GABSPLAT_GRAD_ABS_MEAN2D) != 0;
    if (!geom || !geom->views || !geom->tiles || !cams || num_views < 1 || n < 0 || n >= (1ll << 31) ||
        !grad2d || !accum || !denom || geom->k < 0 || geom->k > GABSPLAT_MAX_K ||
        (grad_flags & ~GABSPLAT_GRAD_ABS_MEAN2D) != 0 || (abs_stat && !accum_abs))
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (n == 0) return GABSPLAT_OK;
    GS_REQUIRE_DEVICE();
    hipLaunchKernelGGL(k_densify_stats, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), geom->views, n, geom->tiles, grad2d,
                       grad2d_stride(geom->k, grad_flags), abs_stat ? 10 + 3 * geom->k : -1, accum, accum_abs,
                       denom);
    return hipGetLastError() == hipSuccess ? GABSPLAT_OK : GABSPLAT_ERR_HIP;
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

size_t gabsplat_densify_workspace_size(int64_t n) {
  if (n < 0) return 0;
  return (size_t)(3 * ((n + kDenBlock - 1) / kDenBlock + 1) + 8) * 4;
}

gabsplat_status gabsplat_densify(const gabsplat_scene* in, const float* accum, const float* denom,
                                 const float* accum_abs, const float* normals, const gabsplat_densify_params* prm,
                                 const gabsplat_scene_out* out, int64_t out_capacity, uint32_t* src_index,
                                 uint32_t* tag, int64_t* d_n_out, int32_t* d_overflow, void* ws, size_t ws_bytes,
                                 void* stream) {
  try {
    if (!in || !prm || !out || !d_n_out || !d_overflow || in->n < 0 || in->n >= (1ll << 31) || out_capacity < 0 ||
        out_capacity >= (1ll << 32) || in->k < 0 || in->k > GABSPLAT_MAX_K || prm->split_count < 1 ||
        prm->split_count > 8)
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (in->n > 0 && (!in->means || !in->scales || !in->quats || !in->opacities || !accum || !denom || !normals ||
                      (in->k > 0 && (!in->freqs || !in->weights)) || ((in->sh == nullptr) == (in->colors == nullptr))))
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (out->k != in->k || (out->sh == nullptr) != (in->sh == nullptr) || !src_index || !tag)
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (in->n > 0 && prm->abs_grad_threshold > 0.f && !accum_abs) return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (!ws || ws_bytes < gabsplat_densify_workspace_size(in->n)) return GABSPLAT_ERR_WORKSPACE_TOO_SMALL;
    GS_REQUIRE_DEVICE();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nblocks = (int)((in->n + kDenBlock - 1) / kDenBlock);
    uint32_t* counts = static_cast<uint32_t*>(ws);
    uint32_t* totals = counts + 3 * (size_t)(nblocks + 1);
    if (nblocks > 0)
      hipLaunchKernelGGL(k_densify_count, dim3(nblocks), dim3(256), 0, s, *in, accum, denom, accum_abs, *prm,
                         counts);
    hipLaunchKernelGGL(k_densify_scan, dim3(1), dim3(256), 0, s, counts, nblocks, prm->split_count, out_capacity,
                       totals, d_n_out, d_overflow);
    if (nblocks > 0)
      hipLaunchKernelGGL(k_densify_write, dim3(nblocks), dim3(256), 0, s, *in, accum, denom, accum_abs, normals,
                         *prm, counts, totals, *out, src_index, tag);
    return hipGetLastError() == hipSuccess ? GABSPLAT_OK : GABSPLAT_ERR_HIP;
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

gabsplat_status gabsplat_reset_frequency_weights(const gabsplat_scene_out* scene, float weight_value,
                                                 float opacity_cap, void* stream) {
  try {
    if (!scene || scene->n < 0 || scene->n >= (1ll << 31) || scene->k < 0 || scene->k > GABSPLAT_MAX_K ||
        (scene->n > 0 && (!scene->opacities || (scene->k > 0 && !scene->weights))))
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (scene->n == 0) return GABSPLAT_OK;
    GS_REQUIRE_DEVICE();
    hipLaunchKernelGGL(k_reset_weights, dim3((unsigned)((scene->n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), *scene, weight_value, opacity_cap);
    return hipGetLastError() == hipSuccess ? GABSPLAT_OK : GABSPLAT_ERR_HIP;
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

}  // extern "C"
