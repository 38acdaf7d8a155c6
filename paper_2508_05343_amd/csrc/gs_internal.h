// Internal declarations of the gfx950 Gabor splatting kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gabsplat.h"

namespace gs {

constexpr int kTile = 16;
constexpr int kBlock = 256;                    // threads per tile workgroup (4 wave64)
constexpr float kAlphaMin = 1.0f / 255.0f;     // skip threshold on alpha
constexpr float kAlphaMax = 0.99f;             // alpha clamp
constexpr float kTMin = 1e-4f;                 // transmittance stop
constexpr float kDilation = 0.3f;              // px^2 added to the 2D covariance
constexpr float kMip2dVariance = 0.1f;         // px^2 of the 2D anti-aliasing filter
constexpr float kMip2dMinRatio = 1e-6f;        // floor of det S / det(S + 0.1 I)
// Bit 31 of a tile's end in the tile ranges: the tile's list is grouped by
// the bin sort but not yet in depth order.  The tile-count bin sort without
// keys leaves lists of up to kBlendSortCap pairs so marked, and the forward
// blend orders such a list (in place in vals) before blending it.
constexpr uint32_t kUnsortedBit = 0x80000000u;
constexpr int kBlendSortCap = 1024;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
// log2(1/255): o G < 1/255  <=>  q + log2 o < kLog2AlphaMin
constexpr float kLog2AlphaMin = -7.9943534368588578f;

// One scene as seen by the kernels (device copy of gabsplat_scene).
struct SceneEntry {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  const float* colors;
  const float* freqs;
  const float* weights;
  const float* filter3d;  // [n] 3D filter variance (GABSPLAT_FLAG_MIP_3D)
  const float* rows;      // [n][row_floats(k)] quats, freqs, weights by primitive, or null
  int64_t n;
  int32_t k;
  int32_t sh_degree;  // -1 for precomputed colours
  int32_t flags;      // GABSPLAT_FLAG_*
  int32_t pad;
};

// One view (camera + where its items, tiles and pixels live).
struct ViewEntry {
  float R[9];
  float t[3];
  float campos[3];
  float fx, fy, cx, cy, near_plane;
  float bg[3];
  int32_t width, height, tiles_x, tiles_y;
  int32_t tile_offset;   // first global tile id of this view
  int32_t scene;         // index into the scene table
  int64_t item_offset;   // first item of this view
  int64_t pixel_offset;  // first pixel of this view (image uses 3x)
};

// Device view table: header, then views, then scenes.
struct ViewTableHeader {
  int32_t num_views;
  int32_t num_scenes;
  int32_t total_tiles;
  int32_t pad;
  int64_t total_items;
  int64_t total_pixels;
};

inline size_t view_table_bytes(int num_views, int num_scenes) {
  return sizeof(ViewTableHeader) + sizeof(ViewEntry) * (size_t)num_views +
         sizeof(SceneEntry) * (size_t)num_scenes;
}

__host__ __device__ inline const ViewEntry* table_views(const void* t) {
  return reinterpret_cast<const ViewEntry*>(reinterpret_cast<const char*>(t) + sizeof(ViewTableHeader));
}
__host__ __device__ inline const SceneEntry* table_scenes(const void* t, int num_views) {
  return reinterpret_cast<const SceneEntry*>(reinterpret_cast<const char*>(t) + sizeof(ViewTableHeader) +
                                             sizeof(ViewEntry) * (size_t)num_views);
}

// Render record: the fields of gabsplat_geom.rec (10 + 3k floats, the mean's
// float32 rounding residuals at 10 + 3k and 11 + 3k), padded to float4s.
__host__ __device__ constexpr int record_stride(int k) { return (12 + 3 * k + 3) & ~3; }
__host__ __device__ constexpr int record_mean_lo(int k) { return 10 + 3 * k; }
inline int record_floats(int k) { return record_stride(k); }
// floats per row of gabsplat_scene.rows: quaternion, 3k frequencies, k weights, zeros to whole 128-byte lines
__host__ __device__ constexpr int row_stride(int k) { return (4 + 4 * k + 31) & ~31; }
__host__ __device__ inline int grad2d_floats(int k) { return (10 + 3 * k + 3) & ~3; }
__host__ __device__ inline int grad2d_stride(int k, int grad_flags) {
  return (grad_flags & GABSPLAT_GRAD_ABS_MEAN2D) ? (12 + 3 * k + 3) & ~3 : grad2d_floats(k);
}

// Host-side packed copy of the table (built by the API layer).
struct HostTable {
  ViewTableHeader hdr;
  ViewEntry* views;    // host array [num_views]
  SceneEntry* scenes;  // host array [num_scenes]
};

// Whether the current HIP device is a gfx950 (GABSPLAT_OK), is not
// (GABSPLAT_ERR_UNSUPPORTED_DEVICE), or cannot be queried (GABSPLAT_ERR_HIP).
// Asked once per device; every entry point that launches work checks it after
// its argument checks (so invalid arguments are reported without a device).
gabsplat_status device_status();
#define GS_REQUIRE_DEVICE()                                       \
  do {                                                            \
    const gabsplat_status ds_ = ::gs::device_status();             \
    if (ds_ != GABSPLAT_OK) return ds_;                           \
  } while (0)

// --- launchers (each returns hipSuccess or the first launch error) ---------
hipError_t upload_table(void* d_table, const HostTable& h, hipStream_t s);
// Copies `bytes` (a multiple of 4) of host memory to device memory with small
// kernels whose arguments carry the data (no copy engine, no host sync).
hipError_t upload_words(void* d_dst, const void* h_src, size_t bytes, hipStream_t s);

hipError_t launch_pack_rows(const gabsplat_scene& sc, float* rows, hipStream_t s);
hipError_t launch_preprocess(const void* d_table, const HostTable& h, const gabsplat_geom& g,
                             hipStream_t s);

struct BinSortPlan {
  int64_t items;
  int64_t capacity;
  int32_t total_tiles;
  int32_t tile_bits;
  size_t bytes;
  // offsets of each workspace region
  size_t off_counters, off_dkeys_a, off_dkeys_b, off_dvals_a, off_dvals_b, off_offsets, off_chunks;
  size_t off_tkeys_a, off_tkeys_b, off_pvals_b, off_hist, off_look_scan, off_tcount, off_tcursor, off_rs_hist, off_tcmat, off_tcpair_a, off_tcpair_b;
  int64_t parts_items, parts_pairs;
};
BinSortPlan plan_bin_sort(int64_t items, int64_t capacity, int32_t total_tiles);

hipError_t launch_bin_sort(const gabsplat_geom& g, const BinSortPlan& p, void* ws, uint64_t* keys,
                           uint32_t* vals, uint32_t* ranges, int64_t* d_num_pairs, int32_t* d_overflow,
                           hipStream_t s);

hipError_t launch_render_fwd(const void* d_table, const HostTable& h, const gabsplat_geom& g,
                             int k, uint32_t* vals, uint32_t* ranges, float* image,
                             float* final_T, uint32_t* n_contrib, uint32_t* eval_counts,
                             float* freq_map, const int32_t* d_overflow, hipStream_t s);

hipError_t launch_render_bwd(const void* d_table, const HostTable& h, const gabsplat_geom& g,
                             int k, const uint32_t* vals, const uint32_t* ranges,
                             const float* final_T, const uint32_t* n_contrib, const float* dl_dimage,
                             float* grad2d, bool abs_mean2d, const int32_t* d_overflow, hipStream_t s);

hipError_t launch_preprocess_bwd(const void* d_table, const HostTable& h, const gabsplat_geom& g,
                                 int scene_index, const gabsplat_scene_grads& gr,
                                 const int32_t* d_overflow, hipStream_t s);

size_t loss_workspace_bytes(int c, int h, int w);
hipError_t launch_loss(const float* x, const float* y, int c, int h, int w, float lambda,
                       float* d_loss, float* dl_dx, void* ws, hipStream_t s);

// generic fill kernel (used instead of memset so that callers may capture)
hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_clear_grad2d(const uint32_t* tiles, float* grad2d, int64_t items, int gf, hipStream_t s);

}  // namespace gs
