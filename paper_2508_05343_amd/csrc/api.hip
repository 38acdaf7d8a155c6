// C ABI of the gfx950 Gabor splatting library: argument validation, the view
// table, and kernel launches.  No allocation, no synchronisation (except
// gabsplat_read_overflow, documented as synchronous).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <vector>

#include "gabsplat.h"
#include "gs_internal.h"

namespace gs {

// The table is written to device memory by a kernel whose argument carries
// the bytes, so the upload is ordered on the stream and needs neither pinned
// host memory nor a host wait.
constexpr int kChunkWords = 448;
struct WordChunk {
  uint32_t n;
  uint32_t w[kChunkWords];
};

__global__ void k_store_words(uint32_t* __restrict__ dst, WordChunk c) {
  for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

gabsplat_status device_status() {
  constexpr int kMaxDevices = 64;
  static std::atomic<int> cache[kMaxDevices];  // 0 unknown, 1 gfx950, 2 other
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GABSPLAT_ERR_HIP;
  int c = (dev >= 0 && dev < kMaxDevices) ? cache[dev].load(std::memory_order_relaxed) : 0;
  if (c == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return GABSPLAT_ERR_HIP;
    c = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
    if (dev >= 0 && dev < kMaxDevices) cache[dev].store(c, std::memory_order_relaxed);
  }
  return c == 1 ? GABSPLAT_OK : GABSPLAT_ERR_UNSUPPORTED_DEVICE;
}

hipError_t upload_table(void* d_table, const HostTable& h, hipStream_t s) {
  const size_t bytes = view_table_bytes(h.hdr.num_views, h.hdr.num_scenes);
  std::vector<uint32_t> buf((bytes + 3) / 4, 0u);
  char* p = reinterpret_cast<char*>(buf.data());
  std::memcpy(p, &h.hdr, sizeof(ViewTableHeader));
  std::memcpy(p + sizeof(ViewTableHeader), h.views, sizeof(ViewEntry) * h.hdr.num_views);
  std::memcpy(p + sizeof(ViewTableHeader) + sizeof(ViewEntry) * h.hdr.num_views, h.scenes,
              sizeof(SceneEntry) * h.hdr.num_scenes);
  return upload_words(d_table, buf.data(), buf.size() * 4, s);
}

hipError_t upload_words(void* d_dst, const void* h_src, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  uint32_t* dst = static_cast<uint32_t*>(d_dst);
  const uint32_t* src = static_cast<const uint32_t*>(h_src);
  for (size_t off = 0; off < words; off += kChunkWords) {
    WordChunk c;
    c.n = (uint32_t)((words - off) < (size_t)kChunkWords ? (words - off) : (size_t)kChunkWords);
    std::memcpy(c.w, src + off, c.n * 4);
    hipLaunchKernelGGL(k_store_words, dim3(1), dim3(256), 0, s, dst + off, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace gs

using namespace gs;

namespace {

struct TableBuild {
  ViewTableHeader hdr{};
  std::vector<ViewEntry> views;
  std::vector<SceneEntry> scenes;
  HostTable host() {
    HostTable h;
    h.hdr = hdr;
    h.views = views.data();
    h.scenes = scenes.data();
    return h;
  }
};

bool valid_scene(const gabsplat_scene& s) {
  if (s.n < 0 || s.n >= (1ll << 31)) return false;
  if (s.k < 0 || s.k > GABSPLAT_MAX_K) return false;
  if (s.n == 0) return true;
  if (!s.means || !s.scales || !s.quats || !s.opacities) return false;
  if ((s.sh == nullptr) == (s.colors == nullptr)) return false;
  if (s.sh && (s.sh_degree < 0 || s.sh_degree > GABSPLAT_MAX_SH_DEGREE)) return false;
  if (s.k > 0 && (!s.freqs || !s.weights)) return false;
  if ((s.flags & GABSPLAT_FLAG_MIP_3D) && !s.filter3d) return false;
  if (s.rows && (reinterpret_cast<uintptr_t>(s.rows) & 15) != 0) return false;
  return true;
}

bool valid_camera(const gabsplat_camera& c) {
  if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384) return false;
  if (!(c.fx > 0.f) || !(c.fy > 0.f)) return false;
  return true;
}

// Builds the host table; returns INVALID_ARGUMENT on any inconsistency.
gabsplat_status build_table(const gabsplat_scene* scenes, int32_t num_scenes, const int32_t* scene_of_view,
                            const gabsplat_camera* cams, int32_t num_views, TableBuild& tb) {
  if (!scenes || !cams || num_scenes < 1 || num_views < 1 || num_views > GABSPLAT_MAX_VIEWS ||
      num_scenes > GABSPLAT_MAX_VIEWS)
    return GABSPLAT_ERR_INVALID_ARGUMENT;
  const int32_t k = scenes[0].k;
  const bool use_sh = scenes[0].sh != nullptr;
  const int32_t deg = use_sh ? scenes[0].sh_degree : -1;
  const int32_t flags = scenes[0].flags;
  tb.scenes.resize(num_scenes);
  for (int i = 0; i < num_scenes; ++i) {
    const gabsplat_scene& s = scenes[i];
    if (!valid_scene(s)) return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (s.k != k || (s.sh != nullptr) != use_sh || (use_sh && s.sh_degree != deg) || s.flags != flags ||
        (s.rows != nullptr) != (scenes[0].rows != nullptr) ||
        (s.flags & ~(GABSPLAT_FLAG_ATTENUATION | GABSPLAT_FLAG_MIP_2D | GABSPLAT_FLAG_MIP_3D)) != 0)
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    SceneEntry& e = tb.scenes[i];
    e.means = s.means; e.scales = s.scales; e.quats = s.quats; e.opac = s.opacities;
    e.sh = s.sh; e.colors = s.colors; e.freqs = s.freqs; e.weights = s.weights;
    e.filter3d = (s.flags & GABSPLAT_FLAG_MIP_3D) ? s.filter3d : nullptr;
    e.rows = s.rows;
    e.n = s.n; e.k = s.k; e.sh_degree = deg; e.flags = s.flags; e.pad = 0;
  }
  tb.views.resize(num_views);
  int64_t items = 0, pixels = 0, tiles = 0;
  for (int v = 0; v < num_views; ++v) {
    const gabsplat_camera& c = cams[v];
    if (!valid_camera(c)) return GABSPLAT_ERR_INVALID_ARGUMENT;
    const int sc = scene_of_view ? scene_of_view[v] : 0;
    if (sc < 0 || sc >= num_scenes) return GABSPLAT_ERR_INVALID_ARGUMENT;
    ViewEntry& e = tb.views[v];
    for (int r = 0; r < 3; ++r) {
      for (int q = 0; q < 3; ++q) e.R[3 * r + q] = c.world_to_cam[4 * r + q];
      e.t[r] = c.world_to_cam[4 * r + 3];
      e.campos[r] = c.cam_pos[r];
      e.bg[r] = c.bg[r];
    }
    e.fx = c.fx; e.fy = c.fy; e.cx = c.cx; e.cy = c.cy; e.near_plane = c.near_plane;
    e.width = c.width; e.height = c.height;
    e.tiles_x = (c.width + kTile - 1) / kTile;
    e.tiles_y = (c.height + kTile - 1) / kTile;
    e.tile_offset = (int32_t)tiles;
    e.scene = sc;
    e.item_offset = items;
    e.pixel_offset = pixels;
    items += tb.scenes[sc].n;
    pixels += (int64_t)c.width * c.height;
    tiles += (int64_t)e.tiles_x * e.tiles_y;
    if (tiles >= (1ll << 31) || items >= (1ll << 32)) return GABSPLAT_ERR_INVALID_ARGUMENT;
  }
  tb.hdr.num_views = num_views;
  tb.hdr.num_scenes = num_scenes;
  tb.hdr.total_tiles = (int32_t)tiles;
  tb.hdr.total_items = items;
  tb.hdr.total_pixels = pixels;
  return GABSPLAT_OK;
}

int64_t total_tiles_of(const gabsplat_camera* cams, int32_t num_views) {
  int64_t t = 0;
  for (int v = 0; v < num_views; ++v)
    t += (int64_t)((cams[v].width + kTile - 1) / kTile) * ((cams[v].height + kTile - 1) / kTile);
  return t;
}

gabsplat_status hip_status(hipError_t e) { return e == hipSuccess ? GABSPLAT_OK : GABSPLAT_ERR_HIP; }

}  // namespace

extern "C" {

int32_t gabsplat_abi_version(void) { return GABSPLAT_ABI_VERSION; }

const char* gabsplat_status_string(gabsplat_status s) {
  switch (s) {
    case GABSPLAT_OK: return "ok";
    case GABSPLAT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case GABSPLAT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case GABSPLAT_ERR_CAPACITY_EXCEEDED: return "pair capacity exceeded";
    case GABSPLAT_ERR_HIP: return "HIP runtime error";
    case GABSPLAT_ERR_UNSUPPORTED_DEVICE: return "unsupported device (gfx950 required)";
    case GABSPLAT_ERR_SCRATCH_LIMIT: return "problem larger than the static scratch of the allocation-free entry point";
  }
  return "unknown status";
}

int32_t gabsplat_record_floats(int32_t k) { return (k < 0 || k > GABSPLAT_MAX_K) ? -1 : record_floats(k); }
int32_t gabsplat_row_floats(int32_t k) { return (k < 0 || k > GABSPLAT_MAX_K) ? -1 : row_stride(k); }
int32_t gabsplat_grad2d_floats(int32_t k) { return (k < 0 || k > GABSPLAT_MAX_K) ? -1 : grad2d_floats(k); }
int32_t gabsplat_grad2d_stride(int32_t k, int32_t grad_flags) {
  if (k < 0 || k > GABSPLAT_MAX_K || (grad_flags & ~GABSPLAT_GRAD_ABS_MEAN2D) != 0) return -1;
  return grad2d_stride(k, grad_flags);
}

size_t gabsplat_views_bytes(int32_t num_views, int32_t num_scenes) {
  if (num_views < 0 || num_scenes < 0) return 0;
  return view_table_bytes(num_views, num_scenes);
}

size_t gabsplat_bin_sort_workspace_size(int64_t items, int64_t pair_capacity, int64_t total_tiles) {
  if (items < 0 || pair_capacity < 0 || total_tiles < 0 || total_tiles >= (1ll << 31)) return 0;
  return plan_bin_sort(items, pair_capacity, (int32_t)total_tiles).bytes;
}

gabsplat_status gabsplat_check_device(void) {
  try {
    return device_status();
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

gabsplat_status gabsplat_preprocess(const gabsplat_scene* scenes, int32_t num_scenes, const int32_t* scene_of_view,
                                    const gabsplat_camera* cams, int32_t num_views, const gabsplat_geom* geom,
                                    void* stream) {
  try {
    if (!geom || !geom->views) return GABSPLAT_ERR_INVALID_ARGUMENT;
    TableBuild tb;
    gabsplat_status st = build_table(scenes, num_scenes, scene_of_view, cams, num_views, tb);
    if (st != GABSPLAT_OK) return st;
    if (geom->k != tb.scenes[0].k) return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (tb.hdr.total_items > 0 && (!geom->rec || !geom->depth || !geom->rect || !geom->tiles))
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HostTable h = tb.host();
    GS_REQUIRE_DEVICE();
    hipError_t e = upload_table(geom->views, h, s);
    if (e != hipSuccess) return GABSPLAT_ERR_HIP;
    return hip_status(launch_preprocess(geom->views, h, *geom, s));
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

gabsplat_status gabsplat_pack_rows(const gabsplat_scene* scene, float* rows, void* stream) {
  try {
    if (!scene || !rows || (reinterpret_cast<uintptr_t>(rows) & 15) != 0) return GABSPLAT_ERR_INVALID_ARGUMENT;
    gabsplat_scene sc = *scene;
    sc.rows = nullptr;  // the scene's own rows are not read
    if (!valid_scene(sc)) return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (sc.n == 0) return GABSPLAT_OK;
    GS_REQUIRE_DEVICE();
    return hip_status(launch_pack_rows(sc, rows, static_cast<hipStream_t>(stream)));
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

gabsplat_status gabsplat_bin_sort(const gabsplat_geom* geom, const gabsplat_camera* cams, int32_t num_views,
                                  int64_t items, void* ws, size_t ws_bytes, uint64_t* keys, uint32_t* vals,
                                  int64_t pair_capacity, uint32_t* tile_ranges, int64_t* d_num_pairs,
                                  int32_t* d_overflow, void* stream) {
  try {
    if (!geom || !cams || num_views < 1 || num_views > GABSPLAT_MAX_VIEWS || items < 0 || items >= (1ll << 32) ||
        pair_capacity < 0 || pair_capacity >= (1ll << 32) || !d_num_pairs || !d_overflow || !geom->views)
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    for (int v = 0; v < num_views; ++v)
      if (!valid_camera(cams[v])) return GABSPLAT_ERR_INVALID_ARGUMENT;
    const int64_t tiles = total_tiles_of(cams, num_views);
    if (tiles >= (1ll << 31)) return GABSPLAT_ERR_INVALID_ARGUMENT;
    if ((pair_capacity > 0 && !vals) || (tiles > 0 && !tile_ranges)) return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (items > 0 && (!geom->depth || !geom->rect || !geom->tiles)) return GABSPLAT_ERR_INVALID_ARGUMENT;
    const BinSortPlan p = plan_bin_sort(items, pair_capacity, (int32_t)tiles);
    if (!ws || ws_bytes < p.bytes) return GABSPLAT_ERR_WORKSPACE_TOO_SMALL;
    GS_REQUIRE_DEVICE();
    return hip_status(launch_bin_sort(*geom, p, ws, keys, vals, tile_ranges, d_num_pairs, d_overflow,
                                      static_cast<hipStream_t>(stream)));
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

gabsplat_status gabsplat_render_fwd(const gabsplat_geom* geom, uint32_t* vals, uint32_t* tile_ranges,
                                    const gabsplat_camera* cams, int32_t num_views, float* image, float* final_T,
                                    uint32_t* n_contrib, uint32_t* eval_counts, float* freq_map,
                                    const int32_t* d_overflow, void* stream) {
  try {
    if (!geom || !geom->views || !geom->rec || !geom->depth || geom->k < 0 || geom->k > GABSPLAT_MAX_K || !cams ||
        num_views < 1 || num_views > GABSPLAT_MAX_VIEWS || !tile_ranges || !image || !final_T || !n_contrib)
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    for (int v = 0; v < num_views; ++v)
      if (!valid_camera(cams[v])) return GABSPLAT_ERR_INVALID_ARGUMENT;
    const int64_t tiles = total_tiles_of(cams, num_views);
    if (tiles >= (1ll << 31)) return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (tiles > 0 && !vals) return GABSPLAT_ERR_INVALID_ARGUMENT;
    HostTable h{};
    h.hdr.num_views = num_views;
    h.hdr.total_tiles = (int32_t)tiles;
    GS_REQUIRE_DEVICE();
    return hip_status(launch_render_fwd(geom->views, h, *geom, geom->k, vals, tile_ranges, image, final_T,
                                        n_contrib, eval_counts, freq_map, d_overflow,
                                        static_cast<hipStream_t>(stream)));
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

gabsplat_status gabsplat_render_bwd(const gabsplat_scene* scenes, int32_t num_scenes, const int32_t* scene_of_view,
                                    const gabsplat_camera* cams, int32_t num_views, const gabsplat_geom* geom,
                                    const uint32_t* vals, const uint32_t* tile_ranges, const float* final_T,
                                    const uint32_t* n_contrib, const float* dl_dimage,
                                    const gabsplat_scene_grads* grads, const int32_t* d_overflow, void* stream) {
  return gabsplat_render_bwd_stages(scenes, num_scenes, scene_of_view, cams, num_views, geom, vals, tile_ranges,
                                    final_T, n_contrib, dl_dimage, grads, d_overflow,
                                    GABSPLAT_BWD_BLEND | GABSPLAT_BWD_PROJECT, stream);
}

gabsplat_status gabsplat_render_bwd_stages(const gabsplat_scene* scenes, int32_t num_scenes,
                                           const int32_t* scene_of_view, const gabsplat_camera* cams,
                                           int32_t num_views, const gabsplat_geom* geom, const uint32_t* vals,
                                           const uint32_t* tile_ranges, const float* final_T,
                                           const uint32_t* n_contrib, const float* dl_dimage,
                                           const gabsplat_scene_grads* grads, const int32_t* d_overflow,
                                           int32_t stages, void* stream) {
  try {
    if (!geom || !geom->views || !geom->rec || !geom->tiles || !grads || !tile_ranges || !final_T || !n_contrib || !dl_dimage)
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (stages < 1 || (stages & ~(GABSPLAT_BWD_BLEND | GABSPLAT_BWD_PROJECT)) != 0) return GABSPLAT_ERR_INVALID_ARGUMENT;
    TableBuild tb;
    gabsplat_status st = build_table(scenes, num_scenes, scene_of_view, cams, num_views, tb);
    if (st != GABSPLAT_OK) return st;
    if (tb.scenes[0].k != geom->k) return GABSPLAT_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < num_scenes; ++i) {
      const gabsplat_scene_grads& g = grads[i];
      if (!g.grad2d || (g.flags & ~GABSPLAT_GRAD_ABS_MEAN2D) != 0 || g.flags != grads[0].flags)
        return GABSPLAT_ERR_INVALID_ARGUMENT;
      if (scenes[i].sh && g.colors) return GABSPLAT_ERR_INVALID_ARGUMENT;
      if (scenes[i].colors && g.sh) return GABSPLAT_ERR_INVALID_ARGUMENT;
      if (i > 0 && g.grad2d != grads[0].grad2d) return GABSPLAT_ERR_INVALID_ARGUMENT;
    }
    if (tb.hdr.total_tiles > 0 && !vals) return GABSPLAT_ERR_INVALID_ARGUMENT;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HostTable h = tb.host();
    const bool abs_mean2d = (grads[0].flags & GABSPLAT_GRAD_ABS_MEAN2D) != 0;
    GS_REQUIRE_DEVICE();
    if (stages & GABSPLAT_BWD_BLEND) {
      hipError_t e = launch_clear_grad2d(geom->tiles, grads[0].grad2d, tb.hdr.total_items,
                                         grad2d_stride(geom->k, grads[0].flags), s);
      if (e != hipSuccess) return GABSPLAT_ERR_HIP;
      e = launch_render_bwd(geom->views, h, *geom, geom->k, vals, tile_ranges, final_T, n_contrib, dl_dimage,
                            grads[0].grad2d, abs_mean2d, d_overflow, s);
      if (e != hipSuccess) return GABSPLAT_ERR_HIP;
    }
    if (stages & GABSPLAT_BWD_PROJECT) {
      for (int i = 0; i < num_scenes; ++i) {
        const hipError_t e = launch_preprocess_bwd(geom->views, h, *geom, i, grads[i], d_overflow, s);
        if (e != hipSuccess) return GABSPLAT_ERR_HIP;
      }
    }
    return GABSPLAT_OK;
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

size_t gabsplat_loss_workspace_size(int32_t channels, int32_t height, int32_t width) {
  if (channels < 1 || height < 1 || width < 1) return 0;
  return loss_workspace_bytes(channels, height, width);
}

gabsplat_status gabsplat_loss_l1_dssim(const float* x, const float* y, int32_t channels, int32_t height,
                                       int32_t width, float lambda, float* d_loss, float* dl_dx, void* ws,
                                       size_t ws_bytes, void* stream) {
  try {
    if (!x || !y || !d_loss || !dl_dx || channels < 1 || height < 1 || width < 1 || height > 65535 * 16 ||
        width > 65535 * 16 || channels > 65535 || !(lambda >= 0.f && lambda <= 1.f))
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (!ws || ws_bytes < loss_workspace_bytes(channels, height, width)) return GABSPLAT_ERR_WORKSPACE_TOO_SMALL;
    GS_REQUIRE_DEVICE();
    return hip_status(launch_loss(x, y, channels, height, width, lambda, d_loss, dl_dx, ws,
                                  static_cast<hipStream_t>(stream)));
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

gabsplat_status gabsplat_read_overflow(const int32_t* d_overflow, void* stream) {
  try {
    if (!d_overflow) return GABSPLAT_ERR_INVALID_ARGUMENT;
    int32_t v = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&v, d_overflow, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess) return GABSPLAT_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GABSPLAT_ERR_HIP;
    return v ? GABSPLAT_ERR_CAPACITY_EXCEEDED : GABSPLAT_OK;
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

}  // extern "C"
