// Variance of Mip-Splatting's 3D smoothing filter per primitive: the
// anti-aliasing the paper combines with its Gabor primitive (Sec. 4.1,
// Table 1).  The sampling rate of a camera at a primitive is its focal length
// over the primitive's depth; the filter variance is s / r^2 for the largest
// rate r over the cameras whose grown frustum holds the mean, and primitives
// no camera sees take the largest variance of the others.
//
// Three launches over the primitives: rates and per-block maxima, one block
// reducing the block maxima, and a fill of the unseen entries.  The camera
// table lives in the caller's workspace.
#include <hip/hip_runtime.h>

#include <vector>

#include "gs_internal.h"

namespace gs {

struct MipCam {
  float R[9];  // world -> camera rotation, row-major
  float t[3];
  float fmax, fx, fy, cx, cy, near_plane, width, height;
};
static_assert(sizeof(MipCam) == 20 * sizeof(float), "camera record layout");

constexpr int kMipBlock = 256;

inline size_t mip_cam_bytes(int ncams) { return ((size_t)ncams * sizeof(MipCam) + 255) & ~(size_t)255; }
inline int64_t mip_blocks(int64_t n) { return (n + kMipBlock - 1) / kMipBlock; }

__device__ __forceinline__ float block_max_256(float m, float* s_w) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = m;
  __syncthreads();
  return fmaxf(fmaxf(s_w[0], s_w[1]), fmaxf(s_w[2], s_w[3]));
}

// out[i] = s / r^2, or -1 when no camera sees primitive i; bmax[block] = the
// block's largest variance (float bits; variances are >= 0, so their bit
// patterns order like the values).
__global__ __launch_bounds__(kMipBlock) void k_mip_rate(const float* __restrict__ means, int64_t n,
                                                        const MipCam* __restrict__ cams, int ncams, float s,
                                                        float margin, float* __restrict__ out,
                                                        uint32_t* __restrict__ bmax) {
  __shared__ float s_w[kMipBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kMipBlock + threadIdx.x;
  float best = 0.f;
  bool seen = false;
  if (i < n) {
    const float x = means[i], y = means[n + i], z = means[2 * n + i];
    for (int c = 0; c < ncams; ++c) {
      const MipCam& C = cams[c];
      const float pz = fmaf(C.R[6], x, fmaf(C.R[7], y, fmaf(C.R[8], z, C.t[2])));
      if (!(pz > C.near_plane)) continue;
      const float px = fmaf(C.R[0], x, fmaf(C.R[1], y, fmaf(C.R[2], z, C.t[0])));
      const float py = fmaf(C.R[3], x, fmaf(C.R[4], y, fmaf(C.R[5], z, C.t[1])));
      const float iz = 1.0f / pz;
      const float u = fmaf(C.fx * px, iz, C.cx), v = fmaf(C.fy * py, iz, C.cy);
      const bool inside = u >= -margin * C.width && u <= (1.0f + margin) * C.width &&
                          v >= -margin * C.height && v <= (1.0f + margin) * C.height;
      if (inside) {
        best = fmaxf(best, C.fmax * iz);
        seen = true;
      }
    }
    out[i] = seen ? s / (best * best) : -1.0f;
  }
  const float m = block_max_256(seen ? s / (best * best) : 0.f, s_w);
  if (threadIdx.x == 0) bmax[blockIdx.x] = __float_as_uint(m);
}

// One block: bmax[nb] = max over bmax[0 .. nb).
__global__ __launch_bounds__(kMipBlock) void k_mip_max(uint32_t* __restrict__ bmax, int64_t nb) {
  __shared__ float s_w[kMipBlock / 64];
  float m = 0.f;
  for (int64_t b = threadIdx.x; b < nb; b += kMipBlock) m = fmaxf(m, __uint_as_float(bmax[b]));
  m = block_max_256(m, s_w);
  if (threadIdx.x == 0) bmax[nb] = __float_as_uint(m);
}

__global__ __launch_bounds__(kMipBlock) void k_mip_fill(float* __restrict__ out, int64_t n,
                                                        const uint32_t* __restrict__ gmax) {
  const int64_t i = (int64_t)blockIdx.x * kMipBlock + threadIdx.x;
  if (i < n && out[i] < 0.f) out[i] = __uint_as_float(*gmax);
}

}  // namespace gs

using namespace gs;

extern "C" {

size_t gabsplat_mip_filter3d_workspace_size(int64_t n, int32_t num_cams) {
  if (n < 0 || n >= (1ll << 31) || num_cams < 1 || num_cams > GABSPLAT_MAX_VIEWS) return 0;
  return mip_cam_bytes(num_cams) + (size_t)(mip_blocks(n) + 1) * sizeof(uint32_t);
}

gabsplat_status gabsplat_mip_filter3d(const float* means, int64_t n, const gabsplat_camera* cams,
                                      int32_t num_cams, float s, float margin, float* filter3d, void* ws,
                                      size_t ws_bytes, void* stream) {
  try {
    if (!cams || num_cams < 1 || num_cams > GABSPLAT_MAX_VIEWS || n < 0 || n >= (1ll << 31) || !(s >= 0.f) ||
        !(margin >= 0.f) || (n > 0 && (!means || !filter3d)))
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    for (int c = 0; c < num_cams; ++c)
      if (cams[c].width < 1 || cams[c].height < 1 || !(cams[c].fx > 0.f) || !(cams[c].fy > 0.f))
        return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (n == 0) return GABSPLAT_OK;
    if (!ws || ws_bytes < gabsplat_mip_filter3d_workspace_size(n, num_cams)) return GABSPLAT_ERR_WORKSPACE_TOO_SMALL;
    GS_REQUIRE_DEVICE();
    std::vector<MipCam> table((size_t)num_cams);
    for (int c = 0; c < num_cams; ++c) {
      const gabsplat_camera& g = cams[c];
      MipCam& m = table[c];
      for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) m.R[3 * r + q] = g.world_to_cam[4 * r + q];
        m.t[r] = g.world_to_cam[4 * r + 3];
      }
      m.fmax = g.fx > g.fy ? g.fx : g.fy;
      m.fx = g.fx; m.fy = g.fy; m.cx = g.cx; m.cy = g.cy;
      m.near_plane = g.near_plane;
      m.width = (float)g.width;
      m.height = (float)g.height;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    MipCam* d_cams = static_cast<MipCam*>(ws);
    uint32_t* bmax = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + mip_cam_bytes(num_cams));
    if (upload_words(d_cams, table.data(), table.size() * sizeof(MipCam), st) != hipSuccess) return GABSPLAT_ERR_HIP;
    const int64_t nb = mip_blocks(n);
    hipLaunchKernelGGL(k_mip_rate, dim3((unsigned)nb), dim3(kMipBlock), 0, st, means, n, d_cams, num_cams, s, margin,
                       filter3d, bmax);
    hipLaunchKernelGGL(k_mip_max, dim3(1), dim3(kMipBlock), 0, st, bmax, nb);
    hipLaunchKernelGGL(k_mip_fill, dim3((unsigned)nb), dim3(kMipBlock), 0, st, filter3d, n, bmax + nb);
    return hipGetLastError() == hipSuccess ? GABSPLAT_OK : GABSPLAT_ERR_HIP;
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}

}  // extern "C"
