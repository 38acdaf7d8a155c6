// K9: photometric loss (1 - lambda) L1 + lambda (1 - SSIM) and its gradient
// (Sec. 3.4.1, lambda = 0.2).  SSIM uses an 11x11 Gaussian window (sigma 1.5)
// with zero padding; the five local moments are separable filters staged in
// LDS per 32x16 output tile (horizontal pass: runs of 4 outputs per lane from
// registers; vertical pass: pairs of rows per lane).  With A1 = 2 mx my + C1, A2 = 2 sxy + C2,
// B1 = mx^2 + my^2 + C1, B2 = sxx + syy + C2 and s = A1 A2 / (B1 B2):
//   ds/dmx  = s (2 my / A1 - 2 my / A2 - 2 mx / B1 + 2 mx / B2)
//   ds/dExx = -s / B2,   ds/dExy = 2 s / A2
// (Exx, Exy the filtered x^2 and x y), and since the window is symmetric the
// adjoint of each filter is the filter itself:
//   dL/dx = G*(g ds/dmx) + 2 x G*(g ds/dExx) + y G*(g ds/dExy),  g = -lambda / N.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "gs_internal.h"

namespace gs {

constexpr int kWin = 11;
constexpr int kHalo = 5;
constexpr int kTX = 32, kTY = 16;        // output tile of one 256-lane block
constexpr int kSY = kTY + 2 * kHalo;     // staged rows (26)
constexpr int kSX = kTX + 2 * kHalo;     // staged columns (42)
constexpr int kSP = 44;                  // LDS row pitch: 16-byte aligned rows
constexpr int kRun = 4;                  // horizontal outputs per lane
constexpr int kRuns = kTX / kRun;        // runs per row (8)
constexpr int kHLanes = kSY * kRuns;     // lanes busy in the horizontal pass (208)

struct Window {
  float g[kWin];
};

static Window gaussian_window() {
  Window w;
  double s = 0.0, v[kWin];
  for (int i = 0; i < kWin; ++i) {
    const double d = i - kHalo;
    v[i] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    s += v[i];
  }
  for (int i = 0; i < kWin; ++i) w.g[i] = (float)(v[i] / s);
  return w;
}

__device__ __forceinline__ float block_sum(float v, float* s_red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_red[w] = v;
  __syncthreads();
  float tot = 0.f;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += s_red[i];
  __syncthreads();
  return tot;
}

// Stages the (kSY x kSX) neighbourhood of the block's output tile of NM
// planes (zero outside the image) into LDS rows of pitch kSP.
template <int NM>
__device__ __forceinline__ void stage_planes(const float* const (&src)[NM], int H, int W, int ox, int oy,
                                             float (*dst)[kSY][kSP]) {
  for (int i = threadIdx.x; i < kSY * kSX; i += 256) {
    const int r = i / kSX, q = i - r * kSX;
    const int gy = oy + r - kHalo, gx = ox + q - kHalo;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const size_t o = (size_t)gy * W + gx;
#pragma unroll
    for (int m = 0; m < NM; ++m) dst[m][r][q] = in ? src[m][o] : 0.f;
  }
}

// The kRun + kWin - 1 = 14 staged values a run of 4 outputs reads, from a row
// position that is a multiple of 4 (three 16-byte and one 8-byte LDS read).
constexpr int kRunIn = kRun + kWin - 1;
__device__ __forceinline__ void load_run(const float* row, float (&v)[kRunIn]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float4 t = reinterpret_cast<const float4*>(row)[j];
    v[4 * j] = t.x; v[4 * j + 1] = t.y; v[4 * j + 2] = t.z; v[4 * j + 3] = t.w;
  }
  const float2 t = reinterpret_cast<const float2*>(row)[6];
  v[12] = t.x;
  v[13] = t.y;
}

// Output tile of a block.  Consecutive workgroups go to the GPU's 8 XCDs in
// turn and each XCD has its own L2, while the staged halos of neighbouring
// tiles overlap: neighbours should run on one XCD.  Workgroup b (linear id,
// x fastest) runs on XCD b % 8, so the blocks with b % 8 = j take the j-th
// contiguous run of tiles (runs of ceil(n/8) tiles, then of floor(n/8)): a
// permutation of the tiles, whatever order the dispatch actually uses.
constexpr uint32_t kXcds = 8;
struct TileId {
  int x, y, c;
  uint32_t linear;
};

__device__ __forceinline__ TileId xcd_tile() {
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  const uint32_t n = gx * gy * gridDim.z;
  const uint32_t b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t q = n / kXcds, r = n % kXcds, j = b % kXcds, k = b / kXcds;
  const uint32_t t = j < r ? j * (q + 1) + k : r * (q + 1) + (j - r) * q + k;
  TileId id;
  id.x = (int)(t % gx);
  id.y = (int)((t / gx) % gy);
  id.c = (int)(t / (gx * gy));
  id.linear = t;
  return id;
}

// pass 1: moments, SSIM map, per-pixel factors for the backward, partial sums
__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Window win, float lambda, float inv_n,
                                                  float* __restrict__ f3, float* __restrict__ partial,
                                                  uint32_t* __restrict__ counter) {
  __shared__ __align__(16) float s_in[2][kSY][kSP];
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *counter = 0u;
  __shared__ __align__(16) float s_h[5][kSY][kTX];
  __shared__ float s_red[4];
  const TileId tid = xcd_tile();
  const int c = tid.c;
  const int ox = tid.x * kTX, oy = tid.y * kTY;
  const size_t plane = (size_t)H * W;
  const float* const src[2] = {x + c * plane, y + c * plane};
  stage_planes<2>(src, H, W, ox, oy, s_in);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kHLanes) {  // horizontal pass: lane = (row, run of 4 outputs)
    const int r = t / kRuns, q0 = (t % kRuns) * kRun;
    float xv[kRunIn], yv[kRunIn];
    load_run(&s_in[0][r][q0], xv);
    load_run(&s_in[1][r][q0], yv);
    float a[kRun], b[kRun], aa[kRun], bb[kRun], ab[kRun];
#pragma unroll
    for (int o = 0; o < kRun; ++o) a[o] = b[o] = aa[o] = bb[o] = ab[o] = 0.f;
#pragma unroll
    for (int j = 0; j < kRunIn; ++j) {
      const float xx = xv[j] * xv[j], yy = yv[j] * yv[j], xy = xv[j] * yv[j];
#pragma unroll
      for (int o = 0; o < kRun; ++o) {
        const int k = j - o;
        if (k >= 0 && k < kWin) {
          const float g = win.g[k];
          a[o] = fmaf(g, xv[j], a[o]);
          b[o] = fmaf(g, yv[j], b[o]);
          aa[o] = fmaf(g, xx, aa[o]);
          bb[o] = fmaf(g, yy, bb[o]);
          ab[o] = fmaf(g, xy, ab[o]);
        }
      }
    }
    *reinterpret_cast<float4*>(&s_h[0][r][q0]) = make_float4(a[0], a[1], a[2], a[3]);
    *reinterpret_cast<float4*>(&s_h[1][r][q0]) = make_float4(b[0], b[1], b[2], b[3]);
    *reinterpret_cast<float4*>(&s_h[2][r][q0]) = make_float4(aa[0], aa[1], aa[2], aa[3]);
    *reinterpret_cast<float4*>(&s_h[3][r][q0]) = make_float4(bb[0], bb[1], bb[2], bb[3]);
    *reinterpret_cast<float4*>(&s_h[4][r][q0]) = make_float4(ab[0], ab[1], ab[2], ab[3]);
  }
  __syncthreads();
  // vertical pass: lane = (column, pair of rows)
  const int q = t % kTX, r0 = (t / kTX) * 2;
  float m[5][2];
#pragma unroll
  for (int mm = 0; mm < 5; ++mm) {
    m[mm][0] = m[mm][1] = 0.f;
#pragma unroll
    for (int j = 0; j < kWin + 1; ++j) {
      const float v = s_h[mm][r0 + j][q];
      if (j < kWin) m[mm][0] = fmaf(win.g[j], v, m[mm][0]);
      if (j >= 1) m[mm][1] = fmaf(win.g[j - 1], v, m[mm][1]);
    }
  }
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  const float g = -lambda * inv_n;
  const size_t nn = plane * gridDim.z;
  float ssim = 0.f, l1 = 0.f;
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int gy = oy + r0 + o, gx = ox + q;
    if (gy < H && gx < W) {
      const float mx = m[0][o], my = m[1][o];
      const float sxx = m[2][o] - mx * mx, syy = m[3][o] - my * my, sxy = m[4][o] - mx * my;
      const float A1 = 2.f * mx * my + C1, A2 = 2.f * sxy + C2;
      const float B1 = mx * mx + my * my + C1, B2 = sxx + syy + C2;
      // four hardware reciprocals (about 1 ulp) instead of seven IEEE
      // divisions; A1, B1 >= C1 and B2 >= C2 (up to rounding of the moments),
      // A2 takes the sign of the covariance
      const float rA1 = __builtin_amdgcn_rcpf(A1), rA2 = __builtin_amdgcn_rcpf(A2);
      const float rB1 = __builtin_amdgcn_rcpf(B1), rB2 = __builtin_amdgcn_rcpf(B2);
      const float s = (A1 * A2) * (rB1 * rB2);
      ssim += s;
      l1 += fabsf(s_in[0][r0 + o + kHalo][q + kHalo] - s_in[1][r0 + o + kHalo][q + kHalo]);
      const size_t off = c * plane + (size_t)gy * W + gx;
      const float gs = g * s;
      f3[off] = 2.f * gs * (my * (rA1 - rA2) + mx * (rB2 - rB1));
      f3[nn + off] = -gs * rB2;
      f3[2 * nn + off] = 2.f * gs * rA2;
    }
  }
  const float ts = block_sum(ssim, s_red);
  const float tl = block_sum(l1, s_red);
  if (threadIdx.x == 0) {
    partial[2 * (size_t)tid.linear] = tl;
    partial[2 * (size_t)tid.linear + 1] = ts;
  }
}

// Sum of the per-tile partials, folded into the SSIM backward (which runs
// after the forward wrote every partial): its first nparts blocks, by linear
// block id, each reduce a contiguous slice; the last of them to finish
// (completion counter, zeroed by k_ssim_fwd and again by that block) adds the
// slice sums in slice order, so the result does not depend on which finishes
// last.  Slice sums are published and read with agent-scope atomics (the
// XCDs' L2s are not coherent).
constexpr int kFinalBlocks = 256;
constexpr int kFinalSlice = 2048;  // partial pairs per slice (before the cap)

__device__ __forceinline__ void loss_final_part(const float* __restrict__ partial, int nb, float lambda,
                                                float inv_n, float* __restrict__ part2,
                                                uint32_t* __restrict__ counter, float* __restrict__ d_loss,
                                                int part, int nparts, float* s_red, int* s_last) {
  const int per = (nb + nparts - 1) / nparts;
  const int b0 = part * per, b1 = min(nb, b0 + per);
  float l1 = 0.f, ss = 0.f;
  for (int i = b0 + (int)threadIdx.x; i < b1; i += 256) {
    l1 += partial[2 * i];
    ss += partial[2 * i + 1];
  }
  l1 = block_sum(l1, s_red);
  ss = block_sum(ss, s_red);
  if (threadIdx.x == 0) {
    __hip_atomic_store(&part2[2 * part], l1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&part2[2 * part + 1], ss, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t done = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    *s_last = done == (uint32_t)nparts - 1;
  }
  __syncthreads();
  if (!*s_last) return;
  float a = 0.f, b = 0.f;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    a += __hip_atomic_load(&part2[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b += __hip_atomic_load(&part2[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  a = block_sum(a, s_red);
  b = block_sum(b, s_red);
  if (threadIdx.x == 0) {
    *d_loss = (1.f - lambda) * a * inv_n + lambda * (1.f - b * inv_n);
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// pass 2: filter the three factor maps and combine
__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Window win, float lambda, float inv_n,
                                                  const float* __restrict__ f3, float* __restrict__ dl_dx,
                                                  const float* __restrict__ partial, int nb, int nfin,
                                                  float* __restrict__ part2, uint32_t* __restrict__ counter,
                                                  float* __restrict__ d_loss) {
  __shared__ __align__(16) float s_f[3][kSY][kSP];
  __shared__ __align__(16) float s_h[3][kSY][kTX];
  __shared__ float s_red[4];
  __shared__ int s_last;
  const TileId tid = xcd_tile();
  const int c = tid.c;
  const int ox = tid.x * kTX, oy = tid.y * kTY;
  const size_t plane = (size_t)H * W;
  const size_t nn = plane * gridDim.z;
  const float* const src[3] = {f3 + c * plane, f3 + nn + c * plane, f3 + 2 * nn + c * plane};
  stage_planes<3>(src, H, W, ox, oy, s_f);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < kHLanes) {
    const int r = t / kRuns, q0 = (t % kRuns) * kRun;
#pragma unroll
    for (int mm = 0; mm < 3; ++mm) {
      float v[kRunIn];
      load_run(&s_f[mm][r][q0], v);
      float acc[kRun];
#pragma unroll
      for (int o = 0; o < kRun; ++o) {
        acc[o] = 0.f;
#pragma unroll
        for (int k = 0; k < kWin; ++k) acc[o] = fmaf(win.g[k], v[o + k], acc[o]);
      }
      *reinterpret_cast<float4*>(&s_h[mm][r][q0]) = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
  }
  __syncthreads();
  const int q = t % kTX, r0 = (t / kTX) * 2;
  float m[3][2];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    m[mm][0] = m[mm][1] = 0.f;
#pragma unroll
    for (int j = 0; j < kWin + 1; ++j) {
      const float v = s_h[mm][r0 + j][q];
      if (j < kWin) m[mm][0] = fmaf(win.g[j], v, m[mm][0]);
      if (j >= 1) m[mm][1] = fmaf(win.g[j - 1], v, m[mm][1]);
    }
  }
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int gy = oy + r0 + o, gx = ox + q;
    if (gy < H && gx < W) {
      const size_t off = c * plane + (size_t)gy * W + gx;
      const float xv = x[off], yv = y[off];
      const float diff = xv - yv;
      const float sgn = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
      dl_dx[off] = (1.f - lambda) * inv_n * sgn + m[0][o] + 2.f * xv * m[1][o] + yv * m[2][o];
    }
  }
  const uint32_t lb = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  if (lb < (uint32_t)nfin)
    loss_final_part(partial, nb, lambda, inv_n, part2, counter, d_loss, (int)lb, nfin, s_red, &s_last);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t loss_workspace_bytes(int c, int h, int w) {
  const size_t nb = (size_t)((w + kTX - 1) / kTX) * ((h + kTY - 1) / kTY) * c;
  return align256((size_t)3 * c * h * w * 4 + nb * 2 * 4) + kFinalBlocks * 2 * 4 + 256;
}

hipError_t launch_loss(const float* x, const float* y, int c, int h, int w, float lambda, float* d_loss,
                       float* dl_dx, void* ws, hipStream_t s) {
  const Window win = gaussian_window();
  const dim3 grid((w + kTX - 1) / kTX, (h + kTY - 1) / kTY, c);
  const int nb = grid.x * grid.y * grid.z;
  float* f3 = static_cast<float*>(ws);
  float* partial = f3 + (size_t)3 * c * h * w;
  char* tail = static_cast<char*>(ws) + align256((size_t)3 * c * h * w * 4 + (size_t)nb * 2 * 4);
  float* part2 = reinterpret_cast<float*>(tail);
  uint32_t* counter = reinterpret_cast<uint32_t*>(tail + kFinalBlocks * 2 * 4);
  const float inv_n = (float)(1.0 / ((double)c * h * w));
  int nfin = (nb + kFinalSlice - 1) / kFinalSlice;
  nfin = nfin < 1 ? 1 : (nfin > kFinalBlocks ? kFinalBlocks : nfin);
  hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, x, y, h, w, win, lambda, inv_n, f3, partial, counter);
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, x, y, h, w, win, lambda, inv_n, f3, dl_dx, partial, nb, nfin,
                     part2, counter, d_loss);
  return hipGetLastError();
}

}  // namespace gs

// ------------------------------------------------ allocation-free entry point
// The scratch of gabsplat_loss_l1_dssim_noalloc (the workspace of launch_loss:
// SSIM maps, per-tile partial sums, completion counter).  The code object
// holds one copy per GPU; in host code `scratch` names no device memory, so
// the host only ever uses the address hipGetSymbolAddress returns for the
// current GPU, looked up once per GPU and kept.
static __device__ __align__(256) unsigned char scratch[GABSPLAT_LOSS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of GPU `dev`'s scratch: looked up with that GPU current the
// first time, then kept.
hipError_t device_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" gabsplat_status gabsplat_loss_l1_dssim_noalloc(const float* x, const float* y, int32_t channels,
                                                          int32_t height, int32_t width, float lambda,
                                                          float* d_loss, float* dl_dx, void* stream) {
  try {
    if (!x || !y || !d_loss || !dl_dx || channels < 1 || height < 1 || width < 1 || height > 65535 * 16 ||
        width > 65535 * 16 || channels > 65535 || !(lambda >= 0.f && lambda <= 1.f))
      return GABSPLAT_ERR_INVALID_ARGUMENT;
    if (gs::loss_workspace_bytes(channels, height, width) > GABSPLAT_LOSS_NOALLOC_SCRATCH_BYTES)
      return GABSPLAT_ERR_SCRATCH_LIMIT;
    GS_REQUIRE_DEVICE();
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    if (hipStreamGetDevice(s, &dev) != hipSuccess) return GABSPLAT_ERR_HIP;
    void* ws = nullptr;
    if (device_scratch(dev, &ws) != hipSuccess) return GABSPLAT_ERR_HIP;
    return gs::launch_loss(x, y, channels, height, width, lambda, d_loss, dl_dx, ws, s) == hipSuccess
               ? GABSPLAT_OK
               : GABSPLAT_ERR_HIP;
  } catch (...) {
    return GABSPLAT_ERR_HIP;
  }
}
