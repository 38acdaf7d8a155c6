// K9: photometric loss (1 - lambda) L1 + lambda (1 - SSIM) and its gradient
// (Sec. 3.4.1, lambda = 0.2).  SSIM uses an 11x11 Gaussian window (sigma 1.5)
// with zero padding; the five local moments are separable filters staged in
// LDS per 16x16 tile.  With A1 = 2 mx my + C1, A2 = 2 sxy + C2,
// B1 = mx^2 + my^2 + C1, B2 = sxx + syy + C2 and s = A1 A2 / (B1 B2):
//   ds/dmx  = s (2 my / A1 - 2 my / A2 - 2 mx / B1 + 2 mx / B2)
//   ds/dExx = -s / B2,   ds/dExy = 2 s / A2
// (Exx, Exy the filtered x^2 and x y), and since the window is symmetric the
// adjoint of each filter is the filter itself:
//   dL/dx = G*(g ds/dmx) + 2 x G*(g ds/dExx) + y G*(g ds/dExy),  g = -lambda / N.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs_internal.h"

namespace gs {

constexpr int kWin = 11;
constexpr int kHalo = 5;
constexpr int kLT = 16;                 // output tile
constexpr int kLS = kLT + 2 * kHalo;    // staged region 26x26

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

// pass 1: moments, SSIM map, per-pixel factors for the backward, partial sums
__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Window win, float lambda, float inv_n,
                                                  float* __restrict__ f3, float* __restrict__ partial) {
  __shared__ float s_x[kLS][kLS], s_y[kLS][kLS];
  __shared__ float s_h[5][kLS][kLT];
  __shared__ float s_red[4];
  const int c = blockIdx.z;
  const int ox = blockIdx.x * kLT, oy = blockIdx.y * kLT;
  const size_t plane = (size_t)H * W;
  const float* xc = x + c * plane;
  const float* yc = y + c * plane;
  for (int i = threadIdx.x; i < kLS * kLS; i += 256) {
    const int r = i / kLS, q = i % kLS;
    const int gy = oy + r - kHalo, gx = ox + q - kHalo;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    s_x[r][q] = in ? xc[(size_t)gy * W + gx] : 0.f;
    s_y[r][q] = in ? yc[(size_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kLS * kLT; i += 256) {
    const int r = i / kLT, q = i % kLT;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      const float xv = s_x[r][q + k], yv = s_y[r][q + k], g = win.g[k];
      a = fmaf(g, xv, a);
      b = fmaf(g, yv, b);
      aa = fmaf(g, xv * xv, aa);
      bb = fmaf(g, yv * yv, bb);
      ab = fmaf(g, xv * yv, ab);
    }
    s_h[0][r][q] = a; s_h[1][r][q] = b; s_h[2][r][q] = aa; s_h[3][r][q] = bb; s_h[4][r][q] = ab;
  }
  __syncthreads();
  const int r = threadIdx.x / kLT, q = threadIdx.x % kLT;
  const int gy = oy + r, gx = ox + q;
  float mx = 0.f, my = 0.f, exx = 0.f, eyy = 0.f, exy = 0.f;
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
    const float g = win.g[k];
    mx = fmaf(g, s_h[0][r + k][q], mx);
    my = fmaf(g, s_h[1][r + k][q], my);
    exx = fmaf(g, s_h[2][r + k][q], exx);
    eyy = fmaf(g, s_h[3][r + k][q], eyy);
    exy = fmaf(g, s_h[4][r + k][q], exy);
  }
  const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
  float ssim = 0.f, l1 = 0.f;
  if (gy < H && gx < W) {
    const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
    const float A1 = 2.f * mx * my + C1, A2 = 2.f * sxy + C2;
    const float B1 = mx * mx + my * my + C1, B2 = sxx + syy + C2;
    const float s = (A1 * A2) / (B1 * B2);
    ssim = s;
    l1 = fabsf(s_x[r + kHalo][q + kHalo] - s_y[r + kHalo][q + kHalo]);
    const float g = -lambda * inv_n;
    const size_t o = c * plane + (size_t)gy * W + gx;
    const size_t nn = plane * gridDim.z;
    f3[o] = g * s * (2.f * my / A1 - 2.f * my / A2 - 2.f * mx / B1 + 2.f * mx / B2);
    f3[nn + o] = g * (-s / B2);
    f3[2 * nn + o] = g * (2.f * s / A2);
  }
  const float ts = block_sum(ssim, s_red);
  const float tl = block_sum(l1, s_red);
  if (threadIdx.x == 0) {
    const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partial[2 * b] = tl;
    partial[2 * b + 1] = ts;
  }
}

// pass 2: filter the three factor maps and combine
__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x, const float* __restrict__ y, int H,
                                                  int W, Window win, float lambda, float inv_n,
                                                  const float* __restrict__ f3, float* __restrict__ dl_dx) {
  __shared__ float s_f[3][kLS][kLS];
  __shared__ float s_h[3][kLS][kLT];
  const int c = blockIdx.z;
  const int ox = blockIdx.x * kLT, oy = blockIdx.y * kLT;
  const size_t plane = (size_t)H * W;
  const size_t nn = plane * gridDim.z;
  for (int i = threadIdx.x; i < kLS * kLS; i += 256) {
    const int r = i / kLS, q = i % kLS;
    const int gy = oy + r - kHalo, gx = ox + q - kHalo;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const size_t o = c * plane + (size_t)gy * W + gx;
    s_f[0][r][q] = in ? f3[o] : 0.f;
    s_f[1][r][q] = in ? f3[nn + o] : 0.f;
    s_f[2][r][q] = in ? f3[2 * nn + o] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kLS * kLT; i += 256) {
    const int r = i / kLT, q = i % kLT;
    float a = 0.f, b = 0.f, d = 0.f;
#pragma unroll
    for (int k = 0; k < kWin; ++k) {
      const float g = win.g[k];
      a = fmaf(g, s_f[0][r][q + k], a);
      b = fmaf(g, s_f[1][r][q + k], b);
      d = fmaf(g, s_f[2][r][q + k], d);
    }
    s_h[0][r][q] = a; s_h[1][r][q] = b; s_h[2][r][q] = d;
  }
  __syncthreads();
  const int r = threadIdx.x / kLT, q = threadIdx.x % kLT;
  const int gy = oy + r, gx = ox + q;
  if (gy >= H || gx >= W) return;
  float a = 0.f, b = 0.f, d = 0.f;
#pragma unroll
  for (int k = 0; k < kWin; ++k) {
    const float g = win.g[k];
    a = fmaf(g, s_h[0][r + k][q], a);
    b = fmaf(g, s_h[1][r + k][q], b);
    d = fmaf(g, s_h[2][r + k][q], d);
  }
  const size_t o = c * plane + (size_t)gy * W + gx;
  const float xv = x[o], yv = y[o];
  const float diff = xv - yv;
  const float sgn = diff > 0.f ? 1.f : (diff < 0.f ? -1.f : 0.f);
  dl_dx[o] = (1.f - lambda) * inv_n * sgn + a + 2.f * xv * b + yv * d;
}

__global__ __launch_bounds__(256) void k_loss_final(const float* __restrict__ partial, int nb, float lambda,
                                                    float inv_n, float* __restrict__ d_loss) {
  __shared__ float s_red[4];
  float l1 = 0.f, ss = 0.f;
  for (int i = threadIdx.x; i < nb; i += 256) {
    l1 += partial[2 * i];
    ss += partial[2 * i + 1];
  }
  l1 = block_sum(l1, s_red);
  ss = block_sum(ss, s_red);
  if (threadIdx.x == 0) *d_loss = (1.f - lambda) * l1 * inv_n + lambda * (1.f - ss * inv_n);
}

size_t loss_workspace_bytes(int c, int h, int w) {
  const size_t nb = (size_t)((w + kLT - 1) / kLT) * ((h + kLT - 1) / kLT) * c;
  return (size_t)3 * c * h * w * 4 + nb * 2 * 4 + 256;
}

hipError_t launch_loss(const float* x, const float* y, int c, int h, int w, float lambda, float* d_loss,
                       float* dl_dx, void* ws, hipStream_t s) {
  const Window win = gaussian_window();
  const dim3 grid((w + kLT - 1) / kLT, (h + kLT - 1) / kLT, c);
  const int nb = grid.x * grid.y * grid.z;
  float* f3 = static_cast<float*>(ws);
  float* partial = f3 + (size_t)3 * c * h * w;
  const float inv_n = (float)(1.0 / ((double)c * h * w));
  hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, x, y, h, w, win, lambda, inv_n, f3, partial);
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, x, y, h, w, win, lambda, inv_n, f3, dl_dx);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, partial, nb, lambda, inv_n, d_loss);
  return hipGetLastError();
}

}  // namespace gs
