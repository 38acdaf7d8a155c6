// K1 (projection of every (view, primitive) item) and K8 (its backward).
//
// Geometry (Sec. 3.1 EWA splatting, Sec. 3.3 frequency projection): with
// T the first two rows of J W and M = R(q) diag(s) (so Sigma = M M^T), the
// rows r0, r1 of A = T M give the raw 2D covariance A A^T = [[r0.r0, r0.r1],
// [r0.r1, r1.r1]] and, by the Lagrange identity, its determinant |r0 x r1|^2
// without cancellation.  The 2D frequency (T Sigma T^T)^-1 T Sigma f is
// evaluated as (v_x . f, v_y . f) with v_x = M (r1 x c) / |c|^2 and
// v_y = M (c x r0) / |c|^2, c = r0 x r1 (the adjugate of A A^T written with
// cross products), so each component costs two dot products.
#include <hip/hip_runtime.h>

#include "gs_internal.h"

namespace gs {

// ---------------------------------------------------------------- helpers
struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ float dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross3(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 add3(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 scale3(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }

// Real spherical harmonics, degree <= 3, ordered l = 0..3, m = -l..l, without
// the Condon-Shortley phase.  Constants are K_l^m (times sqrt 2 for m != 0)
// times the leading factor of d^|m| P_l / dz^|m| for the polynomial written.
constexpr float kY00 = 0.28209479177387814f;
constexpr float kY1 = 0.48860251190291992f;
constexpr float kY2a = 1.0925484305920792f;   // xy, yz, xz
constexpr float kY2b = 0.31539156525252005f;  // 3z^2 - 1
constexpr float kY2c = 0.54627421529603959f;  // x^2 - y^2
constexpr float kY3a = 0.59004358992664352f;  // y(3x^2 - y^2), x(x^2 - 3y^2)
constexpr float kY3b = 2.8906114426405538f;   // xyz
constexpr float kY3c = 0.45704579946446572f;  // y(5z^2 - 1), x(5z^2 - 1)
constexpr float kY3d = 0.37317633259011540f;  // z(5z^2 - 3)
constexpr float kY3e = 1.4453057213202769f;   // z(x^2 - y^2)

__device__ __forceinline__ void sh_basis(float x, float y, float z, int deg, float* Y) {
#pragma unroll
  for (int b = 1; b < 16; ++b) Y[b] = 0.f;
  Y[0] = kY00;
  if (deg < 1) return;
  Y[1] = kY1 * y;
  Y[2] = kY1 * z;
  Y[3] = kY1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kY2a * x * y;
  Y[5] = kY2a * y * z;
  Y[6] = kY2b * (3.0f * zz - 1.0f);
  Y[7] = kY2a * x * z;
  Y[8] = kY2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = kY3a * y * (3.0f * xx - yy);
  Y[10] = kY3b * x * y * z;
  Y[11] = kY3c * y * (5.0f * zz - 1.0f);
  Y[12] = kY3d * z * (5.0f * zz - 3.0f);
  Y[13] = kY3c * x * (5.0f * zz - 1.0f);
  Y[14] = kY3e * z * (xx - yy);
  Y[15] = kY3a * x * (xx - 3.0f * yy);
}

// Ambient gradient of each basis polynomial w.r.t. (x, y, z).
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, int deg, V3* dY) {
#pragma unroll
  for (int b = 0; b < 16; ++b) dY[b] = v3(0.f, 0.f, 0.f);
  if (deg < 1) return;
  dY[1] = v3(0.f, kY1, 0.f);
  dY[2] = v3(0.f, 0.f, kY1);
  dY[3] = v3(kY1, 0.f, 0.f);
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  dY[4] = v3(kY2a * y, kY2a * x, 0.f);
  dY[5] = v3(0.f, kY2a * z, kY2a * y);
  dY[6] = v3(0.f, 0.f, 6.0f * kY2b * z);
  dY[7] = v3(kY2a * z, 0.f, kY2a * x);
  dY[8] = v3(2.0f * kY2c * x, -2.0f * kY2c * y, 0.f);
  if (deg < 3) return;
  dY[9] = v3(6.0f * kY3a * x * y, kY3a * (3.0f * xx - 3.0f * yy), 0.f);
  dY[10] = v3(kY3b * y * z, kY3b * x * z, kY3b * x * y);
  dY[11] = v3(0.f, kY3c * (5.0f * zz - 1.0f), 10.0f * kY3c * y * z);
  dY[12] = v3(0.f, 0.f, kY3d * (15.0f * zz - 3.0f));
  dY[13] = v3(kY3c * (5.0f * zz - 1.0f), 0.f, 10.0f * kY3c * x * z);
  dY[14] = v3(2.0f * kY3e * x * z, -2.0f * kY3e * y * z, kY3e * (xx - yy));
  dY[15] = v3(kY3a * (3.0f * xx - 3.0f * yy), -6.0f * kY3a * x * y, 0.f);
}

// Everything the forward computes for one item, kept for the backward.
struct Geo {
  float tx, ty, tz, inv_tz;
  float ux, uy, uxc, uyc;
  bool clamp_x, clamp_y;
  float a0, a1;        // fx / tz, fy / tz
  V3 T0, T1;           // rows of J W
  float qn[4], qlen;
  float Rq[3][3];
  float s[3];
  V3 r0, r1;           // rows of T M
  float ra, rb, rc;    // raw 2D covariance
  V3 c;                // r0 x r1
  float D;             // |c|^2 = det of the raw covariance
  float det;           // det of the dilated covariance
  float conic[3];
  V3 ux_, uy_;         // r1 x c, c x r0
  V3 vx, vy;           // M ux_ / D, M uy_ / D
  float M[3][3];
};

__device__ __forceinline__ float depth_key(const float* R, const float* t, float x, float y, float z) {
  return __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(R[6], x), __fmul_rn(R[7], y)), __fmul_rn(R[8], z)), t[2]);
}

// Geometry of one item; `tz` is the fp32 depth key, `dil` the px^2 added to
// the 2D covariance (the 0.3 dilation, or the 0.1 anti-aliasing filter).
__device__ __forceinline__ void geometry(const ViewEntry& V, float mx, float my, float mz, float tz,
                                         const float* q, const float* s, float dil, Geo& g) {
  const float* R = V.R;
  g.tx = fmaf(R[0], mx, fmaf(R[1], my, fmaf(R[2], mz, V.t[0])));
  g.ty = fmaf(R[3], mx, fmaf(R[4], my, fmaf(R[5], mz, V.t[1])));
  g.tz = tz;
  g.inv_tz = 1.0f / tz;
  const float Wf = (float)V.width, Hf = (float)V.height;
  const float lox = (-0.15f * Wf - V.cx) / V.fx, hix = (1.15f * Wf - V.cx) / V.fx;
  const float loy = (-0.15f * Hf - V.cy) / V.fy, hiy = (1.15f * Hf - V.cy) / V.fy;
  g.ux = g.tx * g.inv_tz;
  g.uy = g.ty * g.inv_tz;
  g.clamp_x = !(g.ux > lox && g.ux < hix);
  g.clamp_y = !(g.uy > loy && g.uy < hiy);
  g.uxc = fminf(fmaxf(g.ux, lox), hix);
  g.uyc = fminf(fmaxf(g.uy, loy), hiy);
  g.a0 = V.fx * g.inv_tz;
  g.a1 = V.fy * g.inv_tz;
  g.T0 = v3(g.a0 * (R[0] - g.uxc * R[6]), g.a0 * (R[1] - g.uxc * R[7]), g.a0 * (R[2] - g.uxc * R[8]));
  g.T1 = v3(g.a1 * (R[3] - g.uyc * R[6]), g.a1 * (R[4] - g.uyc * R[7]), g.a1 * (R[5] - g.uyc * R[8]));

  const float qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  g.qlen = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  const float iq = 1.0f / g.qlen;
  const float w = qw * iq, x = qx * iq, y = qy * iq, z = qz * iq;
  g.qn[0] = w; g.qn[1] = x; g.qn[2] = y; g.qn[3] = z;
  g.Rq[0][0] = 1.f - 2.f * (y * y + z * z);
  g.Rq[0][1] = 2.f * (x * y - w * z);
  g.Rq[0][2] = 2.f * (x * z + w * y);
  g.Rq[1][0] = 2.f * (x * y + w * z);
  g.Rq[1][1] = 1.f - 2.f * (x * x + z * z);
  g.Rq[1][2] = 2.f * (y * z - w * x);
  g.Rq[2][0] = 2.f * (x * z - w * y);
  g.Rq[2][1] = 2.f * (y * z + w * x);
  g.Rq[2][2] = 1.f - 2.f * (x * x + y * y);
  g.s[0] = s[0]; g.s[1] = s[1]; g.s[2] = s[2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) g.M[i][j] = g.Rq[i][j] * s[j];
  const float T0a[3] = {g.T0.x, g.T0.y, g.T0.z}, T1a[3] = {g.T1.x, g.T1.y, g.T1.z};
  float r0[3], r1[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    r0[j] = T0a[0] * g.M[0][j] + T0a[1] * g.M[1][j] + T0a[2] * g.M[2][j];
    r1[j] = T1a[0] * g.M[0][j] + T1a[1] * g.M[1][j] + T1a[2] * g.M[2][j];
  }
  g.r0 = v3(r0[0], r0[1], r0[2]);
  g.r1 = v3(r1[0], r1[1], r1[2]);
  g.ra = dot3(g.r0, g.r0);
  g.rb = dot3(g.r0, g.r1);
  g.rc = dot3(g.r1, g.r1);
  g.c = cross3(g.r0, g.r1);
  g.D = dot3(g.c, g.c);
  g.det = g.D + dil * (g.ra + g.rc) + dil * dil;
  const float idet = 1.0f / g.det;
  g.conic[0] = (g.rc + dil) * idet;
  g.conic[1] = -g.rb * idet;
  g.conic[2] = (g.ra + dil) * idet;
  g.ux_ = cross3(g.r1, g.c);
  g.uy_ = cross3(g.c, g.r0);
  if (g.D > 0.f) {
    const float iD = 1.0f / g.D;
    g.vx = v3((g.M[0][0] * g.ux_.x + g.M[0][1] * g.ux_.y + g.M[0][2] * g.ux_.z) * iD,
              (g.M[1][0] * g.ux_.x + g.M[1][1] * g.ux_.y + g.M[1][2] * g.ux_.z) * iD,
              (g.M[2][0] * g.ux_.x + g.M[2][1] * g.ux_.y + g.M[2][2] * g.ux_.z) * iD);
    g.vy = v3((g.M[0][0] * g.uy_.x + g.M[0][1] * g.uy_.y + g.M[0][2] * g.uy_.z) * iD,
              (g.M[1][0] * g.uy_.x + g.M[1][1] * g.uy_.y + g.M[1][2] * g.uy_.z) * iD,
              (g.M[2][0] * g.uy_.x + g.M[2][1] * g.uy_.y + g.M[2][2] * g.uy_.z) * iD);
  } else {
    g.vx = v3(0.f, 0.f, 0.f);
    g.vy = v3(0.f, 0.f, 0.f);
  }
}

// Camera-space position of a mean in double precision from the float32
// inputs (the same transform as the depth key, unrounded).
__device__ __forceinline__ void camera_point_f64(const ViewEntry& V, float mx, float my, float mz, double (&t)[3]) {
  const float* R = V.R;
  const double X = mx, Y = my, Z = mz;
  t[0] = (double)R[0] * X + (double)R[1] * Y + (double)R[2] * Z + (double)V.t[0];
  t[1] = (double)R[3] * X + (double)R[4] * Y + (double)R[5] * Z + (double)V.t[1];
  t[2] = (double)R[6] * X + (double)R[7] * Y + (double)R[8] * Z + (double)V.t[2];
}

// The image-plane mean of one item in double precision.  In float32 the mean
// is only held to an ulp of its pixel coordinates (1.2e-4 px near x = 1000),
// which moves alpha by up to ~1e-3 relative at the steep edge of a small
// footprint; the record keeps the mean as a float pair (rounded value +
// residual) and the blend forms the tile-relative offset from both.
__device__ __forceinline__ void precise_mean(const ViewEntry& V, float mx, float my, float mz, double (&mu)[2]) {
  double t[3];
  camera_point_f64(V, mx, my, mz, t);
  const double iz = 1.0 / t[2];
  mu[0] = (double)V.fx * t[0] * iz + (double)V.cx;
  mu[1] = (double)V.fy * t[1] * iz + (double)V.cy;
}

// The frequency basis (v_x, v_y) of geometry() in double precision (the
// camera-space depth unrounded): the frequency dot products v . f cancel in
// float32 to ~1e-5 of their terms, in double they are exact to the final
// rounding.  Returns false when the raw 2D covariance is singular (the
// frequencies are then zero).
__device__ __forceinline__ bool precise_frequency_basis(const ViewEntry& V, float mx, float my, float mz,
                                                        const float* q, const float* s, double (&vx)[3],
                                                        double (&vy)[3]) {
  const float* R = V.R;
  double t[3];
  camera_point_f64(V, mx, my, mz, t);
  const double fx = V.fx, fy = V.fy, cx = V.cx, cy = V.cy;
  const double iz = 1.0 / t[2];
  const double Wd = V.width, Hd = V.height;
  const double uxc = fmin(fmax(t[0] * iz, (-0.15 * Wd - cx) / fx), (1.15 * Wd - cx) / fx);
  const double uyc = fmin(fmax(t[1] * iz, (-0.15 * Hd - cy) / fy), (1.15 * Hd - cy) / fy);
  const double a0 = fx * iz, a1 = fy * iz;
  const double T0[3] = {a0 * (R[0] - uxc * R[6]), a0 * (R[1] - uxc * R[7]), a0 * (R[2] - uxc * R[8])};
  const double T1[3] = {a1 * (R[3] - uyc * R[6]), a1 * (R[4] - uyc * R[7]), a1 * (R[5] - uyc * R[8])};
  const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  const double iq = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw * iq, x = qx * iq, y = qy * iq, z = qz * iq;
  const double Rq[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                           {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                           {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  double M[3][3], r0[3], r1[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = Rq[i][j] * (double)s[j];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    r0[j] = T0[0] * M[0][j] + T0[1] * M[1][j] + T0[2] * M[2][j];
    r1[j] = T1[0] * M[0][j] + T1[1] * M[1][j] + T1[2] * M[2][j];
  }
  const double c[3] = {r0[1] * r1[2] - r0[2] * r1[1], r0[2] * r1[0] - r0[0] * r1[2], r0[0] * r1[1] - r0[1] * r1[0]};
  const double D = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  if (!(D > 0.0)) {
    vx[0] = vx[1] = vx[2] = vy[0] = vy[1] = vy[2] = 0.0;
    return false;
  }
  // r1 x c and c x r0, mapped through M, over |c|^2
  const double ux[3] = {r1[1] * c[2] - r1[2] * c[1], r1[2] * c[0] - r1[0] * c[2], r1[0] * c[1] - r1[1] * c[0]};
  const double uy[3] = {c[1] * r0[2] - c[2] * r0[1], c[2] * r0[0] - c[0] * r0[2], c[0] * r0[1] - c[1] * r0[0]};
  const double iD = 1.0 / D;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vx[i] = (M[i][0] * ux[0] + M[i][1] * ux[1] + M[i][2] * ux[2]) * iD;
    vy[i] = (M[i][0] * uy[0] + M[i][1] * uy[1] + M[i][2] * uy[2]) * iD;
  }
  return true;
}

constexpr float kTwoPiSq = 19.739208802178716f;  // 2 pi^2

__device__ __forceinline__ V3 mat_vec(const float (&M)[3][3], V3 x) {
  return v3(M[0][0] * x.x + M[0][1] * x.y + M[0][2] * x.z, M[1][0] * x.x + M[1][1] * x.y + M[1][2] * x.z,
            M[2][0] * x.x + M[2][1] * x.y + M[2][2] * x.z);
}
__device__ __forceinline__ V3 mat_t_vec(const float (&M)[3][3], V3 x) {
  return v3(M[0][0] * x.x + M[1][0] * x.y + M[2][0] * x.z, M[0][1] * x.x + M[1][1] * x.y + M[2][1] * x.z,
            M[0][2] * x.x + M[1][2] * x.y + M[2][2] * x.z);
}

// Variance along the ray of f . x given the image point: with A = T M and
// c = r0 x r1 spanning A's null space, f^T Sigma f - (T Sigma f)^T (T Sigma
// T^T)^-1 T Sigma f = (M^T f . c)^2 / |c|^2 = (f . M c)^2 / D.  For a
// degenerate 2D footprint (D = 0) the whole f^T Sigma f remains.
__device__ __forceinline__ float ray_variance(const Geo& g, V3 u, V3 f) {
  if (g.D > 0.f) {
    const float s = dot3(f, u);
    return s * s / g.D;
  }
  const V3 mf = mat_t_vec(g.M, f);
  return dot3(mf, mf);
}

// ------------------------------------------------------------------ K1
// Two phases per block of 1024 items.  Phase 1 (every item, coalesced): depth
// key, near and opacity culls, and a conservative screen test: the 2D
// covariance's diagonal is at most |J W|_F^2 max(s)^2 + 0.3 (W orthonormal,
// the largest eigenvalue of Sigma is max(s)^2), so an item whose box of that
// half-width misses the image cannot be visible.  Survivors are compacted in
// LDS so that phase 2 (full EWA projection, SH colour, 2D frequencies, exact
// rect) runs on dense wavefronts instead of wavefronts that are mostly culled.
constexpr int kPreItems = 4;
constexpr int kPreBlock = 256 * kPreItems;

// The scene attributes are device memory, but their pointers come out of the
// view table, so the compiler cannot tell and emits flat loads (64-bit
// addresses, waits on both memory counters).  gptr() states it: global loads.
typedef const __attribute__((address_space(1))) float* gfloat_ptr;
typedef const __attribute__((address_space(1))) float4* gfloat4_ptr;
__device__ __forceinline__ gfloat_ptr gptr(const float* p) { return (gfloat_ptr)p; }

// The nv (<= 48) colour values of primitive i, stored row by row, into
// v[0..nv) (zeros after): 16-byte loads when every row starts on a 16-byte
// boundary, else one float at a time.
template <typename P>
__device__ __forceinline__ void load_colour_row(P base, int64_t i, int nv, float (&v)[48]) {
  const P row = base + i * nv;
  if ((nv & 3) == 0 && (reinterpret_cast<uintptr_t>(base) & 15) == 0) {
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (4 * j < nv) {
        x.x = row[4 * j];
        x.y = row[4 * j + 1];
        x.z = row[4 * j + 2];
        x.w = row[4 * j + 3];
      }
      v[4 * j] = x.x;
      v[4 * j + 1] = x.y;
      v[4 * j + 2] = x.z;
      v[4 * j + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 48; ++j) v[j] = j < nv ? row[j] : 0.f;
  }
}

// The quaternion of primitive i of S: from its row (ROWS, one 16-byte load)
// or its four planes.
template <bool ROWS>
__device__ __forceinline__ void load_quat(const SceneEntry& S, int64_t n, int64_t i, int rs, float (&q)[4]) {
  if constexpr (ROWS) {
    const gfloat_ptr r = gptr(S.rows) + i * rs;  // 16-byte aligned: adjacent loads merge
    q[0] = r[0]; q[1] = r[1]; q[2] = r[2]; q[3] = r[3];
  } else {
    q[0] = gptr(S.quats)[i]; q[1] = gptr(S.quats)[n + i]; q[2] = gptr(S.quats)[2 * n + i];
    q[3] = gptr(S.quats)[3 * n + i];
  }
}

// The frequencies (3K, component-major) then the weights (K) of primitive i
// of S: from its row (ROWS, K 16-byte loads after the quaternion) or the planes.
template <int K, bool ROWS>
__device__ __forceinline__ void load_freq_weights(const SceneEntry& S, int64_t n, int64_t i, int rs,
                                                  float (&fw)[K > 0 ? 4 * K : 1]) {
  if constexpr (ROWS) {
    const gfloat_ptr r = gptr(S.rows) + i * rs + 4;
#pragma unroll
    for (int j = 0; j < 4 * K; ++j) fw[j] = r[j];
  } else {
#pragma unroll
    for (int j = 0; j < 3 * K; ++j) fw[j] = gptr(S.freqs)[(int64_t)j * n + i];
#pragma unroll
    for (int j = 0; j < K; ++j) fw[3 * K + j] = gptr(S.weights)[(int64_t)j * n + i];
  }
}

template <int K, bool ROWS>
__global__ __launch_bounds__(256) void k_preprocess(const void* __restrict__ table,
                                                    float* __restrict__ rec,
                                                    float* __restrict__ depth_out,
                                                    uint32_t* __restrict__ rect_out,
                                                    uint32_t* __restrict__ tiles_out) {
  constexpr int RF = record_stride(K);
  __shared__ uint16_t s_cand[kPreBlock];
  __shared__ uint32_t s_wave[4];
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const ViewEntry& V = table_views(table)[blockIdx.y];
  const SceneEntry& S = table_scenes(table, hdr->num_views)[V.scene];
  const int64_t n = S.n;
  const int64_t base = (int64_t)blockIdx.x * kPreBlock;
  if (base >= n) return;
  const int t = threadIdx.x;
  const float Wf = (float)V.width, Hf = (float)V.height;
  const bool mip3d = (S.flags & GABSPLAT_FLAG_MIP_3D) != 0;
  const bool mip2d = (S.flags & GABSPLAT_FLAG_MIP_2D) != 0;
  const float dil = mip2d ? kMip2dVariance : kDilation;

  // ---- phase 1
  uint32_t cand = 0;
#pragma unroll
  for (int j = 0; j < kPreItems; ++j) {
    const int64_t i = base + j * 256 + t;
    if (i >= n) continue;
    const int64_t item = V.item_offset + i;
    const float mx = gptr(S.means)[i], my = gptr(S.means)[n + i], mz = gptr(S.means)[2 * n + i];
    const float tz = depth_key(V.R, V.t, mx, my, mz);
    depth_out[item] = tz;
    const float o = gptr(S.opac)[i];
    bool ok = (tz > V.near_plane) && (o * 255.0f > 1.0f);
    if (ok) {
      float smax = fmaxf(fmaxf(gptr(S.scales)[i], gptr(S.scales)[n + i]), gptr(S.scales)[2 * n + i]);
      if (mip3d) smax = sqrtf(fmaf(smax, smax, gptr(S.filter3d)[i]));
      const float* R = V.R;
      const float tx = fmaf(R[0], mx, fmaf(R[1], my, fmaf(R[2], mz, V.t[0])));
      const float ty = fmaf(R[3], mx, fmaf(R[4], my, fmaf(R[5], mz, V.t[1])));
      const float iz = 1.0f / tz;
      const float mux = fmaf(V.fx * tx, iz, V.cx), muy = fmaf(V.fy * ty, iz, V.cy);
      const float lox = (-0.15f * Wf - V.cx) / V.fx, hix = (1.15f * Wf - V.cx) / V.fx;
      const float loy = (-0.15f * Hf - V.cy) / V.fy, hiy = (1.15f * Hf - V.cy) / V.fy;
      const float ux = fminf(fmaxf(tx * iz, lox), hix), uy = fminf(fmaxf(ty * iz, loy), hiy);
      const float a0 = V.fx * iz, a1 = V.fy * iz;
      const float jf2 = a0 * a0 * (1.0f + ux * ux) + a1 * a1 * (1.0f + uy * uy);
      const float kk = sqrtf(fmaxf(2.0f * kLn2 * log2f(255.0f * o), 0.0f));
      const float rb = 1.01f * kk * sqrtf(jf2 * smax * smax + dil) + 1.0f;
      // also keep anything whose numbers are not finite: phase 2 decides
      ok = !(mux + rb < 0.0f || mux - rb > Wf || muy + rb < 0.0f || muy - rb > Hf);
    }
    if (ok) {
      cand |= 1u << j;
    } else {
      reinterpret_cast<uint2*>(rect_out)[item] = make_uint2(0u, 0u);
      tiles_out[item] = 0;
    }
  }
  // ---- compact the candidates of the block (order does not matter)
  uint32_t nc = (uint32_t)__popc(cand);
  const int w = t >> 6, l = t & 63;
  uint32_t inc = nc;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, 64);
    if (l >= d) inc += o;
  }
  if (l == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t off = 0, total = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    off += (q < w) ? s_wave[q] : 0u;
    total += s_wave[q];
  }
  uint32_t pos = off + inc - nc;
#pragma unroll
  for (int j = 0; j < kPreItems; ++j)
    if ((cand >> j) & 1u) s_cand[pos++] = (uint16_t)(j * 256 + t);
  __syncthreads();

  // ---- phase 2
  for (uint32_t c = t; c < total; c += 256) {
    const int64_t i = base + s_cand[c];
    const int64_t item = V.item_offset + i;
    const float mx = gptr(S.means)[i], my = gptr(S.means)[n + i], mz = gptr(S.means)[2 * n + i];
    const float tz = depth_out[item];
    const float o = gptr(S.opac)[i];
    float q[4];
    load_quat<ROWS>(S, n, i, row_stride(K), q);
    float sc[3] = {gptr(S.scales)[i], gptr(S.scales)[n + i], gptr(S.scales)[2 * n + i]};
    // filtered envelope: scales sqrt(s^2 + v), opacity times prod s / sqrt(s^2 + v)
    float oe = o;
    if (mip3d) {
      const float fv = gptr(S.filter3d)[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float sf = sqrtf(fmaf(sc[j], sc[j], fv));
        oe *= sc[j] / sf;
        sc[j] = sf;
      }
    }
    Geo g;
    geometry(V, mx, my, mz, tz, q, sc, dil, g);
    if (mip2d) oe *= sqrtf(fmaxf(g.D / g.det, kMip2dMinRatio));
    // compiler-only barriers around the double-precision part: the loads of
    // the frequencies, weights and colour row stay after it instead of being
    // hoisted above it, which keeps the kernel within 128 VGPRs (four
    // wavefronts per SIMD, the whole grid resident at once; 147 VGPRs and
    // three wavefronts without them)
    asm volatile("" ::: "memory");
    double mu_d[2];
    precise_mean(V, mx, my, mz, mu_d);
    const float mux = (float)mu_d[0], muy = (float)mu_d[1];
    const float mux_lo = (float)(mu_d[0] - (double)mux), muy_lo = (float)(mu_d[1] - (double)muy);
    // exact support of o G >= 1/255: d^T C d <= 2 ln(255 o)
    const float kk = sqrtf(fmaxf(2.0f * kLn2 * log2f(255.0f * oe), 0.0f));
    const float rx = kk * sqrtf(g.ra + dil), ry = kk * sqrtf(g.rc + dil);
    const float px0 = fmaxf(ceilf(mux - rx - 0.5f), 0.0f);
    const float px1 = fminf(floorf(mux + rx - 0.5f), (float)(V.width - 1));
    const float py0 = fmaxf(ceilf(muy - ry - 0.5f), 0.0f);
    const float py1 = fminf(floorf(muy + ry - 0.5f), (float)(V.height - 1));
    const bool vis = (g.det > 0.f) && (px0 <= px1) && (py0 <= py1) && (oe * 255.0f > 1.0f);
    uint2 rect = make_uint2(0u, 0u);
    uint32_t ntiles = 0;
    if (vis) {
      const uint32_t x0 = (uint32_t)px0 >> 4, x1 = ((uint32_t)px1 >> 4) + 1;
      const uint32_t y0 = (uint32_t)py0 >> 4, y1 = ((uint32_t)py1 >> 4) + 1;
      rect = make_uint2(x0 | (y0 << 16), x1 | (y1 << 16));
      ntiles = (x1 - x0) * (y1 - y0);
      float r[RF];
      r[0] = mux;
      r[1] = muy;
      r[record_mean_lo(K)] = mux_lo;
      r[record_mean_lo(K) + 1] = muy_lo;
      r[2] = -0.5f * kLog2e * g.conic[0];
      r[3] = -kLog2e * g.conic[1];
      r[4] = -0.5f * kLog2e * g.conic[2];
      r[5] = log2f(oe);
      // frequencies first: their double-precision basis is dead before the colour row is loaded
      float wsum = 0.f;
      const bool atten = (S.flags & GABSPLAT_FLAG_ATTENUATION) != 0;
      const V3 u = mat_vec(g.M, g.c);
      double vx_d[3], vy_d[3];
      precise_frequency_basis(V, mx, my, mz, q, sc, vx_d, vy_d);
      asm volatile("" ::: "memory");
      float fw[K > 0 ? 4 * K : 1];
      load_freq_weights<K, ROWS>(S, n, i, row_stride(K), fw);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const V3 f = v3(fw[3 * k], fw[3 * k + 1], fw[3 * k + 2]);
        const float wk = fw[3 * K + k];
        r[10 + 3 * k] = (float)(vx_d[0] * f.x + vx_d[1] * f.y + vx_d[2] * f.z);
        r[11 + 3 * k] = (float)(vy_d[0] * f.x + vy_d[1] * f.y + vy_d[2] * f.z);
        r[12 + 3 * k] = atten ? wk * __expf(-kTwoPiSq * ray_variance(g, u, f)) : wk;
        wsum += wk;
      }
      r[9] = 1.0f - wsum;
      if (S.sh_degree >= 0) {
        const V3 d = v3(mx - V.campos[0], my - V.campos[1], mz - V.campos[2]);
        const float il = 1.0f / sqrtf(dot3(d, d));
        float Y[16];
        const int deg = S.sh_degree;
        sh_basis(d.x * il, d.y * il, d.z * il, deg, Y);
        const int nd = (deg + 1) * (deg + 1);
        float shv[48];
        load_colour_row(gptr(S.sh), i, 3 * nd, shv);
        float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
        for (int b = 0; b < 16; ++b) {  // compile-time bound keeps Y in registers
          if (b < nd) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) col[ch] = fmaf(Y[b], shv[b * 3 + ch], col[ch]);
          }
        }
        r[6] = fmaxf(col[0], 0.f);
        r[7] = fmaxf(col[1], 0.f);
        r[8] = fmaxf(col[2], 0.f);
      } else {
        r[6] = gptr(S.colors)[3 * i];
        r[7] = gptr(S.colors)[3 * i + 1];
        r[8] = gptr(S.colors)[3 * i + 2];
      }
#pragma unroll
      for (int jj = record_mean_lo(K) + 2; jj < RF; ++jj) r[jj] = 0.f;
      float4* dst = reinterpret_cast<float4*>(rec + item * RF);
#pragma unroll
      for (int jj = 0; jj < RF / 4; ++jj) dst[jj] = make_float4(r[4 * jj], r[4 * jj + 1], r[4 * jj + 2], r[4 * jj + 3]);
    }
    reinterpret_cast<uint2*>(rect_out)[item] = rect;
    tiles_out[item] = ntiles;
  }
}

// ------------------------------------------------------------------ K8
// Two kernels run one after the other over the primitives of scene
// `scene_index`, 256 per block: the geometry part (mean through the
// projection, scale, rotation, opacity, frequencies, weights) and the colour
// part (SH or RGB coefficients, plus the view-direction term of the mean
// gradient, added to what the geometry part wrote).  A block stages the
// attributes of its primitives that some view sees into LDS rows (from the
// planar arrays, loads of consecutive primitives of one plane per
// instruction; from the colour arrays, each primitive's own row), runs the
// chain rule once per such primitive over its views (deterministic
// accumulation, no atomics), puts the gradients back into the same row and
// writes the gradients of all 256 primitives out at once -- plane by plane,
// or as the one contiguous run of colour rows -- with zeros for the
// primitives no view sees, unless accumulating.
constexpr int kBwdBlock = 256;

// Geometry row: mean 3, scale 3, quaternion 4, opacity 1, frequencies 3K, weights K
template <int K>
struct GeoRow {
  static constexpr int NP = 11 + 4 * K;  // odd for every K: conflict-free LDS rows
};

template <int K>
__device__ __forceinline__ const float* geo_src(const SceneEntry& S, int p) {
  if (p < 3) return S.means + (int64_t)p * S.n;
  if (p < 6) return S.scales + (int64_t)(p - 3) * S.n;
  if (p < 10) return S.quats + (int64_t)(p - 6) * S.n;
  if (p < 11) return S.opac;
  if (p < 11 + 3 * K) return S.freqs + (int64_t)(p - 11) * S.n;
  return S.weights + (int64_t)(p - 11 - 3 * K) * S.n;
}

template <int K>
__device__ __forceinline__ float* geo_dst(const gabsplat_scene_grads& gr, int64_t n, int p) {
  if (p < 3) return gr.means ? gr.means + (int64_t)p * n : nullptr;
  if (p < 6) return gr.scales ? gr.scales + (int64_t)(p - 3) * n : nullptr;
  if (p < 10) return gr.quats ? gr.quats + (int64_t)(p - 6) * n : nullptr;
  if (p < 11) return gr.opacities;
  if (p < 11 + 3 * K) return gr.freqs ? gr.freqs + (int64_t)(p - 11) * n : nullptr;
  return gr.weights ? gr.weights + (int64_t)(p - 11 - 3 * K) * n : nullptr;
}

// Chain rule of the geometry part for primitive i, parameters in row P (LDS);
// the gradients replace them in the same layout.  grad2d rows are `gstride`
// floats apart; the first round_up(10 + 3K, 4) are read.  FILT compiles in
// the anti-aliasing filters (flags GABSPLAT_FLAG_MIP_*), so that the plain
// variant keeps its register budget.
template <int K, bool FILT>
__device__ __forceinline__ void geo_bwd_one(const void* __restrict__ table, int scene_index,
                                            const uint32_t* __restrict__ tiles, const float* __restrict__ depth,
                                            const float* __restrict__ grad2d, int gstride, int64_t i, float* P) {
  constexpr int GF = (10 + 3 * K + 3) & ~3;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const int nv = hdr->num_views;
  const ViewEntry* views = table_views(table);
  const SceneEntry& S = table_scenes(table, nv)[scene_index];
  const float mx = P[0], my = P[1], mz = P[2];
  const float s_in[3] = {P[3], P[4], P[5]};
  const float q[4] = {P[6], P[7], P[8], P[9]};
  const float o = P[10];
  const bool mip3d = FILT && (S.flags & GABSPLAT_FLAG_MIP_3D) != 0;
  const bool mip2d = FILT && (S.flags & GABSPLAT_FLAG_MIP_2D) != 0;
  const float dil = mip2d ? kMip2dVariance : kDilation;
  // scales the projection sees (filtered: sqrt(s^2 + v))
  const float fv = mip3d ? S.filter3d[i] : 0.f;
  float s[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) s[j] = mip3d ? sqrtf(fmaf(s_in[j], s_in[j], fv)) : s_in[j];
  float g5 = 0.f;  // sum over views of dL/d rec[5]

  V3 gmean = v3(0.f, 0.f, 0.f);
  float gs[3] = {0.f, 0.f, 0.f};
  float gq[4] = {0.f, 0.f, 0.f, 0.f};
  float go = 0.f;
  V3 gf[K > 0 ? K : 1];
  float gw[K > 0 ? K : 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    gf[k] = v3(0.f, 0.f, 0.f);
    gw[k] = 0.f;
  }
  for (int v = 0; v < nv; ++v) {
    const ViewEntry& V = views[v];
    if (V.scene != scene_index) continue;
    const int64_t item = V.item_offset + i;
    if (tiles[item] == 0) continue;
    const float* g2 = grad2d + item * (int64_t)gstride;
    float G2[GF];
#pragma unroll
    for (int j = 0; j < GF / 4; ++j) {
      const float4 t4 = reinterpret_cast<const float4*>(g2)[j];
      G2[4 * j] = t4.x; G2[4 * j + 1] = t4.y; G2[4 * j + 2] = t4.z; G2[4 * j + 3] = t4.w;
    }
    Geo g;
    geometry(V, mx, my, mz, depth[item], q, s, dil, g);

    // ---- opacity: rec[5] = log2(o) [+ sum_j log2(s_j / s'_j)] [+ log2 of the 2D factor]
    go += G2[5] / (o * kLn2);
    g5 += G2[5];

    // ---- conic record terms -> dilated covariance (a, b, c)
    const float dQ00 = -0.5f * kLog2e * G2[2];
    const float dQ01 = -kLog2e * G2[3];
    const float dQ11 = -0.5f * kLog2e * G2[4];
    const float ca = g.ra + dil, cb = g.rb, cc = g.rc + dil;
    const float id2 = 1.0f / (g.det * g.det);
    float dra = (-cc * cc * dQ00 + cb * cc * dQ01 - cb * cb * dQ11) * id2;
    float drc = (-cb * cb * dQ00 + ca * cb * dQ01 - ca * ca * dQ11) * id2;
    float drb = (2.f * cb * cc * dQ00 - (ca * cc + cb * cb) * dQ01 + 2.f * ca * cb * dQ11) * id2;
    // 2D filter factor: rec[5] += log2(D / det) / 2 with D = ra rc - rb^2 and
    // det = ca cc - rb^2 (a floored ratio has zero derivative)
    if (mip2d && g.D / g.det > kMip2dMinRatio) {
      const float c5 = 0.5f * G2[5] * kLog2e;
      const float iD = 1.0f / g.D, idt = 1.0f / g.det;
      dra += c5 * (g.rc * iD - cc * idt);
      drc += c5 * (g.ra * iD - ca * idt);
      drb += c5 * 2.f * g.rb * (idt - iD);
    }
    V3 gr0 = add3(scale3(g.r0, 2.f * dra), scale3(g.r1, drb));
    V3 gr1 = add3(scale3(g.r1, 2.f * drc), scale3(g.r0, drb));
    float gM[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) gM[a][b] = 0.f;

    // ---- 2D frequencies f2d_k = (vx . f_k, vy . f_k) and cosine weights
    // record weight w'_k = w_k a_k (a_k = exp(-2 pi^2 v_k) or 1), DC weight 1 - sum w
    const bool atten = (S.flags & GABSPLAT_FLAG_ATTENUATION) != 0;
    const V3 u = mat_vec(g.M, g.c);
    V3 gu = v3(0.f, 0.f, 0.f);
    float gD_att = 0.f;
    V3 gvx = v3(0.f, 0.f, 0.f), gvy = v3(0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const V3 f = v3(P[11 + 3 * k], P[12 + 3 * k], P[13 + 3 * k]);
      const float gx = G2[10 + 3 * k], gy = G2[11 + 3 * k], gwr = G2[12 + 3 * k];
      gvx = add3(gvx, scale3(f, gx));
      gvy = add3(gvy, scale3(f, gy));
      gf[k] = add3(gf[k], add3(scale3(g.vx, gx), scale3(g.vy, gy)));
      if (atten) {
        const float wk = P[11 + 3 * K + k];
        const float v = ray_variance(g, u, f);
        const float a = __expf(-kTwoPiSq * v);
        gw[k] += gwr * a - G2[9];
        const float gv_ = -kTwoPiSq * a * wk * gwr;  // dL/dv_k
        if (g.D > 0.f) {
          const float sdot = dot3(f, u);
          const float c2 = 2.f * sdot / g.D * gv_;
          gf[k] = add3(gf[k], scale3(u, c2));
          gu = add3(gu, scale3(f, c2));
          gD_att += -gv_ * v / g.D;
        } else {
          // v = |M^T f|^2: dv/df = 2 M M^T f, dv/dM = 2 f (M^T f)^T
          const V3 mf = mat_t_vec(g.M, f);
          gf[k] = add3(gf[k], scale3(mat_vec(g.M, mf), 2.f * gv_));
          const float fa[3] = {f.x, f.y, f.z}, ma[3] = {mf.x, mf.y, mf.z};
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2)
#pragma unroll
            for (int b2 = 0; b2 < 3; ++b2) gM[a2][b2] += 2.f * gv_ * fa[a2] * ma[b2];
        }
      } else {
        gw[k] += gwr - G2[9];
      }
    }
    if (K > 0 && g.D > 0.f) {
      const float iD = 1.0f / g.D;
      const float gvxa[3] = {gvx.x, gvx.y, gvx.z}, gvya[3] = {gvy.x, gvy.y, gvy.z};
      const float uxa[3] = {g.ux_.x, g.ux_.y, g.ux_.z}, uya[3] = {g.uy_.x, g.uy_.y, g.uy_.z};
      const float gua[3] = {gu.x, gu.y, gu.z}, ca[3] = {g.c.x, g.c.y, g.c.z};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) gM[a][b] += (gvxa[a] * uxa[b] + gvya[a] * uya[b]) * iD + gua[a] * ca[b];
      // M^T gvx / D, M^T gvy / D
      const V3 gux = scale3(mat_t_vec(g.M, gvx), iD);
      const V3 guy = scale3(mat_t_vec(g.M, gvy), iD);
      const float gD = -(dot3(g.vx, gvx) + dot3(g.vy, gvy)) * iD + gD_att;
      // ux_ = r1 x c ; uy_ = c x r0 ; u = M c ; D = c.c ; c = r0 x r1
      V3 gc = mat_t_vec(g.M, gu);
      gr1 = add3(gr1, cross3(g.c, gux));
      gc = add3(gc, cross3(gux, g.r1));
      gc = add3(gc, cross3(g.r0, guy));
      gr0 = add3(gr0, cross3(guy, g.c));
      gc = add3(gc, scale3(g.c, 2.f * gD));
      gr0 = add3(gr0, cross3(g.r1, gc));
      gr1 = add3(gr1, cross3(gc, g.r0));
    }

    // ---- A = T M: rows r0 = T0 M, r1 = T1 M
    const float T0a[3] = {g.T0.x, g.T0.y, g.T0.z}, T1a[3] = {g.T1.x, g.T1.y, g.T1.z};
    const float gr0a[3] = {gr0.x, gr0.y, gr0.z}, gr1a[3] = {gr1.x, gr1.y, gr1.z};
    float gT0[3], gT1[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      gT0[l] = gr0a[0] * g.M[l][0] + gr0a[1] * g.M[l][1] + gr0a[2] * g.M[l][2];
      gT1[l] = gr1a[0] * g.M[l][0] + gr1a[1] * g.M[l][1] + gr1a[2] * g.M[l][2];
#pragma unroll
      for (int j = 0; j < 3; ++j) gM[l][j] += T0a[l] * gr0a[j] + T1a[l] * gr1a[j];
    }
    // ---- M = Rq diag(s)
    float gR[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) gR[a][b] = gM[a][b] * s[b];
#pragma unroll
    for (int b = 0; b < 3; ++b) gs[b] += gM[0][b] * g.Rq[0][b] + gM[1][b] * g.Rq[1][b] + gM[2][b] * g.Rq[2][b];
    {
      const float w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
      float gqn[4];
      gqn[0] = 2.f * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
      gqn[1] = 2.f * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - w * gR[1][2] + z * gR[2][0] + w * gR[2][1]) -
               4.f * x * (gR[1][1] + gR[2][2]);
      gqn[2] = 2.f * (x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] - w * gR[2][0] + z * gR[2][1]) -
               4.f * y * (gR[0][0] + gR[2][2]);
      gqn[3] = 2.f * (-w * gR[0][1] + x * gR[0][2] + w * gR[1][0] + y * gR[1][2] + x * gR[2][0] + y * gR[2][1]) -
               4.f * z * (gR[0][0] + gR[1][1]);
      const float pr = gqn[0] * w + gqn[1] * x + gqn[2] * y + gqn[3] * z;
      const float il = 1.0f / g.qlen;
      gq[0] += (gqn[0] - w * pr) * il;
      gq[1] += (gqn[1] - x * pr) * il;
      gq[2] += (gqn[2] - y * pr) * il;
      gq[3] += (gqn[3] - z * pr) * il;
    }
    // ---- T = J2 R (depends on t through tz and the clamped ratios)
    const float* R = V.R;
    float gtx = 0.f, gty = 0.f, gtz = 0.f;
    {
      const float ga0 = (gT0[0] * g.T0.x + gT0[1] * g.T0.y + gT0[2] * g.T0.z) / g.a0;
      const float ga1 = (gT1[0] * g.T1.x + gT1[1] * g.T1.y + gT1[2] * g.T1.z) / g.a1;
      const float guxc = -g.a0 * (gT0[0] * R[6] + gT0[1] * R[7] + gT0[2] * R[8]);
      const float guyc = -g.a1 * (gT1[0] * R[6] + gT1[1] * R[7] + gT1[2] * R[8]);
      gtz += -(ga0 * g.a0 + ga1 * g.a1) * g.inv_tz;
      if (!g.clamp_x) {
        gtx += guxc * g.inv_tz;
        gtz += -guxc * g.ux * g.inv_tz;
      }
      if (!g.clamp_y) {
        gty += guyc * g.inv_tz;
        gtz += -guyc * g.uy * g.inv_tz;
      }
    }
    // ---- mu2d = (fx tx / tz + cx, fy ty / tz + cy)
    gtx += V.fx * g.inv_tz * G2[0];
    gty += V.fy * g.inv_tz * G2[1];
    gtz += -(V.fx * g.tx * G2[0] + V.fy * g.ty * G2[1]) * g.inv_tz * g.inv_tz;
    // ---- t = R mu + t0
    gmean = add3(gmean, v3(R[0] * gtx + R[3] * gty + R[6] * gtz, R[1] * gtx + R[4] * gty + R[7] * gtz,
                           R[2] * gtx + R[5] * gty + R[8] * gtz));
  }
  P[0] = gmean.x; P[1] = gmean.y; P[2] = gmean.z;
  if (mip3d) {
    // s' = sqrt(s^2 + v): ds'/ds = s / s'; the opacity factor adds
    // d/ds log2(s / s') = v / (ln 2 s s'^2) per unit of rec[5]
#pragma unroll
    for (int j = 0; j < 3; ++j) P[3 + j] = gs[j] * (s_in[j] / s[j]) + g5 * kLog2e * fv / (s_in[j] * s[j] * s[j]);
  } else {
    P[3] = gs[0]; P[4] = gs[1]; P[5] = gs[2];
  }
  P[6] = gq[0]; P[7] = gq[1]; P[8] = gq[2]; P[9] = gq[3];
  P[10] = go;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    P[11 + 3 * k] = gf[k].x;
    P[12 + 3 * k] = gf[k].y;
    P[13 + 3 * k] = gf[k].z;
    P[11 + 3 * K + k] = gw[k];
  }
}

// Colour part for primitive i of a scene with SH degree DEG (-1: RGB), mean
// m and colour coefficients shv (SH [(DEG+1)^2][3] or RGB 3, zeros after):
// adds the coefficient gradients of every view that sees it to g[0..) (an
// LDS row, which keeps them out of the register budget) and returns the
// view-direction term of the mean gradient.
template <int DEG>
__device__ __forceinline__ V3 colour_bwd_one(const void* __restrict__ table, int scene_index,
                                             const uint32_t* __restrict__ tiles, const float* __restrict__ grad2d,
                                             int gf_stride, int64_t i, V3 m, const float (&shv)[48], float* g) {
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const int nv = hdr->num_views;
  const ViewEntry* views = table_views(table);
  constexpr int nd = DEG >= 0 ? (DEG + 1) * (DEG + 1) : 0;
  V3 gmean = v3(0.f, 0.f, 0.f);
  for (int v = 0; v < nv; ++v) {
    const ViewEntry& V = views[v];
    if (V.scene != scene_index) continue;
    const int64_t item = V.item_offset + i;
    if (tiles[item] == 0) continue;
    const float* g2 = grad2d + item * (int64_t)gf_stride;
    const float G2c[3] = {g2[6], g2[7], g2[8]};
    if constexpr (DEG >= 0) {
      const V3 d = v3(m.x - V.campos[0], m.y - V.campos[1], m.z - V.campos[2]);
      const float il = 1.0f / sqrtf(dot3(d, d));
      const V3 dir = scale3(d, il);
      float Y[16];
      V3 dY[16];
      sh_basis(dir.x, dir.y, dir.z, DEG, Y);
      sh_basis_grad(dir.x, dir.y, dir.z, DEG, dY);
      float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
      for (int b = 0; b < nd; ++b)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) col[ch] = fmaf(Y[b], shv[b * 3 + ch], col[ch]);
      float drgb[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) drgb[ch] = col[ch] < 0.f ? 0.f : G2c[ch];
      V3 gdir = v3(0.f, 0.f, 0.f);
#pragma unroll
      for (int b = 0; b < nd; ++b) {
        float acc = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          g[b * 3 + ch] += Y[b] * drgb[ch];
          acc += shv[b * 3 + ch] * drgb[ch];
        }
        gdir = add3(gdir, scale3(dY[b], acc));
      }
      const float pr = dot3(dir, gdir);
      gmean = add3(gmean, scale3(add3(gdir, scale3(dir, -pr)), il));
    } else {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) g[ch] += G2c[ch];
    }
  }
  return gmean;
}

template <int K, bool FILT>
__global__ __launch_bounds__(kBwdBlock) void k_preprocess_bwd(const void* __restrict__ table, int scene_index,
                                                              const uint32_t* __restrict__ tiles,
                                                              const float* __restrict__ depth,
                                                              const float* __restrict__ grad2d,
                                                              gabsplat_scene_grads gr,
                                                              const int32_t* __restrict__ d_overflow) {
  constexpr int PITCH = GeoRow<K>::NP;
  const int gstride = grad2d_stride(K, gr.flags);
  __shared__ float s_row[kBwdBlock * PITCH];
  __shared__ int16_t s_prim[kBwdBlock];
  __shared__ uint32_t s_wave[kBwdBlock / 64];
  if (d_overflow != nullptr && *d_overflow != 0) return;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const int nv = hdr->num_views;
  const ViewEntry* views = table_views(table);
  const SceneEntry& S = table_scenes(table, nv)[scene_index];
  const int64_t n = S.n;
  const int64_t base = (int64_t)blockIdx.x * kBwdBlock;
  if (base >= n) return;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int64_t i = base + t;
  const bool in = i < n;
  bool vis = false;
  for (int v = 0; v < nv && in && !vis; ++v)
    vis = views[v].scene == scene_index && tiles[views[v].item_offset + i] != 0;
  // slot of a visible primitive among the block's visible ones (in order)
  const uint64_t bal = __ballot(vis);
  const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
  if (l == 0) s_wave[w] = (uint32_t)__popcll(bal);
  __syncthreads();
  int before = 0, count = 0;
#pragma unroll
  for (int q = 0; q < kBwdBlock / 64; ++q) {
    before += q < w ? (int)s_wave[q] : 0;
    count += (int)s_wave[q];
  }
  const int slot = vis ? before + __popcll(bal & lt) : -1;
  const bool acc = gr.accumulate != 0;
  if (count == 0 && acc) return;
  if (count > 0) {
    if (vis) {
      s_prim[slot] = (int16_t)t;
      float* row = s_row + slot * PITCH;
      // every load of the row is issued before the first LDS store
      float v[GeoRow<K>::NP];
#pragma unroll
      for (int p = 0; p < GeoRow<K>::NP; ++p) v[p] = geo_src<K>(S, p)[i];
#pragma unroll
      for (int p = 0; p < GeoRow<K>::NP; ++p) row[p] = v[p];
    }
    __syncthreads();
    if (t < count) geo_bwd_one<K, FILT>(table, scene_index, tiles, depth, grad2d, gstride, base + s_prim[t],
                                        s_row + t * PITCH);
    __syncthreads();
  }
  if (!in) return;
  // gradient planes, one plane per step over the block's 256 primitives
  const float* row = s_row + (slot >= 0 ? slot : 0) * PITCH;
#pragma unroll
  for (int p = 0; p < GeoRow<K>::NP; ++p) {
    float* d = geo_dst<K>(gr, n, p);
    if (d == nullptr) continue;
    if (acc) {
      if (vis) d[i] += row[p];
    } else {
      d[i] = vis ? row[p] : 0.f;
    }
  }
}

// The colour part: one wavefront per 64 consecutive primitives, one lane per
// primitive.  Visible lanes read their own colour row (the colour arrays hold
// one row per primitive), run the chain rule and leave the gradient row in
// LDS; the wavefront then writes its 64 rows -- one contiguous run -- with
// consecutive lanes on consecutive float4s, or floats where rows are not whole
// float4s (zeros for the primitives no view sees, unless accumulating).
constexpr int kColBlock = 64;

template <int DEG>
__global__ __launch_bounds__(kColBlock) void k_colour_bwd(const void* __restrict__ table, int scene_index,
                                                          const uint32_t* __restrict__ tiles,
                                                          const float* __restrict__ grad2d, gabsplat_scene_grads gr,
                                                          int gstride, const int32_t* __restrict__ d_overflow) {
  constexpr int NC = DEG >= 0 ? (DEG + 1) * (DEG + 1) * 3 : 3;  // colour values per primitive
  __shared__ __align__(16) float s_g[kColBlock * NC];
  if (d_overflow != nullptr && *d_overflow != 0) return;
  const ViewTableHeader* hdr = reinterpret_cast<const ViewTableHeader*>(table);
  const int nv = hdr->num_views;
  const ViewEntry* views = table_views(table);
  const SceneEntry& S = table_scenes(table, nv)[scene_index];
  const int64_t n = S.n;
  const int64_t base = (int64_t)blockIdx.x * kColBlock;
  const int l = threadIdx.x;
  const int64_t i = base + l;
  bool vis = false;
  for (int v = 0; v < nv && i < n && !vis; ++v)
    vis = views[v].scene == scene_index && tiles[views[v].item_offset + i] != 0;
  const uint64_t vmask = __ballot(vis);
  const bool acc = gr.accumulate != 0;
  if (vmask == 0 && acc) return;
  float* cd = DEG >= 0 ? gr.sh : gr.colors;
  if (vis) {
    float v[48];
    load_colour_row(DEG >= 0 ? S.sh : S.colors, i, NC, v);
    const V3 m = v3(S.means[i], S.means[n + i], S.means[2 * n + i]);
    float* g = s_g + l * NC;
#pragma unroll
    for (int a = 0; a < NC; ++a) g[a] = 0.f;
    const V3 gm = colour_bwd_one<DEG>(table, scene_index, tiles, grad2d, gstride, i, m, v, g);
    if (gr.means) {  // after the geometry part has written the mean gradient
      gr.means[i] += gm.x;
      gr.means[n + i] += gm.y;
      gr.means[2 * n + i] += gm.z;
    }
  }
  __syncthreads();
  if (cd == nullptr) return;
  const int cnt = (int)(n - base < kColBlock ? n - base : kColBlock);
  float* dst = cd + base * NC;
  if constexpr (NC % 4 == 0) {
    // rows of whole float4s (SH degree 1 or 3): the run as float4s, a quarter
    // of the store instructions (the run starts on a 16-byte boundary when
    // the array does, as base * NC floats is a multiple of 4)
    if ((reinterpret_cast<uintptr_t>(cd) & 15) == 0) {
      constexpr int NC4 = NC / 4;
      float4* d4 = reinterpret_cast<float4*>(dst);
      const float4* g4 = reinterpret_cast<const float4*>(s_g);
#pragma unroll
      for (int j = 0; j < NC4; ++j) {
        const int e = j * kColBlock + l;  // float4 e of the run: primitive e / NC4
        const int p = e / NC4;
        if (p < cnt) {
          const bool pv = (vmask >> p) & 1ull;
          if (acc) {
            if (pv) {
              float4 a = d4[e];
              const float4 q = g4[e];
              a.x += q.x;
              a.y += q.y;
              a.z += q.z;
              a.w += q.w;
              d4[e] = a;
            }
          } else {
            d4[e] = pv ? g4[e] : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
      }
      return;
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int e = j * kColBlock + l;  // float e of the run: primitive e / NC, value e % NC
    const int p = e / NC;
    if (p < cnt) {
      const bool pv = (vmask >> p) & 1ull;
      if (acc) {
        if (pv) dst[e] += s_g[e];
      } else {
        dst[e] = pv ? s_g[e] : 0.f;
      }
    }
  }
}

// ------------------------------------------------------------- launchers
template <int K>
static hipError_t pre_k(const void* d_table, const HostTable& h, const gabsplat_geom& g, hipStream_t s) {
  int64_t max_n = 0;
  for (int v = 0; v < h.hdr.num_views; ++v) {
    const int64_t n = h.scenes[h.views[v].scene].n;
    if (n > max_n) max_n = n;
  }
  if (max_n == 0) return hipSuccess;
  dim3 grid((unsigned)((max_n + kPreBlock - 1) / kPreBlock), (unsigned)h.hdr.num_views);
  if (h.scenes[0].rows != nullptr)  // every scene of the call has rows or none has
    hipLaunchKernelGGL((k_preprocess<K, true>), grid, dim3(256), 0, s, d_table, g.rec, g.depth, g.rect, g.tiles);
  else
    hipLaunchKernelGGL((k_preprocess<K, false>), grid, dim3(256), 0, s, d_table, g.rec, g.depth, g.rect, g.tiles);
  return hipGetLastError();
}

// gabsplat_pack_rows: a block transposes 64 primitives through LDS -- loads
// of consecutive primitives of one plane, then the 64 rows written as one
// contiguous run (zeros after the 4 + 4k used floats of each row).
constexpr int kPackRows = 64, kPackPitch = 65;  // row_stride(k) <= 64 columns; odd pitch
__global__ __launch_bounds__(256) void k_pack_rows(const float* __restrict__ quats, const float* __restrict__ freqs,
                                                   const float* __restrict__ weights, int64_t n, int k, int rs,
                                                   float* __restrict__ rows) {
  __shared__ float s[kPackRows * kPackPitch];
  const int64_t i0 = (int64_t)blockIdx.x * kPackRows;
  const int nrow = (int)min((int64_t)kPackRows, n - i0);
  const int used = 4 + 4 * k;
  for (int e = threadIdx.x; e < used * kPackRows; e += 256) {
    const int c = e / kPackRows, r = e - c * kPackRows;
    if (r < nrow) {
      const float* src = c < 4 ? quats + (int64_t)c * n
                               : (c < 4 + 3 * k ? freqs + (int64_t)(c - 4) * n : weights + (int64_t)(c - 4 - 3 * k) * n);
      s[r * kPackPitch + c] = src[i0 + r];
    }
  }
  __syncthreads();
  float* dst = rows + i0 * rs;
  for (int e = threadIdx.x; e < nrow * rs; e += 256) {
    const int r = e / rs, c = e - r * rs;
    dst[e] = c < used ? s[r * kPackPitch + c] : 0.f;
  }
}

hipError_t launch_pack_rows(const gabsplat_scene& sc, float* rows, hipStream_t s) {
  static_assert(row_stride(GABSPLAT_MAX_K) <= kPackPitch - 1, "a row fits the LDS pitch");
  const int64_t blocks = (sc.n + kPackRows - 1) / kPackRows;  // n < 2^31: fewer than 2^25 blocks
  hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)blocks), dim3(256), 0, s, sc.quats, sc.freqs, sc.weights, sc.n,
                     (int)sc.k, row_stride(sc.k), rows);
  return hipGetLastError();
}

hipError_t launch_preprocess(const void* d_table, const HostTable& h, const gabsplat_geom& g, hipStream_t s) {
  switch (h.scenes[0].k) {
    case 0: return pre_k<0>(d_table, h, g, s);
    case 1: return pre_k<1>(d_table, h, g, s);
    case 2: return pre_k<2>(d_table, h, g, s);
    case 3: return pre_k<3>(d_table, h, g, s);
    case 4: return pre_k<4>(d_table, h, g, s);
    case 5: return pre_k<5>(d_table, h, g, s);
    case 6: return pre_k<6>(d_table, h, g, s);
    case 7: return pre_k<7>(d_table, h, g, s);
    case 8: return pre_k<8>(d_table, h, g, s);
  }
  return hipErrorInvalidValue;
}

template <int K>
static hipError_t pbwd_k(const void* d_table, const HostTable& h, const gabsplat_geom& g, int sc,
                         const gabsplat_scene_grads& gr, const int32_t* ov, hipStream_t s) {
  const int64_t n = h.scenes[sc].n;
  if (n == 0) return hipSuccess;
  // geometry / frequency / opacity part, then the colour part (which adds
  // its view-direction term to the mean gradient): two register budgets
  const dim3 grid((unsigned)((n + kBwdBlock - 1) / kBwdBlock));
  if (h.scenes[sc].flags & (GABSPLAT_FLAG_MIP_2D | GABSPLAT_FLAG_MIP_3D))
    hipLaunchKernelGGL((k_preprocess_bwd<K, true>), grid, dim3(256), 0, s, d_table, sc, g.tiles, g.depth,
                       gr.grad2d, gr, ov);
  else
    hipLaunchKernelGGL((k_preprocess_bwd<K, false>), grid, dim3(256), 0, s, d_table, sc, g.tiles, g.depth,
                       gr.grad2d, gr, ov);
  const int gs = grad2d_stride(K, gr.flags);
  const dim3 cgr((unsigned)((n + kColBlock - 1) / kColBlock));
  const void* t = d_table;
  const uint32_t* tl = g.tiles;
  switch (h.scenes[sc].sh_degree) {  // -1: RGB colours
    case -1: hipLaunchKernelGGL(k_colour_bwd<-1>, cgr, dim3(kColBlock), 0, s, t, sc, tl, gr.grad2d, gr, gs, ov); break;
    case 0: hipLaunchKernelGGL(k_colour_bwd<0>, cgr, dim3(kColBlock), 0, s, t, sc, tl, gr.grad2d, gr, gs, ov); break;
    case 1: hipLaunchKernelGGL(k_colour_bwd<1>, cgr, dim3(kColBlock), 0, s, t, sc, tl, gr.grad2d, gr, gs, ov); break;
    case 2: hipLaunchKernelGGL(k_colour_bwd<2>, cgr, dim3(kColBlock), 0, s, t, sc, tl, gr.grad2d, gr, gs, ov); break;
    default: hipLaunchKernelGGL(k_colour_bwd<3>, cgr, dim3(kColBlock), 0, s, t, sc, tl, gr.grad2d, gr, gs, ov);
  }
  return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const void* d_table, const HostTable& h, const gabsplat_geom& g, int sc,
                                 const gabsplat_scene_grads& gr, const int32_t* ov, hipStream_t s) {
  switch (h.scenes[sc].k) {
    case 0: return pbwd_k<0>(d_table, h, g, sc, gr, ov, s);
    case 1: return pbwd_k<1>(d_table, h, g, sc, gr, ov, s);
    case 2: return pbwd_k<2>(d_table, h, g, sc, gr, ov, s);
    case 3: return pbwd_k<3>(d_table, h, g, sc, gr, ov, s);
    case 4: return pbwd_k<4>(d_table, h, g, sc, gr, ov, s);
    case 5: return pbwd_k<5>(d_table, h, g, sc, gr, ov, s);
    case 6: return pbwd_k<6>(d_table, h, g, sc, gr, ov, s);
    case 7: return pbwd_k<7>(d_table, h, g, sc, gr, ov, s);
    case 8: return pbwd_k<8>(d_table, h, g, sc, gr, ov, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace gs
