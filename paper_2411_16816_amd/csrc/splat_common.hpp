// splat_common.hpp -- device-side sensor table and the per-element arithmetic shared by the
// projection, rasterisation and adjoint kernels of libsplat (SplatAD, arXiv 2411.16816).
//
// Everything here is __host__ __device__ so the same arithmetic can be compiled for the host.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "splat.h"

#define HD __host__ __device__ __forceinline__

namespace splat {

constexpr float kTwoPi = 6.28318530717958647692f;   // float32 nearest to 2 pi (0x40C90FDB)
constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvTwoPi = 0.159154943091895335769f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;
constexpr int kBlock = 256;                  // lanes per rasterisation workgroup (4 x wave64)
// Binning supertiles (log2 of their width and height in tiles, at most 8 x 8): camera records
// cover about six tiles per side, lidar records (azimuth x elevation) about two by four.
constexpr int kStLogCamera = 3;
constexpr int kStLogLidar = 2;

enum SensorKind : int32_t { kCamera = 0, kLidar = 1 };

// One sensor as the kernels see it (built on the host from SplatCamera / SplatLidar).
struct alignas(16) DevSensor {
  int32_t kind;
  int32_t feat_off, n_ch;      // blended feature columns
  int32_t n_tiles;             // tiles of this sensor
  int64_t tile_base;           // global numbering inside the rig
  int32_t st_x, st_y;          // binning supertiles per row / column of the tile grid
  int32_t st_wl, st_hl;        // log2 of a supertile's width / height in tiles
  int64_t st_base;             // first supertile (global numbering inside the rig)
  int64_t ray_base;
  int64_t feat_base;
  int64_t n_rays;
  float R[9], t[3], lin[3], ang[3];
  float t_rs, eps2d;
  float t_off;                 // camera time offset (0 for lidars)
  // camera
  float fx, fy, cx, cy, near_p, far_p, limx, limy;   // limx/limy <= 0: no Jacobian clamp
  int32_t width, height, tile_w, tile_h, tiles_x, tiles_y;
  // lidar
  float r_min, r_max, az_w;    // az_w = fl(tile_az * az_res): azimuth width of a tile
  int32_t m_az, m_el;          // M_phi, M_omega
  const float* ray_az;
  const float* ray_el;
  const float* ray_t;
  const float* ray_range;      // measured ranges (line-of-sight sum) or null
  const uint16_t* ray_prio;    // training-time cap: per-ray priorities, or null (render every ray)
  float los_eps;
  float bounds[SPLAT_MAX_EL_TILES + 1];
};

struct f2 { float x, y; };

// ------------------------------------------------------------------------------------------
// correctly rounded division and floor for the tile arithmetic (bit-exact with IEEE float32)
// ------------------------------------------------------------------------------------------
HD float div_rn(float a, float b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __fdiv_rn(a, b);
#else
  return a / b;
#endif
}

// Reciprocal, square root and reciprocal square root of the projection: one hardware
// instruction each on the device (about 1 ulp, against the ten or so instructions of the
// correctly rounded forms), the IEEE operations on the host.  The tile arithmetic keeps div_rn.
HD float rcp_p(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
HD float sqrt_p(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}
HD float rsqrt_p(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rsqf(x);
#else
  return 1.0f / sqrtf(x);
#endif
}

// Z-order cell of a lidar ray inside its tile, on `cell_bits` bits: the tile is cut into
// 2^ab x 2^eb cells (ab = ceil(cell_bits / 2) azimuth bits, eb = floor(cell_bits / 2) elevation
// bits; azimuth from the fractional part of az / w, elevation from (el - b_e) / (b_{e+1} - b_e),
// float32 with correctly rounded divisions) and the cell's coordinates are interleaved: azimuth
// bit i at 2i, elevation bit i at 2i + 1 (the last azimuth bit on top when ab > eb).  Rays in
// consecutive codes are close together.
HD uint32_t ray_cell_code(float az_over_w, float el, float b_lo, float b_hi, int cell_bits) {
  const int ab = (cell_bits + 1) >> 1, eb = cell_bits >> 1;
  const float fa = az_over_w - floorf(az_over_w);
  const float fe = div_rn(el - b_lo, b_hi - b_lo);
  int qa = (int)(fa * (float)(1 << ab)), qe = (int)(fe * (float)(1 << eb));
  qa = qa < 0 ? 0 : (qa > (1 << ab) - 1 ? (1 << ab) - 1 : qa);
  qe = qe < 0 ? 0 : (qe > (1 << eb) - 1 ? (1 << eb) - 1 : qe);
  uint32_t z = 0;
  for (int i = 0; i < ab; ++i) z |= (((uint32_t)qa >> i) & 1u) << (2 * i);
  for (int i = 0; i < eb; ++i) z |= (((uint32_t)qe >> i) & 1u) << (2 * i + 1);
  return z;
}

HD int32_t floor_div_clamped(float x, float w) {
  float q = floorf(div_rn(x, w));
  const float lim = 16777216.0f;
  q = q < -lim ? -lim : (q > lim ? lim : q);
  return (int32_t)q;
}

// ------------------------------------------------------------------------------------------
// Gaussian covariance (Sec. 3.1): Sigma = M M^T, M = R(q) diag(exp(l)).  Returns M (row-major)
// ------------------------------------------------------------------------------------------
struct QuatRot {
  float qn[4];   // normalised quaternion (w,x,y,z)
  float inv_n;   // 1 / |q|
  float R[9];
};

HD void quat_rot(const float q[4], QuatRot& o) {
  float n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
  float inv = rsqrt_p(n2);
  o.inv_n = inv;
  float w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
  o.qn[0] = w; o.qn[1] = x; o.qn[2] = y; o.qn[3] = z;
  o.R[0] = 1.f - 2.f * (y * y + z * z); o.R[1] = 2.f * (x * y - w * z); o.R[2] = 2.f * (x * z + w * y);
  o.R[3] = 2.f * (x * y + w * z); o.R[4] = 1.f - 2.f * (x * x + z * z); o.R[5] = 2.f * (y * z - w * x);
  o.R[6] = 2.f * (x * z - w * y); o.R[7] = 2.f * (y * z + w * x); o.R[8] = 1.f - 2.f * (x * x + y * y);
}

// adjoint of quat_rot: dR (row-major 3x3) -> dq (raw quaternion), through the normalisation
HD void quat_rot_vjp(const QuatRot& o, const float dR[9], float dq[4]) {
  float w = o.qn[0], x = o.qn[1], y = o.qn[2], z = o.qn[3];
  float gw = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
  float gx = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] - 2.f * x * dR[8]);
  float gy = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] - 2.f * y * dR[8]);
  float gz = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
  // q_hat = q / |q|: dq = (g - q_hat (q_hat . g)) / |q|
  float dot = w * gw + x * gx + y * gy + z * gz;
  dq[0] = (gw - w * dot) * o.inv_n;
  dq[1] = (gx - x * dot) * o.inv_n;
  dq[2] = (gy - y * dot) * o.inv_n;
  dq[3] = (gz - z * dot) * o.inv_n;
}

HD void mat3_mul(const float A[9], const float B[9], float C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[i * 3 + j] = A[i * 3 + 0] * B[0 * 3 + j] + A[i * 3 + 1] * B[1 * 3 + j] + A[i * 3 + 2] * B[2 * 3 + j];
}

HD void mat3_vec(const float A[9], const float v[3], float o[3]) {
  o[0] = A[0] * v[0] + A[1] * v[1] + A[2] * v[2];
  o[1] = A[3] * v[0] + A[4] * v[1] + A[5] * v[2];
  o[2] = A[6] * v[0] + A[7] * v[1] + A[8] * v[2];
}

HD void mat3t_vec(const float A[9], const float v[3], float o[3]) {
  o[0] = A[0] * v[0] + A[3] * v[1] + A[6] * v[2];
  o[1] = A[1] * v[0] + A[4] * v[1] + A[7] * v[2];
  o[2] = A[2] * v[0] + A[5] * v[1] + A[8] * v[2];
}

HD void cross3(const float a[3], const float b[3], float o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// ------------------------------------------------------------------------------------------
// Projection of one Gaussian into one sensor (forward).  Keeps every intermediate the adjoint
// needs so forward and adjoint share one definition.
// ------------------------------------------------------------------------------------------
struct ProjInter {
  // common
  float mu[3];        // sensor-frame mean
  float W[9];         // R_sensor * R(q) * diag(s): Sigma_s = W W^T
  float vrel[3];      // relative velocity in the sensor frame
  float J[9];         // camera: rows 0-1 used (2x3); lidar: full J^S
  float T[6];         // J2 W (2x3): Sigma2 = T T^T
  float a2, b2, c2;   // Sigma2
  float det2, detp;   // det Sigma2, det (Sigma2 + sI)
  float ratio;        // det2 / detp
  // camera
  float iz;
  bool clx, cly;      // Jacobian clamp active
  float tx, ty;       // (clamped) x/z, y/z
  // lidar
  float rho, r, rho2, r2;
};

struct ProjOut {
  float mean[2], vel[2];
  float conic[3], o_eff;
  float box[4];
  float depth, v_r;
  int32_t rect[4];
  int32_t n_tiles;
  bool nonfinite;
};

HD bool finite_f(float v) { return v == v && v - v == 0.0f; }

HD void dilate_and_box(const DevSensor& S, float opac, ProjInter& I, ProjOut& o) {
  const float s = S.eps2d;
  // det(T T^T) = |T0 x T1|^2 (no cancellation), det(Sigma2 + sI) = det2 + s (a2 + c2) + s^2
  float t0[3] = {I.T[0], I.T[1], I.T[2]}, t1[3] = {I.T[3], I.T[4], I.T[5]}, cr[3];
  cross3(t0, t1, cr);
  I.det2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
  float a = I.a2 + s, c = I.c2 + s, b = I.b2;
  I.detp = I.det2 + s * (I.a2 + I.c2) + s * s;
  float inv = rcp_p(I.detp);
  o.conic[0] = c * inv;
  o.conic[1] = -b * inv;
  o.conic[2] = a * inv;
  I.ratio = I.det2 * inv;
  o.o_eff = opac * sqrt_p(I.ratio);
  float hr = 0.5f * S.t_rs;
  float ex = 3.0f * sqrt_p(a) + fabsf(o.vel[0]) * hr;
  float ey = 3.0f * sqrt_p(c) + fabsf(o.vel[1]) * hr;
  // centred on the mean at the sensor's time offset (the middle of the exposure; 0 for lidars)
  const float cx = fmaf(o.vel[0], S.t_off, o.mean[0]), cy = fmaf(o.vel[1], S.t_off, o.mean[1]);
  o.box[0] = cx - ex;
  o.box[1] = cy - ey;
  o.box[2] = cx + ex;
  o.box[3] = cy + ey;
}

HD void sensor_frame(const DevSensor& S, const float mu_w[3], const float M[9], const float vg[3], ProjInter& I) {
  mat3_vec(S.R, mu_w, I.mu);
  I.mu[0] += S.t[0]; I.mu[1] += S.t[1]; I.mu[2] += S.t[2];
  mat3_mul(S.R, M, I.W);
  float wxm[3], rv[3];
  cross3(S.ang, I.mu, wxm);
  mat3_vec(S.R, vg, rv);
  I.vrel[0] = -wxm[0] - S.lin[0] + rv[0];
  I.vrel[1] = -wxm[1] - S.lin[1] + rv[1];
  I.vrel[2] = -wxm[2] - S.lin[2] + rv[2];
}

HD void sigma2_from_T(ProjInter& I) {
  I.a2 = I.T[0] * I.T[0] + I.T[1] * I.T[1] + I.T[2] * I.T[2];
  I.b2 = I.T[0] * I.T[3] + I.T[1] * I.T[4] + I.T[2] * I.T[5];
  I.c2 = I.T[3] * I.T[3] + I.T[4] * I.T[4] + I.T[5] * I.T[5];
}

HD void mul_J2_W(const float J[9], const float W[9], float T[6]) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      T[i * 3 + j] = J[i * 3 + 0] * W[0 * 3 + j] + J[i * 3 + 1] * W[1 * 3 + j] + J[i * 3 + 2] * W[2 * 3 + j];
}

// camera (Sec. 3.2; Eq. pixel_velocity).  Returns false when culled by depth.
HD bool project_camera_core(const DevSensor& S, ProjInter& I, ProjOut& o) {
  float x = I.mu[0], y = I.mu[1], z = I.mu[2];
  if (!(z > S.near_p && z < S.far_p)) return false;
  I.iz = rcp_p(z);
  o.mean[0] = S.fx * x * I.iz + S.cx;
  o.mean[1] = S.fy * y * I.iz + S.cy;
  float tx = x * I.iz, ty = y * I.iz;
  I.clx = I.cly = false;
  if (S.limx > 0.f) {
    if (tx > S.limx) { tx = S.limx; I.clx = true; } else if (tx < -S.limx) { tx = -S.limx; I.clx = true; }
    if (ty > S.limy) { ty = S.limy; I.cly = true; } else if (ty < -S.limy) { ty = -S.limy; I.cly = true; }
  }
  I.tx = tx; I.ty = ty;
  I.J[0] = S.fx * I.iz; I.J[1] = 0.f; I.J[2] = -S.fx * tx * I.iz;
  I.J[3] = 0.f; I.J[4] = S.fy * I.iz; I.J[5] = -S.fy * ty * I.iz;
  I.J[6] = I.J[7] = I.J[8] = 0.f;
  mul_J2_W(I.J, I.W, I.T);
  sigma2_from_T(I);
  o.vel[0] = I.J[0] * I.vrel[0] + I.J[2] * I.vrel[2];
  o.vel[1] = I.J[4] * I.vrel[1] + I.J[5] * I.vrel[2];
  o.depth = z;
  o.v_r = 0.f;
  return true;
}

// lidar (Sec. 3.3: spherical projection, the printed J^S, v^S).  Returns false when culled by range.
HD bool project_lidar_core(const DevSensor& S, ProjInter& I, ProjOut& o) {
  float x = I.mu[0], y = I.mu[1], z = I.mu[2];
  I.rho2 = x * x + y * y;
  I.r2 = I.rho2 + z * z;
  I.rho = sqrt_p(I.rho2);
  I.r = sqrt_p(I.r2);
  if (!(I.r >= S.r_min && I.r <= S.r_max && I.rho >= 1e-4f * I.r)) return false;
  float phi = atan2f(y, x);
  if (phi < 0.f) phi += kTwoPi;
  if (phi >= kTwoPi) phi = 0.f;
  o.mean[0] = phi;
  float irho2 = rcp_p(I.rho2), ir2 = rcp_p(I.r2), irho = rcp_p(I.rho), ir = rcp_p(I.r);
  o.mean[1] = asinf(z * ir);
  float w = ir2 * irho;
  I.J[0] = -y * irho2; I.J[1] = x * irho2; I.J[2] = 0.f;
  I.J[3] = -x * z * w; I.J[4] = -y * z * w; I.J[5] = I.rho * ir2;
  I.J[6] = x * ir; I.J[7] = y * ir; I.J[8] = z * ir;
  mul_J2_W(I.J, I.W, I.T);
  sigma2_from_T(I);
  float v3[3];
  mat3_vec(I.J, I.vrel, v3);
  o.vel[0] = v3[0];
  o.vel[1] = v3[1];
  o.v_r = v3[2];
  o.depth = I.r;
  return true;
}

// tile rectangle of a camera box (lower floor(lo/T), upper floor(hi/T) + 1, clamped)
HD void camera_rect(const DevSensor& S, ProjOut& o) {
  int32_t x0 = floor_div_clamped(o.box[0], (float)S.tile_w);
  int32_t x1 = floor_div_clamped(o.box[2], (float)S.tile_w) + 1;
  int32_t y0 = floor_div_clamped(o.box[1], (float)S.tile_h);
  int32_t y1 = floor_div_clamped(o.box[3], (float)S.tile_h) + 1;
  x0 = x0 < 0 ? 0 : (x0 > S.tiles_x ? S.tiles_x : x0);
  x1 = x1 < 0 ? 0 : (x1 > S.tiles_x ? S.tiles_x : x1);
  y0 = y0 < 0 ? 0 : (y0 > S.tiles_y ? S.tiles_y : y0);
  y1 = y1 < 0 ? 0 : (y1 > S.tiles_y ? S.tiles_y : y1);
  int32_t nx = x1 - x0, ny = y1 - y0;
  nx = nx < 0 ? 0 : nx;
  ny = ny < 0 ? 0 : ny;
  o.rect[0] = x0; o.rect[1] = y0; o.rect[2] = nx; o.rect[3] = ny;
  o.n_tiles = nx * ny;
}

// number of elevation boundaries <= v
HD int32_t count_le(const DevSensor& S, float v) {
  int32_t c = 0;
  for (int k = 0; k <= S.m_el; ++k) c += (S.bounds[k] <= v) ? 1 : 0;
  return c;
}

// lidar tile rectangle (App. A): azimuth start wrapped into [0, M_phi) and a span clamped to
// M_phi; elevation tiles [last boundary <= lo, last boundary <= hi + 1).
HD void lidar_rect(const DevSensor& S, ProjOut& o) {
  const int32_t M = S.m_az;
  float lo_a = o.box[0], hi_a = o.box[2];
  float lo_w = lo_a < 0.f ? lo_a + kTwoPi : lo_a;
  float hi_w = hi_a > kTwoPi ? hi_a - kTwoPi : hi_a;
  int32_t low = floor_div_clamped(lo_w, S.az_w) - (lo_a < 0.f ? M : 0);
  int32_t high = floor_div_clamped(hi_w, S.az_w) + 1 + (hi_a > kTwoPi ? M : 0);
  int32_t n = high - low;
  int32_t start;
  if (n >= M) { start = 0; n = M; }
  else { start = ((low % M) + M) % M; n = n < 0 ? 0 : n; }
  int32_t e0 = count_le(S, o.box[1]) - 1;
  int32_t e1 = count_le(S, o.box[3]);
  e0 = e0 < 0 ? 0 : (e0 > S.m_el ? S.m_el : e0);
  e1 = e1 > S.m_el ? S.m_el : e1;
  int32_t ne = e1 - e0;
  ne = ne < 0 ? 0 : ne;
  o.rect[0] = start; o.rect[1] = e0; o.rect[2] = n; o.rect[3] = ne;
  o.n_tiles = n * ne;
}

// Tile (sensor-local id) at (row, col) of a record's rectangle r = (x0, y0, w, h); lidar
// azimuth tiles wrap modulo M_phi (x0 < M_phi and w <= M_phi, so one subtraction suffices).
HD int64_t rect_tile_rc(const DevSensor& S, const int4 r, int row, int col) {
  if (S.kind == kCamera) return (int64_t)(r.y + row) * S.tiles_x + (r.x + col);
  int a = r.x + col;
  a -= a >= S.m_az ? S.m_az : 0;
  return (int64_t)(r.y + row) * S.m_az + a;
}

// Tile of the j-th entry of rectangle r: entries are numbered row-major.
HD int64_t rect_tile(const DevSensor& S, const int4 r, int j) { return rect_tile_rc(S, r, j / r.z, j % r.z); }

// Inverse of rect_tile: the entry number of sensor-local tile t inside rectangle r.
HD int rect_entry(const DevSensor& S, const int4 r, int64_t t) {
  if (S.kind == kCamera) {
    const int tx = (int)(t % S.tiles_x), ty = (int)(t / S.tiles_x);
    return (ty - r.y) * r.z + (tx - r.x);
  }
  const int a = (int)(t % S.m_az), e = (int)(t / S.m_az);
  int da = a - r.x;
  if (da < 0) da += S.m_az;
  return (e - r.y) * r.z + da;
}

// Full forward projection of Gaussian (mu_w, M, vg, opac) into sensor S.  n_tiles = 0 = culled.
HD void project_one(const DevSensor& S, const float mu_w[3], const float M[9], const float vg[3], float opac,
                    ProjInter& I, ProjOut& o) {
  o.n_tiles = 0;
  o.nonfinite = false;
  sensor_frame(S, mu_w, M, vg, I);
  // a non-finite mean fails every depth / range comparison: count it rather than cull it silently
  if (!(finite_f(I.mu[0]) && finite_f(I.mu[1]) && finite_f(I.mu[2]))) { o.nonfinite = true; return; }
  bool ok = (S.kind == kCamera) ? project_camera_core(S, I, o) : project_lidar_core(S, I, o);
  if (!ok) return;
  dilate_and_box(S, opac, I, o);
  bool fin = finite_f(o.mean[0]) && finite_f(o.mean[1]) && finite_f(o.vel[0]) && finite_f(o.vel[1]) &&
             finite_f(o.conic[0]) && finite_f(o.conic[1]) && finite_f(o.conic[2]) && finite_f(o.o_eff) &&
             finite_f(o.box[0]) && finite_f(o.box[1]) && finite_f(o.box[2]) && finite_f(o.box[3]) &&
             finite_f(o.v_r) && finite_f(o.depth);
  if (!fin) { o.nonfinite = true; return; }
  if (!(o.o_eff >= kAlphaMin)) return;
  if (S.kind == kCamera) {
    if (!(o.box[0] < (float)S.width && o.box[2] > 0.f && o.box[1] < (float)S.height && o.box[3] > 0.f)) return;
    camera_rect(S, o);
  } else {
    if (!(o.box[3] > S.bounds[0] && o.box[1] < S.bounds[S.m_el])) return;
    lidar_rect(S, o);
  }
}

HD void gaussian_M(const float q[4], const float ls[3], QuatRot& qr, float s[3], float M[9]) {
  quat_rot(q, qr);
  s[0] = expf(ls[0]); s[1] = expf(ls[1]); s[2] = expf(ls[2]);
  for (int i = 0; i < 3; ++i) {
    M[i * 3 + 0] = qr.R[i * 3 + 0] * s[0];
    M[i * 3 + 1] = qr.R[i * 3 + 1] * s[1];
    M[i * 3 + 2] = qr.R[i * 3 + 2] * s[2];
  }
}

// ------------------------------------------------------------------------------------------
// Adjoint of project_one for a kept record.  Inputs: gradients of the record quantities the
// rasteriser reads (mean, vel, conic, o_eff, depth (z | r), v_r).  Outputs are ADDED to
// dmu_w, dM (dL/dM of Sigma = M M^T), dvg, dopac.
// ------------------------------------------------------------------------------------------
struct RecGrad {
  float mean[2], vel[2], conic[3], o_eff, depth, v_r;
};

// dvrel_out (optional): the gradient with respect to the sensor-frame relative velocity, from
// which the sensor's own velocity gradients follow (vrel = -ang x mu - lin + R vg).
HD void project_one_vjp(const DevSensor& S, const float M[9], float opac, const ProjInter& I, const ProjOut& o,
                        const RecGrad& g, float dmu_w[3], float dM[9], float dvg[3], float* dopac,
                        float* dvrel_out = nullptr) {
  const float s = S.eps2d;
  // --- o_eff = opac * sqrt(ratio), ratio = det2 / detp
  float sq = sqrt_p(I.ratio);
  *dopac += g.o_eff * sq;
  float d_ratio = (I.ratio > 0.f) ? g.o_eff * opac * 0.5f * rcp_p(sq) : 0.f;
  float inv = rcp_p(I.detp);
  float d_det2 = d_ratio * inv;
  float d_detp = -d_ratio * I.det2 * inv * inv;
  // --- conic = (c, -b, a) / detp with a = a2 + s, c = c2 + s, b = b2
  float a = I.a2 + s, c = I.c2 + s, b = I.b2;
  d_detp += -(g.conic[0] * c - g.conic[1] * b + g.conic[2] * a) * inv * inv;
  float d_a = g.conic[2] * inv, d_b = -g.conic[1] * inv, d_c = g.conic[0] * inv;
  // detp = det2 + s (a2 + c2) + s^2
  d_det2 += d_detp;
  d_a += d_detp * s;
  d_c += d_detp * s;
  // --- box extents are not differentiated (they only decide candidacy)
  // --- a2 = |T0|^2, b2 = T0.T1, c2 = |T1|^2, det2 = |T0 x T1|^2
  float dT[6];
  for (int j = 0; j < 3; ++j) {
    dT[j] = 2.f * d_a * I.T[j] + d_b * I.T[3 + j];
    dT[3 + j] = 2.f * d_c * I.T[3 + j] + d_b * I.T[j];
  }
  {
    float t0[3] = {I.T[0], I.T[1], I.T[2]}, t1[3] = {I.T[3], I.T[4], I.T[5]}, cr[3], gcr[3], u[3];
    cross3(t0, t1, cr);
    gcr[0] = 2.f * d_det2 * cr[0]; gcr[1] = 2.f * d_det2 * cr[1]; gcr[2] = 2.f * d_det2 * cr[2];
    // d(t0 x t1) = dt0 x t1 + t0 x dt1  ->  dt0 = t1 x gcr, dt1 = gcr x t0
    cross3(t1, gcr, u);
    dT[0] += u[0]; dT[1] += u[1]; dT[2] += u[2];
    cross3(gcr, t0, u);
    dT[3] += u[0]; dT[4] += u[1]; dT[5] += u[2];
  }
  // --- T = J2 W: dJ2 = dT W^T, dW = J2^T dT
  float dJ[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < 2; ++i)
    for (int k = 0; k < 3; ++k)
      dJ[i * 3 + k] = dT[i * 3 + 0] * I.W[k * 3 + 0] + dT[i * 3 + 1] * I.W[k * 3 + 1] + dT[i * 3 + 2] * I.W[k * 3 + 2];
  float dW[9];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      dW[k * 3 + j] = I.J[0 * 3 + k] * dT[0 * 3 + j] + I.J[1 * 3 + k] * dT[1 * 3 + j];
  // --- velocity v = J vrel (rows 0..1, plus row 2 for lidar)
  float gv[3] = {g.vel[0], g.vel[1], (S.kind == kLidar) ? g.v_r : 0.f};
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) dJ[i * 3 + k] += gv[i] * I.vrel[k];
  float dvrel[3];
  mat3t_vec(I.J, gv, dvrel);
  if (dvrel_out) {
    dvrel_out[0] = dvrel[0];
    dvrel_out[1] = dvrel[1];
    dvrel_out[2] = dvrel[2];
  }
  // --- sensor-frame mean gradient
  float dmu[3] = {0, 0, 0};
  if (S.kind == kCamera) {
    float x = I.mu[0], y = I.mu[1];
    float iz = I.iz;
    // mean (u,v)
    dmu[0] += g.mean[0] * S.fx * iz;
    dmu[1] += g.mean[1] * S.fy * iz;
    dmu[2] += -(g.mean[0] * S.fx * x + g.mean[1] * S.fy * y) * iz * iz;
    // depth = z
    dmu[2] += g.depth;
    // J00 = fx/z, J11 = fy/z, J02 = -fx tx / z, J12 = -fy ty / z (tx = x/z unless clamped)
    float d_iz = dJ[0] * S.fx + dJ[4] * S.fy - dJ[2] * S.fx * I.tx - dJ[5] * S.fy * I.ty;
    float d_tx = -dJ[2] * S.fx * iz, d_ty = -dJ[5] * S.fy * iz;
    if (!I.clx) { dmu[0] += d_tx * iz; d_iz += d_tx * x; }
    if (!I.cly) { dmu[1] += d_ty * iz; d_iz += d_ty * y; }
    dmu[2] += -d_iz * iz * iz;
  } else {
    float x = I.mu[0], y = I.mu[1], z = I.mu[2];
    float irho2 = rcp_p(I.rho2), ir2 = rcp_p(I.r2), irho = rcp_p(I.rho), ir = rcp_p(I.r);
    float w = ir2 * irho;
    // mean (phi, omega) and depth r: their gradients are rows of J^S
    float gm[3] = {g.mean[0], g.mean[1], g.depth};
    float t3[3];
    mat3t_vec(I.J, gm, t3);
    dmu[0] += t3[0]; dmu[1] += t3[1]; dmu[2] += t3[2];
    // entries of J^S as functions of (x, y, z)
    float g_irho2 = -y * dJ[0] + x * dJ[1];
    dmu[0] += irho2 * dJ[1];
    dmu[1] += -irho2 * dJ[0];
    float g_w = -x * z * dJ[3] - y * z * dJ[4];
    dmu[0] += -z * w * dJ[3];
    dmu[1] += -z * w * dJ[4];
    dmu[2] += -(x * dJ[3] + y * dJ[4]) * w;
    float g_ir2 = irho * g_w + I.rho * dJ[5];
    float g_irho = ir2 * g_w;
    float g_rho = ir2 * dJ[5];
    float g_ir = x * dJ[6] + y * dJ[7] + z * dJ[8];
    dmu[0] += ir * dJ[6];
    dmu[1] += ir * dJ[7];
    dmu[2] += ir * dJ[8];
    float g_rho2 = -irho2 * irho2 * g_irho2;
    g_rho += -irho * irho * g_irho;
    float g_r2 = -ir2 * ir2 * g_ir2;
    float g_r = -ir * ir * g_ir;
    g_rho2 += g_rho * 0.5f * irho;
    g_r2 += g_r * 0.5f * ir;
    g_rho2 += g_r2;
    dmu[2] += 2.f * z * g_r2;
    dmu[0] += 2.f * x * g_rho2;
    dmu[1] += 2.f * y * g_rho2;
  }
  // vrel = -ang x mu - lin + R vg: the adjoint of mu -> -(ang x mu) is g -> ang x g
  {
    float c3[3];
    cross3(S.ang, dvrel, c3);
    dmu[0] += c3[0]; dmu[1] += c3[1]; dmu[2] += c3[2];
    float t3[3];
    mat3t_vec(S.R, dvrel, t3);
    dvg[0] += t3[0]; dvg[1] += t3[1]; dvg[2] += t3[2];
  }
  // mu_s = R mu_w + t
  {
    float t3[3];
    mat3t_vec(S.R, dmu, t3);
    dmu_w[0] += t3[0]; dmu_w[1] += t3[1]; dmu_w[2] += t3[2];
  }
  // W = R M: dM += R^T dW
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      dM[k * 3 + j] += S.R[0 * 3 + k] * dW[0 * 3 + j] + S.R[1 * 3 + k] * dW[1 * 3 + j] + S.R[2 * 3 + k] * dW[2 * 3 + j];
}

// adjoint of gaussian_M: dM -> dq (raw), dlog_scale
HD void gaussian_M_vjp(const QuatRot& qr, const float s[3], const float dM[9], float dq[4], float dls[3]) {
  float dR[9];
  for (int i = 0; i < 3; ++i) {
    dR[i * 3 + 0] = dM[i * 3 + 0] * s[0];
    dR[i * 3 + 1] = dM[i * 3 + 1] * s[1];
    dR[i * 3 + 2] = dM[i * 3 + 2] * s[2];
  }
  for (int j = 0; j < 3; ++j)
    dls[j] = (dM[0 * 3 + j] * qr.R[0 * 3 + j] + dM[1 * 3 + j] * qr.R[1 * 3 + j] + dM[2 * 3 + j] * qr.R[2 * 3 + j]) * s[j];
  quat_rot_vjp(qr, dR, dq);
}

// ------------------------------------------------------------------------------------------
// Per (ray, Gaussian) evaluation shared bit-for-bit by the forward and adjoint rasterisers.
// ------------------------------------------------------------------------------------------

// BOX candidacy of a camera pixel / lidar ray (azimuth modular, see lidar_rect)
HD bool box_contains(bool lidar, float px, float py, const float bx[4]) {
  bool in_y = (py >= bx[1]) && (py < bx[3]);
  bool in_x;
  if (!lidar) {
    in_x = (px >= bx[0]) && (px < bx[2]);
  } else {
    in_x = (px >= bx[0] && px < bx[2]) || (bx[0] < 0.f && px >= bx[0] + kTwoPi) ||
           (bx[2] > kTwoPi && px < bx[2] - kTwoPi);
  }
  return in_x && in_y;
}

#if defined(__HIP_DEVICE_COMPILE__)
#define SPLAT_FMA(a, b, c) __builtin_fmaf(a, b, c)
#else
#define SPLAT_FMA(a, b, c) fmaf(a, b, c)
#endif

constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kLn2 = 0.693147180559945309417f;

// The conic (a, b, c) of Eq. delta in base-2 form: exp(-sigma) = 2^s with
// s = A dx^2 + B dx dy + C dy^2, A = -a log2(e) / 2, B = -b log2(e), C = -c log2(e) / 2.
// The rasterisers stage this form (and the opacity in .w), so one exp2 evaluates a Gaussian.
HD float4 conic_exp2(float4 cn) {
  return make_float4(cn.x * (-0.5f * kLog2e), cn.y * -kLog2e, cn.z * (-0.5f * kLog2e), cn.w);
}

HD float exp2_fast(float s) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_exp2f(s);
#else
  return exp2f(s);
#endif
}

struct PairEval {
  float dx, dy;   // ray minus the mean at the ray's time (lidar azimuth reduced to [-pi, pi))
  float tx;       // A dx + B dy
  float cy;       // C dy
  float G;        // exp(-sigma), Eq. delta
  float oG;       // opacity x G: Eq. alpha before its clamp
};

// Eq. delta and the unclamped Eq. alpha for a ray at (px, py, t) and a Gaussian whose mean
// moves as (mv.x + mv.z t, mv.y + mv.w t), with its conic in conic_exp2 form.  Explicit fma so
// that the forward and the adjoint evaluate identical arithmetic.
HD void eval_pair(bool lidar, float px, float py, float t, float4 mv, float4 ce, PairEval& e) {
  float dx = px - SPLAT_FMA(mv.z, t, mv.x);
  const float dy = py - SPLAT_FMA(mv.w, t, mv.y);
  if (lidar) {
    // azimuth difference reduced to [-pi, pi): the rolling-shutter shift v t of a Gaussian close
    // to the sensor can span several turns, so the reduction is modular, not a single wrap
    const float k = floorf(SPLAT_FMA(dx, kInvTwoPi, 0.5f));
    dx = SPLAT_FMA(-k, kTwoPi, dx);
  }
  e.dx = dx;
  e.dy = dy;
  e.tx = SPLAT_FMA(ce.x, dx, ce.y * dy);
  e.cy = ce.z * dy;
  e.G = exp2_fast(SPLAT_FMA(dx, e.tx, e.cy * dy));
  e.oG = ce.w * e.G;
}

// Eq. alpha's clamp: min(o G, 0.99)
HD float clamp_alpha(float oG) { return fminf(oG, kAlphaMax); }

}  // namespace splat
