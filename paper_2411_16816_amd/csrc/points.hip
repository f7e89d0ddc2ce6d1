// points.hip -- lidar points to rasterisation rays (SplatAD, arXiv 2411.16816, App. A "Lidar
// points to rasterization points").
//
// A sweep arrives as world points with the ego motion compensated (every point expressed as if
// captured at the sweep's reference time).  Each point is moved back to where the sensor saw it
// at its own capture time t, under the sensor's constant linear and angular velocity (the motion
// the rolling-shutter model gives a static Gaussian: relative velocity -w x x - v), and converted
// to spherical coordinates:
//   x_l = R x_w + t_s,   x_cap = x_l + t (-w x x_l - v),
//   azimuth = atan2(y, x) in [0, 2 pi),   elevation = asin(z / r),   range = r = |x_cap|.
// The azimuth and elevation are the ray the rasteriser renders at time t; the range is the
// measured range of the line-of-sight sum.
//
// Streaming and HBM-bound: 28 B per point (12 B point + 4 B time in, 12 B out).  Each thread
// maps four consecutive points with 16-byte loads and stores (three for the points, one for
// the times) when every array is 16-byte aligned; a grid-stride loop covers any size.
#include <cfloat>

#include "kernels.hpp"

namespace splat {

struct PointsXform {
  float R[9], t[3], v[3], w[3];
};

__device__ __forceinline__ void point_to_ray(const PointsXform& X, float px, float py, float pz, float tt, float& az,
                                             float& el, float& rg) {
  // sensor frame at the reference time
  float x = fmaf(X.R[0], px, fmaf(X.R[1], py, fmaf(X.R[2], pz, X.t[0])));
  float y = fmaf(X.R[3], px, fmaf(X.R[4], py, fmaf(X.R[5], pz, X.t[1])));
  float z = fmaf(X.R[6], px, fmaf(X.R[7], py, fmaf(X.R[8], pz, X.t[2])));
  // relative to the sensor at the capture time: x + t (-(w x x) - v)
  const float cx = X.w[1] * z - X.w[2] * y;
  const float cy = X.w[2] * x - X.w[0] * z;
  const float cz = X.w[0] * y - X.w[1] * x;
  x = fmaf(-tt, cx + X.v[0], x);
  y = fmaf(-tt, cy + X.v[1], y);
  z = fmaf(-tt, cz + X.v[2], z);
  const float r = sqrtf(x * x + y * y + z * z);
  if (!(r <= FLT_MAX)) {   // non-finite input: a ray outside every tile
    az = el = rg = __builtin_nanf("");
    return;
  }
  float phi = atan2f(y, x);
  if (phi < 0.f) phi += kTwoPi;
  if (phi >= kTwoPi) phi = 0.f;   // -0 or a tiny negative angle rounded up to 2 pi
  float s = r > 0.f ? z / r : 0.f;
  s = fminf(fmaxf(s, -1.f), 1.f);
  az = phi;
  el = asinf(s);
  rg = r;
}

__global__ void k_points_to_rays(const float* __restrict__ pts, const float* __restrict__ tm, int64_t n,
                                 PointsXform X, float* __restrict__ az, float* __restrict__ el,
                                 float* __restrict__ rg, int vec) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; 4 * q < n; q += stride) {
    const int64_t i0 = 4 * q;
    if (vec && i0 + 4 <= n) {
      const float4* p4 = reinterpret_cast<const float4*>(pts) + 3 * q;
      const float4 a = p4[0], b = p4[1], c = p4[2];
      const float4 t4 = reinterpret_cast<const float4*>(tm)[q];
      float4 oa, oe, orr;
      point_to_ray(X, a.x, a.y, a.z, t4.x, oa.x, oe.x, orr.x);
      point_to_ray(X, a.w, b.x, b.y, t4.y, oa.y, oe.y, orr.y);
      point_to_ray(X, b.z, b.w, c.x, t4.z, oa.z, oe.z, orr.z);
      point_to_ray(X, c.y, c.z, c.w, t4.w, oa.w, oe.w, orr.w);
      reinterpret_cast<float4*>(az)[q] = oa;
      reinterpret_cast<float4*>(el)[q] = oe;
      if (rg) reinterpret_cast<float4*>(rg)[q] = orr;
    } else {
      for (int k = 0; k < 4; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        float a, e, r;
        point_to_ray(X, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], tm[i], a, e, r);
        az[i] = a;
        el[i] = e;
        if (rg) rg[i] = r;
      }
    }
  }
}

}  // namespace splat

using namespace splat;

extern "C" {

int splat_lidar_points_to_rays(int64_t n, const float* points, const float* times, const float* R,
                               const float* t, const float* lin_vel, const float* ang_vel, float* ray_az,
                               float* ray_el, float* ray_range, void* stream) {
  if (n < 0 || !R || !t) return SPLAT_ERR_INVALID_ARG;
  if (n == 0) return SPLAT_OK;
  if (!points || !times || !ray_az || !ray_el) return SPLAT_ERR_INVALID_ARG;
  PointsXform X;
  for (int k = 0; k < 9; ++k) X.R[k] = R[k];
  for (int k = 0; k < 3; ++k) {
    X.t[k] = t[k];
    X.v[k] = lin_vel ? lin_vel[k] : 0.f;
    X.w[k] = ang_vel ? ang_vel[k] : 0.f;
  }
  const uintptr_t al = (uintptr_t)points | (uintptr_t)times | (uintptr_t)ray_az | (uintptr_t)ray_el |
                       (uintptr_t)ray_range;
  const int vec = (al & 15) == 0;
  int64_t blocks = div_up(div_up(n, 4), 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_points_to_rays, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, points, times, n, X,
                     ray_az, ray_el, ray_range, vec);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

}  // extern "C"
