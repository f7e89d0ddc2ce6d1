// rig_build.hpp -- host-side validation of SplatCamera / SplatLidar and their conversion into
// the device sensor table (DevSensor).
#pragma once

#include <math.h>
#include <string.h>

#include "splat_common.hpp"

namespace splat {

inline bool finite_all(const float* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(v[i])) return false;
  return true;
}

// Limits of the binning kernels: a rectangle's width and wrap column are packed into 16 bits
// each, and a record's tile count into the top 24 bits of its 64-bit depth key.
constexpr int64_t kMaxRowTiles = 65535;
constexpr int64_t kMaxSensorTiles = ((int64_t)1 << 24) - 1;

// returns SPLAT_OK, SPLAT_ERR_INVALID_ARG, or SPLAT_ERR_UNSUPPORTED (beyond the limits above)
inline int build_camera(const SplatCamera& c, DevSensor& d) {
  memset(&d, 0, sizeof(d));
  if (c.width <= 0 || c.height <= 0 || c.tile_w <= 0 || c.tile_h <= 0) return SPLAT_ERR_INVALID_ARG;
  if (c.tile_w * c.tile_h > kBlock) return SPLAT_ERR_INVALID_ARG;
  if (!(c.fx > 0.f) || !(c.fy > 0.f) || !(c.near_plane > 0.f) || !(c.far_plane > c.near_plane)) return SPLAT_ERR_INVALID_ARG;
  if (!(c.eps2d >= 0.f) || !(c.t_rs >= 0.f) || !(c.jac_clamp >= 0.f)) return SPLAT_ERR_INVALID_ARG;
  if (c.n_channels < 0 || c.n_channels > SPLAT_MAX_CHANNELS || c.feat_offset < 0) return SPLAT_ERR_INVALID_ARG;
  if (!finite_all(c.R, 9) || !finite_all(c.t, 3) || !finite_all(c.lin_vel, 3) || !finite_all(c.ang_vel, 3))
    return SPLAT_ERR_INVALID_ARG;
  if (!isfinite(c.cx) || !isfinite(c.cy) || !isfinite(c.time_offset)) return SPLAT_ERR_INVALID_ARG;
  d.kind = kCamera;
  d.feat_off = c.feat_offset;
  d.n_ch = c.n_channels;
  memcpy(d.R, c.R, sizeof(d.R));
  memcpy(d.t, c.t, sizeof(d.t));
  memcpy(d.lin, c.lin_vel, sizeof(d.lin));
  memcpy(d.ang, c.ang_vel, sizeof(d.ang));
  d.t_rs = c.t_rs;
  d.eps2d = c.eps2d;
  d.t_off = c.time_offset;
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  d.near_p = c.near_plane; d.far_p = c.far_plane;
  if (c.jac_clamp > 0.f) {
    d.limx = c.jac_clamp * 0.5f * (float)c.width / c.fx;
    d.limy = c.jac_clamp * 0.5f * (float)c.height / c.fy;
  } else {
    d.limx = d.limy = -1.f;
  }
  d.width = c.width; d.height = c.height;
  d.tile_w = c.tile_w; d.tile_h = c.tile_h;
  const int64_t tx = ((int64_t)c.width + c.tile_w - 1) / c.tile_w, ty = ((int64_t)c.height + c.tile_h - 1) / c.tile_h;
  if (tx > kMaxRowTiles || tx * ty > kMaxSensorTiles) return SPLAT_ERR_UNSUPPORTED;
  d.tiles_x = (int32_t)tx;
  d.tiles_y = (int32_t)ty;
  d.n_tiles = d.tiles_x * d.tiles_y;
  d.st_wl = d.st_hl = kStLogCamera;
  d.st_x = (d.tiles_x + (1 << d.st_wl) - 1) >> d.st_wl;
  d.st_y = (d.tiles_y + (1 << d.st_hl) - 1) >> d.st_hl;
  d.n_rays = (int64_t)c.width * c.height;
  return SPLAT_OK;
}

inline int build_lidar(const SplatLidar& l, DevSensor& d) {
  memset(&d, 0, sizeof(d));
  if (l.tile_az <= 0 || l.n_az_tiles <= 0 || l.n_el_tiles <= 0 || l.n_el_tiles > SPLAT_MAX_EL_TILES) return SPLAT_ERR_INVALID_ARG;
  if (!(l.az_res > 0.f) || !(l.r_min >= 0.f) || !(l.r_max > l.r_min) || !(l.eps2d >= 0.f) || !(l.t_rs >= 0.f))
    return SPLAT_ERR_INVALID_ARG;
  if (l.elev_bounds == nullptr || l.n_rays < 0) return SPLAT_ERR_INVALID_ARG;
  if (!(l.los_eps >= 0.f) || !isfinite(l.los_eps)) return SPLAT_ERR_INVALID_ARG;
  if (l.n_rays > 0 && (l.ray_az == nullptr || l.ray_el == nullptr || l.ray_t == nullptr)) return SPLAT_ERR_INVALID_ARG;
  if (l.n_channels < 0 || l.n_channels > SPLAT_MAX_CHANNELS || l.feat_offset < 0) return SPLAT_ERR_INVALID_ARG;
  if (!finite_all(l.R, 9) || !finite_all(l.t, 3) || !finite_all(l.lin_vel, 3) || !finite_all(l.ang_vel, 3))
    return SPLAT_ERR_INVALID_ARG;
  for (int k = 0; k <= l.n_el_tiles; ++k) {
    if (!isfinite(l.elev_bounds[k])) return SPLAT_ERR_INVALID_ARG;
    if (k > 0 && !(l.elev_bounds[k] > l.elev_bounds[k - 1])) return SPLAT_ERR_INVALID_ARG;
  }
  if (l.n_az_tiles > kMaxRowTiles || (int64_t)l.n_az_tiles * l.n_el_tiles > kMaxSensorTiles) return SPLAT_ERR_UNSUPPORTED;
  float az_w = (float)l.tile_az * l.az_res;
  // the azimuth tiles must cover a full turn: M_phi * N_phi * res >= 2 pi (up to rounding)
  if ((double)l.n_az_tiles * (double)az_w < 2.0 * M_PI * (1.0 - 1e-6)) return SPLAT_ERR_INVALID_ARG;
  if ((double)(l.n_az_tiles - 1) * (double)az_w >= 2.0 * M_PI) return SPLAT_ERR_INVALID_ARG;
  d.kind = kLidar;
  d.feat_off = l.feat_offset;
  d.n_ch = l.n_channels;
  memcpy(d.R, l.R, sizeof(d.R));
  memcpy(d.t, l.t, sizeof(d.t));
  memcpy(d.lin, l.lin_vel, sizeof(d.lin));
  memcpy(d.ang, l.ang_vel, sizeof(d.ang));
  d.t_rs = l.t_rs;
  d.eps2d = l.eps2d;
  d.r_min = l.r_min;
  d.r_max = l.r_max;
  d.az_w = az_w;
  d.m_az = l.n_az_tiles;
  d.m_el = l.n_el_tiles;
  for (int k = 0; k <= l.n_el_tiles; ++k) d.bounds[k] = l.elev_bounds[k];
  d.ray_az = l.ray_az;
  d.ray_el = l.ray_el;
  d.ray_t = l.ray_t;
  d.ray_range = l.ray_range;
  d.los_eps = l.los_eps;
  d.ray_prio = l.ray_priority;
  d.n_tiles = l.n_az_tiles * l.n_el_tiles;
  d.st_wl = d.st_hl = kStLogLidar;
  d.st_x = (d.m_az + (1 << d.st_wl) - 1) >> d.st_wl;
  d.st_y = (d.m_el + (1 << d.st_hl) - 1) >> d.st_hl;
  d.n_rays = l.n_rays;
  return SPLAT_OK;
}

}  // namespace splat
