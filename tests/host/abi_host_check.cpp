// Host-side checks of the C ABI, built with AddressSanitizer and UndefinedBehaviorSanitizer
// (host code only) by tests/test_host_sanitizers.py: sensor validation over valid and invalid
// cameras and lidars, workspace sizing over edge sizes, and the argument checks of the entry
// points, which must reject bad arguments before touching a device.  Prints one line per
// failed expectation and "host abi checks: N passed"; exits non-zero on any failure.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <limits>
#include <vector>

#include "splat.h"

static int g_pass = 0, g_fail = 0;

static void expect(bool ok, const char* what) {
  if (ok) {
    ++g_pass;
  } else {
    ++g_fail;
    printf("FAIL: %s\n", what);
  }
}

static SplatCamera camera() {
  SplatCamera c;
  memset(&c, 0, sizeof(c));
  for (int i = 0; i < 3; ++i) c.R[4 * i] = 1.f;
  c.fx = c.fy = 500.f;
  c.cx = 320.f;
  c.cy = 240.f;
  c.width = 640;
  c.height = 480;
  c.t_rs = 0.03f;
  c.eps2d = 0.3f;
  c.near_plane = 0.01f;
  c.far_plane = 1000.f;
  c.jac_clamp = 1.3f;
  c.n_channels = 3;
  c.tile_w = c.tile_h = 16;
  return c;
}

static std::vector<float> g_bounds = {-0.4f, -0.2f, 0.f, 0.1f, 0.2f};

static SplatLidar lidar(const float* az, const float* el, const float* t, int64_t n) {
  SplatLidar l;
  memset(&l, 0, sizeof(l));
  for (int i = 0; i < 3; ++i) l.R[4 * i] = 1.f;
  l.t_rs = 0.1f;
  l.eps2d = 1e-6f;
  l.r_min = 0.5f;
  l.r_max = 200.f;
  l.az_res = 2.f * (float)M_PI / 1024.f;
  l.tile_az = 32;
  l.n_az_tiles = 32;
  l.n_el_tiles = (int32_t)g_bounds.size() - 1;
  l.elev_bounds = g_bounds.data();
  l.n_rays = n;
  l.ray_az = az;
  l.ray_el = el;
  l.ray_t = t;
  l.n_channels = 8;
  return l;
}

static void check_cameras() {
  const float nan = std::numeric_limits<float>::quiet_NaN(), inf = std::numeric_limits<float>::infinity();
  SplatCamera c = camera();
  expect(splat_check_camera(&c) == SPLAT_OK, "valid camera");
  expect(splat_check_camera(nullptr) == SPLAT_ERR_INVALID_ARG, "null camera");
  struct Case {
    const char* what;
    void (*edit)(SplatCamera&);
  };
  static float s_nan, s_inf;
  s_nan = nan;
  s_inf = inf;
  const Case bad[] = {
      {"zero width", [](SplatCamera& x) { x.width = 0; }},
      {"negative height", [](SplatCamera& x) { x.height = -4; }},
      {"zero tile", [](SplatCamera& x) { x.tile_w = 0; }},
      {"tile above 256 pixels", [](SplatCamera& x) { x.tile_w = 32; x.tile_h = 16; }},
      {"zero focal", [](SplatCamera& x) { x.fx = 0.f; }},
      {"nan focal", [](SplatCamera& x) { x.fy = s_nan; }},
      {"far before near", [](SplatCamera& x) { x.far_plane = 0.001f; }},
      {"negative near", [](SplatCamera& x) { x.near_plane = -1.f; }},
      {"negative dilation", [](SplatCamera& x) { x.eps2d = -0.1f; }},
      {"negative shutter", [](SplatCamera& x) { x.t_rs = -0.01f; }},
      {"negative clamp", [](SplatCamera& x) { x.jac_clamp = -1.f; }},
      {"too many channels", [](SplatCamera& x) { x.n_channels = SPLAT_MAX_CHANNELS + 1; }},
      {"negative feature offset", [](SplatCamera& x) { x.feat_offset = -1; }},
      {"nan rotation", [](SplatCamera& x) { x.R[3] = s_nan; }},
      {"inf translation", [](SplatCamera& x) { x.t[1] = s_inf; }},
      {"nan velocity", [](SplatCamera& x) { x.lin_vel[2] = s_nan; }},
      {"inf principal point", [](SplatCamera& x) { x.cx = s_inf; }},
      {"nan time offset", [](SplatCamera& x) { x.time_offset = s_nan; }},
  };
  for (const Case& k : bad) {
    SplatCamera x = camera();
    k.edit(x);
    expect(splat_check_camera(&x) == SPLAT_ERR_INVALID_ARG, k.what);
  }
  SplatCamera wide = camera();   // more tiles per row than the binning supports
  wide.width = 70000 * 16;
  wide.height = 16;
  expect(splat_check_camera(&wide) == SPLAT_ERR_UNSUPPORTED, "tiles per row beyond the limit");
}

static void check_lidars() {
  const float nan = std::numeric_limits<float>::quiet_NaN();
  float az[4] = {0.1f, 1.f, 2.f, 3.f}, el[4] = {0.f, 0.05f, -0.1f, 0.15f}, t[4] = {0.f, 0.01f, -0.02f, 0.03f};
  SplatLidar l = lidar(az, el, t, 4);
  expect(splat_check_lidar(&l) == SPLAT_OK, "valid lidar");
  expect(splat_check_lidar(nullptr) == SPLAT_ERR_INVALID_ARG, "null lidar");
  SplatLidar x = l;
  x.elev_bounds = nullptr;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "null elevation bounds");
  std::vector<float> unsorted = {-0.4f, 0.1f, 0.f, 0.2f};
  x = l;
  x.elev_bounds = unsorted.data();
  x.n_el_tiles = 3;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "unsorted elevation bounds");
  std::vector<float> with_nan = {-0.4f, nan, 0.2f};
  x = l;
  x.elev_bounds = with_nan.data();
  x.n_el_tiles = 2;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "nan elevation bound");
  x = l;
  x.n_el_tiles = SPLAT_MAX_EL_TILES + 1;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "too many elevation tiles");
  x = l;
  x.n_az_tiles = 31;   // 31 x 32 steps of 2 pi / 1024 do not cover a turn
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "azimuth tiles short of a turn");
  x = l;
  x.n_az_tiles = 34;   // the 34th tile starts past 2 pi
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "azimuth tiles past a turn");
  x = l;
  x.ray_az = nullptr;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "rays without azimuths");
  x = l;
  x.n_rays = 0;
  x.ray_az = x.ray_el = x.ray_t = nullptr;
  expect(splat_check_lidar(&x) == SPLAT_OK, "lidar without rays");
  x = l;
  x.r_max = x.r_min;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "empty range window");
  x = l;
  x.los_eps = -1.f;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "negative line-of-sight margin");
  x = l;
  x.az_res = 0.f;
  expect(splat_check_lidar(&x) == SPLAT_ERR_INVALID_ARG, "zero azimuth resolution");
  x = l;
  x.tile_az = 1;
  x.n_az_tiles = 70000;
  x.az_res = 2.f * (float)M_PI / 70000.f;
  expect(splat_check_lidar(&x) == SPLAT_ERR_UNSUPPORTED, "azimuth tiles beyond the limit");
}

static void check_sizes() {
  expect(splat_compose_workspace_bytes(0) > 0, "composition workspace for no actors");
  expect(splat_compose_workspace_bytes(10) == 10 * 24 * sizeof(float), "composition workspace per actor");
  expect(splat_lidar_decode_workspace_bytes(-1, 8) == 0, "decoder workspace for negative rays");
  expect(splat_lidar_decode_workspace_bytes(262144, 8) > 0, "decoder workspace for a sweep");
  expect(splat_camera_decode_workspace_bytes(0, 10) == 0, "camera decoder workspace for zero width");
  expect(splat_camera_decode_workspace_bytes(1920, 1080) >= (size_t)1920 * 1080 * 32 * sizeof(float),
         "camera decoder workspace holds an activation map");
  expect(splat_mcmc_relocate_workspace_bytes(-3) == 0, "relocation workspace for negative n");
  expect(splat_mcmc_relocate_workspace_bytes(1) > 0 && splat_mcmc_relocate_workspace_bytes(1 << 21) >
                                                            splat_mcmc_relocate_workspace_bytes(1),
         "relocation workspace grows with n");
  expect(splat_set_adjoint_row_limit(-1) == SPLAT_ERR_INVALID_ARG, "negative adjoint row limit");
  expect(splat_set_adjoint_row_limit(SPLAT_ADJOINT_ROW_LIMIT) == SPLAT_OK, "default adjoint row limit");
  for (int code = -2; code <= 6; ++code) expect(splat_status_string(code) != nullptr, "status string");
  expect(strcmp(splat_status_string(SPLAT_ERR_CAPACITY), "capacity exceeded") == 0, "capacity status text");
}

static void check_argument_errors() {
  // every call below has an invalid argument the library detects before any device work
  expect(splat_project_camera(nullptr, nullptr, 0, 1, nullptr, nullptr, nullptr) == SPLAT_ERR_INVALID_ARG,
         "project without Gaussians");
  expect(splat_bin_sort_camera(nullptr, 0, 1, 10, nullptr, nullptr, nullptr, 0, nullptr, nullptr) ==
             SPLAT_ERR_INVALID_ARG,
         "bin/sort without a rig");
  expect(splat_rig_create(0, 0, nullptr) == SPLAT_ERR_INVALID_ARG, "rig without an output");
  SplatRig* rig = nullptr;
  expect(splat_rig_create(-1, 2, &rig) == SPLAT_ERR_INVALID_ARG, "rig with negative cameras");
  expect(splat_rig_create(SPLAT_MAX_SENSORS, 1, &rig) == SPLAT_ERR_INVALID_ARG, "rig beyond the sensor limit");
  SplatActors actors;
  memset(&actors, 0, sizeof(actors));
  actors.n = -1;
  expect(splat_compose(10, nullptr, nullptr, nullptr, nullptr, &actors, nullptr, nullptr, nullptr, nullptr) ==
             SPLAT_ERR_INVALID_ARG,
         "composition with a negative actor count");
  actors.n = SPLAT_COMPOSE_NOALLOC_MAX_ACTORS + 1;
  float dummy[16] __attribute__((aligned(16))) = {};
  int32_t ids[4] = {};
  SplatActorGrads dg;
  memset(&dg, 0, sizeof(dg));
  actors.rot = actors.trans = dummy;
  expect(splat_compose_bwd_noalloc(4, dummy, dummy, ids, &actors, dummy, dummy, dummy, dummy, dummy, nullptr, &dg,
                                   nullptr) == SPLAT_ERR_CAPACITY,
         "no-allocation composition adjoint beyond its actor limit");
  expect(splat_lidar_points_to_rays(-1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, nullptr) == SPLAT_ERR_INVALID_ARG,
         "points to rays with a negative count");
  expect(splat_mcmc_relocate(nullptr, nullptr, 0.005f, 51, nullptr, nullptr, nullptr, 0, nullptr) ==
             SPLAT_ERR_INVALID_ARG,
         "relocation without state");
}

int main() {
  check_cameras();
  check_lidars();
  check_sizes();
  check_argument_errors();
  printf("host abi checks: %d passed, %d failed\n", g_pass, g_fail);
  return g_fail == 0 ? 0 : 1;
}
