// api.hip -- the C ABI of libsplat (declared in include/splat.h): host-side validation, the rig
// (device sensor table), workspace sizing, and dispatch to the kernel launchers.
#include <atomic>
#include <new>
#include <string.h>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "rig_build.hpp"

using namespace splat;

struct SplatRig {
  int32_t n_cam = 0, n_lid = 0;
  DevSensor* d_table = nullptr;     // device copy, read by every kernel
  DevSensor* h_pinned = nullptr;    // pinned staging for asynchronous uploads
  std::vector<DevSensor> host;      // host copy used for launch configuration
  hipEvent_t uploaded = nullptr;
  // bin/sort's side stream (default priority) and its fork / join events
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // queue order of the last batched bin/sort per lists (keyed by the work buffer): true when it
  // grouped the items by kind, which the adjoint's two-loop kernel relies on
  mutable std::unordered_map<const void*, bool> grouped_queue;
  bool upload_pending = false;
  bool is_set = false;
  int n_cu = 0;                     // compute units of the rig's device (persistent grids)
  uint64_t layout_gen = 0;          // bumped when a launch-shaping field of any sensor changes
  SplatRigLayout layout;
};

// Fields that shape launches (grid sizes, buffer extents, validation); everything else a kernel
// reads from the device table at run time.
static bool same_layout(const DevSensor& a, const DevSensor& b) {
  return a.kind == b.kind && a.n_tiles == b.n_tiles && a.n_rays == b.n_rays && a.n_ch == b.n_ch &&
         a.feat_off == b.feat_off && a.st_x == b.st_x && a.st_y == b.st_y;
}

// one thread: the device's constant-rate wall clock at the point the stream reaches the launch
__global__ void k_device_clock(unsigned long long* dst) { *dst = (unsigned long long)wall_clock64(); }

extern "C" {

int splat_device_clock(unsigned long long* dst, void* stream) {
  if (!dst) return SPLAT_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_device_clock, dim3(1), dim3(1), 0, (hipStream_t)stream, dst);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

int splat_device_clock_hz(int64_t* hz) {
  if (!hz) return SPLAT_ERR_INVALID_ARG;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SPLAT_ERR_DEVICE;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return SPLAT_ERR_DEVICE;
  *hz = (int64_t)khz * 1000;
  return SPLAT_OK;
}

const char* splat_status_string(int code) {
  switch (code) {
    case SPLAT_OK: return "ok";
    case SPLAT_ERR_INVALID_ARG: return "invalid argument";
    case SPLAT_ERR_CAPACITY: return "capacity exceeded";
    case SPLAT_ERR_DEVICE: return "device error";
    case SPLAT_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

int splat_version(void) { return 1; }

int splat_check_camera(const SplatCamera* c) {
  if (!c) return SPLAT_ERR_INVALID_ARG;
  DevSensor d;
  return build_camera(*c, d);
}

int splat_check_lidar(const SplatLidar* l) {
  if (!l) return SPLAT_ERR_INVALID_ARG;
  DevSensor d;
  return build_lidar(*l, d);
}

int splat_rig_create(int32_t n_cameras, int32_t n_lidars, SplatRig** out) {
  if (!out || n_cameras < 0 || n_lidars < 0 || n_cameras + n_lidars <= 0 || n_cameras + n_lidars > SPLAT_MAX_SENSORS)
    return SPLAT_ERR_INVALID_ARG;
  *out = nullptr;
  SplatRig* r = new (std::nothrow) SplatRig();
  if (!r) return SPLAT_ERR_DEVICE;
  r->n_cam = n_cameras;
  r->n_lid = n_lidars;
  const int n = n_cameras + n_lidars;
  r->host.resize(n);
  size_t bytes = sizeof(DevSensor) * n;
  if (hipMalloc((void**)&r->d_table, bytes) != hipSuccess) { delete r; return SPLAT_ERR_DEVICE; }
  if (hipHostMalloc((void**)&r->h_pinned, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(r->d_table);
    delete r;
    return SPLAT_ERR_DEVICE;
  }
  if (hipEventCreateWithFlags(&r->uploaded, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(r->d_table);
    (void)hipHostFree(r->h_pinned);
    delete r;
    return SPLAT_ERR_DEVICE;
  }
  if (hipStreamCreateWithFlags(&r->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&r->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&r->join, hipEventDisableTiming) != hipSuccess) {
    splat_rig_destroy(r);
    return SPLAT_ERR_DEVICE;
  }
  memset(&r->layout, 0, sizeof(r->layout));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&r->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    r->n_cu = 0;
  *out = r;
  return SPLAT_OK;
}

void splat_rig_destroy(SplatRig* r) {
  if (!r) return;
  if (r->upload_pending) (void)hipEventSynchronize(r->uploaded);
  (void)hipEventDestroy(r->uploaded);
  if (r->join) (void)hipEventDestroy(r->join);
  if (r->fork) (void)hipEventDestroy(r->fork);
  if (r->side) (void)hipStreamDestroy(r->side);
  (void)hipFree(r->d_table);
  (void)hipHostFree(r->h_pinned);
  delete r;
}

int splat_rig_set(SplatRig* r, const SplatCamera* cams, const SplatLidar* lidars, void* stream) {
  if (!r) return SPLAT_ERR_INVALID_ARG;
  if ((r->n_cam > 0 && !cams) || (r->n_lid > 0 && !lidars)) return SPLAT_ERR_INVALID_ARG;
  const int n = r->n_cam + r->n_lid;
  std::vector<DevSensor> tab(n);
  for (int i = 0; i < r->n_cam; ++i)
    if (int rc = build_camera(cams[i], tab[i])) return rc;
  for (int i = 0; i < r->n_lid; ++i)
    if (int rc = build_lidar(lidars[i], tab[r->n_cam + i])) return rc;
  SplatRigLayout L;
  memset(&L, 0, sizeof(L));
  L.n_sensors = n;
  L.n_cameras = r->n_cam;
  int64_t st_base = 0;
  for (int i = 0; i < n; ++i) {
    tab[i].st_base = st_base;
    st_base += (int64_t)tab[i].st_x * tab[i].st_y;
    tab[i].tile_base = L.tile_base[i];
    tab[i].ray_base = L.ray_base[i];
    tab[i].feat_base = L.feat_base[i];
    L.tile_base[i + 1] = L.tile_base[i] + tab[i].n_tiles;
    L.ray_base[i + 1] = L.ray_base[i] + tab[i].n_rays;
    L.feat_base[i + 1] = L.feat_base[i] + tab[i].n_rays * tab[i].n_ch;
  }
  if (L.tile_base[n] >= ((int64_t)1 << 31) - 1 || L.ray_base[n] >= ((int64_t)1 << 31) - 1) return SPLAT_ERR_UNSUPPORTED;
  if (r->upload_pending && hipEventSynchronize(r->uploaded) != hipSuccess) return SPLAT_ERR_DEVICE;
  memcpy(r->h_pinned, tab.data(), sizeof(DevSensor) * n);
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(r->d_table, r->h_pinned, sizeof(DevSensor) * n, hipMemcpyHostToDevice, s) != hipSuccess)
    return SPLAT_ERR_DEVICE;
  if (hipEventRecord(r->uploaded, s) != hipSuccess) return SPLAT_ERR_DEVICE;
  r->upload_pending = true;
  bool same = r->is_set;
  for (int i = 0; same && i < n; ++i) same = same_layout(r->host[i], tab[i]);
  if (!same) ++r->layout_gen;
  r->host = tab;
  r->layout = L;
  r->is_set = true;
  return SPLAT_OK;
}

int splat_rig_layout(const SplatRig* r, SplatRigLayout* out) {
  if (!r || !out || !r->is_set) return SPLAT_ERR_INVALID_ARG;
  *out = r->layout;
  return SPLAT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// kind: kCamera / kLidar for the plain per-kind calls, -1 for the batched form (any mix)
static int make_view(const SplatRig* r, int32_t first, int32_t count, int kind, int64_t n_gauss, CallView& v) {
  if (!r || !r->is_set || count <= 0 || first < 0 || first + count > r->n_cam + r->n_lid || n_gauss < 0)
    return SPLAT_ERR_INVALID_ARG;
  v.sens = r->d_table + first;
  v.host = r->host.data() + first;
  v.count = count;
  v.n_gauss = n_gauss;
  v.n_tiles = 0;
  v.n_supertiles = 0;
  v.n_rays = 0;
  v.c_max = 0;
  v.has_lidar = false;
  v.ray_cap = false;
  v.lidar_ray0 = -1;
  v.lidar_tile0 = 0;
  for (int i = 0; i < count; ++i) {
    const DevSensor& d = v.host[i];
    if (kind >= 0 && d.kind != kind) return SPLAT_ERR_INVALID_ARG;
    if (d.kind == kLidar && !v.has_lidar) {
      v.has_lidar = true;
      v.lidar_ray0 = v.n_rays;
      v.lidar_tile0 = v.n_tiles;
    }
    v.ray_cap = v.ray_cap || (d.kind == kLidar && d.ray_prio != nullptr);
    v.n_tiles += d.n_tiles;
    v.n_supertiles += (int64_t)d.st_x * d.st_y;
    v.n_rays += d.n_rays;
    v.c_max = d.n_ch > v.c_max ? d.n_ch : v.c_max;
  }
  if (!v.has_lidar) {
    v.lidar_ray0 = v.n_rays;
    v.lidar_tile0 = v.n_tiles;
  }
  // a batched call over a single sensor runs that sensor's per-kind kernels: with one sensor the
  // queue has nothing to balance, and a plain grid walks the tiles in image order
  const bool single = kind < 0 && count == 1;
  v.lidar = (kind == kLidar) || (single && v.host[0].kind == kLidar);
  v.queue = kind < 0 && count > 1;
  v.n_cu = r->n_cu;
  v.side = r->side;
  v.fork = r->fork;
  v.join = r->join;
  if ((int64_t)count * n_gauss >= ((int64_t)1 << 32)) return SPLAT_ERR_UNSUPPORTED;
  // the capped ray sort keys are (lidar bin, 16-bit priority) in 32 bits
  if (v.ray_cap && v.n_tiles + 1 - v.lidar_tile0 > 65536) return SPLAT_ERR_UNSUPPORTED;
  return SPLAT_OK;
}

static int check_gaussians(const SplatGaussians* g, const CallView& v) {
  if (!g || g->n != v.n_gauss || g->n < 0) return SPLAT_ERR_INVALID_ARG;
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacities)) return SPLAT_ERR_INVALID_ARG;
  if (g->c_total < 0) return SPLAT_ERR_INVALID_ARG;
  for (int i = 0; i < v.count; ++i) {
    const DevSensor& d = v.host[i];
    if (d.n_ch > 0 && (d.feat_off + d.n_ch > g->c_total || (g->n > 0 && !g->features))) return SPLAT_ERR_INVALID_ARG;
  }
  if (((uintptr_t)g->quats & 15) != 0) return SPLAT_ERR_INVALID_ARG;   // read as float4 rows
  return SPLAT_OK;
}

static int check_proj(const SplatProjected* p, const CallView& v) {
  if (!p || p->n_records != (int64_t)v.count * v.n_gauss) return SPLAT_ERR_INVALID_ARG;
  if (p->n_records > 0 && (!p->mv || !p->cn || !p->box || !p->dv || !p->dkey || !p->rect || !p->n_tiles))
    return SPLAT_ERR_INVALID_ARG;
  if ((((uintptr_t)p->mv | (uintptr_t)p->cn | (uintptr_t)p->box | (uintptr_t)p->rect) & 15) != 0 ||
      (((uintptr_t)p->dv | (uintptr_t)p->dkey) & 7) != 0)
    return SPLAT_ERR_INVALID_ARG;
  return SPLAT_OK;
}

static int check_lists(const SplatTileLists* L, const CallView& v) {
  // list positions are 32-bit unsigned inside bin/sort: k_cap < 2^32
  if (!L || L->k_cap < 0 || L->k_cap >= ((int64_t)1 << 32)) return SPLAT_ERR_INVALID_ARG;
  if ((L->k_cap > 0 && !L->gauss) || !L->tile_range || !L->entry_base) return SPLAT_ERR_INVALID_ARG;
  if (((uintptr_t)L->tile_range & 15) != 0 || ((uintptr_t)L->entry_base & 7) != 0) return SPLAT_ERR_INVALID_ARG;
  if (v.has_lidar || v.queue) {
    if ((v.has_lidar && !L->ray_order) || !L->ray_range || !L->work || !L->n_work) return SPLAT_ERR_INVALID_ARG;
    if ((((uintptr_t)L->ray_range | (uintptr_t)L->work) & 7) != 0) return SPLAT_ERR_INVALID_ARG;
    if (L->work_cap < work_capacity(v.n_tiles, v.n_rays)) return SPLAT_ERR_INVALID_ARG;
  }
  return SPLAT_OK;
}

static int check_out(const SplatRenderOut* o, const CallView& v) {
  if (!o || !o->depth || !o->alpha || !o->t_final || !o->last) return SPLAT_ERR_INVALID_ARG;
  if (v.c_max > 0 && !o->feat) return SPLAT_ERR_INVALID_ARG;
  return SPLAT_OK;
}

static int dev_err(hipError_t e) { return e == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE; }

static int project_impl(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count, int kind,
                        const SplatProjected* out, SplatStatus* st, void* stream) {
  CallView v;
  int rc = make_view(r, first, count, kind, g ? g->n : -1, v);
  if (rc) return rc;
  if ((rc = check_gaussians(g, v)) || (rc = check_proj(out, v))) return rc;
  return dev_err(launch_project(v, *g, *out, st, (hipStream_t)stream));
}

static int bin_sort_impl(const SplatRig* r, int32_t first, int32_t count, int kind, int64_t n_gaussians,
                         const SplatProjected* proj, const SplatTileLists* lists, void* ws, size_t ws_bytes,
                         SplatStatus* st, void* stream) {
  CallView v;
  int rc = make_view(r, first, count, kind, n_gaussians, v);
  if (rc) return rc;
  if ((rc = check_proj(proj, v)) || (rc = check_lists(lists, v))) return rc;
  Workspace w = carve_workspace(nullptr, (int64_t)count * n_gaussians, lists->k_cap, v.n_tiles, v.n_rays, v.c_max);
  if (!ws || ws_bytes < w.bytes || ((uintptr_t)ws & 255) != 0) return SPLAT_ERR_INVALID_ARG;
  w = carve_workspace(ws, (int64_t)count * n_gaussians, lists->k_cap, v.n_tiles, v.n_rays, v.c_max);
  const int rc2 = dev_err(launch_bin_sort(v, *proj, *lists, w, st, (hipStream_t)stream));
  if (v.queue) r->grouped_queue[lists->work] = rc2 == SPLAT_OK && w.rows;
  else if (lists->work) r->grouped_queue.erase(lists->work);
  return rc2;
}

// Measurement hook (splat_time_next_raster): consumed by the next rasterise call of this thread.
static thread_local KernelTimer t_next_timer;

static KernelTimer take_timer() {
  KernelTimer t = t_next_timer;
  t_next_timer = KernelTimer();
  return t;
}

static int raster_fwd_impl(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count, int kind,
                           const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                           const SplatRenderOut* out, SplatStatus* st, void* stream) {
  CallView v;
  int rc = make_view(r, first, count, kind, g ? g->n : -1, v);
  if (rc) return rc;
  if (support != SPLAT_SUPPORT_BOX && support != SPLAT_SUPPORT_TILE) return SPLAT_ERR_INVALID_ARG;
  if ((rc = check_gaussians(g, v)) || (rc = check_proj(proj, v)) || (rc = check_lists(lists, v)) ||
      (rc = check_out(out, v)))
    return rc;
  return dev_err(launch_raster_fwd(v, *g, *proj, *lists, support, *out, st, (hipStream_t)stream, take_timer()));
}

// Largest k_cap whose adjoint keeps per-entry rows (process-wide, splat_set_adjoint_row_limit).
static std::atomic<int64_t> g_row_limit{SPLAT_ADJOINT_ROW_LIMIT};

namespace splat {
int64_t adjoint_row_limit() { return g_row_limit.load(); }
}  // namespace splat

// One launch clears what the adjoint accumulates into: the slot flags, the touched-record flags,
// the atomic part (where lidar tiles can be split, and for every record when the call keeps no
// rows), the queue counter and the long-record list counts.
static hipError_t adjoint_clears(const CallView& v, const Workspace& w, const SplatTileLists& L, int64_t n_gauss,
                                 hipStream_t s) {
  FillSegments f;
  if (w.rows) f.add(w.flags, div_up(L.k_cap, 4));
  f.add(w.rflag, div_up((int64_t)v.count * n_gauss, 4));
  if (v.has_lidar || !w.rows) {
    // with rows only lidar records (the call's last sensors) receive atomic parts, from the
    // items of split lidar tiles: zero theirs when bin_sort found such a tile (n_work[2])
    int k_lid = 0;
    while (w.rows && k_lid < v.count && v.host[k_lid].kind != kLidar) ++k_lid;
    f.add(w.g2d + (int64_t)k_lid * n_gauss * kNV, (int64_t)(v.count - k_lid) * n_gauss * kNV, 0u,
          w.rows ? L.n_work + 2 : nullptr);
  }
  f.add(w.qctr, 1);
  if (w.rows) f.add(w.n_long, kLongParts);
  return launch_fill_segments(f, s);
}

static int raster_bwd_impl(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count, int kind,
                           const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                           const SplatRenderOut* saved, const float* dF, const float* dD, const float* dA,
                           const SplatGrads* gr, void* ws, size_t ws_bytes, void* stream) {
  CallView v;
  int rc = make_view(r, first, count, kind, g ? g->n : -1, v);
  if (rc) return rc;
  if (support != SPLAT_SUPPORT_BOX && support != SPLAT_SUPPORT_TILE) return SPLAT_ERR_INVALID_ARG;
  if ((rc = check_gaussians(g, v)) || (rc = check_proj(proj, v)) || (rc = check_lists(lists, v))) return rc;
  if (!saved || !saved->t_final || !saved->last || !dD || !dA || (v.c_max > 0 && !dF)) return SPLAT_ERR_INVALID_ARG;
  if (!gr || !gr->means || !gr->log_scales || !gr->quats || !gr->opacities || (v.c_max > 0 && !gr->features))
    return SPLAT_ERR_INVALID_ARG;
  Workspace w = carve_workspace(nullptr, (int64_t)count * g->n, lists->k_cap, v.n_tiles, v.n_rays, v.c_max);
  if (!ws || ws_bytes < w.bytes || ((uintptr_t)ws & 255) != 0) return SPLAT_ERR_INVALID_ARG;
  w = carve_workspace(ws, (int64_t)count * g->n, lists->k_cap, v.n_tiles, v.n_rays, v.c_max);
  if (v.queue) {
    const auto q = r->grouped_queue.find(lists->work);
    v.queue_grouped = q != r->grouped_queue.end() && q->second;
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = adjoint_clears(v, w, *lists, g->n, s);
  if (e == hipSuccess)
    e = launch_raster_bwd(v, *g, *proj, *lists, support, *saved, dF, dD, dA, w, gr->features, gr->sensor_time_offset, s,
                          take_timer());
  if (e == hipSuccess) e = launch_project_bwd(v, *g, *proj, *lists, w, *gr, s);
  return dev_err(e);
}

extern "C" {

int splat_set_adjoint_row_limit(int64_t max_entries) {
  if (max_entries < 0) return SPLAT_ERR_INVALID_ARG;
  g_row_limit.store(max_entries);
  return SPLAT_OK;
}

size_t splat_workspace_bytes(const SplatRig* r, int32_t first, int32_t count, int64_t n_gaussians, int64_t k_cap) {
  CallView v;
  if (make_view(r, first, count, -1, n_gaussians, v) != SPLAT_OK || k_cap < 0) return 0;
  return carve_workspace(nullptr, (int64_t)count * n_gaussians, k_cap, v.n_tiles, v.n_rays, v.c_max).bytes;
}

int splat_project(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count, const SplatProjected* out,
                  SplatStatus* st, void* stream) {
  return project_impl(g, r, first, count, -1, out, st, stream);
}
int splat_bin_sort(const SplatRig* r, int32_t first, int32_t count, int64_t n_gaussians, const SplatProjected* proj,
                   const SplatTileLists* lists, void* ws, size_t ws_bytes, SplatStatus* st, void* stream) {
  return bin_sort_impl(r, first, count, -1, n_gaussians, proj, lists, ws, ws_bytes, st, stream);
}
int splat_rasterize_fwd(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                        const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                        const SplatRenderOut* out, SplatStatus* st, void* stream) {
  return raster_fwd_impl(g, r, first, count, -1, proj, lists, support, out, st, stream);
}
int splat_rasterize_bwd(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                        const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                        const SplatRenderOut* saved, const float* d_feat, const float* d_depth, const float* d_alpha,
                        const SplatGrads* grads, void* ws, size_t ws_bytes, void* stream) {
  return raster_bwd_impl(g, r, first, count, -1, proj, lists, support, saved, d_feat, d_depth, d_alpha, grads, ws,
                         ws_bytes, stream);
}

int splat_project_camera(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                         const SplatProjected* out, SplatStatus* st, void* stream) {
  return project_impl(g, r, first, count, kCamera, out, st, stream);
}
int splat_project_lidar(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                        const SplatProjected* out, SplatStatus* st, void* stream) {
  return project_impl(g, r, first, count, kLidar, out, st, stream);
}
int splat_bin_sort_camera(const SplatRig* r, int32_t first, int32_t count, int64_t n_gaussians,
                          const SplatProjected* proj, const SplatTileLists* lists, void* ws, size_t ws_bytes,
                          SplatStatus* st, void* stream) {
  return bin_sort_impl(r, first, count, kCamera, n_gaussians, proj, lists, ws, ws_bytes, st, stream);
}
int splat_bin_sort_lidar(const SplatRig* r, int32_t first, int32_t count, int64_t n_gaussians,
                         const SplatProjected* proj, const SplatTileLists* lists, void* ws, size_t ws_bytes,
                         SplatStatus* st, void* stream) {
  return bin_sort_impl(r, first, count, kLidar, n_gaussians, proj, lists, ws, ws_bytes, st, stream);
}
int splat_rasterize_fwd_camera(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                               const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                               const SplatRenderOut* out, SplatStatus* st, void* stream) {
  return raster_fwd_impl(g, r, first, count, kCamera, proj, lists, support, out, st, stream);
}
int splat_rasterize_fwd_lidar(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                              const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                              const SplatRenderOut* out, SplatStatus* st, void* stream) {
  return raster_fwd_impl(g, r, first, count, kLidar, proj, lists, support, out, st, stream);
}
int splat_rasterize_bwd_camera(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                               const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                               const SplatRenderOut* saved, const float* d_feat, const float* d_depth,
                               const float* d_alpha, const SplatGrads* grads, void* ws, size_t ws_bytes, void* stream) {
  return raster_bwd_impl(g, r, first, count, kCamera, proj, lists, support, saved, d_feat, d_depth, d_alpha, grads,
                         ws, ws_bytes, stream);
}
int splat_rasterize_bwd_lidar(const SplatGaussians* g, const SplatRig* r, int32_t first, int32_t count,
                              const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                              const SplatRenderOut* saved, const float* d_feat, const float* d_depth,
                              const float* d_alpha, const SplatGrads* grads, void* ws, size_t ws_bytes, void* stream) {
  return raster_bwd_impl(g, r, first, count, kLidar, proj, lists, support, saved, d_feat, d_depth, d_alpha, grads,
                         ws, ws_bytes, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Pipelines: one step captured into a hipGraph.
// ---------------------------------------------------------------------------------------------
struct SplatPipeline {
  const SplatRig* rig = nullptr;
  uint64_t layout_gen = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void pipeline_free(SplatPipeline* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
}

// The step's launches, in order, on `s` (validation included).
static int step_launches(const SplatRig* r, int32_t first, int32_t count, const SplatStep* st, hipStream_t s) {
  const bool bwd = (st->flags & SPLAT_STEP_BACKWARD) != 0;
  const SplatGaussians* g = &st->gaussians;
  if (st->status) {
    hipError_t e = launch_fill_i32((int32_t*)st->status, sizeof(SplatStatus) / 4, 0, s);
    if (e != hipSuccess) return dev_err(e);
  }
  if (bwd && (st->flags & SPLAT_STEP_ZERO_GRADS)) {   // the gradient accumulators, one launch
    const SplatGrads& gr = st->grads;
    const int64_t n = g->n;
    if (!gr.means || !gr.log_scales || !gr.quats || !gr.opacities) return SPLAT_ERR_INVALID_ARG;
    FillSegments f;
    f.add(gr.means, 3 * n);
    f.add(gr.log_scales, 3 * n);
    f.add(gr.quats, 4 * n);
    f.add(gr.opacities, n);
    f.add(gr.velocities, 3 * n);
    f.add(gr.features, n * g->c_total);
    hipError_t e = launch_fill_segments(f, s);
    if (e != hipSuccess) return dev_err(e);
  }
  int rc = project_impl(g, r, first, count, -1, &st->proj, st->status, s);
  if (!rc) rc = bin_sort_impl(r, first, count, -1, g->n, &st->proj, &st->lists, st->ws, st->ws_bytes, st->status, s);
  SplatStatus* const fwd_status = (st->flags & SPLAT_STEP_COUNT_PAIRS) ? st->status : nullptr;
  if (!rc) rc = raster_fwd_impl(g, r, first, count, -1, &st->proj, &st->lists, st->support, &st->out, fwd_status, s);
  if (!rc && bwd)
    rc = raster_bwd_impl(g, r, first, count, -1, &st->proj, &st->lists, st->support, &st->out, st->d_feat,
                         st->d_depth, st->d_alpha, &st->grads, st->ws, st->ws_bytes, s);
  return rc;
}

extern "C" {

int splat_time_next_raster(void* start_event, void* stop_event) {
  if ((start_event == nullptr) != (stop_event == nullptr)) return SPLAT_ERR_INVALID_ARG;
  t_next_timer.start = (hipEvent_t)start_event;
  t_next_timer.stop = (hipEvent_t)stop_event;
  return SPLAT_OK;
}

int splat_pipeline_create(const SplatRig* r, int32_t first, int32_t count, const SplatStep* step,
                          SplatPipeline** out) {
  if (!out || !step) return SPLAT_ERR_INVALID_ARG;
  t_next_timer = KernelTimer();   // no event records inside a captured graph
  *out = nullptr;
  CallView v;
  int rc = make_view(r, first, count, -1, step->gaussians.n, v);
  if (rc) return rc;
  SplatPipeline* p = new (std::nothrow) SplatPipeline();
  if (!p) return SPLAT_ERR_DEVICE;
  p->rig = r;
  p->layout_gen = r->layout_gen;
  if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
    pipeline_free(p);
    return SPLAT_ERR_DEVICE;
  }
  if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    pipeline_free(p);
    return SPLAT_ERR_DEVICE;
  }
  rc = step_launches(r, first, count, step, p->cap);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(p->cap, &graph);
  p->graph = graph;
  if (rc == SPLAT_OK && ec != hipSuccess) rc = SPLAT_ERR_DEVICE;
  if (rc == SPLAT_OK && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = SPLAT_ERR_DEVICE;
  // move the graph's launch setup to creation time instead of the first run
  if (rc == SPLAT_OK && (hipGraphUpload(p->exec, p->cap) != hipSuccess || hipStreamSynchronize(p->cap) != hipSuccess))
    rc = SPLAT_ERR_DEVICE;
  if (rc != SPLAT_OK) {
    pipeline_free(p);
    return rc;
  }
  *out = p;
  return SPLAT_OK;
}

int splat_pipeline_run(SplatPipeline* p, void* stream) {
  if (!p) return SPLAT_ERR_INVALID_ARG;
  if (p->rig->layout_gen != p->layout_gen) return SPLAT_ERR_INVALID_ARG;
  return dev_err(hipGraphLaunch(p->exec, (hipStream_t)stream));
}

void splat_pipeline_destroy(SplatPipeline* p) { pipeline_free(p); }

}  // extern "C"
