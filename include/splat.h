/*
 * splat.h -- C ABI of libsplat: a differentiable, tile-based Gaussian rasterizer for cameras
 * and spinning lidars on AMD Instinct MI355X (gfx950).
 *
 * The operation is the rendering core of SplatAD (arXiv 2411.16816):
 *   - Gaussians with opacity o, mean mu, covariance from scale + quaternion, and features
 *     (Sec. 3.1) are projected into a camera image plane (Sec. 3.2) or into lidar spherical
 *     coordinates (azimuth, elevation, range) (Sec. 3.3, Eq. spherical_projection),
 *     with rolling-shutter velocities (Eq. pixel_velocity, App. D and the lidar v^S);
 *   - binned into tiles (16x16 pixels in the paper; lidar tiles of N_phi azimuth steps by
 *     N_omega channels, App. A) and depth-sorted per tile (z for cameras, range for lidar);
 *   - alpha-composited front to back per pixel or per supplied lidar ray (Eqs. t_pix,
 *     alpha_blend, alpha, delta), also blending depth / rolling-shutter corrected range and
 *     opacity, with an optional median range (Sec. 3.3);
 *   - differentiated by a hand-written adjoint (Sec. 3.4, "Implementation").
 *
 * Conventions for every call
 *   - Return value: SPLAT_OK or an error code; no C++ exception crosses the ABI.  Arguments are
 *     validated on the host before anything is launched; an invalid call launches nothing.
 *   - All array pointers inside SplatGaussians, SplatProjected, SplatTileLists, SplatRenderOut
 *     and SplatGrads are DEVICE pointers owned by the caller (float32 row-major, int32 indices,
 *     int64 offsets).  Host structs themselves are read during the call only.
 *   - Every call is stream-ordered and asynchronous on `stream` (a hipStream_t, NULL = default
 *     stream).  No call synchronises the host or allocates device memory, so every call may be
 *     captured into a hipGraph.  Scratch memory comes from a caller-provided workspace.
 *   - Asynchronous conditions (intersection overflow, non-finite Gaussians, invalid rays) are
 *     recorded in a caller-provided device SplatStatus; read it after the stream completes.
 *   - Inputs are never modified.  Gradients are ACCUMULATED (+=) into SplatGrads.
 *   - A call covers the sensors [first, first + count) of a rig.  Such a call is self-contained:
 *     its records, tile ids, ray ids and outputs are numbered from the first sensor of the call
 *     ("local" numbering), so one-sensor calls (plain mode) and all-sensor calls (batched mode)
 *     use the same layout rules.  SplatRigLayout gives every offset.
 */
#ifndef SPLAT_H_
#define SPLAT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPLAT_OK 0
#define SPLAT_ERR_INVALID_ARG 1
#define SPLAT_ERR_CAPACITY 2
#define SPLAT_ERR_DEVICE 3
#define SPLAT_ERR_UNSUPPORTED 4

#define SPLAT_MAX_EL_TILES 64         /* lidar elevation tiles (M_omega) per sensor */
#define SPLAT_MAX_SENSORS 1024        /* sensors per rig */
#define SPLAT_MAX_CHANNELS 48         /* blended feature channels per sensor */
#define SPLAT_RAYS_PER_ITEM 256       /* lidar rays per rasterisation work item (App. A) */

/* candidate rule of the rasterisers */
#define SPLAT_SUPPORT_BOX 0   /* Gaussians whose 3-sigma + rolling-shutter box contains the ray */
#define SPLAT_SUPPORT_TILE 1  /* every Gaussian listed for the ray's tile (paper-literal) */

/* Status written by the device.  Zero it before a sequence of calls; fields accumulate. */
typedef struct SplatStatus {
  unsigned long long n_isect;     /* intersections (tile, Gaussian) of the last bin/sort      */
  unsigned long long k_cap;       /* capacity the last bin/sort was given                      */
  unsigned int overflow;          /* non-zero if n_isect exceeded k_cap (lists left empty)     */
  unsigned int n_nonfinite;       /* (Gaussian, sensor) projections culled because of non-finite
                                     values: a non-finite sensor-frame mean, or a non-finite
                                     projected mean, velocity, conic, o_eff, box or depth of a
                                     Gaussian inside the depth / range limits                   */
  unsigned int n_rays_invalid;    /* lidar rays outside [0, 2pi) x [b_0, b_M): output zeros    */
  unsigned int n_rays_time;       /* lidar rays with |t| > t_rs / 2 (still rendered)           */
  unsigned long long n_pairs;     /* (ray, Gaussian) pairs the forward rasterisers evaluated
                                     (box test passed, alpha computed); counted when the
                                     forward call is given a status                          */
  unsigned long long n_stopped;   /* rays whose walk ended early because the next blend would
                                     take the transmittance below 1e-4; counted with n_pairs */
} SplatStatus;

/* Gaussians (Sec. 3.1).  Device arrays. */
typedef struct SplatGaussians {
  int64_t n;
  const float* means;       /* [n,3] world frame                                              */
  const float* log_scales;  /* [n,3] scale = exp(log_scale)                                   */
  const float* quats;       /* [n,4] (w,x,y,z), normalised inside                             */
  const float* opacities;   /* [n]   in (0,1)                                                  */
  const float* velocities;  /* [n,3] world-frame velocity of each Gaussian, or NULL (zero)     */
  const float* features;    /* [n,c_total] base colour and features                           */
  int32_t c_total;
} SplatGaussians;

/* Pinhole camera (Sec. 3.2).  x_c = R x_w + t with x right, y down, z forward.  Velocities are
 * in the camera frame.  t_rs is the rolling-shutter time between first and last row; pixel
 * row v is captured at t = ((v + 1/2) / height - 1/2) t_rs (Eq. t_pix, pixel centres). */
typedef struct SplatCamera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float lin_vel[3];
  float ang_vel[3];
  float t_rs;
  float eps2d;       /* EWA dilation s of Eq. alpha (0.3 in the paper)                           */
  float near_plane;  /* cull z <= near_plane                                                    */
  float far_plane;   /* cull z >= far_plane                                                     */
  float jac_clamp;   /* x/z, y/z clamped to +-jac_clamp * (size/2)/f inside J (0 = off)        */
  int32_t feat_offset, n_channels;  /* blended feature columns [offset, offset + n_channels)   */
  int32_t tile_w, tile_h;           /* pixels per tile; tile_w * tile_h <= 256, both >= 1      */
  float time_offset; /* [s] camera timestamp minus the middle of the exposure (Sec. 3.2): pixel
                        row times are (p_v / H - 1/2) t_rs + time_offset, and the rolling-shutter
                        box is centred on the mean at time_offset.  0 = centred exposure.    */
} SplatCamera;

/* Spinning lidar (Sec. 3.3, App. A).  x_l = R x_w + t with x forward, y left, z up.
 * Azimuth tiles are tile_az * az_res wide and there are n_az_tiles of them (M_phi, with
 * M_phi * tile_az * az_res >= 2 pi); elevation tiles are [elev_bounds[k], elev_bounds[k+1]).
 * Rays are supplied (azimuth in [0, 2pi), elevation, time relative to the middle of the sweep). */
typedef struct SplatLidar {
  float R[9];
  float t[3];
  float lin_vel[3];
  float ang_vel[3];
  float t_rs;        /* sweep duration                                                         */
  float eps2d;       /* dilation in rad^2                                                      */
  float r_min, r_max;
  float az_res;      /* azimuth step [rad]                                                     */
  int32_t tile_az;   /* N_phi                                                                  */
  int32_t n_az_tiles;/* M_phi                                                                  */
  int32_t n_el_tiles;/* M_omega (<= SPLAT_MAX_EL_TILES)                                        */
  const float* elev_bounds;  /* HOST array [n_el_tiles + 1], strictly increasing [rad]          */
  int64_t n_rays;
  const float* ray_az;       /* device [n_rays] */
  const float* ray_el;       /* device [n_rays] */
  const float* ray_t;        /* device [n_rays] */
  int32_t feat_offset, n_channels;
  const float* ray_range;    /* device [n_rays] measured range of each ray, or NULL: enables the
                                line-of-sight sum (training-details appendix, loss term L_los)  */
  float los_eps;             /* line-of-sight margin [m] (0.8 in the paper), >= 0               */
  const uint16_t* ray_priority;  /* device [n_rays] or NULL.  Non-NULL selects the training-time
                                cap of App. A: a tile renders at most SPLAT_RAYS_PER_ITEM rays,
                                those of smallest priority (ties: smaller ray index); its other
                                rays are dropped (SplatRenderOut.dropped): they get the outputs of
                                a ray that meets no Gaussian and their upstream gradients are
                                ignored.  Fresh uniform priorities each step shuffle the rays.
                                NULL: every ray is rendered (a crowded tile takes several work
                                items).  A call with any such lidar supports at most 65535 lidar
                                tiles (SPLAT_ERR_UNSUPPORTED otherwise).                        */
} SplatLidar;

/* Opaque rig: a device-resident table of sensors (cameras first, then lidars). */
typedef struct SplatRig SplatRig;

/* Offsets of every sensor in the rig's global numbering (host copy). */
typedef struct SplatRigLayout {
  int32_t n_sensors;       /* n_cameras + n_lidars; sensor s < n_cameras is a camera          */
  int32_t n_cameras;
  int64_t tile_base[SPLAT_MAX_SENSORS + 1];      /* first tile of each sensor; [n] = total      */
  int64_t ray_base[SPLAT_MAX_SENSORS + 1];       /* first ray (pixel) of each sensor           */
  int64_t feat_base[SPLAT_MAX_SENSORS + 1];      /* first float of each sensor's feature rows  */
} SplatRigLayout;

/* Projected records, one per (sensor, Gaussian): record = (s - first) * n + gaussian.
 * Device arrays, caller-allocated with count * n records. */
typedef struct SplatProjected {
  int64_t n_records;
  float* mv;        /* [n_records,4] mean (u,v) | (phi,omega), and its velocity               */
  float* cn;        /* [n_records,4] conic (a,b,c) of (Sigma + sI)^-1 = [[a,b],[b,c]], o_eff    */
  float* box;       /* [n_records,4] lo_u, lo_v, hi_u, hi_v of the 3-sigma + RS box          */
  float* dv;        /* [n_records,2] depth (z | range) and range velocity (lidar; 0 camera)    */
  unsigned long long* dkey; /* [n_records] IEEE bits of the depth (z | range) evaluated in
                       float64 from the float32 inputs.  Gaussians are ordered by the 32-bit
                       key (e << 27) | (mantissa >> 25), e = binary exponent + 16 clamped to
                       [0, 31] (key 0 below 2^-16, all ones from 2^16 on): 2^-27 relative
                       resolution (a float32 depth has 2^-24); equal keys keep Gaussian-id
                       order                                                                */
  int32_t* rect;    /* [n_records,4] tiles: camera (x0, y0, nx, ny); lidar (az0, el0, naz, nel) */
  int32_t* n_tiles; /* [n_records] tiles touched (0 = culled)                                 */
} SplatProjected;

/* Per-tile depth-ordered lists.  Tile ids are local to the call. */
typedef struct SplatTileLists {
  int64_t k_cap;          /* capacity of gauss[], 0 <= k_cap < 2^32                           */
  int32_t* gauss;         /* [k_cap] Gaussian ids, grouped by tile, by (depth, id) inside      */
  int64_t* tile_range;    /* [n_tiles, 2] [start, end) into gauss (16-byte aligned)           */
  int64_t* entry_base;    /* [count * N] written by bin_sort for records with n_tiles > 0:
                             the number of the record's first (tile, Gaussian) entry.  Entries
                             are numbered record by record in record order, each record's tiles
                             in the row-major order of its rectangle, so record r owns the
                             numbers [entry_base[r], entry_base[r] + n_tiles[r]).  The adjoint
                             keeps one gradient row per entry number in its workspace.         */
  /* lidar only (NULL for camera calls): */
  int32_t* ray_order;     /* [n_rays] local ray ids grouped by tile (invalid rays last)         */
  int32_t* ray_range;     /* [n_tiles + 1, 2] [start, end) into ray_order; entry n_tiles =
                             invalid rays                                                      */
  int32_t* work;          /* [work_cap, 2] work items (tile, first position in ray_order; camera
                             tiles of a batched call are items (tile, 0))                       */
  int32_t* n_work;        /* [3] number of work items; queue counter of the persistent kernels;
                             1 when a lidar tile of the call has more than SPLAT_RAYS_PER_ITEM
                             rays (its items add their gradients atomically), else 0          */
  int64_t work_cap;       /* >= n_tiles + ceil(n_rays / 256) + 1                               */
} SplatTileLists;

/* Rendered outputs (local ray numbering).  feat rows are n_channels of the ray's sensor. */
typedef struct SplatRenderOut {
  float* feat;      /* [sum_s rays_s * C_s]                                                   */
  float* depth;     /* [n_rays] blended z (camera) or RS-corrected range (lidar)              */
  float* alpha;     /* [n_rays] 1 - T_final                                                   */
  float* t_final;   /* [n_rays] final transmittance (saved for the adjoint)                   */
  int32_t* last;    /* [n_rays] 1 + position in the tile list of the last blended Gaussian    */
  float* median;    /* [n_rays] median range of lidar rays (camera rays: not written) or NULL */
  unsigned long long* sensor_done;  /* [count] or NULL: for latency measurement, each sensor's
                       entry is raised (atomic max) to the device wall clock (splat_device_clock
                       ticks) when a work item of that sensor finishes in a rasteriser call
                       given this struct (the forward's `out`, or the adjoint's `saved`); the
                       caller zeroes it.  Items of lidar rays outside every tile are not timed. */
  float* los;       /* [n_rays] or NULL: lidar rays' line-of-sight sum, the alphas of the Gaussians
                       the ray blends whose corrected range r + v_r t is below ray_range - los_eps
                       (0 without ray_range; camera rays: not written)                         */
  const float* d_los;  /* [n_rays] or NULL: upstream gradient of `los`, read by the adjoint from
                       its `saved` struct (NULL = zero)                                          */
  uint8_t* dropped; /* [n_rays] or NULL: 1 for lidar rays dropped by the training-time cap
                       (SplatLidar.ray_priority), else 0; written by the forward for lidar rays
                       (camera rays: not written)                                              */
} SplatRenderOut;

/* Gradient accumulators (+=), device arrays shaped like SplatGaussians. */
typedef struct SplatGrads {
  float* means;       /* [n,3] */
  float* log_scales;  /* [n,3] */
  float* quats;       /* [n,4] */
  float* opacities;   /* [n]   */
  float* velocities;  /* [n,3] or NULL */
  float* features;    /* [n,c_total] */
  /* Sensor parameters of the call's sensors [first, first + count) (index k = sensor - first),
   * accumulated (+=) when non-NULL: */
  float* sensor_lin_vel;      /* [count,3] dL/d lin_vel (sensor frame)                          */
  float* sensor_ang_vel;      /* [count,3] dL/d ang_vel (sensor frame)                          */
  float* sensor_time_offset;  /* [count] dL/d time_offset of cameras (lidar entries untouched)  */
} SplatGrads;

const char* splat_status_string(int code);
int splat_version(void);

/* Host-only validation of one sensor description (no device call): SPLAT_OK,
 * SPLAT_ERR_INVALID_ARG, or SPLAT_ERR_UNSUPPORTED for a valid sensor beyond the kernels'
 * limits: more than 65535 tiles across a row (camera tiles_x, lidar n_az_tiles) or 2^24 tiles
 * or more in total.  splat_rig_set applies the same checks and returns the same codes. */
int splat_check_camera(const SplatCamera* cam);
int splat_check_lidar(const SplatLidar* lidar);

/* ---- rig -------------------------------------------------------------------------------
 * splat_rig_create allocates the rig's device table, and a second stream (default priority)
 * with two events on the current device, onto which bin/sort forks the ray binning for the
 * length of the call (not a hot-path call).  One rig's calls are issued from one host thread
 * at a time: they share that stream and those events.  splat_rig_set
 * validates the sensors on the host and uploads them asynchronously on `stream` from pinned
 * host memory (it waits only for the rig's previous upload).  Cameras get sensor ids
 * 0..n_cameras-1, lidars n_cameras..n_cameras+n_lidars-1. */
int splat_rig_create(int32_t n_cameras, int32_t n_lidars, SplatRig** out);
int splat_rig_set(SplatRig* rig, const SplatCamera* cams, const SplatLidar* lidars, void* stream);
int splat_rig_layout(const SplatRig* rig, SplatRigLayout* out);
void splat_rig_destroy(SplatRig* rig);

/* Workspace bytes needed by any call on sensors [first, first+count) of `rig` with
 * `n_gaussians` Gaussians and list capacity k_cap.  The bin/sort buffers and the adjoint's
 * buffers overlay each other; the adjoint's part is one gradient row per list entry
 * (k_cap x (10 + channel bucket) floats, channel buckets 4/8/16/32/48, rows padded to 16 bytes),
 * k_cap flag bytes and 10 floats per record — without the rows and flags when k_cap exceeds
 * the adjoint row limit (splat_set_adjoint_row_limit).  Nothing in it outlives a call. */
size_t splat_workspace_bytes(const SplatRig* rig, int32_t first, int32_t count, int64_t n_gaussians,
                             int64_t k_cap);

/* The adjoint keeps one gradient row per list entry as long as the call's k_cap is at most
 * this many entries (default SPLAT_ADJOINT_ROW_LIMIT: about 60 GB of rows at 16 channels);
 * larger calls (a whole sensor sweep in one call) keep none: every work item adds its
 * per-Gaussian sums to the record's gradient with float atomics, whose rounding then depends
 * on scheduling.  Process-wide; the same limit must hold from splat_workspace_bytes to the
 * adjoint call that uses the workspace.  For memory-bound callers and tests.  Negative:
 * SPLAT_ERR_INVALID_ARG. */
#define SPLAT_ADJOINT_ROW_LIMIT (1LL << 29)
int splat_set_adjoint_row_limit(int64_t max_entries);

/* ---- a1 / a2: projection (Sec. 3.2 "Projection, tiling, and sorting", "Rolling shutter";
 * Sec. 3.3 "Projection"; App. D).  Per (Gaussian, sensor): sensor-frame mean and covariance,
 * projected mean, J Sigma J^T, RS velocity J(-w x mu - v + R v_g), dilation, conic,
 * o_eff = o sqrt(det(Sigma2) / det(Sigma2 + sI)), box = mean +- (3 sqrt(diag(Sigma2 + sI)) +
 * |v| t_rs / 2), culling (depth / range limits, box outside the image or elevation span,
 * o_eff < 1/255, non-finite) and the tile rectangle.  Culled records get n_tiles = 0 and no
 * other field; non-finite projections are counted in status->n_nonfinite (status may be NULL).
 * Sensors of the call must be all cameras (resp. all lidars). */
int splat_project_camera(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                         const SplatProjected* out, SplatStatus* status, void* stream);
int splat_project_lidar(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                        const SplatProjected* out, SplatStatus* status, void* stream);

/* ---- a3 / a4: tile binning + depth sort (Sec. 3.2; Sec. 3.3 "Tiling and sorting"; App. A).
 * Orders records by depth (stable, so equal depths keep Gaussian-id order) and writes, for
 * every tile, the ids of the Gaussians whose rectangle contains it in that order (the order
 * of a stable (tile | depth) key sort) with per-tile [start, end) ranges into gauss.  The
 * lists of different tiles are laid out in an order of the library's choosing (tile_range
 * says where each is).  The lidar variant also bins the supplied rays into their tiles (a ray
 * is a box of zero extent, App. A) and cuts every tile's rays into work items of <= 256 rays;
 * that part reads no Gaussian data and runs on the rig's second stream, forked from `stream`
 * at the start of the call and joined back before it ends (graph capture included).
 * More than k_cap (tile, Gaussian) pairs: every list is left empty (memory-safe),
 * status->overflow is set and status->n_isect holds the needed capacity. */
int splat_bin_sort_camera(const SplatRig* rig, int32_t first, int32_t count, int64_t n_gaussians,
                          const SplatProjected* proj, const SplatTileLists* lists, void* ws,
                          size_t ws_bytes, SplatStatus* status, void* stream);
int splat_bin_sort_lidar(const SplatRig* rig, int32_t first, int32_t count, int64_t n_gaussians,
                         const SplatProjected* proj, const SplatTileLists* lists, void* ws,
                         size_t ws_bytes, SplatStatus* status, void* stream);

/* ---- a5 / a6: rasterisation forward (Eqs. t_pix, alpha_blend, alpha, delta; Sec. 3.3 for
 * the range blend r + v_r t and the median).  alpha = min(0.99, o_eff exp(-sigma)); alpha <
 * 1/255 is skipped; blending stops before a Gaussian that would take T below 1e-4. */
int splat_rasterize_fwd_camera(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                               const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                               const SplatRenderOut* out, SplatStatus* status, void* stream);
int splat_rasterize_fwd_lidar(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                              const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                              const SplatRenderOut* out, SplatStatus* status, void* stream);

/* ---- a8: batched form.  The same four steps for any mix of the rig's sensors in one call
 * (cameras and lidars together): one projection launch reading every Gaussian once for all
 * sensors; one bin/sort over every sensor's tiles that also builds a global work queue of
 * camera tiles and lidar ray chunks (the lidar chunks first, then the camera tiles, each part
 * ordered by descending list length); and persistent rasterisers (forward and adjoint) whose
 * workgroups drain that queue.  A call over a single sensor (count == 1) runs that sensor's
 * per-kind kernels instead (no queue; work holds lidar chunks only, as in the per-kind call).
 * Lists need ray_order (if any lidar), ray_range, work and n_work.  Results are bit-identical
 * to the per-sensor calls (BOX support).  Gradients agree with the per-sensor calls to float
 * rounding: a workgroup adds its wavefronts' partial sums in LDS in scheduling order. */
int splat_project(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                  const SplatProjected* out, SplatStatus* status, void* stream);
int splat_bin_sort(const SplatRig* rig, int32_t first, int32_t count, int64_t n_gaussians,
                   const SplatProjected* proj, const SplatTileLists* lists, void* ws, size_t ws_bytes,
                   SplatStatus* status, void* stream);
int splat_rasterize_fwd(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                        const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                        const SplatRenderOut* out, SplatStatus* status, void* stream);
int splat_rasterize_bwd(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                        const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                        const SplatRenderOut* saved, const float* d_feat, const float* d_depth,
                        const float* d_alpha, const SplatGrads* grads, void* ws, size_t ws_bytes, void* stream);

/* ---- a7: rasterisation backward + projection adjoint.  Walks each ray's list back to front
 * from `last`, recovering T_i = T_{i+1} / (1 - alpha_i) from the saved T_final.  A work item
 * sums each Gaussian's gradient over its rays (wavefront, then workgroup) and stores it as one
 * row per (tile, Gaussian) entry at the entry's number (see entry_base); work items
 * of a lidar tile with more than SPLAT_RAYS_PER_ITEM rays share the tile and add atomically
 * instead, and so do all work items of a call beyond the adjoint row limit
 * (splat_set_adjoint_row_limit).  Each record's rows are then summed in a fixed order and chained to means,
 * log-scales, quaternions, opacities, velocities and features.  Needs the lists written by
 * bin_sort for the same projection.  d_feat / d_depth / d_alpha are the upstream gradients of
 * SplatRenderOut feat/depth/alpha. */
int splat_rasterize_bwd_camera(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                               const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                               const SplatRenderOut* saved, const float* d_feat, const float* d_depth,
                               const float* d_alpha, const SplatGrads* grads, void* ws, size_t ws_bytes,
                               void* stream);
int splat_rasterize_bwd_lidar(const SplatGaussians* g, const SplatRig* rig, int32_t first, int32_t count,
                              const SplatProjected* proj, const SplatTileLists* lists, int32_t support,
                              const SplatRenderOut* saved, const float* d_feat, const float* d_depth,
                              const float* d_alpha, const SplatGrads* grads, void* ws, size_t ws_bytes,
                              void* stream);

/* ---- a8: one step captured as a hipGraph.  A pipeline records, for the sensors
 * [first, first + count) of a rig, the launches of one step of the batched form: zero *status
 * (fill kernel), zero the gradients (if SPLAT_STEP_ZERO_GRADS), splat_project, splat_bin_sort,
 * splat_rasterize_fwd and, with SPLAT_STEP_BACKWARD, splat_rasterize_bwd, all on the buffers of
 * `step` (validated at creation exactly as those calls validate them).  The forward is given
 * the status (and so counts evaluated pairs, a slower walk) only with SPLAT_STEP_COUNT_PAIRS;
 * projection and bin/sort always report into it.  splat_pipeline_run
 * launches the graph on `stream`: one host call per step instead of one per kernel.
 *   - Graph kernels read the sensor table at run time, so poses, velocities, shutter times and
 *     ray arrays may change between runs through splat_rig_set on the same stream.  A change of
 *     any sensor's kind, tile count, ray count, channel count or feature offset invalidates the
 *     pipeline: splat_pipeline_run then returns SPLAT_ERR_INVALID_ARG and launches nothing.
 *   - The buffers of `step` are captured by address: they must stay allocated, and their
 *     contents are read/written by every run (inputs may change between runs).
 *   - The graph holds no memset node (zeroing uses fill kernels) and allocates nothing.
 *   - Creating a pipeline captures on an internal stream and instantiates the graph; it is not a
 *     hot-path call.  Runs of one pipeline on different streams must not overlap. */
/* ---- measurement hook.  The next splat_rasterize_fwd* or splat_rasterize_bwd* call made by
 * the calling host thread records hipEvent_t `start_event` on its stream right before its
 * rasteriser kernel and `stop_event` right after it (not around the zero fills or, in the
 * adjoint, the gradient sums and the projection adjoint), then forgets them.  Both NULL
 * clears a pending request; exactly one NULL is SPLAT_ERR_INVALID_ARG.  Creating a pipeline
 * clears it too (graphs hold no event records).  For benchmarks: per-kernel time without a
 * profiler. */
int splat_time_next_raster(void* start_event, void* stop_event);

#define SPLAT_STEP_BACKWARD 1    /* include the adjoint                                   */
#define SPLAT_STEP_ZERO_GRADS 2  /* zero every gradient array first (else they accumulate) */
#define SPLAT_STEP_COUNT_PAIRS 4 /* the forward counts evaluated pairs into status->n_pairs  */

typedef struct SplatStep {
  SplatGaussians gaussians;
  SplatProjected proj;
  SplatTileLists lists;
  SplatRenderOut out;        /* forward outputs; the saved state of the adjoint              */
  int32_t support;           /* SPLAT_SUPPORT_BOX or SPLAT_SUPPORT_TILE                      */
  int32_t flags;             /* SPLAT_STEP_*                                                 */
  const float* d_feat;       /* upstream gradients (backward only)                           */
  const float* d_depth;
  const float* d_alpha;
  SplatGrads grads;          /* accumulated (backward only)                                  */
  void* ws;                  /* workspace of splat_workspace_bytes(rig, first, count, n, k_cap) */
  size_t ws_bytes;
  SplatStatus* status;       /* zeroed at the start of every run; may be NULL                */
} SplatStep;

typedef struct SplatPipeline SplatPipeline;

int splat_pipeline_create(const SplatRig* rig, int32_t first, int32_t count, const SplatStep* step,
                          SplatPipeline** out);
int splat_pipeline_run(SplatPipeline* pipeline, void* stream);
void splat_pipeline_destroy(SplatPipeline* pipeline);

/* ---- device clock, for latency measurement: splat_device_clock writes the device's
 * constant-rate wall clock to *dst (device memory) when the stream reaches the call (one tiny
 * kernel); splat_device_clock_hz gives its rate in ticks per second for the current device. */
int splat_device_clock(unsigned long long* dst, void* stream);
int splat_device_clock_hz(int64_t* hz);

/* ---- scene-graph composition at a capture time (Sec. 3.1 "Scene representation"; the actor
 * velocity term of Eq. pixel_velocity, Sec. 3.2, and App. D "Rolling shutter details").
 * The scene is a static background plus rigid actors.  Gaussian i with actor_id[i] = a in
 * [0, n) holds its mean and rotation in the frame of actor a's box; composing writes the
 * world-frame arrays that the projection calls read (SplatGaussians.means / quats / velocities):
 *     mu_w = R_a mu + t_a,     q_w = q_a (x) q,     v_w = R_a (w_a x mu + v_a)
 * with q_a = q_b (x) dq / |dq| (q_b normalised; the rotation offset acts in the actor frame),
 * R_a = R(q_a), t_a = t_b + dt (world frame), v_a = v_b + dv and w_a in the actor frame, and
 * (x) the Hamilton product (R(a (x) b) = R(a) R(b)).  Gaussians with a negative id, or an id
 * >= n, are static background: mean and rotation are copied, and the world velocity is the
 * input velocity (zero when `velocities` is NULL).  All arrays are device arrays; quaternion
 * arrays must be 16-byte aligned (SPLAT_ERR_INVALID_ARG otherwise). */
typedef struct SplatActors {
  int32_t n;                    /* actors                                                     */
  const float* rot;             /* [n,4] base rotation q_b (w,x,y,z), actor -> world         */
  const float* trans;           /* [n,3] base translation t_b, world frame                   */
  const float* rot_offset;      /* [n,4] learnable rotation offset dq (w,x,y,z) or NULL      */
  const float* trans_offset;    /* [n,3] learnable translation offset dt or NULL             */
  const float* lin_vel;         /* [n,3] linear velocity v_b, actor frame, or NULL (zero)    */
  const float* lin_vel_offset;  /* [n,3] learnable velocity offset dv or NULL                */
  const float* ang_vel;         /* [n,3] angular velocity w_a, actor frame, or NULL (zero)   */
} SplatActors;

/* Gradient accumulators (+=) of the learnable actor arrays, device arrays shaped like them;
 * a NULL member is skipped (rot_offset also when SplatActors.rot_offset is NULL). */
typedef struct SplatActorGrads {
  float* rot_offset;      /* [n,4] */
  float* trans_offset;    /* [n,3] */
  float* lin_vel_offset;  /* [n,3] */
  float* ang_vel;         /* [n,3] */
} SplatActorGrads;

/* Composes n Gaussians: means [n,3], quats [n,4], velocities [n,3] or NULL, actor_id [n]
 * (int32) -> means_w [n,3], quats_w [n,4], vel_w [n,3].  Outputs must not overlap the inputs.
 * n = 0 is a no-op.  Stream-ordered, allocates nothing. */
int splat_compose(int64_t n, const float* means, const float* quats, const float* velocities,
                  const int32_t* actor_id, const SplatActors* actors, float* means_w, float* quats_w,
                  float* vel_w, void* stream);
/* Workspace of splat_compose_bwd: one 24-float accumulator per actor. */
size_t splat_compose_workspace_bytes(int32_t n_actors);
/* Adjoint of splat_compose.  Upstream gradients d_means_w [n,3], d_quats_w [n,4], d_vel_w [n,3]
 * (e.g. the projection adjoint's SplatGrads means / quats / velocities); accumulates (+=)
 * d_means [n,3] and d_quats [n,4] of the local arrays, d_velocities [n,3] of static Gaussians
 * (skipped when NULL), and the actor gradients.  ws must hold
 * splat_compose_workspace_bytes(actors->n) bytes (SPLAT_ERR_CAPACITY otherwise); its contents
 * are overwritten.  Calls sharing a workspace must not overlap.  Per-actor sums use float
 * atomics, so their rounding depends on scheduling. */
int splat_compose_bwd(int64_t n, const float* means, const float* quats, const int32_t* actor_id,
                      const SplatActors* actors, const float* d_means_w, const float* d_quats_w,
                      const float* d_vel_w, float* d_means, float* d_quats, float* d_velocities,
                      const SplatActorGrads* d_actors, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): splat_compose_bwd with the per-actor accumulators in a
 * library-owned device array instead of a caller workspace.  The array holds
 * SPLAT_COMPOSE_NOALLOC_MAX_ACTORS actors (24 floats each, 1.5 MiB); each GPU the call runs on
 * keeps its own copy until the process ends.  actors->n above the maximum: SPLAT_ERR_CAPACITY,
 * nothing launched.  Arguments, outputs and the other error codes are those of
 * splat_compose_bwd.  Allocates nothing.  Every call on one GPU shares that GPU's array: the call
 * clears what it uses (a fill kernel, stream-ordered), and calls that overlap on one GPU (other
 * streams or threads) race and give wrong actor gradients. */
#define SPLAT_COMPOSE_NOALLOC_MAX_ACTORS 16384
int splat_compose_bwd_noalloc(int64_t n, const float* means, const float* quats, const int32_t* actor_id,
                              const SplatActors* actors, const float* d_means_w, const float* d_quats_w,
                              const float* d_vel_w, float* d_means, float* d_quats, float* d_velocities,
                              const SplatActorGrads* d_actors, void* stream);

/* ---- lidar points to rasterisation rays (App. A, "Lidar points to rasterization points") ----
 * A sweep's n points arrive with the ego motion compensated: world coordinates as if the whole
 * sweep were captured at its reference time (the middle of the sweep), with each point's capture
 * time relative to it in `times`.  Each point is expressed in the sensor frame at the reference
 * time, x_l = R x_w + t (R row-major, as in SplatLidar), moved back to the sensor at its own
 * capture time under the sensor's constant linear and angular velocity (sensor frame, as in
 * SplatLidar): x_cap = x_l + time (-ang_vel x x_l - lin_vel), and converted to spherical
 * coordinates: ray_az = atan2(y, x) in [0, 2 pi), ray_el = asin(z / r), ray_range = r = |x_cap|.
 * With `times` as the ray times, the outputs are a SplatLidar's ray_az / ray_el / ray_range.
 * A point at the sensor origin gets azimuth and elevation 0; a non-finite point gets NaN
 * outputs (rays outside every tile, counted in SplatStatus.n_rays_invalid).
 * points: device [n,3]; times, ray_az, ray_el: device [n]; ray_range: device [n] or NULL;
 * R [9], t [3]: HOST arrays (required); lin_vel, ang_vel: HOST [3] or NULL (zero).  Outputs
 * must not overlap the inputs.  n = 0 is a no-op; n < 0 or a missing required pointer gives
 * SPLAT_ERR_INVALID_ARG.  Stream-ordered, allocates nothing. */
int splat_lidar_points_to_rays(int64_t n, const float* points, const float* times, const float* R,
                               const float* t, const float* lin_vel, const float* ang_vel, float* ray_az,
                               float* ray_el, float* ray_range, void* stream);

/* ---- lidar decoder (Sec. 3.3; the training-details appendix: two layers, hidden width 32) ----
 * Per lidar ray, the rendered feature row F (n_feat channels, rows of n_feat floats as the lidar
 * rasteriser writes them) and the ray's unit direction in the sensor frame,
 * d = (cos el cos az, cos el sin az, sin el), are decoded by a two-layer MLP:
 *   h = ReLU(W1 [F, d] + b1),  z = W2 h + b2,  intensity = sigmoid(z0),  drop = sigmoid(z1).
 * The weights are device arrays (row-major); trained values are not needed to define the op. */
typedef struct SplatLidarMLP {
  int32_t n_feat;     /* C, 0..32                                                               */
  const float* w1;    /* [32, C + 3]: columns 0..C-1 multiply F, C..C+2 multiply d             */
  const float* b1;    /* [32]                                                                   */
  const float* w2;    /* [2, 32]: row 0 intensity, row 1 ray drop                               */
  const float* b2;    /* [2]                                                                    */
} SplatLidarMLP;

/* Weight-gradient accumulators (+=), device arrays shaped like SplatLidarMLP's; NULL skips one. */
typedef struct SplatLidarMLPGrads {
  float* w1;
  float* b1;
  float* w2;
  float* b2;
} SplatLidarMLPGrads;

/* Decodes n_rays rays: feat [n_rays, C], ray_az / ray_el [n_rays] (the rays the features were
 * rendered for) -> intensity [n_rays], drop_prob [n_rays] (either may be NULL).  n_rays = 0 is a
 * no-op; C outside 0..32 or a missing weight array gives SPLAT_ERR_INVALID_ARG.  Stream-ordered,
 * allocates nothing. */
int splat_lidar_decode(int64_t n_rays, const float* feat, const float* ray_az, const float* ray_el,
                       const SplatLidarMLP* mlp, float* intensity, float* drop_prob, void* stream);
/* Workspace of splat_lidar_decode_bwd (per-workgroup partial weight gradients); 0 = invalid. */
size_t splat_lidar_decode_workspace_bytes(int64_t n_rays, int32_t n_feat);
/* Adjoint of splat_lidar_decode.  Upstream gradients d_intensity, d_drop_prob [n_rays] (either
 * NULL = zero) -> d_feat [n_rays, C] (+=, or NULL) and the weight gradients (+=).  The weight
 * gradients are sums over rays, added in a fixed order (deterministic).  Workspace: caller-owned,
 * at least splat_lidar_decode_workspace_bytes bytes (SPLAT_ERR_CAPACITY otherwise).
 * Stream-ordered, allocates nothing. */
int splat_lidar_decode_bwd(int64_t n_rays, const float* feat, const float* ray_az, const float* ray_el,
                           const SplatLidarMLP* mlp, const float* d_intensity, const float* d_drop_prob,
                           float* d_feat, const SplatLidarMLPGrads* d_mlp, void* ws, size_t ws_bytes,
                           void* stream);

/* ---- camera decoder (Sec. 3.2; the training-details appendix: two residual blocks of width 32,
 * kernel size 3, then a final linear layer) ------------------------------------------------------
 * Per pixel x = [F, d, e]: the camera's rendered feature row F (its first n_feat channels), the
 * unit world-frame direction d of the ray through the pixel centre (camera frame
 * ((u+1/2-cx)/fx, (v+1/2-cy)/fy, 1) normalised, rotated by R^T), and the camera embedding e.
 *   h0 = ReLU(conv_in(x)),  r_k = ReLU(conv_k1(h_{k-1})),  h_k = ReLU(h_{k-1} + conv_k2(r_k))
 *   (M, b) = W_out h_2 + b_out,   I = M * F[0:3] + b            (k = 1, 2)
 * Convolutions: 3x3, stride 1, zero padding, bias, cross-correlation.  Weights are device
 * arrays in OIHW order; trained values are not needed to define the op.  Arithmetic is FP32
 * throughout (the 3x3 convolutions on the matrix cores). */
typedef struct SplatCameraCNN {
  int32_t n_feat;             /* D_f >= 3 (F[0:3] is the colour); D_f + 3 + n_embed <= 32      */
  int32_t n_embed;            /* E, 0..8                                                       */
  const float* embed;         /* [E] this camera's embedding                                   */
  const float* w_in;          /* [32, D_f + 3 + E, 3, 3]                                       */
  const float* b_in;          /* [32]                                                          */
  const float* w_block[4];    /* [32, 32, 3, 3]: block 1 conv 1, conv 2, block 2 conv 1, conv 2 */
  const float* b_block[4];    /* [32]                                                          */
  const float* w_out;         /* [6, 32]: rows 0-2 M, rows 3-5 b                               */
  const float* b_out;         /* [6]                                                           */
} SplatCameraCNN;

/* Gradient accumulators (+=) shaped like SplatCameraCNN's arrays; NULL skips one. */
typedef struct SplatCameraCNNGrads {
  float* embed;
  float* w_in;
  float* b_in;
  float* w_block[4];
  float* b_block[4];
  float* w_out;
  float* b_out;
} SplatCameraCNNGrads;

/* Workspace of the camera decoder for a width x height camera: the activations (six images of
 * 32 channels) that the adjoint reads, three gradient images and partial sums.  0 = invalid. */
size_t splat_camera_decode_workspace_bytes(int32_t width, int32_t height);
/* Decodes one camera: feat [H*W, C] (C = cam->n_channels, or n_feat when that is 0; rows as the
 * camera rasteriser writes them) -> image [H*W, 3].  Writes the activations into ws (caller-
 * owned, 256-byte aligned, >= splat_camera_decode_workspace_bytes, SPLAT_ERR_CAPACITY
 * otherwise).  Invalid sizes or missing arrays give SPLAT_ERR_INVALID_ARG.  Stream-ordered,
 * allocates nothing. */
int splat_camera_decode(const SplatCamera* cam, const float* feat, const SplatCameraCNN* cnn, float* image,
                        void* ws, size_t ws_bytes, void* stream);
/* Adjoint of splat_camera_decode.  d_image [H*W, 3] -> d_feat [H*W, C] (+=, or NULL) and the
 * weight and embedding gradients (+=).  ws must hold what the last splat_camera_decode with the
 * same camera, features and weights wrote.  Weight gradients are sums over pixels added in a
 * fixed order (deterministic).  Stream-ordered, allocates nothing. */
int splat_camera_decode_bwd(const SplatCamera* cam, const float* feat, const SplatCameraCNN* cnn,
                            const float* d_image, float* d_feat, const SplatCameraCNNGrads* d_cnn, void* ws,
                            size_t ws_bytes, void* stream);

/* ---- MCMC regulariser (training-details appendix) -------------------------------------------
 * The opacity and scale regularisation of the MCMC densification strategy:
 *   L = lambda_o sum_i |o_i| + lambda_s sum_i sum_j |sqrt(eig_j(Sigma_i))|
 * (the paper: lambda_o = 0.005, lambda_s = 0.001).  With Sigma = R diag(exp(2 l)) R^T the square
 * roots of the eigenvalues are exp(l_j) whatever the rotation.  Adds L to *value (device float,
 * or NULL) and dL/do = lambda_o sign(o), dL/dl = lambda_s exp(l) to grads->opacities and
 * grads->log_scales (each may be NULL, as may `grads`; other members are not touched).  The
 * value is summed in float32, per workgroup and then atomically (its last bits depend on the
 * order); the gradients are exact elementwise.  n = 0 is a no-op; non-finite lambdas give
 * SPLAT_ERR_INVALID_ARG.  Stream-ordered, allocates nothing. */
int splat_mcmc_regularizer(const SplatGaussians* g, float lambda_o, float lambda_s, float* value,
                           const SplatGrads* grads, void* stream);

/* ---- MCMC relocation of dead Gaussians (the MCMC densification strategy the paper adopts,
 * with at most 5M Gaussians) -------------------------------------------------------------------
 * Gaussian arrays the call updates in place (same layout as SplatGaussians). */
typedef struct SplatGaussianState {
  int64_t n;
  float* means;        /* [n,3] */
  float* log_scales;   /* [n,3] */
  float* quats;        /* [n,4] */
  float* opacities;    /* [n]   */
  float* velocities;   /* [n,3] or NULL */
  float* features;     /* [n,c_total] */
  int32_t c_total;
} SplatGaussianState;

/* Workspace of splat_mcmc_relocate (weights, their scan, a lookup table of the draw, counts, new
 * values); 0 = invalid. */
size_t splat_mcmc_relocate_workspace_bytes(int64_t n);
/* A Gaussian with opacity <= dead_opacity (0.005 in the strategy), or a non-finite one, is
 * dead; each dead Gaussian becomes a copy of an alive target drawn with probability
 * proportional to opacity, and every target shared by N Gaussians (itself and N - 1 copies,
 * N capped at n_max, 51 in the strategy) gets
 *   o' = 1 - (1 - o)^(1/N),   log-scales + log(o / sum_{k=1..N} C(N,k) (-1)^(k+1) o'^k / sqrt(k)),
 * which keeps the integral of the N copies' composited opacity profile along each axis equal to
 * the original's.  The copies take the target's mean, rotation, velocity, features and the new
 * opacity and log-scales.  The draw is exact integer arithmetic from the caller's randoms
 * u [n] (uint32, one per Gaussian, read for dead ones): weights floor(min(o, 1) 2^24) of alive
 * Gaussians, r = floor(u * total / 2^32), the target the first Gaussian whose inclusive weight
 * sum exceeds r.  With no alive Gaussian nothing changes.  target [n] (or NULL): the target of
 * each relocated Gaussian, -1 otherwise (for resetting optimiser state); n_relocated (device,
 * or NULL): += the number relocated.  All arrays are device arrays; ws caller-owned, 256-byte
 * aligned, >= splat_mcmc_relocate_workspace_bytes (SPLAT_ERR_CAPACITY otherwise); n >= 2^31
 * gives SPLAT_ERR_UNSUPPORTED.  Stream-ordered, allocates nothing. */
int splat_mcmc_relocate(const SplatGaussianState* g, const uint32_t* u, float dead_opacity, int32_t n_max,
                        int32_t* target, unsigned long long* n_relocated, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SPLAT_H_ */
