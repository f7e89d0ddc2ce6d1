// raster.hip -- tile rasterisation of cameras and lidars, forward and adjoint
// (SplatAD, arXiv 2411.16816: Sec. 3.2 "Rasterization", Eqs. t_pix, alpha_blend, alpha, delta;
// Sec. 3.3 "Rasterization" with the rolling-shutter range r + v_r t and the median range;
// App. A for rays supplied per tile and idle lanes helping to stage Gaussians).
//
// One 256-lane workgroup (4 x wave64) per work item: a camera tile (one lane per pixel) or a
// lidar tile chunk of <= 256 supplied rays.  The tile's depth-ordered list is walked in batches
// of 256 Gaussians; every lane (idle ones too) stages one Gaussian's record and features into
// LDS, then every lane composites the batch front to back.  A wavefront stops iterating once
// all its lanes are saturated (ballot), the workgroup once all lanes are (barrier count).
//
// The adjoint walks the same list back to front from each ray's `last`, recovering
// T_i = T_{i+1} / (1 - alpha_i) from the saved final transmittance.  Per-Gaussian gradients
// are summed across the wavefront (reduce-scatter over permlane swaps and DPP), across the
// workgroup in LDS, and stored as one row per (tile, Gaussian) entry at the entry's number
// (record-major), where the projection adjoint sums each record's rows in a fixed order.  Only work
// items of lidar tiles split over several items add their rows with global atomics.
#include "kernels.hpp"
#include "wave_ops.hpp"

namespace splat {

struct RasterArgs {
  const DevSensor* sens;
  int count;
  int64_t N;
  int64_t n_tiles;           // tiles of the call (lidar: also the invalid-ray bin id)
  const float4* mv;
  const float4* cn;
  const float4* box;
  const float2* dv;
  const int32_t* gauss;
  const longlong2* tile_range;
  const int4* rect;
  const int64_t* entry_base;
  const float* features;
  int c_total;
  const int32_t* ray_order;
  const int2* ray_range;
  const int2* work;
  const int32_t* n_work;
};

struct FwdOut {
  float* feat;
  float* depth;
  float* alpha;
  float* t_final;
  int32_t* last;
  float* median;
  unsigned long long* n_pairs;   // evaluated-pair counter, or null
  unsigned long long* n_stopped; // early-stopped ray counter (with n_pairs)
  unsigned long long* sensor_done;  // per-sensor completion clock (atomic max), or null
  float* los;                       // lidar line-of-sight sums, or null
  uint8_t* dropped;                 // lidar rays dropped by the training-time cap, or null
};

struct BwdIn {
  const float* t_final;
  const int32_t* last;
  const float* dF;
  const float* dD;
  const float* dA;
  float* slots;      // [k_cap, slot_stride] rows written by work items that own their tile
  uint8_t* flags;    // [k_cap] set for every row written
  uint8_t* rflag;    // [n_rec] set for every record given a gradient (row or atomic)
  float* g2d;        // [n_rec, kNV] atomic part from work items of split lidar tiles (every
                     // work item when rows are not kept)
  bool rows;         // per-entry rows kept (else every work item adds atomically)
  float* dfeat;      // features gradient (atomic part, split lidar tiles)
  unsigned long long* sensor_done;  // per-sensor completion clock (atomic max), or null
  float* d_toff;     // [count] camera time-offset gradients (+=), or null
  const float* d_los;  // upstream gradient of the lidar line-of-sight sums, or null
};

// Latency stamp of a finished work item: the sensor's entry rises to the device wall clock.
__device__ __forceinline__ void stamp_done(unsigned long long* done, int s) {
  if (done && threadIdx.x == 0) atomicMax(done + s, (unsigned long long)wall_clock64());
}

__device__ __forceinline__ int sensor_of_tile(const DevSensor* sens, int count, int64_t t) {
  int lo = 0, hi = count - 1;
  const int64_t b0 = sens[0].tile_base;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sens[mid].tile_base - b0 <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int sensor_of_ray_r(const DevSensor* sens, int count, int64_t r) {
  int lo = 0, hi = count - 1;
  const int64_t b0 = sens[0].ray_base;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sens[mid].ray_base - b0 <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// What one lane of a work item renders.
struct RayCtx {
  bool valid;
  float px, py, t;
  int64_t ray;        // local ray id of the call
  int64_t feat_off;   // first float of this ray's feature row in the output
  int s;              // sensor (call-local index)
  int C;              // channels
  int64_t start, end; // the tile's list range
  bool invalid_bin;   // lidar work item of rays outside every tile
  float los_thr;      // lidar line-of-sight threshold: measured range - margin (-inf: none)
  bool dropped;       // lidar ray dropped by the training-time cap (renders nothing)
};

// A value known to be the same in every lane, held in scalar registers.
__device__ __forceinline__ int64_t uniform_i64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane setup for one work item: a camera tile (all its pixels) or a chunk of <= 256 rays of a
// lidar tile starting at position `pos` of ray_order (tile == n_tiles: rays outside every tile).
template <bool LIDAR>
__device__ __forceinline__ void setup_ray(const RasterArgs& a, int64_t tile, int pos, RayCtx& c, int tid) {
  if (!LIDAR) {
    c.s = sensor_of_tile(a.sens, a.count, tile);
    const DevSensor& S = a.sens[c.s];
    int64_t tl = tile - (S.tile_base - a.sens[0].tile_base);
    int tx = (int)(tl % S.tiles_x), ty = (int)(tl / S.tiles_x);
    // tiles made of 8x8 blocks give each wavefront an 8x8 pixel block (a compact footprint, so
    // fewer wavefronts are partly covered by a Gaussian); other tiles are row-major
    int lx, ly;
    bool in_tile;
    if ((S.tile_w & 7) == 0 && (S.tile_h & 7) == 0) {
      const int blk = tid >> 6, l = tid & 63, bpr = S.tile_w >> 3;
      lx = (blk % bpr) * 8 + (l & 7);
      ly = (blk / bpr) * 8 + (l >> 3);
      in_tile = blk < bpr * (S.tile_h >> 3);
    } else {
      lx = tid % S.tile_w;
      ly = tid / S.tile_w;
      in_tile = tid < S.tile_w * S.tile_h;
    }
    int x = tx * S.tile_w + lx, y = ty * S.tile_h + ly;
    c.valid = in_tile && x < S.width && y < S.height;
    c.px = (float)x + 0.5f;
    c.py = (float)y + 0.5f;
    // Eq. t_pix at the pixel centre, plus the camera's time offset (timestamp - mid-exposure)
    c.t = (c.py / (float)S.height - 0.5f) * S.t_rs + S.t_off;
    int64_t pix = (int64_t)y * S.width + x;
    c.ray = (S.ray_base - a.sens[0].ray_base) + pix;
    c.feat_off = (S.feat_base - a.sens[0].feat_base) + pix * S.n_ch;
    c.C = S.n_ch;
    c.invalid_bin = false;
    c.los_thr = -INFINITY;
    c.dropped = false;
  } else {
    int2 rr = a.ray_range[tile];
    int64_t p = (int64_t)pos + tid;
    c.valid = p < rr.y;
    c.invalid_bin = (tile == a.n_tiles);
    int64_t r = c.valid ? (int64_t)a.ray_order[p] : 0;
    if (!c.valid) r = a.ray_order[pos];   // any ray of the item: keeps the sensor uniform
    c.ray = r;
    c.s = c.invalid_bin ? sensor_of_ray_r(a.sens, a.count, r) : sensor_of_tile(a.sens, a.count, tile);
    const DevSensor& S = a.sens[c.s];
    int64_t j = r - (S.ray_base - a.sens[0].ray_base);
    c.feat_off = (S.feat_base - a.sens[0].feat_base) + j * S.n_ch;
    c.C = S.n_ch;
    if (c.valid) {
      c.px = S.ray_az[j];
      c.py = S.ray_el[j];
      c.t = S.ray_t[j];
    } else {
      c.px = c.py = c.t = 0.f;
    }
    c.los_thr = (c.valid && S.ray_range) ? S.ray_range[j] - S.los_eps : -INFINITY;
    // training-time cap (App. A): a tile's rays past the first work item (its first
    // SPLAT_RAYS_PER_ITEM rays in priority order) are dropped; uniform over the work item
    c.dropped = S.ray_prio != nullptr && !c.invalid_bin && (int64_t)pos - rr.x >= SPLAT_RAYS_PER_ITEM;
  }
  // the invalid-ray bin (tile == n_tiles) has no Gaussian list: read an in-bounds entry and drop
  // it; a work item of dropped rays renders an empty list
  const bool empty = LIDAR && (c.invalid_bin || c.dropped);
  const longlong2 tr = a.tile_range[(LIDAR && c.invalid_bin) ? 0 : tile];
  // the same for every lane of the work item: say so, so that the list walks count in scalars
  c.start = uniform_i64(empty ? 0 : tr.x);
  c.end = uniform_i64(empty ? 0 : tr.y);
}

// One staged Gaussian in LDS, contiguous so that one address reaches all of it (float4 units):
//   [0] mean at t = 0 and its image-plane velocity (mx, my, vx, vy)
//   [1] conic in conic_exp2 form and opacity (A, B, C, o)
//   [2] BOX (x0, y0, x1, y1)
//   [3] depth value and rate, B / 2 and 2 vy (d0, dr, B/2, 2 vy); the last two serve the adjoint
//   [4 ...] features, CMAX channels (zero past the sensor's)
// Every lane reads the same record at a time (an LDS broadcast, free of bank conflicts).  The
// record stride is an odd number of float4 so that the staging writes, one record per lane,
// spread over all banks.
constexpr int rec4(int cmax) { return (4 + cmax / 4) | 1; }

// Returns the staged Gaussian's record (sensor * N + Gaussian id), -1 for lanes past the batch.
template <int CMAX>
__device__ __forceinline__ int64_t stage_batch(const RasterArgs& a, const RayCtx& c, int64_t b0, int64_t b1,
                                               float4* rec) {
  const int tid = threadIdx.x;
  const int64_t idx = b0 + tid;
  int64_t r = -1;
  if (idx < b1) {
    const int64_t g = a.gauss[idx];
    r = (int64_t)c.s * a.N + g;
    float4* o = rec + tid * rec4(CMAX);
    const float4 mv = a.mv[r];
    const float4 ce = conic_exp2(a.cn[r]);
    const float2 dv = a.dv[r];
    o[0] = mv;
    o[1] = ce;
    o[2] = a.box[r];
    o[3] = make_float4(dv.x, dv.y, 0.5f * ce.y, 2.f * mv.w);
    const DevSensor& S = a.sens[c.s];
    const float* f = a.features + g * a.c_total + S.feat_off;
#pragma unroll
    for (int c4 = 0; c4 < CMAX / 4; ++c4) {
      float4 v;
      v.x = (4 * c4 + 0 < c.C) ? f[4 * c4 + 0] : 0.f;
      v.y = (4 * c4 + 1 < c.C) ? f[4 * c4 + 1] : 0.f;
      v.z = (4 * c4 + 2 < c.C) ? f[4 * c4 + 2] : 0.f;
      v.w = (4 * c4 + 3 < c.C) ? f[4 * c4 + 3] : 0.f;
      o[4 + c4] = v;
    }
  }
  return r;
}

// wavefront-uniform tests on a lane predicate (scalar compares of the lane mask)
__device__ __forceinline__ uint64_t lane_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool wave_any(bool p) { return lane_mask(p) != 0; }

// Lane mask of a camera's box_contains over the wavefront, combined from one mask per compare:
// the mask of a single compare is its result register, while that of a combined predicate is
// rebuilt with two vector instructions.
__device__ __forceinline__ uint64_t camera_box_mask(float px, float py, float4 b) {
  return lane_mask(py >= b.y) & lane_mask(py < b.w) & lane_mask(px >= b.x) & lane_mask(px < b.z);
}

// ------------------------------------------------------------------------------------------
// forward
// ------------------------------------------------------------------------------------------
// Gaussians staged per batch of the forward walk (one per lane of the first kFwdBatch lanes).
// Half the workgroup: the smaller LDS footprint lets register use, not LDS, bound occupancy.
constexpr int kFwdBatch = 128;

template <int CMAX>
struct FwdSmem {
  float4 rec[kFwdBatch * rec4(CMAX)];
};

// Counters of a workgroup's forward items, summed over every item the workgroup renders and
// added to the status once per wavefront at the end of the kernel (a persistent workgroup
// renders many items; per-item global atomics on two addresses would contend).  `pairs` is the
// wavefront's count (uniform over its lanes), `stopped` a per-lane count.
struct FwdCount {
  unsigned long long pairs = 0, stopped = 0;
  __device__ void flush(const FwdOut& o) {
    if (!o.n_pairs) return;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) stopped += __shfl_xor(stopped, d, 64);
    if ((threadIdx.x & 63) == 0) {
      if (pairs) atomicAdd(o.n_pairs, pairs);
      if (stopped) atomicAdd(o.n_stopped, stopped);
    }
  }
};

// COUNT: also count the evaluated pairs (the counting launch; the others leave the counter out)
template <int CMAX, bool LIDAR, bool TILE, bool COUNT, typename SM>
__device__ __forceinline__ void fwd_item(const RasterArgs& a, const FwdOut& o, int64_t tile, int pos, SM& sm,
                                         FwdCount& cnt) {
  constexpr int R4 = rec4(CMAX);
  static_assert(sizeof(sm.rec) / sizeof(sm.rec[0]) >= kFwdBatch * R4, "record staging");
  RayCtx c;
  setup_ray<LIDAR>(a, tile, pos, c, threadIdx.x);
  float T = 1.f, D = 0.f, med = 0.f, los = 0.f;
  float F[CMAX];
#pragma unroll
  for (int k = 0; k < CMAX; ++k) F[k] = 0.f;
  int last = 0;
  unsigned long long pairs = 0;
  unsigned stopped = 0;
  // A lane's state is all numbers, no flags carried from one Gaussian to the next (the lane
  // masks of such flags cost scalar instructions on every iteration): `on` scales the lane's
  // alphas, 1 while it renders and 0 once it has stopped (or has no ray), so that it blends
  // nothing more.  `live` is the wavefront's mask of lanes with on = 1.
  float on = c.valid ? 1.f : 0.f;
  uint64_t live = lane_mask(c.valid);
  for (int64_t b0 = c.start; b0 < c.end; b0 += kFwdBatch) {
    if (__syncthreads_count(on > 0.f) == 0) break;
    const int64_t b1 = (b0 + kFwdBatch < c.end) ? b0 + kFwdBatch : c.end;
    if (kFwdBatch == kBlock || threadIdx.x < kFwdBatch) stage_batch<CMAX>(a, c, b0, b1, sm.rec);
    __syncthreads();
    const int nb = (int)(b1 - b0);
    // Branch-free over the lanes: a lane's decisions (box, alpha threshold, stop) become selects,
    // and a lane that does not blend the Gaussian adds exact zeros.  Only wavefront-uniform
    // branches remain, tested on lane masks of single compares: skip a Gaussian that no live
    // lane blends, leave the batch once every lane has stopped (a finished wavefront still
    // takes part in the workgroup's barriers).
    for (int j = 0; live != 0 && j < nb; ++j) {
      const float4* r = sm.rec + j * R4;
      const float4 bx = r[2], m = r[0], ce = r[1];
      bool in = true;
      uint64_t cand = live;
      if (!TILE) {
        const float bxa[4] = {bx.x, bx.y, bx.z, bx.w};
        in = box_contains(LIDAR, c.px, c.py, bxa);
        cand = LIDAR ? cand & lane_mask(in) : cand & camera_box_mask(c.px, c.py, bx);
      }
      if (cand == 0) continue;
      if (COUNT) pairs += (unsigned long long)__builtin_popcountll(cand);
      float4 f[CMAX / 4];
#pragma unroll
      for (int c4 = 0; c4 < CMAX / 4; ++c4) f[c4] = r[4 + c4];
      const float2 d = *reinterpret_cast<const float2*>(r + 3);
      PairEval e;
      eval_pair(LIDAR, c.px, c.py, c.t, m, ce, e);
      const float alpha = clamp_alpha(e.oG) * on;
      const bool pass = alpha >= kAlphaMin;
      const uint64_t blend = cand & lane_mask(pass);
      if (blend == 0) continue;
      const float Tn = SPLAT_FMA(-alpha, T, T);
      const bool low = Tn < kTStop;
      const uint64_t stop_m = blend & lane_mask(low);
      const bool act = in && pass && !low;
      const float w = act ? alpha * T : 0.f;
      const float gv = LIDAR ? SPLAT_FMA(d.y, c.t, d.x) : d.x;
#pragma unroll
      for (int c4 = 0; c4 < CMAX / 4; ++c4) {
        F[4 * c4 + 0] = SPLAT_FMA(w, f[c4].x, F[4 * c4 + 0]);
        F[4 * c4 + 1] = SPLAT_FMA(w, f[c4].y, F[4 * c4 + 1]);
        F[4 * c4 + 2] = SPLAT_FMA(w, f[c4].z, F[4 * c4 + 2]);
        F[4 * c4 + 3] = SPLAT_FMA(w, f[c4].w, F[4 * c4 + 3]);
      }
      D = SPLAT_FMA(w, gv, D);
      if (LIDAR) {
        los += (act && gv < c.los_thr) ? alpha : 0.f;   // line-of-sight sum
        // median range: the Gaussian across which the transmittance falls below 1/2 (T only
        // decreases, so this happens at most once)
        med = (act && T >= 0.5f && Tn < 0.5f) ? gv : med;
      }
      T = act ? Tn : T;
      last = act ? (int)(b0 + j - c.start) + 1 : last;
      if (stop_m) {   // uniform: some lane stops here
        const bool stop = in && pass && low;
        on = stop ? 0.f : on;
        stopped += stop ? 1u : 0u;
        live &= ~stop_m;
      }
    }
  }
  __syncthreads();   // LDS is reused by the next item of a persistent workgroup
  cnt.pairs += pairs;
  cnt.stopped += stopped;
  if (!(LIDAR && c.invalid_bin)) stamp_done(o.sensor_done, c.s);
  if (!c.valid) return;
  float* fo = o.feat + c.feat_off;
#pragma unroll
  for (int k = 0; k < CMAX; ++k)
    if (k < c.C) fo[k] = F[k];
  o.depth[c.ray] = D;
  o.alpha[c.ray] = 1.f - T;
  o.t_final[c.ray] = T;
  o.last[c.ray] = last;
  if (LIDAR && o.median) o.median[c.ray] = med;
  if (LIDAR && o.los) o.los[c.ray] = los;
  if (LIDAR && o.dropped) o.dropped[c.ray] = c.dropped ? 1 : 0;
}

// plain form: one workgroup per work item (camera: tile = block; lidar: work[block])
template <int CMAX, bool LIDAR, bool TILE>
__global__ __launch_bounds__(kBlock) void k_raster_fwd(RasterArgs a, FwdOut o) {
  __shared__ FwdSmem<CMAX> sm;
  FwdCount cnt;
  if (!LIDAR) {
    if (o.n_pairs) fwd_item<CMAX, false, TILE, true>(a, o, blockIdx.x, 0, sm, cnt);
    else fwd_item<CMAX, false, TILE, false>(a, o, blockIdx.x, 0, sm, cnt);
  } else {
    if ((int64_t)blockIdx.x >= (int64_t)a.n_work[0]) return;
    const int2 w = a.work[blockIdx.x];
    if (o.n_pairs) fwd_item<CMAX, true, TILE, true>(a, o, w.x, w.y, sm, cnt);
    else fwd_item<CMAX, true, TILE, false>(a, o, w.x, w.y, sm, cnt);
  }
  cnt.flush(o);
}

// Fetch the next queue entry for the whole workgroup (persistent kernels).
__device__ __forceinline__ int next_item(int32_t* counter, int* s_slot) {
  if (threadIdx.x == 0) *s_slot = atomicAdd(counter, 1);
  __syncthreads();
  const int it = *s_slot;
  __syncthreads();
  return it;
}

__device__ __forceinline__ bool item_is_lidar(const RasterArgs& a, int64_t tile) {
  return tile >= a.n_tiles || a.sens[sensor_of_tile(a.sens, a.count, tile)].kind == kLidar;
}

constexpr int cmax_max(int a, int b) { return a > b ? a : b; }

// persistent form: workgroups drain the cost-ordered queue of camera tiles and lidar chunks;
// camera items are compiled for the cameras' channel bucket CMC, lidar items for the lidars' CML
template <int CMC, int CML, bool TILE>
__global__ __launch_bounds__(kBlock) void k_raster_fwd_queue(RasterArgs a, FwdOut o, int32_t* counter) {
  __shared__ FwdSmem<cmax_max(CMC, CML)> sm;
  __shared__ int s_slot;
  FwdCount cnt;
  const int n_items = a.n_work[0];
  if (o.n_pairs) {
    for (;;) {
      const int it = next_item(counter, &s_slot);
      if (it >= n_items) break;
      const int2 w = a.work[it];
      if (item_is_lidar(a, w.x)) fwd_item<CML, true, TILE, true>(a, o, w.x, w.y, sm, cnt);
      else fwd_item<CMC, false, TILE, true>(a, o, w.x, 0, sm, cnt);
    }
  } else {
    for (;;) {
      const int it = next_item(counter, &s_slot);
      if (it >= n_items) break;
      const int2 w = a.work[it];
      if (item_is_lidar(a, w.x)) fwd_item<CML, true, TILE, false>(a, o, w.x, w.y, sm, cnt);
      else fwd_item<CMC, false, TILE, false>(a, o, w.x, 0, sm, cnt);
    }
  }
  cnt.flush(o);
}

// ------------------------------------------------------------------------------------------
// adjoint
// ------------------------------------------------------------------------------------------

template <int CMAX>
struct BwdShape {
  static constexpr int V = kNV + CMAX;   // values reduced per (ray, Gaussian)
};

// The adjoint runs a work item's 256 rays on 128 lanes (two wavefronts), two rays per lane: a
// lane adds its two rays' values for a Gaussian before the wavefront reduction, which so runs
// once per two (ray, Gaussian) pairs.  Camera: wavefront w covers pixel rows 8w .. 8w + 7 of the
// 16 x 16 tile (its lanes' two 8 x 8 blocks); lidar: ray slots (2w + p) 64 + lane of the item.
constexpr int kBwdLanes = 128;
constexpr int kRpl = kBlock / kBwdLanes;   // rays per lane
constexpr int kBwdBatch = 64;              // Gaussians staged per batch (one per lane of wavefront 0)

template <int CMAX>
struct BwdSmem {
  static constexpr int kCmax = CMAX;   // the launch's channel bucket: sets the gradient row stride
  float4 rec[kBwdBatch * rec4(CMAX)];
  float acc[BwdShape<CMAX>::V][kBwdBatch];
  int used[kBwdBatch];
  int maxlast;
  float toff;   // the item's time-offset gradient, summed over its wavefronts
};

// The adjoint reduces the geometric values of a pair in the basis of the conic_exp2 form, where
// they cost the fewest operations; these constants turn a reduced value into the gradient of
//   0, 1  the mean at t = 0,      2, 3  the velocity,     4, 5, 6  the conic (a, b, c),
//   7     the opacity o,          8, 9  the depth value and its rate (lidar: range, v_r),
// (with u = A dx + B dy the value 0 sums dL/ds (2 A dx + B dy) / ln 2, value 1 sums
// dL/ds (B dx / 2 + C dy) / ln 2, values 4-6 sum dL/ds (dx^2, dx dy, dy^2) / ln 2, where
// s = log2 exp(-sigma); dx = px - mx gives the sign of the mean's terms).
__device__ __forceinline__ constexpr float value_scale(int k) {
  return (k == 0 || k == 2) ? -kLn2
       : (k == 1 || k == 3) ? -2.f * kLn2
       : (k == 4 || k == 6) ? -0.5f
       : (k == 5) ? -1.f
       : 1.f;
}

template <int CMAX, bool LIDAR, bool TILE, typename SM>
__device__ __forceinline__ void bwd_item(const RasterArgs& a, const BwdIn& b, int64_t tile, int pos, SM& sm) {
  using SH = BwdShape<CMAX>;
  constexpr int R4 = rec4(CMAX);
  constexpr int P = kRpl;
  static_assert(SH::V <= 64, "channels");
  static_assert(sizeof(sm.acc) / sizeof(sm.acc[0]) >= SH::V, "accumulator rows");
  static_assert(sizeof(sm.rec) / sizeof(sm.rec[0]) >= kBwdBatch * R4, "record staging");
  auto& s_acc = sm.acc;
  int* s_used = sm.used;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  RayCtx c[P];
#pragma unroll
  for (int p = 0; p < P; ++p) setup_ray<LIDAR>(a, tile, pos, c[p], (P * wave + p) * 64 + lane);
  if (LIDAR && c[0].invalid_bin) return;    // uniform over the workgroup (not timed)
  float T[P], dATf[P], dD[P], bufD[P], dlos[P], S_dot[P];
  float dF[P][CMAX];
  int last_l[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T[p] = 1.f;
    float dA = 0.f;
    dD[p] = bufD[p] = dlos[p] = S_dot[p] = 0.f;
    last_l[p] = 0;
#pragma unroll
    for (int k = 0; k < CMAX; ++k) dF[p][k] = 0.f;
    if (c[p].valid) {
      T[p] = b.t_final[c[p].ray];
      last_l[p] = b.last[c[p].ray];
      dD[p] = b.dD[c[p].ray];
      dA = b.dA[c[p].ray];
      if (LIDAR && b.d_los) dlos[p] = b.d_los[c[p].ray];
      const float* g = b.dF + c[p].feat_off;
#pragma unroll
      for (int k = 0; k < CMAX; ++k)
        if (k < c[p].C) dF[p][k] = g[k];
    }
    dATf[p] = dA * T[p];
  }
  if (tid == 0) {
    sm.maxlast = 0;
    sm.toff = 0.f;
  }
  for (int k = tid; k < SH::V * kBwdBatch; k += kBwdLanes) (&s_acc[0][0])[k] = 0.f;
  if (tid < kBwdBatch) s_used[tid] = 0;
  __syncthreads();
  const int my_last = last_l[0] > last_l[1] ? last_l[0] : last_l[1];
  if (my_last > 0) atomicMax(&sm.maxlast, my_last);
  __syncthreads();
  const int64_t n_proc = sm.maxlast;
  __syncthreads();           // everyone has read maxlast before it can be reset by the next item
  if (n_proc == 0) {         // uniform
    stamp_done(b.sensor_done, c[0].s);
    return;
  }
  const int64_t start = c[0].start;
  const DevSensor& S = a.sens[c[0].s];
  const int64_t tile_local = tile - (S.tile_base - a.sens[0].tile_base);
  // a lidar tile with more rays than one item holds is shared by several items; without
  // per-entry rows every item adds atomically
  const bool split = !b.rows || (LIDAR && (a.ray_range[tile].y - a.ray_range[tile].x > SPLAT_RAYS_PER_ITEM));
  // gradient rows have the stride of the launch's bucket (the workspace's), whatever this
  // item's own channel bucket
  constexpr int SW = slot_stride(SM::kCmax);
  static_assert(SM::kCmax >= CMAX, "row stride");
  // values reduced across the wavefront: a camera has no range-velocity term (value 9)
  constexpr int VR = LIDAR ? SH::V : SH::V - 1;
  bool my_store;
  const int my_slot = scatter_slot<VR>(lane, my_store);
  const int my_idx = (!LIDAR && my_slot >= kNV - 1) ? my_slot + 1 : my_slot;   // accumulator row
  float tacc = 0.f;    // camera: dL/dt of this lane's pairs (mean at time t moves with the velocity)
  for (int64_t b0 = start + ((n_proc - 1) / kBwdBatch) * kBwdBatch; b0 >= start; b0 -= kBwdBatch) {
    const int64_t b1 = (b0 + kBwdBatch < start + n_proc) ? b0 + kBwdBatch : start + n_proc;
    // lane j of wavefront 0 stages Gaussian j of the batch and, after the walk, stores its
    // results: its record and gradient row are looked up now, beside the staging loads
    int64_t my_rec = -1, my_row = 0;
    if (tid < kBwdBatch) {
      my_rec = stage_batch<CMAX>(a, c[0], b0, b1, sm.rec);
      if (my_rec >= 0 && !split) my_row = a.entry_base[my_rec] + rect_entry(S, a.rect[my_rec], tile_local);
    }
    __syncthreads();
    const int nb = (int)(b1 - b0);
    for (int j = nb - 1; j >= 0; --j) {
      const float4* r = sm.rec + j * R4;
      const int posj = (int)(b0 + j - start);
      bool act[P];
      uint64_t cand[P];
      const float4 bx = r[2];
#pragma unroll
      for (int p = 0; p < P; ++p) {   // an invalid lane has last_l = 0
        act[p] = posj < last_l[p];
        cand[p] = lane_mask(act[p]);
        if (!TILE) {
          const float bxa[4] = {bx.x, bx.y, bx.z, bx.w};
          act[p] = act[p] && box_contains(LIDAR, c[p].px, c[p].py, bxa);
          cand[p] = LIDAR ? lane_mask(act[p]) : cand[p] & camera_box_mask(c[p].px, c[p].py, bx);
        }
      }
      if ((cand[0] | cand[1]) == 0) continue;
      const float4 m = r[0], ce = r[1], d = r[3];
      PairEval e[P];
      float alpha[P];
      uint64_t blend = 0;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        eval_pair(LIDAR, c[p].px, c[p].py, c[p].t, m, ce, e[p]);
        alpha[p] = clamp_alpha(e[p].oG);
        const bool pass = alpha[p] >= kAlphaMin;
        blend |= cand[p] & lane_mask(pass);
        act[p] = act[p] && pass;
      }
      if (blend == 0) continue;
      float v[SH::V];
#pragma unroll
      for (int k = 0; k < SH::V; ++k) v[k] = 0.f;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        // branch-free: inactive rays use alpha_eff = 0 and contribute exact zeros
        const float a_eff = act[p] ? alpha[p] : 0.f;
        const float ra = act[p] ? __builtin_amdgcn_rcpf(1.f - alpha[p]) : 1.f;
        T[p] = T[p] * ra;                   // transmittance in front of this Gaussian
        const float w = a_eff * T[p];
        float fd = 0.f;
#pragma unroll
        for (int c4 = 0; c4 < CMAX / 4; ++c4) {
          const float4 f = r[4 + c4];
          fd = SPLAT_FMA(f.x, dF[p][4 * c4 + 0], fd);
          fd = SPLAT_FMA(f.y, dF[p][4 * c4 + 1], fd);
          fd = SPLAT_FMA(f.z, dF[p][4 * c4 + 2], fd);
          fd = SPLAT_FMA(f.w, dF[p][4 * c4 + 3], fd);
        }
#pragma unroll
        for (int k = 0; k < CMAX; ++k) v[kNV + k] = SPLAT_FMA(w, dF[p][k], v[kNV + k]);
        const float gv = LIDAR ? SPLAT_FMA(d.y, c[p].t, d.x) : d.x;
        const float fdS = fd - S_dot[p], gvB = gv - bufD[p];
        const float acc = SPLAT_FMA(gvB, dD[p], fdS);
        S_dot[p] = SPLAT_FMA(a_eff, fdS, S_dot[p]);
        bufD[p] = SPLAT_FMA(a_eff, gvB, bufD[p]);
        // line-of-sight sum: its upstream gradient adds directly to the alpha of Gaussians in front
        float dalpha = SPLAT_FMA(T[p], acc, dATf[p] * ra);
        if (LIDAR) dalpha += (gv < c[p].los_thr) ? dlos[p] : 0.f;
        dalpha = act[p] ? dalpha : 0.f;
        // Eq. alpha's clamp cuts the dependence on G; ga = dL/ds / ln 2 with s = log2 G
        const bool clamped = e[p].oG > kAlphaMax;
        const float ga = clamped ? 0.f : dalpha * e[p].oG;
        const float dg = w * dD[p];
        const float e0 = ga * SPLAT_FMA(ce.x, e[p].dx, e[p].tx);
        const float e1 = ga * SPLAT_FMA(d.z, e[p].dx, e[p].cy);
        v[0] += e0;
        v[1] += e1;
        v[2] = SPLAT_FMA(e0, c[p].t, v[2]);
        v[3] = SPLAT_FMA(e1, c[p].t, v[3]);
        const float gx = ga * e[p].dx;
        v[4] = SPLAT_FMA(gx, e[p].dx, v[4]);
        v[5] = SPLAT_FMA(gx, e[p].dy, v[5]);
        v[6] = SPLAT_FMA(ga * e[p].dy, e[p].dy, v[6]);
        v[7] += clamped ? 0.f : dalpha * e[p].G;
        v[8] += dg;
        if (LIDAR) v[9] = SPLAT_FMA(dg, c[p].t, v[9]);
        if (!LIDAR) tacc = SPLAT_FMA(e0, m.z, SPLAT_FMA(e1, d.w, tacc));
      }
      float r_own;
      if constexpr (LIDAR) {
        r_own = wave_reduce_scatter<VR>(v);
      } else {   // value 9 is zero for a camera: reduce the others
        float u[VR];
#pragma unroll
        for (int k = 0; k < VR; ++k) u[k] = v[k < kNV - 1 ? k : k + 1];
        r_own = wave_reduce_scatter<VR>(u);
      }
      if (my_store) atomicAdd(&s_acc[my_idx][j], r_own);
      if (lane == 0) s_used[j] = 1;
    }
    __syncthreads();
    if (tid < nb && s_used[tid]) {
      const int64_t rec = my_rec;
      const int64_t g = rec - (int64_t)c[0].s * a.N;
      b.rflag[rec] = 1;   // idempotent: every writer stores the same byte
      if (!split) {
        // this item is the only one of its tile: the entry's row is complete, store it
        const int64_t p = my_row;
        float4* row = reinterpret_cast<float4*>(b.slots + p * SW);
#pragma unroll
        for (int q = 0; q < SW / 4; ++q) {
          float x[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) x[u] = (4 * q + u < SH::V) ? s_acc[4 * q + u][tid] * value_scale(4 * q + u) : 0.f;
          row[q] = make_float4(x[0], x[1], x[2], x[3]);
        }
        b.flags[p] = 1;
      } else {
        float* gp = b.g2d + rec * kNV;
#pragma unroll
        for (int k = 0; k < kNV; ++k) atomicAdd(gp + k, s_acc[k][tid] * value_scale(k));
        float* fp = b.dfeat + g * a.c_total + S.feat_off;
#pragma unroll
        for (int k = 0; k < CMAX; ++k)
          if (k < c[0].C) atomicAdd(fp + k, s_acc[kNV + k][tid]);
      }
#pragma unroll
      for (int k = 0; k < SH::V; ++k) s_acc[k][tid] = 0.f;
      s_used[tid] = 0;
    }
    __syncthreads();
  }
  if (!LIDAR && b.d_toff) {   // uniform: the item's time-offset gradient, one global add
    tacc *= -kLn2;            // the velocity terms of values 0 and 1 (see value_scale)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) tacc += __shfl_xor(tacc, d, 64);
    if (lane == 0) atomicAdd(&sm.toff, tacc);
    __syncthreads();
    if (tid == 0) atomicAdd(b.d_toff + c[0].s, sm.toff);
  }
  stamp_done(b.sensor_done, c[0].s);
}

template <int CMAX, bool LIDAR, bool TILE>
__global__ __launch_bounds__(kBwdLanes) void k_raster_bwd(RasterArgs a, BwdIn b) {
  __shared__ BwdSmem<CMAX> sm;
  if (!LIDAR) {
    bwd_item<CMAX, false, TILE>(a, b, blockIdx.x, 0, sm);
  } else {
    if ((int64_t)blockIdx.x >= (int64_t)a.n_work[0]) return;
    const int2 w = a.work[blockIdx.x];
    bwd_item<CMAX, true, TILE>(a, b, w.x, w.y, sm);
  }
}

// Item kinds an adjoint queue kernel renders (the queue holds its lidar items first and its
// n_cam camera items last).  Every form is held to 128 VGPRs (4 waves per SIMD): the camera-only
// and lidar-only kernels fit in 119 and 112; the kernel holding both would take 146 and spills
// 76 bytes per lane in its per-item set-up instead, which measures faster than 3 waves.
// kItemsGrouped: both kinds, the queue grouped by kind (the adjoint keeps rows): one loop over
// the lidar part, then one over the camera part, which halves the combined kernel's spills.
enum : int { kItemsCamera = 1, kItemsLidar = 2, kItemsBoth = 3, kItemsGrouped = 4 };

template <int CMC, int CML, bool TILE, int KINDS>
__global__ __launch_bounds__(kBwdLanes) __attribute__((amdgpu_waves_per_eu(4)))
void k_raster_bwd_queue(RasterArgs a, BwdIn b, int32_t* counter, int n_cam) {
  __shared__ BwdSmem<cmax_max(CMC, CML)> sm;
  __shared__ int s_slot;
  const int n_items = a.n_work[0];
  const int lo = KINDS == kItemsCamera ? n_items - n_cam : 0;   // this kernel's part of the queue
  const int hi = KINDS == kItemsLidar ? n_items - n_cam : n_items;
  if constexpr (KINDS == kItemsGrouped) {
    int it = next_item(counter, &s_slot);
    for (; it < n_items; it = next_item(counter, &s_slot)) {   // the lidar items come first
      const int2 w = a.work[it];
      if (!item_is_lidar(a, w.x)) break;   // uniform over the workgroup
      bwd_item<CML, true, TILE>(a, b, w.x, w.y, sm);
    }
    for (; it < n_items; it = next_item(counter, &s_slot)) {
      const int2 w = a.work[it];
      bwd_item<CMC, false, TILE>(a, b, w.x, 0, sm);
    }
  } else {
    for (;;) {
      const int it = lo + next_item(counter, &s_slot);
      if (it >= hi) break;
      const int2 w = a.work[it];
      if (KINDS == kItemsLidar || (KINDS == kItemsBoth && item_is_lidar(a, w.x)))
        bwd_item<CML, true, TILE>(a, b, w.x, w.y, sm);
      else
        bwd_item<CMC, false, TILE>(a, b, w.x, 0, sm);
    }
  }
}

// ------------------------------------------------------------------------------------------
// launch
// ------------------------------------------------------------------------------------------
static RasterArgs make_args(const CallView& v, const SplatGaussians& g, const SplatProjected& p, const SplatTileLists& L) {
  RasterArgs a;
  a.sens = v.sens;
  a.count = v.count;
  a.N = v.n_gauss;
  a.n_tiles = v.n_tiles;
  a.mv = (const float4*)p.mv;
  a.cn = (const float4*)p.cn;
  a.box = (const float4*)p.box;
  a.dv = (const float2*)p.dv;
  a.gauss = L.gauss;
  a.tile_range = (const longlong2*)L.tile_range;
  a.rect = (const int4*)p.rect;
  a.entry_base = L.entry_base;
  a.features = g.features;
  a.c_total = g.c_total;
  a.ray_order = L.ray_order;
  a.ray_range = (const int2*)L.ray_range;
  a.work = (const int2*)L.work;
  a.n_work = L.n_work;
  return a;
}

template <int CMAX, bool LIDAR>
static void fwd_dispatch(dim3 grid, hipStream_t s, int support, const RasterArgs& a, const FwdOut& o) {
  if (support == SPLAT_SUPPORT_TILE)
    hipLaunchKernelGGL((k_raster_fwd<CMAX, LIDAR, true>), grid, dim3(kBlock), 0, s, a, o);
  else
    hipLaunchKernelGGL((k_raster_fwd<CMAX, LIDAR, false>), grid, dim3(kBlock), 0, s, a, o);
}

template <int CMAX, bool LIDAR>
static void bwd_dispatch(dim3 grid, hipStream_t s, int support, const RasterArgs& a, const BwdIn& b) {
  if (support == SPLAT_SUPPORT_TILE)
    hipLaunchKernelGGL((k_raster_bwd<CMAX, LIDAR, true>), grid, dim3(kBwdLanes), 0, s, a, b);
  else
    hipLaunchKernelGGL((k_raster_bwd<CMAX, LIDAR, false>), grid, dim3(kBwdLanes), 0, s, a, b);
}

// persistent grid: as many workgroups as can be resident at once, capped by the item capacity
template <typename K>
static unsigned persistent_grid(K kernel, const CallView& v, int64_t items, int block) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t g = (int64_t)per_cu * (v.n_cu > 0 ? v.n_cu : 256);
  if (g > items) g = items;
  return (unsigned)(g < 1 ? 1 : g);
}

template <int CMC, int CML, bool TILE>
static void fwd_queue_launch(const CallView& v, int64_t items, hipStream_t s, const RasterArgs& a, const FwdOut& o,
                             int32_t* counter) {
  auto k = k_raster_fwd_queue<CMC, CML, TILE>;
  hipLaunchKernelGGL(k, dim3(persistent_grid(k, v, items, kBlock)), dim3(kBlock), 0, s, a, o, counter);
}

// The adjoint over the queue: one persistent kernel, compiled for the call's item kinds (a call
// of cameras only, or of lidars only, gets that kind's register allocation).
template <int CMC, int CML, bool TILE>
static hipError_t bwd_queue_launch(const CallView& v, int64_t items, hipStream_t s, const RasterArgs& a,
                                   const BwdIn& b, int32_t* counter) {
  const int n_cam = (int)v.lidar_tile0;   // one item per camera tile
  if (!v.has_lidar) {
    auto k = k_raster_bwd_queue<CMC, CML, TILE, kItemsCamera>;
    hipLaunchKernelGGL(k, dim3(persistent_grid(k, v, items, kBwdLanes)), dim3(kBwdLanes), 0, s, a, b, counter, n_cam);
  } else if (n_cam == 0) {
    auto k = k_raster_bwd_queue<CMC, CML, TILE, kItemsLidar>;
    hipLaunchKernelGGL(k, dim3(persistent_grid(k, v, items, kBwdLanes)), dim3(kBwdLanes), 0, s, a, b, counter, 0);
  } else if (v.queue_grouped && b.rows) {   // the queue is grouped by kind (binsort.hip, k_queue_keys)
    auto k = k_raster_bwd_queue<CMC, CML, TILE, kItemsGrouped>;
    hipLaunchKernelGGL(k, dim3(persistent_grid(k, v, items, kBwdLanes)), dim3(kBwdLanes), 0, s, a, b, counter, n_cam);
  } else {
    auto k = k_raster_bwd_queue<CMC, CML, TILE, kItemsBoth>;
    hipLaunchKernelGGL(k, dim3(persistent_grid(k, v, items, kBwdLanes)), dim3(kBwdLanes), 0, s, a, b, counter, n_cam);
  }
  return hipGetLastError();
}

// Channel buckets of the persistent kernels: the cameras' and the lidars' (a call's lidars with
// 8 channels beside wider cameras get the 8-channel code; other mixes use one bucket for both).
static void queue_buckets(const CallView& v, int& cmc, int& cml) {
  int c_cam = 0, c_lid = 0;
  for (int i = 0; i < v.count; ++i) {
    const DevSensor& d = v.host[i];
    if (d.kind == kCamera) c_cam = d.n_ch > c_cam ? d.n_ch : c_cam;
    else c_lid = d.n_ch > c_lid ? d.n_ch : c_lid;
  }
  cmc = cmax_bucket(v.c_max);
  cml = cmc;
  if (c_lid > 0 && cmax_bucket(c_lid) == 8 && cmc > 8) cml = 8;
}

hipError_t launch_raster_fwd(const CallView& v, const SplatGaussians& g, const SplatProjected& p,
                             const SplatTileLists& L, int support, const SplatRenderOut& out, SplatStatus* st,
                             hipStream_t s, const KernelTimer& timer) {
  RasterArgs a = make_args(v, g, p, L);
  FwdOut o{out.feat, out.depth, out.alpha, out.t_final, out.last, out.median, st ? &st->n_pairs : nullptr,
           st ? &st->n_stopped : nullptr, out.sensor_done, out.los,
           out.dropped};
  const int cm = cmax_bucket(v.c_max);
  if (v.queue) {
    const int64_t items = L.work_cap;
    if (items <= 0) return hipSuccess;
    int32_t* counter = L.n_work + 1;
    hipError_t e = launch_fill_i32(counter, 1, 0, s);
    if (e != hipSuccess) return e;
    const bool tile = support == SPLAT_SUPPORT_TILE;
    int cmc, cml;
    queue_buckets(v, cmc, cml);
#define FWDQ_CASE(CM, CL)                                                     \
  if (cmc == CM && cml == CL) {                                               \
    if (tile) fwd_queue_launch<CM, CL, true>(v, items, s, a, o, counter);     \
    else fwd_queue_launch<CM, CL, false>(v, items, s, a, o, counter);         \
  }
    if (timer.start) (void)hipEventRecord(timer.start, s);
    FWDQ_CASE(4, 4)
    FWDQ_CASE(8, 8)
    FWDQ_CASE(16, 16)
    FWDQ_CASE(16, 8)
    FWDQ_CASE(32, 32)
    FWDQ_CASE(32, 8)
    FWDQ_CASE(48, 48)
    FWDQ_CASE(48, 8)
#undef FWDQ_CASE
    if (timer.stop) (void)hipEventRecord(timer.stop, s);
    return hipGetLastError();
  }
  const int64_t items = v.lidar ? L.work_cap : v.n_tiles;
  if (items <= 0) return hipSuccess;
  dim3 grid((unsigned)items);
#define FWD_CASE(CM)                                           \
  case CM:                                                     \
    if (v.lidar) fwd_dispatch<CM, true>(grid, s, support, a, o); \
    else fwd_dispatch<CM, false>(grid, s, support, a, o);      \
    break;
  if (timer.start) (void)hipEventRecord(timer.start, s);
  switch (cm) {
    FWD_CASE(4)
    FWD_CASE(8)
    FWD_CASE(16)
    FWD_CASE(32)
    FWD_CASE(48)
  }
#undef FWD_CASE
  if (timer.stop) (void)hipEventRecord(timer.stop, s);
  return hipGetLastError();
}

hipError_t launch_raster_bwd(const CallView& v, const SplatGaussians& g, const SplatProjected& p,
                             const SplatTileLists& L, int support, const SplatRenderOut& saved, const float* dF,
                             const float* dD, const float* dA, const Workspace& w, float* dfeat, float* d_toff,
                             hipStream_t s, const KernelTimer& timer) {
  RasterArgs a = make_args(v, g, p, L);
  BwdIn b{saved.t_final, saved.last, dF, dD, dA, w.slots, w.flags, w.rflag, w.g2d, w.rows, dfeat, saved.sensor_done,
          d_toff, saved.d_los};
  const int cm = cmax_bucket(v.c_max);
  if (w.stride != slot_stride(cm)) return hipErrorInvalidValue;
  if (v.queue) {
    const int64_t items = L.work_cap;
    if (items <= 0) return hipSuccess;
    hipError_t e = hipSuccess;   // w.qctr was cleared by the caller
    const bool tile = support == SPLAT_SUPPORT_TILE;
    int cmc, cml;
    queue_buckets(v, cmc, cml);
#define BWDQ_CASE(CM, CL)                                                          \
  if (cmc == CM && cml == CL) {                                                    \
    e = tile ? bwd_queue_launch<CM, CL, true>(v, items, s, a, b, w.qctr)           \
             : bwd_queue_launch<CM, CL, false>(v, items, s, a, b, w.qctr);         \
    if (e != hipSuccess) return e;                                                 \
  }
    if (timer.start) (void)hipEventRecord(timer.start, s);
    BWDQ_CASE(4, 4)
    BWDQ_CASE(8, 8)
    BWDQ_CASE(16, 16)
    BWDQ_CASE(16, 8)
    BWDQ_CASE(32, 32)
    BWDQ_CASE(32, 8)
    BWDQ_CASE(48, 48)
    BWDQ_CASE(48, 8)
#undef BWDQ_CASE
    if (timer.stop) (void)hipEventRecord(timer.stop, s);
    return hipGetLastError();
  }
  const int64_t items = v.lidar ? L.work_cap : v.n_tiles;
  if (items <= 0) return hipSuccess;
  dim3 grid((unsigned)items);
#define BWD_CASE(CM)                                           \
  case CM:                                                     \
    if (v.lidar) bwd_dispatch<CM, true>(grid, s, support, a, b); \
    else bwd_dispatch<CM, false>(grid, s, support, a, b);      \
    break;
  if (timer.start) (void)hipEventRecord(timer.start, s);
  switch (cm) {
    BWD_CASE(4)
    BWD_CASE(8)
    BWD_CASE(16)
    BWD_CASE(32)
    BWD_CASE(48)
  }
#undef BWD_CASE
  if (timer.stop) (void)hipEventRecord(timer.stop, s);
  return hipGetLastError();
}

}  // namespace splat
