// kernels.hpp -- launchers of the libsplat kernels (host side), called by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "splat_common.hpp"

namespace splat {

// tile sizes of the sort / scan kernels
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;     // 4096 elements per block
constexpr int kRadixBits = 8;
// radix sort tiles: 2048 keys per 256-thread block (8 per thread); smaller than the scans' so
// that a few million keys still spread over several blocks per compute unit
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kScanThreads * kRadixItems;
constexpr int kRadixBins = 1 << kRadixBits;

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Gradient values of one record read by the projection adjoint: mean.x, mean.y, vel.x, vel.y,
// conic a, b, c, o_eff, depth (z | r), v_r.
constexpr int kNV = 10;

// channel counts are compiled in buckets
inline int cmax_bucket(int c) { return c <= 4 ? 4 : c <= 8 ? 8 : c <= 16 ? 16 : c <= 32 ? 32 : 48; }

// Floats per adjoint slot row: kNV geometric values then the bucket's channels, padded to a
// float4 multiple.
constexpr int slot_stride(int cmax_b) { return (kNV + cmax_b + 3) & ~3; }

// The list of long-record chunks is appended through this many counters (wavefront w uses
// counter w % kLongParts), so that no single counter takes every wavefront's atomic.  A
// partition holds at most one chunk per record of its wavefronts plus one per 1024 listed
// entries of all records.
constexpr int kLongParts = 64;
inline int64_t long_part_cap(int64_t n_rec, int64_t k_cap) {
  return div_up(div_up(n_rec, 64), kLongParts) * 64 + div_up(k_cap, 1024) + 1;
}

// Views of the device buffers of one call (local numbering), shared by the launchers.
struct CallView {
  const DevSensor* sens;   // device table entries [first, first + count)
  const DevSensor* host;   // host copies of the same entries
  int32_t count;
  int64_t n_gauss;
  int64_t n_tiles;         // tiles of the call
  int64_t n_supertiles;    // binning supertiles of the call (<= n_tiles)
  int64_t n_rays;          // rays of the call
  bool lidar;              // plain lidar call (all sensors are lidars)
  bool queue;              // batched form: any mix of sensors, persistent queue rasterisers
  bool has_lidar;          // at least one lidar in the call
  bool ray_cap;            // a lidar of the call renders at most SPLAT_RAYS_PER_ITEM rays per tile
  int64_t lidar_ray0;      // local id of the first lidar ray (cameras precede lidars in a rig)
  int64_t lidar_tile0;     // local id of the first lidar tile
  int c_max;               // max n_channels over the call
  int n_cu;                // compute units of the device (persistent grid)
  // second stream of the rig's device and two events: bin/sort forks the ray binning (which
  // reads no Gaussian data) onto it and joins it back before the queue; null: one stream
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // the adjoint's queue is known to hold its lidar items first, then its camera items (the
  // order bin/sort built for these lists when the adjoint keeps rows)
  bool queue_grouped = false;
};

inline int64_t work_capacity(int64_t n_tiles, int64_t n_rays) {
  return n_tiles + (n_rays + SPLAT_RAYS_PER_ITEM - 1) / SPLAT_RAYS_PER_ITEM + 1;
}

// ---- workspace carving (sizes in bytes, 256-aligned) ----------------------------------------
struct Workspace {
  // bin/sort
  uint64_t* dkeys[2];     // [n_rec] packed depth keys of the visible records
  uint32_t* dvals[2];
  int64_t* coff;          // [n_rec] first (supertile, record) entry of each visible record, depth order
  void* scan_part;        // block partials of the record scans (16 bytes per block)
  uint32_t* ckeys[2];     // [k_cap] supertile of each (supertile, record) entry
  uint64_t* cvals[2];     // [k_cap] Gaussian id | covered tile rows << 32 | columns << 40
  uint2* crange;          // [supertiles] [start, end) of each supertile's entries
  int64_t* item_first;    // [supertiles + 1] first item of each supertile; [n] = items
  uint2* item_st;         // [items] (supertile, sensor) of each item
  uint32_t* xcount;       // [64 items + 1] per (item, tile) entry counts, then their scan
  uint32_t* xpart;
  uint32_t* hist;         // [256 * max_blocks + partials]
  uint32_t* coltotal;     // [256] digit totals of a radix pass
  uint32_t* rhist;        // the ray sort's own histograms and digit totals (it may run beside the
  uint32_t* rcoltotal;    // record sorts, on the side stream)
  uint32_t* rkeys[2];     // [n_rays]
  uint32_t* rvals[2];
  int64_t* wcount;        // [n_tiles + 2]
  int64_t* wpart;
  uint32_t* qkeys[2];     // [work_cap] queue cost keys
  uint32_t* qvals[2];
  int2* qtmp;             // [work_cap] unordered work items
  int64_t* scalars;       // [4] device scalars of the call (visible records, entry counts, items)
  // adjoint (overlays the bin/sort buffers: the two are never live in one call)
  bool rows;              // per-entry rows kept (k_cap within the adjoint row limit)
  float* slots;           // [k_cap, slot_stride] per-entry gradient rows, indexed by entry number
  uint8_t* flags;         // [k_cap] 1 = slot row written by this adjoint call
  float* g2d;             // [n_rec, kNV] atomically accumulated part (lidar tiles split over items;
                          // every record when rows are not kept)
  uint8_t* rflag;         // [n_rec] 1 = the adjoint produced a gradient for the record
  uint32_t* long_list;    // [kLongParts * long_cap] (record, chunk) pairs of long touched records
  int32_t* n_long;        // [kLongParts] partition counts
  int32_t* qctr;          // [1] queue counter of the persistent adjoint
  int64_t long_cap;       // records per partition
  int stride;             // slot_stride(cmax_bucket(c_max))
  size_t bytes;
};

Workspace carve_workspace(void* base, int64_t n_rec, int64_t k_cap, int64_t n_tiles, int64_t n_rays, int c_max);

// Largest k_cap whose adjoint keeps per-entry rows (splat_set_adjoint_row_limit).
int64_t adjoint_row_limit();

// ---- launchers ------------------------------------------------------------------------------
hipError_t launch_project(const CallView& v, const SplatGaussians& g, const SplatProjected& p, SplatStatus* st,
                          hipStream_t s);
hipError_t launch_project_bwd(const CallView& v, const SplatGaussians& g, const SplatProjected& p,
                              const SplatTileLists& L, const Workspace& w, const SplatGrads& gr, hipStream_t s);
hipError_t launch_bin_sort(const CallView& v, const SplatProjected& p, const SplatTileLists& L, const Workspace& w,
                           SplatStatus* st, hipStream_t s);
// Optional events recorded on the launch stream right before and after the rasteriser kernel.
struct KernelTimer {
  hipEvent_t start = nullptr, stop = nullptr;
};

hipError_t launch_raster_fwd(const CallView& v, const SplatGaussians& g, const SplatProjected& p,
                             const SplatTileLists& L, int support, const SplatRenderOut& o, SplatStatus* st,
                             hipStream_t s, const KernelTimer& timer);
// The adjoint's launchers expect w.flags (with rows), w.rflag, the atomic part of w.g2d, w.qctr
// and w.n_long cleared by the caller (one fill launch for all of them).
hipError_t launch_raster_bwd(const CallView& v, const SplatGaussians& g, const SplatProjected& p,
                             const SplatTileLists& L, int support, const SplatRenderOut& saved, const float* dF,
                             const float* dD, const float* dA, const Workspace& w, float* dfeat, float* d_toff,
                             hipStream_t s, const KernelTimer& timer);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// several word arrays filled by one launch
constexpr int kMaxFillSegs = 6;
struct FillSegments {
  struct Seg {
    uint32_t* p;
    int64_t n;             // words
    uint32_t value;        // bit pattern (0.0f = 0)
    const int32_t* cond;   // device flag: the segment is filled only if *cond != 0 (null: always)
  } seg[kMaxFillSegs];
  int count = 0;
  void add(void* p, int64_t n, uint32_t value = 0u, const int32_t* cond = nullptr) {
    if (p && n > 0 && count < kMaxFillSegs) seg[count++] = Seg{(uint32_t*)p, n, value, cond};
  }
};
hipError_t launch_fill_segments(const FillSegments& f, hipStream_t s);
// exclusive scan of in[0..n) into out (may alias in); part: div_up(n, kScanTile) + 1 entries,
// the last of which receives the total
hipError_t launch_exclusive_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* part, hipStream_t s);

}  // namespace splat
