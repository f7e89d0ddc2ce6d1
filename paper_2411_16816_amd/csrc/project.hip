// project.hip -- projection of Gaussians into cameras and lidars, and its adjoint
// (SplatAD, arXiv 2411.16816: Sec. 3.1; Sec. 3.2 "Projection, tiling, and sorting" and
// "Rolling shutter"; Sec. 3.3 "Projection"; App. D).
//
// One thread per Gaussian.  Its parameters are read once (coalesced: consecutive threads read
// consecutive rows) and projected into every sensor of the call, so a batched call over S
// sensors reads the Gaussian arrays once instead of S times.  Records are written SoA
// (record = sensor * N + gaussian); culled records only write n_tiles = 0.
#include "kernels.hpp"
#include "wave_ops.hpp"

namespace splat {

struct GaussLoad {
  float mu[3], ls[3], q[4], vg[3], op;
};

__device__ __forceinline__ void load_gaussian(const SplatGaussians& g, int64_t i, GaussLoad& o) {
  o.mu[0] = g.means[3 * i + 0]; o.mu[1] = g.means[3 * i + 1]; o.mu[2] = g.means[3 * i + 2];
  o.ls[0] = g.log_scales[3 * i + 0]; o.ls[1] = g.log_scales[3 * i + 1]; o.ls[2] = g.log_scales[3 * i + 2];
  float4 q = reinterpret_cast<const float4*>(g.quats)[i];
  o.q[0] = q.x; o.q[1] = q.y; o.q[2] = q.z; o.q[3] = q.w;
  o.op = g.opacities[i];
  if (g.velocities) {
    o.vg[0] = g.velocities[3 * i + 0]; o.vg[1] = g.velocities[3 * i + 1]; o.vg[2] = g.velocities[3 * i + 2];
  } else {
    o.vg[0] = o.vg[1] = o.vg[2] = 0.f;
  }
}

// Depth used to ORDER Gaussians (Sec. 3.2: z of the camera-frame mean; Sec. 3.3: range of the
// lidar-frame mean), evaluated in float64 from the float32 inputs.  The float32 depth that is
// blended is unchanged; only the ordering key is exact enough that Gaussians whose float32
// depths coincide still sort by their true depth.  Positive doubles order like their bits.
__device__ __forceinline__ unsigned long long depth_key(const DevSensor& S, const float mu[3]) {
  double m[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    m[i] = (double)S.R[3 * i + 0] * mu[0] + (double)S.R[3 * i + 1] * mu[1] + (double)S.R[3 * i + 2] * mu[2] +
           (double)S.t[i];
  double d = (S.kind == kCamera) ? m[2] : sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  d = d > 0.0 ? d : 0.0;
  return (unsigned long long)__double_as_longlong(d);
}

__global__ __launch_bounds__(256) void k_project(const DevSensor* __restrict__ sens, int count, SplatGaussians g,
                                                 float4* __restrict__ mv, float4* __restrict__ cn,
                                                 float4* __restrict__ box, float2* __restrict__ dv,
                                                 unsigned long long* __restrict__ dkey,
                                                 int4* __restrict__ rect, int32_t* __restrict__ n_tiles,
                                                 SplatStatus* st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  GaussLoad G;
  load_gaussian(g, i, G);
  QuatRot qr;
  float s[3], M[9];
  gaussian_M(G.q, G.ls, qr, s, M);
  unsigned nonfin = 0;
  for (int k = 0; k < count; ++k) {
    ProjInter I;
    ProjOut o;
    project_one(sens[k], G.mu, M, G.vg, G.op, I, o);
    const int64_t r = (int64_t)k * g.n + i;
    n_tiles[r] = o.n_tiles;
    nonfin += o.nonfinite ? 1u : 0u;
    if (o.n_tiles > 0) {
      mv[r] = make_float4(o.mean[0], o.mean[1], o.vel[0], o.vel[1]);
      cn[r] = make_float4(o.conic[0], o.conic[1], o.conic[2], o.o_eff);
      box[r] = make_float4(o.box[0], o.box[1], o.box[2], o.box[3]);
      dv[r] = make_float2(o.depth, o.v_r);
      dkey[r] = depth_key(sens[k], G.mu);
      rect[r] = make_int4(o.rect[0], o.rect[1], o.rect[2], o.rect[3]);
    }
  }
  if (nonfin && st) atomicAdd(&st->n_nonfinite, nonfin);
}

// Records with more entries than this are summed by the whole wavefront, shorter ones by their
// own lane.
constexpr int kCoopEntries = 32;

// Bit j of the result is the flag of position base + j, for j < n <= kCoopEntries.  Reads the
// aligned 32-bit words that cover [base, base + n) all at once (independent loads, no branch per
// position); the flag array is padded to a multiple of 4 bytes and base + n <= its length.
__device__ __forceinline__ uint32_t flag_mask(const uint8_t* __restrict__ flags, int64_t base, int n) {
  constexpr int kWords = (kCoopEntries + 3) / 4 + 1;
  const int64_t a0 = base & ~(int64_t)3;
  const int off = (int)(base - a0);
  const int nw = (off + n + 3) >> 2;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(flags + a0);
  uint64_t m = 0;
#pragma unroll
  for (int k = 0; k < kWords; ++k) {
    const uint32_t x = w[k < nw ? k : nw - 1];   // in bounds: re-reads the last word past nw
    const uint32_t nib = (x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u);
    m |= (k < nw ? (uint64_t)nib : 0ull) << (4 * k);
  }
  m >>= off;
  return (uint32_t)(m & ((1ull << n) - 1ull));
}

template <int SW, int V>
__device__ __forceinline__ void add_row(const float* __restrict__ row, float (&acc)[V]) {
  const float4* q = reinterpret_cast<const float4*>(row);
#pragma unroll
  for (int u = 0; u < SW / 4; ++u) {
    const float4 x = q[u];
    if (4 * u + 0 < V) acc[4 * u + 0] += x.x;
    if (4 * u + 1 < V) acc[4 * u + 1] += x.y;
    if (4 * u + 2 < V) acc[4 * u + 2] += x.z;
    if (4 * u + 3 < V) acc[4 * u + 3] += x.w;
  }
}

// Long records are summed in chunks of kChunk positions, one wavefront per chunk and
// kChunk / 64 positions per lane.
constexpr int kChunk = 1024;
constexpr int kLanePositions = kChunk / 64;

__device__ __forceinline__ int listed_entries(int nt, int64_t base, int64_t k_cap) {
  const int64_t room = k_cap - base;   // entries at or beyond k_cap were never listed
  return room <= 0 ? 0 : (nt < room ? nt : (int)room);
}

// Work items (record, chunk) for every record that the adjoint touched and that has more than
// kCoopEntries listed entries, appended to partition ((record / 64) % kLongParts) of `list`:
// one atomic per 64 records that hold such a record, spread over kLongParts counters.  A
// wavefront covers 64 x kRecPerLane records (lane l: records l, l + 64, ...).  The list order
// varies from run to run; the sums do not.
constexpr int kRecPerLane = 4;

__global__ __launch_bounds__(256) void k_long_records(const int32_t* __restrict__ n_tiles,
                                                      const uint8_t* __restrict__ rflag,
                                                      const int64_t* __restrict__ entry_base, int64_t n_rec,
                                                      int64_t k_cap, uint2* __restrict__ list, int64_t cap,
                                                      int32_t* __restrict__ n_list) {
  const int lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 * kRecPerLane) + lane;
  int nt[kRecPerLane];
  bool hit[kRecPerLane];
#pragma unroll
  for (int j = 0; j < kRecPerLane; ++j) {   // unconditional loads, in bounds, all in flight together
    const int64_t r = r0 + 64 * j;
    const int64_t rc = r < n_rec ? r : n_rec - 1;
    nt[j] = n_tiles[rc];
    hit[j] = r < n_rec && rflag[rc] != 0;
  }
#pragma unroll
  for (int j = 0; j < kRecPerLane; ++j) {
    const int64_t r = r0 + 64 * j;
    int chunks = 0;
    if (hit[j] && nt[j] > kCoopEntries) chunks = (listed_entries(nt[j], entry_base[r], k_cap) + kChunk - 1) / kChunk;
    if (__ballot(chunks > 0) == 0) continue;   // uniform over the wavefront
    int incl = chunks;   // inclusive prefix over the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int part = (int)((r >> 6) % kLongParts);   // one partition per 64 consecutive records
    int first = 0;
    if (lane == 63) first = atomicAdd(n_list + part, incl);
    first = __shfl(first, 63, 64);
    uint2* dst = list + part * cap + first + (incl - chunks);
    for (int c = 0; c < chunks; ++c) dst[c] = make_uint2((uint32_t)r, (uint32_t)c);
  }
}

// One wavefront per (record, chunk): lane l sums the flagged rows at chunk positions l, l + 64,
// l + 128, ... (so that each load instruction of the wavefront reads 64 consecutive rows), two
// rows in flight; the wavefront reduces, and the chunk's total is stored into the row of the
// chunk's first position, flagged 2 (zeros if no row was written).  Only this wavefront touches
// the chunk's rows.  Items are numbered partition by partition.
constexpr int kLongRowsInFlight = 2;

template <int CMAX>
__global__ __launch_bounds__(256) void k_slot_reduce_long(const uint2* __restrict__ list, int64_t cap,
                                                          const int32_t* __restrict__ n_list,
                                                          const int32_t* __restrict__ n_tiles,
                                                          const int64_t* __restrict__ entry_base, float* slots,
                                                          uint8_t* flags, int64_t k_cap) {
  constexpr int V = kNV + CMAX;
  constexpr int SW = slot_stride(CMAX);
  constexpr int G = kLongRowsInFlight;
  static_assert(kLongParts == 64, "one partition count per lane");
  static_assert(kLanePositions % G == 0, "row groups");
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  // inclusive prefix of the partition counts, one per lane
  int incl = n_list[lane];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const int64_t total = __shfl(incl, 63, 64);
  bool store;
  const int idx = scatter_slot<V>(lane, store);
  for (int64_t it = wave; it < total; it += n_waves) {
    const int part = (int)__popcll(__ballot(incl <= it));   // partitions that end at or before it
    const int before = part == 0 ? 0 : __shfl(incl, part - 1, 64);
    const uint2 item = list[part * cap + (it - before)];
    const uint32_t r = item.x;
    const int64_t base = entry_base[r];
    const int n = listed_entries(n_tiles[r], base, k_cap);
    const int64_t c0 = base + (int64_t)item.y * kChunk;       // the chunk's first row
    const int64_t lim = (int64_t)n - (int64_t)item.y * kChunk;  // positions of the chunk (> 0)
    uint32_t on = 0;   // bit k: the lane's position k * 64 + lane holds a written row
#pragma unroll
    for (int k = 0; k < kLanePositions; ++k) {
      const int j = k * 64 + lane;
      const bool w = flags[c0 + (j < lim ? j : 0)] != 0;   // in bounds: position 0 for j >= lim
      on |= (j < lim && w) ? 1u << k : 0u;
    }
    float sum_v[V];
#pragma unroll
    for (int v = 0; v < V; ++v) sum_v[v] = 0.f;
#pragma unroll 1
    for (int k0 = 0; k0 < kLanePositions; k0 += G) {
      float rv[G][V];
#pragma unroll
      for (int u = 0; u < G; ++u) {
#pragma unroll
        for (int v = 0; v < V; ++v) rv[u][v] = 0.f;
        if ((on >> (k0 + u)) & 1u) add_row<SW>(slots + (c0 + (int64_t)(k0 + u) * 64 + lane) * SW, rv[u]);
      }
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int v = 0; v < V; ++v) sum_v[v] += rv[u][v];
    }
    const float sum = wave_reduce_scatter<V>(sum_v);
    if (store) slots[c0 * SW + idx] = sum;
    if (lane == 0) flags[c0] = 2;
  }
}

constexpr int kGaussPerLane = 4;   // Gaussians per lane of the projection adjoint and the row sums

// Gradient of every touched record, 64 x kGaussPerLane Gaussians per wavefront (lane l:
// Gaussians l, l + 64, ...; the flags of one sensor's records loaded together), sensors in
// order per Gaussian: the sum of the rasteriser's rows over the record's entries (positions [entry_base, entry_base + n_tiles) of
// the slot array, rows whose flag is set; a long record's total sits in its first row), taken
// in a fixed order so that the result does not depend on scheduling.  The geometric part (kNV
// values) goes to g2d[rec] (added to the atomic part of split lidar tiles when `accumulate` and
// bin_sort found such a tile, *split != 0), the channel part to the features gradient.
// Untouched records have no gradient and are skipped here and in the projection adjoint.
template <int CMAX>
__global__ __launch_bounds__(256) void k_slot_reduce(const DevSensor* __restrict__ sens, int count, int64_t N,
                                                     int c_total, const int32_t* __restrict__ n_tiles,
                                                     const uint8_t* __restrict__ rflag,
                                                     const int64_t* __restrict__ entry_base,
                                                     const float* __restrict__ slots,
                                                     const uint8_t* __restrict__ flags, int64_t k_cap,
                                                     bool accumulate, const int32_t* __restrict__ split,
                                                     float* __restrict__ g2d, float* __restrict__ dfeat) {
  constexpr int V = kNV + CMAX;
  constexpr int SW = slot_stride(CMAX);
  const int lane = threadIdx.x & 63;
  const int64_t i0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 * kGaussPerLane) + lane;
  for (int k = 0; k < count; ++k) {
    uint32_t tm = 0;   // bit j: record (k, i0 + 64 j) was touched; flags loaded together
#pragma unroll
    for (int j = 0; j < kGaussPerLane; ++j) {
      const int64_t i = i0 + 64 * j;
      const int64_t ic = i < N ? i : N - 1;   // unconditional loads, in bounds
      tm |= (rflag[(int64_t)k * N + ic] != 0 && i < N) ? 1u << j : 0u;
    }
    for (; tm != 0; tm &= tm - 1) {
      const int64_t i = i0 + 64 * __builtin_ctz(tm);
      const int64_t r = (int64_t)k * N + i;
      const int nt = n_tiles[r];
      const int64_t base = entry_base[r];
      const int n = listed_entries(nt, base, k_cap);
      float acc[V];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = 0.f;
      if (nt > kCoopEntries) {
        // chunk totals from k_slot_reduce_long, in chunk order
        const int nc = (n + kChunk - 1) / kChunk;
        for (int c = 0; c < nc; ++c) add_row<SW>(slots + (base + (int64_t)c * kChunk) * SW, acc);
      } else if (n > 0) {
        uint32_t fm = flag_mask(flags, base, n);
        while (fm) {   // two rows in flight per iteration
          const int j0 = __builtin_ctz(fm);
          fm &= fm - 1;
          const bool two = fm != 0;
          const int j1 = two ? __builtin_ctz(fm) : j0;
          if (two) fm &= fm - 1;
          float r0[V], r1[V];
#pragma unroll
          for (int v = 0; v < V; ++v) r0[v] = r1[v] = 0.f;
          add_row<SW>(slots + (base + j0) * SW, r0);
          add_row<SW>(slots + (base + j1) * SW, r1);
#pragma unroll
          for (int v = 0; v < V; ++v) acc[v] += two ? r0[v] + r1[v] : r0[v];
        }
      }
      // lidar records add to the atomic part of split tiles; camera rows are only ever written here
      float* q = g2d + r * kNV;
      const bool add = accumulate && sens[k].kind == kLidar && *split != 0;
#pragma unroll
      for (int v = 0; v < kNV; ++v) q[v] = add ? q[v] + acc[v] : acc[v];
      if (dfeat) {
        const DevSensor& S = sens[k];
        float* fp = dfeat + i * c_total + S.feat_off;
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
          if (c < S.n_ch) fp[c] += acc[kNV + c];
      }
    }
  }
}

// Projection adjoint of one Gaussian (i < N, with a gradient in at least one record when `live`):
// chains every touched record's g2d gradient (mean.x, mean.y, vel.x, vel.y, conic a, b, c,
// o_eff, depth (z | r), v_r) through the projection, the call's sensors in order, and adds the
// result to the Gaussian's gradients.  With sensor-velocity gradients requested (uniform), every
// touched record also contributes dL/dlin = -g and dL/dang = g x mu_s (g = dL/dvrel, mu_s the
// sensor-frame mean), summed per sensor over the wavefront with a reduce-scatter and one atomic
// per value; then every lane of the wavefront calls this together.
__device__ __forceinline__ void project_bwd_one(const DevSensor* __restrict__ sens, int count, const SplatGaussians& g,
                                                const uint8_t* __restrict__ rflag, const float* __restrict__ g2d,
                                                const SplatGrads& gr, int64_t i, bool live, bool want_s, int slot,
                                                bool store) {
  GaussLoad G;
  QuatRot qr;
  float s[3], M[9];
  if (live) {
    load_gaussian(g, i, G);
    gaussian_M(G.q, G.ls, qr, s, M);
  }
  float dmu[3] = {0.f, 0.f, 0.f}, dM[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, dvg[3] = {0.f, 0.f, 0.f};
  float dop = 0.f;
  bool any = false;
  for (int k = 0; k < count; ++k) {
    const int64_t r = (int64_t)k * g.n + i;
    const bool hit = live && rflag[r] != 0;   // a gradient reached this record
    float sv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (hit) {
      const float* q = g2d + r * kNV;
      RecGrad rg;
      rg.mean[0] = q[0]; rg.mean[1] = q[1]; rg.vel[0] = q[2]; rg.vel[1] = q[3];
      rg.conic[0] = q[4]; rg.conic[1] = q[5]; rg.conic[2] = q[6]; rg.o_eff = q[7];
      rg.depth = q[8]; rg.v_r = q[9];
      ProjInter I;
      ProjOut o;
      project_one(sens[k], G.mu, M, G.vg, G.op, I, o);
      float dv[3];
      project_one_vjp(sens[k], M, G.op, I, o, rg, dmu, dM, dvg, &dop, dv);
      any = true;
      if (want_s) {
        float c3[3];
        cross3(dv, I.mu, c3);
        sv[0] = -dv[0]; sv[1] = -dv[1]; sv[2] = -dv[2];
        sv[3] = c3[0]; sv[4] = c3[1]; sv[5] = c3[2];
      }
    }
    if (want_s && __ballot(hit) != 0) {   // uniform
      const float x = wave_reduce_scatter<6>(sv);
      if (store) {
        float* dst = slot < 3 ? gr.sensor_lin_vel : gr.sensor_ang_vel;
        if (dst) atomicAdd(dst + 3 * k + (slot % 3), x);
      }
    }
  }
  if (!live || !any) return;
  float dq[4], dls[3];
  gaussian_M_vjp(qr, s, dM, dq, dls);
  gr.means[3 * i + 0] += dmu[0]; gr.means[3 * i + 1] += dmu[1]; gr.means[3 * i + 2] += dmu[2];
  gr.log_scales[3 * i + 0] += dls[0]; gr.log_scales[3 * i + 1] += dls[1]; gr.log_scales[3 * i + 2] += dls[2];
  gr.quats[4 * i + 0] += dq[0]; gr.quats[4 * i + 1] += dq[1]; gr.quats[4 * i + 2] += dq[2]; gr.quats[4 * i + 3] += dq[3];
  gr.opacities[i] += dop;
  if (gr.velocities) {
    gr.velocities[3 * i + 0] += dvg[0]; gr.velocities[3 * i + 1] += dvg[1]; gr.velocities[3 * i + 2] += dvg[2];
  }
}

// Projection adjoint over the call's Gaussians.  A wavefront covers 64 x kGaussPerLane of them
// (lane l: Gaussians l, l + 64, ...): the gradient flags of all of them are loaded first, all
// in flight together, and only the groups of 64 that hold a touched Gaussian run the projection
// adjoint — most Gaussians of a scene receive no gradient, and the kernel's register use (3
// wavefronts per SIMD) would otherwise spend most of its time launching wavefronts that only
// test their flags.
__global__ __launch_bounds__(256) void k_project_bwd(const DevSensor* __restrict__ sens, int count, SplatGaussians g,
                                                     const uint8_t* __restrict__ rflag, const float* __restrict__ g2d,
                                                     SplatGrads gr) {
  const int lane = threadIdx.x & 63;
  const int64_t i0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 * kGaussPerLane) + lane;
  uint32_t tm = 0;   // bit j: Gaussian i0 + 64 j received a gradient in some record
  for (int k = 0; k < count; ++k) {
#pragma unroll
    for (int j = 0; j < kGaussPerLane; ++j) {
      const int64_t i = i0 + 64 * j;
      const int64_t ic = i < g.n ? i : g.n - 1;   // unconditional loads, in bounds
      const bool f = rflag[(int64_t)k * g.n + ic] != 0;
      tm |= (f && i < g.n) ? 1u << j : 0u;
    }
  }
  if (__ballot(tm != 0) == 0) return;   // uniform over the wavefront
  const bool want_s = gr.sensor_lin_vel || gr.sensor_ang_vel;   // uniform
  bool store = false;
  const int slot = want_s ? scatter_slot<6>(lane, store) : 0;
#pragma unroll 1
  for (int j = 0; j < kGaussPerLane; ++j) {
    const bool live = ((tm >> j) & 1u) != 0;
    if (__ballot(live) == 0) continue;   // uniform: nothing to add for this group
    project_bwd_one(sens, count, g, rflag, g2d, gr, i0 + 64 * j, live, want_s, slot, store);
  }
}

hipError_t launch_project(const CallView& v, const SplatGaussians& g, const SplatProjected& p, SplatStatus* st,
                          hipStream_t s) {
  if (g.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_project, dim3((unsigned)div_up(g.n, 256)), dim3(256), 0, s, v.sens, v.count, g, (float4*)p.mv,
                     (float4*)p.cn, (float4*)p.box, (float2*)p.dv, p.dkey, (int4*)p.rect, p.n_tiles, st);
  return hipGetLastError();
}

hipError_t launch_project_bwd(const CallView& v, const SplatGaussians& g, const SplatProjected& p,
                              const SplatTileLists& L, const Workspace& w, const SplatGrads& gr, hipStream_t s) {
  if (g.n <= 0) return hipSuccess;
  const int cm = cmax_bucket(v.c_max);
  if (w.stride != slot_stride(cm)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)div_up(g.n, 256));
  const dim3 grid_bwd((unsigned)div_up(g.n, 256 * kGaussPerLane));
  float* dfeat = v.c_max > 0 ? gr.features : nullptr;
  const int64_t n_rec = (int64_t)v.count * g.n;
  if (!w.rows) {   // every work item added its sums to g2d and the features gradient
    hipLaunchKernelGGL(k_project_bwd, grid_bwd, dim3(256), 0, s, v.sens, v.count, g, (const uint8_t*)w.rflag,
                       (const float*)w.g2d, gr);
    return hipGetLastError();
  }
  if (w.long_cap != long_part_cap(n_rec, L.k_cap)) return hipErrorInvalidValue;
  // w.n_long was cleared by the caller before the rasteriser adjoint
  hipLaunchKernelGGL(k_long_records, dim3((unsigned)div_up(n_rec, 256 * kRecPerLane)), dim3(256), 0, s, (const int32_t*)p.n_tiles,
                     (const uint8_t*)w.rflag, (const int64_t*)L.entry_base, n_rec, L.k_cap, (uint2*)w.long_list,
                     w.long_cap, w.n_long);
  const int64_t long_blocks = div_up(n_rec, 4) < 4096 ? div_up(n_rec, 4) : 4096;
#define SR_CASE(CM)                                                                                               \
  case CM:                                                                                                        \
    hipLaunchKernelGGL(k_slot_reduce_long<CM>, dim3((unsigned)long_blocks), dim3(256), 0, s,                      \
                       (const uint2*)w.long_list, w.long_cap, (const int32_t*)w.n_long,                           \
                       (const int32_t*)p.n_tiles, (const int64_t*)L.entry_base, w.slots, w.flags, L.k_cap);       \
    hipLaunchKernelGGL(k_slot_reduce<CM>, grid_bwd, dim3(256), 0, s, v.sens, v.count, g.n, g.c_total,                 \
                       (const int32_t*)p.n_tiles, (const uint8_t*)w.rflag, (const int64_t*)L.entry_base,          \
                       (const float*)w.slots, (const uint8_t*)w.flags, L.k_cap, v.has_lidar,                      \
                       (const int32_t*)L.n_work + 2, w.g2d, dfeat);                                               \
    break;
  switch (cm) {
    SR_CASE(4)
    SR_CASE(8)
    SR_CASE(16)
    SR_CASE(32)
    SR_CASE(48)
  }
#undef SR_CASE
  hipLaunchKernelGGL(k_project_bwd, grid_bwd, dim3(256), 0, s, v.sens, v.count, g, (const uint8_t*)w.rflag,
                     (const float*)w.g2d, gr);
  return hipGetLastError();
}

}  // namespace splat
