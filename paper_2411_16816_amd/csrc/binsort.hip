// binsort.hip -- tile binning and depth sorting (SplatAD, arXiv 2411.16816: Sec. 3.2
// "Projection, tiling, and sorting"; Sec. 3.3 "Tiling and sorting"; App. A).
//
// Pipeline of one call (on the call's stream, step 6 on the rig's side stream when there is
// one; no host synchronisation):
//   1. one scan over the records in record order counts the visible records and their
//      (tile, Gaussian) entries, gives each visible record its entry numbers (the adjoint's
//      gradient rows) and compacts the visible records with a 32-bit key of their float64 depth;
//   2. the visible records are stably sorted by that key, so equal keys keep record
//      (= Gaussian id) order;
//   3. tiles are grouped into supertiles (camera 8 x 8 tiles, lidar 4 x 4); a scan in depth
//      order gives every record the place of its (supertile, record) entries, one per supertile
//      its rectangle meets, and they are written in depth order;
//   4. a stable radix sort by supertile groups those entries, each supertile's in depth order,
//      and gives each supertile its range of entries (with at most 256 supertiles the sort is
//      one pass and its scatter writes the ranges from the digit totals; else a ranges pass);
//   5. each supertile's entries are cut into items of at most 256; per item, the entries
//      meeting each of the supertile's tiles (64 or 16) are counted (wavefront ballots), one scan of the
//      counts gives every tile its list range and every item its first position in each list,
//      and the items write the Gaussian ids straight into the lists, ranked by ballot prefix.
//      Every list holds its tile's Gaussians in (depth, id) order, the ordering the paper gets
//      from sorting (tile | depth) keys, while only the compact supertile entries are sorted;
//   6. lidar: rays are binned into their tiles (a ray is a box of zero extent, App. A), invalid
//      rays go to an extra bin, and every tile's rays are cut into work items of <= 256 rays.
//      This reads no Gaussian data: with a side stream it runs beside steps 1-5.
//
// The radix sort is an LDS-histogram reduce-then-scan sort with 8-bit digits: per-block digit
// histograms (wavefront ballots aggregate equal digits before LDS atomics), a device-wide
// scan, and a stable per-block scatter that ranks equal digits with 64-lane ballots.  No pass
// depends on inter-workgroup forward progress.
#include "kernels.hpp"

namespace splat {

// ------------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

template <typename T>
hipError_t fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = div_up(n, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t s) { return fill<float>(p, n, v, s); }

// Up to kMaxFillSegs arrays of 32-bit words filled by one launch (each segment grid-strided by
// the whole grid).
__global__ void k_fill_segments(FillSegments f) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < f.count; ++k) {
    if (f.seg[k].cond && *f.seg[k].cond == 0) continue;   // uniform: the segment is not needed
    uint32_t* p = f.seg[k].p;
    const uint32_t v = f.seg[k].value;
    for (int64_t i = t0; i < f.seg[k].n; i += stride) p[i] = v;
  }
}

hipError_t launch_fill_segments(const FillSegments& f, hipStream_t s) {
  int64_t most = 0;
  for (int k = 0; k < f.count; ++k) most = f.seg[k].n > most ? f.seg[k].n : most;
  if (most <= 0) return hipSuccess;
  int64_t blocks = div_up(most, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_segments, dim3((unsigned)blocks), dim3(256), 0, s, f);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) { return fill<int32_t>(p, n, v, s); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int64_t shfl_up_i64(int64_t v, int d) {
  int lo = __shfl_up((int)(uint32_t)(uint64_t)v, d, 64);
  int hi = __shfl_up((int)(uint32_t)((uint64_t)v >> 32), d, 64);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
__device__ __forceinline__ uint32_t shfl_up_t(uint32_t v, int d) { return (uint32_t)__shfl_up((int)v, d, 64); }
__device__ __forceinline__ int64_t shfl_up_t(int64_t v, int d) { return shfl_up_i64(v, d); }

// Two int64 counters scanned together (trivially constructible, so it can live in LDS).
struct P64 {
  int64_t a, b;
  P64() = default;
  __device__ P64(int v) : a(v), b(v) {}
  __device__ P64(int64_t x, int64_t y) : a(x), b(y) {}
  __device__ P64& operator+=(const P64& o) {
    a += o.a;
    b += o.b;
    return *this;
  }
};
__device__ __forceinline__ P64 operator+(P64 x, const P64& y) { return x += y; }
__device__ __forceinline__ P64 operator-(P64 x, const P64& y) { return P64(x.a - y.a, x.b - y.b); }
__device__ __forceinline__ P64 shfl_up_t(P64 v, int d) { return P64(shfl_up_i64(v.a, d), shfl_up_i64(v.b, d)); }

// exclusive scan across a 256-thread block; `tmp` holds 4 entries
template <typename T>
__device__ T block_exclusive_scan(T v, T* tmp, T& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = shfl_up_t(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[wid] = x;
  __syncthreads();
  T pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    T s = tmp[w];
    pre += (w < wid) ? s : (T)0;
    tot += s;
  }
  total = tot;
  __syncthreads();
  return pre + x - v;
}

// ------------------------------------------------------------------------------------------
// device-wide exclusive scan (reduce, scan of partials, downsweep); Load(i) gives element i
// ------------------------------------------------------------------------------------------
struct LoadU32 {
  const uint32_t* p;
  __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct LoadI64 {
  const int64_t* p;
  __device__ int64_t operator()(int64_t i) const { return p[i]; }
};

// Elements scanned: the capacity n, or fewer when the count is only known on the device
// (n_dev non-null: min(n, *n_dev)).  Blocks wholly past that count do nothing, except that the
// block holding the last element (block 0 when there is none) closes the scan.
__device__ __forceinline__ int64_t scan_count(const int64_t* n_dev, int64_t n) {
  if (!n_dev) return n;
  const int64_t m = *n_dev;
  return m < 0 ? 0 : (m < n ? m : n);
}
// Elements per thread and per block of a scan over T: 16-byte elements take half as many, so
// that a block's LDS tile stays at 34 KB (four blocks per compute unit).
template <typename T>
constexpr int scan_items() { return sizeof(T) > 8 ? kScanItems / 2 : kScanItems; }
template <typename T>
constexpr int scan_tile() { return kScanThreads * scan_items<T>(); }

template <typename T>
__device__ __forceinline__ int64_t scan_last_block(int64_t n_eff) { return n_eff > 0 ? (n_eff - 1) / scan_tile<T>() : 0; }

template <typename T, typename Load>
__global__ __launch_bounds__(256) void k_scan_reduce(Load ld, int64_t n, const int64_t* n_dev, T* __restrict__ part) {
  __shared__ T tmp[4];
  const int64_t n_eff = scan_count(n_dev, n);
  constexpr int kItems = scan_items<T>();
  const int64_t base = (int64_t)blockIdx.x * scan_tile<T>();   // < n: the grid has div_up(n, tile) blocks
  if ((int64_t)blockIdx.x > scan_last_block<T>(n_eff)) {      // uniform: contributes nothing
    if (threadIdx.x == 0) part[blockIdx.x] = (T)0;
    return;
  }
  const int64_t hi = n_eff > 0 ? n_eff - 1 : 0;
  T acc = 0;
  // indices clamped into [0, n_eff): every load is issued unconditionally, back to back
#pragma unroll 4
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kScanThreads + threadIdx.x;
    const T x = ld(i < hi ? i : hi);
    acc += i < n_eff ? x : (T)0;
  }
  T total;
  block_exclusive_scan<T>(acc, tmp, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Up to this many blocks every down-sweep block sums the block totals before it itself (one
// launch fewer); beyond it a single block scans the totals first.
constexpr int64_t kScanFusedBlocks = 4096;

// single block: exclusive scan of part[0..nb) in place, part[nb] = total
template <typename T>
__global__ __launch_bounds__(256) void k_scan_partials(T* __restrict__ part, int64_t nb) {
  __shared__ T tmp[4];
  T carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += 256) {
    int64_t i = b0 + threadIdx.x;
    T v = i < nb ? part[i] : (T)0;
    T total;
    T ex = block_exclusive_scan<T>(v, tmp, total);
    if (i < nb) part[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

// Per-element work of a scan, in two phases so that the loads of several elements are issued
// before any of their stores: In load(i, value) reads what element i needs, then
// operator()(i, prefix, value, in) writes; finish(total) runs once with the grand total.
struct NoVisit {
  struct In {};
  template <typename T>
  __device__ In load(int64_t, T) const { return In{}; }
  template <typename T>
  __device__ void operator()(int64_t, T, T, In) const {}
  template <typename T>
  __device__ void finish(T) const {}
};

// Writes the grand total to *dst (no per-element work).
struct StoreTotal {
  int64_t* dst;
  struct In {};
  template <typename T>
  __device__ In load(int64_t, T) const { return In{}; }
  template <typename T>
  __device__ void operator()(int64_t, T, T, In) const {}
  __device__ void finish(int64_t total) const { *dst = total; }
};

// Block b: exclusive scan of its tile, offset by the total of the blocks before it: with
// `fused`, the sum of the block totals part[0..b) (read by the block itself; the closing block
// writes the grand total to part[nb]), otherwise part[b] as scanned by k_scan_partials.  Every
// element i is handed to the visitor with its prefix and its value; the closing block's first
// thread hands it the grand total (vis.finish).  `out` may be null (visitor only).
template <typename T, typename Load, typename Visit>
__global__ __launch_bounds__(256) void k_scan_down(Load ld, int64_t n, const int64_t* n_dev, T* __restrict__ part,
                                                   int64_t nb, bool fused, T* __restrict__ out, Visit vis) {
  // element li of the tile lives at pad(li) = li + li / 16: a thread's 16 consecutive
  // elements then start 17 apart, which spreads the per-thread pass over the LDS banks
  constexpr int kItems = scan_items<T>();
  constexpr int kTile = scan_tile<T>();
  __shared__ T tile[kTile + kTile / kItems];
  __shared__ T tmp[4];
  auto pad = [](int li) { return li + li / kItems; };
  const int64_t n_eff = scan_count(n_dev, n);
  const int64_t last = scan_last_block<T>(n_eff);
  if ((int64_t)blockIdx.x > last) return;   // uniform
  const int64_t hi = n_eff > 0 ? n_eff - 1 : 0;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  T xs[kItems];   // the tile's loads are issued first and stay in flight while the blocks
                  // before this one are summed
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kScanThreads + threadIdx.x;
    xs[r] = ld(i < hi ? i : hi);
  }
  T before;
  if (fused) {
    T pb = 0;
    for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) pb += part[i];
    block_exclusive_scan<T>(pb, tmp, before);
  } else {
    before = part[blockIdx.x];
  }
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + (int64_t)r * kScanThreads + threadIdx.x;
    tile[pad(r * kScanThreads + threadIdx.x)] = i < n_eff ? xs[r] : (T)0;
  }
  __syncthreads();
  T loc[kItems];
  T acc = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    loc[k] = acc;
    acc += tile[pad(threadIdx.x * kItems + k)];
  }
  T total;
  T pre = block_exclusive_scan<T>(acc, tmp, total) + before;
  if ((int64_t)blockIdx.x == last && threadIdx.x == 0) {
    if (fused) part[nb] = before + total;
    vis.finish(before + total);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k) tile[pad(threadIdx.x * kItems + k)] = pre + loc[k];
  __syncthreads();
  const T end = before + total;   // exclusive prefix after the block
  constexpr int kBatch = 4;
#pragma unroll
  for (int r0 = 0; r0 < kItems; r0 += kBatch) {
    T p[kBatch], gap[kBatch];
    typename Visit::In in[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int li = (r0 + u) * kScanThreads + threadIdx.x;
      const int64_t i = base + li;
      p[u] = tile[pad(li)];
      gap[u] = (li + 1 < kTile ? tile[pad(li + 1)] : end) - p[u];   // element i's value
      if (i < n_eff) in[u] = vis.load(i, gap[u]);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int64_t i = base + (r0 + u) * kScanThreads + threadIdx.x;
      if (i < n_eff) {
        if (out) out[i] = p[u];
        vis(i, p[u], gap[u], in[u]);
      }
    }
  }
}

// the scan of no elements: total 0
template <typename T, typename Visit>
__global__ void k_scan_empty(T* part, Visit vis) {
  part[0] = (T)0;
  vis.finish((T)0);
}

// exclusive scan of n elements (fewer when n_dev is given, see scan_count) into out[0..n)
// (out may alias the loaded array: each block reads its tile before writing it; out may be
// null); part[nb] receives the total
template <typename T, typename Load, typename Visit = NoVisit>
hipError_t device_scan(Load ld, int64_t n, T* out, T* part, hipStream_t s, Visit vis = Visit(),
                       const int64_t* n_dev = nullptr) {
  int64_t nb = div_up(n, scan_tile<T>());
  if (nb == 0) {
    hipLaunchKernelGGL((k_scan_empty<T, Visit>), dim3(1), dim3(1), 0, s, part, vis);
    return hipGetLastError();
  }
  // one block needs no block totals (the fused down-sweep sums none before block 0)
  if (nb > 1)
    hipLaunchKernelGGL((k_scan_reduce<T, Load>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, ld, n, n_dev, part);
  const bool fused = nb <= kScanFusedBlocks;
  if (!fused) hipLaunchKernelGGL((k_scan_partials<T>), dim3(1), dim3(256), 0, s, part, nb);
  hipLaunchKernelGGL((k_scan_down<T, Load, Visit>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, ld, n, n_dev, part,
                     nb, fused, out, vis);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// radix sort: stable, 8-bit digits, keys and values uint32
// ------------------------------------------------------------------------------------------
// Lanes of the wavefront whose (valid) digit equals this lane's: one ballot per digit bit.
// Always 8 bits, unrolled; a narrower digit has zero high bits, whose ballots change nothing.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(valid && bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ int64_t sort_count(const int64_t* n_ptr, int64_t n_cap) {
  if (!n_ptr) return n_cap;
  int64_t n = *n_ptr;
  return n < n_cap ? n : n_cap;
}

// Per-block digit counts of one kRadixTile-key tile, counted with LDS atomics into one histogram per
// wavefront (order does not matter for counting), written digit-major: hist[d * nb + block] with
// nb = the grid's block count, so that the per-digit scans over the blocks read contiguous runs.
// Blocks past the key count write nothing (nothing reads their counts).
template <typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const K* __restrict__ keys, const int64_t* n_ptr, int64_t n_cap,
                                                    int shift, int bits, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[4][kRadixBins];
  const int tid = threadIdx.x, wid = tid >> 6;
  const int64_t n = sort_count(n_ptr, n_cap);
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  if (base >= n) return;   // uniform
  cnt[0][tid] = cnt[1][tid] = cnt[2][tid] = cnt[3][tid] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  uint32_t d[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int64_t i = base + (int64_t)r * kScanThreads + tid;
    const uint32_t x = (uint32_t)(keys[i < n ? i : n - 1] >> shift) & mask;   // unconditional load
    d[r] = i < n ? x : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r)
    if (d[r] != 0xFFFFFFFFu) atomicAdd(&cnt[wid][d[r]], 1u);
  __syncthreads();
  hist[(int64_t)tid * gridDim.x + blockIdx.x] = cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
}

// One block per digit d: exclusive scan of the digit's counts over the blocks that hold keys
// (in place, row d of the nb_grid-wide digit-major table), and the digit's total.
__global__ __launch_bounds__(256) void k_radix_colscan(uint32_t* __restrict__ hist, const int64_t* n_ptr,
                                                       int64_t n_cap, int64_t nb_grid, uint32_t* __restrict__ coltotal) {
  __shared__ uint32_t tmp[4];
  const int d = blockIdx.x;
  const int64_t nb = (sort_count(n_ptr, n_cap) + kRadixTile - 1) / kRadixTile;
  uint32_t* row = hist + (int64_t)d * nb_grid;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t x = b < nb ? row[b] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<uint32_t>(x, tmp, total);
    if (b < nb) row[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) coltotal[d] = carry;
}

// Stable scatter of one block tile (kRadixTile keys).  Wavefront w owns the contiguous quarter
// of the tile and walks it in kRadixItems rounds of 64 keys: ballot matching of
// the digit gives each key its rank among the round's equal digits, and a wave-private running
// count per digit (LDS, touched only by that wavefront) carries the rank across rounds.  One
// block scan then turns (digit, wavefront) counts into offsets, keys are staged in LDS in digit
// order and written out so that consecutive lanes write consecutive addresses of a digit's
// output run (coalesced), at the block's global digit offsets: the digit's start (exclusive
// scan of the digit totals, done here) plus the earlier blocks' counts of the digit.
//
// range_out (single-pass sorts, may be null): block 0 also writes every digit d < n_range its
// output run [start, end), which for a sort over one digit is the key's range in the output.
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_radix_scatter(const K* __restrict__ kin, const V* __restrict__ vin,
                                                       K* __restrict__ kout, V* __restrict__ vout,
                                                       const int64_t* n_ptr, int64_t n_cap, int shift, int bits,
                                                       const uint32_t* __restrict__ hist,
                                                       const uint32_t* __restrict__ coltotal,
                                                       uint2* __restrict__ range_out, int n_range) {
  constexpr int kPerWave = kRadixTile / 4;
  __shared__ K s_k[kRadixTile];
  __shared__ V s_v[kRadixTile];
  __shared__ uint32_t gbase[kRadixBins];
  __shared__ uint32_t lcum[kRadixBins];
  __shared__ uint32_t wc[4][kRadixBins];   // per-wavefront running counts, then offsets
  __shared__ uint32_t tmp[4];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  const int64_t n = sort_count(n_ptr, n_cap);
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  const bool ranges = range_out && blockIdx.x == 0;   // block 0 writes them even with no keys
  if (base >= n && !ranges) return;                   // both uniform over the block
  {
    uint32_t dtot;
    const uint32_t c = coltotal[tid];
    const uint32_t dstart = block_exclusive_scan<uint32_t>(c, tmp, dtot);
    if (ranges && tid < n_range) range_out[tid] = make_uint2(dstart, dstart + c);
    if (base >= n) return;
    gbase[tid] = dstart + hist[(int64_t)tid * gridDim.x + blockIdx.x];
  }
  const int cnt = (int)((n - base) < kRadixTile ? (n - base) : kRadixTile);
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t lt = lanemask_lt();
  wc[0][tid] = wc[1][tid] = wc[2][tid] = wc[3][tid] = 0u;
  K key[kRadixItems];
  V val[kRadixItems];
  uint32_t rank[kRadixItems];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const int li = wid * kPerWave + r * 64 + lane;
    const int lc = li < cnt ? li : cnt - 1;   // unconditional loads; lanes past cnt are invalid below
    key[r] = kin[base + lc];
    val[r] = vin[base + lc];
  }
  __syncthreads();
  uint32_t* run = wc[wid];
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    const bool valid = wid * kPerWave + r * 64 + lane < cnt;
    const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
    const uint64_t m = match_digit(d, valid);
    const uint32_t before = valid ? run[d] : 0u;
    rank[r] = before + (uint32_t)__popcll(m & lt);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (valid && (m & lt) == 0) run[d] = before + (uint32_t)__popcll(m);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  // digit totals -> block offsets; per-wavefront offsets inside each digit
  const uint32_t c0 = wc[0][tid], c1 = wc[1][tid], c2 = wc[2][tid], c3 = wc[3][tid];
  uint32_t total;
  const uint32_t dcum = block_exclusive_scan<uint32_t>(c0 + c1 + c2 + c3, tmp, total);
  lcum[tid] = dcum;
  wc[0][tid] = dcum;
  wc[1][tid] = dcum + c0;
  wc[2][tid] = dcum + c0 + c1;
  wc[3][tid] = dcum + c0 + c1 + c2;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixItems; ++r) {
    if (wid * kPerWave + r * 64 + lane < cnt) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
      const uint32_t li = wc[wid][d] + rank[r];
      s_k[li] = key[r];
      s_v[li] = val[r];
    }
  }
  __syncthreads();
  // coalesced write-out
  for (int i = tid; i < cnt; i += kScanThreads) {
    const K k = s_k[i];
    const uint32_t d = (uint32_t)(k >> shift) & mask;
    const uint32_t pos = gbase[d] + (uint32_t)i - lcum[d];
    kout[pos] = k;
    vout[pos] = s_v[i];
  }
}

// Digit width of every pass but possibly the last for a sort over total_bits: the fewest
// passes of at most kRadixBits, with the bits spread evenly (14 bits: 7 + 7 rather than 8 + 6),
// so that no pass scatters into many more digit runs than it needs.
static inline int radix_pass_bits(int total_bits) {
  const int passes = (total_bits + kRadixBits - 1) / kRadixBits;
  return (total_bits + passes - 1) / passes;
}

// Sorts (k[cur], v[cur]) stably by key bits [lo_bit, lo_bit + total_bits).  On return `cur`
// indexes the sorted keys; the sorted values are in v[cur], or in `final_vals` when it is
// non-null.  n_ptr (device) gives the element count when non-null, capped by n_cap; only the
// blocks that hold keys do work.  Three launches per pass: histograms, per-digit scans over
// the blocks, scatter.  range_out (may be null): for a sort of one pass, the [start, end) of
// every key value below n_range is also written, by the scatter; nothing for more passes.
template <typename K, typename V>
static hipError_t radix_sort(K* k[2], V* v[2], int& cur, const int64_t* n_ptr, int64_t n_cap, int lo_bit,
                             int total_bits, uint32_t* hist, uint32_t* coltotal, V* final_vals, hipStream_t s,
                             uint2* range_out = nullptr, int n_range = 0) {
  if (total_bits < 1) total_bits = 1;
  const int passes = (total_bits + kRadixBits - 1) / kRadixBits;
  if (passes > 1) range_out = nullptr;
  const int per = radix_pass_bits(total_bits);   // bits spread evenly over the passes
  const int64_t nb = div_up(n_cap, kRadixTile);
  if (nb == 0) return hipSuccess;
  for (int p = 0; p < passes; ++p) {
    const int shift = lo_bit + p * per;
    const int bits = (total_bits - p * per) < per ? (total_bits - p * per) : per;
    hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)nb), dim3(256), 0, s, (const K*)k[cur], n_ptr, n_cap, shift,
                       bits, hist);
    hipLaunchKernelGGL(k_radix_colscan, dim3(kRadixBins), dim3(256), 0, s, hist, n_ptr, n_cap, nb, coltotal);
    V* vdst = (p == passes - 1 && final_vals) ? final_vals : v[1 - cur];
    hipLaunchKernelGGL((k_radix_scatter<K, V>), dim3((unsigned)nb), dim3(256), 0, s, (const K*)k[cur], (const V*)v[cur],
                       k[1 - cur], vdst, n_ptr, n_cap, shift, bits, (const uint32_t*)hist, (const uint32_t*)coltotal,
                       range_out, n_range);
    cur = 1 - cur;
  }
  return hipGetLastError();
}

static int bits_for(int64_t n_values) {   // bits needed for values 0..n_values-1
  int b = 0;
  while (b < 31 && ((int64_t)1 << b) < n_values) ++b;
  return b < 1 ? 1 : b;
}

// bits of a ray's cell code: the rest of the bin's last radix digit (none when the bin fills it)
static int ray_cell_bits(int bin_bits) {
  const int c = (kRadixBits - bin_bits % kRadixBits) % kRadixBits;
  return bin_bits + c <= 32 ? c : 0;
}

// ------------------------------------------------------------------------------------------
// binning kernels
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int64_t local_tile_base(const DevSensor* sens, int s) {
  return sens[s].tile_base - sens[0].tile_base;
}

// 32-bit sort key of a positive float64 depth: 5 bits of binary exponent over [2^-16, 2^16)
// and the top 27 mantissa bits (2^-27 relative resolution, 8x finer than a float32 depth),
// monotone in the depth; depths outside that range clamp to the first / last key (ties then
// keep Gaussian-id order).  Four 8-bit radix passes.
constexpr int kDepthKeyBits = 32;

__device__ __forceinline__ uint64_t depth_sort_key(unsigned long long bits) {
  const int e = (int)((bits >> 52) & 0x7FF) - (1023 - 16);
  if (e < 0) return 0ull;
  if (e > 31) return (1ull << kDepthKeyBits) - 1ull;
  return ((uint64_t)e << 27) | ((bits & 0xFFFFFFFFFFFFFull) >> 25);
}

// Device scalars of one bin/sort call (workspace `scalars`).
enum : int {
  kScVisible = 0,    // visible records (n_tiles > 0)
  kScEntries = 1,    // (tile, Gaussian) entries K, uncapped
  kScCoarse = 2,     // (supertile, record) entries; 0 when K exceeds the capacity
  kScItemsX = 3,     // elements of the per-item count array: 64 x items + 1
  kScCount = 4
};

// sensor (index into the call's table) of record rec = s * N + g; exact for rec < 2^32
__device__ __forceinline__ int record_sensor(int64_t rec, int64_t N, int count) {
  if (count <= 1) return 0;
  int s = (int)((float)rec * __builtin_amdgcn_rcpf((float)N));
  s -= ((int64_t)s * N > rec) ? 1 : 0;
  s += ((int64_t)(s + 1) * N <= rec) ? 1 : 0;
  return s;
}

// ---- supertiles --------------------------------------------------------------------------------
// A sensor's tile grid (camera tiles_x x tiles_y; lidar M_phi x M_omega) is cut into supertiles
// of 2^st_wl x 2^st_hl tiles, numbered row-major (st_x per row), after the supertiles of the
// call's earlier sensors.  Tile (row, col) is tile f = (row % h) * 8 + col % w of supertile
// (row / h, col / w) (tiles are numbered with a stride of 8 whatever the width).
__device__ __forceinline__ int grid_stride(const DevSensor& S) { return S.kind == kCamera ? S.tiles_x : S.m_az; }
__device__ __forceinline__ int grid_rows(const DevSensor& S) { return S.kind == kCamera ? S.tiles_y : S.m_el; }

// Supertiles a rectangle (x0, y0, w, h) meets: rows [r0, r0 + nr) and, in each, the columns
// [c0, c0 + nc0) followed by [0, nc1) (the second run only for a lidar rectangle that wraps the
// azimuth seam into supertile columns it does not already cover).
struct StSpan {
  int r0, nr, c0, nc0, nc1;
};

__device__ __forceinline__ StSpan st_span(const DevSensor& S, const int4 rc) {
  StSpan p;
  p.r0 = rc.y >> S.st_hl;
  p.nr = ((rc.y + rc.w - 1) >> S.st_hl) - p.r0 + 1;
  const int M = grid_stride(S);
  if (S.kind == kCamera || rc.x + rc.z <= M) {
    p.c0 = rc.x >> S.st_wl;
    p.nc0 = ((rc.x + rc.z - 1) >> S.st_wl) - p.c0 + 1;
    p.nc1 = 0;
  } else {
    const int a = rc.x >> S.st_wl;                    // [a, st_x) then [0, e]
    const int e = (rc.x + rc.z - 1 - M) >> S.st_wl;
    if (e >= a) {                                     // the two runs meet: every column
      p.c0 = 0;
      p.nc0 = S.st_x;
      p.nc1 = 0;
    } else {
      p.c0 = a;
      p.nc0 = S.st_x - a;
      p.nc1 = e + 1;
    }
  }
  return p;
}

// bits [max(lo, 0), min(hi, cap)) of a mask of at most 8 bits
__device__ __forceinline__ uint32_t span_bits(int lo, int hi, int cap) {
  const int a = lo > 0 ? lo : 0;
  const int b = hi < cap ? hi : cap;
  return b > a ? ((1u << b) - 1u) & ~((1u << a) - 1u) : 0u;
}

// Tiles of supertile (sr, sc) inside rectangle rc, as the rows (bit r: tile row sr * h + r) and
// the columns (bit c: tile column sc * w + c) it covers there; tile f = r * 8 + c is inside
// exactly when both bits are set.  A lidar rectangle's columns are [x0, x0 + w) modulo M_phi,
// i.e. the columns of [x0, x0 + w) and of [x0 - M_phi, x0 + w - M_phi) inside the grid.
__device__ __forceinline__ void st_rows_cols(const DevSensor& S, const int4 rc, int sr, int sc, uint32_t& rows,
                                             uint32_t& cols) {
  const int M = grid_stride(S);
  const int x0 = sc << S.st_wl, y0 = sr << S.st_hl;
  const int wcap = M - x0 < (1 << S.st_wl) ? M - x0 : (1 << S.st_wl);
  cols = span_bits(rc.x - x0, rc.x + rc.z - x0, wcap);
  if (S.kind != kCamera) cols |= span_bits(rc.x - M - x0, rc.x + rc.z - M - x0, wcap);
  rows = span_bits(rc.y - y0, rc.y + rc.w - y0, 1 << S.st_hl);
}

// Visitor of the record-order scan of (visible, tile count) pairs.  A visible record gets its
// entry base (the record-order prefix of the tile counts: record r owns the adjoint slots
// [entry_base, entry_base + n_tiles)) and, at its compacted position, its depth key with the
// number of supertiles it meets in the top 24 bits (read back in depth order by the next scan).
// The closing block stores the visible and entry counts and the status.
struct VisibleVisit {
  const DevSensor* sens;
  int count;
  int64_t N;
  const int4* rect;
  const unsigned long long* dkey;
  int64_t* entry_base;
  uint64_t* keys;
  uint32_t* vals;
  int64_t* scalars;
  int64_t k_cap;
  SplatStatus* st;
  struct In {
    int4 rc;
    unsigned long long dk;
  };
  __device__ In load(int64_t i, P64 v) const {
    In in;
    if (v.a != 0) {
      in.rc = rect[i];
      in.dk = dkey[i];
    }
    return in;
  }
  __device__ void operator()(int64_t i, P64 p, P64 v, const In& in) const {
    if (v.a == 0) return;
    entry_base[i] = p.b;
    const DevSensor& S = sens[record_sensor(i, N, count)];
    const StSpan sp = st_span(S, in.rc);
    const uint64_t n_st = (uint64_t)(sp.nr * (sp.nc0 + sp.nc1));
    keys[p.a] = (n_st << kDepthKeyBits) | depth_sort_key(in.dk);
    vals[p.a] = (uint32_t)i;
  }
  __device__ void finish(P64 total) const {
    scalars[kScVisible] = total.a;
    scalars[kScEntries] = total.b;
    if (st) {
      st->n_isect = (unsigned long long)total.b;
      st->k_cap = (unsigned long long)k_cap;
      if (total.b > k_cap) st->overflow = 1u;
    }
  }
};

struct LoadVisibleTiles {
  const int32_t* n_tiles;
  __device__ P64 operator()(int64_t i) const {
    const int32_t nt = n_tiles[i];
    return nt > 0 ? P64((int64_t)1, (int64_t)nt) : P64(0);
  }
};

// supertile count of the i-th visible record in depth order, from its sorted packed key
// (entries past the visible count hold stale keys and count zero)
struct LoadPackedCount {
  const uint64_t* keys;
  const int64_t* n_vis;
  __device__ int64_t operator()(int64_t i) const {
    const uint64_t k = keys[i];
    return i < *n_vis ? (int64_t)(k >> kDepthKeyBits) : 0;
  }
};

// Closing step of the depth-order scan of supertile counts: the (supertile, record) entry
// count, or 0 when the (tile, Gaussian) entries overflow the capacity (the lists are then left
// empty).
struct CoarseCount {
  int64_t* scalars;
  int64_t cap;
  struct In {};
  template <typename T>
  __device__ In load(int64_t, T) const { return In{}; }
  template <typename T>
  __device__ void operator()(int64_t, T, T, In) const {}
  __device__ void finish(int64_t total) const {
    scalars[kScCoarse] = (scalars[kScEntries] > cap || total > cap) ? 0 : total;
  }
};

// A (supertile, record) entry's value: the Gaussian id in the low 32 bits, then the tile rows
// (bits 32-39) and columns (bits 40-47) of the supertile that the record's rectangle covers.
__device__ __forceinline__ uint64_t coarse_value(uint32_t gid, uint32_t rows, uint32_t cols) {
  return (uint64_t)gid | ((uint64_t)rows << 32) | ((uint64_t)cols << 40);
}

// Entry j (row-major over its supertile span) of a record: the supertile key and the value.
__device__ __forceinline__ void coarse_entry(const DevSensor& S, uint32_t st0, const int4 rc, const StSpan& sp,
                                             uint32_t gid, int j, uint32_t& key, uint64_t& val) {
  const int nc = sp.nc0 + sp.nc1;
  const int r = j / nc, c = j - r * nc;
  const int sr = sp.r0 + r;
  const int sc = c < sp.nc0 ? sp.c0 + c : c - sp.nc0;
  uint32_t rows, cols;
  st_rows_cols(S, rc, sr, sc, rows, cols);
  key = st0 + (uint32_t)sr * (uint32_t)S.st_x + (uint32_t)sc;
  val = coarse_value(gid, rows, cols);
}

// Visible record i (depth order) writes its (local supertile, record) entries from its offset
// coff[i] on.  Each lane writes the first kEmitOwn entries of its own record; the entries
// beyond that of the wavefront's larger records are then written by the whole wavefront, one
// record at a time, 64 entries per step.  The grid also empties the first n_st supertile
// ranges ([0, 0)) when the supertile sort leaves them to a ranges pass (n_st = 0 otherwise).
constexpr int kEmitOwn = 4;

__global__ __launch_bounds__(256) void k_coarse_emit(const DevSensor* __restrict__ sens, int count, int64_t N,
                                                     const int4* __restrict__ rect, const uint32_t* __restrict__ order,
                                                     const int64_t* __restrict__ coff,
                                                     const int64_t* __restrict__ scalars, int64_t n_cap,
                                                     uint32_t* __restrict__ ckeys, uint64_t* __restrict__ cvals,
                                                     int64_t cap, uint32_t* __restrict__ crange, int64_t n_st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  for (int64_t z = i; z < 2 * n_st; z += (int64_t)gridDim.x * blockDim.x) crange[z] = 0u;
  const bool valid = i < n_cap && i < scalars[kScVisible] && scalars[kScCoarse] != 0;
  uint32_t rec = 0, gid = 0;
  int64_t q0 = 0;
  int s = 0, cnt = 0;
  int4 rc = make_int4(0, 0, 0, 0);
  StSpan sp{0, 0, 0, 0, 0};
  if (valid) {
    rec = order[i];
    q0 = coff[i];
    s = record_sensor(rec, N, count);
    rc = rect[rec];
    sp = st_span(sens[s], rc);
    gid = (uint32_t)((int64_t)rec - (int64_t)s * N);
    cnt = sp.nr * (sp.nc0 + sp.nc1);
  }
  if (valid) {
    const DevSensor& S = sens[s];
    const uint32_t st0 = (uint32_t)(S.st_base - sens[0].st_base);
    for (int j = 0; j < cnt && j < kEmitOwn; ++j) {
      uint32_t key;
      uint64_t val;
      coarse_entry(S, st0, rc, sp, gid, j, key, val);
      if (q0 + j < cap) {
        ckeys[q0 + j] = key;
        cvals[q0 + j] = val;
      }
    }
  }
  uint64_t heavy = __ballot(cnt > kEmitOwn);
  while (heavy) {   // uniform
    const int l = __ffsll((unsigned long long)heavy) - 1;
    heavy &= heavy - 1;
    const int sl = __builtin_amdgcn_readlane(s, l);
    const int4 rl = make_int4(__builtin_amdgcn_readlane(rc.x, l), __builtin_amdgcn_readlane(rc.y, l),
                              __builtin_amdgcn_readlane(rc.z, l), __builtin_amdgcn_readlane(rc.w, l));
    const StSpan pl{__builtin_amdgcn_readlane(sp.r0, l), __builtin_amdgcn_readlane(sp.nr, l),
                    __builtin_amdgcn_readlane(sp.c0, l), __builtin_amdgcn_readlane(sp.nc0, l),
                    __builtin_amdgcn_readlane(sp.nc1, l)};
    const uint32_t gl = (uint32_t)__builtin_amdgcn_readlane((int)gid, l);
    const int64_t ql = ((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)q0, l)) |
                       ((int64_t)__builtin_amdgcn_readlane((int)(q0 >> 32), l) << 32);
    const int cl = __builtin_amdgcn_readlane(cnt, l);
    const DevSensor& S = sens[sl];
    const uint32_t st0 = (uint32_t)(S.st_base - sens[0].st_base);
    for (int j = kEmitOwn + lane; j < cl; j += 64) {
      uint32_t key;
      uint64_t val;
      coarse_entry(S, st0, rl, pl, gl, j, key, val);
      if (ql + j < cap) {
        ckeys[ql + j] = key;
        cvals[ql + j] = val;
      }
    }
  }
}

// Coarse entries are cut into items of at most kItemEntries consecutive entries of one
// supertile; every supertile has at least one item (possibly empty), whose first one also
// writes the supertile's tile ranges.  One wavefront handles an item.
constexpr int kItemEntries = 256;

inline int64_t item_capacity(int64_t n_supertiles, int64_t k_cap) { return n_supertiles + div_up(k_cap, kItemEntries); }

struct LoadItemCount {
  const uint2* crange;
  int64_t n_st;
  __device__ int64_t operator()(int64_t i) const {
    if (i >= n_st) return 0;
    const uint2 r = crange[i];
    const int64_t c = (int64_t)(r.y - r.x);
    return c > kItemEntries ? (c + kItemEntries - 1) / kItemEntries : 1;
  }
};

// the count array: 64 x items counts, then a zero (so that the scan's last element is the total)
struct LoadCountX {
  const uint32_t* cnt;
  const int64_t* n_x;
  __device__ uint32_t operator()(int64_t i) const { return i + 1 < *n_x ? cnt[i] : 0u; }
};

// Closing step of the scan of item counts over supertiles: the count array's size.
struct ItemsVisit {
  int64_t* scalars;
  struct In {};
  template <typename T>
  __device__ In load(int64_t, T) const { return In{}; }
  template <typename T>
  __device__ void operator()(int64_t, T, T, In) const {}
  __device__ void finish(int64_t total) const { scalars[kScItemsX] = total * 64 + 1; }
};

// One wavefront per supertile b: item_st[item] = (b, sensor of b) for each of its items.
__global__ __launch_bounds__(256) void k_item_table(const DevSensor* __restrict__ sens, int count,
                                                    const int64_t* __restrict__ item_first, int64_t n_st,
                                                    uint2* __restrict__ item_st) {
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= n_st) return;   // uniform over the wavefront
  int lo = 0, hi = count - 1;   // last sensor whose first supertile <= b
  const int64_t b0 = sens[0].st_base;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sens[mid].st_base - b0 <= b) lo = mid; else hi = mid - 1;
  }
  const int64_t first = item_first[b], n = item_first[b + 1] - first;
  for (int64_t j = threadIdx.x & 63; j < n; j += 64) item_st[first + j] = make_uint2((uint32_t)b, (uint32_t)lo);
}

// the item's supertile (its index in the call and its sensor), first entry and entry count
struct ItemView {
  int64_t st, first_item, n_items;
  int s;
  int sr, sc;
  int64_t p0;
  int cnt;
};

__device__ __forceinline__ ItemView item_view(const DevSensor* sens, const uint2* item_st, const int64_t* item_first,
                                              const uint2* crange, int64_t it) {
  ItemView v;
  const uint2 bs = item_st[it];
  v.st = bs.x;
  v.s = (int)bs.y;
  v.first_item = item_first[bs.x];
  v.n_items = item_first[bs.x + 1] - v.first_item;
  const DevSensor& S = sens[v.s];
  const int q = (int)((int64_t)bs.x - (S.st_base - sens[0].st_base));
  v.sr = q / S.st_x;
  v.sc = q - v.sr * S.st_x;
  const uint2 r = crange[bs.x];
  v.p0 = (int64_t)r.x + (it - v.first_item) * kItemEntries;
  const int64_t rest = (int64_t)r.y - v.p0;
  v.cnt = (int)(rest < 0 ? 0 : (rest > kItemEntries ? kItemEntries : rest));
  return v;
}

// Position of (item it, tile f of its supertile) in the count array: supertile-major, then f,
// then the supertile's items, so that one exclusive scan of the array gives every item the
// first list position of each of its tiles, the supertiles' tiles laid out one after another.
__device__ __forceinline__ int64_t count_slot(const ItemView& v, int64_t it, int f) {
  return v.first_item * 64 + (int64_t)f * v.n_items + (it - v.first_item);
}

// The items of supertiles [st_lo, st_hi) are spread over a fixed grid; wavefront w of block b
// takes items first + b * 4 + w + k * 4 * grid.
#define FOR_EACH_ITEM(it)                                                                          \
  const int64_t it_end_ = item_first[st_hi];                                                       \
  for (int64_t it = item_first[st_lo] + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); it < it_end_; \
       it += (int64_t)gridDim.x * 4)

// An item's coarse entries (at most kItemEntries = 4 rounds of 64, one per lane), loaded up
// front; an entry past the item covers nothing.
constexpr int kItemRounds = kItemEntries / 64;
static_assert(kItemRounds * 64 == kItemEntries, "items are whole rounds of 64 entries");

struct ItemEntries {
  uint64_t val[kItemRounds];
};

__device__ __forceinline__ void load_item(const ItemView& v, const uint64_t* __restrict__ cvals, int lane,
                                          ItemEntries& e) {
#pragma unroll
  for (int k = 0; k < kItemRounds; ++k) {
    const int j = k * 64 + lane;
    e.val[k] = j < v.cnt ? cvals[v.p0 + j] : 0ull;
  }
}

__device__ __forceinline__ uint32_t entry_rows(uint64_t val) { return (uint32_t)(val >> 32) & 0xFFu; }
__device__ __forceinline__ uint32_t entry_cols(uint64_t val) { return (uint32_t)(val >> 40) & 0xFFu; }

// Ballots of one round over supertiles of 2^WL x 2^HL tiles: rb[y] = lanes covering tile row
// y, cb[x] = lanes covering tile column x; the lanes covering tile (y, x) are rb[y] & cb[x].
// my = that set for the lane's own tile f = lane = y * 8 + x (empty for lanes outside).
template <int WL, int HL>
struct RoundBallots {
  uint64_t rb[1 << HL], cb[1 << WL];
  uint64_t my;
};

template <int WL, int HL>
__device__ __forceinline__ void round_ballots(uint32_t rows, uint32_t cols, int lane, RoundBallots<WL, HL>& b) {
  uint64_t myr = 0, myc = 0;
#pragma unroll
  for (int k = 0; k < (1 << HL); ++k) {
    b.rb[k] = __ballot((rows >> k) & 1u);
    myr = (lane >> 3) == k ? b.rb[k] : myr;
  }
#pragma unroll
  for (int k = 0; k < (1 << WL); ++k) {
    b.cb[k] = __ballot((cols >> k) & 1u);
    myc = (lane & 7) == k ? b.cb[k] : myc;
  }
  b.my = myr & myc;
}

// Per item of the supertiles [st_lo, st_hi) (all of one supertile shape): the number of its
// coarse entries meeting each tile f of the supertile (lane f accumulates), written to the
// count array.
template <int WL, int HL>
__global__ __launch_bounds__(256) void k_st_count(const DevSensor* __restrict__ sens,
                                                  const uint64_t* __restrict__ cvals, const uint2* __restrict__ crange,
                                                  const int64_t* __restrict__ item_first,
                                                  const uint2* __restrict__ item_st, int64_t st_lo, int64_t st_hi,
                                                  uint32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  FOR_EACH_ITEM(it) {
    const ItemView v = item_view(sens, item_st, item_first, crange, it);
    ItemEntries e;
    load_item(v, cvals, lane, e);
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItemRounds; ++k) {
      if (k * 64 >= v.cnt) break;   // uniform
      RoundBallots<WL, HL> b;
      round_ballots<WL, HL>(entry_rows(e.val[k]), entry_cols(e.val[k]), lane, b);
      acc += (uint32_t)__popcll(b.my);
    }
    cnt[count_slot(v, it, lane)] = acc;
  }
}

// Per item of the supertiles [st_lo, st_hi): every coarse entry's Gaussian id goes to each of
// its tiles' lists, at the item's scanned first position for that tile plus the entry's rank
// among the item's earlier entries meeting the same tile (lanes below it in the tile's ballot
// set; lane f carries tile f's next position across rounds), so each list keeps the depth order
// of the coarse entries.  The tiles are visited in a uniform loop over the round's nonempty
// (row, column) ballot pairs.  The first item of a supertile also writes its tiles' [start,
// end) ranges.
template <int WL, int HL>
__global__ __launch_bounds__(256) void k_st_place(const DevSensor* __restrict__ sens,
                                                  const uint64_t* __restrict__ cvals, const uint2* __restrict__ crange,
                                                  const int64_t* __restrict__ item_first,
                                                  const uint2* __restrict__ item_st, int64_t st_lo, int64_t st_hi,
                                                  const uint32_t* __restrict__ pos0, int64_t k_cap,
                                                  int32_t* __restrict__ gauss, longlong2* __restrict__ tile_range) {
  const int lane = threadIdx.x & 63;
  FOR_EACH_ITEM(it) {
    const ItemView v = item_view(sens, item_st, item_first, crange, it);
    ItemEntries e;
    load_item(v, cvals, lane, e);
    const uint32_t start = pos0[count_slot(v, it, lane)];
    if (it == v.first_item) {   // the supertile's tile ranges (tiles inside the sensor's grid)
      const DevSensor& S = sens[v.s];
      const int fy = lane >> 3, fx = lane & 7;
      const int row = (v.sr << HL) + fy, col = (v.sc << WL) + fx;
      if (fy < (1 << HL) && fx < (1 << WL) && row < grid_rows(S) && col < grid_stride(S)) {
        const int64_t t = (S.tile_base - sens[0].tile_base) + (int64_t)row * grid_stride(S) + col;
        const uint32_t end = pos0[v.first_item * 64 + (int64_t)(lane + 1) * v.n_items];
        tile_range[t] = make_longlong2((long long)start, (long long)end);
      }
    }
    uint32_t run = start;
#pragma unroll
    for (int k = 0; k < kItemRounds; ++k) {
      if (k * 64 >= v.cnt) break;   // uniform
      const uint32_t rows = entry_rows(e.val[k]), cols = entry_cols(e.val[k]);
      RoundBallots<WL, HL> b;
      round_ballots<WL, HL>(rows, cols, lane, b);
      const int32_t gid = (int32_t)(uint32_t)e.val[k];
#pragma unroll
      for (int y = 0; y < (1 << HL); ++y) {
        if (b.rb[y] == 0) continue;   // uniform
#pragma unroll
        for (int x = 0; x < (1 << WL); ++x) {
          const uint64_t m = b.rb[y] & b.cb[x];
          if (m == 0) continue;   // uniform
          const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)run, y * 8 + x);
          const uint32_t p = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if (((rows >> y) & (cols >> x) & 1u) && (int64_t)p < k_cap) gauss[p] = gid;
        }
      }
      run += (uint32_t)__popcll(b.my);
    }
  }
}

constexpr int kRangeItems = 8;   // sorted keys per thread of k_ranges

// [start, end) of every key's run in a sorted key array; keys that do not occur keep the range
// the caller filled in.  Thread t of a block handles elements base + j * 256 + t (coalesced).
// The run of key k is range[(k >> shift) + offset].
// R2: int2 (ray bins) or uint2 (coarse entries, up to 2^32 - 1 of them)
template <typename R2>
__global__ void k_ranges(const uint32_t* __restrict__ keys, const int64_t* n_ptr, int64_t n_cap, R2* __restrict__ range,
                         int shift, int64_t offset) {
  using E = decltype(R2::x);
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * kRangeItems + threadIdx.x;
  const int64_t n = sort_count(n_ptr, n_cap);
  if ((int64_t)blockIdx.x * blockDim.x * kRangeItems >= n) return;   // uniform; n >= 1 below
  auto at = [&](int64_t i) { return keys[i < 0 ? 0 : (i < n ? i : n - 1)] >> shift; };   // clamped: no branch per load
  uint32_t cur[kRangeItems], prev[kRangeItems], next[kRangeItems];
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const int64_t i = base + (int64_t)j * blockDim.x;
    const uint32_t c = at(i), p = at(i - 1), x = at(i + 1);
    cur[j] = i < n ? c : 0xFFFFFFFFu;
    prev[j] = (i > 0 && i <= n) ? p : 0xFFFFFFFFu;
    next[j] = i + 1 < n ? x : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const int64_t i = base + (int64_t)j * blockDim.x;
    if (i >= n) break;
    if (prev[j] != cur[j]) range[cur[j] + offset].x = (E)i;
    if (next[j] != cur[j]) range[cur[j] + offset].y = (E)(i + 1);
  }
}

// ---- lidar rays ------------------------------------------------------------------------------
__device__ __forceinline__ int sensor_of_ray(const DevSensor* sens, int count, int64_t r) {
  int lo = 0, hi = count - 1;
  const int64_t b0 = sens[0].ray_base;
  while (lo < hi) {   // last sensor whose local ray base <= r
    int mid = (lo + hi + 1) >> 1;
    if (sens[mid].ray_base - b0 <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// lidar rays [r0, r0 + n) of the call -> (key, ray id) pairs at [0, n); key = ((bin - t0) <<
// cell_bits) | cell, bin = the ray's tile (n_tiles: outside every tile), t0 = the call's first
// lidar tile, cell = ray_cell_code inside the tile (0 outside), or the ray's 16-bit priority
// when its lidar caps the rays per tile (training time).  The grid also empties the n_bins ray
// ranges ([0, 0)), which the ranges pass after the ray sort fills in.
__global__ void k_ray_keys(const DevSensor* __restrict__ sens, int count, int64_t r0, int64_t n, int64_t n_tiles,
                           int64_t t0, int cell_bits, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                           SplatStatus* st, int32_t* __restrict__ ray_range, int64_t n_bins) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t z = q; z < 2 * n_bins; z += (int64_t)gridDim.x * blockDim.x) ray_range[z] = 0;
  if (q >= n) return;
  const int64_t r = r0 + q;
  int s = sensor_of_ray(sens, count, r);
  const DevSensor& S = sens[s];
  int64_t j = r - (S.ray_base - sens[0].ray_base);
  float az = S.ray_az[j], el = S.ray_el[j], t = S.ray_t[j];
  bool ok = (az >= 0.f) && (az < kTwoPi) && (el >= S.bounds[0]) && (el < S.bounds[S.m_el]) && finite_f(t);
  uint32_t tile = (uint32_t)n_tiles, cell = 0;
  if (ok) {
    const float u = div_rn(az, S.az_w);
    int a = floor_div_clamped(az, S.az_w) % S.m_az;
    int e = count_le(S, el) - 1;
    tile = (uint32_t)(local_tile_base(sens, s) + (int64_t)e * S.m_az + a);
    // training-time cap: the ray's priority orders the tile (its first rays are the ones kept)
    cell = S.ray_prio ? (uint32_t)S.ray_prio[j] : ray_cell_code(u, el, S.bounds[e], S.bounds[e + 1], cell_bits);
  } else if (st) {
    atomicAdd(&st->n_rays_invalid, 1u);
  }
  if (ok && st && fabsf(t) > 0.5f * S.t_rs * (1.0f + 1e-6f) + 1e-9f) atomicAdd(&st->n_rays_time, 1u);
  keys[q] = ((tile - (uint32_t)t0) << cell_bits) | cell;
  vals[q] = (uint32_t)r;
}

__device__ __forceinline__ bool camera_tile(const DevSensor* sens, int count, int64_t t, int64_t n_tiles) {
  if (t >= n_tiles) return false;
  int lo = 0, hi = count - 1;
  const int64_t b0 = sens[0].tile_base;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (sens[mid].tile_base - b0 <= t) lo = mid; else hi = mid - 1;
  }
  return sens[lo].kind == kCamera;
}

// work items per bin: one per camera tile, ceil(rays / 256) per lidar tile and for the bin of
// rays outside every tile (bin n_tiles); also clears the split flag n_work[2], which k_work_emit
// sets
__global__ void k_work_count(const DevSensor* __restrict__ sens, int count, const int2* __restrict__ range,
                             int64_t n_tiles, int64_t* __restrict__ cnt, int32_t* __restrict__ n_work) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) n_work[2] = 0;
  if (t > n_tiles) return;
  if (camera_tile(sens, count, t, n_tiles)) {
    cnt[t] = 1;
    return;
  }
  int2 r = range[t];
  int64_t c = r.y - r.x;
  cnt[t] = c > 0 ? (c + SPLAT_RAYS_PER_ITEM - 1) / SPLAT_RAYS_PER_ITEM : 0;
}

__global__ void k_work_emit(const DevSensor* __restrict__ sens, int count, const int2* __restrict__ range,
                            int64_t n_tiles, const int64_t* __restrict__ woff, int64_t work_cap,
                            int2* __restrict__ work, int32_t* __restrict__ n_work) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    int64_t tot = woff[n_tiles + 1];
    *n_work = (int32_t)(tot < work_cap ? tot : work_cap);
  }
  if (t > n_tiles) return;
  int64_t o = woff[t];
  if (camera_tile(sens, count, t, n_tiles)) {
    if (o < work_cap) work[o] = make_int2((int)t, 0);
    return;
  }
  int2 r = range[t];
  if (t < n_tiles && r.y - r.x > SPLAT_RAYS_PER_ITEM) n_work[2] = 1;   // a split lidar tile
  for (int p = r.x; p < r.y; p += SPLAT_RAYS_PER_ITEM, ++o)
    if (o < work_cap) work[o] = make_int2((int)t, p);
}

// Order of the persistent queue: longest processing time first, sorted (stably) by the
// descending estimated cost of an item, from an 8-bit log-scale code of its tile list length (4
// bits of exponent, 4 of mantissa: buckets of about 6 %).  Two forms:
//   grouped (the adjoint keeps per-entry rows): the lidar items, then the camera items, each
//     part by cost (key (camera << 7) | (127 - code / 2)): each kind's records stay hot in
//     cache while its items run;
//   mixed (the adjoint adds every pair atomically): one cost order over both kinds, a lidar
//     chunk's list counted 4x longer (key 255 - min(255, code + 32 if lidar)): interleaving the
//     kinds spreads the atomic traffic over the kernel's run.
__device__ __forceinline__ uint32_t length_code(int64_t len) {
  const uint32_t x = (uint32_t)(len < 0xFFFFF ? len : 0xFFFFF) + 1u;   // >= 1
  const int e = 31 - __clz(x);                                       // 0..20
  const uint32_t m = e >= 4 ? (x >> (e - 4)) & 15u : (x << (4 - e)) & 15u;
  const uint32_t c = ((uint32_t)e << 4) | m;
  return c < 255u ? c : 255u;
}

// tiles [0, lidar_tile0) are camera tiles (cameras precede lidars in a call)
__global__ void k_queue_keys(const int2* __restrict__ work, const int32_t* __restrict__ n_work,
                             const longlong2* __restrict__ tile_range, int64_t n_tiles, int64_t lidar_tile0,
                             bool grouped, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_work) return;
  int64_t t = work[i].x;
  int64_t len = 0;
  if (t < n_tiles) {
    const longlong2 r = tile_range[t];
    len = r.y - r.x;
  }
  const bool camera = t < lidar_tile0;
  const uint32_t c = length_code(len);
  if (grouped) {
    keys[i] = (camera ? 128u : 0u) | (127u - (c >> 1));
  } else {
    const uint32_t w = c + (camera ? 0u : 32u);
    keys[i] = 255u - (w < 255u ? w : 255u);
  }
  vals[i] = (uint32_t)i;
}

__global__ void k_queue_gather(const int2* __restrict__ src, const uint32_t* __restrict__ order,
                               const int32_t* __restrict__ n_work, int2* __restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_work) return;
  dst[i] = src[order[i]];
}

// ------------------------------------------------------------------------------------------
// host driver
// ------------------------------------------------------------------------------------------
static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

Workspace carve_workspace(void* base, int64_t n_rec, int64_t k_cap, int64_t n_tiles, int64_t n_rays, int c_max) {
  Workspace w;
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* r = base ? (void*)(p + off) : nullptr;
    off += align256(bytes);
    return r;
  };
  int64_t nrec = n_rec < 1 ? 1 : n_rec;
  int64_t kc = k_cap < 1 ? 1 : k_cap;
  int64_t nr = n_rays < 1 ? 1 : n_rays;
  // the longest sort sharing `hist`: records, coarse entries or queue entries
  const int64_t wq = work_capacity(n_tiles, nr) + 1;
  int64_t max_n = nrec > kc ? nrec : kc;
  max_n = max_n > wq ? max_n : wq;
  int64_t max_blocks = div_up(max_n, kRadixTile);
  for (int i = 0; i < 2; ++i) w.dkeys[i] = (uint64_t*)take(nrec * 8);
  for (int i = 0; i < 2; ++i) w.dvals[i] = (uint32_t*)take(nrec * 4);
  w.coff = (int64_t*)take(nrec * 8);
  w.scan_part = take((div_up(nrec > n_tiles + 2 ? nrec : n_tiles + 2, scan_tile<P64>()) + 2) * 16);
  for (int i = 0; i < 2; ++i) w.ckeys[i] = (uint32_t*)take(kc * 4);
  for (int i = 0; i < 2; ++i) w.cvals[i] = (uint64_t*)take(kc * 8);
  const int64_t nst = n_tiles < 1 ? 1 : n_tiles;   // supertiles <= tiles
  w.crange = (uint2*)take(nst * 8);
  w.item_first = (int64_t*)take((nst + 1) * 8);
  w.item_st = (uint2*)take(item_capacity(nst, kc) * 8);
  const int64_t xcap = item_capacity(nst, kc) * 64 + 1;
  w.xcount = (uint32_t*)take(xcap * 4);
  w.xpart = (uint32_t*)take((div_up(xcap, kScanTile) + 2) * 4);
  w.hist = (uint32_t*)take((size_t)kRadixBins * max_blocks * 4 + 64);
  w.coltotal = (uint32_t*)take(kRadixBins * 4);
  w.rhist = (uint32_t*)take((size_t)kRadixBins * div_up(nr, kRadixTile) * 4 + 64);
  w.rcoltotal = (uint32_t*)take(kRadixBins * 4);
  for (int i = 0; i < 2; ++i) w.rkeys[i] = (uint32_t*)take(nr * 4);
  for (int i = 0; i < 2; ++i) w.rvals[i] = (uint32_t*)take(nr * 4);
  const int64_t wcap = work_capacity(n_tiles, nr) + 1;
  for (int i = 0; i < 2; ++i) w.qkeys[i] = (uint32_t*)take(wcap * 4);
  for (int i = 0; i < 2; ++i) w.qvals[i] = (uint32_t*)take(wcap * 4);
  w.qtmp = (int2*)take(wcap * 8);
  w.wcount = (int64_t*)take((n_tiles + 2) * 8);
  w.wpart = (int64_t*)take((div_up(n_tiles + 2, kScanTile) + 2) * 8);
  w.scalars = (int64_t*)take(kScCount * 8);
  const size_t sort_bytes = off;
  // adjoint buffers start over at the base
  off = 0;
  w.stride = slot_stride(cmax_bucket(c_max));
  w.rows = k_cap <= adjoint_row_limit();
  const int64_t kr = w.rows ? kc : 1;   // rows and flags only while they are kept
  w.slots = (float*)take((size_t)kr * w.stride * 4);
  w.flags = (uint8_t*)take((size_t)div_up(kr, 4) * 4);
  w.g2d = (float*)take((size_t)nrec * kNV * 4);
  w.rflag = (uint8_t*)take((size_t)div_up(nrec, 4) * 4);
  w.long_cap = w.rows ? long_part_cap(nrec, kc) : 1;
  w.long_list = (uint32_t*)take((size_t)kLongParts * w.long_cap * 8);
  w.n_long = (int32_t*)take(kLongParts * 4);
  w.qctr = (int32_t*)take(4);
  w.bytes = off > sort_bytes ? off : sort_bytes;
  return w;
}

// 6. lidar rays -> tiles; work item counts and offsets; work items (lidar chunks, and camera
//    tiles in the batched form; there into qtmp, ordered by the queue pass).  Reads no Gaussian
//    data, so it may run on a stream of its own beside steps 1-5.
static hipError_t launch_ray_bins(const CallView& v, const SplatTileLists& L, const Workspace& w, SplatStatus* st,
                                  hipStream_t s) {
  hipError_t e;
  const int64_t bins = v.n_tiles + 1;
  const int64_t r0 = v.lidar_ray0;
  const int64_t nr = v.n_rays - r0;
  if (nr > 0) {
    // rays grouped by tile, and inside a tile in Z-order of their cells (compact work items);
    // the cell code fills the unused bits of the bin's last radix digit, so it adds no pass
    // (under the training-time cap 16 bits of priority take its place, and add passes)
    const int64_t t0 = v.lidar_tile0;
    const int bin_bits = bits_for(bins - t0);
    const int cell_bits = v.ray_cap ? 16 : ray_cell_bits(bin_bits);   // make_view keeps bin_bits <= 16
    hipLaunchKernelGGL(k_ray_keys, dim3((unsigned)div_up(nr, 256)), dim3(256), 0, s, v.sens, v.count, r0, nr,
                       v.n_tiles, t0, cell_bits, w.rkeys[0], w.rvals[0], st, L.ray_range, bins);
    uint32_t* rk[2] = {w.rkeys[0], w.rkeys[1]};
    uint32_t* rv[2] = {w.rvals[0], w.rvals[1]};
    int rcur = 0;
    if ((e = radix_sort<uint32_t, uint32_t>(rk, rv, rcur, nullptr, nr, 0, bin_bits + cell_bits, w.rhist,
                                            w.rcoltotal, (uint32_t*)L.ray_order, s)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_ranges<int2>, dim3((unsigned)div_up(nr, 256 * kRangeItems)), dim3(256), 0, s,
                       (const uint32_t*)rk[rcur], (const int64_t*)nullptr, nr, (int2*)L.ray_range, cell_bits, t0);
  } else if ((e = fill<int32_t>(L.ray_range, 2 * bins, 0, s)) != hipSuccess) {
    return e;
  }
  hipLaunchKernelGGL(k_work_count, dim3((unsigned)div_up(bins, 256)), dim3(256), 0, s, v.sens, v.count,
                     (const int2*)L.ray_range, v.n_tiles, w.wcount, L.n_work);
  // per-bin offsets, and the total behind them for k_work_emit
  if ((e = device_scan<int64_t>(LoadI64{w.wcount}, bins, w.wcount, w.wpart, s, StoreTotal{w.wcount + bins})) !=
      hipSuccess)
    return e;
  int2* wdst = v.queue ? w.qtmp : (int2*)L.work;
  hipLaunchKernelGGL(k_work_emit, dim3((unsigned)div_up(bins, 256)), dim3(256), 0, s, v.sens, v.count,
                     (const int2*)L.ray_range, v.n_tiles, (const int64_t*)w.wcount, L.work_cap, wdst, L.n_work);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const CallView& v, const SplatProjected& p, const SplatTileLists& L, const Workspace& w,
                           SplatStatus* st, hipStream_t s) {
  const int64_t n_rec = (int64_t)v.count * v.n_gauss;
  hipError_t e;
  int64_t* const sc = w.scalars;
  // 6. first, so that it overlaps the rest: on the side stream, forked from the call's stream
  const bool rays = v.has_lidar || v.queue;
  const bool fork = rays && v.side && v.fork && v.join;
  if (rays) {
    if (fork) {
      if ((e = hipEventRecord(v.fork, s)) != hipSuccess || (e = hipStreamWaitEvent(v.side, v.fork, 0)) != hipSuccess)
        return e;
    }
    if ((e = launch_ray_bins(v, L, w, st, fork ? v.side : s)) != hipSuccess) return e;
    if (fork && (e = hipEventRecord(v.join, v.side)) != hipSuccess) return e;
  }
  // 1. one record-order scan of (visible, tile count): entry bases, the visible records'
  //    packed depth keys compacted in record order, the counts and the overflow status
  if ((e = device_scan<P64>(LoadVisibleTiles{p.n_tiles}, n_rec, (P64*)nullptr, (P64*)w.scan_part, s,
                            VisibleVisit{v.sens, v.count, v.n_gauss, (const int4*)p.rect,
                                         (const unsigned long long*)p.dkey, L.entry_base, w.dkeys[0], w.dvals[0], sc,
                                         L.k_cap, st})) != hipSuccess)
    return e;
  // 2. stable sort of the visible records by the 32-bit depth key (ties keep record order)
  uint64_t* dk[2] = {w.dkeys[0], w.dkeys[1]};
  uint32_t* dvv[2] = {w.dvals[0], w.dvals[1]};
  int cur = 0;
  if ((e = radix_sort<uint64_t, uint32_t>(dk, dvv, cur, sc + kScVisible, n_rec, 0, kDepthKeyBits, w.hist, w.coltotal,
                                nullptr, s)) != hipSuccess)
    return e;
  // 3. depth-order scan of the supertile counts, emitting (supertile, record) entries in depth
  //    order
  if ((e = device_scan<int64_t>(LoadPackedCount{dk[cur], sc + kScVisible}, n_rec, w.coff, (int64_t*)w.scan_part, s,
                                CoarseCount{sc, L.k_cap}, sc + kScVisible)) != hipSuccess)
    return e;
  const int64_t n_st = v.n_supertiles;
  // with at most kRadixBins supertiles step 4 is one radix pass, whose scatter writes the
  // supertile ranges; otherwise the emit clears them and a ranges pass fills them in
  const bool one_pass = n_st <= kRadixBins && L.k_cap > 0;
  if (n_rec > 0)
    hipLaunchKernelGGL(k_coarse_emit, dim3((unsigned)div_up(n_rec, 256)), dim3(256), 0, s, v.sens, v.count, v.n_gauss,
                       (const int4*)p.rect, (const uint32_t*)dvv[cur], (const int64_t*)w.coff, (const int64_t*)sc, n_rec,
                       w.ckeys[0], w.cvals[0], L.k_cap, (uint32_t*)w.crange, one_pass ? (int64_t)0 : n_st);
  else if ((e = fill<int32_t>((int32_t*)w.crange, 2 * n_st, 0, s)) != hipSuccess)   // [0, 0): empty
    return e;
  // 4. stable sort of the entries by supertile: each supertile's records stay in depth order
  uint32_t* ck[2] = {w.ckeys[0], w.ckeys[1]};
  uint64_t* cv[2] = {w.cvals[0], w.cvals[1]};
  int ccur = 0;
  if ((e = radix_sort<uint32_t, uint64_t>(ck, cv, ccur, sc + kScCoarse, L.k_cap, 0, bits_for(n_st), w.hist, w.coltotal,
                                nullptr, s, one_pass ? w.crange : nullptr, (int)(one_pass ? n_st : 0))) != hipSuccess)
    return e;
  if (L.k_cap > 0 && !one_pass)
    hipLaunchKernelGGL(k_ranges<uint2>, dim3((unsigned)div_up(L.k_cap, 256 * kRangeItems)), dim3(256), 0, s,
                       (const uint32_t*)ck[ccur], (const int64_t*)(sc + kScCoarse), L.k_cap, w.crange, 0, (int64_t)0);
  // 5. items of <= kItemEntries entries per supertile; per item and tile the entry counts; their
  //    scan gives every tile its list range and every item its first positions; placement
  if ((e = device_scan<int64_t>(LoadItemCount{w.crange, n_st}, n_st + 1, w.item_first, (int64_t*)w.scan_part, s,
                                ItemsVisit{sc})) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_item_table, dim3((unsigned)div_up(n_st, 4)), dim3(256), 0, s, v.sens, v.count,
                     (const int64_t*)w.item_first, n_st, w.item_st);
  // cameras precede lidars: supertiles [0, st_cam) have the camera shape, the rest the lidar one
  int64_t st_cam = 0;
  for (int i = 0; i < v.count; ++i)
    if (v.host[i].kind == kCamera) st_cam += (int64_t)v.host[i].st_x * v.host[i].st_y;
  const int64_t icap = item_capacity(n_st, L.k_cap);
  int64_t grid = div_up(icap, 4);
  const int64_t gmax = (int64_t)(v.n_cu > 0 ? v.n_cu : 256) * 16;
  if (grid > gmax) grid = gmax;
  const uint64_t* cvs = cv[ccur];
  if (st_cam > 0)
    hipLaunchKernelGGL((k_st_count<kStLogCamera, kStLogCamera>), dim3((unsigned)grid), dim3(256), 0, s, v.sens, cvs,
                       (const uint2*)w.crange, (const int64_t*)w.item_first, (const uint2*)w.item_st, (int64_t)0, st_cam,
                       w.xcount);
  if (st_cam < n_st)
    hipLaunchKernelGGL((k_st_count<kStLogLidar, kStLogLidar>), dim3((unsigned)grid), dim3(256), 0, s, v.sens, cvs,
                       (const uint2*)w.crange, (const int64_t*)w.item_first, (const uint2*)w.item_st, st_cam, n_st,
                       w.xcount);
  if ((e = device_scan<uint32_t>(LoadCountX{w.xcount, sc + kScItemsX}, icap * 64 + 1, w.xcount, w.xpart, s,
                                 NoVisit(), sc + kScItemsX)) != hipSuccess)
    return e;
  if (st_cam > 0)
    hipLaunchKernelGGL((k_st_place<kStLogCamera, kStLogCamera>), dim3((unsigned)grid), dim3(256), 0, s, v.sens, cvs,
                       (const uint2*)w.crange, (const int64_t*)w.item_first, (const uint2*)w.item_st, (int64_t)0, st_cam,
                       (const uint32_t*)w.xcount, L.k_cap, L.gauss, (longlong2*)L.tile_range);
  if (st_cam < n_st)
    hipLaunchKernelGGL((k_st_place<kStLogLidar, kStLogLidar>), dim3((unsigned)grid), dim3(256), 0, s, v.sens, cvs,
                       (const uint2*)w.crange, (const int64_t*)w.item_first, (const uint2*)w.item_st, st_cam, n_st,
                       (const uint32_t*)w.xcount, L.k_cap, L.gauss, (longlong2*)L.tile_range);
  // join the ray binning; the batched form then orders its work items by cost
  if (fork && (e = hipStreamWaitEvent(s, v.join, 0)) != hipSuccess) return e;
  if (v.queue) {
    const int64_t bins = v.n_tiles + 1;
    // the work items never exceed work_capacity (the workspace's queue buffers and histograms
    // are sized for that many), whatever larger capacity the lists declare
    const int64_t wmax = work_capacity(v.n_tiles, v.n_rays) + 1;
    const int64_t wcap = L.work_cap < wmax ? L.work_cap : wmax;
    hipLaunchKernelGGL(k_queue_keys, dim3((unsigned)div_up(wcap, 256)), dim3(256), 0, s, (const int2*)w.qtmp,
                       (const int32_t*)L.n_work, (const longlong2*)L.tile_range, v.n_tiles, v.lidar_tile0, w.rows,
                       w.qkeys[0], w.qvals[0]);
    uint32_t* qk[2] = {w.qkeys[0], w.qkeys[1]};
    uint32_t* qv[2] = {w.qvals[0], w.qvals[1]};
    int qcur = 0;
    // item count: the scan total (clamped to the capacity by the sort)
    if ((e = radix_sort<uint32_t, uint32_t>(qk, qv, qcur, w.wcount + bins, wcap, 0, 8, w.hist, w.coltotal, nullptr, s)) !=
        hipSuccess)
      return e;
    hipLaunchKernelGGL(k_queue_gather, dim3((unsigned)div_up(wcap, 256)), dim3(256), 0, s, (const int2*)w.qtmp,
                       (const uint32_t*)qv[qcur], (const int32_t*)L.n_work, (int2*)L.work);
  }
  return hipGetLastError();
}

hipError_t launch_exclusive_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* part, hipStream_t s) {
  return device_scan<int64_t>(LoadI64{in}, n, out, part, s);
}

}  // namespace splat
