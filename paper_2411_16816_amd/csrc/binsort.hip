// binsort.hip -- tile binning and depth sorting (SplatAD, arXiv 2411.16816: Sec. 3.2
// "Projection, tiling, and sorting"; Sec. 3.3 "Tiling and sorting"; App. A).
//
// Pipeline of one call (all on the stream, no host synchronisation):
//   1. the visible records are compacted and stably sorted by a 40-bit key of their float64
//      depth, so equal keys keep record (= Gaussian id) order;
//   2. an exclusive scan of n_tiles in that order gives every record its slot range;
//   3. every record emits (local tile id, Gaussian id) pairs into its slots;
//   4. a stable LSD radix sort on the tile id groups the pairs by tile; inside a tile they stay in
//      (depth, id) order, which is the ordering the paper obtains from its (tile | depth) keys;
//   5. per-tile [start, end) ranges;
//   6. lidar: rays are binned into their tiles (a ray is a box of zero extent, App. A), invalid
//      rays go to an extra bin, and every tile's rays are cut into work items of <= 256 rays.
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
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) { return fill<int32_t>(p, n, v, s); }

__global__ void k_copy_i64(const int64_t* __restrict__ src, int64_t* __restrict__ dst) { *dst = *src; }

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

template <typename T, typename Load>
__global__ __launch_bounds__(256) void k_scan_reduce(Load ld, int64_t n, T* __restrict__ part) {
  __shared__ T tmp[4];
  int64_t base = (int64_t)blockIdx.x * kScanTile;   // < n: the grid has div_up(n, kScanTile) blocks
  T acc = 0;
  // indices clamped into [0, n): every load is issued unconditionally, back to back
#pragma unroll 4
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)r * kScanThreads + threadIdx.x;
    const T x = ld(i < n ? i : n - 1);
    acc += i < n ? x : (T)0;
  }
  T total;
  block_exclusive_scan<T>(acc, tmp, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Up to this many blocks every down-sweep block sums the block totals before it itself (one
// launch fewer); beyond it a single block scans the totals first.
constexpr int64_t kScanFusedBlocks = 1024;

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

// Block b: exclusive scan of its tile, offset by the total of the blocks before it: with
// `fused`, the sum of the block totals part[0..b) (read by the block itself; the last block
// writes the grand total to part[nb]), otherwise part[b] as scanned by k_scan_partials.
// no per-element work besides the scan
struct NoVisit {
  template <typename T>
  __device__ void operator()(int64_t, T, T) const {}
};

template <typename T, typename Load, typename Visit>
__global__ __launch_bounds__(256) void k_scan_down(Load ld, int64_t n, T* __restrict__ part, int64_t nb, bool fused,
                                                   T* __restrict__ out, Visit vis) {
  // element li of the tile lives at pad(li) = li + li / 16: a thread's 16 consecutive
  // elements then start 17 apart, which spreads the per-thread pass over the LDS banks
  __shared__ T tile[kScanTile + kScanTile / kScanItems];
  __shared__ T tmp[4];
  auto pad = [](int li) { return li + (li >> 4); };
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  T before;
  if (fused) {
    T pb = 0;
    for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) pb += part[i];
    block_exclusive_scan<T>(pb, tmp, before);
  } else {
    before = part[blockIdx.x];
  }
#pragma unroll 4
  for (int r = 0; r < kScanItems; ++r) {
    const int64_t i = base + (int64_t)r * kScanThreads + threadIdx.x;
    const T x = ld(i < n ? i : n - 1);
    tile[pad(r * kScanThreads + threadIdx.x)] = i < n ? x : (T)0;
  }
  __syncthreads();
  T loc[kScanItems];
  T acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    loc[k] = acc;
    acc += tile[pad(threadIdx.x * kScanItems + k)];
  }
  T total;
  T pre = block_exclusive_scan<T>(acc, tmp, total) + before;
  if (fused && blockIdx.x == nb - 1 && threadIdx.x == 0) part[nb] = before + total;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) tile[pad(threadIdx.x * kScanItems + k)] = pre + loc[k];
  __syncthreads();
  const T end = before + total;   // exclusive prefix after the block
#pragma unroll 4
  for (int r = 0; r < kScanItems; ++r) {
    const int li = r * kScanThreads + threadIdx.x;
    const int64_t i = base + li;
    if (i < n) {
      const T p = tile[pad(li)];
      out[i] = p;
      vis(i, p, (li + 1 < kScanTile ? tile[pad(li + 1)] : end) - p);   // element i's value is the gap
    }
  }
}

// exclusive scan of n elements into out[0..n) (out may alias the loaded array: each block
// reads its tile before writing it); part[nb] receives the total
template <typename T, typename Load, typename Visit = NoVisit>
hipError_t device_scan(Load ld, int64_t n, T* out, T* part, hipStream_t s, Visit vis = Visit()) {
  int64_t nb = div_up(n, kScanTile);
  if (nb == 0) {
    hipLaunchKernelGGL((k_fill<T>), dim3(1), dim3(64), 0, s, part, (int64_t)1, (T)0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_scan_reduce<T, Load>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, ld, n, part);
  const bool fused = nb <= kScanFusedBlocks;
  if (!fused) hipLaunchKernelGGL((k_scan_partials<T>), dim3(1), dim3(256), 0, s, part, nb);
  hipLaunchKernelGGL((k_scan_down<T, Load, Visit>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, ld, n, part, nb,
                     fused, out, vis);
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

// Per-block digit counts of one 4096-key tile, counted with LDS atomics into one histogram per
// wavefront (order does not matter for counting), written digit-major: hist[d * nb + block].
template <typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const K* __restrict__ keys, const int64_t* n_ptr, int64_t n_cap,
                                                    int shift, int bits, uint32_t* __restrict__ hist, int64_t nb) {
  __shared__ uint32_t cnt[4][kRadixBins];
  const int tid = threadIdx.x, wid = tid >> 6;
  cnt[0][tid] = cnt[1][tid] = cnt[2][tid] = cnt[3][tid] = 0;
  __syncthreads();
  const int64_t n = sort_count(n_ptr, n_cap);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const uint32_t mask = (1u << bits) - 1u;
  if (base < n) {
    uint32_t d[kScanItems];
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
      const int64_t i = base + (int64_t)r * kScanThreads + tid;
      const uint32_t x = (uint32_t)(keys[i < n ? i : n - 1] >> shift) & mask;   // unconditional load
      d[r] = i < n ? x : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int r = 0; r < kScanItems; ++r)
      if (d[r] != 0xFFFFFFFFu) atomicAdd(&cnt[wid][d[r]], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nb + blockIdx.x] = cnt[0][tid] + cnt[1][tid] + cnt[2][tid] + cnt[3][tid];
}

// Stable scatter of one block tile (4096 keys).  Wavefront w owns the contiguous quarter
// [1024 w, 1024 w + 1024) of the tile and walks it in 16 rounds of 64 keys: ballot matching of
// the digit gives each key its rank among the round's equal digits, and a wave-private running
// count per digit (LDS, touched only by that wavefront) carries the rank across rounds.  One
// block scan then turns (digit, wavefront) counts into offsets, keys are staged in LDS in digit
// order and written out so that consecutive lanes write consecutive addresses of a digit's
// output run (coalesced), at the block's global digit offsets from the scanned histogram.
template <typename K>
__global__ __launch_bounds__(256) void k_radix_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                       K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       const int64_t* n_ptr, int64_t n_cap, int shift, int bits,
                                                       const uint32_t* __restrict__ hist, int64_t nb) {
  constexpr int kPerWave = kScanTile / 4;
  __shared__ K s_k[kScanTile];
  __shared__ uint32_t s_v[kScanTile];
  __shared__ uint32_t gbase[kRadixBins];
  __shared__ uint32_t lcum[kRadixBins];
  __shared__ uint32_t wc[4][kRadixBins];   // per-wavefront running counts, then offsets
  __shared__ uint32_t tmp[4];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  const int64_t n = sort_count(n_ptr, n_cap);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n) return;   // uniform over the block
  const int cnt = (int)((n - base) < kScanTile ? (n - base) : kScanTile);
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t lt = lanemask_lt();
  gbase[tid] = hist[(int64_t)tid * nb + blockIdx.x];
  wc[0][tid] = wc[1][tid] = wc[2][tid] = wc[3][tid] = 0u;
  K key[kScanItems];
  uint32_t val[kScanItems], rank[kScanItems];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int li = wid * kPerWave + r * 64 + lane;
    const int lc = li < cnt ? li : cnt - 1;   // unconditional loads; lanes past cnt are invalid below
    key[r] = kin[base + lc];
    val[r] = vin[base + lc];
  }
  __syncthreads();
  uint32_t* run = wc[wid];
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
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
  for (int r = 0; r < kScanItems; ++r) {
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
// non-null.  n_ptr (device) gives the element count when non-null, capped by n_cap.
// `first_hist_ready`: the caller already wrote the first pass's digit counts into `hist`.
template <typename K>
static hipError_t radix_sort(K* k[2], uint32_t* v[2], int& cur, const int64_t* n_ptr, int64_t n_cap, int lo_bit,
                             int total_bits, uint32_t* hist, uint32_t* hist_part, uint32_t* final_vals, hipStream_t s,
                             bool first_hist_ready = false) {
  if (total_bits < 1) total_bits = 1;
  const int passes = (total_bits + kRadixBits - 1) / kRadixBits;
  const int per = radix_pass_bits(total_bits);   // bits spread evenly over the passes
  const int64_t nb = div_up(n_cap, kScanTile);
  if (nb == 0) return hipSuccess;
  for (int p = 0; p < passes; ++p) {
    const int shift = lo_bit + p * per;
    const int bits = (total_bits - p * per) < per ? (total_bits - p * per) : per;
    if (!(p == 0 && first_hist_ready))
      hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)nb), dim3(256), 0, s, (const K*)k[cur], n_ptr, n_cap, shift,
                         bits, hist, nb);
    hipError_t e = device_scan<uint32_t>(LoadU32{hist}, (int64_t)kRadixBins * nb, hist, hist_part, s);
    if (e != hipSuccess) return e;
    uint32_t* vdst = (p == passes - 1 && final_vals) ? final_vals : v[1 - cur];
    hipLaunchKernelGGL(k_radix_scatter<K>, dim3((unsigned)nb), dim3(256), 0, s, (const K*)k[cur],
                       (const uint32_t*)v[cur], k[1 - cur], vdst, n_ptr, n_cap, shift, bits, (const uint32_t*)hist, nb);
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

// compaction of the visible records with their float64 depth keys (upper 48 bits)
struct LoadVisible {
  const int32_t* n_tiles;
  __device__ int64_t operator()(int64_t i) const { return n_tiles[i] > 0 ? 1 : 0; }
};

// 40-bit sort key of a positive float64 depth: 5 bits of binary exponent over [2^-16, 2^16)
// and the top 35 mantissa bits (2^-35 relative resolution), monotone in the depth; depths
// outside that range clamp to the first / last key (ties then keep Gaussian-id order).
constexpr int kDepthKeyBits = 40;

__device__ __forceinline__ uint64_t depth_sort_key(unsigned long long bits) {
  const int e = (int)((bits >> 52) & 0x7FF) - (1023 - 16);
  if (e < 0) return 0ull;
  if (e > 31) return (1ull << kDepthKeyBits) - 1ull;
  return ((uint64_t)e << 35) | ((bits & 0xFFFFFFFFFFFFFull) >> 17);
}

// The record's tile count rides in the key's top 24 bits (the sort looks only at the low
// kDepthKeyBits), so that the scan of the counts in depth order reads the sorted keys
// contiguously instead of gathering by record.  A sensor has fewer than 2^24 tiles.
__global__ void k_compact_visible(const int32_t* __restrict__ n_tiles, const unsigned long long* __restrict__ dkey,
                                  const int64_t* __restrict__ pos, int64_t n_rec, uint64_t* __restrict__ keys,
                                  uint32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rec) return;
  const int32_t nt = n_tiles[i];
  if (nt <= 0) return;
  int64_t p = pos[i];
  keys[p] = ((uint64_t)nt << kDepthKeyBits) | depth_sort_key(dkey[i]);
  vals[p] = (uint32_t)i;
}

// tile count of the i-th visible record in depth order, from its sorted packed key (entries
// past the visible count hold stale keys and count zero)
struct LoadPackedTiles {
  const uint64_t* keys;
  const int64_t* n_vis;
  __device__ int64_t operator()(int64_t i) const {
    const uint64_t k = keys[i];
    return i < *n_vis ? (int64_t)(k >> kDepthKeyBits) : 0;
  }
};

__global__ void k_finalize_count(const int64_t* __restrict__ total, int64_t k_cap, int64_t* __restrict__ n_sort,
                                 SplatStatus* st) {
  int64_t K = *total;
  *n_sort = K < k_cap ? K : k_cap;
  if (st) {
    st->n_isect = (unsigned long long)K;
    st->k_cap = (unsigned long long)k_cap;
    if (K > k_cap) st->overflow = 1u;
  }
}

constexpr int kEmitTile = kScanTile;   // output slots per workgroup of the emit kernel = one radix tile
constexpr int kEmitThreads = 512;
constexpr int kEmitPer = kEmitTile / kEmitThreads;   // consecutive slots per thread
constexpr int kEmitRecs = kEmitTile + 1;             // records that can meet one workgroup's slots
static_assert(kEmitPer == 8, "k_emit stores a thread's slots as two 16-byte vectors");

// q = floor(a / b) for 0 <= a < 2^24, b >= 1, from a float reciprocal with an exact correction.
__device__ __forceinline__ int div_small(int a, int b) {
  int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
  q -= (q * b > a) ? 1 : 0;
  q += ((q + 1) * b <= a) ? 1 : 0;
  return q;
}

// Thread t emits the kEmitPer consecutive slots k0 + t kEmitPer + j.  Slot k belongs to the
// visible record r (depth order) with offs[r] <= k < offs[r + 1]; the records that can own a
// slot of the workgroup are bstart[b] .. bstart[b + 1] (at most kEmitRecs).  They are staged
// first, all in parallel: every record's first slot relative to k0 and a descriptor
//   {Gaussian id, key of the rectangle's first tile, width | wrap column << 16, row stride},
// where the key of entry (row, col) of the rectangle is first + row * stride + col, minus the
// stride once col reaches the wrap column (lidar azimuth wrap; cameras never wrap).  A thread
// then finds its first slot's record by binary search and walks its slots through LDS only
// (every visible record has >= 1 slot, so the walk advances at most one record per slot).
// Keys and ids are stored straight from registers (each thread's slots are contiguous).  A
// workgroup's slots are exactly one tile of the radix sort that follows, so it also writes that
// tile's counts of the first pass's digit (key & digit_mask: hist[d * nb + block], zero
// for blocks past the last slot).
__global__ __launch_bounds__(kEmitThreads) void k_emit(const DevSensor* __restrict__ sens, int count, int64_t N,
                                                       const int4* __restrict__ rect,
                                                       const uint32_t* __restrict__ order,
                                                       const int64_t* __restrict__ offs,
                                                       const int64_t* __restrict__ n_vis,
                                                       const int64_t* __restrict__ n_slots,
                                                       const int64_t* __restrict__ bstart, uint32_t* __restrict__ keys,
                                                       uint32_t* __restrict__ vals, uint32_t* __restrict__ hist,
                                                       int64_t nb, uint32_t digit_mask) {
  __shared__ uint4 s_desc[kEmitRecs];
  __shared__ int16_t s_off[kEmitRecs + 1];   // first slot - k0, clamped to [0, kEmitTile + 1]
  __shared__ uint32_t s_cnt[kRadixBins];
  __shared__ int s_off0;                     // first slot - k0 of record 0 (<= 0), unclamped
  const int tid = threadIdx.x;
  const int64_t K = *n_slots;
  const int64_t k0 = (int64_t)blockIdx.x * kEmitTile;
  if (tid < kRadixBins) s_cnt[tid] = 0;
  if (k0 >= K) {   // uniform
    if (tid < kRadixBins) hist[(int64_t)tid * nb + blockIdx.x] = 0;
    return;
  }
  const int64_t r0 = bstart[blockIdx.x];
  const int64_t used = (K + kEmitTile - 1) / kEmitTile;   // workgroups with slots; bstart is set for each
  const int64_t r_last = blockIdx.x + 1 < used ? bstart[blockIdx.x + 1] : *n_vis - 1;
  const int nrec = (int)(r_last - r0 + 1 < kEmitRecs ? r_last - r0 + 1 : kEmitRecs);
  // stage the records, three rounds per iteration with clamped (always valid) indices so that
  // their loads are issued together
  constexpr int kU = 3;
  for (int i0 = 0; i0 < nrec; i0 += kU * kEmitThreads) {
    int64_t rel[kU];
    uint32_t rec[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kEmitThreads + tid;
      const int64_t r = r0 + (i < nrec ? i : nrec - 1);
      rel[u] = offs[r] - k0;
      rec[u] = order[r];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * kEmitThreads + tid;
      int s = 0;
      if (count > 1) {
        s = (int)((float)rec[u] * __builtin_amdgcn_rcpf((float)N));
        s -= ((int64_t)s * N > (int64_t)rec[u]) ? 1 : 0;
        s += ((int64_t)(s + 1) * N <= (int64_t)rec[u]) ? 1 : 0;
      }
      const DevSensor& S = sens[s];
      const int4 rc = rect[rec[u]];
      const bool cam = S.kind == kCamera;
      const uint32_t stride = (uint32_t)(cam ? S.tiles_x : S.m_az);
      const uint32_t first = (uint32_t)(S.tile_base - sens[0].tile_base) + (uint32_t)rc.y * stride + (uint32_t)rc.x;
      const uint32_t wrap = (uint32_t)(cam ? rc.z : S.m_az - rc.x);
      if (i < nrec) {
        s_desc[i] = make_uint4(rec[u] - (uint32_t)s * (uint32_t)N, first, (uint32_t)rc.z | (wrap << 16), stride);
        const int64_t v = rel[u] < 0 ? 0 : (rel[u] > kEmitTile + 1 ? kEmitTile + 1 : rel[u]);
        s_off[i] = (int16_t)v;
        if (i == 0) s_off0 = (int)rel[u];
      }
    }
  }
  if (tid == 0) s_off[nrec] = (int16_t)(kEmitTile + 1);
  __syncthreads();
  const int nk = (int)((K - k0) < kEmitTile ? (K - k0) : kEmitTile);
  const int j0 = tid * kEmitPer;
  uint32_t kk[kEmitPer], gg[kEmitPer];
  if (j0 < nk) {
    int lo = 0, hi = nrec - 1;   // last record with s_off[lo] <= j0 (s_off[0] = 0)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= j0) lo = mid; else hi = mid - 1;
    }
    uint4 d = s_desc[lo];
    int nxt = s_off[lo + 1];
    int w = (int)(d.z & 0xFFFFu), wrap = (int)(d.z >> 16);
    const int jj = j0 - (lo == 0 ? s_off0 : (int)s_off[lo]);
    int row = div_small(jj, w), col = jj - row * w;
#pragma unroll
    for (int j = 0; j < kEmitPer; ++j) {
      const int q = j0 + j;
      if (q < nk && q >= nxt) {   // the next record starts here (it is staged: its first slot < nk)
        ++lo;
        d = s_desc[lo];
        nxt = s_off[lo + 1];
        w = (int)(d.z & 0xFFFFu);
        wrap = (int)(d.z >> 16);
        row = 0;
        col = 0;
      }
      const uint32_t key = d.y + (uint32_t)row * d.w + (uint32_t)col - (col >= wrap ? d.w : 0u);
      kk[j] = key;
      gg[j] = d.x;
      if (q < nk) atomicAdd(&s_cnt[key & digit_mask], 1u);
      if (++col == w) {
        col = 0;
        ++row;
      }
    }
    uint32_t* kp = keys + k0 + j0;
    uint32_t* vp = vals + k0 + j0;
    if (j0 + kEmitPer <= nk && ((((uintptr_t)kp) | ((uintptr_t)vp)) & 15) == 0) {
      reinterpret_cast<uint4*>(kp)[0] = make_uint4(kk[0], kk[1], kk[2], kk[3]);
      reinterpret_cast<uint4*>(kp)[1] = make_uint4(kk[4], kk[5], kk[6], kk[7]);
      reinterpret_cast<uint4*>(vp)[0] = make_uint4(gg[0], gg[1], gg[2], gg[3]);
      reinterpret_cast<uint4*>(vp)[1] = make_uint4(gg[4], gg[5], gg[6], gg[7]);
    } else {
#pragma unroll
      for (int j = 0; j < kEmitPer; ++j)
        if (j0 + j < nk) {
          kp[j] = kk[j];
          vp[j] = gg[j];
        }
    }
  }
  __syncthreads();
  if (tid < kRadixBins) hist[(int64_t)tid * nb + blockIdx.x] = s_cnt[tid];
}

// Visitor of the offsets scan over the visible records in depth order: record i (value = its
// tile count, exclusive prefix a) owns slots [a, a + count); writes entry_base[record] = a and
// the first record of every emit block whose first slot falls in that range.
struct EntryVisit {
  const uint32_t* order;
  const int64_t* n_vis;
  int64_t* entry_base;
  int64_t* bstart;
  int64_t n_blocks;
  __device__ void operator()(int64_t i, int64_t a, int64_t cnt) const {
    if (i >= *n_vis) return;
    entry_base[order[i]] = a;
    for (int64_t kb = (a + kEmitTile - 1) / kEmitTile; kb < n_blocks && kb * kEmitTile < a + cnt; ++kb) bstart[kb] = i;
  }
};

constexpr int kRangeItems = 8;   // sorted keys per thread of k_ranges

// [start, end) of every key's run in a sorted key array; keys that do not occur keep the range
// the caller filled in.  Thread t of a block handles elements base + j * 256 + t (coalesced).
// The run of key k is range[(k >> shift) + offset].
__global__ void k_ranges(const uint32_t* __restrict__ keys, const int64_t* n_ptr, int64_t n_cap, int2* __restrict__ range,
                         int shift, int64_t offset) {
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
    if (prev[j] != cur[j]) range[cur[j] + offset].x = (int)i;
    if (next[j] != cur[j]) range[cur[j] + offset].y = (int)(i + 1);
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
// when its lidar caps the rays per tile (training time)
__global__ void k_ray_keys(const DevSensor* __restrict__ sens, int count, int64_t r0, int64_t n, int64_t n_tiles,
                           int64_t t0, int cell_bits, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                           SplatStatus* st) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
// rays outside every tile (bin n_tiles)
__global__ void k_work_count(const DevSensor* __restrict__ sens, int count, const int2* __restrict__ range,
                             int64_t n_tiles, int64_t* __restrict__ cnt) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
  for (int p = r.x; p < r.y; p += SPLAT_RAYS_PER_ITEM, ++o)
    if (o < work_cap) work[o] = make_int2((int)t, p);
}

// Longest-processing-time order of the persistent queue: items sorted (stably) by descending
// length of their tile's Gaussian list, in buckets of about 6 %: the key is 255 minus an 8-bit
// log-scale code of the length (4 bits of exponent, 4 bits of mantissa).
__device__ __forceinline__ uint32_t length_code(int64_t len) {
  const uint32_t x = (uint32_t)(len < 0xFFFFF ? len : 0xFFFFF) + 1u;   // >= 1
  const int e = 31 - __clz(x);                                       // 0..20
  const uint32_t m = e >= 4 ? (x >> (e - 4)) & 15u : (x << (4 - e)) & 15u;
  const uint32_t c = ((uint32_t)e << 4) | m;
  return c < 255u ? c : 255u;
}

__global__ void k_queue_keys(const int2* __restrict__ work, const int32_t* __restrict__ n_work,
                             const int2* __restrict__ tile_range, int64_t n_tiles, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_work) return;
  int64_t t = work[i].x;
  int64_t len = 0;
  if (t < n_tiles) {
    int2 r = tile_range[t];
    len = r.y - r.x;
  }
  keys[i] = 255u - length_code(len);
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
  int64_t max_n = nrec > kc ? nrec : kc;
  max_n = max_n > nr ? max_n : nr;
  int64_t max_blocks = div_up(max_n, kScanTile);
  for (int i = 0; i < 2; ++i) w.dkeys[i] = (uint64_t*)take(nrec * 8);
  for (int i = 0; i < 2; ++i) w.dvals[i] = (uint32_t*)take(nrec * 4);
  w.offs = (int64_t*)take((nrec + 1) * 8);
  w.scan_part = (int64_t*)take((div_up(nrec > n_tiles + 2 ? nrec : n_tiles + 2, kScanTile) + 2) * 8);
  for (int i = 0; i < 2; ++i) w.tkeys[i] = (uint32_t*)take(kc * 4);
  w.tvals = (uint32_t*)take(kc * 4);
  w.hist = (uint32_t*)take((size_t)kRadixBins * max_blocks * 4 + 64);
  w.hist_part = (uint32_t*)take((div_up((int64_t)kRadixBins * max_blocks, kScanTile) + 2) * 4);
  for (int i = 0; i < 2; ++i) w.rkeys[i] = (uint32_t*)take(nr * 4);
  for (int i = 0; i < 2; ++i) w.rvals[i] = (uint32_t*)take(nr * 4);
  const int64_t wcap = work_capacity(n_tiles, nr) + 1;
  for (int i = 0; i < 2; ++i) w.qkeys[i] = (uint32_t*)take(wcap * 4);
  for (int i = 0; i < 2; ++i) w.qvals[i] = (uint32_t*)take(wcap * 4);
  w.qtmp = (int2*)take(wcap * 8);
  w.wcount = (int64_t*)take((n_tiles + 2) * 8);
  w.wpart = (int64_t*)take((div_up(n_tiles + 2, kScanTile) + 2) * 8);
  w.scalars = (int64_t*)take(4 * 8);
  w.bstart = (int64_t*)take((size_t)(div_up(kc, kEmitTile) + 1) * 8);
  const size_t sort_bytes = off;
  // adjoint buffers start over at the base
  off = 0;
  w.stride = slot_stride(cmax_bucket(c_max));
  w.slots = (float*)take((size_t)kc * w.stride * 4);
  w.flags = (uint8_t*)take((size_t)div_up(kc, 4) * 4);
  w.g2d = (float*)take((size_t)nrec * kNV * 4);
  w.rflag = (uint8_t*)take((size_t)div_up(nrec, 4) * 4);
  w.long_cap = long_part_cap(nrec, kc);
  w.long_list = (uint32_t*)take((size_t)kLongParts * w.long_cap * 8);
  w.n_long = (int32_t*)take(kLongParts * 4);
  w.bytes = off > sort_bytes ? off : sort_bytes;
  return w;
}

hipError_t launch_bin_sort(const CallView& v, const SplatProjected& p, const SplatTileLists& L, const Workspace& w,
                           SplatStatus* st, hipStream_t s) {
  const int64_t n_rec = (int64_t)v.count * v.n_gauss;
  hipError_t e;
  int64_t* n_sort = w.scalars;   // min(K, k_cap)
  // 1. visible records, compacted in record order, then stably sorted by the 40-bit depth key
  int64_t* n_vis = n_sort + 1;
  if ((e = device_scan<int64_t>(LoadVisible{p.n_tiles}, n_rec, w.offs, w.scan_part, s)) != hipSuccess) return e;
  const int64_t nb0 = div_up(n_rec, kScanTile);
  hipLaunchKernelGGL(k_copy_i64, dim3(1), dim3(1), 0, s, (const int64_t*)(w.scan_part + nb0), n_vis);
  if (n_rec > 0)
    hipLaunchKernelGGL(k_compact_visible, dim3((unsigned)div_up(n_rec, 256)), dim3(256), 0, s, (const int32_t*)p.n_tiles,
                       (const unsigned long long*)p.dkey, (const int64_t*)w.offs, n_rec, w.dkeys[0], w.dvals[0]);
  uint64_t* dk[2] = {w.dkeys[0], w.dkeys[1]};
  uint32_t* dvv[2] = {w.dvals[0], w.dvals[1]};
  int cur = 0;
  if ((e = radix_sort<uint64_t>(dk, dvv, cur, n_vis, n_rec, 0, kDepthKeyBits, w.hist, w.hist_part,
                                nullptr, s)) != hipSuccess)
    return e;
  const uint32_t* order = dvv[cur];
  // 2. slot ranges
  const int64_t emit_blocks = div_up(L.k_cap, kEmitTile);
  if ((e = device_scan<int64_t>(LoadPackedTiles{dk[cur], n_vis}, n_rec, w.offs, w.scan_part, s,
                                EntryVisit{order, n_vis, L.entry_base, w.bstart, emit_blocks})) != hipSuccess)
    return e;
  int64_t nb = div_up(n_rec, kScanTile);
  hipLaunchKernelGGL(k_finalize_count, dim3(1), dim3(1), 0, s, (const int64_t*)(w.scan_part + nb), L.k_cap, n_sort, st);
  // 3. emit: the final tile-sort pass must land its values in lists->gauss
  const int tbits = bits_for(v.n_tiles);
  const int passes = (tbits + kRadixBits - 1) / kRadixBits;
  uint32_t* tv[2];
  if (passes % 2 == 0) { tv[0] = (uint32_t*)L.gauss; tv[1] = w.tvals; }
  else { tv[0] = w.tvals; tv[1] = (uint32_t*)L.gauss; }
  if (n_rec > 0 && L.k_cap > 0)
    hipLaunchKernelGGL(k_emit, dim3((unsigned)emit_blocks), dim3(kEmitThreads), 0, s, v.sens, v.count, v.n_gauss,
                       (const int4*)p.rect, order, (const int64_t*)w.offs, (const int64_t*)n_vis,
                       (const int64_t*)n_sort, (const int64_t*)w.bstart, w.tkeys[0], tv[0], w.hist,
                       div_up(L.k_cap, kScanTile), (1u << radix_pass_bits(tbits)) - 1u);
  // 4. stable sort by tile
  uint32_t* tk[2] = {w.tkeys[0], w.tkeys[1]};
  int tcur = 0;
  if ((e = radix_sort<uint32_t>(tk, tv, tcur, n_sort, L.k_cap, 0, tbits, w.hist, w.hist_part, nullptr, s,
                                n_rec > 0 && L.k_cap > 0)) != hipSuccess)
    return e;
  // 5. ranges
  if ((e = fill<int32_t>(L.tile_range, 2 * v.n_tiles, 0, s)) != hipSuccess) return e;
  if (L.k_cap > 0)
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)div_up(L.k_cap, 256 * kRangeItems)), dim3(256), 0, s, (const uint32_t*)tk[tcur],
                       (const int64_t*)n_sort, L.k_cap, (int2*)L.tile_range, 0, (int64_t)0);
  // 6. lidar rays -> tiles; work items (lidar chunks, and camera tiles in the batched form)
  if (v.has_lidar || v.queue) {
    const int64_t bins = v.n_tiles + 1;
    const int64_t r0 = v.lidar_ray0;
    const int64_t nr = v.n_rays - r0;
    if ((e = fill<int32_t>(L.ray_range, 2 * bins, 0, s)) != hipSuccess) return e;
    if (nr > 0) {
      // rays grouped by tile, and inside a tile in Z-order of their cells (compact work items);
      // the cell code fills the unused bits of the bin's last radix digit, so it adds no pass
      // (under the training-time cap 16 bits of priority take its place, and add passes)
      const int64_t t0 = v.lidar_tile0;
      const int bin_bits = bits_for(bins - t0);
      const int cell_bits = v.ray_cap ? 16 : ray_cell_bits(bin_bits);   // make_view keeps bin_bits <= 16
      hipLaunchKernelGGL(k_ray_keys, dim3((unsigned)div_up(nr, 256)), dim3(256), 0, s, v.sens, v.count, r0, nr,
                         v.n_tiles, t0, cell_bits, w.rkeys[0], w.rvals[0], st);
      uint32_t* rk[2] = {w.rkeys[0], w.rkeys[1]};
      uint32_t* rv[2] = {w.rvals[0], w.rvals[1]};
      int rcur = 0;
      if ((e = radix_sort<uint32_t>(rk, rv, rcur, nullptr, nr, 0, bin_bits + cell_bits, w.hist, w.hist_part,
                                    (uint32_t*)L.ray_order, s)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(k_ranges, dim3((unsigned)div_up(nr, 256 * kRangeItems)), dim3(256), 0, s, (const uint32_t*)rk[rcur],
                         (const int64_t*)nullptr, nr, (int2*)L.ray_range, cell_bits, t0);
    }
    hipLaunchKernelGGL(k_work_count, dim3((unsigned)div_up(bins, 256)), dim3(256), 0, s, v.sens, v.count,
                       (const int2*)L.ray_range, v.n_tiles, w.wcount);
    if ((e = device_scan<int64_t>(LoadI64{w.wcount}, bins, w.wcount, w.wpart, s)) != hipSuccess) return e;
    // the total lands in wpart[nb]; copy it behind the per-bin offsets for k_work_emit
    const int64_t wnb = div_up(bins, kScanTile);
    hipLaunchKernelGGL(k_copy_i64, dim3(1), dim3(1), 0, s, (const int64_t*)(w.wpart + wnb), w.wcount + bins);
    int2* wdst = v.queue ? w.qtmp : (int2*)L.work;
    hipLaunchKernelGGL(k_work_emit, dim3((unsigned)div_up(bins, 256)), dim3(256), 0, s, v.sens, v.count,
                       (const int2*)L.ray_range, v.n_tiles, (const int64_t*)w.wcount, L.work_cap, wdst, L.n_work);
    if (v.queue) {
      const int64_t wcap = L.work_cap;
      hipLaunchKernelGGL(k_queue_keys, dim3((unsigned)div_up(wcap, 256)), dim3(256), 0, s, (const int2*)w.qtmp,
                         (const int32_t*)L.n_work, (const int2*)L.tile_range, v.n_tiles, w.qkeys[0], w.qvals[0]);
      uint32_t* qk[2] = {w.qkeys[0], w.qkeys[1]};
      uint32_t* qv[2] = {w.qvals[0], w.qvals[1]};
      int qcur = 0;
      // item count: the scan total (clamped to the capacity by the sort)
      if ((e = radix_sort<uint32_t>(qk, qv, qcur, w.wcount + bins, wcap, 0, 8, w.hist, w.hist_part, nullptr, s)) !=
          hipSuccess)
        return e;
      hipLaunchKernelGGL(k_queue_gather, dim3((unsigned)div_up(wcap, 256)), dim3(256), 0, s, (const int2*)w.qtmp,
                         (const uint32_t*)qv[qcur], (const int32_t*)L.n_work, (int2*)L.work);
    }
  }
  return hipGetLastError();
}

hipError_t launch_exclusive_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* part, hipStream_t s) {
  return device_scan<int64_t>(LoadI64{in}, n, out, part, s);
}

}  // namespace splat
