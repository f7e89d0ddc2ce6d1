// mcmc.hip -- the MCMC regulariser of the training-details appendix (SplatAD, arXiv 2411.16816;
// the opacity and scale regularisation of the MCMC densification strategy the paper adopts):
//   L = lambda_o sum_i |o_i| + lambda_S sum_i sum_j |sqrt(eig_j(Sigma_i))|.
// With Sigma = R diag(exp(2 l)) R^T (Sec. 3.1) the eigenvalues are exp(2 l_j) for any rotation,
// so the scale term is lambda_S sum exp(l_j): no rotation enters, and dL/dl_j = lambda_S exp(l_j),
// dL/do = lambda_o sign(o).
//
// HBM-bound: per Gaussian it reads o and l (16 B) and read-modify-writes their gradients
// (32 B).  A grid-stride loop over groups of four Gaussians (16-byte accesses); L is summed per
// wavefront, then per workgroup through LDS, and added to the caller's scalar with one atomic per
// workgroup.
#include <cmath>

#include "kernels.hpp"
#include "wave_ops.hpp"

namespace splat {

__device__ __forceinline__ float sgnf(float o) { return o > 0.f ? 1.f : (o < 0.f ? -1.f : 0.f); }

// Four Gaussians per thread with 16-byte accesses when every array is 16-byte aligned (their
// log-scale rows then span three float4), one per thread otherwise and for the tail.
__global__ __launch_bounds__(256) void k_mcmc_reg(int64_t n, const float* __restrict__ opac,
                                                  const float* __restrict__ log_scales, float lam_o, float lam_s,
                                                  float* __restrict__ value, float* __restrict__ d_opac,
                                                  float* __restrict__ d_ls, int vec) {
  __shared__ float s_part[4];
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n4 = vec ? n / 4 : 0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride) {
    const float4 o = reinterpret_cast<const float4*>(opac)[q];
    const float4* lp = reinterpret_cast<const float4*>(log_scales) + 3 * q;
    const float4 l0 = lp[0], l1 = lp[1], l2 = lp[2];
    const float e[12] = {expf(l0.x), expf(l0.y), expf(l0.z), expf(l0.w), expf(l1.x), expf(l1.y),
                         expf(l1.z), expf(l1.w), expf(l2.x), expf(l2.y), expf(l2.z), expf(l2.w)};
    float se = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) se += e[k];
    acc += lam_o * (fabsf(o.x) + fabsf(o.y) + fabsf(o.z) + fabsf(o.w)) + lam_s * se;
    if (d_opac) {
      float4 g = reinterpret_cast<float4*>(d_opac)[q];
      g.x += lam_o * sgnf(o.x);
      g.y += lam_o * sgnf(o.y);
      g.z += lam_o * sgnf(o.z);
      g.w += lam_o * sgnf(o.w);
      reinterpret_cast<float4*>(d_opac)[q] = g;
    }
    if (d_ls) {
      float4* gp = reinterpret_cast<float4*>(d_ls) + 3 * q;
      float4 g0 = gp[0], g1 = gp[1], g2 = gp[2];
      g0.x += lam_s * e[0]; g0.y += lam_s * e[1]; g0.z += lam_s * e[2]; g0.w += lam_s * e[3];
      g1.x += lam_s * e[4]; g1.y += lam_s * e[5]; g1.z += lam_s * e[6]; g1.w += lam_s * e[7];
      g2.x += lam_s * e[8]; g2.y += lam_s * e[9]; g2.z += lam_s * e[10]; g2.w += lam_s * e[11];
      gp[0] = g0;
      gp[1] = g1;
      gp[2] = g2;
    }
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float o = opac[i];
    const float s0 = expf(log_scales[3 * i]), s1 = expf(log_scales[3 * i + 1]), s2 = expf(log_scales[3 * i + 2]);
    acc += lam_o * fabsf(o) + lam_s * (s0 + s1 + s2);
    if (d_opac) d_opac[i] += lam_o * sgnf(o);
    if (d_ls) {
      d_ls[3 * i] += lam_s * s0;
      d_ls[3 * i + 1] += lam_s * s1;
      d_ls[3 * i + 2] += lam_s * s2;
    }
  }
  if (!value) return;   // uniform
  float v[1] = {acc};
  acc = wave_reduce_scatter<1>(v);   // one value: every lane ends with the wavefront's sum
  if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(value, s_part[0] + s_part[1] + s_part[2] + s_part[3]);
}

}  // namespace splat

using namespace splat;

extern "C" {

int splat_mcmc_regularizer(const SplatGaussians* g, float lambda_o, float lambda_s, float* value,
                           const SplatGrads* grads, void* stream) {
  if (!g || g->n < 0 || !std::isfinite(lambda_o) || !std::isfinite(lambda_s)) return SPLAT_ERR_INVALID_ARG;
  if (g->n == 0) return SPLAT_OK;
  if (!g->opacities || !g->log_scales) return SPLAT_ERR_INVALID_ARG;
  float* d_o = grads ? grads->opacities : nullptr;
  float* d_l = grads ? grads->log_scales : nullptr;
  if (!value && !d_o && !d_l) return SPLAT_OK;
  const uintptr_t al = (uintptr_t)g->opacities | (uintptr_t)g->log_scales | (uintptr_t)d_o | (uintptr_t)d_l;
  const int vec = (al & 15) == 0;
  // few workgroups, each striding over many Gaussians: every workgroup adds its part of L with
  // one atomic on the same address, and those atomics serialise
  int64_t blocks = div_up(vec ? div_up(g->n, 4) : g->n, 256);
  if (blocks > 512) blocks = 512;
  hipLaunchKernelGGL(k_mcmc_reg, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, g->n, g->opacities,
                     g->log_scales, lambda_o, lambda_s, value, d_o, d_l, vec);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Relocation of dead Gaussians (the MCMC densification strategy the paper adopts): a Gaussian
// with opacity <= the dead threshold takes the place of an alive one drawn with probability
// proportional to opacity; a target shared by N Gaussians gets o' = 1 - (1 - o)^(1/N) and its
// scales times o / sum_{k=1..N} C(N, k) (-1)^(k+1) o'^k / sqrt(k) (the N copies' composited
// profile integrates to the original's).  The draw is exact integer arithmetic: weights
// floor(o * 2^24) (alive only), their exclusive scan, r = floor(u * total / 2^32) from the
// caller's 32-bit random u, the target the first Gaussian whose inclusive sum exceeds r.
// Passes: weights, their scan, a lookup table of the draw (for every 2^s-wide range of r the first
// Gaussian that can be its target, one entry per four Gaussians), the draw (a short binary search
// between two table entries, one atomic count per dead Gaussian), new opacity and scales of each
// target (FP64), copies.
// ---------------------------------------------------------------------------------------------
namespace splat {

constexpr float kWeightOne = 16777216.f;   // 2^24

__global__ void k_reloc_weights(const float* __restrict__ o, int64_t n, float thr, int64_t* __restrict__ w,
                                int32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float oi = o[i];
  w[i] = oi > thr ? (int64_t)fminf(floorf(oi * kWeightOne), kWeightOne) : 0;
  counts[i] = 0;
}

// the first j in [lo, hi] whose inclusive sum (excl[j + 1], or the total) exceeds r; the caller
// guarantees that it lies in that range
__device__ inline int64_t first_exceeding(const int64_t* __restrict__ excl, int64_t n, int64_t total, int64_t r,
                                          int64_t lo, int64_t hi) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t inc = mid + 1 < n ? excl[mid + 1] : total;
    if (inc > r) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// bucket width 2^s of the lookup table: the smallest s with (total - 1) >> s < n_lut
__device__ inline int lut_shift(int64_t total, int64_t n_lut) {
  int s = 0;
  while (((total - 1) >> s) >= n_lut) ++s;
  return s;
}

inline int64_t reloc_lut_entries(int64_t n) { return n > 4 ? (n + 3) / 4 : 1; }

// lut[b] = the target of r = b << s, for b <= (total - 1) >> s
__global__ void k_reloc_lut(const int64_t* __restrict__ excl, int64_t n, const int64_t* __restrict__ total_p,
                            int64_t n_lut, int32_t* __restrict__ lut) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = *total_p;
  if (total <= 0) return;
  const int s = lut_shift(total, n_lut);
  if (b > ((total - 1) >> s)) return;
  lut[b] = (int32_t)first_exceeding(excl, n, total, b << s, 0, n - 1);
}

// grid-stride over the Gaussians; targets are nondecreasing in r, so the target of r lies between
// the table entries of its bucket and of the next one (the last Gaussian for the last bucket)
__global__ __launch_bounds__(256) void k_reloc_draw(const float* __restrict__ o, int64_t n, float thr,
                                                    const uint32_t* __restrict__ u, const int64_t* __restrict__ excl,
                                                    const int64_t* __restrict__ total_p, int64_t n_lut,
                                                    const int32_t* __restrict__ lut, int32_t* __restrict__ counts,
                                                    int32_t* __restrict__ target,
                                                    unsigned long long* __restrict__ n_moved) {
  __shared__ unsigned int s_moved;
  if (threadIdx.x == 0) s_moved = 0;
  __syncthreads();
  const int64_t total = *total_p;
  const int s = total > 0 ? lut_shift(total, n_lut) : 0;
  const int64_t last_b = total > 0 ? (total - 1) >> s : 0;
  unsigned int moved = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t t = -1;
    if (!(o[i] > thr) && total > 0) {
      const uint64_t T = (uint64_t)total, ui = u[i];
      const int64_t r = (int64_t)((T >> 32) * ui + (((T & 0xffffffffull) * ui) >> 32));   // < total
      const int64_t b = r >> s;
      const int64_t lo = lut[b], hi = b < last_b ? (int64_t)lut[b + 1] : n - 1;
      t = (int32_t)first_exceeding(excl, n, total, r, lo, hi);
      atomicAdd(&counts[t], 1);
      ++moved;
    }
    target[i] = t;
  }
  if (!n_moved) return;   // uniform
  if (moved) atomicAdd(&s_moved, moved);
  __syncthreads();
  if (threadIdx.x == 0 && s_moved) atomicAdd(n_moved, (unsigned long long)s_moved);
}

__global__ void k_reloc_update(const float* __restrict__ o, const float* __restrict__ ls, int64_t n,
                               const int32_t* __restrict__ counts, int n_max, float* __restrict__ new_o,
                               float* __restrict__ new_ls) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || counts[i] == 0) return;
  int N = counts[i] + 1;
  N = N < n_max ? N : n_max;
  const double od = o[i];
  const double on = 1.0 - pow(1.0 - od, 1.0 / N);
  double denom = 0.0, c = 1.0, p = 1.0;   // c = C(N, k), p = o'^k
  for (int k = 1; k <= N; ++k) {
    c = c * (double)(N - k + 1) / (double)k;
    p *= on;
    denom += ((k & 1) ? c : -c) * p / sqrt((double)k);
  }
  const double lf = log(od / denom);
  new_o[i] = (float)on;
  for (int d = 0; d < 3; ++d) new_ls[3 * i + d] = (float)((double)ls[3 * i + d] + lf);
}

__global__ void k_reloc_apply(SplatGaussianState g, const int32_t* __restrict__ target,
                              const int32_t* __restrict__ counts, const float* __restrict__ new_o,
                              const float* __restrict__ new_ls) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  const int64_t t = target[i];
  if (t >= 0) {   // a dead Gaussian becomes a copy of its (alive, never written here) target
    for (int d = 0; d < 3; ++d) g.means[3 * i + d] = g.means[3 * t + d];
    for (int d = 0; d < 4; ++d) g.quats[4 * i + d] = g.quats[4 * t + d];
    if (g.velocities)
      for (int d = 0; d < 3; ++d) g.velocities[3 * i + d] = g.velocities[3 * t + d];
    if (g.features)
      for (int d = 0; d < g.c_total; ++d) g.features[i * g.c_total + d] = g.features[t * g.c_total + d];
    g.opacities[i] = new_o[t];
    for (int d = 0; d < 3; ++d) g.log_scales[3 * i + d] = new_ls[3 * t + d];
  } else if (counts[i] > 0) {
    g.opacities[i] = new_o[i];
    for (int d = 0; d < 3; ++d) g.log_scales[3 * i + d] = new_ls[3 * i + d];
  }
}

struct RelocWs {
  int64_t* w;
  int64_t* part;
  int32_t* counts;
  int32_t* target;
  int32_t* lut;
  float* new_o;
  float* new_ls;
  size_t bytes;
};

inline RelocWs carve_reloc(void* base, int64_t n) {
  RelocWs r;
  char* b = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {   // base == nullptr: sizes only, pointers stay null
    char* p = b ? b + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  r.w = (int64_t*)take(n * sizeof(int64_t));
  r.part = (int64_t*)take((div_up(n, kScanTile) + 1) * sizeof(int64_t));
  r.counts = (int32_t*)take(n * sizeof(int32_t));
  r.target = (int32_t*)take(n * sizeof(int32_t));
  r.lut = (int32_t*)take(reloc_lut_entries(n) * sizeof(int32_t));
  r.new_o = (float*)take(n * sizeof(float));
  r.new_ls = (float*)take(3 * n * sizeof(float));
  r.bytes = off;
  return r;
}

}  // namespace splat

extern "C" {

size_t splat_mcmc_relocate_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return carve_reloc(nullptr, n > 0 ? n : 1).bytes;
}

int splat_mcmc_relocate(const SplatGaussianState* g, const uint32_t* u, float dead_opacity, int32_t n_max,
                        int32_t* target, unsigned long long* n_relocated, void* ws, size_t ws_bytes, void* stream) {
  if (!g || g->n < 0 || n_max < 1 || !std::isfinite(dead_opacity)) return SPLAT_ERR_INVALID_ARG;
  if (g->n == 0) return SPLAT_OK;
  if (g->n >= ((int64_t)1 << 31)) return SPLAT_ERR_UNSUPPORTED;
  if (!u || !g->means || !g->log_scales || !g->quats || !g->opacities || (g->c_total > 0 && !g->features) ||
      g->c_total < 0)
    return SPLAT_ERR_INVALID_ARG;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < splat_mcmc_relocate_workspace_bytes(g->n)) return SPLAT_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  RelocWs w = carve_reloc(ws, g->n);
  int32_t* tgt = target ? target : w.target;
  const unsigned nb = (unsigned)div_up(g->n, 256);
  hipLaunchKernelGGL(k_reloc_weights, dim3(nb), dim3(256), 0, s, (const float*)g->opacities, g->n, dead_opacity, w.w,
                     w.counts);
  if (launch_exclusive_scan_i64(w.w, g->n, w.w, w.part, s) != hipSuccess) return SPLAT_ERR_DEVICE;
  const int64_t* excl = w.w;
  const int64_t* total = w.part + div_up(g->n, kScanTile);
  const int64_t n_lut = reloc_lut_entries(g->n);
  hipLaunchKernelGGL(k_reloc_lut, dim3((unsigned)div_up(n_lut, 256)), dim3(256), 0, s, excl, g->n, total, n_lut,
                     w.lut);
  // a bounded grid: one atomic per workgroup on the shared count
  const unsigned nd = nb < 2048 ? nb : 2048;
  hipLaunchKernelGGL(k_reloc_draw, dim3(nd), dim3(256), 0, s, (const float*)g->opacities, g->n, dead_opacity, u,
                     excl, total, n_lut, (const int32_t*)w.lut, w.counts, tgt, n_relocated);
  hipLaunchKernelGGL(k_reloc_update, dim3(nb), dim3(256), 0, s, (const float*)g->opacities,
                     (const float*)g->log_scales, g->n, (const int32_t*)w.counts, (int)n_max, w.new_o, w.new_ls);
  hipLaunchKernelGGL(k_reloc_apply, dim3(nb), dim3(256), 0, s, *g, (const int32_t*)tgt, (const int32_t*)w.counts,
                     (const float*)w.new_o, (const float*)w.new_ls);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

}  // extern "C"
