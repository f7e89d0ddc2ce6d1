// decoders.hip -- the lidar decoder of the rendered features (SplatAD, arXiv 2411.16816, Sec. 3.3;
// the training-details appendix gives its size: two layers, hidden width 32).
//
// Per lidar ray, the rendered feature row F (C channels) and the ray's unit direction
// d = (cos el cos az, cos el sin az, sin el) in the sensor frame are decoded:
//   h = ReLU(W1 [F, d] + b1),  z = W2 h + b2,  intensity = sigmoid(z0),  drop = sigmoid(z1).
//
// Both directions read the weights by scalar loads (every lane uses the same weight: they sit in
// SGPRs, which vector instructions take as operands).  Forward: one thread per ray, about
// 32 (C + 5) FMAs per ray; HBM moves the feature row, the angles and the two outputs.  Adjoint: one wavefront per workgroup, persistent over chunks of 64 rays (one per
// lane).  Each lane recomputes its ray's forward, writes dL/dF (+=) and sums the output layer's
// gradients (W2, b2: 66 numbers) over its rays in registers.  The first layer's gradients
// [dW1 | db1] = sum over rays of dpre^T [x, 1] are a contraction over rays: the lane stages x
// and the pre-activation gradient dpre in LDS and the wavefront contracts its 64 rows on the
// matrix cores (16x16x4 FP32), accumulating across chunks.  At the end every workgroup stores
// its partial sums (the W2 / b2 sums reduced over its lanes), and a second kernel adds them in
// workgroup order: deterministic, no atomics.
#include "kernels.hpp"
#include "reduce.hpp"
#include "wave_ops.hpp"

namespace splat {

constexpr int kDecHidden = 32;
constexpr int kDecBlock = 128;
constexpr int kDecMaxC = 32;

inline int dec_outputs(int C) { return kDecHidden * (C + 3) + kDecHidden + 2 * kDecHidden + 2; }

__device__ __forceinline__ float sigmoid_f(float z) { return 1.f / (1.f + expf(-z)); }

// vec: C == CM and the rows are 16-byte aligned (whole-row vector loads)
template <int CM>
__device__ __forceinline__ void load_ray(const float* feat, const float* az, const float* el, int64_t r, int C,
                                         bool vec, float (&F)[CM], float (&d)[3]) {
  if (vec) {
    const float4* row = reinterpret_cast<const float4*>(feat + r * CM);
#pragma unroll
    for (int q = 0; q < CM / 4; ++q) {
      const float4 v = row[q];
      F[4 * q] = v.x;
      F[4 * q + 1] = v.y;
      F[4 * q + 2] = v.z;
      F[4 * q + 3] = v.w;
    }
  } else {
    const float* row = feat + r * C;
#pragma unroll
    for (int k = 0; k < CM; ++k) F[k] = k < C ? row[k] : 0.f;
  }
  float sa, ca, se, ce;
  sincosf(az[r], &sa, &ca);
  sincosf(el[r], &se, &ce);
  d[0] = ce * ca;
  d[1] = ce * sa;
  d[2] = se;
}

// Weights are read through the constant address space: every lane reads the same weight, so
// they come in by scalar loads into SGPRs, which the vector instructions use directly (no LDS
// traffic).  EX: the feature count is exactly CM, known at compile time, so a row's loads
// merge; otherwise feature weights past C read the row's last feature weight, which multiplies a
// zero feature.
typedef const __attribute__((address_space(4))) float* ConstF;

template <int CM, bool EX>
__device__ __forceinline__ float hidden_pre_s(ConstF w1, ConstF b1, int C, int j, const float (&F)[CM],
                                              const float (&d)[3]) {
  const int Cn = EX ? CM : C, row = j * (Cn + 3), last = Cn > 0 ? Cn - 1 : 0;
  float p = b1[j];
#pragma unroll
  for (int k = 0; k < CM; ++k) p = fmaf(w1[row + (EX || k < Cn ? k : last)], F[k], p);
  p = fmaf(w1[row + Cn], d[0], p);
  p = fmaf(w1[row + Cn + 1], d[1], p);
  return fmaf(w1[row + Cn + 2], d[2], p);
}

template <int CM, bool EX>
__global__ __launch_bounds__(kDecBlock) void k_lidar_decode(int64_t n, const float* __restrict__ feat,
                                                            const float* __restrict__ az, const float* __restrict__ el,
                                                            SplatLidarMLP m, float* __restrict__ intensity,
                                                            float* __restrict__ drop, int vec) {
  const ConstF w1 = (ConstF)m.w1, b1 = (ConstF)m.b1, w2 = (ConstF)m.w2, b2 = (ConstF)m.b2;
  const int C = EX ? CM : m.n_feat;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    float F[CM], d[3];
    load_ray<CM>(feat, az, el, r, C, vec != 0, F, d);
    float z0 = b2[0], z1 = b2[1];
#pragma unroll 4
    for (int j = 0; j < kDecHidden; ++j) {
      const float h = fmaxf(hidden_pre_s<CM, EX>(w1, b1, C, j, F, d), 0.f);
      z0 = fmaf(w2[j], h, z0);
      z1 = fmaf(w2[kDecHidden + j], h, z1);
    }
    if (intensity) intensity[r] = sigmoid_f(z0);
    if (drop) drop[r] = sigmoid_f(z1);
  }
}

// N-tiles of 16 columns of the x rows: [F (CM), d (3), 1] padded with zeros
template <int CM>
constexpr int dec_xtiles() { return (CM + 4 + 15) / 16; }

constexpr int kDecChunk = 64;   // rays per chunk of the adjoint: one per lane of its wavefront

// One chunk's rows for the first-layer contraction (+1 column: conflict-free row writes)
template <int CM>
struct DecRows {
  float x[kDecChunk][16 * dec_xtiles<CM>() + 1];   // [F (zero beyond C), d, 1, 0...]
  float dpre[kDecChunk][kDecHidden + 1];            // pre-activation, then its gradient
};

typedef float decx4 __attribute__((ext_vector_type(4)));

// at least 3 wavefronts per SIMD: the output-layer sums take 66 registers per lane
template <int CM, bool EX>
__global__ __launch_bounds__(kDecChunk) __attribute__((amdgpu_waves_per_eu(3)))
void k_lidar_decode_bwd(int64_t n, const float* __restrict__ feat, const float* __restrict__ az,
                        const float* __restrict__ el, SplatLidarMLP m, const float* __restrict__ d_int,
                        const float* __restrict__ d_drop, float* __restrict__ d_feat, float* __restrict__ partial,
                        int n_out, int vec) {
  constexpr int NXT = dec_xtiles<CM>();
  constexpr int NT = 2 * NXT;   // [dW1 | db1] blocks: hidden rows 16 (b / NXT) .., x columns 16 (b % NXT) ..
  // hidden units per unrolled step: a runtime feature count keeps more addresses in registers
  constexpr int UNR = EX ? 4 : 2;
  __shared__ DecRows<CM> S;
  const ConstF w1 = (ConstF)m.w1, b1 = (ConstF)m.b1, w2 = (ConstF)m.w2, b2 = (ConstF)m.b2;
  const int C = EX ? CM : m.n_feat, XC = C + 3, last = C > 0 ? C - 1 : 0;
  const int nw1 = kDecHidden * XC, nb1 = nw1 + kDecHidden, nw2 = nb1 + 2 * kDecHidden;
  decx4 acc[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) acc[i] = decx4{0.f, 0.f, 0.f, 0.f};
  float gw2[2 * kDecHidden];   // this lane's sums of dz_c h_j over its rays: W2[c][j] at c * 32 + j
#pragma unroll
  for (int i = 0; i < 2 * kDecHidden; ++i) gw2[i] = 0.f;
  float gb0 = 0.f, gb1 = 0.f;
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int64_t step = (int64_t)gridDim.x * kDecChunk;
  for (int64_t base = (int64_t)blockIdx.x * kDecChunk; base < n; base += step) {
    __syncthreads();   // weights staged / the previous chunk's rows consumed
    // Lanes past the end work on the last ray with zero upstream gradients: they add nothing,
    // and every load of the chunk is unconditional (issued together, not one branch at a time).
    const int64_t r = base + lane;
    const bool valid = r < n;
    const int64_t rr = valid ? r : n - 1;
    float F[CM], d[3];
    if (vec) {   // uniform: C == CM, 16-byte rows
      const float4* row = reinterpret_cast<const float4*>(feat + rr * CM);
#pragma unroll
      for (int q = 0; q < CM / 4; ++q) {
        const float4 v = row[q];
        F[4 * q] = v.x;
        F[4 * q + 1] = v.y;
        F[4 * q + 2] = v.z;
        F[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < CM; ++k) F[k] = k < C ? feat[rr * C + k] : 0.f;
    }
    const float a_r = az[rr], e_r = el[rr];
    float di = d_int ? d_int[rr] : 0.f, dd = d_drop ? d_drop[rr] : 0.f;
    di = valid ? di : 0.f;
    dd = valid ? dd : 0.f;
    {
      float sa, ca, se, ce;
      sincosf(a_r, &sa, &ca);
      sincosf(e_r, &se, &ce);
      d[0] = ce * ca;
      d[1] = ce * sa;
      d[2] = se;
    }
#pragma unroll
    for (int k = 0; k < CM; ++k) S.x[lane][k] = F[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) S.x[lane][CM + k] = d[k];   // x = [F, d]: direction after the features
#pragma unroll
    for (int k = CM + 3; k < 16 * NXT; ++k) S.x[lane][k] = k == CM + 3 ? 1.f : 0.f;   // ones: the bias
    // forward again; the pre-activations wait in this lane's own LDS row
    float z0 = b2[0], z1 = b2[1];
#pragma unroll UNR
    for (int j = 0; j < kDecHidden; ++j) {
      const float p = hidden_pre_s<CM, EX>(w1, b1, C, j, F, d);
      S.dpre[lane][j] = p;
      const float h = fmaxf(p, 0.f);
      z0 = fmaf(w2[j], h, z0);
      z1 = fmaf(w2[kDecHidden + j], h, z1);
    }
    const float s0 = sigmoid_f(z0), s1 = sigmoid_f(z1);
    const float g0 = di * s0 * (1.f - s0);
    const float g1 = dd * s1 * (1.f - s1);
    gb0 += g0;
    gb1 += g1;
    // output layer: sums of dz_c h_j (a pass of its own, fully unrolled: the sums stay in
    // registers, while the first layer's loop below is only partly unrolled)
#pragma unroll
    for (int j = 0; j < kDecHidden; ++j) {
      const float h = fmaxf(S.dpre[lane][j], 0.f);
      gw2[j] = fmaf(g0, h, gw2[j]);
      gw2[kDecHidden + j] = fmaf(g1, h, gw2[kDecHidden + j]);
    }
    float dF[CM];
#pragma unroll
    for (int k = 0; k < CM; ++k) dF[k] = 0.f;
#pragma unroll UNR
    for (int j = 0; j < kDecHidden; ++j) {
      const float p = S.dpre[lane][j];
      const float t = fmaf(w2[j], g0, w2[kDecHidden + j] * g1);
      const float dp = t * (p > 0.f ? 1.f : 0.f);   // ReLU'
      S.dpre[lane][j] = dp;
      const int row = j * XC;
#pragma unroll
      for (int k = 0; k < CM; ++k) dF[k] = fmaf(w1[row + (EX || k < C ? k : last)], dp, dF[k]);
    }
    if (d_feat && valid) {
      if (vec) {
        float4* row = reinterpret_cast<float4*>(d_feat + r * CM);
#pragma unroll
        for (int q = 0; q < CM / 4; ++q) {
          float4 v = row[q];
          v.x += dF[4 * q];
          v.y += dF[4 * q + 1];
          v.z += dF[4 * q + 2];
          v.w += dF[4 * q + 3];
          row[q] = v;
        }
      } else {
        float* row = d_feat + r * C;
#pragma unroll
        for (int k = 0; k < CM; ++k)
          if (k < C) row[k] += dF[k];
      }
    }
    __syncthreads();
    // [dW1 | db1] += dpre^T [x, 1] over the chunk's 64 rays: K in 16 steps of 4 rows (4 s + lk)
    // (the blocks' accumulation chains are independent: interleaved, their latencies overlap)
#pragma unroll 4
    for (int s4 = 0; s4 < kDecChunk / 4; ++s4) {
      const int q = 4 * s4 + lk;
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const int jh = b / NXT, nt = b % NXT;
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(S.dpre[q][16 * jh + li], S.x[q][16 * nt + li], acc[b], 0, 0, 0);
      }
    }
  }
  float* dst = partial + (int64_t)blockIdx.x * n_out;
  // D[i][j] of a block: lane j + 16 (i / 4), element i % 4
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int jh = b / NXT, nt = b % NXT;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 16 * jh + 4 * lk + e, col = 16 * nt + li;
      const float v = acc[b][e];
      if (col < C) dst[j * XC + col] = v;                                     // feature columns of W1
      else if (col >= CM && col < CM + 3) dst[j * XC + C + (col - CM)] = v;   // direction columns
      else if (col == CM + 3) dst[nw1 + j] = v;                               // b1
    }
  }
  // W2: one value per lane after the wavefront's reduce-scatter; b2: two wavefront sums
  bool store;
  const int slot = scatter_slot<2 * kDecHidden>(lane, store);
  const float w2sum = wave_reduce_scatter<2 * kDecHidden>(gw2);
  if (store) dst[nb1 + slot] = w2sum;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    gb0 += __shfl_xor(gb0, o, 64);
    gb1 += __shfl_xor(gb1, o, 64);
  }
  if (lane == 0) {
    dst[nw2] = gb0;
    dst[nw2 + 1] = gb1;
  }
}

// weight gradients (+=) from the column sums of the workgroups' partials
struct MlpGradStore {
  SplatLidarMLPGrads g;
  int C;
  __device__ void operator()(int o, float s) const {
    const int nw1 = kDecHidden * (C + 3), nb1 = nw1 + kDecHidden, nw2 = nb1 + 2 * kDecHidden;
    if (o < nw1) { if (g.w1) g.w1[o] += s; }
    else if (o < nb1) { if (g.b1) g.b1[o - nw1] += s; }
    else if (o < nw2) { if (g.w2) g.w2[o - nb1] += s; }
    else if (g.b2) g.b2[o - nw2] += s;
  }
};

// Workgroups of the adjoint: at most kDecBwdMaxGrid (which sizes the partial sums), at most one
// per chunk of rays, and no more than the device holds at once (the grid is persistent).
constexpr int kDecBwdMaxGrid = 8192;

static int bwd_blocks(int64_t n) {
  int64_t b = div_up(n, kDecChunk);
  return (int)(b < kDecBwdMaxGrid ? (b < 1 ? 1 : b) : kDecBwdMaxGrid);
}

// returns the grid: the number of partial-sum rows written
template <int CM, bool EX>
static int launch_decode_bwd(int64_t n, const float* feat, const float* az, const float* el, const SplatLidarMLP& m,
                              const float* d_int, const float* d_drop, float* d_feat, float* partial, int n_out,
                              int vec, hipStream_t s) {
  int dev = 0, n_cu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
    n_cu = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lidar_decode_bwd<CM, EX>, kDecChunk, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t resident = (int64_t)n_cu * per_cu;
  const int b = bwd_blocks(n), grid = (int)(b < resident ? b : resident);
  hipLaunchKernelGGL((k_lidar_decode_bwd<CM, EX>), dim3((unsigned)grid), dim3(kDecChunk), 0, s, n, feat, az, el, m,
                     d_int, d_drop, d_feat, partial, n_out, vec);
  return grid;
}

static bool mlp_ok(const SplatLidarMLP* m) {
  return m && m->n_feat >= 0 && m->n_feat <= kDecMaxC && m->w1 && m->b1 && m->w2 && m->b2;
}

}  // namespace splat

using namespace splat;

extern "C" {

int splat_lidar_decode(int64_t n_rays, const float* feat, const float* ray_az, const float* ray_el,
                       const SplatLidarMLP* mlp, float* intensity, float* drop_prob, void* stream) {
  if (n_rays < 0 || !mlp_ok(mlp)) return SPLAT_ERR_INVALID_ARG;
  if (n_rays == 0 || (!intensity && !drop_prob)) return SPLAT_OK;
  if ((mlp->n_feat > 0 && !feat) || !ray_az || !ray_el) return SPLAT_ERR_INVALID_ARG;
  int64_t blocks = div_up(n_rays, kDecBlock);
  if (blocks > 4096) blocks = 4096;
  const int C = mlp->n_feat;
  const int vec = ((C == 8 || C == 16 || C == 32) && ((uintptr_t)feat & 15) == 0) ? 1 : 0;
  const dim3 g((unsigned)blocks), blk(kDecBlock);
  hipStream_t s = (hipStream_t)stream;
  if (C == 8) hipLaunchKernelGGL((k_lidar_decode<8, true>), g, blk, 0, s, n_rays, feat, ray_az, ray_el, *mlp, intensity, drop_prob, vec);
  else if (C == 16) hipLaunchKernelGGL((k_lidar_decode<16, true>), g, blk, 0, s, n_rays, feat, ray_az, ray_el, *mlp, intensity, drop_prob, vec);
  else if (C == 32) hipLaunchKernelGGL((k_lidar_decode<32, true>), g, blk, 0, s, n_rays, feat, ray_az, ray_el, *mlp, intensity, drop_prob, vec);
  else if (C < 8) hipLaunchKernelGGL((k_lidar_decode<8, false>), g, blk, 0, s, n_rays, feat, ray_az, ray_el, *mlp, intensity, drop_prob, vec);
  else if (C < 16) hipLaunchKernelGGL((k_lidar_decode<16, false>), g, blk, 0, s, n_rays, feat, ray_az, ray_el, *mlp, intensity, drop_prob, vec);
  else hipLaunchKernelGGL((k_lidar_decode<32, false>), g, blk, 0, s, n_rays, feat, ray_az, ray_el, *mlp, intensity, drop_prob, vec);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

size_t splat_lidar_decode_workspace_bytes(int64_t n_rays, int32_t n_feat) {
  if (n_rays < 0 || n_feat < 0 || n_feat > kDecMaxC) return 0;
  return (size_t)bwd_blocks(n_rays) * dec_outputs(n_feat) * sizeof(float);
}

int splat_lidar_decode_bwd(int64_t n_rays, const float* feat, const float* ray_az, const float* ray_el,
                           const SplatLidarMLP* mlp, const float* d_intensity, const float* d_drop_prob,
                           float* d_feat, const SplatLidarMLPGrads* d_mlp, void* ws, size_t ws_bytes, void* stream) {
  if (n_rays < 0 || !mlp_ok(mlp) || !d_mlp) return SPLAT_ERR_INVALID_ARG;
  if (n_rays == 0) return SPLAT_OK;
  if ((mlp->n_feat > 0 && !feat) || !ray_az || !ray_el) return SPLAT_ERR_INVALID_ARG;
  if (!ws || ws_bytes < splat_lidar_decode_workspace_bytes(n_rays, mlp->n_feat)) return SPLAT_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  const int C = mlp->n_feat, n_out = dec_outputs(C);
  float* partial = (float*)ws;
  // vec: the feature rows (and the gradient rows) are whole 16-byte aligned rows of the kernel's width
  const int cm = C <= 8 ? 8 : C <= 16 ? 16 : 32;
  const int vec = (C == cm && ((uintptr_t)feat & 15) == 0 && ((uintptr_t)d_feat & 15) == 0) ? 1 : 0;
  const float *di = d_intensity, *dd = d_drop_prob;
  const SplatLidarMLP& w = *mlp;
  int nb;
  if (C == 8) nb = launch_decode_bwd<8, true>(n_rays, feat, ray_az, ray_el, w, di, dd, d_feat, partial, n_out, vec, s);
  else if (C == 16) nb = launch_decode_bwd<16, true>(n_rays, feat, ray_az, ray_el, w, di, dd, d_feat, partial, n_out, vec, s);
  else if (C == 32) nb = launch_decode_bwd<32, true>(n_rays, feat, ray_az, ray_el, w, di, dd, d_feat, partial, n_out, vec, s);
  else if (C < 8) nb = launch_decode_bwd<8, false>(n_rays, feat, ray_az, ray_el, w, di, dd, d_feat, partial, n_out, vec, s);
  else if (C < 16) nb = launch_decode_bwd<16, false>(n_rays, feat, ray_az, ray_el, w, di, dd, d_feat, partial, n_out, vec, s);
  else nb = launch_decode_bwd<32, false>(n_rays, feat, ray_az, ray_el, w, di, dd, d_feat, partial, n_out, vec, s);
  launch_column_sums((const float*)partial, n_out, nb, n_out, MlpGradStore{*d_mlp, mlp->n_feat}, s);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

}  // extern "C"
