// decoders.hip -- the lidar decoder of the rendered features (SplatAD, arXiv 2411.16816, Sec. 3.3;
// the training-details appendix gives its size: two layers, hidden width 32).
//
// Per lidar ray, the rendered feature row F (C channels) and the ray's unit direction
// d = (cos el cos az, cos el sin az, sin el) in the sensor frame are decoded:
//   h = ReLU(W1 [F, d] + b1),  z = W2 h + b2,  intensity = sigmoid(z0),  drop = sigmoid(z1).
//
// Forward: one thread per ray, the weights staged in LDS (every lane reads the same weight: LDS
// broadcasts), about 32 (C + 5) FMAs per ray; HBM moves the feature row, the angles and the
// two outputs.  Adjoint: one thread per ray recomputes the forward, writes dL/dF (+=) and stages
// its input x, hidden pre-activation gradient, hidden output and output gradient in LDS; the
// weight gradients are contractions over rays, so each thread then sums its share of the
// (W1, b1, W2, b2) entries over the workgroup's 128 rays from LDS into registers, across the
// chunks a persistent workgroup takes.  Every workgroup stores its partial sums, and a second
// kernel adds them in workgroup order: deterministic, no atomics.
#include "kernels.hpp"
#include "reduce.hpp"

namespace splat {

constexpr int kDecHidden = 32;
constexpr int kDecBlock = 128;
constexpr int kDecMaxC = 32;

inline int dec_outputs(int C) { return kDecHidden * (C + 3) + kDecHidden + 2 * kDecHidden + 2; }

// Laid out for 16-byte LDS reads: per hidden unit j its feature-weight row (zero beyond C), its
// direction weights with its bias, and its two output weights.
template <int CM>
struct __align__(16) DecWeights {
  float4 w1f[kDecHidden][CM / 4];   // feature columns of W1
  float4 aux[kDecHidden];           // (W1 direction columns 0..2, b1)
  float2 w2p[kDecHidden];           // (W2[0][j], W2[1][j])
  float b2[2];
};

template <int CM>
__device__ void stage_weights(DecWeights<CM>& W, const SplatLidarMLP& m) {
  const int C = m.n_feat;
  float* w1f = reinterpret_cast<float*>(&W.w1f[0][0]);
  for (int i = threadIdx.x; i < kDecHidden * CM; i += blockDim.x) {
    const int j = i / CM, k = i % CM;
    w1f[i] = k < C ? m.w1[j * (C + 3) + k] : 0.f;
  }
  for (int j = threadIdx.x; j < kDecHidden; j += blockDim.x) {
    const float* r = m.w1 + j * (C + 3) + C;
    W.aux[j] = make_float4(r[0], r[1], r[2], m.b1[j]);
    W.w2p[j] = make_float2(m.w2[j], m.w2[kDecHidden + j]);
  }
  if (threadIdx.x < 2) W.b2[threadIdx.x] = m.b2[threadIdx.x];
}

__device__ __forceinline__ float sigmoid_f(float z) { return 1.f / (1.f + expf(-z)); }

template <int CM>
__device__ __forceinline__ void load_ray(const float* feat, const float* az, const float* el, int64_t r, int C,
                                         float (&F)[CM], float (&d)[3]) {
  const float* row = feat + r * C;
#pragma unroll
  for (int k = 0; k < CM; ++k) F[k] = k < C ? row[k] : 0.f;
  float sa, ca, se, ce;
  sincosf(az[r], &sa, &ca);
  sincosf(el[r], &se, &ce);
  d[0] = ce * ca;
  d[1] = ce * sa;
  d[2] = se;
}

template <int CM>
__device__ __forceinline__ float hidden_pre(const DecWeights<CM>& W, int j, const float (&F)[CM], const float (&d)[3]) {
  const float4 a = W.aux[j];
  float p = a.w;
#pragma unroll
  for (int q = 0; q < CM / 4; ++q) {
    const float4 w = W.w1f[j][q];
    p = fmaf(w.x, F[4 * q], p);
    p = fmaf(w.y, F[4 * q + 1], p);
    p = fmaf(w.z, F[4 * q + 2], p);
    p = fmaf(w.w, F[4 * q + 3], p);
  }
  p = fmaf(a.x, d[0], p);
  p = fmaf(a.y, d[1], p);
  return fmaf(a.z, d[2], p);
}

template <int CM>
__global__ __launch_bounds__(kDecBlock) void k_lidar_decode(int64_t n, const float* __restrict__ feat,
                                                            const float* __restrict__ az, const float* __restrict__ el,
                                                            SplatLidarMLP m, float* __restrict__ intensity,
                                                            float* __restrict__ drop) {
  __shared__ DecWeights<CM> W;
  stage_weights<CM>(W, m);
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    float F[CM], d[3];
    load_ray<CM>(feat, az, el, r, m.n_feat, F, d);
    float z0 = W.b2[0], z1 = W.b2[1];
#pragma unroll 4
    for (int j = 0; j < kDecHidden; ++j) {
      const float h = fmaxf(hidden_pre<CM>(W, j, F, d), 0.f);
      const float2 w2 = W.w2p[j];
      z0 = fmaf(w2.x, h, z0);
      z1 = fmaf(w2.y, h, z1);
    }
    if (intensity) intensity[r] = sigmoid_f(z0);
    if (drop) drop[r] = sigmoid_f(z1);
  }
}

// LDS rows of one chunk of rays for the weight-gradient contraction
// N-tiles of 16 columns of the x rows: [F (CM), d (3), 1] padded with zeros
template <int CM>
constexpr int dec_xtiles() { return (CM + 4 + 15) / 16; }

template <int CM>
struct DecStage {
  float x[kDecBlock][16 * dec_xtiles<CM>() + 1];   // [F (zero beyond C), d, 1, 0...]
  float dpre[kDecBlock][kDecHidden + 1];
  float h[kDecBlock][3 * 16 + 1];                   // [h (32), 1, 0...]
  float dz[kDecBlock][2];
};

typedef float decx4 __attribute__((ext_vector_type(4)));

template <int CM>
__global__ __launch_bounds__(kDecBlock) void k_lidar_decode_bwd(int64_t n, const float* __restrict__ feat,
                                                                const float* __restrict__ az,
                                                                const float* __restrict__ el, SplatLidarMLP m,
                                                                const float* __restrict__ d_int,
                                                                const float* __restrict__ d_drop,
                                                                float* __restrict__ d_feat, float* __restrict__ partial,
                                                                int n_out) {
  constexpr int NXT = dec_xtiles<CM>();
  constexpr int NTILE = 2 * NXT + 3;             // dW1|db1: 2 x NXT blocks; dW2|db2: 3 blocks
  constexpr int NPW = (NTILE + 1) / 2;           // blocks per wavefront (two wavefronts)
  __shared__ DecWeights<CM> W;
  __shared__ DecStage<CM> S;
  stage_weights<CM>(W, m);
  const int C = m.n_feat, XC = C + 3;
  const int nw1 = kDecHidden * XC, nb1 = nw1 + kDecHidden, nw2 = nb1 + 2 * kDecHidden;
  decx4 acc[NPW];
#pragma unroll
  for (int i = 0; i < NPW; ++i) acc[i] = decx4{0.f, 0.f, 0.f, 0.f};
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  // a ray's inputs; those of the next chunk are loaded while the current chunk is computed
  // (the kernel is latency-bound on these loads otherwise)
  struct RayIn {
    float F[CM];
    float az, el, di, dd;
  };
  auto fetch = [&](int64_t rr, RayIn& in) {
    if (rr >= n) return;
    const float* row = feat + rr * C;
#pragma unroll
    for (int k = 0; k < CM; ++k) in.F[k] = k < C ? row[k] : 0.f;
    in.az = az[rr];
    in.el = el[rr];
    in.di = d_int ? d_int[rr] : 0.f;
    in.dd = d_drop ? d_drop[rr] : 0.f;
  };
  const int64_t step = (int64_t)gridDim.x * kDecBlock;
  RayIn cur{};
  fetch((int64_t)blockIdx.x * kDecBlock + t, cur);
  for (int64_t base = (int64_t)blockIdx.x * kDecBlock; base < n; base += step) {
    __syncthreads();   // weights staged / the previous chunk's rows consumed
    const int64_t r = base + t;
    RayIn nxt{};   // stays zero past the last chunk
    fetch(r + step, nxt);
    float old[CM];   // the feature-gradient row this ray adds to
#pragma unroll
    for (int k = 0; k < CM; ++k) old[k] = (d_feat && r < n && k < C) ? d_feat[r * C + k] : 0.f;
    if (r < n) {
      float F[CM], d[3];
#pragma unroll
      for (int k = 0; k < CM; ++k) F[k] = cur.F[k];
      {
        float sa, ca, se, ce;
        sincosf(cur.az, &sa, &ca);
        sincosf(cur.el, &se, &ce);
        d[0] = ce * ca;
        d[1] = ce * sa;
        d[2] = se;
      }
      float z0 = W.b2[0], z1 = W.b2[1];
      // forward again; the pre-activations wait in this ray's LDS row (the lane's own row)
#pragma unroll 2
      for (int j = 0; j < kDecHidden; ++j) {
        const float p = hidden_pre<CM>(W, j, F, d);
        const float h = fmaxf(p, 0.f);
        S.dpre[t][j] = p;
        S.h[t][j] = h;
        const float2 w2 = W.w2p[j];
        z0 = fmaf(w2.x, h, z0);
        z1 = fmaf(w2.y, h, z1);
      }
      const float s0 = sigmoid_f(z0), s1 = sigmoid_f(z1);
      const float g0 = cur.di * s0 * (1.f - s0);
      const float g1 = cur.dd * s1 * (1.f - s1);
      S.dz[t][0] = g0;
      S.dz[t][1] = g1;
#pragma unroll
      for (int k = 0; k < CM; ++k) S.x[t][k] = F[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) S.x[t][CM + k] = d[k];   // x = [F, d]: direction after the features
#pragma unroll
      for (int k = CM + 3; k < 16 * NXT; ++k) S.x[t][k] = k == CM + 3 ? 1.f : 0.f;   // ones: the bias
#pragma unroll
      for (int k = kDecHidden; k < 48; ++k) S.h[t][k] = k == kDecHidden ? 1.f : 0.f;
      float dF[CM];
#pragma unroll
      for (int k = 0; k < CM; ++k) dF[k] = 0.f;
#pragma unroll 2
      for (int j = 0; j < kDecHidden; ++j) {
        const float2 w2 = W.w2p[j];
        const float dp = S.dpre[t][j] > 0.f ? fmaf(w2.x, g0, w2.y * g1) : 0.f;
        S.dpre[t][j] = dp;
#pragma unroll
        for (int q = 0; q < CM / 4; ++q) {
          const float4 w = W.w1f[j][q];
          dF[4 * q] = fmaf(w.x, dp, dF[4 * q]);
          dF[4 * q + 1] = fmaf(w.y, dp, dF[4 * q + 1]);
          dF[4 * q + 2] = fmaf(w.z, dp, dF[4 * q + 2]);
          dF[4 * q + 3] = fmaf(w.w, dp, dF[4 * q + 3]);
        }
      }
      if (d_feat) {
        float* row = d_feat + r * C;
#pragma unroll
        for (int k = 0; k < CM; ++k)
          if (k < C) row[k] = old[k] + dF[k];
      }
    } else {
#pragma unroll
      for (int j = 0; j < kDecHidden; ++j) S.dpre[t][j] = 0.f;
#pragma unroll
      for (int j = 0; j < 48; ++j) S.h[t][j] = 0.f;
      S.dz[t][0] = S.dz[t][1] = 0.f;
#pragma unroll
      for (int k = 0; k < 16 * NXT; ++k) S.x[t][k] = 0.f;
    }
    __syncthreads();
    // Weight gradients: contractions over the chunk's rays on the matrix cores (16x16x4 FP32),
    // K = 128 rays in 32 steps (rows 4 s + lk).  Blocks 0 .. 2 NXT - 1: [dW1 | db1] =
    // dpre^T [x, 1] (M: hidden 16 jh .. +15, N: x columns 16 nt .. +15); blocks 2 NXT .. +2:
    // [dW2 | db2] = dz^T [h, 1] (M: the two outputs padded to 16, N: h columns 16 nt .. +15).
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
      const int b = wave + 2 * i;
      if (b >= NTILE) break;
#pragma unroll 4
      for (int s = 0; s < kDecBlock / 4; ++s) {
        const int q = 4 * s + lk;
        float av, bv;
        if (b < 2 * NXT) {
          const int jh = b / NXT, nt = b % NXT;
          av = S.dpre[q][16 * jh + li];
          bv = S.x[q][16 * nt + li];
        } else {
          const int nt = b - 2 * NXT;
          av = li < 2 ? S.dz[q][li] : 0.f;
          bv = S.h[q][16 * nt + li];
        }
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[i], 0, 0, 0);
      }
    }
    cur = nxt;
  }
  // D[i][j] of a block: lane j + 16 (i / 4), element i % 4
  float* dst = partial + (int64_t)blockIdx.x * n_out;
#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int b = wave + 2 * i;
    if (b >= NTILE) break;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 4 * lk + e;
      const float v = acc[i][e];
      if (b < 2 * NXT) {
        const int jh = b / NXT, nt = b % NXT;
        const int j = 16 * jh + row, col = 16 * nt + li;
        if (col < C) dst[j * XC + col] = v;                                 // feature columns of W1
        else if (col >= CM && col < CM + 3) dst[j * XC + C + (col - CM)] = v;   // direction columns
        else if (col == CM + 3) dst[nw1 + j] = v;                         // b1
      } else {
        const int nt = b - 2 * NXT;
        const int c = row, col = 16 * nt + li;
        if (c < 2) {
          if (col < kDecHidden) dst[nb1 + c * kDecHidden + col] = v;      // W2
          else if (col == kDecHidden) dst[nw2 + c] = v;                   // b2
        }
      }
    }
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

static int bwd_blocks(int64_t n) {
  int64_t b = div_up(n, kDecBlock);
  return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

static bool mlp_ok(const SplatLidarMLP* m) {
  return m && m->n_feat >= 0 && m->n_feat <= kDecMaxC && m->w1 && m->b1 && m->w2 && m->b2;
}

}  // namespace splat

using namespace splat;

#define SPLAT_DEC_DISPATCH(C, KERNEL, ...)                                                             \
  do {                                                                                                 \
    if ((C) <= 8) hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                                          \
    else if ((C) <= 16) hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);                                   \
    else hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__);                                                  \
  } while (0)

extern "C" {

int splat_lidar_decode(int64_t n_rays, const float* feat, const float* ray_az, const float* ray_el,
                       const SplatLidarMLP* mlp, float* intensity, float* drop_prob, void* stream) {
  if (n_rays < 0 || !mlp_ok(mlp)) return SPLAT_ERR_INVALID_ARG;
  if (n_rays == 0 || (!intensity && !drop_prob)) return SPLAT_OK;
  if ((mlp->n_feat > 0 && !feat) || !ray_az || !ray_el) return SPLAT_ERR_INVALID_ARG;
  int64_t blocks = div_up(n_rays, kDecBlock);
  if (blocks > 4096) blocks = 4096;
  SPLAT_DEC_DISPATCH(mlp->n_feat, k_lidar_decode, dim3((unsigned)blocks), dim3(kDecBlock), 0, (hipStream_t)stream,
                     n_rays, feat, ray_az, ray_el, *mlp, intensity, drop_prob);
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
  const int nb = bwd_blocks(n_rays), n_out = dec_outputs(mlp->n_feat);
  float* partial = (float*)ws;
  SPLAT_DEC_DISPATCH(mlp->n_feat, k_lidar_decode_bwd, dim3((unsigned)nb), dim3(kDecBlock), 0, s, n_rays, feat,
                     ray_az, ray_el, *mlp, d_intensity, d_drop_prob, d_feat, partial, n_out);
  launch_column_sums((const float*)partial, n_out, nb, n_out, MlpGradStore{*d_mlp, mlp->n_feat}, s);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

}  // extern "C"
