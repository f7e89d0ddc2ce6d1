// cnn.hip -- the camera decoder of the rendered features (SplatAD, arXiv 2411.16816, Sec. 3.2: a
// small CNN maps the feature image, the ray directions and a camera embedding to a per-pixel
// affine map of the rendered colour; the training-details appendix: two residual blocks of
// width 32, kernel size 3, then a final linear layer).
//
//   x  = [F, d, e]                       (D_f + 3 + E <= 32 channels, zero-padded to 32)
//   h0 = ReLU(conv_in(x)),  r_k = ReLU(conv_k1(h_{k-1})),  h_k = ReLU(h_{k-1} + conv_k2(r_k))
//   (M, b) = W_out h_2 + b_out,  I = M * F_rgb + b
//
// Activations are NHWC float32 with 32 channels.  The 3x3 convolutions are dense contractions
// (K = 9 taps x 32 channels per output) and run on the matrix cores: v_mfma_f32_16x16x4_f32
// (FP32 in, FP32 accumulate, so results match an FP32 reference to rounding).
//   * forward / input-gradient convolution (k_conv3x3): a workgroup computes a 16 x 16-pixel
//     tile for all 32 output channels from its 18 x 18 input halo staged in LDS; each wavefront
//     owns 4 pixel rows.  In an MFMA the A operand is 16 pixels x 4 channels, the B operand 4
//     channels x 16 output channels; the contraction order inside a tap is permuted so that a
//     lane's eight A values of a tap are eight consecutive channels of one pixel (two 16-byte
//     LDS reads), with B loaded to match.  The input gradient is the same convolution over the
//     output gradient with the weights flipped and transposed (read in place, not copied).
//   * weight gradient (k_conv3x3_wgrad): dW[tap][ci][co] = sum_p x[p + tap][ci] dy[p][co] is a
//     contraction over pixels; persistent workgroups stage 8 x 16-pixel tiles (and the input
//     halo) in LDS, each wavefront accumulates 9 of the 36 (tap, 16 ci, 16 co) output blocks in
//     registers, and a second kernel adds the workgroups' partial sums in a fixed order.
//   * the stem input, the 1x1 head and their adjoints are per-pixel kernels.
#include "kernels.hpp"
#include "reduce.hpp"

namespace splat {

constexpr int kCC = 32;            // padded channel count of every activation
constexpr int kTS = 16;            // forward tile side
constexpr int kHalo = kTS + 2;     // 18
constexpr int kLS = 36;            // floats per pixel in LDS (32 + 4: 16-byte aligned rows)
constexpr int kWTH = 8;            // weight-gradient tile: 8 rows x 16 columns
constexpr int kWOut = 9 * kCC * kCC + kCC;   // partial sums per workgroup: dW [tap][ci][co], db
constexpr int kHeadOut = 6 * kCC + 6;        // dW_out [6][32], db_out [6]
constexpr int kCnnBlock = 128;               // per-pixel kernels with LDS contractions

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Stages an R x Cw pixel window of a 32-channel NHWC image whose top-left pixel is (y0, x0) into
// LDS rows of kLS floats (zeros outside the image).  Every load of a thread is issued before its
// first LDS store, so the window's global loads are all in flight at once.
template <int R, int Cw>
__device__ __forceinline__ void stage_window(const float* __restrict__ img, int H, int W, int y0, int x0, float* dst) {
  constexpr int kVec = R * Cw * 8;
  constexpr int kPer = (kVec + 255) / 256;
  float4 v[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int i = threadIdx.x + 256 * j;
    v[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < kVec) {
      const int pix = i >> 3, q = i & 7;
      const int y = y0 + pix / Cw, x = x0 + pix % Cw;
      if (y >= 0 && y < H && x >= 0 && x < W) v[j] = reinterpret_cast<const float4*>(img + ((int64_t)y * W + x) * 32)[q];
    }
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int i = threadIdx.x + 256 * j;
    if (i < kVec) *reinterpret_cast<float4*>(&dst[(i >> 3) * kLS + (i & 7) * 4]) = v[j];
  }
}

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct ConvArgs {
  const float* in;      // [H*W][32]
  float* out;           // [H*W][32]
  const float* w;       // [co_n][ci_n][3][3] (OIHW)
  int ci_n, co_n;       // channels of w
  int transpose;        // 0: out[co] = sum w[co][ci][t] in[p + t][ci]; 1: input gradient
  const float* bias;    // [co_n] or null
  const float* addend;  // [H*W][32] or null, added before the activation
  const float* mask;    // [H*W][32] or null: out = v where mask > 0, else 0
  int relu;
  int H, W;
};

// B operand element: the weight taking input channel `cin` of the convolution's input to its
// output channel `cout` at tap (ky, kx); zero outside the weight's channels.
__device__ __forceinline__ float conv_w(const ConvArgs& a, int cin, int cout, int ky, int kx) {
  if (!a.transpose) {
    if (cin >= a.ci_n || cout >= a.co_n) return 0.f;
    return a.w[((cout * a.ci_n + cin) * 3 + ky) * 3 + kx];
  }
  // input gradient: the input holds gradients of the layer's outputs (co), the output its inputs (ci)
  if (cin >= a.co_n || cout >= a.ci_n) return 0.f;
  return a.w[((cin * a.ci_n + cout) * 3 + (2 - ky)) * 3 + (2 - kx)];
}

constexpr int kFrag = 9 * 8 * 2 * 64;   // B fragments of one convolution: [tap][step][half][lane]

// The B operands of every MFMA of k_conv3x3 in lane order, so that the convolution loads each
// tap's fragments as coalesced rows (and flips / transposes the weights for the input gradient
// here, once per launch, instead of per load).
__global__ void k_conv_frag(ConvArgs a, float* __restrict__ frag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kFrag) return;
  const int lane = i & 63, h = (i >> 6) & 1, s = (i >> 7) & 7, tap = i >> 10;
  frag[i] = conv_w(a, 8 * (lane >> 4) + s, 16 * h + (lane & 15), tap / 3, tap % 3);
}

__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a, const float* __restrict__ frag) {
  __shared__ __align__(16) float s_in[kHalo * kHalo * kLS];
  const int tiles_x = (a.W + kTS - 1) / kTS;
  const int tx0 = (int)(blockIdx.x % tiles_x) * kTS, ty0 = (int)(blockIdx.x / tiles_x) * kTS;
  stage_window<kHalo, kHalo>(a.in, a.H, a.W, ty0 - 1, tx0 - 1, s_in);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  floatx4 acc[4][2];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int h = 0; h < 2; ++h) acc[r][h] = floatx4{0.f, 0.f, 0.f, 0.f};
  float bf[8][2], bn[8][2];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int h = 0; h < 2; ++h) bf[s][h] = frag[(s * 2 + h) * 64 + lane];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap % 3;
    // the next tap's fragments are in flight while this tap's MFMAs run
    const int tn = tap < 8 ? tap + 1 : tap;
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) bn[s][h] = frag[((tn * 8 + s) * 2 + h) * 64 + lane];
    float av[4][8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int py = wave * 4 + r;
      const float* src = &s_in[((py + ky) * kHalo + li + kx) * kLS + 8 * lk];
      const float4 a0 = *reinterpret_cast<const float4*>(src);
      const float4 a1 = *reinterpret_cast<const float4*>(src + 4);
      av[r][0] = a0.x; av[r][1] = a0.y; av[r][2] = a0.z; av[r][3] = a0.w;
      av[r][4] = a1.x; av[r][5] = a1.y; av[r][6] = a1.z; av[r][7] = a1.w;
    }
    // eight independent accumulators between two MFMAs on the same one
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[r][0] = mfma4(av[r][s], bf[s][0], acc[r][0]);
        acc[r][1] = mfma4(av[r][s], bf[s][1], acc[r][1]);
      }
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) bf[s][h] = bn[s][h];
  }
  // D[i][j]: pixel column 4 lk + e of the row, output channel 16 h + li
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int y = ty0 + wave * 4 + r;
    if (y >= a.H) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int x = tx0 + 4 * lk + e;
      if (x >= a.W) continue;
      const int64_t base = ((int64_t)y * a.W + x) * kCC;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int co = 16 * h + li;
        float v = acc[r][h][e];
        if (a.bias && co < (a.transpose ? a.ci_n : a.co_n)) v += a.bias[co];
        if (a.addend) v += a.addend[base + co];
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.mask) v = a.mask[base + co] > 0.f ? v : 0.f;
        a.out[base + co] = v;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const float* __restrict__ x, const float* __restrict__ dy,
                                                        int H, int W, float* __restrict__ partial) {
  __shared__ __align__(16) float s_x[(kWTH + 2) * kHalo * kLS];
  __shared__ __align__(16) float s_dy[kWTH * kTS * kLS];
  __shared__ float s_b[8][kCC];
  const int tiles_x = (W + kTS - 1) / kTS, tiles_y = (H + kWTH - 1) / kWTH;
  const int n_tiles = tiles_x * tiles_y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  floatx4 acc[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
  float accb = 0.f;
  const int bco = threadIdx.x & 31, bg = threadIdx.x >> 5;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int tx0 = (tile % tiles_x) * kTS, ty0 = (tile / tiles_x) * kWTH;
    __syncthreads();   // the previous tile's LDS reads are done
    stage_window<kWTH + 2, kHalo>(x, H, W, ty0 - 1, tx0 - 1, s_x);
    stage_window<kWTH, kTS>(dy, H, W, ty0, tx0, s_dy);
    __syncthreads();
    for (int q = bg; q < kWTH * kTS; q += 8) accb += s_dy[q * kLS + bco];
    // nine independent accumulators (output blocks: tap, input-channel half, output half)
    // between two MFMAs on the same one
#pragma unroll 2
    for (int s = 0; s < kWTH * kTS / 4; ++s) {
      const int pix = 4 * s + lk;
      const int py = pix >> 4, px = pix & 15;
      const float bv0 = s_dy[pix * kLS + li], bv1 = s_dy[pix * kLS + 16 + li];
#pragma unroll
      for (int m = 0; m < 9; ++m) {
        const int t = wave + 4 * m;
        const int tap = t >> 2, ch = (t >> 1) & 1, oh = t & 1;
        const int ky = tap / 3, kx = tap % 3;
        const float av = s_x[((py + ky) * kHalo + px + kx) * kLS + 16 * ch + li];
        acc[m] = mfma4(av, oh ? bv1 : bv0, acc[m]);
      }
    }
  }
  float* dst = partial + (int64_t)blockIdx.x * kWOut;
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    const int t = wave + 4 * m;
    const int tap = t >> 2, ch = (t >> 1) & 1, oh = t & 1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ci = 16 * ch + 4 * lk + e, co = 16 * oh + li;
      dst[(tap * kCC + ci) * kCC + co] = acc[m][e];
    }
  }
  s_b[bg][bco] = accb;
  __syncthreads();
  if (threadIdx.x < kCC) {
    float s = 0.f;
    for (int g = 0; g < 8; ++g) s += s_b[g][threadIdx.x];
    dst[9 * kCC * kCC + threadIdx.x] = s;
  }
}

// dW (OIHW, +=) and db (+=) of one convolution from the column sums of the partials
struct ConvGradStore {
  float* dw;
  float* db;
  int ci_n, co_n;
  __device__ void operator()(int o, float s) const {
    if (o < 9 * kCC * kCC) {
      const int tap = o / (kCC * kCC), ci = (o / kCC) % kCC, co = o % kCC;
      if (dw && ci < ci_n && co < co_n) dw[(co * ci_n + ci) * 9 + tap] += s;
    } else {
      const int co = o - 9 * kCC * kCC;
      if (db && co < co_n) db[co] += s;
    }
  }
};

struct CnnGeo {
  float R[9];         // world -> camera rotation
  float fx, fy, cx, cy;
  int W, H;
};

// x = [F, d, e, 0...] per pixel; eight lanes per pixel, lane q writing channels 4q .. 4q + 3, so
// that a wavefront reads and writes contiguous rows (vec: 16-byte feature rows, C and Df multiples
// of 4)
__global__ __launch_bounds__(256) void k_cnn_input(const float* __restrict__ feat, int C, int Df, int E,
                                                   const float* __restrict__ embed, CnnGeo g, int vec,
                                                   float* __restrict__ x0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = t >> 3;
  const int k0 = 4 * (int)(t & 7);
  if (p >= (int64_t)g.W * g.H) return;
  const float* row = feat + p * C;
  float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
  if (vec && k0 + 4 <= Df) {
    out = *reinterpret_cast<const float4*>(row + k0);
  } else if (k0 < Df + 3 + E) {
    const int u = (int)(p % g.W), v = (int)(p / g.W);
    float dc0 = ((float)u + 0.5f - g.cx) / g.fx, dc1 = ((float)v + 0.5f - g.cy) / g.fy, dc2 = 1.f;
    const float inv = rsqrtf(dc0 * dc0 + dc1 * dc1 + 1.f);
    dc0 *= inv;
    dc1 *= inv;
    dc2 *= inv;
    // world direction R^T d_c
    const float dw0 = g.R[0] * dc0 + g.R[3] * dc1 + g.R[6] * dc2, dw1 = g.R[1] * dc0 + g.R[4] * dc1 + g.R[7] * dc2,
                dw2 = g.R[2] * dc0 + g.R[5] * dc1 + g.R[8] * dc2;
    float o4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + j;
      o4[j] = k < Df            ? row[k]
              : k == Df         ? dw0
              : k == Df + 1     ? dw1
              : k == Df + 2     ? dw2
              : k < Df + 3 + E  ? embed[k - Df - 3]
                                : 0.f;
    }
    out = make_float4(o4[0], o4[1], o4[2], o4[3]);
  }
  reinterpret_cast<float4*>(x0 + p * kCC)[t & 7] = out;
}

// the stem's input gradient: d_feat += dx[0:Df]; per-workgroup sums of dx[Df+3 : Df+3+E] (embedding)
// vec: the host found d_feat 16-byte aligned and C, Df multiples of 4 (16-byte rows)
__global__ __launch_bounds__(256) void k_cnn_input_bwd(const float* __restrict__ dx0, int64_t n, int C, int Df, int E,
                                                        int vec, float* __restrict__ d_feat,
                                                        float* __restrict__ partial_e) {
  __shared__ float s_e[256][9];
  __shared__ float s_p[8][9];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float e[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) e[k] = 0.f;
  if (p < n) {
    const float* src = dx0 + p * kCC;
    float v[kCC];
#pragma unroll
    for (int q = 0; q < 8; ++q) {   // every load issued before any store
      const float4 x = reinterpret_cast<const float4*>(src)[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
    if (d_feat) {
      float* row = d_feat + p * C;
      if (vec) {   // uniform: 16-byte rows
        float4 old[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (4 * q < Df) old[q] = reinterpret_cast<const float4*>(row)[q];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (4 * q < Df)
            reinterpret_cast<float4*>(row)[q] =
                make_float4(old[q].x + v[4 * q], old[q].y + v[4 * q + 1], old[q].z + v[4 * q + 2], old[q].w + v[4 * q + 3]);
      } else {
        float old[kCC];
#pragma unroll
        for (int k = 0; k < kCC; ++k) old[k] = k < Df ? row[k] : 0.f;
#pragma unroll
        for (int k = 0; k < kCC; ++k)
          if (k < Df) row[k] = old[k] + v[k];
      }
    }
    // the embedding's channels Df + 3 .. Df + 3 + E - 1, picked from the registers already loaded
#pragma unroll
    for (int k = 0; k < kCC; ++k)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < E && k == Df + 3 + j) e[j] = v[k];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) s_e[threadIdx.x][k] = e[k];
  __syncthreads();
  if (threadIdx.x < 64) {   // 8 slices of 32 rows per embedding entry, then the 8 slices in order
    const int k = threadIdx.x & 7, part = threadIdx.x >> 3;
    float s = 0.f;
    for (int t = 32 * part; t < 32 * part + 32; ++t) s += s_e[t][k];
    s_p[part][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    float s = 0.f;
    for (int part = 0; part < 8; ++part) s += s_p[part][threadIdx.x];
    partial_e[(int64_t)blockIdx.x * 8 + threadIdx.x] = s;
  }
}

struct HeadW {
  float w[6][kCC];
  float b[6];
};

__device__ __forceinline__ void stage_head(HeadW& Hw, const float* w_out, const float* b_out) {
  for (int i = threadIdx.x; i < 6 * kCC; i += blockDim.x) Hw.w[i / kCC][i % kCC] = w_out[i];
  if (threadIdx.x < 6) Hw.b[threadIdx.x] = b_out[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_cnn_head(const float* __restrict__ h2, const float* __restrict__ feat, int C,
                                                   const float* __restrict__ w_out, const float* __restrict__ b_out,
                                                   int64_t n, float* __restrict__ image) {
  __shared__ HeadW Hw;
  stage_head(Hw, w_out, b_out);
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float z[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) z[o] = Hw.b[o];
  const float4* hp = reinterpret_cast<const float4*>(h2 + p * kCC);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float4 h = hp[q];
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      z[o] = fmaf(Hw.w[o][4 * q], h.x, z[o]);
      z[o] = fmaf(Hw.w[o][4 * q + 1], h.y, z[o]);
      z[o] = fmaf(Hw.w[o][4 * q + 2], h.z, z[o]);
      z[o] = fmaf(Hw.w[o][4 * q + 3], h.w, z[o]);
    }
  }
  const float* f = feat + p * C;
#pragma unroll
  for (int c = 0; c < 3; ++c) image[p * 3 + c] = fmaf(z[c], f[c], z[3 + c]);
}

// head adjoint: dI -> dz -> d_feat (colour part), dpre2 = (W_out^T dz) * [h2 > 0]; dW_out, db_out
// as per-workgroup contractions over the workgroup's pixels (partials, summed later)
__global__ __launch_bounds__(kCnnBlock) void k_cnn_head_bwd(const float* __restrict__ h2, const float* __restrict__ feat,
                                                            int C, const float* __restrict__ w_out,
                                                            const float* __restrict__ b_out, int64_t n,
                                                            const float* __restrict__ d_image, float* __restrict__ d_feat,
                                                            float* __restrict__ dpre2, float* __restrict__ partial) {
  __shared__ HeadW Hw;
  __shared__ float s_h[kCnnBlock][kCC + 1];
  __shared__ float s_dz[kCnnBlock][6];
  stage_head(Hw, w_out, b_out);
  constexpr int NPT = (kHeadOut + kCnnBlock - 1) / kCnnBlock;
  float acc[NPT];
#pragma unroll
  for (int i = 0; i < NPT; ++i) acc[i] = 0.f;
  const int t = threadIdx.x;
  for (int64_t base = (int64_t)blockIdx.x * kCnnBlock; base < n; base += (int64_t)gridDim.x * kCnnBlock) {
    __syncthreads();
    const int64_t p = base + t;
    if (p < n) {
      float h[kCC];
      const float4* hp = reinterpret_cast<const float4*>(h2 + p * kCC);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float4 v = hp[q];
        h[4 * q] = v.x;
        h[4 * q + 1] = v.y;
        h[4 * q + 2] = v.z;
        h[4 * q + 3] = v.w;
      }
      float z[3];
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        float s = Hw.b[o];
#pragma unroll
        for (int c = 0; c < kCC; ++c) s = fmaf(Hw.w[o][c], h[c], s);
        z[o] = s;   // M
      }
      const float* f = feat + p * C;
      float dz[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float di = d_image[p * 3 + c];
        dz[c] = di * f[c];      // dL/dM
        dz[3 + c] = di;         // dL/db
        if (d_feat) d_feat[p * C + c] += di * z[c];
      }
      float4* gp = reinterpret_cast<float4*>(dpre2 + p * kCC);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float g4[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int c = 4 * q + m;
          float s = 0.f;
#pragma unroll
          for (int o = 0; o < 6; ++o) s = fmaf(Hw.w[o][c], dz[o], s);
          g4[m] = h[c] > 0.f ? s : 0.f;
        }
        gp[q] = make_float4(g4[0], g4[1], g4[2], g4[3]);
      }
#pragma unroll
      for (int c = 0; c < kCC; ++c) s_h[t][c] = h[c];
#pragma unroll
      for (int o = 0; o < 6; ++o) s_dz[t][o] = dz[o];
    } else {
#pragma unroll
      for (int c = 0; c < kCC; ++c) s_h[t][c] = 0.f;
#pragma unroll
      for (int o = 0; o < 6; ++o) s_dz[t][o] = 0.f;
    }
    __syncthreads();
    const int rows = (n - base) < kCnnBlock ? (int)(n - base) : kCnnBlock;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
      const int o = t + i * kCnnBlock;
      if (o >= kHeadOut) break;
      float s = 0.f;
      if (o < 6 * kCC) {
        const int oo = o / kCC, c = o % kCC;
        for (int q = 0; q < rows; ++q) s = fmaf(s_dz[q][oo], s_h[q][c], s);
      } else {
        const int oo = o - 6 * kCC;
        for (int q = 0; q < rows; ++q) s += s_dz[q][oo];
      }
      acc[i] += s;
    }
  }
#pragma unroll
  for (int i = 0; i < NPT; ++i) {
    const int o = t + i * kCnnBlock;
    if (o < kHeadOut) partial[(int64_t)blockIdx.x * kHeadOut + o] = acc[i];
  }
}

// ---- workspace --------------------------------------------------------------------------------
struct CnnWs {
  float* act[6];   // x0, h0, r1, h1, r2, h2
  float* g[3];     // gradient buffers
  float* frag;     // B fragments of the convolution being launched
  float* partial;  // partial sums
  size_t bytes;
};

inline int wgrad_blocks(int W, int H) {
  const int tiles = ((W + kTS - 1) / kTS) * ((H + kWTH - 1) / kWTH);
  return tiles < 768 ? tiles : 768;
}
inline int head_blocks(int64_t n) {
  const int64_t b = (n + kCnnBlock - 1) / kCnnBlock;
  return (int)(b < 1024 ? b : 1024);
}
inline int64_t input_bwd_blocks(int64_t n) { return (n + 255) / 256; }

// base == nullptr: sizes only (every pointer stays null; no arithmetic on the null base)
inline CnnWs carve_cnn(void* base, int W, int H) {
  CnnWs w;
  const int64_t n = (int64_t)W * H;
  const size_t act = ((size_t)n * kCC * sizeof(float) + 255) / 256 * 256;
  size_t off = 0;
  char* b = (char*)base;
  auto at = [&](size_t o) { return b ? (float*)(b + o) : nullptr; };
  for (int i = 0; i < 6; ++i, off += act) w.act[i] = at(off);
  for (int i = 0; i < 3; ++i, off += act) w.g[i] = at(off);
  w.frag = at(off);
  off += (size_t)kFrag * sizeof(float);
  size_t part = (size_t)wgrad_blocks(W, H) * kWOut;
  const size_t hp = (size_t)head_blocks(n) * kHeadOut;
  const size_t ep = (size_t)input_bwd_blocks(n) * 8;
  part = part > hp ? part : hp;
  part = part > ep ? part : ep;
  w.partial = at(off);
  off += (part * sizeof(float) + 255) / 256 * 256;
  w.bytes = off;
  return w;
}

static bool cnn_ok(const SplatCamera* cam, const SplatCameraCNN* m) {
  if (!cam || !m || cam->width <= 0 || cam->height <= 0) return false;
  if (m->n_feat < 3 || m->n_embed < 0 || m->n_embed > 8 || m->n_feat + 3 + m->n_embed > kCC) return false;
  if (!m->w_in || !m->b_in || !m->w_out || !m->b_out || (m->n_embed > 0 && !m->embed)) return false;
  for (int k = 0; k < 4; ++k)
    if (!m->w_block[k] || !m->b_block[k]) return false;
  return true;
}

static CnnGeo cnn_geo(const SplatCamera* cam) {
  CnnGeo g;
  for (int k = 0; k < 9; ++k) g.R[k] = cam->R[k];
  g.fx = cam->fx;
  g.fy = cam->fy;
  g.cx = cam->cx;
  g.cy = cam->cy;
  g.W = cam->width;
  g.H = cam->height;
  return g;
}

static hipError_t conv(const float* in, float* out, const float* w, int ci_n, int co_n, int transpose,
                       const float* bias, const float* addend, const float* mask, int relu, int W, int H, float* frag,
                       hipStream_t s) {
  ConvArgs a{in, out, w, ci_n, co_n, transpose, bias, addend, mask, relu, H, W};
  const int tiles = ((W + kTS - 1) / kTS) * ((H + kTS - 1) / kTS);
  hipLaunchKernelGGL(k_conv_frag, dim3((unsigned)(kFrag / 256)), dim3(256), 0, s, a, frag);
  hipLaunchKernelGGL(k_conv3x3, dim3((unsigned)tiles), dim3(256), 0, s, a, (const float*)frag);
  return hipGetLastError();
}

static hipError_t wgrad(const float* x, const float* dy, int ci_n, int co_n, float* dw, float* db, float* partial, int W,
                        int H, hipStream_t s) {
  const int nb = wgrad_blocks(W, H);
  hipLaunchKernelGGL(k_conv3x3_wgrad, dim3((unsigned)nb), dim3(256), 0, s, x, dy, H, W, partial);
  launch_column_sums((const float*)partial, kWOut, nb, kWOut, ConvGradStore{dw, db, ci_n, co_n}, s);
  return hipGetLastError();
}

}  // namespace splat

using namespace splat;

extern "C" {

size_t splat_camera_decode_workspace_bytes(int32_t width, int32_t height) {
  if (width <= 0 || height <= 0) return 0;
  return carve_cnn(nullptr, width, height).bytes;
}

int splat_camera_decode(const SplatCamera* cam, const float* feat, const SplatCameraCNN* cnn, float* image, void* ws,
                        size_t ws_bytes, void* stream) {
  if (!cnn_ok(cam, cnn) || !feat || !image) return SPLAT_ERR_INVALID_ARG;
  const int W = cam->width, H = cam->height;
  const int64_t n = (int64_t)W * H;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < splat_camera_decode_workspace_bytes(W, H)) return SPLAT_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  CnnWs w = carve_cnn(ws, W, H);
  const int C = cam->n_channels > 0 ? cam->n_channels : cnn->n_feat;
  if (cnn->n_feat > C) return SPLAT_ERR_INVALID_ARG;
  const int cin = cnn->n_feat + 3 + cnn->n_embed;
  const int vec = (((uintptr_t)feat & 15) == 0 && ((C | cnn->n_feat) & 3) == 0) ? 1 : 0;
  hipLaunchKernelGGL(k_cnn_input, dim3((unsigned)div_up(8 * n, 256)), dim3(256), 0, s, feat, C, cnn->n_feat,
                     cnn->n_embed, cnn->embed, cnn_geo(cam), vec, w.act[0]);
  hipError_t e = conv(w.act[0], w.act[1], cnn->w_in, cin, kCC, 0, cnn->b_in, nullptr, nullptr, 1, W, H, w.frag, s);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    float* hin = w.act[1 + 2 * k];
    e = conv(hin, w.act[2 + 2 * k], cnn->w_block[2 * k], kCC, kCC, 0, cnn->b_block[2 * k], nullptr, nullptr, 1, W, H,
             w.frag, s);
    if (e == hipSuccess)
      e = conv(w.act[2 + 2 * k], w.act[3 + 2 * k], cnn->w_block[2 * k + 1], kCC, kCC, 0, cnn->b_block[2 * k + 1], hin,
               nullptr, 1, W, H, w.frag, s);
  }
  if (e != hipSuccess) return SPLAT_ERR_DEVICE;
  hipLaunchKernelGGL(k_cnn_head, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, (const float*)w.act[5], feat, C,
                     cnn->w_out, cnn->b_out, n, image);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

int splat_camera_decode_bwd(const SplatCamera* cam, const float* feat, const SplatCameraCNN* cnn, const float* d_image,
                            float* d_feat, const SplatCameraCNNGrads* d_cnn, void* ws, size_t ws_bytes, void* stream) {
  if (!cnn_ok(cam, cnn) || !feat || !d_image || !d_cnn) return SPLAT_ERR_INVALID_ARG;
  const int W = cam->width, H = cam->height;
  const int64_t n = (int64_t)W * H;
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < splat_camera_decode_workspace_bytes(W, H)) return SPLAT_ERR_CAPACITY;
  hipStream_t s = (hipStream_t)stream;
  CnnWs w = carve_cnn(ws, W, H);
  const int C = cam->n_channels > 0 ? cam->n_channels : cnn->n_feat;
  if (cnn->n_feat > C) return SPLAT_ERR_INVALID_ARG;
  const int cin = cnn->n_feat + 3 + cnn->n_embed;
  float *x0 = w.act[0], *h0 = w.act[1], *r1 = w.act[2], *h1 = w.act[3], *r2 = w.act[4], *h2 = w.act[5];
  float *ga = w.g[0], *gb = w.g[1], *gc = w.g[2];
  // head: dpre2 -> ga
  const int hb = head_blocks(n);
  hipLaunchKernelGGL(k_cnn_head_bwd, dim3((unsigned)hb), dim3(kCnnBlock), 0, s, (const float*)h2, feat, C, cnn->w_out,
                     cnn->b_out, n, d_image, d_feat, ga, w.partial);
  launch_column_sums((const float*)w.partial, kHeadOut, hb, 6 * kCC, AddTo{d_cnn->w_out}, s);
  launch_column_sums((const float*)(w.partial + 6 * kCC), kHeadOut, hb, 6, AddTo{d_cnn->b_out}, s);
  hipError_t e = hipGetLastError();
  // blocks, last first: dpre_k in `dp`, h_{k-1}, r_k the saved activations
  float* dp = ga;
  float* spare[2] = {gb, gc};
  for (int k = 1; k >= 0 && e == hipSuccess; --k) {
    float* hin = w.act[1 + 2 * k];
    float* r = w.act[2 + 2 * k];
    float* du = spare[0];
    float* dnext = spare[1];
    // conv_k2: its input r_k, output gradient dpre_k
    e = wgrad(r, dp, kCC, kCC, d_cnn->w_block[2 * k + 1], d_cnn->b_block[2 * k + 1], w.partial, W, H, s);
    if (e == hipSuccess)   // du_k = conv_k2^T(dpre_k) * [r_k > 0]
      e = conv(dp, du, cnn->w_block[2 * k + 1], kCC, kCC, 1, nullptr, nullptr, r, 0, W, H, w.frag, s);
    if (e == hipSuccess)   // conv_k1: input h_{k-1}, output gradient du_k
      e = wgrad(hin, du, kCC, kCC, d_cnn->w_block[2 * k], d_cnn->b_block[2 * k], w.partial, W, H, s);
    if (e == hipSuccess)   // dpre_{k-1} = (dpre_k + conv_k1^T(du_k)) * [h_{k-1} > 0]
      e = conv(du, dnext, cnn->w_block[2 * k], kCC, kCC, 1, nullptr, dp, hin, 0, W, H, w.frag, s);
    spare[0] = dp;
    spare[1] = du;
    dp = dnext;
  }
  (void)h1;
  (void)r1;
  (void)r2;
  (void)h0;
  // stem: dW_in, db_in; dx0 = conv_in^T(dpre0)
  if (e == hipSuccess) e = wgrad(x0, dp, cin, kCC, d_cnn->w_in, d_cnn->b_in, w.partial, W, H, s);
  float* dx0 = spare[0];
  if (e == hipSuccess) e = conv(dp, dx0, cnn->w_in, cin, kCC, 1, nullptr, nullptr, nullptr, 0, W, H, w.frag, s);
  if (e != hipSuccess) return SPLAT_ERR_DEVICE;
  const int64_t eb = input_bwd_blocks(n);
  const int vec = (((uintptr_t)d_feat & 15) == 0 && ((C | cnn->n_feat) & 3) == 0) ? 1 : 0;
  hipLaunchKernelGGL(k_cnn_input_bwd, dim3((unsigned)eb), dim3(256), 0, s, (const float*)dx0, n, C, cnn->n_feat,
                     cnn->n_embed, vec, d_feat, w.partial);
  if (cnn->n_embed > 0) launch_column_sums((const float*)w.partial, 8, (int)eb, cnn->n_embed, AddTo{d_cnn->embed}, s);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

}  // extern "C"
