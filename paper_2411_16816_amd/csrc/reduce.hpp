// reduce.hpp -- fixed-order column sums of per-workgroup partial sums (the weight gradients of
// the decoders are contractions over rays or pixels; each workgroup leaves one row of partials).
#pragma once

#include <hip/hip_runtime.h>

namespace splat {

constexpr int kColWaves = 16;

// Column sums of partial [n_rows, stride] for columns [0, n_cols): a 1024-thread workgroup takes
// 64 consecutive columns (one per lane); wavefront w adds rows w, w + 16, w + 32, ... with four
// running sums in flight, then wavefront 0 adds the 16 wavefront sums in order.  The order of
// every addition is fixed, so the result does not depend on timing.  `st(col, sum)` stores it.
template <class Store>
__global__ __launch_bounds__(1024) void k_column_sums(const float* __restrict__ partial, int64_t stride, int n_rows,
                                                      int n_cols, Store st) {
  __shared__ float s[kColWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + lane;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  if (o < n_cols) {
    int r = w;
    for (; r + 3 * kColWaves < n_rows; r += 4 * kColWaves) {
      a0 += partial[(int64_t)r * stride + o];
      a1 += partial[(int64_t)(r + kColWaves) * stride + o];
      a2 += partial[(int64_t)(r + 2 * kColWaves) * stride + o];
      a3 += partial[(int64_t)(r + 3 * kColWaves) * stride + o];
    }
    for (; r < n_rows; r += kColWaves) a0 += partial[(int64_t)r * stride + o];
  }
  s[w][lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (w == 0 && o < n_cols) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < kColWaves; ++k) t += s[k][lane];
    st(o, t);
  }
}

template <class Store>
inline void launch_column_sums(const float* partial, int64_t stride, int n_rows, int n_cols, Store st, hipStream_t s) {
  if (n_cols <= 0) return;
  hipLaunchKernelGGL(k_column_sums<Store>, dim3((unsigned)((n_cols + 63) / 64)), dim3(64 * kColWaves), 0, s, partial,
                     stride, n_rows, n_cols, st);
}

// dst[col] += sum (dst may be null: nothing stored)
struct AddTo {
  float* dst;
  __device__ void operator()(int o, float v) const {
    if (dst) dst[o] += v;
  }
};

}  // namespace splat
