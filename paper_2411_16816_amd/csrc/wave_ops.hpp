// wave_ops.hpp -- wavefront (64-lane) reductions shared by the rasteriser adjoint and the
// projection adjoint.
#pragma once

#include <hip/hip_runtime.h>

namespace splat {

// Wavefront-scope ordering of LDS accesses between lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

// Wavefront reduce-scatter of V values per lane (V <= 64).  Six levels, one per lane-index bit
// (5 down to 0): at a level with M values per lane, the lanes whose bit is 0 keep positions
// [0, H) and the others positions [H, M), H = ceil(M / 2) (a missing upper partner is a zero),
// each adding its partner lane's copy.  Bit 5 moves data with v_permlane32_swap, bit 4 with
// v_permlane16_swap, bits 3..0 with DPP row_mirror, row_half_mirror and quad permutations.
// Once one value is left the remaining levels are plain sums.  About 2 V instructions in all,
// against 6 V for V separate wavefront reductions; scatter_slot() tells each lane which value
// it ends up holding.
constexpr int rs_half(int m) { return m > 1 ? (m + 1) / 2 : 1; }

template <int M, int N>
__device__ __forceinline__ void rs_swap32(float (&v)[N]) {
  constexpr int H = rs_half(M);
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float hi = (M == 1) ? v[0] : ((i + H < M) ? v[i + H] : 0.f);
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(hi), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

template <int M, int N>
__device__ __forceinline__ void rs_swap16(float (&v)[N]) {
  constexpr int H = rs_half(M);
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float hi = (M == 1) ? v[0] : ((i + H < M) ? v[i + H] : 0.f);
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(hi), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

template <int CTRL, int M, int N>
__device__ __forceinline__ void rs_dpp(float (&v)[N], bool bit) {
  if constexpr (M == 1) {
    v[0] += dpp_f<CTRL>(v[0]);
  } else {
    constexpr int H = rs_half(M);
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float a = v[i];
      const float b = (i + H < M) ? v[i + H] : 0.f;
      const float keep = bit ? b : a;
      const float send = bit ? a : b;
      v[i] = keep + dpp_f<CTRL>(send);
    }
  }
}

template <int V, int N>
__device__ __forceinline__ float wave_reduce_scatter(float (&v)[N]) {
  static_assert(V >= 1 && V <= 64 && N >= V, "V");
  const int lane = threadIdx.x & 63;
  constexpr int M1 = rs_half(V), M2 = rs_half(M1), M3 = rs_half(M2), M4 = rs_half(M3), M5 = rs_half(M4);
  rs_swap32<V>(v);                                  // bit 5
  rs_swap16<M1>(v);                                 // bit 4
  rs_dpp<0x140, M2>(v, (lane >> 3) & 1);            // bit 3: row_mirror (i <-> 15 - i)
  rs_dpp<0x141, M3>(v, (lane >> 2) & 1);            // bit 2: row_half_mirror (i <-> 7 - i)
  rs_dpp<0x4E, M4>(v, (lane >> 1) & 1);             // bit 1: quad_perm [2,3,0,1]
  rs_dpp<0xB1, M5>(v, lane & 1);                    // bit 0: quad_perm [1,0,3,2]
  return v[0];
}

// Which value lane `lane` holds after wave_reduce_scatter<V>, and whether it should store it
// (one lane per value).
template <int V>
__device__ __forceinline__ int scatter_slot(int lane, bool& store) {
  int m = V, real = V, pos = 0;
  bool first = true;   // first lane of a group that holds the same value after plain levels
  for (int b = 5; b >= 0; --b) {
    const bool bit = (lane >> b) & 1;
    if (m > 1) {
      const int h = (m + 1) / 2;
      if (bit) { pos += h; real -= h; } else { real = real < h ? real : h; }
      m = h;
    } else {
      first = first && !bit;
    }
  }
  store = first && real >= 1;
  return pos;
}

}  // namespace splat
