// compose.hip -- scene-graph composition at a capture time and its adjoint (SplatAD, arXiv
// 2411.16816: Sec. 3.1 "Scene representation"; the actor velocity term of Eq. (pixel_velocity)
// in Sec. 3.2 and App. D "Rolling shutter details").
//
// Gaussians of rigid actors hold their mean and rotation in the actor's box frame.  At a capture
// time actor a has pose (R_a, t_a) (actor -> world) and rigid motion (v_a, w_a) in its own frame:
//   mu_w = R_a mu + t_a,   q_w = q_a (x) q,   v_w = R_a (w_a x mu + v_a)
// with q_a = q_b (x) dq / |dq|, t_a = t_b + dt, v_a = v_b + dv (base values and learnable
// offsets).  Static Gaussians keep mean and rotation; their velocity is the input velocity.
//
// One thread per Gaussian (HBM-bound: ~72 B moved per Gaussian forward).  The adjoint writes the
// per-Gaussian gradients directly and sums the per-actor ones (translation, rotation matrix,
// rotation quaternion, linear and angular velocity: 22 floats) over each wavefront's lanes of
// one actor with the reduce-scatter of wave_ops.hpp, one global atomic per value and actor per
// wavefront; a per-actor pass then chains them to the offsets.
#include <mutex>

#include "kernels.hpp"
#include "wave_ops.hpp"

namespace splat {

struct Quat {
  float w, x, y, z;
};

__device__ __forceinline__ Quat qmul(Quat a, Quat b) {   // Hamilton product: R(a b) = R(a) R(b)
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
__device__ __forceinline__ Quat qconj(Quat a) { return {a.w, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ Quat qload(const float* p) { return {p[0], p[1], p[2], p[3]}; }
__device__ __forceinline__ Quat qnorm(Quat a, float* inv_len = nullptr) {
  const float r = rsqrtf(a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z);
  if (inv_len) *inv_len = r;
  return {a.w * r, a.x * r, a.y * r, a.z * r};
}

// rotation matrix of a unit quaternion, row-major
__device__ __forceinline__ void qmat(Quat q, float R[9]) {
  const float w = q.w, x = q.x, y = q.y, z = q.z;
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

struct ActorState {
  Quat qb, dq, qa;   // normalised base rotation, normalised offset, effective rotation
  float inv_dq;      // 1 / |dq| (offset given)
  float R[9], t[3], v[3], w[3];
};

__device__ __forceinline__ void actor_state(const SplatActors& A, int a, ActorState& s) {
  s.qb = qnorm(qload(A.rot + 4 * a));
  s.inv_dq = 1.f;
  s.dq = A.rot_offset ? qnorm(qload(A.rot_offset + 4 * a), &s.inv_dq) : Quat{1.f, 0.f, 0.f, 0.f};
  s.qa = qmul(s.qb, s.dq);
  qmat(s.qa, s.R);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.t[k] = A.trans[3 * a + k] + (A.trans_offset ? A.trans_offset[3 * a + k] : 0.f);
    s.v[k] = (A.lin_vel ? A.lin_vel[3 * a + k] : 0.f) + (A.lin_vel_offset ? A.lin_vel_offset[3 * a + k] : 0.f);
    s.w[k] = A.ang_vel ? A.ang_vel[3 * a + k] : 0.f;
  }
}

__global__ __launch_bounds__(256) void k_compose(int64_t n, const float* __restrict__ means, const float* __restrict__ quats,
                                                 const float* __restrict__ vel, const int32_t* __restrict__ actor_id,
                                                 SplatActors A, float* __restrict__ means_w, float* __restrict__ quats_w,
                                                 float* __restrict__ vel_w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = actor_id[i];
  float mu[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  const float4 q4 = reinterpret_cast<const float4*>(quats)[i];
  if (a < 0 || a >= A.n) {   // static background (ids past the actor count are treated the same way)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      means_w[3 * i + k] = mu[k];
      vel_w[3 * i + k] = vel ? vel[3 * i + k] : 0.f;
    }
    reinterpret_cast<float4*>(quats_w)[i] = q4;
    return;
  }
  ActorState s;
  actor_state(A, a, s);
  float u[3];
  cross3(s.w, mu, u);
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] += s.v[k];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    means_w[3 * i + r] = s.R[3 * r] * mu[0] + s.R[3 * r + 1] * mu[1] + s.R[3 * r + 2] * mu[2] + s.t[r];
    vel_w[3 * i + r] = s.R[3 * r] * u[0] + s.R[3 * r + 1] * u[1] + s.R[3 * r + 2] * u[2];
  }
  const Quat qw = qmul(s.qa, Quat{q4.x, q4.y, q4.z, q4.w});
  reinterpret_cast<float4*>(quats_w)[i] = make_float4(qw.w, qw.x, qw.y, qw.z);
}

constexpr int kActorAcc = 24;   // floats per actor accumulator: dt 3, dR 9, dq_a 4, dv 3, dw 3, pad 2

// Adjoint of k_compose.  Grid-stride over the Gaussians; every wavefront sums the per-actor
// gradients of its lanes actor by actor (lanes of other actors and static lanes contribute
// zeros) and adds them to acc[actor] with one atomic per value.
__global__ __launch_bounds__(256) void k_compose_bwd(int64_t n, const float* __restrict__ means,
                                                     const float* __restrict__ quats, const int32_t* __restrict__ actor_id,
                                                     SplatActors A, const float* __restrict__ gm,
                                                     const float* __restrict__ gq, const float* __restrict__ gv,
                                                     float* __restrict__ d_means, float* __restrict__ d_quats,
                                                     float* __restrict__ d_vel, float* __restrict__ acc) {
  const int lane = threadIdx.x & 63;
  constexpr int V = 22;
  bool store;
  const int slot = scatter_slot<V>(lane, store);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // every lane of a wavefront runs the same number of iterations (the reduction needs them all)
  const int64_t first = i0 - lane;
  for (int64_t base = first; base < n; base += stride) {
    const int64_t i = base + lane;
    const bool in = i < n;
    int a = in ? actor_id[i] : -1;
    if (a >= A.n) a = -1;
    float g_m[3] = {0.f, 0.f, 0.f}, g_v[3] = {0.f, 0.f, 0.f};
    Quat g_q{0.f, 0.f, 0.f, 0.f};
    float mu[3] = {0.f, 0.f, 0.f};
    Quat q{1.f, 0.f, 0.f, 0.f};
    if (in) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        g_m[k] = gm[3 * i + k];
        g_v[k] = gv[3 * i + k];
        mu[k] = means[3 * i + k];
      }
      const float4 g4 = reinterpret_cast<const float4*>(gq)[i];
      g_q = {g4.x, g4.y, g4.z, g4.w};
      const float4 q4 = reinterpret_cast<const float4*>(quats)[i];
      q = {q4.x, q4.y, q4.z, q4.w};
    }
    float vals[V];
#pragma unroll
    for (int k = 0; k < V; ++k) vals[k] = 0.f;
    if (in && a < 0) {   // static: identity composition
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        d_means[3 * i + k] += g_m[k];
        if (d_vel) d_vel[3 * i + k] += g_v[k];
      }
      float4* dq4 = reinterpret_cast<float4*>(d_quats) + i;
      const float4 o = *dq4;
      *dq4 = make_float4(o.x + g_q.w, o.y + g_q.x, o.z + g_q.y, o.w + g_q.z);
    } else if (in) {
      ActorState s;
      actor_state(A, a, s);
      float u[3], gl[3], gm_l[3], t1[3];
      cross3(s.w, mu, u);
#pragma unroll
      for (int k = 0; k < 3; ++k) u[k] += s.v[k];
      // actor-frame images of the upstream gradients: R^T g
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gl[c] = s.R[c] * g_v[0] + s.R[3 + c] * g_v[1] + s.R[6 + c] * g_v[2];
        gm_l[c] = s.R[c] * g_m[0] + s.R[3 + c] * g_m[1] + s.R[6 + c] * g_m[2];
      }
      cross3(gl, s.w, t1);   // d/dmu of R (w x mu): (R^T g_v) x w
#pragma unroll
      for (int k = 0; k < 3; ++k) d_means[3 * i + k] += gm_l[k] + t1[k];
      const Quat dql = qmul(qconj(s.qa), g_q);   // q_w = q_a q: dq = conj(q_a) g
      float4* dq4 = reinterpret_cast<float4*>(d_quats) + i;
      const float4 o = *dq4;
      *dq4 = make_float4(o.x + dql.w, o.y + dql.x, o.z + dql.y, o.w + dql.z);
      // per-actor values
#pragma unroll
      for (int k = 0; k < 3; ++k) vals[k] = g_m[k];                          // dt
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) vals[3 + 3 * r + c] = g_m[r] * mu[c] + g_v[r] * u[c];   // dR
      const Quat dqa = qmul(g_q, qconj(q));                                  // dq_a = g conj(q)
      vals[12] = dqa.w; vals[13] = dqa.x; vals[14] = dqa.y; vals[15] = dqa.z;
#pragma unroll
      for (int k = 0; k < 3; ++k) vals[16 + k] = gl[k];                      // dv = R^T g_v
      cross3(mu, gl, t1);                                                    // dw = mu x R^T g_v
#pragma unroll
      for (int k = 0; k < 3; ++k) vals[19 + k] = t1[k];
    }
    // sum over the wavefront's lanes, one actor at a time
    uint64_t todo = __ballot(in && a >= 0);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const int aa = __shfl(a, leader, 64);
      const bool mine = in && a == aa;
      todo &= ~__ballot(mine);
      float x[V];
#pragma unroll
      for (int k = 0; k < V; ++k) x[k] = mine ? vals[k] : 0.f;
      const float r = wave_reduce_scatter<V>(x);
      if (store) atomicAdd(acc + (int64_t)aa * kActorAcc + slot, r);
    }
  }
}

// d(sum G . R(q)) / dq for the polynomial rotation matrix of a unit quaternion (row-major G)
__device__ __forceinline__ Quat rotmat_grad(Quat q, const float G[9]) {
  const float w = q.w, x = q.x, y = q.y, z = q.z;
  Quat d;
  d.w = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
  d.x = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] + w * G[7] - 2.f * x * G[8]);
  d.y = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] - 2.f * y * G[8]);
  d.z = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
  return d;
}

// Per actor: the summed gradients of (t_a, R_a, q_a, v_a, w_a) chained to the learnable arrays.
__global__ void k_actor_finalize(SplatActors A, const float* __restrict__ acc, SplatActorGrads G) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.n) return;
  const float* s = acc + (int64_t)a * kActorAcc;
  if (G.trans_offset)
    for (int k = 0; k < 3; ++k) G.trans_offset[3 * a + k] += s[k];
  if (G.lin_vel_offset)
    for (int k = 0; k < 3; ++k) G.lin_vel_offset[3 * a + k] += s[16 + k];
  if (G.ang_vel)
    for (int k = 0; k < 3; ++k) G.ang_vel[3 * a + k] += s[19 + k];
  if (G.rot_offset && A.rot_offset) {
    ActorState st;
    actor_state(A, a, st);
    const Quat gr = rotmat_grad(st.qa, s + 3);
    const Quat gqa{s[12] + gr.w, s[13] + gr.x, s[14] + gr.y, s[15] + gr.z};
    const Quat gdn = qmul(qconj(st.qb), gqa);   // q_a = q_b dq^: d dq^ = conj(q_b) g
    // through dq^ = dq / |dq|: (g - dq^ (dq^ . g)) / |dq|
    const float dot = gdn.w * st.dq.w + gdn.x * st.dq.x + gdn.y * st.dq.y + gdn.z * st.dq.z;
    float* o = G.rot_offset + 4 * a;
    o[0] += (gdn.w - st.dq.w * dot) * st.inv_dq;
    o[1] += (gdn.x - st.dq.x * dot) * st.inv_dq;
    o[2] += (gdn.y - st.dq.y * dot) * st.inv_dq;
    o[3] += (gdn.z - st.dq.z * dot) * st.inv_dq;
  }
}

}  // namespace splat

using namespace splat;

static bool actors_ok(const SplatActors* A) {
  return A && A->n >= 0 && (A->n == 0 || (A->rot && A->trans));
}

static int compose_bwd_check(int64_t n, const float* means, const float* quats, const int32_t* actor_id,
                             const SplatActors* actors, const float* d_means_w, const float* d_quats_w,
                             const float* d_vel_w, const float* d_means, const float* d_quats,
                             const SplatActorGrads* d_actors) {
  if (n < 0 || !actors_ok(actors) || !d_actors) return SPLAT_ERR_INVALID_ARG;
  if (n == 0) return SPLAT_OK;
  if (!means || !quats || !actor_id || !d_means_w || !d_quats_w || !d_vel_w || !d_means || !d_quats)
    return SPLAT_ERR_INVALID_ARG;
  if ((((uintptr_t)quats) | ((uintptr_t)d_quats_w) | ((uintptr_t)d_quats)) & 15) return SPLAT_ERR_INVALID_ARG;
  return SPLAT_OK;
}

// The adjoint's launches with the per-actor accumulators in `acc` (actors->n x kActorAcc floats,
// cleared here by a fill kernel so that the sequence stays capturable).
static int compose_bwd_launch(int64_t n, const float* means, const float* quats, const int32_t* actor_id,
                              const SplatActors* actors, const float* d_means_w, const float* d_quats_w,
                              const float* d_vel_w, float* d_means, float* d_quats, float* d_velocities,
                              const SplatActorGrads* d_actors, float* acc, hipStream_t s) {
  if (actors->n > 0 && launch_fill_f32(acc, (int64_t)actors->n * kActorAcc, 0.f, s) != hipSuccess)
    return SPLAT_ERR_DEVICE;
  int64_t blocks = div_up(n, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_compose_bwd, dim3((unsigned)blocks), dim3(256), 0, s, n, means, quats, actor_id, *actors,
                     d_means_w, d_quats_w, d_vel_w, d_means, d_quats, d_velocities, acc);
  if (actors->n > 0)
    hipLaunchKernelGGL(k_actor_finalize, dim3((unsigned)div_up(actors->n, 64)), dim3(64), 0, s, *actors,
                       (const float*)acc, *d_actors);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

// Library-owned accumulators of splat_compose_bwd_noalloc: SPLAT_COMPOSE_NOALLOC_MAX_ACTORS
// actors of kActorAcc floats.  Each GPU holds its own copy at its own address for the life of
// the process.  In host code `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is handed to kernels.
static __device__ __align__(256) float scratch[(size_t)SPLAT_COMPOSE_NOALLOC_MAX_ACTORS * kActorAcc];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mutex;
static float* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the first call there).
static bool scratch_address(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return false;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
    g_scratch_ptr[dev] = (float*)p;
  }
  *out = g_scratch_ptr[dev];
  return true;
}

extern "C" {

int splat_compose(int64_t n, const float* means, const float* quats, const float* velocities, const int32_t* actor_id,
                  const SplatActors* actors, float* means_w, float* quats_w, float* vel_w, void* stream) {
  if (n < 0 || !actors_ok(actors)) return SPLAT_ERR_INVALID_ARG;
  if (n == 0) return SPLAT_OK;
  if (!means || !quats || !actor_id || !means_w || !quats_w || !vel_w) return SPLAT_ERR_INVALID_ARG;
  if ((((uintptr_t)quats) | ((uintptr_t)quats_w)) & 15) return SPLAT_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_compose, dim3((unsigned)div_up(n, 256)), dim3(256), 0, (hipStream_t)stream, n, means, quats,
                     velocities, actor_id, *actors, means_w, quats_w, vel_w);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

size_t splat_compose_workspace_bytes(int32_t n_actors) {
  return (size_t)(n_actors > 0 ? n_actors : 1) * kActorAcc * sizeof(float);
}

int splat_compose_bwd(int64_t n, const float* means, const float* quats, const int32_t* actor_id,
                      const SplatActors* actors, const float* d_means_w, const float* d_quats_w, const float* d_vel_w,
                      float* d_means, float* d_quats, float* d_velocities, const SplatActorGrads* d_actors, void* ws,
                      size_t ws_bytes, void* stream) {
  const int rc = compose_bwd_check(n, means, quats, actor_id, actors, d_means_w, d_quats_w, d_vel_w, d_means, d_quats,
                                   d_actors);
  if (rc != SPLAT_OK || n == 0) return rc;
  if (!ws || ws_bytes < splat_compose_workspace_bytes(actors->n)) return SPLAT_ERR_CAPACITY;
  return compose_bwd_launch(n, means, quats, actor_id, actors, d_means_w, d_quats_w, d_vel_w, d_means, d_quats,
                            d_velocities, d_actors, (float*)ws, (hipStream_t)stream);
}

int splat_compose_bwd_noalloc(int64_t n, const float* means, const float* quats, const int32_t* actor_id,
                              const SplatActors* actors, const float* d_means_w, const float* d_quats_w,
                              const float* d_vel_w, float* d_means, float* d_quats, float* d_velocities,
                              const SplatActorGrads* d_actors, void* stream) {
  const int rc = compose_bwd_check(n, means, quats, actor_id, actors, d_means_w, d_quats_w, d_vel_w, d_means, d_quats,
                                   d_actors);
  if (rc != SPLAT_OK || n == 0) return rc;
  if (actors->n > SPLAT_COMPOSE_NOALLOC_MAX_ACTORS) return SPLAT_ERR_CAPACITY;
  float* acc = nullptr;
  if (!scratch_address(&acc)) return SPLAT_ERR_DEVICE;
  return compose_bwd_launch(n, means, quats, actor_id, actors, d_means_w, d_quats_w, d_vel_w, d_means, d_quats,
                            d_velocities, d_actors, acc, (hipStream_t)stream);
}

}  // extern "C"
