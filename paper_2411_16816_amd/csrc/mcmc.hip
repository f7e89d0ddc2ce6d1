// mcmc.hip -- the MCMC regulariser of the training-details appendix (SplatAD, arXiv 2411.16816;
// the opacity and scale regularisation of the MCMC densification strategy the paper adopts):
//   L = lambda_o sum_i |o_i| + lambda_S sum_i sum_j |sqrt(eig_j(Sigma_i))|.
// With Sigma = R diag(exp(2 l)) R^T (Sec. 3.1) the eigenvalues are exp(2 l_j) for any rotation,
// so the scale term is lambda_S sum exp(l_j): no rotation enters, and dL/dl_j = lambda_S exp(l_j),
// dL/do = lambda_o sign(o).
//
// HBM-bound: per Gaussian it reads o and l (16 B) and read-modify-writes their gradients
// (32 B).  A grid-stride loop; L is summed per wavefront, then per workgroup through LDS, and
// added to the caller's scalar with one atomic per workgroup.
#include <cmath>

#include "kernels.hpp"
#include "wave_ops.hpp"

namespace splat {

__global__ __launch_bounds__(256) void k_mcmc_reg(int64_t n, const float* __restrict__ opac,
                                                  const float* __restrict__ log_scales, float lam_o, float lam_s,
                                                  float* __restrict__ value, float* __restrict__ d_opac,
                                                  float* __restrict__ d_ls) {
  __shared__ float s_part[4];
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float o = opac[i];
    const float s0 = expf(log_scales[3 * i]), s1 = expf(log_scales[3 * i + 1]), s2 = expf(log_scales[3 * i + 2]);
    acc += lam_o * fabsf(o) + lam_s * (s0 + s1 + s2);
    if (d_opac) d_opac[i] += lam_o * (o > 0.f ? 1.f : (o < 0.f ? -1.f : 0.f));
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
  int64_t blocks = div_up(g->n, 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_mcmc_reg, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, g->n, g->opacities,
                     g->log_scales, lambda_o, lambda_s, value, d_o, d_l);
  return hipGetLastError() == hipSuccess ? SPLAT_OK : SPLAT_ERR_DEVICE;
}

}  // extern "C"
