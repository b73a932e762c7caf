// Generator entry points: raw Philox blocks, the float32 ln and Box-Muller
// pairs, exposed so the random streams can be checked bit for bit.
#include "internal.hpp"

namespace leea {

__global__ void rng_philox_kernel(const uint4* __restrict__ ctr, uint32_t k0, uint32_t k1,
                                  uint4* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 c = ctr[i];
  out[i] = philox(c.x, c.y, c.z, c.w, k0, k1);
}

__global__ void rng_ln32_kernel(const float* __restrict__ u, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = ln32(u[i]);
}

__global__ void rng_normal_kernel(const uint2* __restrict__ ab, float2* __restrict__ z,
                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint2 w = ab[i];
  float2 r;
  normal_pair(w.x, w.y, r.x, r.y);
  z[i] = r;
}

static dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_rng_philox(const uint32_t* ctr, uint64_t key, uint32_t* out, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(rng_philox_kernel, grid_for(n), dim3(256), 0, s,
                     reinterpret_cast<const uint4*>(ctr), (uint32_t)key, (uint32_t)(key >> 32),
                     reinterpret_cast<uint4*>(out), n);
  return hipGetLastError();
}

hipError_t launch_rng_ln32(const float* u, float* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(rng_ln32_kernel, grid_for(n), dim3(256), 0, s, u, out, n);
  return hipGetLastError();
}

hipError_t launch_rng_normal_pairs(const uint32_t* ab, float* z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(rng_normal_kernel, grid_for(n), dim3(256), 0, s,
                     reinterpret_cast<const uint2*>(ab), reinterpret_cast<float2*>(z), n);
  return hipGetLastError();
}

}  // namespace leea
