// Operand preparation of the reduced-precision first layer: largest
// magnitudes for the FP8 scales (of the batch, and of every network's W_1)
// and the quantised copy of the batch that the evaluation kernels read.
#include "lowp.hpp"
#include "runs.hpp"

namespace leea {

// FP8 scales of one evaluation: workgroups [0, pop) find the largest
// magnitude of each later layer's weights of network blockIdx.x; the others
// reduce the batch (one workgroup: it writes *x_amax; several: one atomic
// each into a word cleared before the launch).
__global__ __launch_bounds__(256) void fp8_scales_kernel(const float* __restrict__ x, int64_t n,
                                                         uint32_t* __restrict__ x_amax, int xg,
                                                         const float* __restrict__ genomes,
                                                         NetDesc nd, int pop,
                                                         uint32_t* __restrict__ tail) {
  __shared__ uint32_t red[4];
  __shared__ uint32_t lred[4][kTailScales];
  const int j = blockIdx.x;
  if (j < pop) {
    const float* g = genomes + (int64_t)j * nd.stride;
    const int L = nd.L;
    uint32_t m[kTailScales];
#pragma unroll
    for (int l = 0; l < kTailScales; ++l) m[l] = 0u;
    // each later layer's weights on their own (a few thousand values), four
    // independent loads in flight per thread
    for (int l = 1; l < L; ++l) {
      const float* w = g + nd.woff[l];
      const int n = nd.w[l] * nd.w[l + 1];
      uint32_t ml = 0;
      for (int i0 = threadIdx.x; i0 < n; i0 += 4 * 256) {
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = i0 + 256 * k < n ? w[i0 + 256 * k] : 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t a = mag_bits(v[k]);
          ml = a > ml ? a : ml;
        }
      }
#pragma unroll
      for (int q = 1; q < kTailScales; ++q)
        if (q == l) m[q] = ml;
    }
#pragma unroll
    for (int l = 1; l < kTailScales; ++l) {
      const uint32_t w = wave_umax(m[l]);
      if ((threadIdx.x & 63) == 0) lred[threadIdx.x >> 6][l] = w;
    }
    __syncthreads();
    const int l = threadIdx.x;
    if (l >= 1 && l < L) {
      uint32_t r = lred[0][l];
      for (int w = 1; w < 4; ++w) r = lred[w][l] > r ? lred[w][l] : r;
      tail[(int64_t)j * kTailScales + l] = r;
    }
    return;
  }
  const int g = j - pop;
  uint32_t m = 0;
  // the batch is 16-byte aligned with n a multiple of 4: 16-byte loads, four
  // in flight per thread
  const float4* x4 = reinterpret_cast<const float4*>(x);
  const int64_t n4 = n >> 2;
  const int64_t step = (int64_t)xg * 256;
  for (int64_t i0 = (int64_t)g * 256 + threadIdx.x; i0 < n4; i0 += 4 * step) {
    float4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      v[k] = i0 + step * k < n4 ? x4[i0 + step * k] : float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t a = mag_bits(v[k].x), c = mag_bits(v[k].y), d = mag_bits(v[k].z),
               e = mag_bits(v[k].w);
      a = a > c ? a : c;
      d = d > e ? d : e;
      a = a > d ? a : d;
      m = a > m ? a : m;
    }
  }
  m = wave_umax(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = red[0];
    for (int i = 1; i < 4; ++i) r = red[i] > r ? red[i] : r;
    if (xg == 1)
      *x_amax = r;
    else if (r)
      atomicMax(x_amax, r);
  }
}

hipError_t launch_fp8_scales(const float* x, int64_t n, uint32_t* x_amax, const float* genomes,
                             const NetDesc& nd, int pop, uint32_t* tail, hipStream_t s) {
  // the batch: one workgroup up to 16 K values, else at most 256 (one
  // atomic each, after clearing the word)
  int64_t xg = (n + 2047) / 2048;
  xg = n <= 16384 ? 1 : (xg > 256 ? 256 : xg);
  if (xg > 1) {
    const hipError_t e = launch_fill(reinterpret_cast<float*>(x_amax), 1, 0.0f, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fp8_scales_kernel, dim3((unsigned)(pop + xg)), dim3(256), 0, s, x, n, x_amax,
                     (int)xg, genomes, nd, pop, tail);
  return hipGetLastError();
}

// amax[j] = max over network j's W_1 of mag_bits; one workgroup per network.
__global__ __launch_bounds__(256) void amax_w1_kernel(const float* __restrict__ genomes,
                                                      NetDesc nd, uint32_t* __restrict__ amax) {
  __shared__ uint32_t red[4];
  const int j = blockIdx.x;
  const float* w = genomes + (int64_t)j * nd.stride + nd.woff[0];
  const int64_t n = (int64_t)nd.w[0] * nd.w[1];  // w[0] % 4 == 0: whole float4s
  const float4* w4 = reinterpret_cast<const float4*>(w);
  uint32_t m = 0;
  for (int64_t i = threadIdx.x; i < (n >> 2); i += 256) {
    const float4 v = w4[i];
    uint32_t a = mag_bits(v.x), b = mag_bits(v.y), c = mag_bits(v.z), d = mag_bits(v.w);
    a = a > b ? a : b;
    c = c > d ? c : d;
    a = a > c ? a : c;
    m = a > m ? a : m;
  }
  m = wave_umax(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = red[0];
    for (int i = 1; i < 4; ++i) r = red[i] > r ? red[i] : r;
    amax[j] = r;
  }
}

// Quantised batch as float values [b][n0] (read by the small-batch kernel,
// which multiplies exact products on the FP32 matrix cores).
template <int DT>
__global__ __launch_bounds__(256) void quantize_values_kernel(const float* __restrict__ x,
                                                              int64_t n,
                                                              const uint32_t* __restrict__ x_amax,
                                                              float* __restrict__ out) {
  const int neg_e = DT == 2 ? -fp8_exponent(*x_amax) : 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = quantize<DT>(x[i], neg_e);
}

// Quantised batch packed for the low-precision matrix cores: [b][kp]
// bfloat16 or E4M3 codes, kp = n0 rounded up to 32, zero padded.  One
// thread per 8 consecutive elements.
template <int DT>
__global__ __launch_bounds__(256) void quantize_packed_kernel(const float* __restrict__ x, int b,
                                                              int n0, int kp,
                                                              const uint32_t* __restrict__ x_amax,
                                                              void* __restrict__ out) {
  const int neg_e = DT == 2 ? -fp8_exponent(*x_amax) : 0;
  const int per_row = kp >> 3;
  const int64_t items = (int64_t)b * per_row;
  for (int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * 256) {
    const int m = (int)(it / per_row);
    const int k = (int)(it - (int64_t)m * per_row) * 8;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = k + e < n0 ? x[(int64_t)m * n0 + k + e] : 0.0f;
    if constexpr (DT == 1) {
      uint4 o;
      o.x = pack_bf16x2(v[0], v[1]);
      o.y = pack_bf16x2(v[2], v[3]);
      o.z = pack_bf16x2(v[4], v[5]);
      o.w = pack_bf16x2(v[6], v[7]);
      reinterpret_cast<uint4*>(out)[it] = o;
    } else {
      uint2 o;
      o.x = pack_fp8x4(ldexpf(v[0], neg_e), ldexpf(v[1], neg_e), ldexpf(v[2], neg_e),
                       ldexpf(v[3], neg_e));
      o.y = pack_fp8x4(ldexpf(v[4], neg_e), ldexpf(v[5], neg_e), ldexpf(v[6], neg_e),
                       ldexpf(v[7], neg_e));
      reinterpret_cast<uint2*>(out)[it] = o;
    }
  }
}

static unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_amax_w1(const float* genomes, const NetDesc& nd, int pop, uint32_t* amax,
                          hipStream_t s) {
  hipLaunchKernelGGL(amax_w1_kernel, dim3((unsigned)pop), dim3(256), 0, s, genomes, nd, amax);
  return hipGetLastError();
}

hipError_t launch_quantize_x(int dt, bool packed, const float* x, int b, int n0, int kp,
                             const uint32_t* x_amax, void* out, hipStream_t s) {
  if (packed) {
    const int64_t items = (int64_t)b * (kp >> 3);
    if (dt == 1)
      hipLaunchKernelGGL(quantize_packed_kernel<1>, dim3(grid_for(items)), dim3(256), 0, s, x, b,
                         n0, kp, x_amax, out);
    else
      hipLaunchKernelGGL(quantize_packed_kernel<2>, dim3(grid_for(items)), dim3(256), 0, s, x, b,
                         n0, kp, x_amax, out);
  } else {
    const int64_t n = (int64_t)b * n0;
    if (dt == 1)
      hipLaunchKernelGGL(quantize_values_kernel<1>, dim3(grid_for(n)), dim3(256), 0, s, x, n,
                         x_amax, (float*)out);
    else
      hipLaunchKernelGGL(quantize_values_kernel<2>, dim3(grid_for(n)), dim3(256), 0, s, x, n,
                         x_amax, (float*)out);
  }
  return hipGetLastError();
}

// Batch in bfloat16, chunk-major for the large-batch kernel that reads W_1
// from its bfloat16 copy: slot it (8 elements) = chunk it / (4 bpad), row
// (it / 4) mod bpad, elements 8 (it mod 4) .. + 7 of the chunk; rows at or
// past b and k at or past n0 are zero.
__global__ __launch_bounds__(256) void quantize_chunks_kernel(const float* __restrict__ x, int b,
                                                              int n0, int bpad, int64_t items,
                                                              uint4* __restrict__ out) {
  for (int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * 256) {
    const int64_t rs = it >> 2;
    const int ch = (int)(rs / bpad);
    const int m = (int)(rs - (int64_t)ch * bpad);
    const int k = ch * 32 + 8 * (int)(it & 3);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (m < b && k + e < n0) ? x[(int64_t)m * n0 + k + e] : 0.0f;
    uint4 o;
    o.x = pack_bf16x2(v[0], v[1]);
    o.y = pack_bf16x2(v[2], v[3]);
    o.z = pack_bf16x2(v[4], v[5]);
    o.w = pack_bf16x2(v[6], v[7]);
    out[it] = o;
  }
}

hipError_t launch_quantize_x_chunks(const float* x, int b, int n0, int kp, int bpad,
                                    uint16_t* xq, hipStream_t s) {
  const int64_t items = (int64_t)(kp >> 5) * bpad * 4;
  hipLaunchKernelGGL(quantize_chunks_kernel, dim3(grid_for(items)), dim3(256), 0, s, x, b, n0,
                     bpad, items, reinterpret_cast<uint4*>(xq));
  return hipGetLastError();
}

// Batch in FP8 E4M3 (scaled by 2^-e_x, e_x from *x_amax), chunk-major for the
// large-batch kernel that reads the FP8 copy of W_1: slot it (16 elements) =
// chunk it / (4 bpad), row (it / 4) mod bpad, elements 16 (it mod 4) .. + 15
// of the 64-element chunk; rows at or past b and k at or past n0 are zero.
__global__ __launch_bounds__(256) void quantize_chunks8_kernel(const float* __restrict__ x, int b,
                                                               int n0, int bpad, int64_t items,
                                                               const uint32_t* __restrict__ x_amax,
                                                               uint4* __restrict__ out) {
  const uint32_t am = *x_amax;
  const int neg_e = am < kNonFinite ? -fp8_exponent(am) : 0;
  for (int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * 256) {
    const int64_t rs = it >> 2;
    const int ch = (int)(rs / bpad);
    const int m = (int)(rs - (int64_t)ch * bpad);
    const int k = ch * 64 + 16 * (int)(it & 3);
    float v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e)
      v[e] = (m < b && k + e < n0) ? ldexpf(x[(int64_t)m * n0 + k + e], neg_e) : 0.0f;
    uint4 o;
    o.x = pack_fp8x4(v[0], v[1], v[2], v[3]);
    o.y = pack_fp8x4(v[4], v[5], v[6], v[7]);
    o.z = pack_fp8x4(v[8], v[9], v[10], v[11]);
    o.w = pack_fp8x4(v[12], v[13], v[14], v[15]);
    out[it] = o;
  }
}

hipError_t launch_quantize_x_chunks8(const float* x, int b, int n0, int kp8, int bpad,
                                     const uint32_t* x_amax, uint8_t* xq, hipStream_t s) {
  const int64_t items = (int64_t)(kp8 >> 6) * bpad * 4;
  hipLaunchKernelGGL(quantize_chunks8_kernel, dim3(grid_for(items)), dim3(256), 0, s, x, b, n0,
                     bpad, items, x_amax, reinterpret_cast<uint4*>(xq));
  return hipGetLastError();
}

// The bfloat16 W_1 copy rebuilt from the genomes (after initialisation or a
// population replaced from outside): slot it of network blockIdx.y = row
// it / (kp / 8), elements 8 (it mod (kp / 8)) .. + 7.
__global__ __launch_bounds__(256) void shadow_w1_kernel(const float* __restrict__ genomes,
                                                        NetDesc nd, W1Shadow wsh,
                                                        int64_t items) {
  const int j = blockIdx.y;
  const int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (it >= items) return;
  const float* __restrict__ W1 = genomes + (int64_t)j * nd.stride + nd.woff[0];
  const int n0 = nd.w[0], n1 = nd.w[1];
  const int per_row = wsh.kp >> 3;
  const int n = (int)(it / per_row);
  const int k = (int)(it - (int64_t)n * per_row) * 8;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (n < n1 && k + e < n0) ? W1[(int64_t)n * n0 + k + e] : 0.0f;
  uint4 o;
  o.x = pack_bf16x2(v[0], v[1]);
  o.y = pack_bf16x2(v[2], v[3]);
  o.z = pack_bf16x2(v[4], v[5]);
  o.w = pack_bf16x2(v[6], v[7]);
  reinterpret_cast<uint4*>(wsh.p + (int64_t)j * wsh.net)[it] = o;
}

hipError_t launch_shadow_w1(const float* genomes, const NetDesc& nd, int pop,
                            const W1Shadow& wsh, hipStream_t s) {
  const int64_t items = wsh.net / 8;
  dim3 grid((unsigned)((items + 255) / 256), (unsigned)pop);
  hipLaunchKernelGGL(shadow_w1_kernel, grid, dim3(256), 0, s, genomes, nd, wsh, items);
  return hipGetLastError();
}

// The FP8 copy of W_1 rebuilt from the genomes (after initialisation, a
// restore or a surrogate step): slot it of network blockIdx.y = row
// it / (kp / 8), elements 8 (it mod (kp / 8)) .. + 7, each scaled by 2^-e_j
// (e_j from bound[j]) and rounded to E4M3; padding zero.  A network whose
// bound is not finite gets zeros (its fitness is NaN through the scale).
__global__ __launch_bounds__(256) void fp8_copy_kernel(const float* __restrict__ genomes,
                                                       NetDesc nd, W1Fp8 w8, int64_t items) {
  const int j = blockIdx.y;
  const int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (it >= items) return;
  const float* __restrict__ W1 = genomes + (int64_t)j * nd.stride + nd.woff[0];
  const int n0 = nd.w[0], n1 = nd.w[1];
  const uint32_t bnd = w8.bound[j];
  const bool fin = bnd < kNonFinite;
  const int neg_e = fin ? -fp8_exponent(bnd) : 0;
  const int per_row = w8.kp >> 3;
  const int n = (int)(it / per_row);
  const int k = (int)(it - (int64_t)n * per_row) * 8;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e)
    v[e] = (fin && n < n1 && k + e < n0) ? ldexpf(W1[(int64_t)n * n0 + k + e], neg_e) : 0.0f;
  uint2 o;
  o.x = pack_fp8x4(v[0], v[1], v[2], v[3]);
  o.y = pack_fp8x4(v[4], v[5], v[6], v[7]);
  reinterpret_cast<uint2*>(w8.p + (int64_t)j * w8.net)[it] = o;
}

hipError_t launch_fp8_copy(const float* genomes, const NetDesc& nd, int pop, const W1Fp8& w8,
                           hipStream_t s) {
  const int64_t items = w8.net / 8;
  dim3 grid((unsigned)((items + 255) / 256), (unsigned)pop);
  hipLaunchKernelGGL(fp8_copy_kernel, grid, dim3(256), 0, s, genomes, nd, w8, items);
  return hipGetLastError();
}

// Quantised batch of every bfloat16 run: values [b][n0] for the small-batch
// kernel (b <= 16), packed [b][kp] otherwise; 256 items per workgroup.
__global__ __launch_bounds__(256) void runs_quantize_kernel(const RunDesc* __restrict__ runs,
                                                            const int* __restrict__ off,
                                                            const int* __restrict__ ids, int n) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  const int64_t it = (int64_t)(blockIdx.x - off[i]) * 256 + threadIdx.x;
  const int n0 = d.nd.w[0];
  if (d.ekind == 0) {
    if (it < (int64_t)d.b * n0) reinterpret_cast<float*>(d.xq)[it] = round_bf16(d.xb[it]);
    return;
  }
  const int per_row = d.kp >> 3;
  if (it >= (int64_t)d.b * per_row) return;
  const int m = (int)(it / per_row);
  const int k = (int)(it - (int64_t)m * per_row) * 8;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = k + e < n0 ? d.xb[(int64_t)m * n0 + k + e] : 0.0f;
  uint4 o;
  o.x = pack_bf16x2(v[0], v[1]);
  o.y = pack_bf16x2(v[2], v[3]);
  o.z = pack_bf16x2(v[4], v[5]);
  o.w = pack_bf16x2(v[6], v[7]);
  reinterpret_cast<uint4*>(d.xq)[it] = o;
}

hipError_t launch_runs_quantize(const RunDesc* runs, const Group& g, hipStream_t s) {
  hipLaunchKernelGGL(runs_quantize_kernel, dim3((unsigned)g.blocks), dim3(256), 0, s, runs, g.off,
                     g.ids, g.n);
  return hipGetLastError();
}

}  // namespace leea
