// Device helpers of the reduced-precision first layer: bfloat16 and OCP FP8
// E4M3 rounding (round to nearest, ties to even, by the gfx950 conversion
// instructions) and the power-of-two FP8 scales.  The scale exponent of an
// operand with largest magnitude amax is the smallest integer e with
// amax <= 448 * 2^e (448 = largest finite E4M3 value); a non-finite amax
// marks the operand as unusable (the fitness it feeds becomes NaN).
#pragma once

#include "internal.hpp"

namespace leea {

constexpr uint32_t kNonFinite = 0x7F800000u;  // |x| bits at or above: inf or NaN

// Magnitude bits of a float: ordered like the magnitudes for finite values,
// above kNonFinite - 1 for infinities and NaNs, so an unsigned max over them
// is the largest magnitude and flags any non-finite value.
__device__ __forceinline__ uint32_t mag_bits(float v) { return __float_as_uint(v) & 0x7FFFFFFFu; }

// Largest of v over the wave.
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = (uint32_t)__shfl_xor((int)v, off);
    v = o > v ? o : v;
  }
  return v;
}

// e for a finite non-negative amax (0 for amax = 0): with amax = m * 2^k,
// m in [0.5, 1), 448 * 2^(k-9) = 0.875 * 2^k covers amax iff m <= 0.875.
__device__ __forceinline__ int fp8_exponent(uint32_t amax_bits) {
  const float a = __uint_as_float(amax_bits);
  if (a == 0.0f) return 0;
  int k;
  const float m = frexpf(a, &k);
  return m <= 0.875f ? k - 9 : k - 8;
}

// 2^(e_x + e_w) for the product of two scaled operands, NaN if either
// operand is not finite.
__device__ __forceinline__ float fp8_factor(uint32_t ax_bits, uint32_t aw_bits) {
  if (ax_bits >= kNonFinite || aw_bits >= kNonFinite) return __builtin_nanf("");
  return ldexpf(1.0f, fp8_exponent(ax_bits) + fp8_exponent(aw_bits));
}

__device__ __forceinline__ float round_bf16(float v) {
  const __bf16 h = (__bf16)v;
  return (float)h;
}

typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// Two floats -> two bfloat16 in one dword (first in the low half); one
// v_cvt_pk_bf16_f32 (round to nearest even, like the scalar conversion).
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  const float2v v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}

// Four floats (already divided by their scale, |v| <= 448) -> four E4M3
// codes in one dword (first in the low byte).
__device__ __forceinline__ uint32_t pack_fp8x4(float a, float b, float c, float d) {
  int p = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  p = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, p, true);
  return (uint32_t)p;
}

// The E4M3 value nearest to v (|v| <= 448), as a float.
__device__ __forceinline__ float round_fp8(float v) {
  const int p = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false);
  return __builtin_amdgcn_cvt_f32_fp8(p, 0);
}

// Quantised value of a weight or input element in the given mode:
// BF16 -> nearest bfloat16; FP8 -> nearest E4M3 of v * 2^-e (still scaled).
template <int DT>
__device__ __forceinline__ float quantize(float v, int neg_e) {
  if constexpr (DT == 1) return round_bf16(v);
  else if constexpr (DT == 2) return round_fp8(ldexpf(v, neg_e));
  else return v;
}

// Largest magnitude bits of n floats at W (global memory or LDS) over the
// workgroup; every thread of the workgroup (a multiple of 64 threads, at most
// 1024) calls it, with the same arguments.
__device__ __forceinline__ uint32_t block_amax(const float* W, int n) {
  __shared__ uint32_t red[16];
  uint32_t m = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t v = mag_bits(W[i]);
    m = v > m ? v : m;
  }
  m = wave_umax(m);
  __syncthreads();  // red is free (an earlier call's readers are done)
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  uint32_t r = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = red[w] > r ? red[w] : r;
  return r;
}

// Largest magnitude bits of a network's later layers (entry l for W_l,
// l >= 1), read once at the start of an evaluation kernel so that the tail
// does not wait on them; given = 0: the tail reduces each layer itself.
struct TailScales {
  uint32_t amax[kMaxLayers];
  int given;
};

__device__ __forceinline__ TailScales load_tail_scales(const uint32_t* p, int L) {
  TailScales t;
  t.given = p != nullptr;
#pragma unroll
  for (int l = 0; l < kMaxLayers; ++l) t.amax[l] = (p && l >= 1 && l < L) ? p[l] : 0u;
  return t;
}

// Scale of a later layer's FP8 weights from their largest magnitude bits:
// neg_e = -e for quantize<2>, fac = 2^e multiplies the layer's sums; a
// non-finite weight gives fac = NaN (the network's fitness becomes NaN).
__device__ __forceinline__ void tail_fp8_scale(uint32_t amax, int& neg_e, float& fac) {
  if (amax >= kNonFinite) {
    neg_e = 0;
    fac = __builtin_nanf("");
  } else {
    const int e = fp8_exponent(amax);
    neg_e = -e;
    fac = ldexpf(1.0f, e);
  }
}

}  // namespace leea
