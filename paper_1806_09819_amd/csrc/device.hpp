// Device-side building blocks shared by the LEEA kernels (gfx950).
//
// * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
//   32x32->64-bit products with key bumps by the Weyl constants.
// * A float32 Box-Muller normal sampler whose every operation is a correctly
//   rounded IEEE float32 +, -, *, / or sqrt in a fixed order with contraction
//   disabled, so it is reproducible bit for bit on any IEEE machine:
//     ln:  exact exponent/mantissa split (m in (sqrt(1/2), sqrt(2)]),
//          s = (m-1)/(m+1), ln m = 2 atanh s by its odd series to s^11,
//          ln u = e*ln2_hi + (e*ln2_lo + ln m) with a 16-bit ln2_hi.
//     sin/cos: Taylor series to x^11 / x^12 on [0, pi/4]; the angle
//          (q + f) * pi/2 is reduced by quarter turns and by f -> 1 - f.
//   Every coefficient is the float32 nearest to the exact value, written as
//   an exactly representable integer ratio the compiler folds in float32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace leea {

// Philox counter purposes (low byte of the last counter word).
enum : uint32_t {
  kInit = 0, kSel = 1, kXo = 2, kMutMask = 3, kMutNorm = 4, kSigma = 5, kBatch = 6
};

enum : int { kOpElite = 0, kOpCross = 1, kOpMut = 2 };

constexpr int kMaxLayers = 8;
constexpr int kMaxWidth = 256;

// Shape of one directly encoded network and where each layer lives in the
// genome (gene offsets; W_l is [w[l]][w[l-1]] row-major, then b_l).
struct NetDesc {
  int L;
  int w[kMaxLayers + 1];
  int64_t woff[kMaxLayers];
  int64_t boff[kMaxLayers];
  int64_t genes;
  int64_t stride;
};

struct Key {
  uint32_t k0, k1, run;
};

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Four words for (purpose, generation, slot, block) under key.
__device__ __forceinline__ uint4 draw(const Key& key, uint32_t purpose, uint32_t gen,
                                      uint32_t slot, uint32_t block) {
  return philox(block, slot, gen, (key.run << 8) | purpose, key.k0, key.k1);
}

__device__ __forceinline__ uint32_t word_of(const uint4& w, int i) {
  return i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w;
}

// ------------------------------------------------------------ sampler ----

__device__ __forceinline__ float ln32(float u) {
#pragma clang fp contract(off)
  const uint32_t bits = __float_as_uint(u);
  int e = (int)(bits >> 23) - 127;
  float m = __uint_as_float((bits & 0x7FFFFFu) | 0x3F800000u);
  if (m > 1.41421356237309504880f) {  // nearest float32 to sqrt(2)
    m = m * 0.5f;
    e = e + 1;
  }
  const float f = m - 1.0f;
  const float t = m + 1.0f;
  const float s = f / t;
  const float z = s * s;
  float p = 1.0f / 11.0f;
  p = p * z;
  p = p + 1.0f / 9.0f;
  p = p * z;
  p = p + 1.0f / 7.0f;
  p = p * z;
  p = p + 1.0f / 5.0f;
  p = p * z;
  p = p + 1.0f / 3.0f;
  const float sz = s * z;
  const float szp = sz * p;
  const float h = s + szp;
  const float lnm = 2.0f * h;
  const float ef = (float)e;
  // ln 2 = ln2_hi + ln2_lo; ln2_hi = 45426 / 65536 has 16 significant bits
  const float hi = ef * (45426.0f / 65536.0f);
  float lo = ef * 1.42860682030941723212e-6f;
  lo = lo + lnm;
  return hi + lo;
}

// sin and cos of x in [0, pi/4]
__device__ __forceinline__ void sincos_quarter(float x, float& s, float& c) {
#pragma clang fp contract(off)
  const float z = x * x;
  float ps = -1.0f / 39916800.0f;  // -1/11!
  ps = ps * z;
  ps = ps + 1.0f / 362880.0f;      // 1/9!
  ps = ps * z;
  ps = ps + -1.0f / 5040.0f;       // -1/7!
  ps = ps * z;
  ps = ps + 1.0f / 120.0f;         // 1/5!
  ps = ps * z;
  ps = ps + -1.0f / 6.0f;          // -1/3!
  const float xz = x * z;
  const float sp = xz * ps;
  s = x + sp;
  float pc = 1.0f / 479001600.0f;  // 1/12!
  pc = pc * z;
  pc = pc + -1.0f / 3628800.0f;    // -1/10!
  pc = pc * z;
  pc = pc + 1.0f / 40320.0f;       // 1/8!
  pc = pc * z;
  pc = pc + -1.0f / 720.0f;        // -1/6!
  pc = pc * z;
  pc = pc + 1.0f / 24.0f;          // 1/4!
  pc = pc * z;
  pc = pc + -0.5f;                 // -1/2!
  const float zp = z * pc;
  c = 1.0f + zp;
}

// Two standard normals from words a (radius) and b (angle).
__device__ __forceinline__ void normal_pair(uint32_t a, uint32_t b, float& z0, float& z1) {
#pragma clang fp contract(off)
  const float u1 = (float)((a >> 8) + 1u) * 5.9604644775390625e-8f;  // * 2^-24
  const float lg = ln32(u1);
  const float r2 = -2.0f * lg;
  const float r = __builtin_sqrtf(r2);
  const uint32_t q = b >> 30;
  const uint32_t fi = (b >> 6) & 0xFFFFFFu;
  const float f = (float)fi * 5.9604644775390625e-8f;
  const bool swap = fi >= (1u << 23);
  const float g = swap ? 1.0f - f : f;
  const float x = g * 1.57079632679489661923f;  // nearest float32 to pi/2
  float s0, c0;
  sincos_quarter(x, s0, c0);
  const float s = swap ? c0 : s0;
  const float c = swap ? s0 : c0;
  // Rotate by q quarter turns: (cos, sin) -> (c, s), (-s, c), (-c, -s),
  // (s, -c) for q = 0..3.  Written without branches (odd q swaps; the sign
  // bits are XORed in, which is exactly IEEE negation): a four-way branch
  // here was compiled into divergent control flow that left the sine of
  // q = 3 lanes unset inside the variation kernel.
  const bool odd = (q & 1u) != 0u;
  const float u = odd ? s : c;
  const float v = odd ? c : s;
  const uint32_t sign_c = ((q + 1u) & 2u) << 30;  // q = 1, 2
  const uint32_t sign_s = (q & 2u) << 30;         // q = 2, 3
  const float cq = __uint_as_float(__float_as_uint(u) ^ sign_c);
  const float sq = __uint_as_float(__float_as_uint(v) ^ sign_s);
  z0 = r * cq;
  z1 = r * sq;
}

__device__ __forceinline__ float4 normals4(uint4 w) {
  float4 z;
  normal_pair(w.x, w.y, z.x, z.y);
  normal_pair(w.z, w.w, z.z, z.w);
  return z;
}

// e^x for |x| <= 80: n = rint(x / ln 2), r = (x - n*ln2_hi) - n*ln2_lo,
// Taylor series of e^r to r^7, exact scaling by 2^n from the exponent bits.
__device__ __forceinline__ float exp32(float x) {
#pragma clang fp contract(off)
  const float t = x * 1.44269504088896340736f;  // nearest float32 to 1/ln 2
  const float n = __builtin_rintf(t);
  const float hi = n * (45426.0f / 65536.0f);
  float r = x - hi;
  const float lo = n * 1.42860682030941723212e-6f;
  r = r - lo;
  float p = 1.0f / 5040.0f;
  p = p * r;
  p = p + 1.0f / 720.0f;
  p = p * r;
  p = p + 1.0f / 120.0f;
  p = p * r;
  p = p + 1.0f / 24.0f;
  p = p * r;
  p = p + 1.0f / 6.0f;
  p = p * r;
  p = p + 0.5f;
  p = p * r;
  p = p + 1.0f;
  p = p * r;
  p = p + 1.0f;
  const float scale = __uint_as_float((uint32_t)((int)n + 127) << 23);
  return p * scale;
}

__device__ __forceinline__ float f4get(const float4& v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

}  // namespace leea
