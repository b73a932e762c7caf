// Device pieces of the genetic operators (paper section 3.2) shared by the
// variation kernel (genetic.hip) and the fused variation + evaluation kernel
// (fused.hip), so both produce bit-identical children:
// * the child's sigma gene under self-adaptation,
// * uniform crossover of one float4 (the coin of gene i is bit 4(t mod 8)+e
//   of word t/8 of Philox block (XO, gen, slot, 64G + q), i = 8192G + 256t +
//   4q + e),
// * arithmetic crossover fl(fl(a + b) * 0.5),
// * Gaussian mutation fl(a + fl(sigma * z)) of the genes whose MUTMASK word
//   is below the threshold, z from block (MUTNORM, gen, slot, i >> 2).
#pragma once

#include "device.hpp"

namespace leea {

typedef float floatv4 __attribute__((ext_vector_type(4)));

// Children are written with non-temporal stores: the evaluation streams them
// back once, and dirty lines left in L2 / the memory-side cache would
// otherwise be written back while it reads, halving its read bandwidth.
__device__ __forceinline__ void store_stream(float4* p, const float4& v) {
  floatv4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<floatv4*>(p));
}

struct VaryParams {
  float sigma;     // mutation strength of this child
  bool all;        // every gene mutates (threshold 2^32)
  uint32_t t32;    // per-gene threshold otherwise
  Key key;
  uint32_t gen;
  uint32_t slot;
  int64_t genes;   // genes at or beyond this index are padding
};

// Sigma gene of the child in slot j under self-adaptive control.
__device__ __forceinline__ float child_sigma(const int4& pl, const float* __restrict__ sig_cur,
                                             const Key& key, uint32_t gen, uint32_t j,
                                             float tau) {
#pragma clang fp contract(off)
  if (pl.x == kOpElite) return sig_cur[pl.y];
  if (pl.x == kOpCross) {
    const float sum = sig_cur[pl.y] + sig_cur[pl.z];
    return sum * 0.5f;
  }
  const uint4 w = draw(key, kSigma, gen, j, 0u);
  float z0, z1;
  normal_pair(w.x, w.y, z0, z1);
  const float t = tau * z0;
  return sig_cur[pl.y] * exp32(t);
}

// Uniform crossover of the float4 holding genes i0 .. i0+3 (i0 % 4 == 0).
__device__ __forceinline__ float4 xo_uniform4(const VaryParams& v, int64_t i0, const float4& a,
                                              const float4& b) {
  const uint32_t G = (uint32_t)(i0 >> 13);
  const int t = (int)((i0 >> 8) & 31);
  const uint32_t q = (uint32_t)((i0 >> 2) & 63);
  const uint4 w = draw(v.key, kXo, v.gen, v.slot, G * 64u + q);
  const uint32_t bits = word_of(w, t >> 3) >> (4 * (t & 7));
  float4 o;
  o.x = (bits & 1u) ? b.x : a.x;
  o.y = (bits & 2u) ? b.y : a.y;
  o.z = (bits & 4u) ? b.z : a.z;
  o.w = (bits & 8u) ? b.w : a.w;
  return o;
}

__device__ __forceinline__ float4 xo_arith4(const float4& a, const float4& b) {
#pragma clang fp contract(off)
  float4 o;
  o.x = (a.x + b.x) * 0.5f;
  o.y = (a.y + b.y) * 0.5f;
  o.z = (a.z + b.z) * 0.5f;
  o.w = (a.w + b.w) * 0.5f;
  return o;
}

// Gaussian mutation of the float4 with index f (genes 4f .. 4f+3).  Padding
// genes (index >= genes) keep their value; they run through the same
// branch-free code so loads can be batched across loop iterations.
__device__ __forceinline__ float4 mutate4(const VaryParams& v, int64_t f, const float4& a) {
#pragma clang fp contract(off)
  const int64_t i0 = 4 * f;
  const float4 z = normals4(draw(v.key, kMutNorm, v.gen, v.slot, (uint32_t)f));
  uint4 mw = make_uint4(0u, 0u, 0u, 0u);
  if (!v.all) mw = draw(v.key, kMutMask, v.gen, v.slot, (uint32_t)f);
  const bool m0 = (v.all || mw.x < v.t32) && i0 + 0 < v.genes;
  const bool m1 = (v.all || mw.y < v.t32) && i0 + 1 < v.genes;
  const bool m2 = (v.all || mw.z < v.t32) && i0 + 2 < v.genes;
  const bool m3 = (v.all || mw.w < v.t32) && i0 + 3 < v.genes;
  const float n0 = v.sigma * z.x;
  const float n1 = v.sigma * z.y;
  const float n2 = v.sigma * z.z;
  const float n3 = v.sigma * z.w;
  float4 o;
  o.x = m0 ? a.x + n0 : a.x;
  o.y = m1 ? a.y + n1 : a.y;
  o.z = m2 ? a.z + n2 : a.z;
  o.w = m3 ? a.w + n3 : a.w;
  return o;
}

}  // namespace leea
