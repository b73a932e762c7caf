// Population initialisation, variation (elites / crossover / mutation) and
// minibatch draw.  All three are HBM-streaming kernels: float4 accesses,
// whole 1 KiB wave-wide segments, and one Philox call per lane per
// 4 (mutation) or 128 (uniform crossover) genes.
#include "internal.hpp"
#include "lowp.hpp"
#include "runs.hpp"
#include "vary_common.hpp"

namespace leea {

// Glorot-uniform weights, zero biases and padding (Algorithm 1, first line;
// section 4.1).  Thread = 4 consecutive genes = one Philox block.
__global__ __launch_bounds__(256) void init_kernel(float* __restrict__ genomes, NetDesc nd,
                                                   Glorot ga, Key key) {
#pragma clang fp contract(off)
  const int j = blockIdx.y;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n4 = nd.stride >> 2;
  if (q >= n4) return;
  const uint4 w = draw(key, kInit, 0, (uint32_t)j, (uint32_t)q);
  float v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = 4 * q + e;
    v[e] = 0.0f;
    for (int l = 0; l < nd.L; ++l) {
      const int64_t w0 = nd.woff[l];
      const int64_t w1 = w0 + (int64_t)nd.w[l + 1] * nd.w[l];
      if (i >= w0 && i < w1) {
        const float u = (float)(word_of(w, e) >> 8) * 5.9604644775390625e-8f;
        float t = 2.0f * u;
        t = t - 1.0f;
        v[e] = t * ga.a[l];
      }
    }
  }
  reinterpret_cast<float4*>(genomes + (int64_t)j * nd.stride)[q] =
      make_float4(v[0], v[1], v[2], v[3]);
}

hipError_t launch_init(float* genomes, const NetDesc& nd, const Glorot& ga, int pop,
                       const Key& key, hipStream_t s) {
  const int64_t n4 = nd.stride >> 2;
  dim3 grid((unsigned)((n4 + 255) / 256), (unsigned)pop);
  hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, s, genomes, nd, ga, key);
  return hipGetLastError();
}

// One wave handles an 8192-gene group G: lane q, step t (0..31) touches the
// float4 at gene 8192 G + 256 t + 4 q, so every step is one contiguous
// 1 KiB access per parent.  Uniform crossover: the lane's 32 steps x 4
// genes use the 128 bits of Philox block (XO, gen, slot, 64 G + q): word
// t/8, bit 4 (t mod 8) + element.  Mutation: the float4 at gene 4f uses
// block f of MUTNORM (four normals) and, when not every gene mutates, block
// f of MUTMASK (four decisions).  Padding genes stay zero.
// Workgroups are dispatched in blockIdx order; slot j = (y * mul) mod pop
// (mul coprime to pop) interleaves the compute-heavy mutation children with
// the bandwidth-bound elites and crossover children instead of running them
// all at the end.
// Self-adaptive mutation strength (sig_cur != NULL): every individual
// carries a sigma gene.  Elites keep theirs, crossover children take the
// parents' mean, mutants take sigma * exp(tau * z) with z the first normal
// of block (SIGMA, gen, slot, 0), and are then mutated with that new sigma.
// Every workgroup of a slot computes the same value; the first writes it.
// kAmax: also accumulate the largest magnitude of each child's W_1 (genes
// [0, w1n), whole float4s since n0 % 4 == 0) into amax[j] (cleared
// beforehand), the FP8 scale of the next evaluation.
// Body of one workgroup: slot j, gene groups 4 gx .. 4 gx + 3 (one per wave).
// The random draws of slot j come from slot j + slot_off of the streams.
// kNorm: also write, per wave, the sum of squared differences between the
// child and parent 1 over the wave's genes to nu[j * ngroups + G].
// kShadow: also write the child's W_1 rounded to bfloat16 into its W1Shadow
// slot (n0 % 4 == 0: a float4 of W_1 is 4 consecutive k of one row, one
// 8-byte store; a wave's stores are contiguous within each row).
// kFp8: also write the child's W_1 into its FP8 copy, scaled by 2^-e with e
// from the child's bound (from its parents' largest magnitudes), which the
// first workgroup of the child stores.
__device__ __forceinline__ uint32_t fp8_child_bound(const int4& pl, const uint32_t* amax,
                                                    float sigma) {
#pragma clang fp contract(off)
  const uint32_t a1 = amax[pl.y];
  if (pl.x == kOpElite) return a1;
  if (pl.x == kOpCross) {
    const uint32_t a2 = amax[pl.z];
    return a1 > a2 ? a1 : a2;  // magnitude bits: NaN above inf above every number
  }
  const float t = __uint_as_float(a1) * (1.0f + 0x1p-20f);
  const float m = 6.0f * sigma;
  return mag_bits(t + m);
}

template <int kXoKind, bool kAmax, bool kNorm = false, bool kShadow = false, bool kFp8 = false>
__device__ __forceinline__ void vary_body(int j, int gx, const float* __restrict__ cur,
                                          float* __restrict__ nxt, const int4* __restrict__ plan,
                                          int64_t stride, int64_t genes, float sigma,
                                          uint64_t thr, Key key, uint32_t gen,
                                          const float* __restrict__ sig_cur,
                                          float* __restrict__ sig_next, float tau,
                                          uint32_t* __restrict__ amax, int64_t w1n,
                                          uint32_t slot_off = 0, float* __restrict__ nu = nullptr,
                                          int ngroups = 0, W1Shadow wsh = W1Shadow{},
                                          W1Fp8 w8 = W1Fp8{}) {
#pragma clang fp contract(off)
  const uint32_t pslot = (uint32_t)j + slot_off;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t G = (int64_t)gx * 4 + wave;
  const int64_t n4 = stride >> 2;
  const int64_t base4 = G * 2048 + lane;
  const int4 pl = plan[j];
  if (sig_cur) {
    sigma = child_sigma(pl, sig_cur, key, gen, pslot, tau);
    if (gx == 0 && threadIdx.x == 0) sig_next[j] = sigma;
  }
  int neg_e8 = 0;
  if (kFp8) {
    const uint32_t bnd = fp8_child_bound(pl, w8.amax_par, sigma);
    if (gx == 0 && threadIdx.x == 0) w8.bound[j] = bnd;
    neg_e8 = bnd < kNonFinite ? -fp8_exponent(bnd) : 0;
  }
  if (G * 2048 >= n4) return;
  const float4* __restrict__ a4 = reinterpret_cast<const float4*>(cur + (int64_t)pl.y * stride);
  const float4* __restrict__ b4 = reinterpret_cast<const float4*>(cur + (int64_t)pl.z * stride);
  float4* __restrict__ d4 = reinterpret_cast<float4*>(nxt + (int64_t)j * stride);
  const int64_t w1f = w1n >> 2;
  uint32_t am = 0;
  float sq = 0.0f;
  auto dist = [&](const float4& o, const float4& a) {
    if (kNorm) {
      const float dx = o.x - a.x, dy = o.y - a.y, dz = o.z - a.z, dw = o.w - a.w;
      sq += dx * dx;
      sq += dy * dy;
      sq += dz * dz;
      sq += dw * dw;
    }
  };
  uint16_t* __restrict__ sh = kShadow ? wsh.p + (int64_t)j * wsh.net : nullptr;
  uint8_t* __restrict__ s8 = (kFp8 && w8.p) ? w8.p + (int64_t)j * w8.net : nullptr;
  auto track = [&](int64_t f, const float4& o) {
    if (kFp8 && s8 && f < w1f) {
      const int g = (int)(4 * f);
      int n = (int)((float)g * w8.rcp_n0);  // g < 2^24: off by at most one
      int k = g - n * w8.n0;
      if (k < 0) {
        n -= 1;
        k += w8.n0;
      } else if (k >= w8.n0) {
        n += 1;
        k -= w8.n0;
      }
      const uint32_t q = pack_fp8x4(ldexpf(o.x, neg_e8), ldexpf(o.y, neg_e8),
                                    ldexpf(o.z, neg_e8), ldexpf(o.w, neg_e8));
      __builtin_nontemporal_store(q, reinterpret_cast<uint32_t*>(s8 + (int64_t)n * w8.kp + k));
    }
    if (kShadow && f < w1f) {
      const int g = (int)(4 * f);
      int n = (int)((float)g * wsh.rcp_n0);  // g < 2^24: off by at most one
      int k = g - n * wsh.n0;
      if (k < 0) {
        n -= 1;
        k += wsh.n0;
      } else if (k >= wsh.n0) {
        n += 1;
        k -= wsh.n0;
      }
      typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
      const u32x2 v = {pack_bf16x2(o.x, o.y), pack_bf16x2(o.z, o.w)};
      // non-temporal like the children themselves: the evaluation reads the
      // copy once, after this whole kernel
      __builtin_nontemporal_store(v, reinterpret_cast<u32x2*>(sh + (int64_t)n * wsh.kp + k));
    }
    if (kAmax && f < w1f) {
      uint32_t a = mag_bits(o.x), b = mag_bits(o.y), c = mag_bits(o.z), d = mag_bits(o.w);
      a = a > b ? a : b;
      c = c > d ? c : d;
      a = a > c ? a : c;
      am = a > am ? a : am;
    }
  };

  if (pl.x == kOpElite) {
#pragma unroll 8
    for (int t = 0; t < 32; ++t) {
      const int64_t f = base4 + 64 * t;
      if (f < n4) {
        const float4 a = a4[f];
        track(f, a);
        store_stream(d4 + f, a);
      }
    }
  } else if (pl.x == kOpCross) {
    if (kXoKind == 0) {
      const uint4 m = draw(key, kXo, gen, pslot, (uint32_t)(G * 64 + lane));
#pragma unroll 8
      for (int t = 0; t < 32; ++t) {
        const int64_t f = base4 + 64 * t;
        if (f < n4) {
          const float4 a = a4[f];
          const float4 b = b4[f];
          const uint32_t bits = word_of(m, t >> 3) >> (4 * (t & 7));
          float4 o;
          o.x = (bits & 1u) ? b.x : a.x;
          o.y = (bits & 2u) ? b.y : a.y;
          o.z = (bits & 4u) ? b.z : a.z;
          o.w = (bits & 8u) ? b.w : a.w;
          track(f, o);
          dist(o, a);
          store_stream(d4 + f, o);
        }
      }
    } else {
#pragma unroll 8
      for (int t = 0; t < 32; ++t) {
        const int64_t f = base4 + 64 * t;
        if (f < n4) {
          const float4 a = a4[f];
          const float4 b = b4[f];
          const float4 o = xo_arith4(a, b);
          track(f, o);
          dist(o, a);
          store_stream(d4 + f, o);
        }
      }
    }
  } else {
    VaryParams vp;
    vp.sigma = sigma;
    vp.all = thr >= (1ull << 32);
    vp.t32 = (uint32_t)thr;
    vp.key = key;
    vp.gen = gen;
    vp.slot = pslot;
    vp.genes = genes;
#pragma unroll 4
    for (int t = 0; t < 32; ++t) {
      const int64_t f = base4 + 64 * t;
      if (f < n4) {
        const float4 a = a4[f];
        if (4 * f >= genes) {  // padding only: skip the draws
          store_stream(d4 + f, a);
          continue;
        }
        const float4 o = mutate4(vp, f, a);
        track(f, o);
        dist(o, a);
        store_stream(d4 + f, o);
      }
    }
  }
  if (kNorm) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (lane == 0) nu[(int64_t)j * ngroups + G] = sq;
  }
  if (kAmax && G * 2048 < w1f) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o = (uint32_t)__shfl_xor((int)am, off);
      am = o > am ? o : am;
    }
    if (lane == 0 && am) atomicMax(amax + j, am);
  }
}

template <int kXoKind, bool kAmax, bool kShadow, bool kFp8>
__global__ __launch_bounds__(256) void vary_kernel(const float* __restrict__ cur,
                                                   float* __restrict__ nxt,
                                                   const int4* __restrict__ plan,
                                                   int64_t stride, int64_t genes, float sigma,
                                                   uint64_t thr, Key key, uint32_t gen, int pop,
                                                   uint32_t mul, const float* __restrict__ sig_cur,
                                                   float* __restrict__ sig_next, float tau,
                                                   uint32_t* __restrict__ amax, int64_t w1n,
                                                   W1Shadow wsh, W1Fp8 w8) {
  const int j = (int)(((uint64_t)blockIdx.y * mul) % (uint32_t)pop);
  vary_body<kXoKind, kAmax, false, kShadow, kFp8>(j, blockIdx.x, cur, nxt, plan, stride, genes,
                                                  sigma, thr, key, gen, sig_cur, sig_next, tau,
                                                  amax, w1n, 0, nullptr, 0, wsh, w8);
}

// Candidate children of the fitness surrogate: plan index j, random draws
// from slot slot_off + j, and the per-wave squared distances to parent 1.
template <int kXoKind>
__global__ __launch_bounds__(256) void vary_cand_kernel(const float* __restrict__ cur,
                                                        float* __restrict__ cand,
                                                        const int4* __restrict__ plan,
                                                        int64_t stride, int64_t genes,
                                                        float sigma, uint64_t thr, Key key,
                                                        uint32_t gen, int n, uint32_t mul,
                                                        uint32_t slot_off, float* __restrict__ nu,
                                                        int ngroups) {
  const int j = (int)(((uint64_t)blockIdx.y * mul) % (uint32_t)n);
  vary_body<kXoKind, false, true>(j, blockIdx.x, cur, cand, plan, stride, genes, sigma, thr, key,
                                  gen, nullptr, nullptr, 0.0f, nullptr, 0, slot_off, nu, ngroups);
}

// A multiplier near pop * 0.618 that is coprime to pop: slot = (y * mul) mod
// pop visits every slot once and spreads the operators over the dispatch.
uint32_t slot_multiplier(int pop) {
  if (pop <= 1) return 1u;
  uint32_t mul = (uint32_t)(pop * 0.6180339887) | 1u;
  auto gcd = [](uint32_t a, uint32_t b) {
    while (b) {
      const uint32_t t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  while (gcd(mul, (uint32_t)pop) != 1u) ++mul;
  return mul;
}

hipError_t launch_vary(const float* cur, float* nxt, const int4* plan, const NetDesc& nd,
                       int pop, int crossover, float sigma, uint64_t mut_threshold,
                       const Key& key, uint32_t gen, const float* sig_cur, float* sig_next,
                       float tau, uint32_t* amax, const W1Shadow& wsh, const W1Fp8& w8,
                       hipStream_t s) {
  const int64_t groups = (nd.stride + 8191) / 8192;
  dim3 grid((unsigned)((groups + 3) / 4), (unsigned)pop);
  const uint32_t mul = slot_multiplier(pop);
  const int64_t w1n = (int64_t)nd.w[0] * nd.w[1];
#define LEEA_VARY(XO, AM, SH, F8)                                                              \
  hipLaunchKernelGGL((vary_kernel<XO, AM, SH, F8>), grid, dim3(256), 0, s, cur, nxt, plan,     \
                     nd.stride, nd.genes, sigma, mut_threshold, key, gen, pop, mul, sig_cur,     \
                     sig_next, tau, amax, w1n, wsh, w8)
  // kind: 0 genomes only; 1 + exact largest |W_1|; 2 + bfloat16 copy; 3 + exact
  // largest |W_1|, the FP8 scale bounds and (if kept) the FP8 copy
  const int kind = amax ? (w8.bound ? 3 : 1) : (wsh.p ? 2 : 0);
  if (crossover == 0) {
    if (kind == 1)
      LEEA_VARY(0, true, false, false);
    else if (kind == 2)
      LEEA_VARY(0, false, true, false);
    else if (kind == 3)
      LEEA_VARY(0, true, false, true);
    else
      LEEA_VARY(0, false, false, false);
  } else {
    if (kind == 1)
      LEEA_VARY(1, true, false, false);
    else if (kind == 2)
      LEEA_VARY(1, false, true, false);
    else if (kind == 3)
      LEEA_VARY(1, true, false, true);
    else
      LEEA_VARY(1, false, false, false);
  }
#undef LEEA_VARY
  return hipGetLastError();
}

hipError_t launch_vary_cand(const float* cur, float* cand, const int4* plan, const NetDesc& nd,
                            int n, int crossover, float sigma, uint64_t thr, const Key& key,
                            uint32_t gen, uint32_t slot_off, float* nu, hipStream_t s) {
  const int64_t groups = (nd.stride + 8191) / 8192;
  dim3 grid((unsigned)((groups + 3) / 4), (unsigned)n);
  const uint32_t mul = slot_multiplier(n);
  if (crossover == 0)
    hipLaunchKernelGGL(vary_cand_kernel<0>, grid, dim3(256), 0, s, cur, cand, plan, nd.stride,
                       nd.genes, sigma, thr, key, gen, n, mul, slot_off, nu, (int)groups);
  else
    hipLaunchKernelGGL(vary_cand_kernel<1>, grid, dim3(256), 0, s, cur, cand, plan, nd.stride,
                       nd.genes, sigma, thr, key, gen, n, mul, slot_off, nu, (int)groups);
  return hipGetLastError();
}

// Max of a 2x2 block; NaN if any of the four is NaN.
__device__ __forceinline__ float max4_nan(float a, float b, float c, float d) {
  float m = a > b ? a : b;
  m = m > c ? m : c;
  m = m > d ? m : d;
  if (a != a || b != b || c != c || d != d) m = __builtin_nanf("");
  return m;
}

// Example k of the batch is row floor(w * n_train / 2^32) of the training
// set, w = word k&3 of block (BATCH, gen, slot 0, k>>2).  One workgroup
// copies one row (float4 granularity; n_in is a multiple of 4).  With
// side > 0 the rows are side x side images that are 2x2 max-pooled on the
// way (section 4.1: the network pools its 28x28 inputs first).
__device__ __forceinline__ void draw_row(int k, const float* __restrict__ x_train,
                                         const int32_t* __restrict__ y_train, int64_t n_train,
                                         int n_in, int side, float* __restrict__ x_out,
                                         int32_t* __restrict__ y_out, const Key& key,
                                         uint32_t gen) {
  const uint4 w = draw(key, kBatch, gen, 0u, (uint32_t)(k >> 2));
  const uint64_t idx = ((uint64_t)word_of(w, k & 3) * (uint64_t)n_train) >> 32;
  if (side == 0) {
    const float4* src = reinterpret_cast<const float4*>(x_train + (int64_t)idx * n_in);
    float4* dst = reinterpret_cast<float4*>(x_out + (int64_t)k * n_in);
    for (int c = threadIdx.x; c < (n_in >> 2); c += 256) dst[c] = src[c];
  } else {
    const float* src = x_train + (int64_t)idx * side * side;
    const int h = side >> 1;
    for (int p = threadIdx.x; p < h * h; p += 256) {
      const int r = p / h;
      const int c = p - r * h;
      const float* q = src + 2 * r * side + 2 * c;
      x_out[(int64_t)k * n_in + p] = max4_nan(q[0], q[1], q[side], q[side + 1]);
    }
  }
  if (threadIdx.x == 0) y_out[k] = y_train[idx];
}

__global__ __launch_bounds__(256) void draw_batch_kernel(const float* __restrict__ x_train,
                                                         const int32_t* __restrict__ y_train,
                                                         int64_t n_train, int n_in, int side,
                                                         float* __restrict__ x_out,
                                                         int32_t* __restrict__ y_out, Key key,
                                                         uint32_t gen) {
  draw_row(blockIdx.x, x_train, y_train, n_train, n_in, side, x_out, y_out, key, gen);
}

hipError_t launch_draw_batch(const float* x_train, const int32_t* y_train, int64_t n_train,
                             int n_in, int side, int b, float* x_out, int32_t* y_out,
                             const Key& key, uint32_t gen, hipStream_t s) {
  hipLaunchKernelGGL(draw_batch_kernel, dim3((unsigned)b), dim3(256), 0, s, x_train, y_train,
                     n_train, n_in, side, x_out, y_out, key, gen);
  return hipGetLastError();
}

__global__ void pool2x2_kernel(const float* __restrict__ x, int64_t n, int side,
                               float* __restrict__ out) {
  const int h = side >> 1;
  const int64_t total = n * h * h;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256) {
    const int64_t e = i / (h * h);
    const int p = (int)(i - e * h * h);
    const int r = p / h;
    const int c = p - r * h;
    const float* q = x + e * side * side + 2 * r * side + 2 * c;
    out[i] = max4_nan(q[0], q[1], q[side], q[side + 1]);
  }
}

hipError_t launch_pool2x2(const float* x, int64_t n, int side, float* out, hipStream_t s) {
  const int64_t total = n * (side / 2) * (side / 2);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pool2x2_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, side, out);
  return hipGetLastError();
}

__global__ void fill_kernel(float* __restrict__ p, int n, float v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill(float* p, int n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ------------------------------------------------- grouped (many runs) --

// Batch rows of every run: workgroup = (run, row); generation = completed
// generations + step (step 0 draws the initial batch).
__global__ __launch_bounds__(256) void runs_draw_kernel(const RunDesc* __restrict__ runs,
                                                        const BatchState* __restrict__ st,
                                                        const int* __restrict__ off,
                                                        const int* __restrict__ ids, int n,
                                                        const float* __restrict__ x_train,
                                                        const int32_t* __restrict__ y_train,
                                                        int64_t n_train, int step) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  draw_row(blockIdx.x - off[i], x_train, y_train, n_train, d.nd.w[0], d.side, d.xb, d.yb, d.key,
           st->gen + (uint32_t)step);
}

hipError_t launch_runs_draw(const RunDesc* runs, const BatchState* st, const Group& g,
                            const float* x_train, const int32_t* y_train, int64_t n_train,
                            int step, hipStream_t s) {
  hipLaunchKernelGGL(runs_draw_kernel, dim3((unsigned)g.blocks), dim3(256), 0, s, runs, st, g.off,
                     g.ids, g.n, x_train, y_train, n_train, step);
  return hipGetLastError();
}

// Variation of every run: workgroup = (run, slot order y, gene-group block
// x) in the same order as the single-run launch; constant sigma.
__global__ __launch_bounds__(256) void runs_vary_kernel(const RunDesc* __restrict__ runs,
                                                        const BatchState* __restrict__ st,
                                                        const int* __restrict__ off,
                                                        const int* __restrict__ ids, int n) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  const int local = blockIdx.x - off[i];
  const int y = local / d.vgx;
  const int x = local - y * d.vgx;
  const int j = (int)(((uint64_t)y * d.mul) % (uint32_t)d.pop);
  const int c = st->cur;
  const uint32_t g = st->gen + 1;
  if (d.crossover == 0)
    vary_body<0, false>(j, x, d.genomes[c], d.genomes[c ^ 1], d.plan, d.nd.stride, d.nd.genes,
                        d.sigma, d.thr, d.key, g, nullptr, nullptr, 0.0f, nullptr, 0);
  else
    vary_body<1, false>(j, x, d.genomes[c], d.genomes[c ^ 1], d.plan, d.nd.stride, d.nd.genes,
                        d.sigma, d.thr, d.key, g, nullptr, nullptr, 0.0f, nullptr, 0);
}

hipError_t launch_runs_vary(const RunDesc* runs, const BatchState* st, const Group& g,
                            hipStream_t s) {
  hipLaunchKernelGGL(runs_vary_kernel, dim3((unsigned)g.blocks), dim3(256), 0, s, runs, st, g.off,
                     g.ids, g.n);
  return hipGetLastError();
}

// The new populations become current: one generation more, buffers and
// inherited fitness swap (every run at once).
__global__ void runs_advance_kernel(BatchState* st) {
  if (threadIdx.x == 0) {
    st->gen += 1;
    st->cur ^= 1;
    st->inh ^= 1;
    st->has_inh = 1;
  }
}

hipError_t launch_runs_advance(BatchState* st, hipStream_t s) {
  hipLaunchKernelGGL(runs_advance_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace leea
