// Learned fitness surrogate that pre-screens over-generated offspring: a
// requested variant of Algorithm 1 that spends predictions instead of
// evaluations.  Each generation keeps the n_E elites, makes k (P - n_E)
// candidate children (slot P + c of the generation's streams), describes
// every candidate by a fixed random +-1 projection of its bfloat16-rounded
// genome (256 values), its parents' adjusted fitness and its distance to
// parent 1, standardises every feature over the generation's candidates,
// predicts its fitness with a 259-64-1 MLP, keeps the P - n_E best
// predictions, evaluates the new population as usual and trains the MLP on
// that evaluation standardised over the kept candidates (full-batch gradient
// steps on the squared error).  Until
// the MLP has trained for `warmup` generations and its Kendall tau on the
// previous generation reaches tau_min, plain LEEA's mix of candidates is
// kept instead.
//
// Kernels: sign bits of the projection (once), candidate plan, the
// projection as a split-K bfloat16 matrix-core product whose signs are
// expanded from bits on the fly, feature assembly and standardisation,
// prediction, screening
// (bitonic sort in LDS), gather of the new population, training (forward,
// gradient, update) and the tau / fallback decision.  Every sum has a fixed
// order.
#include "lowp.hpp"
#include "select_common.hpp"

namespace leea {

constexpr int kFeat = 256;   // projection rows
constexpr int kHid = 64;     // hidden units
constexpr int kIn = kFeat + 3;
constexpr int kFeatLd = 260; // feature row stride (floats)
constexpr uint32_t kSurr = 7u;

typedef float floatx4s __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8s __attribute__((ext_vector_type(8)));

// bits[c][r] = word c & 3 of block (SURR, 0, r, c >> 2): sign bits of genes
// 32 c .. 32 c + 31 in projection row r (a set bit is -1).
__global__ __launch_bounds__(256) void proj_bits_kernel(uint32_t* __restrict__ bits, int nchunks,
                                                        Key key) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)nchunks * kFeat) return;
  const int c = (int)(idx / kFeat);
  const int r = (int)(idx - (int64_t)c * kFeat);
  const uint4 w = draw(key, kSurr, 0u, (uint32_t)r, (uint32_t)(c >> 2));
  bits[idx] = word_of(w, c & 3);
}

hipError_t launch_proj_bits(uint32_t* bits, int nchunks, const Key& key, hipStream_t s) {
  const int64_t n = (int64_t)nchunks * kFeat;
  hipLaunchKernelGGL(proj_bits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, bits,
                     nchunks, key);
  return hipGetLastError();
}

// Glorot-uniform weights from (SURR, 1, slot h, block d >> 2) for the first
// layer and (SURR, 2, slot 0, block h >> 2) for the second; zero biases.
// Parameter layout: W1 [kHid][kIn], b1 [kHid], w2 [kHid], b2 [1].
__global__ __launch_bounds__(256) void mlp_init_kernel(float* __restrict__ prm, Key key, float a1,
                                                       float a2) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int nw1 = kHid * kIn;
  if (i < nw1) {
    const int h = i / kIn;
    const int d = i - h * kIn;
    const uint4 w = draw(key, kSurr, 1u, (uint32_t)h, (uint32_t)(d >> 2));
    const float u = (float)(word_of(w, d & 3) >> 8) * 5.9604644775390625e-8f;
    float t = 2.0f * u;
    t = t - 1.0f;
    prm[i] = t * a1;
  } else if (i < nw1 + kHid) {
    prm[i] = 0.0f;
  } else if (i < nw1 + 2 * kHid) {
    const int h = i - nw1 - kHid;
    const uint4 w = draw(key, kSurr, 2u, 0u, (uint32_t)(h >> 2));
    const float u = (float)(word_of(w, h & 3) >> 8) * 5.9604644775390625e-8f;
    float t = 2.0f * u;
    t = t - 1.0f;
    prm[i] = t * a2;
  } else if (i == nw1 + 2 * kHid) {
    prm[i] = 0.0f;
  }
}

hipError_t launch_mlp_init(float* prm, const Key& key, float a1, float a2, hipStream_t s) {
  const int n = kHid * kIn + 2 * kHid + 1;
  hipLaunchKernelGGL(mlp_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, prm, key,
                     a1, a2);
  return hipGetLastError();
}

// Candidate c: crossover if c < kc, else mutation; parents from slot pop + c.
__global__ __launch_bounds__(256) void cand_plan_kernel(const int32_t* __restrict__ order,
                                                        const float* __restrict__ f_adj, int M,
                                                        int kc, int pop, int n_trunc,
                                                        int selection, int tk, Key key,
                                                        uint32_t gen, int4* __restrict__ cplan,
                                                        float* __restrict__ cf_inh) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= M) return;
  const uint32_t slot = (uint32_t)(pop + c);
  const uint32_t r1 = parent_rank(key, gen, slot, 0, selection, tk, (uint32_t)n_trunc,
                                  (uint32_t)pop);
  const int p1 = order[r1];
  if (c < kc) {
    const uint32_t r2 = parent_rank(key, gen, slot, 1, selection, tk, (uint32_t)n_trunc,
                                    (uint32_t)pop);
    const int p2 = order[r2];
    cplan[c] = make_int4(kOpCross, p1, p2, 0);
    const float sum = f_adj[p1] + f_adj[p2];
    cf_inh[c] = sum * 0.5f;
  } else {
    cplan[c] = make_int4(kOpMut, p1, p1, 0);
    cf_inh[c] = f_adj[p1];
  }
}

hipError_t launch_cand_plan(const int32_t* order, const float* f_adj, int M, int kc, int pop,
                            int n_trunc, int selection, int tk, const Key& key, uint32_t gen,
                            int4* cplan, float* cf_inh, hipStream_t s) {
  hipLaunchKernelGGL(cand_plan_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, order,
                     f_adj, M, kc, pop, n_trunc, selection, tk, key, gen, cplan, cf_inh);
  return hipGetLastError();
}

// Projection part[sp][c][r] = sum over the split's genes i of bf16(x_c[i]) *
// R[r][i]: workgroup = (64 candidates, split sp); per 32-gene chunk the
// candidates' genes are converted to bfloat16 and the 256 rows' sign words
// expanded to +-1.0 bfloat16, both staged in LDS (rows of 64 bytes, 16-byte
// slot s of row r at slot s ^ ((r >> 1) & 3)); wave w multiplies all 64
// candidates by projection rows 64 w .. 64 w + 63 with
// v_mfma_f32_16x16x32_bf16 (lane l: A[l%16][8(l/16)+e], B[8(l/16)+e][l%16]).
__global__ __launch_bounds__(256) void proj_kernel(const float* __restrict__ cand, int64_t stride,
                                                   int M, const uint32_t* __restrict__ bits,
                                                   int nchunks, int cps,
                                                   float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char sa[64 * 64];
  __shared__ __attribute__((aligned(16))) char sb[kFeat * 64];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const int c0 = blockIdx.x * 64;
  const int sp = blockIdx.y;
  const int ch0 = sp * cps;
  const int ch1 = ch0 + cps < nchunks ? ch0 + cps : nchunks;
  // A staging item of this thread: candidate row ar, slot as
  const int ar = tid >> 2;
  const int as = tid & 3;
  const bool av = c0 + ar < M;
  const float* arow = cand + (int64_t)(av ? c0 + ar : 0) * stride;
  floatx4s acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[i][t] = floatx4s{0.f, 0.f, 0.f, 0.f};
  // the next chunk's candidate values and sign word are loaded while the
  // current one is converted and multiplied
  float4 nv0, nv1;
  uint32_t nw = 0;
  auto fetch = [&](int ch) {
    const int k0 = ch * 32;
    nv0 = *reinterpret_cast<const float4*>(arow + k0 + 8 * as);
    nv1 = *reinterpret_cast<const float4*>(arow + k0 + 8 * as + 4);
    nw = bits[(int64_t)ch * kFeat + tid];
  };
  if (ch0 < ch1) fetch(ch0);
  for (int ch = ch0; ch < ch1; ++ch) {
    const float4 v0 = nv0, v1 = nv1;
    const uint32_t w = nw;
    if (ch + 1 < ch1) fetch(ch + 1);
    {  // candidates -> bf16
      uint4 o;
      o.x = pack_bf16x2(v0.x, v0.y);
      o.y = pack_bf16x2(v0.z, v0.w);
      o.z = pack_bf16x2(v1.x, v1.y);
      o.w = pack_bf16x2(v1.z, v1.w);
      if (!av) o = make_uint4(0u, 0u, 0u, 0u);
      *reinterpret_cast<uint4*>(sa + ar * 64 + ((as ^ ((ar >> 1) & 3)) * 16)) = o;
    }
    {  // sign word of row tid -> 32 bf16 of +-1
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        uint32_t d[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const uint32_t v = w >> (8 * s + 2 * p);
          d[p] = 0x3F803F80u | ((v & 1u) << 15) | ((v & 2u) << 30);
        }
        *reinterpret_cast<uint4*>(sb + tid * 64 + ((s ^ ((tid >> 1) & 3)) * 16)) =
            make_uint4(d[0], d[1], d[2], d[3]);
      }
    }
    __syncthreads();
    uint4 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = i * 16 + mn;
      a[i] = *reinterpret_cast<const uint4*>(sa + m * 64 + ((kq ^ ((m >> 1) & 3)) * 16));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = wave * 64 + t * 16 + mn;
      b[t] = *reinterpret_cast<const uint4*>(sb + n * 64 + ((kq ^ ((n >> 1) & 3)) * 16));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf16x8s, a[i]), __builtin_bit_cast(bf16x8s, b[t]), acc[i][t], 0,
            0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = c0 + i * 16 + 4 * kq + e;
        const int n = wave * 64 + t * 16 + mn;
        if (c < M) part[((int64_t)sp * M + c) * kFeat + n] = acc[i][t][e];
      }
}

hipError_t launch_proj(const float* cand, int64_t stride, int M, const uint32_t* bits,
                       int nchunks, int splits, float* part, hipStream_t s) {
  const int cps = (nchunks + splits - 1) / splits;
  hipLaunchKernelGGL(proj_kernel, dim3((unsigned)((M + 63) / 64), (unsigned)splits), dim3(256), 0,
                     s, cand, stride, M, bits, nchunks, cps, part);
  return hipGetLastError();
}

// feat[c] = [scale * sum of the split parts (in split order), f_adj of the
// parents, scale * sqrt(sum of the wave partial squared distances in order)].
__global__ __launch_bounds__(256) void features_kernel(const float* __restrict__ part, int splits,
                                                       int M, const float* __restrict__ nu,
                                                       int ngroups, const int4* __restrict__ cplan,
                                                       const float* __restrict__ f_adj,
                                                       float scale, float* __restrict__ feat) {
#pragma clang fp contract(off)
  const int c = blockIdx.x;
  const int r = threadIdx.x;
  float s = 0.0f;
  for (int sp = 0; sp < splits; ++sp) s += part[((int64_t)sp * M + c) * kFeat + r];
  feat[(int64_t)c * kFeatLd + r] = s * scale;
  if (r == 0) {
    const int4 pl = cplan[c];
    float q = 0.0f;
    for (int g = 0; g < ngroups; ++g) q += nu[(int64_t)c * ngroups + g];
    feat[(int64_t)c * kFeatLd + kFeat] = f_adj[pl.y];
    feat[(int64_t)c * kFeatLd + kFeat + 1] = f_adj[pl.z];
    const float rt = __builtin_sqrtf(q);
    feat[(int64_t)c * kFeatLd + kFeat + 2] = rt * scale;
    feat[(int64_t)c * kFeatLd + kFeat + 3] = 0.0f;
  }
}

hipError_t launch_features(const float* part, int splits, int M, const float* nu, int ngroups,
                           const int4* cplan, const float* f_adj, float scale, float* feat,
                           hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)M), dim3(256), 0, s, part, splits, M, nu,
                     ngroups, cplan, f_adj, scale, feat);
  return hipGetLastError();
}

// Fixed-order sum of one value per thread over a 256-thread workgroup
// (halving tree in LDS); every thread gets the total.
__device__ __forceinline__ float block_sum256(float v, float* red) {
#pragma clang fp contract(off)
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] = red[t] + red[t + off];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

// MLP inputs: feature d of every candidate minus its mean over the M
// candidates, divided by its standard deviation over them (no Bessel
// correction); 0 where that deviation is 0; the projection features then
// times 2^-4 = 1 / sqrt(256), so that the whole projection weighs as much as
// one scalar feature (an exact scaling).  Workgroup = feature d (d = 259,
// the padding column, writes zeros); thread t sums candidates t, t + 256, ...
// in order, then the halving tree.
__global__ __launch_bounds__(256) void standardize_kernel(const float* __restrict__ feat, int M,
                                                          float* __restrict__ z) {
#pragma clang fp contract(off)
  __shared__ float red[256];
  const int d = blockIdx.x;
  const int t = threadIdx.x;
  if (d >= kIn) {
    for (int c = t; c < M; c += 256) z[(int64_t)c * kFeatLd + d] = 0.0f;
    return;
  }
  float s = 0.0f;
  for (int c = t; c < M; c += 256) s += feat[(int64_t)c * kFeatLd + d];
  const float mean = block_sum256(s, red) / (float)M;
  float q = 0.0f;
  for (int c = t; c < M; c += 256) {
    const float dx = feat[(int64_t)c * kFeatLd + d] - mean;
    q += dx * dx;
  }
  const float var = block_sum256(q, red) / (float)M;
  const float sd = __builtin_sqrtf(var);
  const float wgt = d < kFeat ? 0.0625f : 1.0f;  // 1 / sqrt(kFeat), exact
  for (int c = t; c < M; c += 256) {
    const float dx = feat[(int64_t)c * kFeatLd + d] - mean;
    z[(int64_t)c * kFeatLd + d] = sd > 0.0f ? (dx / sd) * wgt : 0.0f;
  }
}

hipError_t launch_standardize(const float* feat, int M, float* z, hipStream_t s) {
  hipLaunchKernelGGL(standardize_kernel, dim3((unsigned)kFeatLd), dim3(256), 0, s, feat, M, z);
  return hipGetLastError();
}

// Training targets: the finite fitness values y[n] minus their mean, divided
// by their standard deviation (1 if it is 0); other values copied.  One
// workgroup, the same fixed-order sums.
__global__ __launch_bounds__(256) void targets_kernel(const float* __restrict__ y, int N,
                                                      float* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ float red[256];
  const int t = threadIdx.x;
  float s = 0.0f, k = 0.0f;
  for (int n = t; n < N; n += 256) {
    const float v = y[n];
    const bool ok = v == v && v != __builtin_inff() && v != -__builtin_inff();
    if (ok) {
      s += v;
      k += 1.0f;
    }
  }
  const float tot = block_sum256(s, red);
  const float cnt = block_sum256(k, red);
  const float mean = cnt > 0.0f ? tot / cnt : 0.0f;
  float q = 0.0f;
  for (int n = t; n < N; n += 256) {
    const float v = y[n];
    const bool ok = v == v && v != __builtin_inff() && v != -__builtin_inff();
    if (ok) {
      const float dv = v - mean;
      q += dv * dv;
    }
  }
  const float var = cnt > 0.0f ? block_sum256(q, red) / cnt : 0.0f;
  float sd = __builtin_sqrtf(var);
  sd = sd > 0.0f ? sd : 1.0f;
  for (int n = t; n < N; n += 256) {
    const float v = y[n];
    const bool ok = v == v && v != __builtin_inff() && v != -__builtin_inff();
    if (ok) {
      const float dv = v - mean;
      out[n] = dv / sd;
    } else {
      out[n] = v;
    }
  }
}

hipError_t launch_targets(const float* y, int N, float* out, hipStream_t s) {
  hipLaunchKernelGGL(targets_kernel, dim3(1), dim3(256), 0, s, y, N, out);
  return hipGetLastError();
}

// MLP forward of rows idx[n] (or n when idx is NULL): pre[n][u] (optional)
// and pred[n].  Workgroup = kFwdRows rows staged in LDS; wave q takes the
// inputs d in [65 q, 65 q + 65) and lane u hidden unit u: each weight it
// loads serves all kFwdRows rows.  The four partial sums of (row, u) are
// added in wave order with the bias; then one thread per row sums the
// hidden units in order.
constexpr int kFwdRows = 16;
constexpr int kFwdSlice = (kIn + 3) / 4;  // 65 inputs per wave

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ prm,
                                                          const float* __restrict__ feat,
                                                          const int32_t* __restrict__ idx, int n,
                                                          float* __restrict__ pre,
                                                          float* __restrict__ pred) {
#pragma clang fp contract(off)
  __shared__ float xs[kFwdRows][kFeatLd];
  __shared__ float hp[4][kFwdRows][kHid];
  const int r0 = blockIdx.x * kFwdRows;
  const int tid = threadIdx.x;
  const int u = tid & 63;
  const int q = tid >> 6;
  // wave q stages rows q, q + 4, ...: whole rows, every load independent
#pragma unroll
  for (int k = 0; k < kFwdRows / 4; ++k) {
    const int r = q + 4 * k;
    const int m = r0 + r;
    const float* __restrict__ src = m < n ? feat + (int64_t)(idx ? idx[m] : m) * kFeatLd : nullptr;
#pragma unroll
    for (int d = u; d < kFeatLd; d += 64) xs[r][d] = src ? src[d] : 0.0f;
  }
  __syncthreads();
  const int d0 = q * kFwdSlice;
  const int d1 = d0 + kFwdSlice < kIn ? d0 + kFwdSlice : kIn;
  const float* __restrict__ w = prm + u * kIn;
  float acc[kFwdRows];
#pragma unroll
  for (int r = 0; r < kFwdRows; ++r) acc[r] = 0.0f;
  for (int d = d0; d < d1; ++d) {
    const float wd = w[d];
#pragma unroll
    for (int r = 0; r < kFwdRows; ++r) acc[r] += wd * xs[r][d];
  }
#pragma unroll
  for (int r = 0; r < kFwdRows; ++r) hp[q][r][u] = acc[r];
  __syncthreads();
  {
    // thread (u, q) finishes rows q, q + 4, q + 8, q + 12 of unit u
    const float bu = prm[kHid * kIn + u];
#pragma unroll
    for (int k = 0; k < kFwdRows / 4; ++k) {
      const int r = q + 4 * k;
      const float v = ((hp[0][r][u] + hp[1][r][u]) + (hp[2][r][u] + hp[3][r][u])) + bu;
      if (pre && r0 + r < n) pre[(int64_t)(r0 + r) * kHid + u] = v;
      xs[r][u] = v > 0.0f ? v : 0.0f;  // the rows' inputs are no longer needed
    }
  }
  __syncthreads();
  if (tid < kFwdRows && r0 + tid < n) {
    const float* w2 = prm + kHid * kIn + kHid;
    float o = 0.0f;
    for (int h = 0; h < kHid; ++h) o += w2[h] * xs[tid][h];
    o += w2[kHid];
    pred[r0 + tid] = o;
  }
}

hipError_t launch_mlp_forward(const float* prm, const float* feat, const int32_t* idx, int n,
                              float* pre, float* pred, hipStream_t s) {
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + kFwdRows - 1) / kFwdRows)),
                     dim3(256), 0, s, prm, feat, idx, n, pre, pred);
  return hipGetLastError();
}

// Number of keys[j], j0 <= j < j1, below own (keys in LDS, 16-byte aligned,
// j0 even): 128-bit reads of two keys, four reads in flight per step.
__device__ __forceinline__ int count_below(const uint64_t* keys, int j0, int j1, uint64_t own) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  const u64x2* k2 = reinterpret_cast<const u64x2*>(keys);
  int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
  int j = j0;
  for (; j + 8 <= j1; j += 8) {
    const u64x2 a = k2[j >> 1], b = k2[(j >> 1) + 1], c = k2[(j >> 1) + 2], d = k2[(j >> 1) + 3];
    r0 += (a.x < own ? 1 : 0) + (a.y < own ? 1 : 0);
    r1 += (b.x < own ? 1 : 0) + (b.y < own ? 1 : 0);
    r2 += (c.x < own ? 1 : 0) + (c.y < own ? 1 : 0);
    r3 += (d.x < own ? 1 : 0) + (d.y < own ? 1 : 0);
  }
  for (; j < j1; ++j) r0 += keys[j] < own ? 1 : 0;
  return (r0 + r1) + (r2 + r3);
}

// Screening: chosen[i] for the N non-elite slots.  With the surrogate on
// (*flag != 0) the N best predictions in rank_key order (descending, ties by
// candidate index, NaN last): every candidate counts the keys below its own
// (the keys are unique, so the counts are the sorted positions; four
// threads per candidate count a quarter of the keys each, from LDS) and
// candidates ranked below N write themselves there; otherwise the first n_c
// crossover and the first n_m mutation candidates.  chosen_pred[i] =
// pred[chosen[i]].  (The sort by counting took 17 us for 3,800 candidates
// against 34 us for a bitonic network in one workgroup.)
constexpr int kScreenCands = 64;  // candidates per workgroup (4 threads each)

__global__ __launch_bounds__(256) void screen_kernel(const float* __restrict__ pred, int M, int N,
                                                     int n_c, int kc,
                                                     const int32_t* __restrict__ flag,
                                                     int32_t* __restrict__ chosen,
                                                     float* __restrict__ chosen_pred) {
  extern __shared__ uint64_t keys[];
  const int tid = threadIdx.x;
  if (*flag == 0) {
    for (int c = blockIdx.x * 256 + tid; c < N; c += gridDim.x * 256) {
      const int k = c < n_c ? c : kc + (c - n_c);
      chosen[c] = k;
      chosen_pred[c] = pred[k];
    }
    return;
  }
  for (int i = tid; i < M; i += 256) keys[i] = rank_key(pred[i], (uint32_t)i);
  __syncthreads();
  const int c = blockIdx.x * kScreenCands + (tid >> 2);
  const int part = tid & 3;
  const int q = ((M + 7) >> 3) * 2;  // a quarter of the keys, even
  const int j0 = part * q < M ? part * q : M;
  const int j1 = j0 + q < M ? j0 + q : M;
  int r = c < M ? count_below(keys, j0, j1, keys[c]) : 0;
  r += __shfl_xor(r, 1);
  r += __shfl_xor(r, 2);
  if (c < M && part == 0 && r < N) {
    chosen[r] = c;
    chosen_pred[r] = pred[c];
  }
}

hipError_t launch_screen(const float* pred, int M, int N, int n_c, int kc, const int32_t* flag,
                         int32_t* chosen, float* chosen_pred, hipStream_t s) {
  hipLaunchKernelGGL(screen_kernel, dim3((unsigned)((M + kScreenCands - 1) / kScreenCands)),
                     dim3(256), (size_t)M * 8, s, pred, M, N, n_c, kc, flag, chosen,
                     chosen_pred);
  return hipGetLastError();
}

// New population: slot j < n_e copies the elite of plan[j]; slot n_e + i
// copies candidate chosen[i]; inherited fitness likewise.
__global__ __launch_bounds__(256) void gather_kernel(const float* __restrict__ cur,
                                                     const float* __restrict__ cand,
                                                     float* __restrict__ nxt, int64_t stride,
                                                     int n_e, const int4* __restrict__ plan,
                                                     const int32_t* __restrict__ chosen,
                                                     const float* __restrict__ f_adj,
                                                     const float* __restrict__ cf_inh,
                                                     float* __restrict__ f_inh_next) {
  const int j = blockIdx.y;
  const float* src = j < n_e ? cur + (int64_t)plan[j].y * stride
                             : cand + (int64_t)chosen[j - n_e] * stride;
  const int64_t n4 = stride >> 2;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  float4* d4 = reinterpret_cast<float4*>(nxt + (int64_t)j * stride);
  for (int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x; f < n4; f += (int64_t)gridDim.x * 256)
    d4[f] = s4[f];
  if (blockIdx.x == 0 && threadIdx.x == 0)
    f_inh_next[j] = j < n_e ? f_adj[plan[j].y] : cf_inh[chosen[j - n_e]];
}

hipError_t launch_gather(const float* cur, const float* cand, float* nxt, int64_t stride,
                         int pop, int n_e, const int4* plan, const int32_t* chosen,
                         const float* f_adj, const float* cf_inh, float* f_inh_next,
                         hipStream_t s) {
  const int64_t n4 = stride >> 2;
  int64_t gx = (n4 + 255) / 256;
  if (gx > 64) gx = 64;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)gx, (unsigned)pop), dim3(256), 0, s, cur, cand,
                     nxt, stride, n_e, plan, chosen, f_adj, cf_inh, f_inh_next);
  return hipGetLastError();
}

// Gradient of mean((pred - y)^2) over the rows with a numeric target
// y[n] = training target of kept candidate n (rows without one contribute
// zeros).  Workgroup (row block, parameter chunk) = kGradRows consecutive
// rows x 256 parameters: it stages the rows' inputs, d[r][u] = e_r w_2[u]
// [pre > 0] (e_r = pred - y), relu(pre) and e_r in LDS and writes, for each
// of its parameters, the sum over the rows in row order (a block of the
// products D^T X, D^T 1, relu(pre)^T e, 1^T e).  The update adds the row
// blocks in order, scales by 2 / rows and takes the step.
constexpr int kGradRows = 32;
constexpr int kParams = kHid * kIn + 2 * kHid + 1;

__device__ __forceinline__ bool finite_f(float t) {
  return t == t && t != __builtin_inff() && t != -__builtin_inff();
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ prm,
                                                       const float* __restrict__ feat,
                                                       const int32_t* __restrict__ idx,
                                                       const float* __restrict__ pre,
                                                       const float* __restrict__ pred,
                                                       const float* __restrict__ y, int N,
                                                       float* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ float xs[kGradRows][kFeatLd];
  __shared__ float ds[kGradRows][kHid];
  __shared__ float hs[kGradRows][kHid];
  __shared__ float es[kGradRows];
  const int blk = blockIdx.x;  // row block
  const int n0 = blk * kGradRows;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nw1 = kHid * kIn;
  // wave w stages rows w, w + 4, ...: the inputs (whole rows), d and relu
  // of every hidden unit (lane = unit) and e
#pragma unroll
  for (int k = 0; k < kGradRows / 4; ++k) {
    const int r = wave + 4 * k;
    const int n = n0 + r;
    const float t = n < N ? y[n] : 0.0f;
    const bool ok = n < N && finite_f(t);
    const float* __restrict__ src = ok ? feat + (int64_t)idx[n] * kFeatLd : nullptr;
#pragma unroll
    for (int d = lane; d < kFeatLd; d += 64) xs[r][d] = src ? src[d] : 0.0f;
    float dv = 0.0f, hv = 0.0f, e = 0.0f;
    if (ok) {
      e = pred[n] - t;
      const float pv = pre[(int64_t)n * kHid + lane];
      dv = pv > 0.0f ? e * prm[nw1 + kHid + lane] : 0.0f;
      hv = pv > 0.0f ? pv : 0.0f;
    }
    ds[r][lane] = dv;
    hs[r][lane] = hv;
    if (lane == 0) es[r] = e;
  }
  __syncthreads();
  float* __restrict__ g = part + (int64_t)blk * kParams;
  const int o = blockIdx.y * 256 + tid;  // parameter
  if (o < kParams) {
    float sum = 0.0f;
    if (o < nw1) {
      const int u = o / kIn;
      const int d = o - u * kIn;
#pragma unroll 8
      for (int r = 0; r < kGradRows; ++r) sum += ds[r][u] * xs[r][d];
    } else if (o < nw1 + kHid) {
      const int u = o - nw1;
#pragma unroll 8
      for (int r = 0; r < kGradRows; ++r) sum += ds[r][u];
    } else if (o < nw1 + 2 * kHid) {
      const int u = o - nw1 - kHid;
#pragma unroll 8
      for (int r = 0; r < kGradRows; ++r) sum += es[r] * hs[r][u];
    } else {
      for (int r = 0; r < kGradRows; ++r) sum += es[r];
    }
    g[o] = sum;
  }
  if (blockIdx.y == 0 && tid == 0) {
    int rows = 0;
    for (int r = 0; r < kGradRows; ++r) rows += (n0 + r < N && finite_f(y[n0 + r])) ? 1 : 0;
    reinterpret_cast<int*>(part + (int64_t)gridDim.x * kParams)[blk] = rows;
  }
}

__global__ __launch_bounds__(256) void mlp_update_kernel(float* __restrict__ prm,
                                                         const float* __restrict__ part,
                                                         int nblk, float lr) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kParams) return;
  const int* cnt = reinterpret_cast<const int*>(part + (int64_t)nblk * kParams);
  int rows = 0;
  float tot = 0.0f;
  for (int k = 0; k < nblk; ++k) {
    tot += part[(int64_t)k * kParams + i];
    rows += cnt[k];
  }
  const float f = rows > 0 ? 2.0f / (float)rows : 0.0f;
  const float step = lr * (tot * f);
  prm[i] = prm[i] - step;
}

int mlp_grad_blocks(int N) { return (N + kGradRows - 1) / kGradRows; }

hipError_t launch_mlp_train_step(float* prm, const float* feat, const int32_t* idx, int N,
                                 const float* y, float* pre, float* pred, float* grad, float lr,
                                 hipStream_t s) {
  hipError_t e = launch_mlp_forward(prm, feat, idx, N, pre, pred, s);
  if (e != hipSuccess) return e;
  const int nblk = mlp_grad_blocks(N);
  if (nblk < 1) return hipSuccess;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)nblk, (kParams + 255) / 256), dim3(256), 0, s,
                     prm, feat, idx, pre, pred, y, N, grad);
  hipLaunchKernelGGL(mlp_update_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, prm, grad,
                     nblk, lr);
  return hipGetLastError();
}

// +1 for a concordant pair, -1 for a discordant one, 0 for a tie or a NaN.
__device__ __forceinline__ int concord(float dp, float dy) {
  const int sp = (dp > 0.0f) - (dp < 0.0f);
  const int sy = (dy > 0.0f) - (dy < 0.0f);
  return sp * sy;
}

// Numerator of Kendall tau-a: workgroup w takes rows i = w, w + G, ...,
// its threads the partners j = i + 1 + t, + 256, ...; the workgroup's sum is
// added to *acc with a 64-bit integer atomic (exact, so the total does not
// depend on the order of the additions).
constexpr int kTauBlocks = 64;

__global__ __launch_bounds__(256) void tau_pairs_kernel(const float* __restrict__ p,
                                                        const float* __restrict__ y, int N,
                                                        unsigned long long* __restrict__ acc) {
  __shared__ int red[4];
  int s = 0;
  for (int i = blockIdx.x; i < N; i += gridDim.x) {
    const float pi = p[i], yi = y[i];
    for (int j = i + 1 + (int)threadIdx.x; j < N; j += 256) s += concord(pi - p[j], yi - y[j]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long t = (long long)red[0] + red[1] + red[2] + red[3];
    if (t) atomicAdd(acc, (unsigned long long)t);
  }
}

// Kendall tau-a of the screening predictions against the evaluated fitness
// of the kept candidates (numerator from tau_pairs_kernel, which this kernel
// clears for the next generation), root mean squared error against their
// training targets (the standardised fitness), and the next generation's
// decision: on when `warmup` generations have trained and tau >= tau_min.
// state = {flag, trained generations, numerator (64 bits)}; stats (and
// stats_out when not NULL) = {surrogate used this generation, tau, rmse,
// trained generations}.
__global__ __launch_bounds__(1024) void surrogate_judge_kernel(const float* __restrict__ p,
                                                               const float* __restrict__ yt, int N,
                                                               int warmup, float tau_min,
                                                               int32_t* __restrict__ state,
                                                               float* __restrict__ stats,
                                                               float* __restrict__ stats_out) {
  __shared__ float sq[1024];
  __shared__ int cnt[1024];
  const int tid = threadIdx.x;
  float e2 = 0.0f;
  int c = 0;
  for (int i = tid; i < N; i += 1024) {
    const float d = p[i] - yt[i];
    if (d == d && d != __builtin_inff() && d != -__builtin_inff()) {
      e2 += d * d;
      ++c;
    }
  }
  sq[tid] = e2;
  cnt[tid] = c;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) {
      sq[tid] += sq[tid + off];
      cnt[tid] += cnt[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(state + 2);
    const long long num = (long long)*acc;
    *acc = 0ull;
    const double pairs = (double)N * (double)(N - 1) / 2.0;
    const float tau = pairs > 0 ? (float)((double)num / pairs) : 0.0f;
    const float rmse = cnt[0] > 0 ? __builtin_sqrtf(sq[0] / (float)cnt[0]) : 0.0f;
    const int trained = state[1] + 1;
    const float st[4] = {(float)state[0], tau, rmse, (float)trained};
    for (int k = 0; k < 4; ++k) {
      stats[k] = st[k];
      if (stats_out) stats_out[k] = st[k];
    }
    state[1] = trained;
    state[0] = (trained >= warmup && tau >= tau_min) ? 1 : 0;
  }
}

hipError_t launch_surrogate_judge(const float* pred, const float* y, const float* yt, int N,
                                  int warmup, float tau_min, int32_t* state, float* stats,
                                  float* stats_out, hipStream_t s) {
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(state + 2);
  if (N > 1)
    hipLaunchKernelGGL(tau_pairs_kernel, dim3(N - 1 < kTauBlocks ? N - 1 : kTauBlocks), dim3(256),
                       0, s, pred, y, N, acc);
  hipLaunchKernelGGL(surrogate_judge_kernel, dim3(1), dim3(1024), 0, s, pred, yt, N, warmup,
                     tau_min, state, stats, stats_out);
  return hipGetLastError();
}

}  // namespace leea
