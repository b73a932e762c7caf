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
  for (int ch = ch0; ch < ch1; ++ch) {
    const int k0 = ch * 32;
    {  // candidates -> bf16
      const float4 v0 = *reinterpret_cast<const float4*>(arow + k0 + 8 * as);
      const float4 v1 = *reinterpret_cast<const float4*>(arow + k0 + 8 * as + 4);
      uint4 o;
      o.x = pack_bf16x2(v0.x, v0.y);
      o.y = pack_bf16x2(v0.z, v0.w);
      o.z = pack_bf16x2(v1.x, v1.y);
      o.w = pack_bf16x2(v1.z, v1.w);
      if (!av) o = make_uint4(0u, 0u, 0u, 0u);
      *reinterpret_cast<uint4*>(sa + ar * 64 + ((as ^ ((ar >> 1) & 3)) * 16)) = o;
    }
    {  // sign word of row tid -> 32 bf16 of +-1
      const uint32_t w = bits[(int64_t)ch * kFeat + tid];
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
// correction); 0 where that deviation is 0.  Workgroup = feature d (d = 259,
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
  for (int c = t; c < M; c += 256) {
    const float dx = feat[(int64_t)c * kFeatLd + d] - mean;
    z[(int64_t)c * kFeatLd + d] = sd > 0.0f ? dx / sd : 0.0f;
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
// and pred[n].  Workgroup = one row, thread u = hidden unit; inputs summed
// in index order, hidden units summed in order by thread 0.
__global__ __launch_bounds__(64) void mlp_forward_kernel(const float* __restrict__ prm,
                                                         const float* __restrict__ feat,
                                                         const int32_t* __restrict__ idx,
                                                         float* __restrict__ pre,
                                                         float* __restrict__ pred) {
#pragma clang fp contract(off)
  __shared__ float hs[kHid];
  const int n = blockIdx.x;
  const int u = threadIdx.x;
  const int row = idx ? idx[n] : n;
  const float* x = feat + (int64_t)row * kFeatLd;
  const float* w = prm + u * kIn;
  float s = 0.0f;
  for (int d = 0; d < kIn; ++d) s += w[d] * x[d];
  s += prm[kHid * kIn + u];
  if (pre) pre[(int64_t)n * kHid + u] = s;
  hs[u] = s > 0.0f ? s : 0.0f;
  __syncthreads();
  if (u == 0) {
    const float* w2 = prm + kHid * kIn + kHid;
    float o = 0.0f;
    for (int h = 0; h < kHid; ++h) o += w2[h] * hs[h];
    o += w2[kHid];
    pred[n] = o;
  }
}

hipError_t launch_mlp_forward(const float* prm, const float* feat, const int32_t* idx, int n,
                              float* pre, float* pred, hipStream_t s) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)n), dim3(64), 0, s, prm, feat, idx, pre,
                     pred);
  return hipGetLastError();
}

// Screening: chosen[i] for the N non-elite slots.  With the surrogate on
// (*flag != 0) the N best predictions (rank_key order: descending, ties by
// candidate index, NaN last); otherwise the first n_c crossover and the
// first n_m mutation candidates.  chosen_pred[i] = pred[chosen[i]].
__global__ __launch_bounds__(1024) void screen_kernel(const float* __restrict__ pred, int M, int n2,
                                                      int N, int n_c, int kc,
                                                      const int32_t* __restrict__ flag,
                                                      int32_t* __restrict__ chosen,
                                                      float* __restrict__ chosen_pred) {
  extern __shared__ uint64_t keys[];
  const int tid = threadIdx.x;
  const bool use = *flag != 0;
  if (use) {
    for (int i = tid; i < n2; i += 1024)
      keys[i] = i < M ? rank_key(pred[i], (uint32_t)i) : ~0ull;
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
      for (int half = size >> 1; half > 0; half >>= 1) {
        for (int i = tid; i < (n2 >> 1); i += 1024) {
          const int lo = 2 * i - (i & (half - 1));
          const int hi = lo + half;
          const bool up = (lo & size) == 0;
          const uint64_t a = keys[lo];
          const uint64_t b = keys[hi];
          if ((a > b) == up) {
            keys[lo] = b;
            keys[hi] = a;
          }
        }
        __syncthreads();
      }
    }
  }
  for (int i = tid; i < N; i += 1024) {
    const int c = use ? (int)(uint32_t)keys[i] : (i < n_c ? i : kc + (i - n_c));
    chosen[i] = c;
    chosen_pred[i] = pred[c];
  }
}

hipError_t launch_screen(const float* pred, int M, int N, int n_c, int kc, const int32_t* flag,
                         int32_t* chosen, float* chosen_pred, hipStream_t s) {
  int n2 = 2;
  while (n2 < M) n2 <<= 1;
  hipLaunchKernelGGL(screen_kernel, dim3(1), dim3(1024), (size_t)n2 * 8, s, pred, M, n2, N, n_c,
                     kc, flag, chosen, chosen_pred);
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
// y[n] = training target of kept candidate n; one thread per parameter.  The
// rows are summed in 8 interleaved partial sums (row n into sum n mod 8, each
// in row order), added in a fixed tree ((s0 + s1) + (s2 + s3)) + ((s4 + s5) +
// (s6 + s7)), so eight rows' loads are in flight at once; then (2 / rows)
// times the total.
__device__ __forceinline__ float grad_term(int i, int n, const float* __restrict__ prm,
                                           const float* __restrict__ feat,
                                           const int32_t* __restrict__ idx,
                                           const float* __restrict__ pre,
                                           const float* __restrict__ pred,
                                           const float* __restrict__ y, int* rows) {
#pragma clang fp contract(off)
  const int nw1 = kHid * kIn;
  const float t = y[n];
  if (!(t == t) || t == __builtin_inff() || t == -__builtin_inff()) return 0.0f;
  ++*rows;
  const float* w2 = prm + nw1 + kHid;
  const float e = pred[n] - t;
  if (i < nw1) {
    const int u = i / kIn;
    const int d = i - u * kIn;
    const float p = pre[(int64_t)n * kHid + u];
    const float ew = e * w2[u];
    return p > 0.0f ? ew * feat[(int64_t)idx[n] * kFeatLd + d] : 0.0f;
  }
  if (i < nw1 + kHid) {
    const int u = i - nw1;
    const float p = pre[(int64_t)n * kHid + u];
    return p > 0.0f ? e * w2[u] : 0.0f;
  }
  if (i < nw1 + 2 * kHid) {
    const int u = i - nw1 - kHid;
    const float p = pre[(int64_t)n * kHid + u];
    return p > 0.0f ? e * p : 0.0f;
  }
  return e;
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ prm,
                                                       const float* __restrict__ feat,
                                                       const int32_t* __restrict__ idx,
                                                       const float* __restrict__ pre,
                                                       const float* __restrict__ pred,
                                                       const float* __restrict__ y, int N,
                                                       float* __restrict__ grad) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int total = kHid * kIn + 2 * kHid + 1;
  if (i >= total) return;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int rows = 0;
  int n = 0;
  for (; n + 8 <= N; n += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] += grad_term(i, n + q, prm, feat, idx, pre, pred, y, &rows);
  }
  for (int q = 0; n + q < N; ++q) s[q] += grad_term(i, n + q, prm, feat, idx, pre, pred, y, &rows);
  const float a = (s[0] + s[1]) + (s[2] + s[3]);
  const float b = (s[4] + s[5]) + (s[6] + s[7]);
  const float tot = a + b;
  const float f = rows > 0 ? 2.0f / (float)rows : 0.0f;
  grad[i] = tot * f;
}

__global__ __launch_bounds__(256) void mlp_update_kernel(float* __restrict__ prm,
                                                         const float* __restrict__ grad, float lr) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kHid * kIn + 2 * kHid + 1) return;
  const float step = lr * grad[i];
  prm[i] = prm[i] - step;
}

hipError_t launch_mlp_train_step(float* prm, const float* feat, const int32_t* idx, int N,
                                 const float* y, float* pre, float* pred, float* grad, float lr,
                                 hipStream_t s) {
  hipError_t e = launch_mlp_forward(prm, feat, idx, N, pre, pred, s);
  if (e != hipSuccess) return e;
  const int total = kHid * kIn + 2 * kHid + 1;
  const unsigned g = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(g), dim3(256), 0, s, prm, feat, idx, pre, pred, y, N,
                     grad);
  hipLaunchKernelGGL(mlp_update_kernel, dim3(g), dim3(256), 0, s, prm, grad, lr);
  return hipGetLastError();
}

// Kendall tau-a of the screening predictions against the evaluated fitness
// of the kept candidates, root mean squared error against their training
// targets (the standardised fitness), and the next
// generation's decision: on when `warmup` generations have trained and
// tau >= tau_min.  state = {flag, trained generations}; stats = {surrogate
// used this generation, tau, rmse, trained generations}.
__global__ __launch_bounds__(1024) void surrogate_judge_kernel(const float* __restrict__ p,
                                                               const float* __restrict__ y,
                                                               const float* __restrict__ yt, int N,
                                                               int warmup, float tau_min,
                                                               int32_t* __restrict__ state,
                                                               float* __restrict__ stats) {
  __shared__ long long part[1024];
  __shared__ float sq[1024];
  __shared__ int cnt[1024];
  const int tid = threadIdx.x;
  long long s = 0;
  for (int i = tid; i < N; i += 1024) {
    const float pi = p[i], yi = y[i];
    for (int j = i + 1; j < N; ++j) {
      const float dp = pi - p[j];
      const float dy = yi - y[j];
      const int sp = (dp > 0.0f) - (dp < 0.0f);
      const int sy = (dy > 0.0f) - (dy < 0.0f);
      s += sp * sy;
    }
  }
  float e2 = 0.0f;
  int c = 0;
  for (int i = tid; i < N; i += 1024) {
    const float d = p[i] - yt[i];
    if (d == d && d != __builtin_inff() && d != -__builtin_inff()) {
      e2 += d * d;
      ++c;
    }
  }
  part[tid] = s;
  sq[tid] = e2;
  cnt[tid] = c;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) {
      part[tid] += part[tid + off];
      sq[tid] += sq[tid + off];
      cnt[tid] += cnt[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double pairs = (double)N * (double)(N - 1) / 2.0;
    const float tau = pairs > 0 ? (float)((double)part[0] / pairs) : 0.0f;
    const float rmse = cnt[0] > 0 ? __builtin_sqrtf(sq[0] / (float)cnt[0]) : 0.0f;
    const int trained = state[1] + 1;
    stats[0] = (float)state[0];
    stats[1] = tau;
    stats[2] = rmse;
    stats[3] = (float)trained;
    state[1] = trained;
    state[0] = (trained >= warmup && tau >= tau_min) ? 1 : 0;
  }
}

hipError_t launch_surrogate_judge(const float* pred, const float* y, const float* yt, int N,
                                  int warmup, float tau_min, int32_t* state, float* stats,
                                  hipStream_t s) {
  hipLaunchKernelGGL(surrogate_judge_kernel, dim3(1), dim3(1024), 0, s, pred, y, yt, N, warmup,
                     tau_min, state, stats);
  return hipGetLastError();
}

}  // namespace leea
