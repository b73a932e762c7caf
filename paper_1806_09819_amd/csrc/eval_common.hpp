// Device pieces shared by the evaluation kernels (evaluate.hip) and the
// fused variation + evaluation kernel (fused.hip): MFMA super-steps, the
// LDS carve-up, layers 2..L and the fused fitness.
#pragma once

#include "internal.hpp"
#include "lowp.hpp"

namespace leea {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One super-step for NT column tiles; consecutive MFMAs go to different
// accumulators so none waits on the previous one's result.
template <int NT>
__device__ __forceinline__ void mfma_superstep(const float4& a, const float4 (&b)[NT],
                                               floatx4 (&acc)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(a.x, b[t].x, acc[t]);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(a.y, b[t].y, acc[t]);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(a.z, b[t].z, acc[t]);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(a.w, b[t].w, acc[t]);
}

// The same super-step with the operands swapped: acc[t] accumulates
// W X^T (neuron 16 t + 4 kq + i of row mn in lane mn + 16 kq), the layout
// the register tail reads.
template <int NT>
__device__ __forceinline__ void mfma_superstep_t(const float4& a, const float4 (&b)[NT],
                                                 floatx4 (&acc)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(b[t].x, a.x, acc[t]);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(b[t].y, a.y, acc[t]);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(b[t].z, a.z, acc[t]);
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = mfma(b[t].w, a.w, acc[t]);
}

__device__ __forceinline__ float relu_keep_nan(float v) { return v < 0.0f ? 0.0f : v; }

__device__ __forceinline__ float4 zero4() { return make_float4(0.f, 0.f, 0.f, 0.f); }

// s_waitcnt immediate: vmcnt <= n, lgkmcnt = 0, expcnt untouched.
constexpr int waitcnt_vm_lgkm0(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4); }

// global_load_lds_dwordx4: lane l copies 16 bytes from g to l + 16 l (the
// LDS base is the wave's).  A device function: kernel lambdas are compiled
// for the host too, where the builtin does not exist.
__device__ __forceinline__ void copy16_to_lds(const char* g, char* l) {
  __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
}

// Non-temporal 16-byte load, for weights that are read exactly once and
// whose cache lines no other wave shares.
__device__ __forceinline__ float4 load_once(const float* p) {
  const floatx4 v = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// One fully connected layer on the matrix cores for rows [0, 16*mtiles):
// out = act(in * W^T + bias).  `in` (LDS, row stride ldi) must hold zeros in
// columns [n_in, round16(n_in)); `out` gets zeros in [n_out, round16(n_out)).
// W is [n_out][n_in] row-major in global memory with n_in and the matrix
// offset multiples of 4.  A wave loads the weight fragments of one column
// tile once and runs G row tiles at a time on independent accumulators, so
// the matrix-core chains overlap (G = 1 for register-tight kernels); every
// output tile accumulates its K range in the same order (s = 0, 1, ... and
// e = 0..3 inside a super-step) whatever G is.  DT != 0: the weights are
// quantised as they are loaded and, for DT = 2, the sums multiplied by wfac
// before the bias (tail_and_fitness).
template <int G, int DT = 0>
static __device__ void mfma_layer(const float* in, int ldi, int n_in, float* out, int ldo, int n_out,
                           const float* W, const float* bias, bool relu, int mtiles,
                           int neg_e = 0, float wfac = 1.0f) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const int ntiles = (n_out + 15) >> 4;
  const int kss = (n_in + 15) >> 4;  // <= 16: widths are at most 256
  // (nt, mt) work of this wave: column tiles nt0, nt0 + nstep, ...; for each
  // of them row tiles mt0, mt0 + mstep, ...
  int nt0, nstep, mt0, mstep;
  if (ntiles >= 4) {
    nt0 = wave, nstep = 4, mt0 = 0, mstep = 1;
  } else {
    const int per = 4 / ntiles;           // waves sharing a column tile
    nt0 = wave % ntiles, nstep = 4, mt0 = wave / ntiles, mstep = per;
    if (wave >= per * ntiles) nt0 = ntiles;  // idle wave (ntiles == 3)
  }
  for (int nt = nt0; nt < ntiles; nt += nstep) {
    const int n = nt * 16 + mn;
    const bool nv = n < n_out;
    const float* wr = W + (int64_t)(nv ? n : 0) * n_in;
    // weight fragments: every lane loads from a valid address (row 0 for
    // columns past n_out, column 0 past n_in) and masks the value, so the
    // loads need no per-lane branch; s < kss is uniform across the wave
    float4 bf[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      bf[s] = zero4();
      if (s < kss) {
        const int k = 16 * s + 4 * kq;
        const bool kv = k < n_in;
        float4 v = *reinterpret_cast<const float4*>(wr + (kv ? k : 0));
        if constexpr (DT != 0) {
          v.x = quantize<DT>(v.x, neg_e);
          v.y = quantize<DT>(v.y, neg_e);
          v.z = quantize<DT>(v.z, neg_e);
          v.w = quantize<DT>(v.w, neg_e);
        }
        if (nv && kv) bf[s] = v;
      }
    }
    const float bb = nv ? bias[n] : 0.0f;
    for (int mt = mt0; mt < mtiles; mt += G * mstep) {
      floatx4 acc[G];
      const float* arow[G];
      bool mv[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        acc[g] = floatx4{0.f, 0.f, 0.f, 0.f};
        const int m = mt + g * mstep;
        mv[g] = m < mtiles;
        arow[g] = in + ((mv[g] ? m : mt) * 16 + mn) * ldi + 4 * kq;
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (s < kss) {
          float4 a[G];
#pragma unroll
          for (int g = 0; g < G; ++g) a[g] = *reinterpret_cast<const float4*>(arow[g] + 16 * s);
#pragma unroll
          for (int g = 0; g < G; ++g) acc[g] = mfma(a[g].x, bf[s].x, acc[g]);
#pragma unroll
          for (int g = 0; g < G; ++g) acc[g] = mfma(a[g].y, bf[s].y, acc[g]);
#pragma unroll
          for (int g = 0; g < G; ++g) acc[g] = mfma(a[g].z, bf[s].z, acc[g]);
#pragma unroll
          for (int g = 0; g < G; ++g) acc[g] = mfma(a[g].w, bf[s].w, acc[g]);
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (mv[g]) {
          const int m = mt + g * mstep;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float v = acc[g][i];
            if constexpr (DT == 2) v = v * wfac;
            v = v + bb;
            if (relu) v = relu_keep_nan(v);
            out[(m * 16 + 4 * kq + i) * ldo + n] = nv ? v : 0.0f;
          }
        }
      }
    }
  }
}

// mfma_layer with as many row tiles per group as this wave has (up to GMAX):
// a wave with fewer row tiles than the group size would multiply copies of
// its last tile for nothing.  The result does not depend on the group size.
template <int GMAX, int DT = 0>
static __device__ void mfma_layer_fit(const float* in, int ldi, int n_in, float* out, int ldo,
                                      int n_out, const float* W, const float* bias, bool relu,
                                      int mtiles, int neg_e = 0, float wfac = 1.0f) {
  const int wave = threadIdx.x >> 6;
  const int ntiles = (n_out + 15) >> 4;
  int mt0 = 0, mstep = 1;
  if (ntiles < 4) {
    mstep = 4 / ntiles;
    mt0 = wave / ntiles;
  }
  const int r = mt0 < mtiles ? (mtiles - mt0 + mstep - 1) / mstep : 0;
  if constexpr (GMAX >= 4) {
    if (r >= 3) {
      mfma_layer<4, DT>(in, ldi, n_in, out, ldo, n_out, W, bias, relu, mtiles, neg_e, wfac);
      return;
    }
  }
  if constexpr (GMAX >= 2) {
    if (r == 2) {
      mfma_layer<2, DT>(in, ldi, n_in, out, ldo, n_out, W, bias, relu, mtiles, neg_e, wfac);
      return;
    }
  }
  mfma_layer<1, DT>(in, ldi, n_in, out, ldo, n_out, W, bias, relu, mtiles, neg_e, wfac);
}

// The same layer on VALU, for hidden widths that are not multiples of 4.
template <int DT = 0>
static __device__ void scalar_layer(const float* in, int ldi, int n_in, float* out, int ldo, int n_out,
                             const float* W, const float* bias, bool relu, int rows,
                             int neg_e = 0, float wfac = 1.0f) {
  const int n16 = (n_out + 15) & ~15;
  for (int idx = threadIdx.x; idx < rows * n16; idx += blockDim.x) {
    const int m = idx / n16;
    const int n = idx - m * n16;
    float v = 0.0f;
    if (n < n_out) {
      const float* a = in + m * ldi;
      const float* w = W + (int64_t)n * n_in;
      for (int k = 0; k < n_in; ++k) v += a[k] * quantize<DT>(w[k], neg_e);
      if constexpr (DT == 2) v = v * wfac;
      v += bias[n];
      if (relu) v = relu_keep_nan(v);
    }
    out[m * ldo + n] = v;
  }
}

// Layers 2..L on the LDS tile of layer-1 activations, then the per-sample
// fitness of the first `rows` rows: log-likelihood (z_y - max z) -
// log sum_k exp(z_k - max z) (Eq. 1, left side) and correctness (first
// maximal logit equals the label); a label outside [0, d) gives NaN.  The
// row sums go to *out in a fixed order (deterministic).
// Layer weights come from tw: W_l at tw + (woff[l] - toff) (the genome in
// global memory with toff = 0, or a copy of the genome's tail in LDS).
// G: row tiles per matrix-core group in the hidden layers (see mfma_layer).
// y == nullptr: the label of row threadIdx.x is ylab (rows <= blockDim.x),
// loaded by the caller ahead of time.  DT: arithmetic of the weights of
// layers 2..L (0 float32; 1 rounded to bfloat16; 2 E4M3 with a power-of-two
// scale per layer from its largest magnitude, whose factor multiplies the
// layer's sums before the bias: ts.amax[l] when given, else reduced here);
// the activations stay float32.  Every thread of the workgroup calls it.
template <int G, int DT = 0>
static __device__ float2 tail_and_fitness(float* lds, const EvalLds& lo, const NetDesc& nd,
                                 const float* tw, int64_t toff, int mtiles, int rows,
                                 int m0, const int32_t* __restrict__ y, bool tail_vec,
                                 float2* __restrict__ out, int ylab = 0,
                                 const TailScales& ts = TailScales{{}, 0}) {
  const float* in = lds + lo.h1;
  int ldi = lo.ld1;
  float* dst = lds + lo.ta;
  for (int l = 1; l < nd.L; ++l) {
    const float* W = tw + (nd.woff[l] - toff);
    const float* bias = tw + (nd.boff[l] - toff);
    const bool relu = l < nd.L - 1;
    int neg_e = 0;
    float wfac = 1.0f;
    if constexpr (DT == 2)
      tail_fp8_scale(ts.given ? ts.amax[l] : block_amax(W, nd.w[l] * nd.w[l + 1]), neg_e, wfac);
    if (tail_vec)
      mfma_layer_fit<G, DT>(in, ldi, nd.w[l], dst, lo.ldt, nd.w[l + 1], W, bias, relu, mtiles,
                            neg_e, wfac);
    else
      scalar_layer<DT>(in, ldi, nd.w[l], dst, lo.ldt, nd.w[l + 1], W, bias, relu, 16 * mtiles,
                       neg_e, wfac);
    __syncthreads();
    in = dst;
    ldi = lo.ldt;
    dst = (dst == lds + lo.ta) ? lds + lo.h1 : lds + lo.ta;
  }
  const int d = nd.w[nd.L];
  float* ll = lds + lo.ll;
  int* cor = reinterpret_cast<int*>(lds + lo.cor);
  for (int m = threadIdx.x; m < rows; m += blockDim.x) {
    const float* z = in + m * ldi;
    const int yy = y ? y[m0 + m] : ylab;
    float mx = z[0];
    int best = 0;
    for (int k = 1; k < d; ++k)
      if (z[k] > mx) {
        mx = z[k];
        best = k;
      }
    float s = 0.0f;
    for (int k = 0; k < d; ++k) s += expf(z[k] - mx);
    ll[m] = (yy >= 0 && yy < d) ? (z[yy] - mx) - logf(s) : __builtin_nanf("");
    cor[m] = (best == yy) ? 1 : 0;
  }
  __syncthreads();
  float2 r = make_float2(0.0f, 0.0f);
  if (threadIdx.x < 64) {
    float s = 0.0f;
    int c = 0;
    for (int m = threadIdx.x; m < rows; m += 64) {
      s += ll[m];
      c += cor[m];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_xor(s, off);
      c += __shfl_xor(c, off);
    }
    if (threadIdx.x == 0) {
      r = make_float2(s, (float)c);
      *out = r;
    }
  }
  return r;  // thread 0: the partial it wrote
}


}  // namespace leea
