// Population-batched forward pass with fused fitness (paper section 3.3:
// batch the whole population into tensor products; Eq. 1 fitness).
//
// Layer 1 of every network reads the same minibatch X [b][n0], so for the
// whole population it is one dense product X * [W1_1 .. W1_P]^T (M = b,
// N = P * n1, K = n0).  One workgroup owns one individual's n1 columns
// (all of its layer-1 neurons) for up to 64 batch rows and accumulates them
// on the matrix cores with v_mfma_f32_16x16x4_f32 (FP32 in, FP32
// accumulate).  Keeping all n1 columns of an individual in one workgroup
// lets the rest of the network and the fitness run in the same kernel on
// the layer-1 tile held in LDS: nothing but two floats per (individual,
// row tile) ever goes back to HBM.
//
// MFMA 16x16x4 f32 operand layout (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; the 4 accumulator values of lane l are
// D[4*(l/16)+i][l%16].  A float4 load of 4 consecutive k per lane feeds 4
// MFMAs: in the e-th one lane (m, kq) contributes k = k0 + 4*kq + e, so the
// four MFMAs together cover k0 .. k0+15 (one "super-step").
//
// Two layer-1 schemes:
// * small batch (b <= 16): one workgroup per individual, 4 waves split the
//   K range; weights stream straight from HBM into registers (each weight
//   is read exactly once; the kernel is bandwidth-bound), X sits in LDS.
// * large batch: workgroup = (row tile of 64, individual); 4 waves split the
//   rows; 16-wide K chunks of W and X are staged through double-buffered
//   LDS so each weight fragment read from HBM serves all 4 waves.
#include "internal.hpp"

namespace leea {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// One super-step for NT column tiles; consecutive MFMAs go to different
// accumulators so none waits on the previous one's result.
template <int NT>
__device__ __forceinline__ void mfma_superstep(const float4& a, const float4 (&b)[NT],
                                               floatx4 (&acc)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t)
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[t].x, acc[t], 0, 0, 0);
#pragma unroll
  for (int t = 0; t < NT; ++t)
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[t].y, acc[t], 0, 0, 0);
#pragma unroll
  for (int t = 0; t < NT; ++t)
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b[t].z, acc[t], 0, 0, 0);
#pragma unroll
  for (int t = 0; t < NT; ++t)
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b[t].w, acc[t], 0, 0, 0);
}

__device__ __forceinline__ float relu_keep_nan(float v) { return v < 0.0f ? 0.0f : v; }

// LDS carve-up shared by both kernels (offsets in floats, set on the host).
struct EvalLds {
  int h1;      // [rows][ld1] layer-1 activations
  int ld1;
  int buf_a;   // [16][ldt] tail activations (ping)
  int buf_b;   // [16][ldt] (pong)
  int ldt;
  int ll;      // [rows] per-sample log-likelihood
  int cor;     // [rows] per-sample correctness (int)
  int total;   // floats of dynamic LDS
};

// Layers 2..L and the fitness of `rows` samples whose layer-1 activations
// are in LDS; writes ll[m] and cor[m] for m < rows.  Per-sample
// log-likelihood: (z_y - max z) - log sum_k exp(z_k - max z) (Eq. 1, left
// side); correct iff the first maximal logit is the label.
__device__ void tail_fitness(const float* __restrict__ genome, const NetDesc& nd,
                             float* lds, const EvalLds& lo, int rows, int m0,
                             const int32_t* __restrict__ y) {
  const int tid = threadIdx.x;
  const int d = nd.w[nd.L];
  float* ll = lds + lo.ll;
  int* cor = reinterpret_cast<int*>(lds + lo.cor);
  for (int r0 = 0; r0 < rows; r0 += 16) {
    const int rc = rows - r0 < 16 ? rows - r0 : 16;
    const float* in = lds + lo.h1 + r0 * lo.ld1;
    int ldin = lo.ld1;
    float* out = lds + lo.buf_a;
    for (int l = 1; l < nd.L; ++l) {
      const int n_in = nd.w[l];
      const int n_out = nd.w[l + 1];
      const float* __restrict__ W = genome + nd.woff[l];
      const float* __restrict__ bias = genome + nd.boff[l];
      const bool last = (l == nd.L - 1);
      for (int idx = tid; idx < rc * n_out; idx += blockDim.x) {
        const int m = idx / n_out;
        const int n = idx - m * n_out;
        const float* a = in + m * ldin;
        const float* w = W + (int64_t)n * n_in;
        float acc = 0.0f;
        for (int k = 0; k < n_in; ++k) acc += a[k] * w[k];
        acc += bias[n];
        out[m * lo.ldt + n] = last ? acc : relu_keep_nan(acc);
      }
      __syncthreads();
      in = out;
      ldin = lo.ldt;
      out = (out == lds + lo.buf_a) ? lds + lo.buf_b : lds + lo.buf_a;
    }
    for (int m = tid; m < rc; m += blockDim.x) {
      const float* z = in + m * ldin;
      const int yy = y[m0 + r0 + m];
      float mx = z[0];
      int best = 0;
      for (int k = 1; k < d; ++k)
        if (z[k] > mx) {
          mx = z[k];
          best = k;
        }
      float s = 0.0f;
      for (int k = 0; k < d; ++k) s += expf(z[k] - mx);
      float v;
      if (yy >= 0 && yy < d)
        v = (z[yy] - mx) - logf(s);
      else
        v = __builtin_nanf("");
      ll[r0 + m] = v;
      cor[r0 + m] = (best == yy) ? 1 : 0;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void write_partial(float* lds, const EvalLds& lo, int rows,
                                              float2* __restrict__ out) {
  if (threadIdx.x == 0) {
    const float* ll = lds + lo.ll;
    const int* cor = reinterpret_cast<const int*>(lds + lo.cor);
    float s = 0.0f;
    int c = 0;
    for (int m = 0; m < rows; ++m) {
      s += ll[m];
      c += cor[m];
    }
    *out = make_float2(s, (float)c);
  }
}

// ---------------------------------------------------------------- small b --
template <int NT>
__global__ __launch_bounds__(256) void eval_small_kernel(const float* __restrict__ genomes,
                                                         NetDesc nd, const float* __restrict__ x,
                                                         const int32_t* __restrict__ y, int b,
                                                         float2* __restrict__ partial,
                                                         EvalLds lo, int ldx, int part_off,
                                                         int ldp) {
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int j = blockIdx.x;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int n0p = (n0 + 15) & ~15;
  const int c4 = n0p >> 2;

  // X rows into LDS, zero beyond b and beyond n0
  for (int idx = tid; idx < 16 * c4; idx += 256) {
    const int m = idx / c4;
    const int c = idx - m * c4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (m < b && 4 * c < n0) v = reinterpret_cast<const float4*>(x + (int64_t)m * n0)[c];
    *reinterpret_cast<float4*>(lds + m * ldx + 4 * c) = v;
  }
  __syncthreads();

  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};

  const float* wrow[NT];
  bool rvalid[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = t * 16 + mn;
    rvalid[t] = r < n1;
    wrow[t] = genome + nd.woff[0] + (int64_t)(rvalid[t] ? r : 0) * n0;
  }
  const int nss = n0p >> 4;
  float4 xa, wb[NT];
  auto load = [&](int s, float4& xo, float4* wo) {
    const int k = 16 * s + 4 * kq;
    xo = *reinterpret_cast<const float4*>(lds + mn * ldx + k);
    const bool kv = k < n0;
#pragma unroll
    for (int t = 0; t < NT; ++t)
      wo[t] = (rvalid[t] && kv) ? *reinterpret_cast<const float4*>(wrow[t] + k)
                                : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  int s = wave;
  if (s < nss) load(s, xa, wb);
  for (; s < nss; s += 4) {
    float4 xn, wn[NT];
    if (s + 4 < nss) load(s + 4, xn, wn);
    mfma_superstep<NT>(xa, wb, acc);
    if (s + 4 < nss) {
      xa = xn;
#pragma unroll
      for (int t = 0; t < NT; ++t) wb[t] = wn[t];
    }
  }
  __syncthreads();  // every wave is done with X in LDS

  // cross-wave reduction of the 4 K-partial tiles, fixed order
  float* part = lds + part_off;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      part[(wave * 16 + 4 * kq + i) * ldp + t * 16 + mn] = acc[t][i];
  __syncthreads();
  const float* __restrict__ b1 = genome + nd.boff[0];
  const bool hidden = nd.L > 1;
  for (int idx = tid; idx < b * n1; idx += 256) {
    const int m = idx / n1;
    const int n = idx - m * n1;
    float v = part[(0 * 16 + m) * ldp + n] + part[(1 * 16 + m) * ldp + n];
    v += part[(2 * 16 + m) * ldp + n];
    v += part[(3 * 16 + m) * ldp + n];
    v += b1[n];
    lds[lo.h1 + m * lo.ld1 + n] = hidden ? relu_keep_nan(v) : v;
  }
  __syncthreads();
  tail_fitness(genome, nd, lds, lo, b, 0, y);
  write_partial(lds, lo, b, partial + j);
}

// ---------------------------------------------------------------- large b --
template <int NT>
__global__ __launch_bounds__(256) void eval_large_kernel(const float* __restrict__ genomes,
                                                         NetDesc nd, const float* __restrict__ x,
                                                         const int32_t* __restrict__ y, int b,
                                                         float2* __restrict__ partial,
                                                         EvalLds lo, int n_mt) {
  extern __shared__ float lds[];
  constexpr int NR = NT * 16;             // staged weight rows
  constexpr int WBUF = 4 * NR * 4;        // floats per W staging buffer
  constexpr int XBUF = 4 * 64 * 4;        // floats per X staging buffer
  constexpr int WITEMS = NR * 4;          // float4 items of one W chunk
  constexpr int WPT = (WITEMS + 255) / 256;
  const int tid = threadIdx.x;
  const int mt = blockIdx.x;
  const int j = blockIdx.y;
  const int m0 = mt * 64;
  const int rows = b - m0 < 64 ? b - m0 : 64;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const float* __restrict__ W1 = genome + nd.woff[0];
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int nss = (n0 + 15) >> 4;
  float* wst = lds;                // [2][4][NR][4]
  float* xst = lds + 2 * WBUF;     // [2][4][64][4]

  float4 wr[WPT];
  float4 xr;
  auto gload = [&](int s) {
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int it = tid + 256 * q;
      const int r = it >> 2;
      const int k = 16 * s + 4 * (it & 3);
      wr[q] = (it < WITEMS && r < n1 && k < n0)
                  ? *reinterpret_cast<const float4*>(W1 + (int64_t)r * n0 + k)
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int m = tid >> 2;
    const int k = 16 * s + 4 * (tid & 3);
    xr = (m < rows && k < n0)
             ? *reinterpret_cast<const float4*>(x + (int64_t)(m0 + m) * n0 + k)
             : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int it = tid + 256 * q;
      if (it < WITEMS)
        *reinterpret_cast<float4*>(wst + buf * WBUF + ((it & 3) * NR + (it >> 2)) * 4) = wr[q];
    }
    *reinterpret_cast<float4*>(xst + buf * XBUF + ((tid & 3) * 64 + (tid >> 2)) * 4) = xr;
  };

  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};

  gload(0);
  sstore(0);
  __syncthreads();
  for (int s = 0; s < nss; ++s) {
    const int buf = s & 1;
    if (s + 1 < nss) gload(s + 1);
    const float4 xa =
        *reinterpret_cast<const float4*>(xst + buf * XBUF + (kq * 64 + wave * 16 + mn) * 4);
    float4 wb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
      wb[t] = *reinterpret_cast<const float4*>(wst + buf * WBUF + (kq * NR + t * 16 + mn) * 4);
    mfma_superstep<NT>(xa, wb, acc);
    if (s + 1 < nss) sstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue: bias + ReLU into the LDS layer-1 tile (staging is dead now)
  const float* __restrict__ b1 = genome + nd.boff[0];
  const bool hidden = nd.L > 1;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int n = t * 16 + mn;
    if (n < n1) {
      const float bb = b1[n];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = wave * 16 + 4 * kq + i;
        const float v = acc[t][i] + bb;
        lds[lo.h1 + m * lo.ld1 + n] = hidden ? relu_keep_nan(v) : v;
      }
    }
  }
  __syncthreads();
  tail_fitness(genome, nd, lds, lo, rows, m0, y);
  write_partial(lds, lo, rows, partial + (int64_t)j * n_mt + mt);
}

// -------------------------------------------------------------- dispatch --

static EvalLds tail_layout(const NetDesc& nd, int rows, int base) {
  EvalLds lo;
  int ldt = 4;
  for (int l = 2; l <= nd.L; ++l) ldt = nd.w[l] > ldt ? nd.w[l] : ldt;
  ldt = ((ldt + 3) & ~3) + 4;
  const int n1p = ((nd.w[1] + 15) & ~15);
  lo.ld1 = n1p + 4;
  lo.h1 = base;
  lo.buf_a = lo.h1 + rows * lo.ld1;
  lo.buf_b = lo.buf_a + 16 * ldt;
  lo.ldt = ldt;
  lo.ll = lo.buf_b + 16 * ldt;
  lo.cor = lo.ll + rows;
  lo.total = lo.cor + rows;
  return lo;
}

static bool small_fits(const NetDesc& nd, int b) {
  if (b > 16) return false;
  const int n0p = (nd.w[0] + 15) & ~15;
  return 16 * (n0p + 4) * 4 <= 64 * 1024;
}

int eval_mtiles(const NetDesc& nd, int b) { return small_fits(nd, b) ? 1 : (b + 63) / 64; }

template <int NT>
static hipError_t launch_nt(const float* genomes, const NetDesc& nd, int pop, const float* x,
                            const int32_t* y, int b, float2* partial, hipStream_t s) {
  if (small_fits(nd, b)) {
    const int n0p = (nd.w[0] + 15) & ~15;
    const int ldx = n0p + 4;
    const int ldp = NT * 16 + 4;
    const int part_off = 0;
    EvalLds lo = tail_layout(nd, 16, part_off + 4 * 16 * ldp);
    int total = lo.total > 16 * ldx ? lo.total : 16 * ldx;
    lo.total = total;
    const size_t bytes = (size_t)total * 4;
    if (bytes > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute((const void*)eval_small_kernel<NT>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)bytes);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(eval_small_kernel<NT>, dim3((unsigned)pop), dim3(256), bytes, s, genomes,
                       nd, x, y, b, partial, lo, ldx, part_off, ldp);
  } else {
    const int n_mt = (b + 63) / 64;
    const int staging = 2 * (4 * NT * 16 * 4) + 2 * (4 * 64 * 4);
    EvalLds lo = tail_layout(nd, 64, 0);
    lo.total = lo.total > staging ? lo.total : staging;
    const size_t bytes = (size_t)lo.total * 4;
    if (bytes > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute((const void*)eval_large_kernel<NT>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)bytes);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(eval_large_kernel<NT>, dim3((unsigned)n_mt, (unsigned)pop), dim3(256),
                       bytes, s, genomes, nd, x, y, b, partial, lo, n_mt);
  }
  return hipGetLastError();
}

hipError_t launch_evaluate(const float* genomes, const NetDesc& nd, int pop, const float* x,
                           const int32_t* y, int b, float2* partial, hipStream_t s) {
  const int nt = (nd.w[1] + 15) / 16;
  switch (nt) {
#define LEEA_NT_CASE(N) \
  case N:               \
    return launch_nt<N>(genomes, nd, pop, x, y, b, partial, s);
    LEEA_NT_CASE(1) LEEA_NT_CASE(2) LEEA_NT_CASE(3) LEEA_NT_CASE(4)
    LEEA_NT_CASE(5) LEEA_NT_CASE(6) LEEA_NT_CASE(7) LEEA_NT_CASE(8)
    LEEA_NT_CASE(9) LEEA_NT_CASE(10) LEEA_NT_CASE(11) LEEA_NT_CASE(12)
    LEEA_NT_CASE(13) LEEA_NT_CASE(14) LEEA_NT_CASE(15) LEEA_NT_CASE(16)
#undef LEEA_NT_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Fitness = (sum of per-sample log-likelihoods) / b, accuracy = correct / b,
// summed over row tiles in order; then the inheritance weighting
// f_adj = fl(fl((1 - alpha) f_inh) + fl(alpha f)) (section 3.1).
__global__ void finalize_kernel(const float2* __restrict__ partial, int pop, int n_mt, int b,
                                const float* __restrict__ f_inh, int use_inh, float alpha,
                                float* f_adj, float* f_raw, float* acc, float* f_adj_out,
                                float* f_raw_out, float* acc_out) {
#pragma clang fp contract(off)
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= pop) return;
  float s = 0.0f, c = 0.0f;
  for (int t = 0; t < n_mt; ++t) {
    const float2 p = partial[(int64_t)j * n_mt + t];
    s += p.x;
    c += p.y;
  }
  const float fb = (float)b;
  const float f = s / fb;
  const float a = c / fb;
  float fa = f;
  if (use_inh) {
    const float oma = 1.0f - alpha;
    const float t1 = oma * f_inh[j];
    const float t2 = alpha * f;
    fa = t1 + t2;
  }
  if (f_adj) f_adj[j] = fa;
  if (f_raw) f_raw[j] = f;
  if (acc) acc[j] = a;
  if (f_adj_out) f_adj_out[j] = fa;
  if (f_raw_out) f_raw_out[j] = f;
  if (acc_out) acc_out[j] = a;
}

hipError_t launch_finalize(const float2* partial, int pop, int n_mt, int b, const float* f_inh,
                           int use_inh, float alpha, float* f_adj, float* f_raw, float* acc,
                           float* f_adj_out, float* f_raw_out, float* acc_out, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((pop + 255) / 256)), dim3(256), 0, s,
                     partial, pop, n_mt, b, f_inh, use_inh, alpha, f_adj, f_raw, acc, f_adj_out,
                     f_raw_out, acc_out);
  return hipGetLastError();
}

}  // namespace leea
