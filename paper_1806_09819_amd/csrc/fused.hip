// Fused variation + evaluation for small batches (b <= 16).
//
// At small batch sizes a generation is bandwidth-bound twice over: the
// variation kernel reads the parents and writes the children (Algorithm 1,
// crossover / mutation / union), then the evaluation streams the children
// back (Algorithm 1, last line).  Here one workgroup per child builds the
// child's genes from its parents in registers -- with exactly the operator
// arithmetic of the variation kernel (vary_common.hpp) -- writes them once,
// and feeds the layer-1 genes straight into the MFMA evaluation of the
// small-batch kernel, in the same MFMA issue order and the same fixed-order
// K-partial reduction, so fitness and children are bit-identical to the
// separate select -> crossover_mutate -> evaluate path.  The genes after
// layer 1's weights (b_1, W_2, b_2, ...) are kept in LDS for the tail layers.
#include "eval_common.hpp"
#include "vary_common.hpp"

namespace leea {

template <int NT>
__global__ __launch_bounds__(256, 3) void vary_eval_small_kernel(
    const float* __restrict__ cur, float* __restrict__ nxt, const int4* __restrict__ plan,
    NetDesc nd, float sigma, uint64_t thr, Key key, uint32_t gen,
    const float* __restrict__ sig_cur, float* __restrict__ sig_next, float tau, int xo_kind,
    int pop, uint32_t mul, const float* __restrict__ x, const int32_t* __restrict__ y, int b,
    float2* __restrict__ partial, EvalLds lo, int tail_lds, int tail_vec) {
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int j = (int)(((uint64_t)blockIdx.x * mul) % (uint32_t)pop);
  const int4 pl = plan[j];
  const int op = pl.x;
  VaryParams vp;
  vp.sigma = sigma;
  if (sig_cur) {
    vp.sigma = child_sigma(pl, sig_cur, key, gen, (uint32_t)j, tau);
    if (tid == 0) sig_next[j] = vp.sigma;
  }
  vp.all = thr >= (1ull << 32);
  vp.t32 = (uint32_t)thr;
  vp.key = key;
  vp.gen = gen;
  vp.slot = (uint32_t)j;
  vp.genes = nd.genes;
  const float4* __restrict__ pa = reinterpret_cast<const float4*>(cur + (int64_t)pl.y * nd.stride);
  const float4* __restrict__ pb = reinterpret_cast<const float4*>(cur + (int64_t)pl.z * nd.stride);
  float4* __restrict__ pc = reinterpret_cast<float4*>(nxt + (int64_t)j * nd.stride);

  // genes from b_1 on: child -> HBM and LDS (tail weights for layers 2..L)
  const int64_t T0 = nd.boff[0];
  const int64_t n4 = nd.stride >> 2;
  float* tl = lds + tail_lds;
  for (int64_t f = (T0 >> 2) + tid; f < n4; f += 256) {
    const float4 a = pa[f];
    float4 c;
    if (op == kOpElite) {
      c = a;
    } else if (op == kOpCross) {
      const float4 bb = pb[f];
      c = xo_kind == 0 ? xo_uniform4(vp, 4 * f, a, bb) : xo_arith4(a, bb);
    } else {
      c = mutate4(vp, f, a);
    }
    store_stream(pc + f, c);
    *reinterpret_cast<float4*>(tl + (4 * f - T0)) = c;
  }

  // layer 1: waves split K (super-step s = wave, wave+4, ...) exactly as in
  // the small-batch evaluation kernel; each weight float4 is a child gene
  // block built from the parents on the fly
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const bool xv = mn < b;
  const float* __restrict__ xrow = x + (int64_t)(xv ? mn : 0) * n0;
  int rowf[NT];  // float4 index of the row start (genomes are < 2^31 floats)
  bool rvalid[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = t * 16 + mn;
    rvalid[t] = r < n1;
    rowf[t] = (int)((nd.woff[0] + (int64_t)(rvalid[t] ? r : 0) * n0) >> 2);
  }
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nss = (n0 + 15) >> 4;
  for (int s = wave; s < nss; s += 4) {
    const int k = 16 * s + 4 * kq;
    const bool kv = k < n0;
    const float4 xa = (xv && kv) ? *reinterpret_cast<const float4*>(xrow + k) : zero4();
    float4 wa[NT], wb2[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) wa[t] = (rvalid[t] && kv) ? pa[rowf[t] + (k >> 2)] : zero4();
    if (op == kOpCross) {
#pragma unroll
      for (int t = 0; t < NT; ++t) wb2[t] = (rvalid[t] && kv) ? pb[rowf[t] + (k >> 2)] : zero4();
    }
    // one tile at a time: child genes, store, then its four MFMAs (the same
    // per-accumulator order as the evaluation kernel's super-step); the
    // scheduling barrier keeps the tiles' random-number chains from being
    // interleaved, which would multiply the live registers
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int f = rowf[t] + (k >> 2);
      const bool v = rvalid[t] && kv;
      float4 c = wa[t];
      if (op == kOpCross)
        c = xo_kind == 0 ? xo_uniform4(vp, 4 * f, wa[t], wb2[t]) : xo_arith4(wa[t], wb2[t]);
      else if (op == kOpMut && v)
        c = mutate4(vp, f, wa[t]);
      if (v) store_stream(pc + f, c);
      acc[t] = mfma(xa.x, c.x, acc[t]);
      acc[t] = mfma(xa.y, c.y, acc[t]);
      acc[t] = mfma(xa.z, c.z, acc[t]);
      acc[t] = mfma(xa.w, c.w, acc[t]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // K-partial tiles summed in the order ((p0 + p1) + p2) + p3, then the
  // bias: tiles 1 and 2 go through LDS buffers A and B, tile 3 through A
  const int ld1 = lo.ld1;
  float* bufA = lds;
  float* bufB = lds + 16 * ld1;
  auto put = [&](float* buf) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) buf[(4 * kq + i) * ld1 + t * 16 + mn] = acc[t][i];
  };
  auto addin = [&](const float* buf) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[t][i] += buf[(4 * kq + i) * ld1 + t * 16 + mn];
  };
  if (wave == 1) put(bufA);
  if (wave == 2) put(bufB);
  __syncthreads();
  if (wave == 0) {
    addin(bufA);
    addin(bufB);
  }
  __syncthreads();
  if (wave == 3) put(bufA);
  __syncthreads();
  if (wave == 0) {
    addin(bufA);
    const bool hidden = nd.L > 1;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = t * 16 + mn;
      const float bb = n < n1 ? tl[n] : 0.0f;  // b_1 is the first tail gene
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = 0.0f;
        if (n < n1) {
          v = acc[t][i] + bb;
          if (hidden) v = relu_keep_nan(v);
        }
        lds[lo.h1 + (4 * kq + i) * ld1 + n] = v;
      }
    }
  }
  __syncthreads();
  tail_and_fitness<1>(lds, lo, nd, tl, T0, 1, b, 0, y, tail_vec != 0, partial + j);
}

// Usable when the batch is small, the tail layers run on MFMA and the genes
// after layer 1's weights fit in LDS next to the evaluation buffers.
static int fused_lds_floats(const NetDesc& nd, EvalLds* out, int* tail_lds) {
  EvalLds lo;
  lo.ld1 = ((nd.w[1] + 15) & ~15) + 4;
  int ldt = 4;
  for (int l = 2; l <= nd.L; ++l) ldt = nd.w[l] > ldt ? nd.w[l] : ldt;
  lo.ldt = ((ldt + 15) & ~15) + 4;
  const int ldmax = lo.ld1 > lo.ldt ? lo.ld1 : lo.ldt;
  lo.h1 = 0;
  lo.ta = 16 * ldmax;
  lo.ll = lo.ta + 16 * lo.ldt;
  lo.cor = lo.ll + 16;
  lo.total = lo.cor + 16;
  int base = lo.total > 2 * 16 * lo.ld1 ? lo.total : 2 * 16 * lo.ld1;
  base = (base + 3) & ~3;
  const int64_t tail = nd.stride - nd.boff[0];
  if (out) *out = lo;
  if (tail_lds) *tail_lds = base;
  return base + (int)tail;
}

bool fused_supported(const NetDesc& nd, int b) {
  if (b > 16 || nd.L < 2) return false;
  for (int l = 1; l < nd.L; ++l)
    if (nd.w[l] % 4 != 0) return false;
  if (nd.boff[0] % 4 != 0) return false;
  const int64_t tail = nd.stride - nd.boff[0];
  if (tail > 24576) return false;
  return (size_t)fused_lds_floats(nd, nullptr, nullptr) * 4 <= 160 * 1024;
}

template <int NT>
static hipError_t launch_fused_nt(const float* cur, float* nxt, const int4* plan,
                                  const NetDesc& nd, int pop, int crossover, float sigma,
                                  uint64_t thr, const Key& key, uint32_t gen,
                                  const float* sig_cur, float* sig_next, float tau,
                                  uint32_t mul, const float* x, const int32_t* y, int b,
                                  float2* partial, hipStream_t s) {
  EvalLds lo;
  int tail_lds = 0;
  const size_t bytes = (size_t)fused_lds_floats(nd, &lo, &tail_lds) * 4;
  if (bytes > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)vary_eval_small_kernel<NT>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(vary_eval_small_kernel<NT>, dim3((unsigned)pop), dim3(256), bytes, s, cur,
                     nxt, plan, nd, sigma, thr, key, gen, sig_cur, sig_next, tau, crossover, pop,
                     mul, x, y, b, partial, lo, tail_lds, 1);
  return hipGetLastError();
}

hipError_t launch_vary_eval(const float* cur, float* nxt, const int4* plan, const NetDesc& nd,
                            int pop, int crossover, float sigma, uint64_t thr, const Key& key,
                            uint32_t gen, const float* sig_cur, float* sig_next, float tau,
                            const float* x, const int32_t* y, int b, float2* partial,
                            hipStream_t s) {
  const uint32_t mul = slot_multiplier(pop);
  switch ((nd.w[1] + 15) / 16) {
#define LEEA_FUSED_CASE(N)                                                                      \
  case N:                                                                                       \
    return launch_fused_nt<N>(cur, nxt, plan, nd, pop, crossover, sigma, thr, key, gen, sig_cur, \
                              sig_next, tau, mul, x, y, b, partial, s);
    LEEA_FUSED_CASE(1) LEEA_FUSED_CASE(2) LEEA_FUSED_CASE(3) LEEA_FUSED_CASE(4)
    LEEA_FUSED_CASE(5) LEEA_FUSED_CASE(6) LEEA_FUSED_CASE(7) LEEA_FUSED_CASE(8)
    LEEA_FUSED_CASE(9) LEEA_FUSED_CASE(10) LEEA_FUSED_CASE(11) LEEA_FUSED_CASE(12)
    LEEA_FUSED_CASE(13) LEEA_FUSED_CASE(14) LEEA_FUSED_CASE(15) LEEA_FUSED_CASE(16)
#undef LEEA_FUSED_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace leea
