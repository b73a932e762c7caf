// Population forward pass with the first layer on the bfloat16 / FP8 matrix
// cores (batches above 16 rows; smaller batches use the FP32 small-batch
// kernel on quantised values, which is bandwidth-bound either way).
//
// Same decomposition as the FP32 large-batch kernel (section 3.3: one
// shared-input product X * [W1_1 .. W1_P]^T, then each network's tail and
// fitness), with these differences:
// * v_mfma_f32_16x16x32_{bf16,fp8_fp8}: lane l supplies A[l%16][8(l/16)+e]
//   and B[8(l/16)+e][l%16] for e = 0..7 (16 bytes of bf16, 8 bytes of fp8)
//   and receives D[4(l/16)+i][l%16]; one instruction covers a 32-wide K
//   chunk, so each staged chunk costs one MFMA per (row tile, column tile).
// * W_1 is read as float32 from the genome and converted while it is
//   staged (bfloat16, or E4M3 of w * 2^-e_w); the batch arrives already
//   quantised and packed [b][kp] (kp = n0 rounded up to 32).
// * Layer 1 is computed transposed (W_1 X^T) for the register tail; a
//   workgroup owns 64*MW rows (MW 1 or 2) and writes one partial sum per 64
//   rows, like the other large-batch kernels, so every shape and kernel
//   gives bit-identical fitness.  (Four row tiles per wave measured slower:
//   their accumulators push the kernel to one wave per SIMD and into
//   accumulator-register shuffling.)
// * FP8 products are rescaled by 2^(e_x + e_w) (exact) before the bias.
// LDS rows hold 32 elements (64 or 32 bytes) in four 8-element slots; slot s
// of row r is stored at slot s ^ ((r >> SH) & 3), which spreads the 16 lanes
// reading one slot column of 16 rows over distinct banks.
#include <string.h>

#include "lowp.hpp"
#include "lp_common.hpp"
#include "runs.hpp"

namespace leea {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int DT>
struct Lp;

template <>
struct Lp<1> {  // bfloat16
  static constexpr int ES = 2;  // bytes per element
  static constexpr int SH = 1;  // swizzle shift
  typedef uint4 Frag;
  static __device__ __forceinline__ floatx4 mma(const Frag& a, const Frag& b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
  // 8 floats -> one slot
  static __device__ __forceinline__ Frag pack(const float4& a, const float4& b, int) {
    Frag f;
    f.x = pack_bf16x2(a.x, a.y);
    f.y = pack_bf16x2(a.z, a.w);
    f.z = pack_bf16x2(b.x, b.y);
    f.w = pack_bf16x2(b.z, b.w);
    return f;
  }
};

template <>
struct Lp<2> {  // OCP FP8 E4M3
  static constexpr int ES = 1;
  static constexpr int SH = 2;
  typedef uint2 Frag;
  static __device__ __forceinline__ floatx4 mma(const Frag& a, const Frag& b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(
        (long)__builtin_bit_cast(unsigned long long, a),
        (long)__builtin_bit_cast(unsigned long long, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ Frag pack(const float4& a, const float4& b, int neg_e) {
    Frag f;
    f.x = pack_fp8x4(ldexpf(a.x, neg_e), ldexpf(a.y, neg_e), ldexpf(a.z, neg_e),
                     ldexpf(a.w, neg_e));
    f.y = pack_fp8x4(ldexpf(b.x, neg_e), ldexpf(b.y, neg_e), ldexpf(b.z, neg_e),
                     ldexpf(b.w, neg_e));
    return f;
  }
};

// Body of one workgroup: network j, row tile wt (rows 64*MW*wt ...).
template <int NT, int MW, int DT, int D, bool RT>
__device__ __forceinline__ void eval_lp_body(int j, int wt, const float* __restrict__ genomes,
                                             const NetDesc& nd, const void* __restrict__ xq,
                                             int kp, const uint32_t* __restrict__ w_amax,
                                             const uint32_t* __restrict__ x_amax,
                                             const int32_t* __restrict__ y, int b,
                                             float2* __restrict__ partial, const EvalLds& lo,
                                             int n_pt, int tail_vec) {
  typedef Lp<DT> T;
  typedef typename T::Frag Frag;
  extern __shared__ float lds[];
  constexpr int ES = T::ES;
  constexpr int FB = 8 * ES;        // bytes per slot (one lane fragment)
  constexpr int RB = 4 * FB;        // bytes per staged row (32 elements)
  constexpr int MT = 64 * MW;       // rows per workgroup
  constexpr int NR = NT * 16;       // staged weight rows
  constexpr int BUF = (NR + MT) * RB;
  constexpr int WITEMS = NR * 4;    // slots of a W chunk
  constexpr int WPT = (WITEMS + 255) / 256;
  constexpr int XPT = MT * 4 / 256;  // = MW

  const int tid = threadIdx.x;
  const int m0 = wt * MT;
  const int rows = b - m0 < MT ? b - m0 : MT;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const float* __restrict__ W1 = genome + nd.woff[0];
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int nch = kp >> 5;
  const char* __restrict__ xb = reinterpret_cast<const char*>(xq);
  const int neg_ew = DT == 2 ? -fp8_exponent(w_amax[j]) : 0;

  // D register stages of global prefetch: chunk ch + D is requested while
  // chunk ch is multiplied, which keeps D chunks of W_1 in flight per
  // workgroup (the per-chunk matrix work alone is far shorter than the
  // memory latency).
  float4 wr[D][WPT][2];
  Frag xr[D][XPT];
  // Every load is issued unconditionally from a clamped (valid) address;
  // out-of-range elements are zeroed only when the stage is stored to LDS.
  // Branch-free loads whose results are untouched until then let the
  // compiler wait for exactly the stage it consumes instead of draining
  // every load in flight.
  auto sel4 = [](bool keep, const float4& v) {
    return make_float4(keep ? v.x : 0.0f, keep ? v.y : 0.0f, keep ? v.z : 0.0f,
                       keep ? v.w : 0.0f);
  };
  auto gload = [&](int ch, float4 (&w)[WPT][2], Frag (&xx)[XPT]) {
    const int k0 = (ch < nch ? ch : nch - 1) * 32;  // past the end: reload the last chunk
#pragma unroll
    for (int qq = 0; qq < WPT; ++qq) {
      const int it = tid + 256 * qq;
      const int row = it >> 2;
      const int k = k0 + 8 * (it & 3);
      const int rc = (it < WITEMS && row < n1) ? row : 0;
      const int ka = k < n0 ? k : n0 - 4;
      const int kb = k + 4 < n0 ? k + 4 : n0 - 4;
      w[qq][0] = *reinterpret_cast<const float4*>(W1 + (int64_t)rc * n0 + ka);
      w[qq][1] = *reinterpret_cast<const float4*>(W1 + (int64_t)rc * n0 + kb);
    }
#pragma unroll
    for (int qq = 0; qq < XPT; ++qq) {
      const int m = (tid + 256 * qq) >> 2;
      const int s = (tid + 256 * qq) & 3;
      const int mc = m < rows ? m : 0;
      xx[qq] = *reinterpret_cast<const Frag*>(xb + ((int64_t)(m0 + mc) * kp + k0 + 8 * s) * ES);
    }
  };
  auto sstore = [&](int ch, int buf, const float4 (&w)[WPT][2], const Frag (&xx)[XPT]) {
    char* wst = reinterpret_cast<char*>(lds) + buf * BUF;
    char* xst = wst + NR * RB;
    const int k0 = ch * 32;
#pragma unroll
    for (int qq = 0; qq < WPT; ++qq) {
      const int it = tid + 256 * qq;
      const int row = it >> 2;
      const int s = it & 3;
      const int k = k0 + 8 * s;
      const bool rv = row < n1;
      if (it < WITEMS)
        *reinterpret_cast<Frag*>(wst + row * RB + ((s ^ ((row >> T::SH) & 3)) * FB)) =
            T::pack(sel4(rv && k < n0, w[qq][0]), sel4(rv && k + 4 < n0, w[qq][1]), neg_ew);
    }
#pragma unroll
    for (int qq = 0; qq < XPT; ++qq) {
      const int it = tid + 256 * qq;
      const int m = it >> 2;
      const int s = it & 3;
      *reinterpret_cast<Frag*>(xst + m * RB + ((s ^ ((m >> T::SH) & 3)) * FB)) =
          m < rows ? xx[qq] : Frag{};
    }
  };

  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  floatx4 acc[MW][NT];
#pragma unroll
  for (int mi = 0; mi < MW; ++mi)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[mi][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](int buf) {
    const char* wst = reinterpret_cast<const char*>(lds) + buf * BUF;
    const char* xst = wst + NR * RB;
    Frag a[MW], bq[NT];
#pragma unroll
    for (int mi = 0; mi < MW; ++mi) {
      const int m = wave * MW * 16 + mi * 16 + mn;
      a[mi] = *reinterpret_cast<const Frag*>(xst + m * RB + ((kq ^ ((m >> T::SH) & 3)) * FB));
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = t * 16 + mn;
      bq[t] = *reinterpret_cast<const Frag*>(wst + n * RB + ((kq ^ ((n >> T::SH) & 3)) * FB));
    }
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[mi][t] = T::mma(bq[t], a[mi], acc[mi][t]);
  };

  // double-buffered LDS: the store of chunk ch (buffer ch & 1) follows the
  // barrier of chunk ch - 1, which every wave reaches only after finishing
  // chunk ch - 2, the last reader of that buffer
#pragma unroll
  for (int s = 0; s < D; ++s) gload(s, wr[s], xr[s]);
  for (int ch0 = 0; ch0 < nch; ch0 += D) {
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int ch = ch0 + s;
      if (ch < nch) {  // uniform across the workgroup
        sstore(ch, ch & 1, wr[s], xr[s]);
        __syncthreads();
        gload(ch + D, wr[s], xr[s]);
        compute(ch & 1);
      }
    }
  }
  __syncthreads();  // staging is dead from here on
  const float fac = DT == 2 ? fp8_factor(*x_amax, w_amax[j]) : 1.0f;
  if constexpr (RT) {  // networks reg_tail_ok() takes
    copy_tail_genes(genome, nd, lds);
    int ylab[MW];
#pragma unroll
    for (int mi = 0; mi < MW; ++mi) {
      const int r = m0 + wave * MW * 16 + mi * 16 + mn;
      ylab[mi] = r < b ? y[r] : 0;
    }
    float* red = lds + reg_tail_copy_floats(nd);
    __syncthreads();
    reg_tail<NT, MW, DT>(acc, fac, lds, nd, m0, wave * MW * 16, b, ylab, red,
                         partial + (int64_t)j * n_pt, m0 / 64);
  } else {
    lds_epilogue<NT, MW, DT>(lds, acc, fac, j, wt, genome, nd, y, b, partial, lo, n_pt,
                             tail_vec);
  }
}

template <int NT, int MW, int DT, int D, bool RT>
__global__ __launch_bounds__(256, MW * NT <= 16 ? 2 : 1) void eval_lp_kernel(const float* __restrict__ genomes,
                                                      NetDesc nd, const void* __restrict__ xq,
                                                      int kp, const uint32_t* __restrict__ w_amax,
                                                      const uint32_t* __restrict__ x_amax,
                                                      const int32_t* __restrict__ y, int b,
                                                      float2* __restrict__ partial, EvalLds lo,
                                                      int n_wt, int n_pt, int pop, int tail_vec) {
  const int Lw = xcd_logical(blockIdx.x, n_wt * pop);
  const int j = Lw / n_wt;
  eval_lp_body<NT, MW, DT, D, RT>(j, Lw - j * n_wt, genomes, nd, xq, kp, w_amax, x_amax, y, b,
                                  partial, lo, n_pt, tail_vec);
}

// ------------------------------------------------------------- dispatch --

struct LpShape {
  int mw, pass_rows;
  size_t lds;
  EvalLds lo;
};

static constexpr size_t kLdsMax = 160 * 1024;
constexpr int kLpStages = 2;

// Dynamic LDS: the staging double buffer, then either the register tail's
// tail genes and row-sum scratch or the 64-row tile of the LDS epilogue.
static size_t lp_bytes(const NetDesc& nd, int mw, int es, EvalLds* lo) {
  const int nt = (nd.w[1] + 15) / 16;
  const size_t staging = 2 * (size_t)(nt * 16 + 64 * mw) * 32 * es;
  *lo = lp_tail_layout(nd, 64);
  const size_t tail = reg_tail_ok(nd)
                          ? (size_t)(reg_tail_copy_floats(nd) + 8 * mw) * 4
                          : (size_t)lo->total * 4;
  const size_t bytes = staging > tail ? staging : tail;
  lo->total = (int)((bytes + 3) / 4);
  return bytes;
}

// Rows per workgroup grow with the batch (more rows share each weight
// chunk) while the accumulators stay within 32 tiles per wave and LDS
// within 160 KB.
static bool lp_shape(const NetDesc& nd, int b, int dt, LpShape* out) {
  const int nt = (nd.w[1] + 15) / 16;
  const int es = dt == 1 ? 2 : 1;
  int mw = b > 64 ? 2 : 1;
  while (mw > 1 && mw * nt > 32) mw >>= 1;
  for (; mw >= 1; mw >>= 1) {
    EvalLds lo;
    const size_t bytes = lp_bytes(nd, mw, es, &lo);
    if (bytes <= kLdsMax) {
      out->mw = mw;
      out->pass_rows = 64;
      out->lds = bytes;
      out->lo = lo;
      return true;
    }
  }
  return false;
}

int eval_lp_ptiles(const NetDesc& nd, int b, int dt) {
  LpShape sh;
  if (!lp_shape(nd, b, dt, &sh)) return 1;
  return (b + sh.pass_rows - 1) / sh.pass_rows;
}

bool eval_lp_supported(const NetDesc& nd, int b, int dt) {
  LpShape sh;
  return lp_shape(nd, b, dt, &sh);
}

bool eval_shape_lp(const NetDesc& nd, int b, int dt, int kind, int mw, EvalShape* out) {
  const int nt = (nd.w[1] + 15) / 16;
  if (nt < 1 || nt > 16 || b < 1 || (dt != 1 && dt != 2)) return false;
  if (kind < 0) {
    EvalShape rows;
    kind = (dt == 1 && eval_shape_f32(nd, b, 4, 1, &rows)) ? 4 : (b <= 16 ? 0 : 2);
  }
  if (kind == 0) {
    if (!eval_shape_f32(nd, b, 0, 1, out)) return false;
    return true;  // small-batch kernel on quantised values
  }
  if (kind == 4)  // 1 KiB-row kernel, bfloat16 only
    return dt == 1 && eval_shape_f32(nd, b, 4, 1, out);
  if (kind != 2) return false;
  LpShape sh;
  if (!lp_shape(nd, b, dt, &sh)) return false;
  if (mw > 0 && mw != sh.mw) {
    if (mw != 1 && mw != 2) return false;
    if (mw * nt > 32) return false;
    const int es = dt == 1 ? 2 : 1;
    EvalLds lo;
    const size_t bytes = lp_bytes(nd, mw, es, &lo);
    if (bytes > kLdsMax) return false;
    sh.mw = mw;
    sh.pass_rows = 64;
    sh.lds = bytes;
    sh.lo = lo;
  }
  EvalShape r;
  memset(&r, 0, sizeof r);
  r.kind = 2;
  r.mw = sh.mw;
  r.n_wt = (b + 64 * sh.mw - 1) / (64 * sh.mw);
  r.n_pt = (b + sh.pass_rows - 1) / sh.pass_rows;
  r.pass_rows = sh.pass_rows;
  r.tail_vec = 1;
  for (int l = 1; l < nd.L; ++l)
    if (nd.w[l] % 4 != 0) r.tail_vec = 0;
  r.lds = sh.lds;
  r.lo = sh.lo;
  *out = r;
  return true;
}

// ------------------------------------------------- grouped (many runs) --

template <int NT, int MW, int DT, bool RT>
__global__ __launch_bounds__(256, MW * NT <= 16 ? 2 : 1) void runs_eval_lp_kernel(
    const RunDesc* __restrict__ runs, const BatchState* __restrict__ st,
    const int* __restrict__ off, const int* __restrict__ ids, int n, int total) {
  const int L = xcd_logical(blockIdx.x, total);
  const int i = find_group(off, n, L);
  const RunDesc& d = runs[ids[i]];
  const int local = L - off[i];
  const int j = local / d.n_wt;
  eval_lp_body<NT, MW, DT, kLpStages, RT>(j, local - j * d.n_wt, d.genomes[st->cur], d.nd, d.xq,
                                          d.kp, nullptr, nullptr, d.yb, d.b, d.partial, d.lo,
                                          d.n_pt, d.tail_vec);
}

template <int NT, int MW, bool RT>
static hipError_t launch_runs_lp3(const RunDesc* runs, const BatchState* st, const Group& g,
                                  hipStream_t s) {
  auto kern = runs_eval_lp_kernel<NT, MW, 1, RT>;
  if (g.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)g.blocks), dim3(256), g.lds, s, runs, st, g.off, g.ids,
                     g.n, g.blocks);
  return hipGetLastError();
}

template <int NT>
static hipError_t launch_runs_lp_nt(int mw, int rt, const RunDesc* runs, const BatchState* st,
                                    const Group& g, hipStream_t s) {
  if (mw == 2)
    return rt ? launch_runs_lp3<NT, 2, true>(runs, st, g, s)
              : launch_runs_lp3<NT, 2, false>(runs, st, g, s);
  return rt ? launch_runs_lp3<NT, 1, true>(runs, st, g, s)
            : launch_runs_lp3<NT, 1, false>(runs, st, g, s);
}

// Grouped launches exist for the bfloat16 first layer (the FP8 scales are
// tracked by the single-run path only).
hipError_t launch_runs_eval_lp(int nt, int mw, int dt, int rt, const RunDesc* runs,
                               const BatchState* st, const Group& g, hipStream_t s) {
  if (dt != 1) return hipErrorInvalidValue;
  switch (nt) {
#define LEEA_RLP_CASE(N) \
  case N:                \
    return launch_runs_lp_nt<N>(mw, rt, runs, st, g, s);
    LEEA_RLP_CASE(1) LEEA_RLP_CASE(2) LEEA_RLP_CASE(3) LEEA_RLP_CASE(4) LEEA_RLP_CASE(5)
    LEEA_RLP_CASE(6) LEEA_RLP_CASE(7) LEEA_RLP_CASE(8) LEEA_RLP_CASE(9) LEEA_RLP_CASE(10)
    LEEA_RLP_CASE(11) LEEA_RLP_CASE(12) LEEA_RLP_CASE(13) LEEA_RLP_CASE(14) LEEA_RLP_CASE(15)
    LEEA_RLP_CASE(16)
#undef LEEA_RLP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <int NT, int MW, int DT, bool RT>
static hipError_t launch_lp4(const float* genomes, const NetDesc& nd, int pop, const void* xq,
                             int kp, const uint32_t* w_amax, const uint32_t* x_amax,
                             const int32_t* y, int b, float2* partial, const LpShape& sh,
                             int tv, hipStream_t s) {
  auto kern = eval_lp_kernel<NT, MW, DT, kLpStages, RT>;
  if (sh.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
    if (e != hipSuccess) return e;
  }
  const int n_wt = (b + 64 * MW - 1) / (64 * MW);
  const int n_pt = (b + 63) / 64;
  hipLaunchKernelGGL(kern, dim3((unsigned)(n_wt * pop)), dim3(256), sh.lds, s, genomes, nd, xq,
                     kp, w_amax, x_amax, y, b, partial, sh.lo, n_wt, n_pt, pop, tv);
  return hipGetLastError();
}

template <int NT, int MW, int DT>
static hipError_t launch_lp3(const float* genomes, const NetDesc& nd, int pop, const void* xq,
                             int kp, const uint32_t* w_amax, const uint32_t* x_amax,
                             const int32_t* y, int b, float2* partial, const LpShape& sh,
                             int tv, hipStream_t s) {
  if (reg_tail_ok(nd))
    return launch_lp4<NT, MW, DT, true>(genomes, nd, pop, xq, kp, w_amax, x_amax, y, b, partial,
                                        sh, tv, s);
  return launch_lp4<NT, MW, DT, false>(genomes, nd, pop, xq, kp, w_amax, x_amax, y, b, partial,
                                       sh, tv, s);
}

template <int NT, int DT>
static hipError_t launch_lp2(const float* genomes, const NetDesc& nd, int pop, const void* xq,
                             int kp, const uint32_t* w_amax, const uint32_t* x_amax,
                             const int32_t* y, int b, float2* partial, const LpShape& sh,
                             int tv, hipStream_t s) {
  if (sh.mw == 2)
    return launch_lp3<NT, 2, DT>(genomes, nd, pop, xq, kp, w_amax, x_amax, y, b, partial, sh, tv,
                                 s);
  if (sh.mw == 1)
    return launch_lp3<NT, 1, DT>(genomes, nd, pop, xq, kp, w_amax, x_amax, y, b, partial, sh, tv,
                                 s);
  return hipErrorInvalidValue;
}

template <int NT>
static hipError_t launch_lp_nt(int dt, const float* genomes, const NetDesc& nd, int pop,
                               const void* xq, int kp, const uint32_t* w_amax,
                               const uint32_t* x_amax, const int32_t* y, int b, float2* partial,
                               hipStream_t s) {
  LpShape sh;
  if (!lp_shape(nd, b, dt, &sh)) return hipErrorInvalidValue;
  int tv = 1;
  for (int l = 1; l < nd.L; ++l)
    if (nd.w[l] % 4 != 0) tv = 0;
  if (dt == 1)
    return launch_lp2<NT, 1>(genomes, nd, pop, xq, kp, w_amax, x_amax, y, b, partial, sh, tv, s);
  return launch_lp2<NT, 2>(genomes, nd, pop, xq, kp, w_amax, x_amax, y, b, partial, sh, tv, s);
}

hipError_t launch_evaluate_lp(int dt, const float* genomes, const NetDesc& nd, int pop,
                              const void* xq, int kp, const uint32_t* w_amax,
                              const uint32_t* x_amax, const int32_t* y, int b, float2* partial,
                              hipStream_t s) {
  switch ((nd.w[1] + 15) / 16) {
#define LEEA_LP_CASE(N) \
  case N:               \
    return launch_lp_nt<N>(dt, genomes, nd, pop, xq, kp, w_amax, x_amax, y, b, partial, s);
    LEEA_LP_CASE(1) LEEA_LP_CASE(2) LEEA_LP_CASE(3) LEEA_LP_CASE(4) LEEA_LP_CASE(5)
    LEEA_LP_CASE(6) LEEA_LP_CASE(7) LEEA_LP_CASE(8) LEEA_LP_CASE(9) LEEA_LP_CASE(10)
    LEEA_LP_CASE(11) LEEA_LP_CASE(12) LEEA_LP_CASE(13) LEEA_LP_CASE(14) LEEA_LP_CASE(15)
    LEEA_LP_CASE(16)
#undef LEEA_LP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace leea
