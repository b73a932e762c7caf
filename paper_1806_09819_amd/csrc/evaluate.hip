// Population-batched forward pass with fused fitness (paper section 3.3:
// batch the whole population into tensor products; Eq. 1 fitness).
//
// Layer 1 of every network reads the same minibatch X [b][n0], so for the
// whole population it is one dense product X * [W1_1 .. W1_P]^T (M = b,
// N = P * n1, K = n0).  A workgroup owns one individual's n1 columns (all of
// its layer-1 neurons) for a tile of batch rows and accumulates them on the
// matrix cores with v_mfma_f32_16x16x4_f32 (FP32 in, FP32 accumulate).
// Keeping all n1 columns of an individual in one workgroup lets the rest of
// the network and the fitness run in the same kernel on the layer-1 tile
// held in LDS: only two floats per (individual, row tile) go back to HBM.
//
// MFMA 16x16x4 f32 operand layout (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; the 4 accumulator values of lane l are
// D[4*(l/16)+i][l%16].  A float4 of 4 consecutive k per lane feeds 4 MFMAs:
// in the e-th one lane (m, kq) contributes k = k0 + 4*kq + e, so the four
// MFMAs together cover k0 .. k0+15 (one "super-step").
//
// Layer-1 schemes:
// * tiny batch (b <= 4, float32): rows of W_1 streamed 1 KiB per load
//   instruction against the batch held in registers, on the vector ALUs.
// * batch <= 8 (float32 or bfloat16): rows of W_1 loaded 1 KiB per
//   instruction, regrouped through a wave-private LDS tile for the
//   16-block 4x4 matrix products (see the 1 KiB-row kernels below).
// * small batch (b <= 16, bandwidth-bound): one workgroup per individual;
//   its 4 waves split the K range, weight fragments stream straight from
//   HBM into registers (every weight is read exactly once), batch fragments
//   come from L2; the four K-partial tiles are summed through LDS.
// * large batch (compute-bound): workgroup = (tile of 64*MW rows,
//   individual), each wave owns 16*MW rows x all n1 columns; 32-wide K
//   chunks of W and X are staged through double-buffered, XOR-swizzled LDS
//   so each weight fragment fetched serves every wave.  Workgroup ids are
//   remapped so all row tiles of one individual run on the same XCD and
//   share its weights in that XCD's L2.
// Layers 2..L run on the matrix cores too (weight fragments as float4 loads
// from L2) whenever the hidden widths are multiples of 4, else on VALU.
#include <string.h>

#include "eval_common.hpp"
#include "lowp.hpp"
#include "lp_common.hpp"
#include "runs.hpp"

namespace leea {

// Per-network finish from the summed partials s (log-likelihoods) and c
// (correct rows): fitness s / b, accuracy c / b, then the inheritance
// weighting f_adj = fl(fl((1 - alpha) f_inh) + fl(alpha f)) (section 3.1).
__device__ __forceinline__ void finalize_values(int j, float s, float c, int b,
                                                const float* __restrict__ f_inh, int use_inh,
                                                float alpha, float* f_adj, float* f_raw,
                                                float* acc, float* f_adj_out, float* f_raw_out,
                                                float* acc_out) {
#pragma clang fp contract(off)
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

// The same finish inside an evaluation kernel whose workgroup wrote the
// network's only partial p (thread 0 holds it): the sum over one tile
// starts from zero as finalize_one's does, so the results are bitwise its.
__device__ __forceinline__ void finalize_in_kernel(int j, float2 p, int b, const FinArgs& fin) {
#pragma clang fp contract(off)
  float s = 0.0f, c = 0.0f;
  s += p.x;
  c += p.y;
  finalize_values(j, s, c, b, fin.f_inh, fin.use_inh, fin.alpha, fin.f_adj, fin.f_raw, fin.acc,
                  fin.f_adj_out, fin.f_raw_out, fin.acc_out);
}

// ---------------------------------------------------------------- small b --
// End of the small-batch kernels (one workgroup per network, 4 waves that
// split K, acc[t] = this wave's K-partial of rows 4 kq + i, neurons
// 16 t + mn): the 4 K-partial tiles -> LDS [wave][16][ld1], summed in a fixed
// order into tile 0, which becomes the layer-1 activations (times fac when
// SCALED, bias, ReLU, zero padding columns); then the tail layers (weights
// in the arithmetic DT, see tail_and_fitness), the fitness and, with fin.on,
// the network's finish.
template <int NT, bool SCALED, int DT = 0>
__device__ __forceinline__ void small_epilogue(const floatx4 (&acc)[NT], float fac, int j,
                                               const float* __restrict__ genome,
                                               const NetDesc& nd, const int32_t* __restrict__ y,
                                               int b, float2* __restrict__ partial,
                                               const EvalLds& lo, int tail_vec,
                                               const FinArgs& fin,
                                               const TailScales& ts = TailScales{{}, 0}) {
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const int n1 = nd.w[1];
  const int ld1 = lo.ld1;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) lds[(wave * 16 + 4 * kq + i) * ld1 + t * 16 + mn] = acc[t][i];
  __syncthreads();
  const float* __restrict__ b1 = genome + nd.boff[0];
  const bool hidden = nd.L > 1;
  for (int idx = tid; idx < 16 * NT * 16; idx += 256) {
    const int m = idx / (NT * 16);
    const int n = idx - m * (NT * 16);
    float v = 0.0f;
    if (n < n1) {
      v = lds[m * ld1 + n] + lds[(16 + m) * ld1 + n];
      v += lds[(32 + m) * ld1 + n];
      v += lds[(48 + m) * ld1 + n];
      if (SCALED) v = v * fac;
      v += b1[n];
      if (hidden) v = relu_keep_nan(v);
    }
    lds[m * ld1 + n] = v;
  }
  __syncthreads();
  const float2 r = tail_and_fitness<1, DT>(lds, lo, nd, genome, 0, 1, b, 0, y, tail_vec != 0,
                                           partial + j, 0, ts);
  if (fin.on && tid == 0) finalize_in_kernel(j, r, b, fin);
}

// DT selects the first layer's arithmetic (0 float32; 1 bfloat16, 2 FP8
// E4M3: x holds the batch already quantised, the weight fragments are
// quantised in registers; products of such values are exact in float32, so
// the FP32 matrix cores sum exactly the reduced-precision products).
template <int NT, int DT>
__device__ __forceinline__ void eval_small_body(int j, const float* __restrict__ genomes,
                                                const NetDesc& nd, const float* __restrict__ x,
                                                const int32_t* __restrict__ y, int b,
                                                float2* __restrict__ partial, const EvalLds& lo,
                                                int tail_vec, const uint32_t* __restrict__ w_amax,
                                                const uint32_t* __restrict__ x_amax,
                                                const FinArgs& fin) {
  extern __shared__ float lds[];
  const int tid = threadIdx.x;
  const int neg_ew = DT == 2 ? -fp8_exponent(w_amax[j]) : 0;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const bool xv = mn < b;
  const float* __restrict__ xrow = x + (int64_t)(xv ? mn : 0) * n0;
  const float* wrow[NT];
  bool rvalid[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = t * 16 + mn;
    rvalid[t] = r < n1;
    wrow[t] = genome + nd.woff[0] + (int64_t)(rvalid[t] ? r : 0) * n0;
  }
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nss = (n0 + 15) >> 4;
  float4 xa, wb[NT];
  auto load = [&](int s, float4& xo, float4* wo) {
    const int k = 16 * s + 4 * kq;
    const bool kv = k < n0;
    xo = (xv && kv) ? *reinterpret_cast<const float4*>(xrow + k) : zero4();
#pragma unroll
    for (int t = 0; t < NT; ++t)
      wo[t] = (rvalid[t] && kv) ? *reinterpret_cast<const float4*>(wrow[t] + k) : zero4();
    if constexpr (DT != 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        wo[t].x = quantize<DT>(wo[t].x, neg_ew);
        wo[t].y = quantize<DT>(wo[t].y, neg_ew);
        wo[t].z = quantize<DT>(wo[t].z, neg_ew);
        wo[t].w = quantize<DT>(wo[t].w, neg_ew);
      }
    }
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

  const float fac = DT == 2 ? fp8_factor(*x_amax, w_amax[j]) : 1.0f;
  small_epilogue<NT, DT == 2, DT>(acc, fac, j, genome, nd, y, b, partial, lo, tail_vec, fin);
}

template <int NT, int DT>
__global__ __launch_bounds__(256, NT > 8 ? 3 : 4) void eval_small_kernel(const float* __restrict__ genomes,
                                                         NetDesc nd, const float* __restrict__ x,
                                                         const int32_t* __restrict__ y, int b,
                                                         float2* __restrict__ partial,
                                                         EvalLds lo, int tail_vec,
                                                         const uint32_t* __restrict__ w_amax,
                                                         const uint32_t* __restrict__ x_amax,
                                                         FinArgs fin) {
  eval_small_body<NT, DT>(blockIdx.x, genomes, nd, x, y, b, partial, lo, tail_vec, w_amax,
                          x_amax, fin);
}

// ------------------------------------------------------- b <= 16, BF16 --
// The small-batch scheme with a bfloat16 first layer on the bfloat16 matrix
// cores: v_mfma_f32_16x16x32_bf16, lane l = (mn, kq) supplying batch row mn
// and W_1 row 16 t + mn at k = 32 s + 8 kq .. + 7 (16 bytes each), waves
// splitting the 32-wide K steps s = wave, wave + 4, ...  FROM_COPY: W_1 comes
// from its bfloat16 copy (W1Shadow: rows padded to 16, K to 32, zeros), half
// the bytes of the float32 genome; otherwise it is read as float32 and
// rounded on the way (the grouped runs, which keep no copy).  The batch is
// read as float32 and rounded in registers.  Both forms round the same
// values the same way (nearest even) and issue the same products in the same
// order, so they are bitwise equal.
__device__ __forceinline__ uint4 pack_bf16x8(const float4& a, const float4& c) {
  return make_uint4(pack_bf16x2(a.x, a.y), pack_bf16x2(a.z, a.w), pack_bf16x2(c.x, c.y),
                    pack_bf16x2(c.z, c.w));
}

__device__ __forceinline__ floatx4 mfma_bf16x32(const uint4& a, const uint4& b, const floatx4& c) {
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

template <int NT, bool FROM_COPY>
__device__ __forceinline__ void eval_small_bf16_body(int j, const float* __restrict__ genomes,
                                                     const NetDesc& nd, const W1Shadow& wsh,
                                                     const float* __restrict__ x,
                                                     const int32_t* __restrict__ y, int b,
                                                     float2* __restrict__ partial,
                                                     const EvalLds& lo, int tail_vec,
                                                     const FinArgs& fin) {
  const int tid = threadIdx.x;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const bool xv = mn < b;
  const float* __restrict__ xrow = x + (int64_t)(xv ? mn : 0) * n0;
  const uint16_t* __restrict__ crow[NT];
  const float* __restrict__ frow[NT];
  bool rvalid[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = t * 16 + mn;
    rvalid[t] = r < n1;
    crow[t] = FROM_COPY ? wsh.p + (int64_t)j * wsh.net + (int64_t)r * wsh.kp : nullptr;
    frow[t] = genome + nd.woff[0] + (int64_t)(rvalid[t] ? r : 0) * n0;
  }
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  auto ld8 = [&](const float* row, int k, bool ok) {
    const float4 a = (ok && k < n0) ? *reinterpret_cast<const float4*>(row + k) : zero4();
    const float4 c = (ok && k + 4 < n0) ? *reinterpret_cast<const float4*>(row + k + 4) : zero4();
    return pack_bf16x8(a, c);
  };
  const int nss = (n0 + 31) >> 5;
  uint4 xa, wb[NT];
  auto load = [&](int s, uint4& xo, uint4* wo) {
    const int k = 32 * s + 8 * kq;
    xo = ld8(xrow, k, xv);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if constexpr (FROM_COPY)
        wo[t] = *reinterpret_cast<const uint4*>(crow[t] + k);
      else
        wo[t] = ld8(frow[t], k, rvalid[t]);
    }
  };
  int s = wave;
  if (s < nss) load(s, xa, wb);
  for (; s < nss; s += 4) {
    uint4 xn, wn[NT];
    if (s + 4 < nss) load(s + 4, xn, wn);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = mfma_bf16x32(xa, wb[t], acc[t]);
    if (s + 4 < nss) {
      xa = xn;
#pragma unroll
      for (int t = 0; t < NT; ++t) wb[t] = wn[t];
    }
  }
  small_epilogue<NT, false, 1>(acc, 1.0f, j, genome, nd, y, b, partial, lo, tail_vec, fin);
}

template <int NT>
__global__ __launch_bounds__(256, NT > 8 ? 3 : 4) void eval_small_bf16_kernel(
    const float* __restrict__ genomes, NetDesc nd, W1Shadow wsh, const float* __restrict__ x,
    const int32_t* __restrict__ y, int b, float2* __restrict__ partial, EvalLds lo, int tail_vec,
    FinArgs fin) {
  if (wsh.p)
    eval_small_bf16_body<NT, true>(blockIdx.x, genomes, nd, wsh, x, y, b, partial, lo, tail_vec,
                                   fin);
  else
    eval_small_bf16_body<NT, false>(blockIdx.x, genomes, nd, wsh, x, y, b, partial, lo, tail_vec,
                                    fin);
}

// ------------------------------------------------------- b <= 16, FP8 --
// The small-batch scheme with an FP8 (E4M3) first layer on the FP8 matrix
// cores, reading W_1 from its FP8 copy (a quarter of the float32 genome's
// bytes).  Lane l = (mn, kq) loads 16 codes of W_1 row 16 t + mn at
// k = 64 s + 16 kq .. + 15 (16 bytes) and the same 16 elements of batch row
// mn (float32, scaled by 2^-e_x and rounded on the way); its first 8 feed one
// v_mfma_f32_16x16x32_fp8_fp8 and its last 8 a second, so the two products
// cover the 64-wide step between them (the K order inside a step is a
// permutation shared by both operands).  Waves split the steps
// s = wave, wave + 4, ...; the sums are multiplied by 2^(e_x + e_w) (NaN if
// either operand is not finite) before the bias.
__device__ __forceinline__ floatx4 mfma_fp8x32(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1,
                                               const floatx4& c) {
  const unsigned long long a = (unsigned long long)a0 | ((unsigned long long)a1 << 32);
  const unsigned long long b = (unsigned long long)b0 | ((unsigned long long)b1 << 32);
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)a, (long)b, c, 0, 0, 0);
}

template <int NT>
__global__ __launch_bounds__(256, NT > 8 ? 3 : 4) void eval_small_fp8_kernel(
    const float* __restrict__ genomes, NetDesc nd, W1Fp8 w8, const float* __restrict__ x,
    const uint32_t* __restrict__ x_amax, const int32_t* __restrict__ y, int b,
    float2* __restrict__ partial, EvalLds lo, int tail_vec, FinArgs fin) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const int n0 = nd.w[0];
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const uint32_t xam = *x_amax;
  const int neg_ex = xam < kNonFinite ? -fp8_exponent(xam) : 0;
  const float fac = fp8_factor(xam, w8.bound[j]);
  const bool xv = mn < b;
  const float* __restrict__ xrow = x + (int64_t)(xv ? mn : 0) * n0;
  const uint8_t* __restrict__ crow[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) crow[t] = w8.p + (int64_t)j * w8.net + (int64_t)(t * 16 + mn) * w8.kp;
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  auto xq4 = [&](int k) {  // 4 batch elements k .. k + 3 -> one word of codes
    const float4 v = (xv && k < n0) ? *reinterpret_cast<const float4*>(xrow + k) : zero4();
    return pack_fp8x4(ldexpf(v.x, neg_ex), ldexpf(v.y, neg_ex), ldexpf(v.z, neg_ex),
                      ldexpf(v.w, neg_ex));
  };
  const int nss = w8.kp >> 6;
  uint4 xa, wb[NT];
  auto load = [&](int s, uint4& xo, uint4* wo) {
    const int k = 64 * s + 16 * kq;
    xo = make_uint4(xq4(k), xq4(k + 4), xq4(k + 8), xq4(k + 12));
#pragma unroll
    for (int t = 0; t < NT; ++t) wo[t] = *reinterpret_cast<const uint4*>(crow[t] + k);
  };
  int s = wave;
  if (s < nss) load(s, xa, wb);
  for (; s < nss; s += 4) {
    uint4 xn, wn[NT];
    if (s + 4 < nss) load(s + 4, xn, wn);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = mfma_fp8x32(xa.x, xa.y, wb[t].x, wb[t].y, acc[t]);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = mfma_fp8x32(xa.z, xa.w, wb[t].z, wb[t].w, acc[t]);
    if (s + 4 < nss) {
      xa = xn;
#pragma unroll
      for (int t = 0; t < NT; ++t) wb[t] = wn[t];
    }
  }
  // the later layers' scales are read here, not at the start: kept through
  // the main loop they cost scalar registers the loop needs (measured 43 vs
  // 39 us at b = 8)
  const TailScales ts =
      load_tail_scales(w8.tail ? w8.tail + (int64_t)j * kTailScales : nullptr, nd.L);
  small_epilogue<NT, true, 2>(acc, fac, j, genome, nd, y, b, partial, lo, tail_vec, fin, ts);
}

// ------------------------------------------ b <= 8, FP32 / BF16, 1 KiB rows --
// Layer 1 from whole 1 KiB spans of W_1 rows on the 16-block matrix
// instructions v_mfma_f32_4x4x1f32 (float32) and v_mfma_f32_4x4x4_16b_bf16
// (bfloat16, 4 k per lane).  Lane l = 4 beta + jj of a wave belongs to block
// beta; block beta multiplies A[i] (supplied by lane 4 beta + i) with B[jj]
// (lane 4 beta + jj) into D[i][jj], held by lane 4 beta + jj in its
// accumulator i.  With A = batch row i of a group of 4 and B = W_1 row jj of
// a group of 4 rows, both at the same k in a block, the 16 blocks cover
// different k and their D tiles are summed over the blocks at the end.
//
// A unit is 1 KiB of a row (256 floats, or 512 bfloat16 of the copy); a
// wave owns one unit of every row it takes (one load instruction per row:
// lane l reads the unit's 16 bytes at 16 l).  Four such loads (rows
// 4 rg .. 4 rg + 3) pass through a wave-private LDS tile that swaps rows and
// lanes within each quad, so that lane (beta, jj) holds row 4 rg + jj at 16
// (float32) or 32 (bfloat16) consecutive columns of block beta, and the
// batch is held in registers at the same columns (two groups of 4 rows).
// The matrix products of 4 rows are followed by a reduce-scatter of the 16
// block sums over the wave (xor 32 halves the group, 16 and 8 the rows, 4
// sums the pair): one value per lane, written to the unit's K-partial tile
// [unit][8][ld1] in LDS.  Loads are raw buffer loads over the network's W_1
// or its copy (rows past n1 and columns past the row lie outside and read
// zero without a memory access) and non-temporal (each line is read once);
// two groups of 4 rows are in flight.  Measured against the 16-row fragment
// walk of eval_small_kernel, which streams the same bytes as 16 rows x 64 B
// per instruction: float32 layer 1 alone 60 us at P = 1000, 784-112, b = 8
// (5.8 TB/s) against about 75 us.  The unit partials meet in LDS in a fixed
// order (unit 0 + 1, + 2, + 3), then the bias, the ReLU and a tail for at
// most 8 rows from a copy of the genome's tail in LDS where it fits (else
// the small-batch kernel's tail from global memory).
constexpr int kRowsMaxB = 8;
constexpr int kRowsUnit = 256;      // floats of a row per load instruction
constexpr int kRowsTile = 4 * 65;   // float4 per wave transpose tile (one float4 pad per row)

// Floats of LDS the kernel uses: the K-partial tiles [4][8][ld1], then the
// four transpose tiles; the activation tile and tail buffers reuse the space.
__host__ __device__ inline int rows_lds_floats(const EvalLds& lo) {
  const int l1 = 4 * kRowsMaxB * lo.ld1 + 4 * 4 * kRowsTile;
  return lo.total > l1 ? lo.total : l1;
}

// Layers 2..L and the fitness of the 1 KiB-row kernels: at most 8 batch
// rows, the weights from the LDS copy of the genome's tail (W_l at
// tw + woff[l] - toff), one output (row, neuron) per thread at a time as a
// float32 dot product (four partial sums by k mod 4, weights rounded as
// loaded for DT 1), then
// one thread per row for the fitness (as tail_and_fitness) and thread 0 for
// the row sums, in row order.  A short chain per thread in place of the
// 16-row matrix tail: at the end of the kernel only the last networks' tails
// are left, and their latency is what shows.
template <int DT>
__device__ float2 rows_tail(float* lds, const EvalLds& lo, const NetDesc& nd, const float* tw,
                            int64_t toff, int b, int ylab, bool vec, float2* __restrict__ out) {
  const int tid = threadIdx.x;
  const float* in = lds + lo.h1;
  int ldi = lo.ld1;
  float* dst = lds + lo.ta;
  for (int l = 1; l < nd.L; ++l) {
    const int n_in = nd.w[l];
    const int n_out = nd.w[l + 1];
    const float* W = tw + (nd.woff[l] - toff);
    const float* bias = tw + (nd.boff[l] - toff);
    const bool relu = l < nd.L - 1;
    for (int idx = tid; idx < kRowsMaxB * n_out; idx += 256) {
      const int m = idx & (kRowsMaxB - 1);
      const int n = idx / kRowsMaxB;
      if (m < b) {
        const float* a = in + m * ldi;
        const float* w = W + n * n_in;
        // four partial sums (k mod 4), added pairwise at the end: four
        // independent chains, and the unrolled loop issues its LDS reads
        // ahead of the multiplies
        float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, v3 = 0.0f;
        int k = 0;
        if (vec) {
#pragma unroll 4
          for (; k + 4 <= n_in; k += 4) {
            const float4 av = *reinterpret_cast<const float4*>(a + k);
            const float4 wv = *reinterpret_cast<const float4*>(w + k);
            v0 = fmaf(av.x, quantize<DT>(wv.x, 0), v0);
            v1 = fmaf(av.y, quantize<DT>(wv.y, 0), v1);
            v2 = fmaf(av.z, quantize<DT>(wv.z, 0), v2);
            v3 = fmaf(av.w, quantize<DT>(wv.w, 0), v3);
          }
        }
        for (; k < n_in; ++k) v0 = fmaf(a[k], quantize<DT>(w[k], 0), v0);
        float v = (v0 + v1) + (v2 + v3);
        v += bias[n];
        if (relu) v = relu_keep_nan(v);
        dst[m * lo.ldt + n] = v;
      }
    }
    __syncthreads();
    in = dst;
    ldi = lo.ldt;
    dst = (dst == lds + lo.ta) ? lds + lo.h1 : lds + lo.ta;
  }
  const int d = nd.w[nd.L];
  float* ll = lds + lo.ll;
  int* cor = reinterpret_cast<int*>(lds + lo.cor);
  if (tid < b) {
    const float* z = in + tid * ldi;
    float mx = z[0];
    int best = 0;
    for (int k = 1; k < d; ++k)
      if (z[k] > mx) {
        mx = z[k];
        best = k;
      }
    float sx = 0.0f;
    for (int k = 0; k < d; ++k) sx += expf(z[k] - mx);
    ll[tid] = (ylab >= 0 && ylab < d) ? (z[ylab] - mx) - logf(sx) : __builtin_nanf("");
    cor[tid] = (best == ylab) ? 1 : 0;
  }
  __syncthreads();
  float2 r = make_float2(0.0f, 0.0f);
  if (tid == 0) {
    float sl = 0.0f;
    int c = 0;
    for (int m = 0; m < b; ++m) {
      sl += ll[m];
      c += cor[m];
    }
    r = make_float2(sl, (float)c);
    *out = r;
  }
  return r;  // thread 0: the partial it wrote
}

// DT 0: float32.  DT 1: bfloat16 products (exact in float32) on
// v_mfma_f32_4x4x4_16b_bf16, K = 4 per block, W_1 from its bfloat16 copy
// (FROM_COPY, 1 KiB = 512 elements per row load) or read as float32 and
// rounded in registers (grouped runs, which keep no copy; the same values in
// the same places, so the two forms are bitwise equal), the batch rounded in
// registers, later layers' weights rounded as the tail loads them.
// A unit is 1 KiB of a row in the copy's element size (256 floats, 512
// bfloat16); units (at most 4) are rounded up to 1, 2 or 4 and the four
// waves take (unit, row phase): wave w owns unit w mod UP and every
// (4 / UP)-th group of rows, so each (unit, row) partial is one wave's.
template <int NT, int DT, bool FROM_COPY>
__device__ __forceinline__ void eval_rows_body(int j, const float* __restrict__ genomes,
                                               const NetDesc& nd, const W1Shadow& wsh,
                                               const float* __restrict__ x,
                                               const int32_t* __restrict__ y, int b,
                                               float2* __restrict__ partial, const EvalLds& lo,
                                               int tail_vec, const FinArgs& fin) {
  extern __shared__ float lds[];
  constexpr int KU = DT == 1 ? 2 * kRowsUnit : kRowsUnit;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int beta = lane >> 2;
  const int jj = lane & 3;
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int ld1 = lo.ld1;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const float* __restrict__ W = genome + nd.woff[0];
  const int U = (n0 + KU - 1) / KU;
  const int UP = U <= 1 ? 1 : (U <= 2 ? 2 : 4);
  const int unit = wave & (UP - 1);
  const int phase = wave / UP;
  const int nphase = 4 / UP;
  const int k0 = KU * unit;
  // the fitness's labels, read ahead (a buffer load: no branch, and no flat
  // access where y comes from a run descriptor, either of which would cost
  // the main loop its exact waits)
  const int ylab = __builtin_amdgcn_raw_buffer_load_b32(
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(y), 0, b * 4, 0x00020000),
      tid < b ? tid * 4 : 0x40000000, 0, 0);
  // the batch at this lane's block columns, rows 4 g + jj (buffer loads:
  // rows past b and columns past n0 read zero): float32 columns
  // k0 + 16 beta + 4 t .. + 3, or bfloat16 columns k0 + 32 beta + 8 t .. + 7
  const __amdgpu_buffer_rsrc_t xs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(x), 0, b * n0 * 4, 0x00020000);
  auto xload = [&](int r, int k) {
    const int off = (r < b && k < n0) ? (r * n0 + k) * 4 : 0x40000000;
    const floatx4 v = __builtin_amdgcn_raw_buffer_load_b128(xs, off, 0, 0);
    return make_float4(v[0], v[1], v[2], v[3]);
  };
  uint4 xr[2][4];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 4 * g + jj;
      if constexpr (DT == 1) {
        const int k = k0 + 32 * beta + 8 * t;
        xr[g][t] = pack_bf16x8(xload(r, k), xload(r, k + 4));
      } else {
        const float4 v = xload(r, k0 + 16 * beta + 4 * t);
        xr[g][t] = make_uint4(__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z),
                              __float_as_uint(v.w));
      }
    }
  // touch one dword of each 128-byte line of the rest of the genome (b_1
  // and layers 2..L, read after layer 1 by the epilogue and the tail; up to
  // 32 KiB) so that those lines are in L2 by then
  const float* __restrict__ rest = genome + nd.boff[0];
  const int rest_bytes = (int)((nd.genes - nd.boff[0]) * 4);
  const float touch = __builtin_amdgcn_raw_buffer_load_b32(
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(rest), 0, rest_bytes, 0x00020000),
      tid * 128 < rest_bytes ? tid * 128 : 0x40000000, 0, 0);
  // W_1 row loads, 16 bytes per lane: rows past n1 and columns past the row
  // lie outside the resource and read zero without a memory access.  The
  // float32 form of DT 1 loads 32 bytes (two float4) and rounds them when
  // the row group is used.
  constexpr int LW = (DT == 1 && !FROM_COPY) ? 2 : 1;
  const __amdgpu_buffer_rsrc_t rs =
      (DT == 1 && FROM_COPY)
          ? __builtin_amdgcn_make_buffer_rsrc(wsh.p + (int64_t)j * wsh.net, 0,
                                              (int)(wsh.net * 2), 0x00020000)
          : __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(W), 0, n1 * n0 * 4, 0x00020000);
  const int kl = k0 + (DT == 1 ? 8 : 4) * lane;
  auto load = [&](int rg, uint4 (&wv)[4][LW]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int row = 4 * rg + t;
#pragma unroll
      for (int h = 0; h < LW; ++h) {
        int off;
        if constexpr (DT == 1 && FROM_COPY)
          off = (row < n1 && kl < wsh.kp) ? (row * wsh.kp + kl) * 2 : 0x40000000;
        else
          off = (row < n1 && kl + 4 * h < n0) ? (row * n0 + kl + 4 * h) * 4 : 0x40000000;
        const floatx4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 2);  // nt
        wv[t][h] = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]),
                              __float_as_uint(v[2]), __float_as_uint(v[3]));
      }
    }
  };
  uint4* tile = reinterpret_cast<uint4*>(lds + 4 * kRowsMaxB * ld1) + wave * kRowsTile;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  const int prow = 4 * (int)b5 + 2 * (int)b4 + (int)b3;  // batch row this lane ends with
  float* part = lds + (unit * kRowsMaxB + prow) * ld1;
  auto compute = [&](int rg, const uint4 (&wv)[4][LW]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if constexpr (LW == 2)
        tile[t * 65 + lane] = pack_bf16x8(
            make_float4(__uint_as_float(wv[t][0].x), __uint_as_float(wv[t][0].y),
                        __uint_as_float(wv[t][0].z), __uint_as_float(wv[t][0].w)),
            make_float4(__uint_as_float(wv[t][1].x), __uint_as_float(wv[t][1].y),
                        __uint_as_float(wv[t][1].z), __uint_as_float(wv[t][1].w)));
      else
        tile[t * 65 + lane] = wv[t][0];
    }
    uint4 T[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) T[t] = tile[jj * 65 + 4 * beta + t];
    floatx4 a0 = {0.f, 0.f, 0.f, 0.f}, a1 = {0.f, 0.f, 0.f, 0.f};
    if constexpr (DT == 1) {
      typedef short shortx4 __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint2 wl = make_uint2(T[t].x, T[t].y), wh = make_uint2(T[t].z, T[t].w);
        a0 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(
            __builtin_bit_cast(shortx4, make_uint2(xr[0][t].x, xr[0][t].y)),
            __builtin_bit_cast(shortx4, wl), a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(
            __builtin_bit_cast(shortx4, make_uint2(xr[1][t].x, xr[1][t].y)),
            __builtin_bit_cast(shortx4, wl), a1, 0, 0, 0);
        a0 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(
            __builtin_bit_cast(shortx4, make_uint2(xr[0][t].z, xr[0][t].w)),
            __builtin_bit_cast(shortx4, wh), a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(
            __builtin_bit_cast(shortx4, make_uint2(xr[1][t].z, xr[1][t].w)),
            __builtin_bit_cast(shortx4, wh), a1, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint32_t w4[4] = {T[t].x, T[t].y, T[t].z, T[t].w};
        const uint32_t x0[4] = {xr[0][t].x, xr[0][t].y, xr[0][t].z, xr[0][t].w};
        const uint32_t x1[4] = {xr[1][t].x, xr[1][t].y, xr[1][t].z, xr[1][t].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a0 = __builtin_amdgcn_mfma_f32_4x4x1f32(__uint_as_float(x0[e]), __uint_as_float(w4[e]),
                                                  a0, 0, 0, 0);
          a1 = __builtin_amdgcn_mfma_f32_4x4x1f32(__uint_as_float(x1[e]), __uint_as_float(w4[e]),
                                                  a1, 0, 0, 0);
        }
      }
    }
    // sum over the 16 blocks (lane bits 2..5): reduce-scatter
    float r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float keep = b5 ? a1[i] : a0[i];
      const float send = b5 ? a0[i] : a1[i];
      r[i] = keep + __shfl_xor(send, 32);
    }
    float r2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float keep = b4 ? r[2 + i] : r[i];
      const float send = b4 ? r[i] : r[2 + i];
      r2[i] = keep + __shfl_xor(send, 16);
    }
    const float r3 = (b3 ? r2[1] : r2[0]) + __shfl_xor(b3 ? r2[0] : r2[1], 8);
    const float r4 = r3 + __shfl_xor(r3, 4);
    const int row = 4 * rg + jj;
    if (!(lane & 4) && row < n1) part[row] = r4;
  };
  // this wave's row groups phase, phase + nphase, ...; two in flight (the
  // scheduling barriers keep each group's loads together so that the waits
  // count exactly the older group)
  const int RG = (n1 + 3) >> 2;
  uint4 w0[4][LW], w1[4][LW];
  load(phase, w0);
  __builtin_amdgcn_sched_barrier(0);
  load(phase + nphase, w1);
  __builtin_amdgcn_sched_barrier(0);
  for (int rg = phase; rg < RG; rg += 2 * nphase) {
    compute(rg, w0);
    __builtin_amdgcn_sched_barrier(0);
    load(rg + 2 * nphase, w0);
    __builtin_amdgcn_sched_barrier(0);
    compute(rg + nphase, w1);
    __builtin_amdgcn_sched_barrier(0);
    load(rg + 3 * nphase, w1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (b < 0) partial[j].x = touch;  // never taken (b >= 1): keeps the touch load
  // the rest of the genome (b_1 and layers 2..L) into the transpose tiles,
  // now free, when it fits there and clear of the tail's own buffers: each
  // wave copies the quarter over its own tile as soon as its loop ends, so
  // the epilogue and the tail read LDS instead of waiting on global memory
  // behind the other networks' streams (one round trip instead of one per
  // layer)
  const int64_t rest_floats = nd.genes - nd.boff[0];
  const int tile0 = 4 * kRowsMaxB * ld1;
  const bool tail_lds = rest_floats <= 4 * 4 * kRowsTile && lo.total <= tile0;
  if (tail_lds) {
    const int n4 = (int)((rest_floats + 3) >> 2);  // float4 of the copy (the last may run
                                                    // past the genome, inside its stride)
    char* dst = reinterpret_cast<char*>(lds + tile0);
    const char* src = reinterpret_cast<const char*>(rest);
    for (int i = wave * kRowsTile; i < (wave + 1) * kRowsTile && i < n4; i += 64)
      if (i + lane < n4 && i + lane < (wave + 1) * kRowsTile)
        copy16_to_lds(src + 16 * (int64_t)(i + lane), dst + 16 * i);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
  }
  __syncthreads();
  // activation rows [0, 8) of the tile [16][ld1], in place over unit 0's
  // partials (each element is read and written by the same thread; the
  // other units' partials, rows 8 and up, are only read): the unit partials
  // summed in a fixed order, bias, ReLU, zero padding columns.  Rows 8..15
  // keep what they hold; every row past the batch is left out of the
  // fitness, and no layer mixes rows.
  const float* __restrict__ b1 = tail_lds ? lds + tile0 : rest;
  const bool hidden = nd.L > 1;
  for (int idx = tid; idx < kRowsMaxB * NT * 16; idx += 256) {
    const int m = idx / (NT * 16);
    const int n = idx - m * (NT * 16);
    float v = 0.0f;
    if (n < n1) {
      v = lds[m * ld1 + n];
      if (UP > 1) v += lds[(kRowsMaxB + m) * ld1 + n];
      if (UP > 2) {
        v += lds[(2 * kRowsMaxB + m) * ld1 + n];
        v += lds[(3 * kRowsMaxB + m) * ld1 + n];
      }
      v += b1[n];
      if (hidden) v = relu_keep_nan(v);
    }
    lds[m * ld1 + n] = v;
  }
  __syncthreads();
  const float2 res =
      tail_lds ? rows_tail<DT>(lds, lo, nd, lds + tile0, nd.boff[0], b, ylab, tail_vec != 0,
                               partial + j)
               : tail_and_fitness<1, DT>(lds, lo, nd, genome, 0, 1, b, 0, nullptr, tail_vec != 0,
                                         partial + j, ylab);
  if (fin.on && tid == 0) finalize_in_kernel(j, res, b, fin);
}

template <int NT>
__global__ __launch_bounds__(256, NT > 8 ? 3 : 4) void eval_rows_kernel(
    const float* __restrict__ genomes, NetDesc nd, const float* __restrict__ x,
    const int32_t* __restrict__ y, int b, float2* __restrict__ partial, EvalLds lo, int tail_vec,
    FinArgs fin) {
  eval_rows_body<NT, 0, false>(blockIdx.x, genomes, nd, W1Shadow{}, x, y, b, partial, lo,
                               tail_vec, fin);
}

// bfloat16 first layer from the copy (single runs)
template <int NT>
__global__ __launch_bounds__(256, NT > 8 ? 3 : 4) void eval_rows_bf16_kernel(
    const float* __restrict__ genomes, NetDesc nd, W1Shadow wsh, const float* __restrict__ x,
    const int32_t* __restrict__ y, int b, float2* __restrict__ partial, EvalLds lo, int tail_vec,
    FinArgs fin) {
  eval_rows_body<NT, 1, true>(blockIdx.x, genomes, nd, wsh, x, y, b, partial, lo, tail_vec, fin);
}

// ------------------------------------------------------- b <= 4, FP32 --
// Layer 1 on the vector ALUs with W_1 streamed row by row.  The K range is
// split in two halves (k < ka and k >= ka, ka = 4 floor(n0 / 8)); waves 0 and
// 1 take the two halves of rows [0, R), waves 2 and 3 those of rows [R, n1)
// (R = ceil(n1 / 2)), so every wave walks one contiguous block of W_1 (its
// half-rows, 1 KiB contiguous per load instruction: lane l reads elements
// 256 kb + 4 l .. + 3 of the half) with a ring of 4 half-rows in flight,
// against the batch held in registers (MB rows padded to a power of two, up
// to 4; the half-K split halves those registers).  Measured in the
// generation loop at P = 1000, 784-112-32-10: 65 / 66 / 67 us at b = 1 / 2 / 4
// against 72 / 101 / 87 us for whole rows taken by one wave with rows
// interleaved across waves.  At tiny batches the matrix cores multiply mostly
// padding and need the 16-row fragment walk of W_1, which streams slower.
// Each half-row's MB lane-partial sums are reduced over the wave by a
// reduce-scatter butterfly (halving the values at xor 32, 16, ... then
// summing the last one), a fixed order whose tree does not depend on MB; the
// two half sums of a row meet in LDS (half 0 + half 1, then the bias), so
// grouped runs that size the registers for 4 rows reproduce single runs bit
// for bit.  Layer-1 activations go to the LDS tile of the small-batch
// kernel, whose tail and fitness follow.  Rows are loaded non-temporally
// (each is read once, by one wave).
constexpr int kStreamBlocks = 2;  // 256-float blocks per half-row: n0 <= 1024

// K split of the row-streaming kernel: floats of the first half.
__host__ __device__ inline int stream_ka(int n0) { return 4 * (n0 / 8); }

// Floats of LDS the row-streaming kernel uses past the tail layout: the two
// half-row partial tiles [2][16][ld1].
__host__ __device__ inline int stream_part_floats(const EvalLds& lo) { return 2 * 16 * lo.ld1; }

// Floats of the copy of the rest of the genome (b_1 and layers 2..L) that
// the row-streaming kernel keeps in LDS past its partial tiles for the
// epilogue and the tail, 0 when that rest is larger than 16 KiB (they then
// read global memory).
constexpr int64_t kStreamTailMax = 4096;
__host__ __device__ inline int stream_tail_floats(const NetDesc& nd) {
  const int64_t r = nd.genes - nd.boff[0];
  return r <= kStreamTailMax ? (int)((r + 3) & ~(int64_t)3) : 0;
}

template <int MB>
__device__ __forceinline__ void eval_stream_body(int j, const float* __restrict__ genomes,
                                                 const NetDesc& nd, const float* __restrict__ x,
                                                 const int32_t* __restrict__ y, int b,
                                                 float2* __restrict__ partial,
                                                 const EvalLds& lo, int tail_vec,
                                                 const FinArgs& fin) {
  extern __shared__ float lds[];
  constexpr int KB = kStreamBlocks;
  constexpr int RF = 4;  // half-rows in flight per wave
  constexpr int LOG2MB = MB == 1 ? 0 : MB == 2 ? 1 : MB == 4 ? 2 : 3;
  static_assert((1 << LOG2MB) == MB, "MB is 1, 2, 4 or 8");
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const float* __restrict__ W1 = genome + nd.woff[0];
  const float* __restrict__ b1 = genome + nd.boff[0];
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int half = wave & 1;
  const int ka = stream_ka(n0);
  const int kbase = half ? ka : 0;
  const int klen = half ? n0 - ka : ka;
  const bool hidden = nd.L > 1;
  const int ld1 = lo.ld1;
  float* h1 = lds + lo.h1;
  float* part = lds + lo.total;  // [half][16][ld1]
  // the fitness's labels, read ahead (a buffer load: no branch in front of
  // the row loop)
  const int ylab = __builtin_amdgcn_raw_buffer_load_b32(
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(y), 0, b * 4, 0x00020000),
      tid < b ? tid * 4 : 0x40000000, 0, 0);
  // with the global-memory matrix tail (a rest of the genome too large for
  // the LDS copy) the 16-row activation tile starts as zeros (padding rows
  // and columns); the tail of at most 8 rows reads only written entries
  const bool tail_in_lds = stream_tail_floats(nd) != 0;
  if (!tail_in_lds)
    for (int i = tid; i < 16 * ld1; i += 256) h1[i] = 0.0f;

  // all loads of the row loop are raw buffer loads: rows past this wave's
  // share and columns past its half lie outside the resources (or are sent
  // there) and read zero without a memory access, so no load sits behind a
  // branch and the waits of the ring count exactly the older half-rows
  const __amdgpu_buffer_rsrc_t xs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(x), 0, b * n0 * 4, 0x00020000);
  float4 xr[MB][KB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = 256 * kb + 4 * lane;
      const int off = (m < b && k < klen) ? (m * n0 + kbase + k) * 4 : 0x40000000;
      const floatx4 v = __builtin_amdgcn_raw_buffer_load_b128(xs, off, 0, 0);
      xr[m][kb] = make_float4(v[0], v[1], v[2], v[3]);
    }
  const int rows_per = (n1 + 1) >> 1;
  const int r0 = (wave >> 1) * rows_per;
  const int R = r0 < n1 ? (n1 - r0 < rows_per ? n1 - r0 : rows_per) : 0;
  const __amdgpu_buffer_rsrc_t ws =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(W1), 0, n1 * n0 * 4, 0x00020000);
  auto loadrow = [&](int r, float4 (&w)[KB]) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = 256 * kb + 4 * lane;
      const int off = (r < R && k < klen) ? ((r0 + r) * n0 + kbase + k) * 4 : 0x40000000;
      const floatx4 v = __builtin_amdgcn_raw_buffer_load_b128(ws, off, 0, 2);  // nt
      w[kb] = make_float4(v[0], v[1], v[2], v[3]);
    }
  };
  if (!tail_in_lds) __syncthreads();  // the zeroed tile before any row is written (uniform)

  // ring of RF half-rows: the load of half-row r + RF is issued as soon as
  // half-row r has been multiplied
  float4 w[RF][KB];
  auto row = [&](int r, int q) {
    float v[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) v[m] = 0.0f;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        v[m] = fmaf(w[q][kb].x, xr[m][kb].x, v[m]);
        v[m] = fmaf(w[q][kb].y, xr[m][kb].y, v[m]);
        v[m] = fmaf(w[q][kb].z, xr[m][kb].z, v[m]);
        v[m] = fmaf(w[q][kb].w, xr[m][kb].w, v[m]);
      }
    __builtin_amdgcn_sched_barrier(0);
    loadrow(r + RF, w[q]);  // past the share: reads nothing
    __builtin_amdgcn_sched_barrier(0);
    // reduce-scatter: after the level with offset 32 >> lvl, a lane with
    // that bit set holds the upper half of the remaining values
#pragma unroll
    for (int lvl = 0; lvl < LOG2MB; ++lvl) {
      const int off = 32 >> lvl;
      const int hv = MB >> (lvl + 1);
      const bool hi = (lane & off) != 0;
#pragma unroll
      for (int i = 0; i < hv; ++i) {
        const float mine = hi ? v[i + hv] : v[i];
        const float send = hi ? v[i] : v[i + hv];
        v[i] = mine + __shfl_xor(send, off);
      }
    }
#pragma unroll
    for (int off = 32 >> LOG2MB; off >= 1; off >>= 1) v[0] += __shfl_xor(v[0], off);
    int m = 0;
#pragma unroll
    for (int lvl = 0; lvl < LOG2MB; ++lvl)
      if (lane & (32 >> lvl)) m += MB >> (lvl + 1);
    if ((lane & (64 / MB - 1)) == 0 && m < b && r < R) part[(half * 16 + m) * ld1 + r0 + r] = v[0];
  };
#pragma unroll
  for (int q = 0; q < RF; ++q) {
    loadrow(q, w[q]);
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int rb = 0; rb < R; rb += RF) {
#pragma unroll
    for (int q = 0; q < RF; ++q) row(rb + q, q);  // rows past R: zeros, not written
  }
  // the rest of the genome into LDS past the partial tiles where it fits,
  // each wave a quarter once its rows are done, for the epilogue and the
  // tail of at most 8 rows (rows_tail)
  const int tail_n = stream_tail_floats(nd);
  float* tail_copy = part + stream_part_floats(lo);
  if (tail_n) {
    const int n4 = tail_n >> 2;
    const int per = (n4 + 3) >> 2;
    const char* src = reinterpret_cast<const char*>(b1);
    char* dst = reinterpret_cast<char*>(tail_copy);
    for (int i = wave * per; i < (wave + 1) * per && i < n4; i += 64)
      if (i + lane < n4 && i + lane < (wave + 1) * per)
        copy16_to_lds(src + 16 * (int64_t)(i + lane), dst + 16 * i);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(0));
  }
  __syncthreads();
  const float* __restrict__ bias1 = tail_n ? tail_copy : b1;
  for (int idx = tid; idx < b * n1; idx += 256) {
    const int m = idx / n1;
    const int n = idx - m * n1;
    float o = part[m * ld1 + n] + part[(16 + m) * ld1 + n];
    o += bias1[n];
    if (hidden) o = relu_keep_nan(o);
    h1[m * ld1 + n] = o;
  }
  __syncthreads();
  const float2 r =
      tail_n ? rows_tail<0>(lds, lo, nd, tail_copy, nd.boff[0], b, ylab, tail_vec != 0,
                            partial + j)
             : tail_and_fitness<1>(lds, lo, nd, genome, 0, 1, b, 0, nullptr, tail_vec != 0,
                                   partial + j, ylab);
  if (fin.on && tid == 0) finalize_in_kernel(j, r, b, fin);
}

template <int MB>
__global__ __launch_bounds__(256, 2) void eval_stream_kernel(const float* __restrict__ genomes,
                                                             NetDesc nd,
                                                             const float* __restrict__ x,
                                                             const int32_t* __restrict__ y, int b,
                                                             float2* __restrict__ partial,
                                                             EvalLds lo, int tail_vec,
                                                             FinArgs fin) {
  eval_stream_body<MB>(blockIdx.x, genomes, nd, x, y, b, partial, lo, tail_vec, fin);
}

// ---------------------------------------------------------------- large b --
// Body of one workgroup: network j, row tile mt (rows 64*MW*mt ...).  RT:
// the tail from registers (networks reg_tail_ok() takes), else from an LDS
// activation tile; separate kernels, so that neither carries the other's
// registers.
template <int NT, int MW, bool RT>
__device__ __forceinline__ void eval_large_body(int j, int mt, const float* __restrict__ genomes,
                                                const NetDesc& nd, const float* __restrict__ x,
                                                const int32_t* __restrict__ y, int b,
                                                float2* __restrict__ partial, const EvalLds& lo,
                                                int n_pt, int tail_vec) {
  extern __shared__ float lds[];
  constexpr int MT = 64 * MW;              // rows per workgroup
  constexpr int NR = NT * 16;              // staged weight rows
  constexpr int WBUF = 8 * NR * 4;         // floats of one W chunk [8][NR][4]
  constexpr int XBUF = 8 * MT * 4;         // floats of one X chunk [8][MT][4]
  constexpr int BUF = WBUF + XBUF;
  constexpr int WITEMS = NR * 8;           // float4 items of a W chunk
  constexpr int WPT = (WITEMS + 255) / 256;
  constexpr int XPT = MT * 8 / 256;

  const int tid = threadIdx.x;
  const int m0 = mt * MT;
  const int rows = b - m0 < MT ? b - m0 : MT;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const float* __restrict__ W1 = genome + nd.woff[0];
  const int n0 = nd.w[0];
  const int n1 = nd.w[1];
  const int nch = (n0 + 31) >> 5;

  // global -> register prefetch of one 32-wide K chunk; item it covers row
  // it/8, k = k0 + 4*(it%8); LDS slot [c][row ^ 2c] with c = it%8 keeps both
  // the stores and the fragment reads free of bank conflicts
  float4 wr[WPT], xr[XPT];
  auto gload = [&](int ch) {
    const int k0 = ch * 32;
#pragma unroll
    for (int qq = 0; qq < WPT; ++qq) {
      const int it = tid + 256 * qq;
      const int row = it >> 3;
      const int k = k0 + 4 * (it & 7);
      wr[qq] = (it < WITEMS && row < n1 && k < n0)
                   ? *reinterpret_cast<const float4*>(W1 + (int64_t)row * n0 + k)
                   : zero4();
    }
#pragma unroll
    for (int qq = 0; qq < XPT; ++qq) {
      const int it = tid + 256 * qq;
      const int m = it >> 3;
      const int k = k0 + 4 * (it & 7);
      xr[qq] = (m < rows && k < n0)
                   ? *reinterpret_cast<const float4*>(x + (int64_t)(m0 + m) * n0 + k)
                   : zero4();
    }
  };
  auto sstore = [&](int buf) {
    float* wst = lds + buf * BUF;
    float* xst = wst + WBUF;
#pragma unroll
    for (int qq = 0; qq < WPT; ++qq) {
      const int it = tid + 256 * qq;
      const int c = it & 7;
      if (it < WITEMS)
        *reinterpret_cast<float4*>(wst + (c * NR + ((it >> 3) ^ (2 * c))) * 4) = wr[qq];
    }
#pragma unroll
    for (int qq = 0; qq < XPT; ++qq) {
      const int it = tid + 256 * qq;
      const int c = it & 7;
      *reinterpret_cast<float4*>(xst + (c * MT + ((it >> 3) ^ (2 * c))) * 4) = xr[qq];
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

  gload(0);
  sstore(0);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) gload(ch + 1);
    const float* wst = lds + buf * BUF;
    const float* xst = wst + WBUF;
#pragma unroll
    for (int ss = 0; ss < 2; ++ss) {
      if (ch * 32 + ss * 16 < n0) {
        const int c = ss * 4 + kq;
        float4 xa[MW], wb[NT];
#pragma unroll
        for (int mi = 0; mi < MW; ++mi)
          xa[mi] = *reinterpret_cast<const float4*>(
              xst + (c * MT + ((wave * MW * 16 + mi * 16 + mn) ^ (2 * c))) * 4);
#pragma unroll
        for (int t = 0; t < NT; ++t)
          wb[t] = *reinterpret_cast<const float4*>(wst + (c * NR + ((t * 16 + mn) ^ (2 * c))) * 4);
#pragma unroll
        for (int mi = 0; mi < MW; ++mi) mfma_superstep_t<NT>(xa[mi], wb, acc[mi]);
      }
    }
    if (ch + 1 < nch) sstore(buf ^ 1);
    __syncthreads();
  }

  // epilogue (staging is dead now): the tail from registers when the
  // network allows it (tail genes copied to LDS first), else 64-row passes
  // over an LDS activation tile; one partial per 64 rows either way
  if constexpr (RT) {
    copy_tail_genes(genome, nd, lds);
    int ylab[MW];
#pragma unroll
    for (int mi = 0; mi < MW; ++mi) {
      const int r = m0 + wave * MW * 16 + mi * 16 + mn;
      ylab[mi] = r < b ? y[r] : 0;
    }
    float* red = lds + reg_tail_copy_floats(nd);
    __syncthreads();
    reg_tail<NT, MW>(acc, 1.0f, lds, nd, m0, wave * MW * 16, b, ylab, red,
                     partial + (int64_t)j * n_pt, m0 / 64);
  } else {
    lds_epilogue<NT, MW>(lds, acc, 1.0f, j, mt, genome, nd, y, b, partial, lo, n_pt, tail_vec);
  }
}

// XCD-aware order (hardware workgroup i runs on XCD i % 8): each XCD gets a
// contiguous range of logical ids, so one individual's row tiles share that
// XCD's L2.
__device__ __forceinline__ int xcd_order(int i, int total) {
  const int q = total >> 3;
  const int r = total & 7;
  const int xcd = i & 7;
  const int kk = i >> 3;
  return xcd < r ? xcd * (q + 1) + kk : r * (q + 1) + (xcd - r) * q + kk;
}

template <int NT, int MW, bool RT>
__global__ __launch_bounds__(256, MW * NT <= 16 ? 2 : 1) void eval_large_kernel(const float* __restrict__ genomes,
                                                         NetDesc nd, const float* __restrict__ x,
                                                         const int32_t* __restrict__ y, int b,
                                                         float2* __restrict__ partial,
                                                         EvalLds lo, int n_wt, int n_pt, int pop,
                                                         int tail_vec) {
  const int L = xcd_order(blockIdx.x, n_wt * pop);
  const int j = L / n_wt;
  eval_large_body<NT, MW, RT>(j, L - j * n_wt, genomes, nd, x, y, b, partial, lo, n_pt, tail_vec);
}

// -------------------------------------------------------------- dispatch --

static int round16(int v) { return (v + 15) & ~15; }

static int tail_width(const NetDesc& nd) {
  int w = 4;
  for (int l = 2; l <= nd.L; ++l) w = nd.w[l] > w ? nd.w[l] : w;
  return round16(w) + 4;
}

static bool tail_vectorizable(const NetDesc& nd) {
  for (int l = 1; l < nd.L; ++l)
    if (nd.w[l] % 4 != 0) return false;
  return true;
}

// Tail regions for a tile of `rows` (padded) rows: the layer-1 tile (also
// the second tail ping-pong buffer), the first tail buffer, per-row results.
static EvalLds tail_layout(const NetDesc& nd, int rows) {
  EvalLds lo;
  lo.ld1 = round16(nd.w[1]) + 4;
  lo.ldt = tail_width(nd);
  const int ldmax = lo.ld1 > lo.ldt ? lo.ld1 : lo.ldt;
  lo.h1 = 0;
  lo.ta = rows * ldmax;
  lo.ll = lo.ta + rows * lo.ldt;
  lo.cor = lo.ll + rows;
  lo.total = lo.cor + rows;
  return lo;
}

static size_t small_lds_bytes(const NetDesc& nd, EvalLds* out) {
  EvalLds lo = tail_layout(nd, 16);
  const int part = 4 * 16 * lo.ld1;  // the four K-partial tiles
  lo.total = lo.total > part ? lo.total : part;
  if (out) *out = lo;
  return (size_t)lo.total * 4;
}

static size_t large_lds_rt(const NetDesc& nd, int nt, int mw, EvalLds* out);

template <int NT, int MW>
static size_t large_lds_bytes(const NetDesc& nd, EvalLds* out) {
  return large_lds_rt(nd, NT, MW, out);
}

static constexpr size_t kMaxLds = 160 * 1024;
static constexpr size_t kTwoPerCu = 80 * 1024;

static bool use_small(int b) { return b <= 16; }

template <int NT>
static int large_mw(const NetDesc& nd, int b) {
  if (b > 64 && large_lds_bytes<NT, 2>(nd, nullptr) <= kTwoPerCu) return 2;
  return 1;
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  if (bytes > kMaxLds) return hipErrorInvalidValue;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// Partial row sums per network: one (small batches) or one per 64 rows.
template <int NT>
static int mtiles_nt(const NetDesc& nd, int b) {
  if (use_small(b)) return 1;
  return (b + 63) / 64;
}

template <int NT, int DT>
static hipError_t launch_small(const float* genomes, const NetDesc& nd, int pop, const float* x,
                               const int32_t* y, int b, float2* partial, const uint32_t* w_amax,
                               const uint32_t* x_amax, hipStream_t s, const FinArgs& fin) {
  const int tv = tail_vectorizable(nd) ? 1 : 0;
  EvalLds lo;
  const size_t bytes = small_lds_bytes(nd, &lo);
  hipError_t e = allow_lds(eval_small_kernel<NT, DT>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eval_small_kernel<NT, DT>), dim3((unsigned)pop), dim3(256), bytes, s,
                     genomes, nd, x, y, b, partial, lo, tv, w_amax, x_amax, fin);
  return hipGetLastError();
}

template <int NT>
static hipError_t launch_small_bf16(const float* genomes, const NetDesc& nd, int pop,
                                    const W1Shadow& wsh, const float* x, const int32_t* y, int b,
                                    float2* partial, hipStream_t s, const FinArgs& fin) {
  const int tv = tail_vectorizable(nd) ? 1 : 0;
  EvalLds lo;
  const size_t bytes = small_lds_bytes(nd, &lo);
  hipError_t e = allow_lds(eval_small_bf16_kernel<NT>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eval_small_bf16_kernel<NT>), dim3((unsigned)pop), dim3(256), bytes, s,
                     genomes, nd, wsh, x, y, b, partial, lo, tv, fin);
  return hipGetLastError();
}

template <int NT>
static hipError_t launch_small_fp8(const float* genomes, const NetDesc& nd, int pop,
                                   const W1Fp8& w8, const float* x, const uint32_t* x_amax,
                                   const int32_t* y, int b, float2* partial, hipStream_t s,
                                   const FinArgs& fin) {
  const int tv = tail_vectorizable(nd) ? 1 : 0;
  EvalLds lo;
  const size_t bytes = small_lds_bytes(nd, &lo);
  hipError_t e = allow_lds(eval_small_fp8_kernel<NT>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eval_small_fp8_kernel<NT>), dim3((unsigned)pop), dim3(256), bytes, s,
                     genomes, nd, w8, x, x_amax, y, b, partial, lo, tv, fin);
  return hipGetLastError();
}

template <int NT, int MW, bool RT>
static hipError_t launch_large(const float* genomes, const NetDesc& nd, int pop, const float* x,
                               const int32_t* y, int b, float2* partial, int n_pt, int tv,
                               hipStream_t s) {
  EvalLds lo;
  const int n_wt = (b + 64 * MW - 1) / (64 * MW);
  const size_t bytes = large_lds_bytes<NT, MW>(nd, &lo);
  hipError_t e = allow_lds(eval_large_kernel<NT, MW, RT>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eval_large_kernel<NT, MW, RT>), dim3((unsigned)(n_wt * pop)), dim3(256),
                     bytes, s, genomes, nd, x, y, b, partial, lo, n_wt, n_pt, pop, tv);
  return hipGetLastError();
}

// 1 KiB-row kernel for b <= 8: n0 a multiple of 4 and at most 4 units of 256.
static size_t rows_lds_bytes(const NetDesc& nd, EvalLds* out) {
  const EvalLds lo = tail_layout(nd, 16);
  if (out) *out = lo;
  return (size_t)rows_lds_floats(lo) * 4;
}

static bool rows_ok(const NetDesc& nd, int b) {
  const int n0 = nd.w[0];
  return b >= 1 && b <= kRowsMaxB && n0 % 4 == 0 && n0 >= 4 && n0 <= 4 * kRowsUnit &&
         (int64_t)nd.w[1] * n0 * 4 < 0x40000000 && rows_lds_bytes(nd, nullptr) <= kMaxLds;
}

template <int NT>
static hipError_t launch_rows(const float* genomes, const NetDesc& nd, int pop, const float* x,
                              const int32_t* y, int b, float2* partial, hipStream_t s,
                              const FinArgs& fin) {
  const int tv = tail_vectorizable(nd) ? 1 : 0;
  EvalLds lo;
  const size_t bytes = rows_lds_bytes(nd, &lo);
  hipError_t e = allow_lds(eval_rows_kernel<NT>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eval_rows_kernel<NT>), dim3((unsigned)pop), dim3(256), bytes, s, genomes,
                     nd, x, y, b, partial, lo, tv, fin);
  return hipGetLastError();
}

template <int NT>
static hipError_t launch_rows_bf16(const float* genomes, const NetDesc& nd, int pop,
                                   const W1Shadow& wsh, const float* x, const int32_t* y, int b,
                                   float2* partial, hipStream_t s, const FinArgs& fin) {
  const int tv = tail_vectorizable(nd) ? 1 : 0;
  EvalLds lo;
  const size_t bytes = rows_lds_bytes(nd, &lo);
  hipError_t e = allow_lds(eval_rows_bf16_kernel<NT>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eval_rows_bf16_kernel<NT>), dim3((unsigned)pop), dim3(256), bytes, s,
                     genomes, nd, wsh, x, y, b, partial, lo, tv, fin);
  return hipGetLastError();
}

// Row-streaming kernel for b <= 4: n0 a multiple of 4 and at most 1024.
static constexpr int kStreamMaxRows = 4;
static size_t stream_lds_bytes(const NetDesc& nd) {
  const EvalLds lo = tail_layout(nd, 16);
  return (size_t)(lo.total + stream_part_floats(lo) + stream_tail_floats(nd)) * 4;
}

static bool stream_ok(const NetDesc& nd, int b) {
  const int n0 = nd.w[0];
  return b >= 1 && b <= kStreamMaxRows && n0 % 4 == 0 && n0 >= 8 &&
         n0 - stream_ka(n0) <= 256 * kStreamBlocks && stream_lds_bytes(nd) <= kMaxLds;
}

static int stream_rows(int b) { return b <= 1 ? 1 : b <= 2 ? 2 : 4; }

template <int MB>
static hipError_t launch_stream_mb(const float* genomes, const NetDesc& nd, int pop,
                                   const float* x, const int32_t* y, int b, float2* partial,
                                   hipStream_t s, const FinArgs& fin) {
  const int tv = tail_vectorizable(nd) ? 1 : 0;
  const EvalLds lo = tail_layout(nd, 16);  // the activation tile and the tail buffers
  const size_t bytes = stream_lds_bytes(nd);      // + the half-row partial tiles
  hipError_t e = allow_lds(eval_stream_kernel<MB>, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eval_stream_kernel<MB>), dim3((unsigned)pop), dim3(256), bytes, s, genomes,
                     nd, x, y, b, partial, lo, tv, fin);
  return hipGetLastError();
}

static hipError_t launch_stream(const float* genomes, const NetDesc& nd, int pop, const float* x,
                                const int32_t* y, int b, float2* partial, hipStream_t s,
                                const FinArgs& fin) {
  switch (stream_rows(b)) {
    case 1:
      return launch_stream_mb<1>(genomes, nd, pop, x, y, b, partial, s, fin);
    case 2:
      return launch_stream_mb<2>(genomes, nd, pop, x, y, b, partial, s, fin);
    default:
      return launch_stream_mb<4>(genomes, nd, pop, x, y, b, partial, s, fin);
  }
}

template <int NT>
static hipError_t launch_nt(const float* genomes, const NetDesc& nd, int pop, const float* x,
                            const int32_t* y, int b, float2* partial, hipStream_t s,
                            const FinArgs* fin, bool* finalized) {
  const int tv = tail_vectorizable(nd) ? 1 : 0;
  const FinArgs none{};
  const bool one_tile = stream_ok(nd, b) || use_small(b);
  if (finalized) *finalized = fin && one_tile;
  if (stream_ok(nd, b))
    return launch_stream(genomes, nd, pop, x, y, b, partial, s, fin ? *fin : none);
  if (rows_ok(nd, b))
    return launch_rows<NT>(genomes, nd, pop, x, y, b, partial, s, fin ? *fin : none);
  if (use_small(b))
    return launch_small<NT, 0>(genomes, nd, pop, x, y, b, partial, nullptr, nullptr, s,
                               fin ? *fin : none);
  const int n_pt = mtiles_nt<NT>(nd, b);
  const bool rt = reg_tail_ok(nd);
  if (rt && eval_lfw_supported(nd, b, large_mw<NT>(nd, b), x))
    return launch_evaluate_lfw(genomes, nd, pop, x, y, b, large_mw<NT>(nd, b), partial, s);
  if (large_mw<NT>(nd, b) == 2)
    return rt ? launch_large<NT, 2, true>(genomes, nd, pop, x, y, b, partial, n_pt, tv, s)
              : launch_large<NT, 2, false>(genomes, nd, pop, x, y, b, partial, n_pt, tv, s);
  return rt ? launch_large<NT, 1, true>(genomes, nd, pop, x, y, b, partial, n_pt, tv, s)
            : launch_large<NT, 1, false>(genomes, nd, pop, x, y, b, partial, n_pt, tv, s);
}

#define LEEA_NT_SWITCH(EXPR, DEFAULT)                                               \
  switch ((nd.w[1] + 15) / 16) {                                                     \
    case 1: { constexpr int N = 1; return EXPR; }                                   \
    case 2: { constexpr int N = 2; return EXPR; }                                   \
    case 3: { constexpr int N = 3; return EXPR; }                                   \
    case 4: { constexpr int N = 4; return EXPR; }                                   \
    case 5: { constexpr int N = 5; return EXPR; }                                   \
    case 6: { constexpr int N = 6; return EXPR; }                                   \
    case 7: { constexpr int N = 7; return EXPR; }                                   \
    case 8: { constexpr int N = 8; return EXPR; }                                   \
    case 9: { constexpr int N = 9; return EXPR; }                                   \
    case 10: { constexpr int N = 10; return EXPR; }                                 \
    case 11: { constexpr int N = 11; return EXPR; }                                 \
    case 12: { constexpr int N = 12; return EXPR; }                                 \
    case 13: { constexpr int N = 13; return EXPR; }                                 \
    case 14: { constexpr int N = 14; return EXPR; }                                 \
    case 15: { constexpr int N = 15; return EXPR; }                                 \
    case 16: { constexpr int N = 16; return EXPR; }                                 \
    default: return DEFAULT;                                                        \
  }

int eval_mtiles(const NetDesc& nd, int b) { LEEA_NT_SWITCH((mtiles_nt<N>(nd, b)), 1) }

bool large_reg_tail(const NetDesc& nd) { return reg_tail_ok(nd); }

bool eval_stream_supported(const NetDesc& nd, int b) { return stream_ok(nd, b); }

bool eval_rows_supported(const NetDesc& nd, int b) { return !stream_ok(nd, b) && rows_ok(nd, b); }

hipError_t launch_evaluate(const float* genomes, const NetDesc& nd, int pop, const float* x,
                           const int32_t* y, int b, float2* partial, hipStream_t s,
                           const FinArgs* fin, bool* finalized) {
  if (finalized) *finalized = false;
  LEEA_NT_SWITCH((launch_nt<N>(genomes, nd, pop, x, y, b, partial, s, fin, finalized)),
                 hipErrorInvalidValue)
}

hipError_t launch_evaluate_small_lp(int dt, const float* genomes, const NetDesc& nd, int pop,
                                    const float* xq, const int32_t* y, int b, float2* partial,
                                    const uint32_t* w_amax, const uint32_t* x_amax,
                                    hipStream_t s) {
  if (dt == 1)
    LEEA_NT_SWITCH((launch_small<N, 1>(genomes, nd, pop, xq, y, b, partial, w_amax, x_amax, s,
                                       FinArgs{})),
                   hipErrorInvalidValue)
  LEEA_NT_SWITCH((launch_small<N, 2>(genomes, nd, pop, xq, y, b, partial, w_amax, x_amax, s,
                                     FinArgs{})),
                 hipErrorInvalidValue)
}

hipError_t launch_evaluate_small_bf16(const float* genomes, const NetDesc& nd, int pop,
                                      const W1Shadow& wsh, const float* x, const int32_t* y,
                                      int b, float2* partial, hipStream_t s, const FinArgs& fin) {
  if (wsh.p && rows_ok(nd, b))
    LEEA_NT_SWITCH((launch_rows_bf16<N>(genomes, nd, pop, wsh, x, y, b, partial, s, fin)),
                   hipErrorInvalidValue)
  LEEA_NT_SWITCH((launch_small_bf16<N>(genomes, nd, pop, wsh, x, y, b, partial, s, fin)),
                 hipErrorInvalidValue)
}

hipError_t launch_evaluate_small_fp8(const float* genomes, const NetDesc& nd, int pop,
                                     const W1Fp8& w8, const float* x, const uint32_t* x_amax,
                                     const int32_t* y, int b, float2* partial, hipStream_t s,
                                     const FinArgs& fin) {
  LEEA_NT_SWITCH((launch_small_fp8<N>(genomes, nd, pop, w8, x, x_amax, y, b, partial, s, fin)),
                 hipErrorInvalidValue)
}

#undef LEEA_NT_SWITCH

// ------------------------------------------------------------- shapes --

// LDS of the large-batch kernel (floats): the staging double buffer, then
// either the tail genes and the row-sum scratch of the register tail or the
// 64-row activation tile of the LDS epilogue.
static size_t large_lds_rt(const NetDesc& nd, int nt, int mw, EvalLds* out) {
  EvalLds lo = lp_tail_layout(nd, 64);
  const int staging = 2 * (8 * nt * 16 * 4 + 8 * 64 * mw * 4);
  const int rt = reg_tail_ok(nd) ? reg_tail_copy_floats(nd) + 8 * mw : 0;
  int total = lo.total > staging ? lo.total : staging;
  total = total > rt ? total : rt;
  lo.total = total;
  if (out) *out = lo;
  return (size_t)lo.total * 4;
}

bool eval_shape_f32(const NetDesc& nd, int b, int kind, int mw, EvalShape* out) {
  const int nt = (nd.w[1] + 15) / 16;
  if (nt < 1 || nt > 16 || b < 1) return false;
  if (kind < 0) kind = stream_ok(nd, b) ? 3 : rows_ok(nd, b) ? 4 : (use_small(b) ? 0 : 1);
  EvalShape sh;
  memset(&sh, 0, sizeof sh);
  sh.tail_vec = tail_vectorizable(nd) ? 1 : 0;
  if (kind == 3) {
    if (!stream_ok(nd, b)) return false;
    sh.kind = 3;
    sh.mw = 1;
    sh.n_wt = 1;
    sh.n_pt = 1;
    sh.pass_rows = 16;
    sh.lo = tail_layout(nd, 16);
    sh.lds = stream_lds_bytes(nd);
  } else if (kind == 4) {
    if (!rows_ok(nd, b)) return false;
    sh.kind = 4;
    sh.mw = 1;
    sh.n_wt = 1;
    sh.n_pt = 1;
    sh.pass_rows = 16;
    sh.lds = rows_lds_bytes(nd, &sh.lo);
  } else if (kind == 0) {
    if (b > 16) return false;
    sh.kind = 0;
    sh.mw = 1;
    sh.n_wt = 1;
    sh.n_pt = 1;
    sh.pass_rows = 16;
    sh.lds = small_lds_bytes(nd, &sh.lo);
  } else if (kind == 1) {
    if (mw <= 0) mw = (b > 64 && large_lds_rt(nd, nt, 2, nullptr) <= kTwoPerCu) ? 2 : 1;
    if (mw != 1 && mw != 2) return false;
    sh.kind = 1;
    sh.mw = mw;
    sh.n_wt = (b + 64 * mw - 1) / (64 * mw);
    sh.n_pt = (b + 63) / 64;
    sh.pass_rows = 64;
    sh.lds = large_lds_rt(nd, nt, mw, &sh.lo);
  } else {
    return false;
  }
  if (sh.lds > kMaxLds) return false;
  *out = sh;
  return true;
}

// ------------------------------------------------- grouped (many runs) --
// Population buffer: the one made by this generation's variation (the
// state advances right after it) or the initial one.

template <int NT, int DT>
__global__ __launch_bounds__(256, NT > 8 ? 3 : 4) void runs_eval_small_kernel(
    const RunDesc* __restrict__ runs, const BatchState* __restrict__ st,
    const int* __restrict__ off, const int* __restrict__ ids, int n) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  if constexpr (DT == 1)  // bfloat16 matrix cores, W_1 rounded on the way (no copy)
    eval_small_bf16_body<NT, false>(blockIdx.x - off[i], d.genomes[st->cur], d.nd, W1Shadow{},
                                    d.xb, d.yb, d.b, d.partial, d.lo, d.tail_vec, FinArgs{});
  else
    eval_small_body<NT, DT>(blockIdx.x - off[i], d.genomes[st->cur], d.nd, d.xb, d.yb, d.b,
                            d.partial, d.lo, d.tail_vec, nullptr, nullptr, FinArgs{});
}

// Row-streaming evaluation of the float32 runs with b <= 4: the batch
// registers sized for 4 rows whatever each run's b (the per-row sums and
// their butterfly tree do not depend on that size, so each run gets
// bitwise what it gets alone).
__global__ __launch_bounds__(256, 2) void runs_eval_stream_kernel(
    const RunDesc* __restrict__ runs, const BatchState* __restrict__ st,
    const int* __restrict__ off, const int* __restrict__ ids, int n) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  eval_stream_body<4>(blockIdx.x - off[i], d.genomes[st->cur], d.nd, d.xb, d.yb, d.b, d.partial,
                      d.lo, d.tail_vec, FinArgs{});
}

// 1 KiB-row evaluation of the float32 runs with b <= 8 (each run's own n0,
// n1 and b; the kernel sizes nothing by them but the epilogue's columns).
template <int NT>
__global__ __launch_bounds__(256, NT > 8 ? 3 : 4) void runs_eval_rows_kernel(
    const RunDesc* __restrict__ runs, const BatchState* __restrict__ st,
    const int* __restrict__ off, const int* __restrict__ ids, int n) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  eval_rows_body<NT, 0, false>(blockIdx.x - off[i], d.genomes[st->cur], d.nd, W1Shadow{}, d.xb,
                               d.yb, d.b, d.partial, d.lo, d.tail_vec, FinArgs{});
}

// bfloat16 runs: W_1 read as float32 and rounded in registers (no copy),
// bitwise what a single run gets from its copy
template <int NT>
__global__ __launch_bounds__(256, 2) void runs_eval_rows_bf16_kernel(
    const RunDesc* __restrict__ runs, const BatchState* __restrict__ st,
    const int* __restrict__ off, const int* __restrict__ ids, int n) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  eval_rows_body<NT, 1, false>(blockIdx.x - off[i], d.genomes[st->cur], d.nd, W1Shadow{}, d.xb,
                               d.yb, d.b, d.partial, d.lo, d.tail_vec, FinArgs{});
}

template <int NT, int MW, bool RT>
__global__ __launch_bounds__(256, MW * NT <= 16 ? 2 : 1) void runs_eval_large_kernel(const RunDesc* __restrict__ runs,
                                                              const BatchState* __restrict__ st,
                                                              const int* __restrict__ off,
                                                              const int* __restrict__ ids, int n,
                                                              int total) {
  const int L = xcd_order(blockIdx.x, total);
  const int i = find_group(off, n, L);
  const RunDesc& d = runs[ids[i]];
  const int local = L - off[i];
  const int j = local / d.n_wt;
  eval_large_body<NT, MW, RT>(j, local - j * d.n_wt, d.genomes[st->cur], d.nd, d.xb, d.yb, d.b,
                              d.partial, d.lo, d.n_pt, d.tail_vec);
}

template <typename K>
static hipError_t allow_lds_any(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int NT, int MW, bool RT>
static hipError_t launch_runs_large(const RunDesc* runs, const BatchState* st, const Group& g,
                                    hipStream_t s) {
  hipError_t e = allow_lds_any(runs_eval_large_kernel<NT, MW, RT>, g.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((runs_eval_large_kernel<NT, MW, RT>), dim3((unsigned)g.blocks), dim3(256),
                     g.lds, s, runs, st, g.off, g.ids, g.n, g.blocks);
  return hipGetLastError();
}

template <int NT>
static hipError_t launch_runs_eval_nt(int kind, int mw, int dt, int rt, const RunDesc* runs,
                                      const BatchState* st, const Group& g, hipStream_t s) {
  hipError_t e;
  if (kind == 3) {
    if (dt != 0) return hipErrorInvalidValue;
    e = allow_lds_any(runs_eval_stream_kernel, g.lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(runs_eval_stream_kernel, dim3((unsigned)g.blocks), dim3(256), g.lds, s, runs,
                       st, g.off, g.ids, g.n);
    return hipGetLastError();
  }
  if (kind == 4) {
    if (dt == 0) {
      e = allow_lds_any(runs_eval_rows_kernel<NT>, g.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((runs_eval_rows_kernel<NT>), dim3((unsigned)g.blocks), dim3(256), g.lds,
                         s, runs, st, g.off, g.ids, g.n);
    } else if (dt == 1) {
      e = allow_lds_any(runs_eval_rows_bf16_kernel<NT>, g.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((runs_eval_rows_bf16_kernel<NT>), dim3((unsigned)g.blocks), dim3(256),
                         g.lds, s, runs, st, g.off, g.ids, g.n);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (kind == 0) {
    if (dt == 0) {
      e = allow_lds_any(runs_eval_small_kernel<NT, 0>, g.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((runs_eval_small_kernel<NT, 0>), dim3((unsigned)g.blocks), dim3(256),
                         g.lds, s, runs, st, g.off, g.ids, g.n);
    } else if (dt == 1) {
      e = allow_lds_any(runs_eval_small_kernel<NT, 1>, g.lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((runs_eval_small_kernel<NT, 1>), dim3((unsigned)g.blocks), dim3(256),
                         g.lds, s, runs, st, g.off, g.ids, g.n);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (kind == 1) {
    if (rt == 2) return launch_runs_lfw(NT, mw, runs, st, g, s);
    if (mw == 1)
      return rt ? launch_runs_large<NT, 1, true>(runs, st, g, s)
                : launch_runs_large<NT, 1, false>(runs, st, g, s);
    return rt ? launch_runs_large<NT, 2, true>(runs, st, g, s)
              : launch_runs_large<NT, 2, false>(runs, st, g, s);
  }
  return launch_runs_eval_lp(NT, mw, dt, rt, runs, st, g, s);
}

hipError_t launch_runs_eval(int kind, int nt, int mw, int dt, int rt, const RunDesc* runs,
                            const BatchState* st, const Group& g, hipStream_t s) {
  switch (nt) {
#define LEEA_RUNS_CASE(N) \
  case N:                 \
    return launch_runs_eval_nt<N>(kind, mw, dt, rt, runs, st, g, s);
    LEEA_RUNS_CASE(1) LEEA_RUNS_CASE(2) LEEA_RUNS_CASE(3) LEEA_RUNS_CASE(4) LEEA_RUNS_CASE(5)
    LEEA_RUNS_CASE(6) LEEA_RUNS_CASE(7) LEEA_RUNS_CASE(8) LEEA_RUNS_CASE(9) LEEA_RUNS_CASE(10)
    LEEA_RUNS_CASE(11) LEEA_RUNS_CASE(12) LEEA_RUNS_CASE(13) LEEA_RUNS_CASE(14)
    LEEA_RUNS_CASE(15) LEEA_RUNS_CASE(16)
#undef LEEA_RUNS_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Fitness = (sum of per-sample log-likelihoods) / b, accuracy = correct / b,
// summed over row tiles in order (finalize_values).
__device__ __forceinline__ void finalize_one(int j, const float2* __restrict__ partial,
                                             int n_mt, int b, const float* __restrict__ f_inh,
                                             int use_inh, float alpha, float* f_adj, float* f_raw,
                                             float* acc, float* f_adj_out, float* f_raw_out,
                                             float* acc_out) {
#pragma clang fp contract(off)
  float s = 0.0f, c = 0.0f;
  for (int t = 0; t < n_mt; ++t) {
    const float2 p = partial[(int64_t)j * n_mt + t];
    s += p.x;
    c += p.y;
  }
  finalize_values(j, s, c, b, f_inh, use_inh, alpha, f_adj, f_raw, acc, f_adj_out, f_raw_out,
                  acc_out);
}

__global__ void finalize_kernel(const float2* __restrict__ partial, int pop, int n_mt, int b,
                                const float* __restrict__ f_inh, int use_inh, float alpha,
                                float* f_adj, float* f_raw, float* acc, float* f_adj_out,
                                float* f_raw_out, float* acc_out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= pop) return;
  finalize_one(j, partial, n_mt, b, f_inh, use_inh, alpha, f_adj, f_raw, acc, f_adj_out,
               f_raw_out, acc_out);
}

__global__ void runs_finalize_kernel(const RunDesc* __restrict__ runs,
                                     const BatchState* __restrict__ st,
                                     const int* __restrict__ off, const int* __restrict__ ids,
                                     int n) {
  const int i = find_group(off, n, blockIdx.x);
  const RunDesc& d = runs[ids[i]];
  const int j = (blockIdx.x - off[i]) * 256 + threadIdx.x;
  if (j >= d.pop) return;
  const int use_inh = st->has_inh && d.alpha != 1.0f;
  finalize_one(j, d.partial, d.n_pt, d.b, d.f_inh[st->inh], use_inh, d.alpha, d.f_adj, d.f_raw,
               d.acc, nullptr, nullptr, nullptr);
}

hipError_t launch_runs_finalize(const RunDesc* runs, const BatchState* st, const Group& g,
                                hipStream_t s) {
  hipLaunchKernelGGL(runs_finalize_kernel, dim3((unsigned)g.blocks), dim3(256), 0, s, runs, st,
                     g.off, g.ids, g.n);
  return hipGetLastError();
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
