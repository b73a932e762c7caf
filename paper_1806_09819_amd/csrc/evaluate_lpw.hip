// Large-batch population forward pass with a bfloat16 first layer that reads
// W_1 from its bfloat16 copy (W1Shadow, written by the variation kernel as
// each child is made) instead of converting the float32 genome on the fly.
//
// Same product as the other bfloat16 kernel (section 3.3: X * [W1_1 .. W1_P]^T,
// one v_mfma_f32_16x16x32_bf16 per (row tile, column tile, 32-wide K chunk),
// FP32 accumulation in K order, then the FP32 tail and fitness), with the
// staging done by the memory system instead of registers:
// * global_load_lds_dwordx4 copies a block of 16 rows x 64 bytes (one
//   32-wide K chunk) straight into LDS: lane l writes bytes 16 l .. 16 l + 15
//   of the 1 KiB block and reads the 16-byte slot that the bank swizzle
//   places at its position, so the swizzle costs nothing.  The batch is
//   chunk-major (a block is 1 KiB contiguous); the W_1 copy is row-major
//   (a block is 16 row pieces of 64 bytes, L2 lines shared with the
//   neighbouring chunk), which keeps the variation kernel's writes of it
//   contiguous.
// * S stages, S - 1 chunks in flight: chunk ch + S - 1 is requested right
//   after the barrier of chunk ch.  The stages are separate static LDS
//   arrays, so the compiler can tell a stage being read from the stages
//   being copied into and adds no wait for copies still in flight (with one
//   array, or the dynamic LDS, it drains every copy before each read).
// * Layer 1 comes out transposed (W_1 X^T) and the tail layers and the
//   fitness run from registers (reg_tail.hpp), reading the tail genes that
//   were requested before the main loop and parked in stage 1 after it.  Every wave
//   issues the same number Q of block copies per chunk (a wave with no block
//   left re-copies its previous one: same bytes to the same place), so
//   "chunk ch has landed" is vmcnt <= (S-2) Q, waited for explicitly before
//   the barrier.  Past the last chunk the last one is copied again into the
//   free stage, which keeps that count exact.
// * No register staging, no conversion: the main loop is copy issue, LDS
//   fragment reads and matrix instructions.
#include <type_traits>

#include "lowp.hpp"
#include "lp_common.hpp"
#include "runs.hpp"

namespace leea {

typedef __bf16 bf16x8w __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx4 mfma_bf16(const uint4& a, const uint4& b, const floatx4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8w, a),
                                                 __builtin_bit_cast(bf16x8w, b), c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma_fp8(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1,
                                            const floatx4& c) {
  const unsigned long long a = (unsigned long long)a0 | ((unsigned long long)a1 << 32);
  const unsigned long long b = (unsigned long long)b0 | ((unsigned long long)b1 << 32);
  return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8((long)a, (long)b, c, 0, 0, 0);
}

// Wait until at most N copies of this wave are in flight and its LDS reads
// are done, then the workgroup barrier; the compiler moves no memory access
// across either side.
template <int N>
__device__ __forceinline__ void wait_copies_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0(N));
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// LDS plan (bytes): a stage holds NT 16-row blocks of W_1 and 4 MW of the
// batch, 64 bytes per row.  After the main loop stage 1 takes the tail genes
// (b_1 .. b_L, up to 20 KiB; the 784-112-32-10 network's take 15.9 KiB) that
// the register tail reads, and stage 0 its row-sum scratch.  As many stages
// (up to four) as fit 80 KiB, which keeps two workgroups per CU; at
// b = 512 four stages measured 3 % faster than three.
constexpr int lpw_stage_bytes(int nt, int mw) { return (nt * 16 + 64 * mw) * 64; }
constexpr int kTailGenesCap = 20 * 1024;
constexpr int lpw_stage1_bytes(int nt, int mw) {
  return lpw_stage_bytes(nt, mw) > kTailGenesCap ? lpw_stage_bytes(nt, mw) : kTailGenesCap;
}
constexpr int lpw_stages(int nt, int mw) {
  return lpw_stage1_bytes(nt, mw) + 3 * lpw_stage_bytes(nt, mw) <= 80 * 1024   ? 4
         : lpw_stage1_bytes(nt, mw) + 2 * lpw_stage_bytes(nt, mw) <= 80 * 1024 ? 3
                                                                                : 2;
}
constexpr int lpw_lds_bytes(int nt, int mw) {
  return lpw_stage1_bytes(nt, mw) + (lpw_stages(nt, mw) - 1) * lpw_stage_bytes(nt, mw);
}

// DT = 1: bfloat16 (32-element K chunks, one v_mfma_f32_16x16x32_bf16 per
// tile pair and chunk).  DT = 2: FP8 E4M3 from the FP8 copy of W_1 and the
// FP8 chunk-major batch (64-element chunks: the 16 bytes of a lane feed two
// v_mfma_f32_16x16x32_fp8_fp8, its first and its last 8 codes, a K
// permutation both operands share); the sums are multiplied by
// 2^(e_x + e_w) (NaN for a non-finite operand) before the bias.  Either way a
// staged row piece is 64 bytes, so the blocks, the swizzle and the stage plan
// are the same.  wp: the copy, wnet bytes per network, wrow bytes per row.
template <int NT, int MW, int DT>
__global__ __launch_bounds__(256, MW * NT <= 16 ? 2 : 1) void eval_lpw_kernel(
    const float* __restrict__ genomes, NetDesc nd, const char* __restrict__ wp, int64_t wnet,
    int64_t wrow, const char* __restrict__ xq, int nch, int bpad,
    const uint32_t* __restrict__ x_amax, const uint32_t* __restrict__ w_bound,
    const uint32_t* __restrict__ tail, const int32_t* __restrict__ y, int b,
    float2* __restrict__ partial, int n_wt, int n_pt, int pop) {
  constexpr int S = lpw_stages(NT, MW);
  constexpr int RB = 64;                // bytes per staged row (32 bfloat16)
  constexpr int MT = 64 * MW;           // rows per workgroup
  constexpr int NR = NT * 16;           // staged weight rows
  constexpr int STG = (NR + MT) * RB;   // bytes per stage
  constexpr int NB = NT + MT / 16;      // 1 KiB blocks per stage
  constexpr int Q = (NB + 3) / 4;       // block copies per wave per stage
  static_assert(Q >= 2, "duplicate copies need a previous block");
  __shared__ __attribute__((aligned(16))) char st0[STG];
  __shared__ __attribute__((aligned(16))) char st1[lpw_stage1_bytes(NT, MW)];
  __shared__ __attribute__((aligned(16))) char st2[S >= 3 ? STG : 16];
  __shared__ __attribute__((aligned(16))) char st3[S >= 4 ? STG : 16];
  // stage by a compile-time index, so that every LDS access names one array
  auto stage_ptr = [&](auto sc) -> char* {
    constexpr int st = decltype(sc)::value;
    if constexpr (st == 0) return st0;
    else if constexpr (st == 1) return st1;
    else if constexpr (st == 2) return st2;
    else return st3;
  };

  const int Lw = xcd_logical(blockIdx.x, n_wt * pop);
  const int j = Lw / n_wt;
  const int wt = Lw - j * n_wt;
  const int m0 = wt * MT;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  // this lane's 16 bytes of a block: row r = lane / 4, physical slot lane % 4,
  // which holds logical slot (lane % 4) ^ ((r >> 1) & 3)
  const int r = lane >> 2;
  const int slot = ((lane & 3) ^ ((r >> 1) & 3)) * 16;
  const char* src[Q];
  int64_t cstride[Q];
  int dst[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int i = q * 4 + wave;
    if (i >= NB) i -= 4;
    if (i < NT) {
      src[q] = wp + (int64_t)j * wnet + (16 * i + r) * wrow + slot;
      cstride[q] = RB;
      dst[q] = i * 1024;
    } else {
      src[q] = xq + (int64_t)(m0 + 16 * (i - NT) + r) * RB + slot;
      cstride[q] = (int64_t)bpad * RB;
      dst[q] = NR * RB + (i - NT) * 1024;
    }
  }
  auto issue = [&](int ch, auto sc) {
    const int64_t c = ch < nch ? ch : nch - 1;
    char* d = stage_ptr(sc);
#pragma unroll
    for (int q = 0; q < Q; ++q)
      copy16_to_lds(src[q] + c * cstride[q], d + dst[q]);
  };

  const int mn = lane & 15;
  const int kq = lane >> 4;

  // What the tail reads from global memory, requested now so that it
  // arrives during the main loop: the labels of this lane's rows and the
  // tail genes (b_1 .. b_L, contiguous from boff[0]), which go to stage 1
  // after the loop.
  int ylab[MW];
#pragma unroll
  for (int mi = 0; mi < MW; ++mi) {
    const int r = m0 + wave * MW * 16 + mi * 16 + mn;
    ylab[mi] = r < b ? y[r] : 0;
  }
  const TailScales ts =
      load_tail_scales(DT == 2 && tail ? tail + (int64_t)j * kTailScales : nullptr, nd.L);
  const int tn = (int)reg_tail_genes(nd);
  constexpr int TQ = kTailGenesCap / 16 / 256;  // float4 per thread
  float4 tv[TQ];
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    const int i = tid + 256 * q;
    tv[q] = 4 * i < tn ? reinterpret_cast<const float4*>(genome + nd.boff[0])[i]
                       : float4{0.f, 0.f, 0.f, 0.f};
  }

  floatx4 acc[MW][NT];
#pragma unroll
  for (int mi = 0; mi < MW; ++mi)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[mi][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  // Fragment offsets within a stage: row m = 16 MW wave + 16 mi + mn of the
  // batch part, row n = 16 t + mn of the weight part, slot kq swizzled by
  // row bits 1..2 (those of mn).  The per-lane parts are hidden from the
  // optimiser: a read at an offset it cannot bound may alias its own
  // stage's copy (whose wait the explicit vmcnt already covers) and nothing
  // else; a read it proves disjoint from every copy gets a wait for all of
  // them.
  int xoff = NR * RB + (wave * MW * 16 + mn) * RB + ((kq ^ ((mn >> 1) & 3)) * 16);
  int woff = mn * RB + ((kq ^ ((mn >> 1) & 3)) * 16);
  asm("" : "+v"(xoff));
  asm("" : "+v"(woff));
  auto compute = [&](auto sc) {
    const char* st = stage_ptr(sc);
    uint4 a[MW], bq[NT];
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
      a[mi] = *reinterpret_cast<const uint4*>(st + xoff + mi * 16 * RB);
#pragma unroll
    for (int t = 0; t < NT; ++t) bq[t] = *reinterpret_cast<const uint4*>(st + woff + t * 16 * RB);
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if constexpr (DT == 1) {
          acc[mi][t] = mfma_bf16(bq[t], a[mi], acc[mi][t]);  // W_1 X^T
        } else {
          acc[mi][t] = mfma_fp8(bq[t].x, bq[t].y, a[mi].x, a[mi].y, acc[mi][t]);
          acc[mi][t] = mfma_fp8(bq[t].z, bq[t].w, a[mi].z, a[mi].w, acc[mi][t]);
        }
      }
  };

  // Stage of chunk ch is ch % S; the loop is unrolled by S so that every
  // stage offset is a constant.  Before the barrier of chunk ch each wave
  // waits for its own copies of chunk ch (later chunks stay in flight) and
  // for its LDS reads of chunk ch - 1, whose stage the copy issued after the
  // barrier overwrites.
  // The main loop runs whole groups of S chunks without a branch inside: at
  // a control-flow join the compiler's own wait analysis forgets which stage
  // a copy in flight targets and drains them all.
  auto step = [&](int ch0, auto sc) {
    constexpr int s = decltype(sc)::value;
    wait_copies_barrier<(S - 2) * Q>();
    issue(ch0 + s + S - 1, std::integral_constant<int, (s + S - 1) % S>{});
    compute(sc);
  };
  issue(0, std::integral_constant<int, 0>{});
  if constexpr (S >= 3) issue(1, std::integral_constant<int, 1>{});
  if constexpr (S >= 4) issue(2, std::integral_constant<int, 2>{});
  int ch0 = 0;
  for (; ch0 + S <= nch; ch0 += S) {
    step(ch0, std::integral_constant<int, 0>{});
    step(ch0, std::integral_constant<int, 1>{});
    if constexpr (S >= 3) step(ch0, std::integral_constant<int, 2>{});
    if constexpr (S >= 4) step(ch0, std::integral_constant<int, 3>{});
  }
  if (ch0 < nch) step(ch0, std::integral_constant<int, 0>{});  // uniform branches
  if constexpr (S >= 3)
    if (ch0 + 1 < nch) step(ch0, std::integral_constant<int, 1>{});
  if constexpr (S >= 4)
    if (ch0 + 2 < nch) step(ch0, std::integral_constant<int, 2>{});
  // every copy has landed and every wave is done with the stages before the
  // epilogue reuses the LDS
  wait_copies_barrier<0>();
#pragma unroll
  for (int q = 0; q < TQ; ++q) reinterpret_cast<float4*>(st1)[tid + 256 * q] = tv[q];
  __syncthreads();
  const float fac = DT == 2 ? fp8_factor(*x_amax, w_bound[j]) : 1.0f;
  reg_tail<NT, MW, DT>(acc, fac, reinterpret_cast<const float*>(st1), nd, m0, wave * MW * 16, b,
                       ylab, reinterpret_cast<float*>(st0), partial + (int64_t)j * n_pt, m0 / 64,
                       ts);
}

// ------------------------------------------------ float32 first layer --
// The same pipeline for the float32 product: 16-float K chunks (64 bytes per
// row, so the blocks, the swizzle and the stage plan are those above) copied
// global -> LDS straight from the genomes' W_1 rows and the row-major batch,
// in place of the register double buffer of the other float32 kernel
// (whose staging loads and LDS stores cost about a tenth of its time at
// b = 512).  Lane (mn, kq) reads the float4 at k = 4 kq .. 4 kq + 3 of its
// row and runs four v_mfma_f32_16x16x4_f32 per tile pair, component e taking
// K-step k = 4 kq + e: the products and their order are exactly those of the
// other kernel, so its results are bitwise equal.  Taken when n0 and n1 are
// multiples of 16 (every copied row is a W_1 row and every chunk is whole);
// batch rows past b are copies of row b - 1, which the register tail leaves
// out of every sum.

// Body of one workgroup: network j, row tile wt (rows 64 MW wt ...).
template <int NT, int MW>
__device__ __forceinline__ void eval_lfw_body(int j, int wt, const float* __restrict__ genomes,
                                              const NetDesc& nd, const float* __restrict__ x,
                                              const int32_t* __restrict__ y, int b,
                                              float2* __restrict__ partial, int n_pt) {
  constexpr int S = lpw_stages(NT, MW);
  constexpr int RB = 64;                // bytes per staged row (16 floats)
  constexpr int MT = 64 * MW;           // rows per workgroup
  constexpr int NR = NT * 16;           // staged weight rows
  constexpr int STG = (NR + MT) * RB;   // bytes per stage
  constexpr int NB = NT + MT / 16;      // 1 KiB blocks per stage
  constexpr int Q = (NB + 3) / 4;       // block copies per wave per stage
  static_assert(Q >= 2, "duplicate copies need a previous block");
  __shared__ __attribute__((aligned(16))) char st0[STG];
  __shared__ __attribute__((aligned(16))) char st1[lpw_stage1_bytes(NT, MW)];
  __shared__ __attribute__((aligned(16))) char st2[S >= 3 ? STG : 16];
  __shared__ __attribute__((aligned(16))) char st3[S >= 4 ? STG : 16];
  auto stage_ptr = [&](auto sc) -> char* {
    constexpr int st = decltype(sc)::value;
    if constexpr (st == 0) return st0;
    else if constexpr (st == 1) return st1;
    else if constexpr (st == 2) return st2;
    else return st3;
  };

  const int m0 = wt * MT;
  const float* __restrict__ genome = genomes + (int64_t)j * nd.stride;
  const int n0 = nd.w[0];
  const int nch = n0 >> 4;

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int r = lane >> 2;
  const int slot = ((lane & 3) ^ ((r >> 1) & 3)) * 16;
  const char* src[Q];
  int dst[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int i = q * 4 + wave;
    if (i >= NB) i -= 4;
    if (i < NT) {
      src[q] = reinterpret_cast<const char*>(genome + nd.woff[0] + (int64_t)(16 * i + r) * n0) +
               slot;
      dst[q] = i * 1024;
    } else {
      int m = m0 + 16 * (i - NT) + r;
      m = m < b ? m : b - 1;
      src[q] = reinterpret_cast<const char*>(x + (int64_t)m * n0) + slot;
      dst[q] = NR * RB + (i - NT) * 1024;
    }
  }
  auto issue = [&](int ch, auto sc) {
    const int64_t c = ch < nch ? ch : nch - 1;
    char* d = stage_ptr(sc);
#pragma unroll
    for (int q = 0; q < Q; ++q) copy16_to_lds(src[q] + c * RB, d + dst[q]);
  };

  const int mn = lane & 15;
  const int kq = lane >> 4;
  int ylab[MW];
#pragma unroll
  for (int mi = 0; mi < MW; ++mi) {
    const int rr = m0 + wave * MW * 16 + mi * 16 + mn;
    ylab[mi] = rr < b ? y[rr] : 0;
  }
  const int tn = (int)reg_tail_genes(nd);
  constexpr int TQ = kTailGenesCap / 16 / 256;
  float4 tv[TQ];
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    const int i = tid + 256 * q;
    tv[q] = 4 * i < tn ? reinterpret_cast<const float4*>(genome + nd.boff[0])[i]
                       : float4{0.f, 0.f, 0.f, 0.f};
  }

  floatx4 acc[MW][NT];
#pragma unroll
  for (int mi = 0; mi < MW; ++mi)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[mi][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  int xoff = NR * RB + (wave * MW * 16 + mn) * RB + ((kq ^ ((mn >> 1) & 3)) * 16);
  int woff = mn * RB + ((kq ^ ((mn >> 1) & 3)) * 16);
  asm("" : "+v"(xoff));
  asm("" : "+v"(woff));
  auto compute = [&](auto sc) {
    const char* st = stage_ptr(sc);
    float4 a[MW], bq[NT];
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
      a[mi] = *reinterpret_cast<const float4*>(st + xoff + mi * 16 * RB);
#pragma unroll
    for (int t = 0; t < NT; ++t) bq[t] = *reinterpret_cast<const float4*>(st + woff + t * 16 * RB);
#pragma unroll
    for (int mi = 0; mi < MW; ++mi) mfma_superstep_t<NT>(a[mi], bq, acc[mi]);  // W_1 X^T
  };

  auto step = [&](int ch0, auto sc) {
    constexpr int s = decltype(sc)::value;
    wait_copies_barrier<(S - 2) * Q>();
    issue(ch0 + s + S - 1, std::integral_constant<int, (s + S - 1) % S>{});
    compute(sc);
  };
  issue(0, std::integral_constant<int, 0>{});
  if constexpr (S >= 3) issue(1, std::integral_constant<int, 1>{});
  if constexpr (S >= 4) issue(2, std::integral_constant<int, 2>{});
  int ch0 = 0;
  for (; ch0 + S <= nch; ch0 += S) {
    step(ch0, std::integral_constant<int, 0>{});
    step(ch0, std::integral_constant<int, 1>{});
    if constexpr (S >= 3) step(ch0, std::integral_constant<int, 2>{});
    if constexpr (S >= 4) step(ch0, std::integral_constant<int, 3>{});
  }
  if (ch0 < nch) step(ch0, std::integral_constant<int, 0>{});  // uniform branches
  if constexpr (S >= 3)
    if (ch0 + 1 < nch) step(ch0, std::integral_constant<int, 1>{});
  if constexpr (S >= 4)
    if (ch0 + 2 < nch) step(ch0, std::integral_constant<int, 2>{});
  wait_copies_barrier<0>();
#pragma unroll
  for (int q = 0; q < TQ; ++q) reinterpret_cast<float4*>(st1)[tid + 256 * q] = tv[q];
  __syncthreads();
  reg_tail<NT, MW>(acc, 1.0f, reinterpret_cast<const float*>(st1), nd, m0, wave * MW * 16, b,
                   ylab, reinterpret_cast<float*>(st0), partial + (int64_t)j * n_pt, m0 / 64);
}

template <int NT, int MW>
__global__ __launch_bounds__(256, MW * NT <= 16 ? 2 : 1) void eval_lfw_kernel(
    const float* __restrict__ genomes, NetDesc nd, const float* __restrict__ x,
    const int32_t* __restrict__ y, int b, float2* __restrict__ partial, int n_wt, int n_pt,
    int pop) {
  const int Lw = xcd_logical(blockIdx.x, n_wt * pop);
  const int j = Lw / n_wt;
  eval_lfw_body<NT, MW>(j, Lw - j * n_wt, genomes, nd, x, y, b, partial, n_pt);
}

// The grouped float32 runs whose networks this kernel takes (one launch per
// class of equal column tiles and row tiles per wave).
template <int NT, int MW>
__global__ __launch_bounds__(256, MW * NT <= 16 ? 2 : 1) void runs_eval_lfw_kernel(
    const RunDesc* __restrict__ runs, const BatchState* __restrict__ st,
    const int* __restrict__ off, const int* __restrict__ ids, int n, int total) {
  const int L = xcd_logical(blockIdx.x, total);
  const int i = find_group(off, n, L);
  const RunDesc& d = runs[ids[i]];
  const int local = L - off[i];
  const int j = local / d.n_wt;
  eval_lfw_body<NT, MW>(j, local - j * d.n_wt, d.genomes[st->cur], d.nd, d.xb, d.yb, d.b,
                        d.partial, d.n_pt);
}

// ------------------------------------------------------------- dispatch --

namespace {

constexpr size_t kLdsMaxW = 160 * 1024;

// Networks the register tail takes, with their tail genes from boff[0] (a
// multiple of 4) fitting stage 1.  Returns the row tiles per wave (0: none).
int lpw_mw(const NetDesc& nd, int b) {
  const int nt = (nd.w[1] + 15) / 16;
  if (nt < 1 || nt > 16 || nd.w[0] % 4 != 0 || b <= 16) return 0;
  if (!reg_tail_ok(nd) || nd.boff[0] % 4 != 0 || reg_tail_copy_floats(nd) * 4 > kTailGenesCap)
    return 0;
  int mw = b > 64 ? 2 : 1;
  while (mw > 1 && mw * nt > 32) mw >>= 1;
  for (; mw >= 1; mw >>= 1)
    if ((size_t)lpw_lds_bytes(nt, mw) <= kLdsMaxW) return mw;
  return 0;
}

// The copy operands of one launch: W_1 copy (bytes per network and per row)
// and the chunk-major batch; FP8 also the scale sources.
struct LpwArgs {
  const char* wp;
  int64_t wnet, wrow;
  const char* xq;
  int nch, bpad;
  const uint32_t* x_amax;
  const uint32_t* w_bound;
  const uint32_t* tail;  // FP8: later layers' largest magnitudes, [pop][kTailScales]
};

template <int NT, int MW, int DT>
hipError_t launch_lpw3(const float* genomes, const NetDesc& nd, int pop, const LpwArgs& a,
                       const int32_t* y, int b, float2* partial, hipStream_t s) {
  const int n_wt = (b + 64 * MW - 1) / (64 * MW);
  const int n_pt = (b + 63) / 64;
  hipLaunchKernelGGL((eval_lpw_kernel<NT, MW, DT>), dim3((unsigned)(n_wt * pop)), dim3(256), 0,
                     s, genomes, nd, a.wp, a.wnet, a.wrow, a.xq, a.nch, a.bpad, a.x_amax,
                     a.w_bound, a.tail, y, b, partial, n_wt, n_pt, pop);
  return hipGetLastError();
}

template <int NT, int DT>
hipError_t launch_lpw_nt(const float* genomes, const NetDesc& nd, int pop, const LpwArgs& a,
                         const int32_t* y, int b, float2* partial, hipStream_t s) {
  const int mw = lpw_mw(nd, b);
  if (mw == 2) return launch_lpw3<NT, 2, DT>(genomes, nd, pop, a, y, b, partial, s);
  if (mw == 1) return launch_lpw3<NT, 1, DT>(genomes, nd, pop, a, y, b, partial, s);
  return hipErrorInvalidValue;
}

template <int DT>
hipError_t launch_lpw_any(const float* genomes, const NetDesc& nd, int pop, const LpwArgs& a,
                          const int32_t* y, int b, float2* partial, hipStream_t s) {
  switch ((nd.w[1] + 15) / 16) {
#define LEEA_LPW_CASE(N) \
  case N:                \
    return launch_lpw_nt<N, DT>(genomes, nd, pop, a, y, b, partial, s);
    LEEA_LPW_CASE(1) LEEA_LPW_CASE(2) LEEA_LPW_CASE(3) LEEA_LPW_CASE(4) LEEA_LPW_CASE(5)
    LEEA_LPW_CASE(6) LEEA_LPW_CASE(7) LEEA_LPW_CASE(8) LEEA_LPW_CASE(9) LEEA_LPW_CASE(10)
    LEEA_LPW_CASE(11) LEEA_LPW_CASE(12) LEEA_LPW_CASE(13) LEEA_LPW_CASE(14) LEEA_LPW_CASE(15)
    LEEA_LPW_CASE(16)
#undef LEEA_LPW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

bool eval_lpw_supported(const NetDesc& nd, int b) { return lpw_mw(nd, b) > 0; }

bool eval_lfw_supported(const NetDesc& nd, int b, int mw, const float* x) {
  const int nt = (nd.w[1] + 15) / 16;
  if (nt < 1 || nt > 16 || (mw != 1 && mw != 2) || b <= 16) return false;
  if (nd.w[0] % 16 != 0 || nd.w[1] % 16 != 0 || nd.stride % 4 != 0 || nd.woff[0] % 4 != 0)
    return false;
  if (reinterpret_cast<uintptr_t>(x) % 16 != 0) return false;
  if (!reg_tail_ok(nd) || nd.boff[0] % 4 != 0 || reg_tail_copy_floats(nd) * 4 > kTailGenesCap)
    return false;
  return (size_t)(mw == 2 ? lpw_lds_bytes(nt, 2) : lpw_lds_bytes(nt, 1)) <= kLdsMaxW;
}

namespace {
template <int NT, int MW>
hipError_t launch_lfw3(const float* genomes, const NetDesc& nd, int pop, const float* x,
                       const int32_t* y, int b, float2* partial, hipStream_t s) {
  const int n_wt = (b + 64 * MW - 1) / (64 * MW);
  const int n_pt = (b + 63) / 64;
  hipLaunchKernelGGL((eval_lfw_kernel<NT, MW>), dim3((unsigned)(n_wt * pop)), dim3(256), 0, s,
                     genomes, nd, x, y, b, partial, n_wt, n_pt, pop);
  return hipGetLastError();
}
}  // namespace

namespace {
template <int NT, int MW>
hipError_t launch_runs_lfw3(const RunDesc* runs, const BatchState* st, const Group& g,
                            hipStream_t s) {
  hipLaunchKernelGGL((runs_eval_lfw_kernel<NT, MW>), dim3((unsigned)g.blocks), dim3(256), 0, s,
                     runs, st, g.off, g.ids, g.n, g.blocks);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_runs_lfw(int nt, int mw, const RunDesc* runs, const BatchState* st,
                           const Group& g, hipStream_t s) {
  if (mw != 1 && mw != 2) return hipErrorInvalidValue;
  switch (nt) {
#define LEEA_RLFW_CASE(N)                                                  \
  case N:                                                                  \
    return mw == 2 ? launch_runs_lfw3<N, 2>(runs, st, g, s)                \
                   : launch_runs_lfw3<N, 1>(runs, st, g, s);
    LEEA_RLFW_CASE(1) LEEA_RLFW_CASE(2) LEEA_RLFW_CASE(3) LEEA_RLFW_CASE(4) LEEA_RLFW_CASE(5)
    LEEA_RLFW_CASE(6) LEEA_RLFW_CASE(7) LEEA_RLFW_CASE(8) LEEA_RLFW_CASE(9) LEEA_RLFW_CASE(10)
    LEEA_RLFW_CASE(11) LEEA_RLFW_CASE(12) LEEA_RLFW_CASE(13) LEEA_RLFW_CASE(14)
    LEEA_RLFW_CASE(15) LEEA_RLFW_CASE(16)
#undef LEEA_RLFW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_evaluate_lfw(const float* genomes, const NetDesc& nd, int pop, const float* x,
                               const int32_t* y, int b, int mw, float2* partial, hipStream_t s) {
  if (!eval_lfw_supported(nd, b, mw, x)) return hipErrorInvalidValue;
  switch ((nd.w[1] + 15) / 16) {
#define LEEA_LFW_CASE(N)                                                            \
  case N:                                                                           \
    return mw == 2 ? launch_lfw3<N, 2>(genomes, nd, pop, x, y, b, partial, s)       \
                   : launch_lfw3<N, 1>(genomes, nd, pop, x, y, b, partial, s);
    LEEA_LFW_CASE(1) LEEA_LFW_CASE(2) LEEA_LFW_CASE(3) LEEA_LFW_CASE(4) LEEA_LFW_CASE(5)
    LEEA_LFW_CASE(6) LEEA_LFW_CASE(7) LEEA_LFW_CASE(8) LEEA_LFW_CASE(9) LEEA_LFW_CASE(10)
    LEEA_LFW_CASE(11) LEEA_LFW_CASE(12) LEEA_LFW_CASE(13) LEEA_LFW_CASE(14) LEEA_LFW_CASE(15)
    LEEA_LFW_CASE(16)
#undef LEEA_LFW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

int eval_lpw_ptiles(const NetDesc& nd, int b) { return (b + 63) / 64; }

hipError_t launch_evaluate_lpw(const float* genomes, const NetDesc& nd, int pop,
                               const W1Shadow& wsh, const uint16_t* xq, int kp, int bpad,
                               const int32_t* y, int b, float2* partial, hipStream_t s) {
  if (!wsh.p || bpad % 128 != 0 || bpad < b) return hipErrorInvalidValue;
  const LpwArgs a{reinterpret_cast<const char*>(wsh.p), wsh.net * 2, (int64_t)wsh.kp * 2,
                  reinterpret_cast<const char*>(xq), kp >> 5, bpad, nullptr, nullptr, nullptr};
  return launch_lpw_any<1>(genomes, nd, pop, a, y, b, partial, s);
}

hipError_t launch_evaluate_lpw8(const float* genomes, const NetDesc& nd, int pop,
                                const W1Fp8& w8, const uint8_t* xq, int bpad,
                                const uint32_t* x_amax, const int32_t* y, int b, float2* partial,
                                hipStream_t s) {
  if (!w8.p || bpad % 128 != 0 || bpad < b) return hipErrorInvalidValue;
  const LpwArgs a{reinterpret_cast<const char*>(w8.p), w8.net, (int64_t)w8.kp,
                  reinterpret_cast<const char*>(xq), w8.kp >> 6, bpad, x_amax, w8.bound,
                  w8.tail};
  return launch_lpw_any<2>(genomes, nd, pop, a, y, b, partial, s);
}

}  // namespace leea
