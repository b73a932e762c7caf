// Layers 2..L and the fitness of the large-batch kernels, computed from
// registers.
//
// The large-batch kernels compute layer 1 transposed, W_1 X^T, so that the
// accumulator of lane l (kq = l / 16, mn = l % 16) for row tile mi and
// column tile t holds neuron 16 t + 4 kq + i (i = 0..3) of row 16 mi + mn.
// That is the B operand of a 16x16x4 FP32 matrix product W_2 h^T in which
// K-step (t, i) covers neurons 16 t + 4 kq + i of the four lane groups: every
// tail layer runs straight from the previous layer's accumulators and leaves
// its own output in the same layout (section 3.3's per-individual tail, with
// no activation tile in LDS and no barrier between layers).  The fitness
// (Eq. 1, left side: log-softmax of the true class; accuracy = first maximal
// logit is the label) then reduces each row across its four lane groups.
//
// Row sums: per 16-row tile a fixed shuffle tree over the 16 rows, then per
// 64-row group a fixed sum of its four tiles, so the partial sums depend on
// neither the workgroup's rows nor the wave that owns a tile.
//
// Supported: up to three layers, tail widths (w[2..L]) at most 64 and every
// hidden width a multiple of 4; reg_tail_ok() checks this on the host.
#pragma once

#include "eval_common.hpp"

namespace leea {

constexpr int kRegTailMax = 4;  // column tiles of a tail layer (<= 64 outputs)

__host__ __device__ inline bool reg_tail_ok(const NetDesc& nd) {
  if (nd.L < 1 || nd.L > 3) return false;
  for (int l = 1; l < nd.L; ++l)
    if (nd.w[l] % 4 != 0) return false;
  for (int l = 2; l <= nd.L; ++l)
    if (nd.w[l] > 16 * kRegTailMax) return false;
  if (nd.L == 1 && nd.w[1] > 16 * kRegTailMax) return false;
  return true;
}

// Genes of the LDS copy the register tail reads: b_1 .. b_L, contiguous
// from boff[0].
__host__ __device__ inline int64_t reg_tail_genes(const NetDesc& nd) {
  return nd.genes - nd.boff[0];
}

// Floats of the LDS copy: the genes, zeros up to the next multiple of 4
// (the last bias is read in fours), then four more zeros that weight
// fragments past n_in read instead of masking.
__host__ __device__ inline int reg_tail_copy_floats(const NetDesc& nd) {
  return (int)((reg_tail_genes(nd) + 3) & ~3) + 4;
}

// That copy, made by the whole workgroup (256 threads).  Caller
// synchronises afterwards.
__device__ __forceinline__ void copy_tail_genes(const float* __restrict__ genome,
                                                const NetDesc& nd, float* tl) {
  const int tn = (int)reg_tail_genes(nd);
  const float* src = genome + nd.boff[0];
  const int n = reg_tail_copy_floats(nd);
  for (int i = threadIdx.x; i < n; i += 256) tl[i] = i < tn ? src[i] : 0.0f;
}

// One tail layer: out[mi][o] (column tile o < TO) = in * W^T + b with `in` =
// the first TI column tiles of the transposed layout, ReLU if hidden; tiles
// TO .. kRegTailMax - 1 of out are zero, and so are columns past n_out.  W
// (n_out x n_in, row-major) and b are in LDS; z4 points at four zeros there.
// Fragments of rows past n_out read row 0 (those columns are zeroed
// afterwards); fragments past n_in read z4 (zero times the zero activations
// there, where a clamped weight could be infinite or NaN).  Every K-step
// loads its TO weight fragments first and then runs its 4 TO MW products
// across all the accumulators, so consecutive products never wait on each
// other; each accumulator still sums its K-steps in order (t, then i).
// DT != 0: weights quantised as they are loaded (quantize<DT>, scale
// exponent neg_e); DT = 2: the sums times wfac before the bias.
template <int MW, int TI, int TO, int TIN, int DT>
__device__ __forceinline__ void reg_layer_t(const floatx4 (&in)[MW][TIN],
                                            floatx4 (&out)[MW][kRegTailMax], const float* W,
                                            const float* bias, const float* z4, int n_in,
                                            int n_out, bool relu, int neg_e, float wfac) {
  static_assert(TI <= TIN && TO <= kRegTailMax, "tile counts");
  const int lane = threadIdx.x & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const float* wr[TO];
#pragma unroll
  for (int o = 0; o < TO; ++o) {
    const int n = 16 * o + mn;
    wr[o] = W + (n < n_out ? n : 0) * n_in;
  }
#pragma unroll
  for (int o = 0; o < kRegTailMax; ++o)
#pragma unroll
    for (int mi = 0; mi < MW; ++mi) out[mi][o] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < TI; ++t) {
    const int k = 16 * t + 4 * kq;
    float4 w[TO];
#pragma unroll
    for (int o = 0; o < TO; ++o) {
      w[o] = *reinterpret_cast<const float4*>(k < n_in ? wr[o] + k : z4);
      if constexpr (DT != 0) {
        w[o].x = quantize<DT>(w[o].x, neg_e);
        w[o].y = quantize<DT>(w[o].y, neg_e);
        w[o].z = quantize<DT>(w[o].z, neg_e);
        w[o].w = quantize<DT>(w[o].w, neg_e);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int o = 0; o < TO; ++o)
#pragma unroll
        for (int mi = 0; mi < MW; ++mi) {
          const float wv = i == 0 ? w[o].x : i == 1 ? w[o].y : i == 2 ? w[o].z : w[o].w;
          out[mi][o] = mfma(wv, in[mi][t][i], out[mi][o]);
        }
  }
#pragma unroll
  for (int o = 0; o < TO; ++o) {
    const int c = 16 * o + 4 * kq;
    const float4 bv = *reinterpret_cast<const float4*>(bias + (c < n_out ? c : 0));
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = out[mi][o][i];
        if constexpr (DT == 2) v = v * wfac;
        v = v + (i == 0 ? bv.x : i == 1 ? bv.y : i == 2 ? bv.z : bv.w);
        if (relu) v = relu_keep_nan(v);
        out[mi][o][i] = c + i < n_out ? v : 0.0f;
      }
  }
}

// reg_layer_t with TO = the column tiles of n_out (1 .. kRegTailMax); for
// DT = 2 the layer's FP8 scale comes from its weights' largest magnitude,
// *tam when given, else reduced here by the workgroup (every thread of the
// workgroup calls this).
template <int MW, int TI, int TIN, int DT>
__device__ __forceinline__ void reg_layer(const floatx4 (&in)[MW][TIN],
                                          floatx4 (&out)[MW][kRegTailMax], const float* W,
                                          const float* bias, const float* z4, int n_in, int n_out,
                                          bool relu, const uint32_t* tam) {
  int neg_e = 0;
  float wfac = 1.0f;
  if constexpr (DT == 2) tail_fp8_scale(tam ? *tam : block_amax(W, n_in * n_out), neg_e, wfac);
  switch ((n_out + 15) >> 4) {
    case 1:
      reg_layer_t<MW, TI, 1, TIN, DT>(in, out, W, bias, z4, n_in, n_out, relu, neg_e, wfac);
      break;
    case 2:
      reg_layer_t<MW, TI, 2, TIN, DT>(in, out, W, bias, z4, n_in, n_out, relu, neg_e, wfac);
      break;
    case 3:
      reg_layer_t<MW, TI, 3, TIN, DT>(in, out, W, bias, z4, n_in, n_out, relu, neg_e, wfac);
      break;
    default:
      reg_layer_t<MW, TI, 4, TIN, DT>(in, out, W, bias, z4, n_in, n_out, relu, neg_e, wfac);
      break;
  }
}

// Log-likelihood and correctness of row 16 mi + mn from its logits
// (transposed layout, TC column tiles of which tc_used are live, d classes);
// every lane of the row's four lane groups gets the same result.
template <int MW, int TC>
__device__ __forceinline__ void reg_fitness(const floatx4 (&z)[MW][TC], int tc_used, int d,
                                            const int (&ylab)[MW], float (&ll)[MW],
                                            int (&cor)[MW]) {
  const int lane = threadIdx.x & 63;
  const int kq = lane >> 4;
#pragma unroll
  for (int mi = 0; mi < MW; ++mi) {
    // first maximal logit: each lane scans its classes in increasing order
    // (a later class wins only if strictly larger), then the lane groups
    // combine (value, class) pairs: larger value wins, equal values go to
    // the lower class; kNone marks a lane group without a class
    constexpr int kNone = 0x7fffffff;
    float mx = -__builtin_inff();
    int best = kNone;
    float zy = 0.0f;
    const int yy = ylab[mi];
#pragma unroll
    for (int c = 0; c < TC; ++c) {
      if (c < tc_used) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * c + 4 * kq + i;
          const float v = z[mi][c][i];
          if (k < d) {
            if (best == kNone || v > mx) {
              mx = v;
              best = k;
            }
            if (k == yy) zy = v;
          }
        }
      }
    }
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      const float om = __shfl_xor(mx, off);
      const int ob = __shfl_xor(best, off);
      if (ob != kNone && (best == kNone || om > mx || (om == mx && ob < best))) {
        mx = om;
        best = ob;
      }
      zy += __shfl_xor(zy, off);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < TC; ++c) {
      if (c < tc_used) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = 16 * c + 4 * kq + i;
          if (k < d) s += expf(z[mi][c][i] - mx);
        }
      }
    }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    ll[mi] = (yy >= 0 && yy < d) ? (zy - mx) - logf(s) : __builtin_nanf("");
    cor[mi] = best == yy ? 1 : 0;
  }
}

// Whole tail from the layer-1 accumulators z (transposed layout, NT tiles):
// bias and activation, layers 2..L, fitness, and the partial sums of this
// workgroup's 64-row groups.  fac scales the accumulators first (FP8).
// tl: the copy_tail_genes copy in LDS (tl[0] = b_1[0]); red: LDS scratch of
// 2 * 4 * MW floats; rows of this wave: r0 + 16 mi + mn (r0 relative to the
// workgroup's first row m0); labels ylab[mi] of those rows (any value for
// rows at or past b).  partial: the network's partials, one per 64-row group,
// g0 = index of the workgroup's first group.  DT: arithmetic of the weights
// of layers 2..L (as in tail_and_fitness); ts: their largest magnitudes, if
// given.
template <int NT, int MW, int DT = 0>
__device__ __forceinline__ void reg_tail(floatx4 (&z)[MW][NT], float fac, const float* tl,
                                         const NetDesc& nd, int m0, int r0, int b,
                                         const int (&ylab)[MW], float* red,
                                         float2* __restrict__ partial, int g0,
                                         const TailScales& ts = TailScales{{}, 0}) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const int n1 = nd.w[1];
  const bool hidden = nd.L > 1;
  // layer 1: fac * z + b_1, ReLU unless it is the output layer
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = 16 * t + 4 * kq;
    float4 bv = zero4();
    if (hidden) {
      bv = *reinterpret_cast<const float4*>(tl + (c < n1 ? c : 0));
    } else {
      bv.x = c < n1 ? tl[c] : 0.0f;
      bv.y = c + 1 < n1 ? tl[c + 1] : 0.0f;
      bv.z = c + 2 < n1 ? tl[c + 2] : 0.0f;
      bv.w = c + 3 < n1 ? tl[c + 3] : 0.0f;
    }
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = z[mi][t][i];
        if (fac != 1.0f) v = v * fac;
        v = v + (i == 0 ? bv.x : i == 1 ? bv.y : i == 2 ? bv.z : bv.w);
        if (hidden) v = relu_keep_nan(v);
        z[mi][t][i] = c + i < n1 ? v : 0.0f;
      }
  }
  float ll[MW];
  int cor[MW];
  const int64_t base = nd.boff[0];
  if (nd.L == 1) {
    reg_fitness<MW, NT>(z, NT, n1, ylab, ll, cor);
  } else {
    const float* z4 = tl + reg_tail_copy_floats(nd) - 4;
    floatx4 h2[MW][kRegTailMax];
    reg_layer<MW, NT, NT, DT>(z, h2, tl + (nd.woff[1] - base), tl + (nd.boff[1] - base), z4, n1,
                              nd.w[2], nd.L > 2, ts.given ? &ts.amax[1] : nullptr);
    const int t2 = (nd.w[2] + 15) >> 4;
    if (nd.L == 2) {
      reg_fitness<MW, kRegTailMax>(h2, t2, nd.w[2], ylab, ll, cor);
    } else {
      floatx4 h3[MW][kRegTailMax];
      const float* W3 = tl + (nd.woff[2] - base);
      const float* b3 = tl + (nd.boff[2] - base);
      switch (t2) {
        case 1:
          reg_layer<MW, 1, kRegTailMax, DT>(h2, h3, W3, b3, z4, nd.w[2], nd.w[3], false,
                                             ts.given ? &ts.amax[2] : nullptr);
          break;
        case 2:
          reg_layer<MW, 2, kRegTailMax, DT>(h2, h3, W3, b3, z4, nd.w[2], nd.w[3], false,
                                             ts.given ? &ts.amax[2] : nullptr);
          break;
        case 3:
          reg_layer<MW, 3, kRegTailMax, DT>(h2, h3, W3, b3, z4, nd.w[2], nd.w[3], false,
                                             ts.given ? &ts.amax[2] : nullptr);
          break;
        default:
          reg_layer<MW, 4, kRegTailMax, DT>(h2, h3, W3, b3, z4, nd.w[2], nd.w[3], false,
                                             ts.given ? &ts.amax[2] : nullptr);
          break;
      }
      reg_fitness<MW, kRegTailMax>(h3, (nd.w[3] + 15) >> 4, nd.w[3], ylab, ll, cor);
    }
  }
  // per 16-row tile: rows past b count zero; a fixed tree over the 16 rows
  const int wave = tid >> 6;
#pragma unroll
  for (int mi = 0; mi < MW; ++mi) {
    const bool rv = m0 + r0 + 16 * mi + mn < b;
    float s = rv ? ll[mi] : 0.0f;
    float c = rv ? (float)cor[mi] : 0.0f;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      s += __shfl_xor(s, off);
      c += __shfl_xor(c, off);
    }
    if (lane == 0) {
      const int tile = wave * MW + mi;  // tile index within the workgroup
      red[2 * tile] = s;
      red[2 * tile + 1] = c;
    }
  }
  __syncthreads();
  // per 64-row group: ((t0 + t1) + (t2 + t3)), groups wholly past b skipped
  constexpr int G = MW;  // 64-row groups per workgroup (4 MW tiles)
  if (tid < G && m0 + 64 * tid < b) {
    const float* r = red + 8 * tid;
    const float s = (r[0] + r[2]) + (r[4] + r[6]);
    const float c = (r[1] + r[3]) + (r[5] + r[7]);
    partial[g0 + tid] = make_float2(s, c);
  }
}

}  // namespace leea
