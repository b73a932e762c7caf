// Pieces shared by the large-batch kernels: the LDS-tile epilogue for
// networks the register tail does not take, the XCD-aware workgroup order,
// and the LDS layout of that epilogue's tail.
#pragma once

#include "eval_common.hpp"
#include "reg_tail.hpp"

namespace leea {

// Epilogue of the large-batch kernels for networks the register tail does
// not take (more than three layers, wide or odd-width tail layers): passes
// of 64 rows over an LDS activation tile.  acc holds layer 1 transposed
// (W_1 X^T: acc[mi][t][i] = neuron 16 t + 4 kq + i of row 16 mi + mn of the
// wave's rows).  The waves owning a pass's rows write fac * acc + b_1 (ReLU
// unless it is the output layer) into the tile, then the tail layers and the
// fitness of the pass run; each pass writes partial[j * n_pt + m0 / 64 + p].
// The tail layers read their weights from tw + (offset - toff) (the genome:
// toff = 0); DT: arithmetic of their weights (tail_and_fitness).
template <int NT, int MW, int DT = 0>
__device__ __forceinline__ void lds_epilogue(float* lds, const floatx4 (&acc)[MW][NT], float fac,
                                             int j, int wt, const float* __restrict__ genome,
                                             const NetDesc& nd, const int32_t* __restrict__ y,
                                             int b, float2* __restrict__ partial,
                                             const EvalLds& lo, int n_pt, int tail_vec) {
  constexpr int MT = 64 * MW;
  constexpr int PR = 64;  // rows per pass
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int mn = lane & 15;
  const int kq = lane >> 4;
  const int m0 = wt * MT;
  const int rows = b - m0 < MT ? b - m0 : MT;
  const int n1 = nd.w[1];
  const float* __restrict__ b1 = genome + nd.boff[0];
  const bool hidden = nd.L > 1;
  float* h1 = lds + lo.h1;
  const int wr0 = wave * MW * 16;  // first row of this wave, inside one pass
  for (int p = 0; p < MW; ++p) {
    const int pr0 = p * PR;
    const int prow = rows - pr0 < PR ? rows - pr0 : PR;
    if (prow <= 0) break;  // uniform across the workgroup
    if (wr0 >= pr0 && wr0 < pr0 + PR) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int c = t * 16 + 4 * kq;
        float bb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) bb[i] = c + i < n1 ? b1[c + i] : 0.0f;
#pragma unroll
        for (int mi = 0; mi < MW; ++mi) {
          float v[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float u = acc[mi][t][i];
            if (fac != 1.0f) u = u * fac;
            u = u + bb[i];
            if (hidden) u = relu_keep_nan(u);
            v[i] = c + i < n1 ? u : 0.0f;
          }
          const int m = wr0 + mi * 16 + mn - pr0;
          *reinterpret_cast<float4*>(h1 + m * lo.ld1 + c) = make_float4(v[0], v[1], v[2], v[3]);
        }
      }
    }
    __syncthreads();
    tail_and_fitness<4, DT>(lds, lo, nd, genome, 0, PR / 16, prow, m0 + pr0, y, tail_vec != 0,
                            partial + (int64_t)j * n_pt + m0 / 64 + p);
    __syncthreads();
  }
}

// XCD-aware order (hardware workgroup i runs on XCD i % 8): consecutive
// logical ids go to the same XCD, so one network's row tiles share its L2.
__device__ __forceinline__ int xcd_logical(int i, int total) {
  const int q = total >> 3;
  const int r8 = total & 7;
  const int xcd = i & 7;
  const int kk = i >> 3;
  return xcd < r8 ? xcd * (q + 1) + kk : r8 * (q + 1) + (xcd - r8) * q + kk;
}

__host__ inline int round16i(int v) { return (v + 15) & ~15; }

__host__ inline EvalLds lp_tail_layout(const NetDesc& nd, int rows) {
  EvalLds lo;
  lo.ld1 = round16i(nd.w[1]) + 4;
  int w = 4;
  for (int l = 2; l <= nd.L; ++l) w = nd.w[l] > w ? nd.w[l] : w;
  lo.ldt = round16i(w) + 4;
  const int ldmax = lo.ld1 > lo.ldt ? lo.ld1 : lo.ldt;
  lo.h1 = 0;
  lo.ta = rows * ldmax;
  lo.ll = lo.ta + rows * lo.ldt;
  lo.cor = lo.ll + rows;
  lo.total = lo.cor + rows;
  return lo;
}

}  // namespace leea
