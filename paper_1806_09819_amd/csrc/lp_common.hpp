// Pieces shared by the reduced-precision large-batch kernels: the epilogue
// that turns layer-1 accumulators into the LDS activation tile and runs the
// FP32 tail and fitness, the XCD-aware workgroup order, and the LDS layout
// of the tail.
#pragma once

#include "eval_common.hpp"

namespace leea {

// Epilogue in passes of pass_rows rows (LDS tile at lds): the waves owning those rows write
// fac * acc + bias (ReLU unless it is the output layer) into the LDS tile,
// then the tail layers and the fitness of the pass run.  A wave's 16 MW rows
// lie inside one pass (pass_rows is a multiple of 64), so whether it writes
// is uniform across the wave.
// The tail layers read their weights from tw + (offset - toff): the genome
// (toff = 0) or a copy of its tail in LDS.  kPre: layer 1's bias
// (b1v[t] = b_1[16 t + lane % 16]) and the labels (ylab[p] = y of row
// 64 p + threadIdx.x, passes of 64 rows) were loaded by the caller before
// its main loop, so no global load waits here.
template <int NT, int MW, int DT, bool kPre = false>
__device__ __forceinline__ void lp_epilogue(float* lds, const floatx4 (&acc)[MW][NT], float fac,
                                            int j, int wt, const float* __restrict__ genome,
                                            const float* tw, int64_t toff,
                                            const NetDesc& nd, const int32_t* __restrict__ y,
                                            int b, float2* __restrict__ partial,
                                            const EvalLds& lo, int n_pt, int pass_rows,
                                            int tail_vec, const float (&b1v)[NT],
                                            const int (&ylab)[MW]) {
  constexpr int MT = 64 * MW;
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
  const int passes = MT / pass_rows;
  const int wr0 = wave * MW * 16;  // first row of this wave
  for (int p = 0; p < passes; ++p) {
    const int pr0 = p * pass_rows;
    const int prow = rows - pr0 < pass_rows ? rows - pr0 : pass_rows;
    const int pidx = wt * passes + p;
    if (prow <= 0 || pidx >= n_pt) break;  // uniform across the workgroup
    if (wr0 >= pr0 && wr0 < pr0 + pass_rows) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int n = t * 16 + mn;
        const bool nv = n < n1;
        const float bb = kPre ? b1v[t] : (nv ? b1[n] : 0.0f);
#pragma unroll
        for (int mi = 0; mi < MW; ++mi)
#pragma unroll
          for (int i2 = 0; i2 < 4; ++i2) {
            const int m = wr0 + mi * 16 + 4 * kq + i2 - pr0;
            float v = acc[mi][t][i2];
            if (DT == 2) v = v * fac;
            v = v + bb;
            if (hidden) v = relu_keep_nan(v);
            h1[m * lo.ld1 + n] = nv ? v : 0.0f;
          }
      }
    }
    __syncthreads();
    int yl = 0;
    if (kPre) {
#pragma unroll
      for (int q = 0; q < MW; ++q)
        if (q == p) yl = ylab[q];
    }
    tail_and_fitness<4>(lds, lo, nd, tw, toff, pass_rows / 16, prow, m0 + pr0, kPre ? nullptr : y,
                        tail_vec != 0, partial + (int64_t)j * n_pt + pidx, yl);
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
