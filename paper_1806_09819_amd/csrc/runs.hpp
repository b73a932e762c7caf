// Many independent EA runs driven together: per-run descriptors in device
// memory and the grouped launches that serve every run of a phase with one
// kernel.  The state that changes from one generation to the next (the
// generation counter and which population buffer is current) lives in
// device memory too, so a captured generation replays unchanged.
#pragma once

#include "internal.hpp"

namespace leea {

// Everything a kernel needs to know about one run (device memory, written
// once by the host).
struct RunDesc {
  NetDesc nd;
  float* genomes[2];
  float* f_adj;
  float* f_raw;
  float* acc;
  float* f_inh[2];
  int4* plan;
  float2* partial;
  float* xb;       // drawn batch [b][n0]
  int32_t* yb;     // [b]
  void* xq;        // quantised batch (reduced-precision first layer)
  Key key;
  uint64_t thr;    // mutation threshold
  float sigma, alpha;
  int pop, n_elite, n_cross, n_trunc, selection, tk, crossover;
  int b, dt, kp, side;
  uint32_t mul;    // variation slot multiplier
  int n2;          // selection sort size
  int vgx;         // variation workgroups per slot (4 gene groups each)
  // evaluation shape (chosen on the host, possibly by the autotuner)
  int ekind;       // 0 small-batch, 1 FP32 large-batch, 2 reduced-precision large-batch
  int emw;         // row tiles of 16 per wave (large kernels)
  int n_wt;        // workgroups per network (row tiles)
  int n_pt;        // partial row tiles per network
  int pass_rows;   // rows per tail pass (reduced-precision kernel)
  int tail_vec;
  EvalLds lo;
};

// Shared by every run: all runs advance one generation per step.
struct BatchState {
  uint32_t gen;    // completed generations
  int cur;         // current population buffer
  int has_inh;     // inherited fitness exists (after the first step)
  int inh;         // current inherited-fitness buffer
};

// A grouped launch: workgroup blk of the launch belongs to run ids[i] with
// off[i] <= blk < off[i + 1]; returns i (ids has n entries, off n + 1).
__device__ __forceinline__ int find_group(const int* __restrict__ off, int n, int blk) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= blk)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Host launchers of the grouped kernels (off / ids in device memory).
struct Group {
  const int* off;  // n + 1 block offsets
  const int* ids;  // n run indices
  int n;
  int blocks;      // off[n]
  size_t lds;      // dynamic LDS of the launch (max over its runs)
};

// Float32 large-batch runs on the global -> LDS kernel (every run of the
// group taken by eval_lfw_supported; nt column tiles, mw row tiles per wave).
hipError_t launch_runs_lfw(int nt, int mw, const RunDesc* runs, const BatchState* st,
                           const Group& g, hipStream_t s);
hipError_t launch_runs_draw(const RunDesc* runs, const BatchState* st, const Group& g,
                            const float* x_train, const int32_t* y_train, int64_t n_train,
                            int step, hipStream_t s);
hipError_t launch_runs_select(const RunDesc* runs, const BatchState* st, const Group& g,
                              hipStream_t s);
hipError_t launch_runs_vary(const RunDesc* runs, const BatchState* st, const Group& g,
                            hipStream_t s);
hipError_t launch_runs_quantize(const RunDesc* runs, const Group& g, hipStream_t s);
// one evaluation class: every run of the group shares (kind, NT, MW, dt) and
// rt, whether the large-batch kernels run its tail from registers (1), and
// for float32 also stage by global -> LDS copies (2)
hipError_t launch_runs_eval(int kind, int nt, int mw, int dt, int rt, const RunDesc* runs,
                            const BatchState* st, const Group& g, hipStream_t s);
hipError_t launch_runs_eval_lp(int nt, int mw, int dt, int rt, const RunDesc* runs,
                               const BatchState* st, const Group& g, hipStream_t s);
hipError_t launch_runs_finalize(const RunDesc* runs, const BatchState* st, const Group& g,
                                hipStream_t s);
hipError_t launch_runs_advance(BatchState* st, hipStream_t s);

}  // namespace leea
