// Rank + selection plan in one single-workgroup kernel (Algorithm 1: sort
// by fitness, elites, parent pairs, mutation parents).
//
// Each slot's fitness becomes a unique 64-bit key: the high word is an
// order-reversing map of the float (larger fitness -> smaller key, -0 -> +0,
// every NaN -> 0xFFFFFFFF), the low word the slot index.  Unique keys make
// the result independent of the sorting algorithm; a bitonic sort over the
// next power of two (padding keys all-ones) then gives the order: in
// registers with lane shuffles up to 1024 keys, in LDS beyond.
#include "internal.hpp"
#include "runs.hpp"
#include "select_common.hpp"

namespace leea {

// Rank + plan of one population by the 1024 threads of a workgroup; keys is
// LDS of n2 (the next power of two >= pop) 64-bit entries.
__device__ void select_body(uint64_t* keys, const float* __restrict__ f_adj, int pop, int n2,
                            int n_elite, int n_cross, int n_trunc, int selection, int tk,
                            const Key& key, uint32_t gen, int4* __restrict__ plan,
                            float* __restrict__ f_inh_next, int32_t* __restrict__ order_out) {
#pragma clang fp contract(off)
  const int tid = threadIdx.x;
  if (n2 <= 1024) {
    // one key per thread: partners less than 64 apart are in the same wave
    // and trade keys by lane shuffles; only the 10 exchange steps over 64 or
    // more (n2 = 1024) go through LDS with barriers.  Element t ends with
    // the smaller key when it is the lower of its pair in an ascending block
    // (t & size == 0) or the upper in a descending one.
    uint64_t a = tid < pop ? rank_key(f_adj[tid], (uint32_t)tid) : ~0ull;
    for (int size = 2; size <= n2; size <<= 1) {
      for (int half = size >> 1; half > 0; half >>= 1) {
        uint64_t b;
        if (half >= 64) {  // uniform
          if (tid < n2) keys[tid] = a;
          __syncthreads();
          b = tid < n2 ? keys[tid ^ half] : a;
          __syncthreads();
        } else {
          const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)a, half);
          const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(a >> 32), half);
          b = ((uint64_t)hi << 32) | lo;
        }
        const bool asc = (tid & size) == 0;
        const bool lower = (tid & half) == 0;
        const uint64_t mn = a < b ? a : b;
        const uint64_t mx = a < b ? b : a;
        a = (lower == asc) ? mn : mx;
      }
    }
    if (tid < n2) keys[tid] = a;
    __syncthreads();
  } else {
    for (int i = tid; i < n2; i += 1024)
      keys[i] = i < pop ? rank_key(f_adj[i], (uint32_t)i) : ~0ull;
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
      for (int half = size >> 1; half > 0; half >>= 1) {
        for (int i = tid; i < (n2 >> 1); i += 1024) {
          const int lo = 2 * i - (i & (half - 1));
          const int hi = lo + half;
          const bool up = (lo & size) == 0;
          const uint64_t a = keys[lo];
          const uint64_t b = keys[hi];
          if ((a > b) == up) {
            keys[lo] = b;
            keys[hi] = a;
          }
        }
        __syncthreads();
      }
    }
  }
  for (int r = tid; r < pop; r += 1024) {
    const int32_t slot = (int32_t)(uint32_t)keys[r];
    if (order_out) order_out[r] = slot;
  }
  // plan: slot j < n_elite copies rank j; then n_cross crossover children;
  // the rest are mutants
  for (int j = tid; j < pop; j += 1024) {
    int op, p1, p2;
    float fi;
    if (j < n_elite) {
      op = kOpElite;
      p1 = p2 = (int)(uint32_t)keys[j];
      fi = f_adj[p1];
    } else if (j < n_elite + n_cross) {
      op = kOpCross;
      const uint32_t r1 = parent_rank(key, gen, (uint32_t)j, 0, selection, tk, n_trunc, pop);
      const uint32_t r2 = parent_rank(key, gen, (uint32_t)j, 1, selection, tk, n_trunc, pop);
      p1 = (int)(uint32_t)keys[r1];
      p2 = (int)(uint32_t)keys[r2];
      const float sum = f_adj[p1] + f_adj[p2];
      fi = sum * 0.5f;
    } else {
      op = kOpMut;
      const uint32_t r1 = parent_rank(key, gen, (uint32_t)j, 0, selection, tk, n_trunc, pop);
      p1 = p2 = (int)(uint32_t)keys[r1];
      fi = f_adj[p1];
    }
    plan[j] = make_int4(op, p1, p2, 0);
    f_inh_next[j] = fi;
  }
}

__global__ __launch_bounds__(1024) void select_kernel(const float* __restrict__ f_adj, int pop,
                                                      int n2, int n_elite, int n_cross,
                                                      int n_trunc, int selection, int tk,
                                                      Key key, uint32_t gen,
                                                      int4* __restrict__ plan,
                                                      float* __restrict__ f_inh_next,
                                                      int32_t* __restrict__ order_out) {
  extern __shared__ uint64_t keys[];
  select_body(keys, f_adj, pop, n2, n_elite, n_cross, n_trunc, selection, tk, key, gen, plan,
              f_inh_next, order_out);
}

hipError_t launch_select(const float* f_adj, int pop, int n_elite, int n_cross, int n_trunc,
                         int selection, int tk, const Key& key, uint32_t gen, int4* plan,
                         float* f_inh_next, int32_t* order, hipStream_t s) {
  int n2 = 1;
  while (n2 < pop) n2 <<= 1;
  if (n2 < 2) n2 = 2;
  const size_t lds = (size_t)n2 * sizeof(uint64_t);
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(1024), lds, s, f_adj, pop, n2, n_elite,
                     n_cross, n_trunc, selection, tk, key, gen, plan, f_inh_next, order);
  return hipGetLastError();
}

// Rank + plan of every run: one workgroup per run; the plan's inherited
// fitness goes to the run's next inherited-fitness buffer.
__global__ __launch_bounds__(1024) void runs_select_kernel(const RunDesc* __restrict__ runs,
                                                           const BatchState* __restrict__ st,
                                                           const int* __restrict__ ids) {
  extern __shared__ uint64_t keys[];
  const RunDesc& d = runs[ids[blockIdx.x]];
  select_body(keys, d.f_adj, d.pop, d.n2, d.n_elite, d.n_cross, d.n_trunc, d.selection, d.tk,
              d.key, st->gen + 1, d.plan, d.f_inh[st->inh ^ 1], nullptr);
}

hipError_t launch_runs_select(const RunDesc* runs, const BatchState* st, const Group& g,
                              hipStream_t s) {
  hipLaunchKernelGGL(runs_select_kernel, dim3((unsigned)g.n), dim3(1024), g.lds, s, runs, st,
                     g.ids);
  return hipGetLastError();
}

}  // namespace leea
