// Host-side launchers of the LEEA kernels (one translation unit per kernel
// family); used only by the C-ABI implementation in api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace leea {

struct Glorot {
  float a[kMaxLayers];
};

// LDS carve-up of the evaluation kernels (offsets and strides in floats).
struct EvalLds {
  int h1;     // layer-1 activations [rows][ld1]; later reused as a tail buffer
  int ld1;
  int ta;     // tail activations [rows][ldt]
  int ldt;
  int ll;     // [rows] per-sample log-likelihood
  int cor;    // [rows] per-sample correctness (int)
  int total;  // floats of dynamic LDS
};

// Launch shape of the evaluation of one network population on b rows:
// kind 0 small-batch kernel (b <= 16), 1 FP32 large-batch, 2 reduced-precision
// large-batch, 3 FP32 row-streaming (b <= 4), 4 FP32 1 KiB-row (b <= 8);
// mw row tiles of 16 per wave;
// n_wt workgroups per network; n_pt partial sums per network.
struct EvalShape {
  int kind, mw, n_wt, n_pt, pass_rows, tail_vec;
  size_t lds;
  EvalLds lo;
};
// kind < 0 / mw <= 0: the default choice.  Returns false if the requested
// shape does not exist for these widths and b.
bool eval_shape_f32(const NetDesc& nd, int b, int kind, int mw, EvalShape* out);
bool eval_shape_lp(const NetDesc& nd, int b, int dt, int kind, int mw, EvalShape* out);

// bfloat16 copy of every network's W_1 read by the large-batch bfloat16
// kernel, row-major with padding: element (n, k) of network j is
// p[j * net + n * kp + k], with the rows padded to nrp = n1 rounded up to 16
// and K to kp = n0 rounded up to 32 (padding zero).  p == nullptr: none.
struct W1Shadow {
  uint16_t* p;
  int64_t net;  // elements per network = nrp * kp
  int n0, nrp, kp;
  float rcp_n0;  // 1 / n0 (row of a W_1 gene index below 2^24: one fix-up step)
};

// FP8 (OCP E4M3) copy of every network's W_1 with its per-network
// power-of-two scale: element (n, k) of network j is p[j * net + n * kp + k],
// the E4M3 code of W_1[n][k] * 2^-e_j, rows padded to nrp = n1 rounded up to
// 16 and K to kp = n0 rounded up to 64 (padding zero).  e_j is the smallest
// integer with B_j <= 448 * 2^e_j for the bound B_j held as magnitude bits in
// bound[j]: the network's largest |W_1| after initialisation or a restore;
// for a child, the bound its parents give (elite: the parent's largest
// magnitude; crossover: the larger parent's; mutant: fl(fl(a (1 + 2^-20)) +
// fl(6 sigma))), which the variation kernel knows before it writes the
// child.  amax_par: the parents' exact largest magnitudes (read by the
// variation kernel).  p == nullptr: no copy.
struct W1Fp8 {
  uint8_t* p;
  int64_t net;
  int n0, nrp, kp;
  float rcp_n0;
  const uint32_t* amax_par;
  uint32_t* bound;
  const uint32_t* tail;  // largest |W_l| of the later layers, [pop][kTailScales] (evaluation)
};

// init.hip / vary.hip / batch.hip
hipError_t launch_init(float* genomes, const NetDesc& nd, const Glorot& ga, int pop,
                       const Key& key, hipStream_t s);
hipError_t launch_vary(const float* cur, float* nxt, const int4* plan, const NetDesc& nd,
                       int pop, int crossover, float sigma, uint64_t mut_threshold,
                       const Key& key, uint32_t gen, const float* sig_cur, float* sig_next,
                       float tau, uint32_t* amax, const W1Shadow& wsh, const W1Fp8& w8,
                       hipStream_t s);
hipError_t launch_draw_batch(const float* x_train, const int32_t* y_train, int64_t n_train,
                             int n_in, int side, int b, float* x_out, int32_t* y_out,
                             const Key& key, uint32_t gen, hipStream_t s);
hipError_t launch_pool2x2(const float* x, int64_t n, int side, float* out, hipStream_t s);
hipError_t launch_fill(float* p, int n, float v, hipStream_t s);
uint32_t slot_multiplier(int pop);

// fused.hip: variation + small-batch evaluation in one kernel
bool fused_supported(const NetDesc& nd, int b);
hipError_t launch_vary_eval(const float* cur, float* nxt, const int4* plan, const NetDesc& nd,
                            int pop, int crossover, float sigma, uint64_t thr, const Key& key,
                            uint32_t gen, const float* sig_cur, float* sig_next, float tau,
                            const float* x, const int32_t* y, int b, float2* partial,
                            hipStream_t s);

// select.hip
hipError_t launch_select(const float* f_adj, int pop, int n_elite, int n_cross, int n_trunc,
                         int selection, int tk, const Key& key, uint32_t gen, int4* plan,
                         float* f_inh_next, int32_t* order, hipStream_t s);

// evaluate.hip
int eval_mtiles(const NetDesc& nd, int b);
// Whether the large-batch kernels run this network's tail from registers.
bool large_reg_tail(const NetDesc& nd);
// Whether float32 evaluation of b rows takes the row-streaming kernel (b <= 4).
bool eval_stream_supported(const NetDesc& nd, int b);
// The 1 KiB-row float32 kernel takes this batch (and the row-streaming one does not).
bool eval_rows_supported(const NetDesc& nd, int b);
// What finalize_kernel writes for one network (fitness = sum / b, accuracy,
// inheritance), for evaluation kernels that hold a network's whole batch in
// one workgroup and finish it themselves; on = 0: they do not.
struct FinArgs {
  const float* f_inh;
  float* f_adj;
  float* f_raw;
  float* acc;
  float* f_adj_out;
  float* f_raw_out;
  float* acc_out;
  float alpha;
  int use_inh;
  int on;
};
// With fin given, the kernels for b <= 16 also do the finalisation (the
// partials are written either way); *finalized tells whether they did.
hipError_t launch_evaluate(const float* genomes, const NetDesc& nd, int pop, const float* x,
                           const int32_t* y, int b, float2* partial, hipStream_t s,
                           const FinArgs* fin = nullptr, bool* finalized = nullptr);
hipError_t launch_finalize(const float2* partial, int pop, int n_mt, int b, const float* f_inh,
                           int use_inh, float alpha, float* f_adj, float* f_raw, float* acc,
                           float* f_adj_out, float* f_raw_out, float* acc_out, hipStream_t s);

// evaluate.hip / evaluate_lp.hip / quant.hip: reduced-precision first layer
// (dt 1 = bfloat16, 2 = FP8 E4M3 with power-of-two scales)
hipError_t launch_evaluate_small_lp(int dt, const float* genomes, const NetDesc& nd, int pop,
                                    const float* xq, const int32_t* y, int b, float2* partial,
                                    const uint32_t* w_amax, const uint32_t* x_amax,
                                    hipStream_t s);
// bfloat16 first layer for b <= 16 on the bfloat16 matrix cores, from the
// W_1 copy (wsh.p != nullptr) or rounding the float32 genome on the way; x is
// the float32 batch; finishes each network itself when fin.on.
hipError_t launch_evaluate_small_bf16(const float* genomes, const NetDesc& nd, int pop,
                                      const W1Shadow& wsh, const float* x, const int32_t* y,
                                      int b, float2* partial, hipStream_t s, const FinArgs& fin);
bool eval_lp_supported(const NetDesc& nd, int b, int dt);
int eval_lp_ptiles(const NetDesc& nd, int b, int dt);
hipError_t launch_evaluate_lp(int dt, const float* genomes, const NetDesc& nd, int pop,
                              const void* xq, int kp, const uint32_t* w_amax,
                              const uint32_t* x_amax, const int32_t* y, int b, float2* partial,
                              hipStream_t s);
// The FP8 scales of one evaluation in one launch: *x_amax over the batch
// x[0..n) and tail[j * kTailScales + l] = the largest magnitude bits of
// network j's W_l for every later layer l = 1 .. L - 1 (0-based).
constexpr int kTailScales = kMaxLayers;
hipError_t launch_fp8_scales(const float* x, int64_t n, uint32_t* x_amax, const float* genomes,
                             const NetDesc& nd, int pop, uint32_t* tail, hipStream_t s);
hipError_t launch_amax_w1(const float* genomes, const NetDesc& nd, int pop, uint32_t* amax,
                          hipStream_t s);
hipError_t launch_quantize_x(int dt, bool packed, const float* x, int b, int n0, int kp,
                             const uint32_t* x_amax, void* out, hipStream_t s);
// The large-batch bfloat16 kernel on the W_1 copy: availability, partial row
// tiles, the batch quantised chunk-major (xq[((k >> 5) * bpad + m) * 32 +
// (k & 31)], rows b .. bpad - 1 zero, bpad = b rounded up to 128), the copy
// rebuilt from the genomes, and the launch.
bool eval_lpw_supported(const NetDesc& nd, int b);
int eval_lpw_ptiles(const NetDesc& nd, int b);
hipError_t launch_quantize_x_chunks(const float* x, int b, int n0, int kp, int bpad,
                                    uint16_t* xq, hipStream_t s);
hipError_t launch_shadow_w1(const float* genomes, const NetDesc& nd, int pop,
                            const W1Shadow& wsh, hipStream_t s);
// The FP8 copy rebuilt from the genomes with the scales of w8.bound.
hipError_t launch_fp8_copy(const float* genomes, const NetDesc& nd, int pop, const W1Fp8& w8,
                           hipStream_t s);
// FP8 first layer for b <= 16 on the FP8 matrix cores from the FP8 copy; the
// batch x (float32) is scaled by 2^-e_x (e_x from *x_amax) and rounded on the
// way; finishes each network itself when fin.on.
hipError_t launch_evaluate_small_fp8(const float* genomes, const NetDesc& nd, int pop,
                                     const W1Fp8& w8, const float* x, const uint32_t* x_amax,
                                     const int32_t* y, int b, float2* partial, hipStream_t s,
                                     const FinArgs& fin);
hipError_t launch_evaluate_lpw(const float* genomes, const NetDesc& nd, int pop,
                               const W1Shadow& wsh, const uint16_t* xq, int kp, int bpad,
                               const int32_t* y, int b, float2* partial, hipStream_t s);
// The same pipeline with an FP8 first layer from the FP8 copy (same shapes as
// eval_lpw_supported): the batch chunk-major in E4M3 codes
// (xq[((k >> 6) * bpad + m) * 64 + (k & 63)], scaled by 2^-e_x, rows b ..
// bpad - 1 zero) from launch_quantize_x_chunks8.
hipError_t launch_quantize_x_chunks8(const float* x, int b, int n0, int kp8, int bpad,
                                     const uint32_t* x_amax, uint8_t* xq, hipStream_t s);
hipError_t launch_evaluate_lpw8(const float* genomes, const NetDesc& nd, int pop,
                                const W1Fp8& w8, const uint8_t* xq, int bpad,
                                const uint32_t* x_amax, const int32_t* y, int b, float2* partial,
                                hipStream_t s);
// The float32 large-batch kernel with LDS staging by global -> LDS copies
// (bitwise equal to the register-staged one): whether it takes a network,
// batch size, row tiles per wave (1 or 2) and batch pointer, and the launch
// (same partials as launch_evaluate).
bool eval_lfw_supported(const NetDesc& nd, int b, int mw, const float* x);
hipError_t launch_evaluate_lfw(const float* genomes, const NetDesc& nd, int pop, const float* x,
                               const int32_t* y, int b, int mw, float2* partial, hipStream_t s);

// genetic.hip / surrogate.hip: the fitness surrogate
hipError_t launch_vary_cand(const float* cur, float* cand, const int4* plan, const NetDesc& nd,
                            int n, int crossover, float sigma, uint64_t thr, const Key& key,
                            uint32_t gen, uint32_t slot_off, float* nu, hipStream_t s);
hipError_t launch_proj_bits(uint32_t* bits, int nchunks, const Key& key, hipStream_t s);
hipError_t launch_mlp_init(float* prm, const Key& key, float a1, float a2, hipStream_t s);
hipError_t launch_cand_plan(const int32_t* order, const float* f_adj, int M, int kc, int pop,
                            int n_trunc, int selection, int tk, const Key& key, uint32_t gen,
                            int4* cplan, float* cf_inh, hipStream_t s);
hipError_t launch_proj(const float* cand, int64_t stride, int M, const uint32_t* bits,
                       int nchunks, int splits, float* part, hipStream_t s);
hipError_t launch_features(const float* part, int splits, int M, const float* nu, int ngroups,
                           const int4* cplan, const float* f_adj, float scale, float* feat,
                           hipStream_t s);
hipError_t launch_mlp_forward(const float* prm, const float* feat, const int32_t* idx, int n,
                              float* pre, float* pred, hipStream_t s);
hipError_t launch_screen(const float* pred, int M, int N, int n_c, int kc, const int32_t* flag,
                         int32_t* chosen, float* chosen_pred, hipStream_t s);
hipError_t launch_gather(const float* cur, const float* cand, float* nxt, int64_t stride,
                         int pop, int n_e, const int4* plan, const int32_t* chosen,
                         const float* f_adj, const float* cf_inh, float* f_inh_next,
                         hipStream_t s);
// The surrogate's training gradient is summed over blocks of rows; grad
// holds mlp_grad_blocks(N) * (parameter count) partial sums followed by as
// many row counts.
int mlp_grad_blocks(int N);
hipError_t launch_mlp_train_step(float* prm, const float* feat, const int32_t* idx, int N,
                                 const float* y, float* pre, float* pred, float* grad, float lr,
                                 hipStream_t s);
hipError_t launch_standardize(const float* feat, int M, float* z, hipStream_t s);
hipError_t launch_targets(const float* y, int N, float* out, hipStream_t s);
hipError_t launch_surrogate_judge(const float* pred, const float* y, const float* yt, int N,
                                  int warmup, float tau_min, int32_t* state, float* stats,
                                  float* stats_out, hipStream_t s);

// rng.hip (generator entry points)
hipError_t launch_rng_philox(const uint32_t* ctr, uint64_t key, uint32_t* out, int64_t n,
                             hipStream_t s);
hipError_t launch_rng_ln32(const float* u, float* out, int64_t n, hipStream_t s);
hipError_t launch_rng_normal_pairs(const uint32_t* ab, float* z, int64_t n, hipStream_t s);

}  // namespace leea
