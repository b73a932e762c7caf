// C ABI of libleea.so: argument validation, workspace carving, the call-order
// state machine of Algorithm 1 and kernel sequencing.  Declarations and the
// contract of every entry point are in include/leea.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "../../include/leea.h"
#include "internal.hpp"

using namespace leea;

namespace {

enum State { kNeedEval = 0, kEvaluated = 1, kSelected = 2 };

// Message of the last failure of a call without a ctx: a fixed buffer, so
// that reporting an error never allocates.
thread_local char g_err[512];

constexpr uint32_t kStateMagic = 0x4C454541u;  // checkpoint tag
constexpr uint32_t kStateVersion = 2u;

}  // namespace

struct leea_ctx {
  leea_config cfg;
  NetDesc nd;
  hipStream_t stream;
  float* genomes[2];
  int cur;
  float* f_adj;
  float* f_raw;
  float* acc;
  float* f_inh;
  float* f_inh_next;
  int4* plan;
  int32_t* order;
  float2* partial;
  float* sig[2];   // self-adaptive sigma genes (ping-pong with the genomes)
  int n_mt_max;
  int side;        // input image side when draw_batch pools 2x2, else 0
  float tau;       // effective self-adaptation rate
  uint32_t gen;
  int state;
  int has_inh;
  float sigma;
  int fused;       // leea_step may fuse variation and small-batch evaluation
  int dt;          // arithmetic of the first layer (LEEA_DT_*)
  int kp;          // n0 rounded up to 32 (packed quantised batch row)
  uint32_t* w_amax[2];  // FP8: largest |W_1| of each network (ping-pong with the genomes)
  uint32_t* x_amax;     // FP8: largest |x| of the batch being evaluated
  void* xq;             // quantised batch (values [b][n0], packed [b][kp] or chunk-major)
  W1Shadow wsh;         // bfloat16 copy of every W_1 (bfloat16 kernels), or none
  W1Fp8 w8;             // FP8 copy of every W_1 with its scale bounds (FP8 kernels)
  uint32_t* w_bound;    // FP8: bound of each network's largest |W_1| (scale of its copy)
  uint32_t* tail_amax;  // FP8: largest |W_l| (l >= 2) of each network, [pop][kTailScales]
  int w8_ok;            // FP8 amax, bounds and copy match the current population
  int wsh_ok;           // the copy matches the current population
  // fitness surrogate (leea_surrogate_attach)
  int sur;
  leea_surrogate_config sc;
  int sM, sN, skc, snc, sngroups, snchunks, ssplits;
  float* scand;
  int4* scplan;
  float* scf_inh;
  float* snu;
  float* spart;
  float* sfeat;
  float* szfeat;   // standardised features (the MLP's inputs)
  float* sytgt;    // standardised fitness of the kept candidates (training targets)
  float* spred;
  int32_t* schosen;
  float* schosen_pred;
  float* spred_t;
  uint32_t* sbits;
  float* sprm;
  float* sgrad;
  float* spre;
  int32_t* sstate;
  float* sstats;
  std::string err;
};

namespace {

leea_status fail(leea_ctx* c, leea_status st, const char* fmt, const char* extra = nullptr) {
  if (c) {
    char buf[512];
    snprintf(buf, sizeof buf, fmt, extra ? extra : "");
    c->err = buf;
  } else {
    snprintf(g_err, sizeof g_err, fmt, extra ? extra : "");
  }
  return st;
}

leea_status dev(leea_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return LEEA_OK;
  if (c) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    c->err = buf;
  } else {
    snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
  }
  return LEEA_EDEVICE;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

leea_status validate(const leea_config* cfg, NetDesc* nd) {
  if (!cfg) return fail(nullptr, LEEA_EINVAL, "config is NULL");
  const int L = cfg->n_layers;
  if (L < 1 || L > LEEA_MAX_LAYERS) return fail(nullptr, LEEA_EINVAL, "n_layers must be 1..8");
  if (cfg->widths[0] < 4 || cfg->widths[0] % 4 != 0 || cfg->widths[0] > 1 << 20)
    return fail(nullptr, LEEA_EINVAL, "widths[0] must be a positive multiple of 4");
  for (int l = 1; l <= L; ++l)
    if (cfg->widths[l] < 1 || cfg->widths[l] > LEEA_MAX_WIDTH)
      return fail(nullptr, LEEA_EINVAL, "widths[1..L] must be in 1..256");
  if (cfg->widths[L] < 2) return fail(nullptr, LEEA_EINVAL, "need at least 2 classes");
  if (cfg->pop < 1 || cfg->pop > LEEA_MAX_POP)
    return fail(nullptr, LEEA_EINVAL, "pop must be in 1..8192");
  if (cfg->n_elite < 0 || cfg->n_cross < 0 || cfg->n_mut < 0 ||
      (int64_t)cfg->n_elite + cfg->n_cross + cfg->n_mut != cfg->pop)
    return fail(nullptr, LEEA_EINVAL, "n_elite + n_cross + n_mut must equal pop");
  if (cfg->n_trunc < 1 || cfg->n_trunc > cfg->pop)
    return fail(nullptr, LEEA_EINVAL, "n_trunc must be in 1..pop");
  if (cfg->selection != LEEA_SEL_TRUNCATION && cfg->selection != LEEA_SEL_TOURNAMENT)
    return fail(nullptr, LEEA_EINVAL, "unknown selection");
  if (cfg->selection == LEEA_SEL_TOURNAMENT && (cfg->tournament_k < 1 || cfg->tournament_k > 16))
    return fail(nullptr, LEEA_EINVAL, "tournament_k must be in 1..16");
  if (cfg->crossover != LEEA_XO_UNIFORM && cfg->crossover != LEEA_XO_ARITHMETIC)
    return fail(nullptr, LEEA_EINVAL, "unknown crossover");
  if (!(cfg->sigma >= 0.0f) || cfg->sigma == __builtin_inff())
    return fail(nullptr, LEEA_EINVAL, "sigma must be finite and >= 0");
  if (!(cfg->alpha >= 0.0f && cfg->alpha <= 1.0f))
    return fail(nullptr, LEEA_EINVAL, "alpha must be in [0, 1]");
  if (cfg->mut_threshold > (1ull << 32))
    return fail(nullptr, LEEA_EINVAL, "mut_threshold must be <= 2^32");
  if (cfg->max_batch < 1 || cfg->max_batch > LEEA_MAX_BATCH)
    return fail(nullptr, LEEA_EINVAL, "max_batch must be in 1..65536");
  for (int l = 0; l < L; ++l)
    if (!(cfg->glorot_a[l] >= 0.0f) || cfg->glorot_a[l] == __builtin_inff())
      return fail(nullptr, LEEA_EINVAL, "glorot_a must be finite and >= 0");
  if (cfg->sigma_mode < LEEA_SIGMA_CONSTANT || cfg->sigma_mode > LEEA_SIGMA_SELF_ADAPTIVE)
    return fail(nullptr, LEEA_EINVAL, "unknown sigma_mode");
  if (cfg->sigma_mode == LEEA_SIGMA_DECAY &&
      !(cfg->sigma_decay_k > 0.0f && cfg->sigma_decay_k < __builtin_inff()))
    return fail(nullptr, LEEA_EINVAL, "sigma_decay_k must be positive and finite");
  if (!(cfg->tau >= 0.0f && cfg->tau <= 10.0f))
    return fail(nullptr, LEEA_EINVAL, "tau must be in [0, 10]");
  if (cfg->input_pool != 0 && cfg->input_pool != 2)
    return fail(nullptr, LEEA_EINVAL, "input_pool must be 0 or 2");
  if (cfg->eval_dtype < LEEA_DT_F32 || cfg->eval_dtype > LEEA_DT_FP8)
    return fail(nullptr, LEEA_EINVAL, "unknown eval_dtype");
  if (cfg->input_pool == 2) {
    const int64_t raw = 4ll * cfg->widths[0];
    int64_t side = (int64_t)sqrt((double)raw);
    while (side * side < raw) ++side;
    if (side * side != raw || side % 2 != 0)
      return fail(nullptr, LEEA_EINVAL, "input_pool needs 4*widths[0] to be an even square");
  }
  NetDesc d;
  memset(&d, 0, sizeof d);
  d.L = L;
  int64_t off = 0;
  for (int l = 0; l <= L; ++l) d.w[l] = cfg->widths[l];
  for (int l = 0; l < L; ++l) {
    d.woff[l] = off;
    off += (int64_t)d.w[l + 1] * d.w[l];
    d.boff[l] = off;
    off += d.w[l + 1];
  }
  d.genes = off;
  d.stride = (off + 63) & ~(int64_t)63;
  if ((int64_t)cfg->pop * d.stride > (1ll << 40))
    return fail(nullptr, LEEA_EINVAL, "population too large");
  if (d.stride > 0xFFFFFFFFll * 4)
    return fail(nullptr, LEEA_EINVAL, "network too large for 32-bit gene blocks");
  if (cfg->eval_dtype != LEEA_DT_F32 && cfg->max_batch > 16 &&
      !eval_lp_supported(d, cfg->max_batch, cfg->eval_dtype))
    return fail(nullptr, LEEA_EINVAL, "reduced-precision evaluation does not fit these widths");
  if (nd) *nd = d;
  return LEEA_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Carve {
  size_t genomes, scalars, plan, order, partial, xq, wsh, w8, tail, total;
};

int padded_k(int n0) { return (n0 + 31) & ~31; }
int round128(int v) { return (v + 127) & ~127; }

// bfloat16 W_1 copy, read by the bfloat16 evaluation kernels at every batch
// size (small batches: half the bytes of the float32 W_1 they would stream
// otherwise); kept when W_1 has fewer than 2^24 genes (the variation kernel
// finds a gene's row with a float reciprocal)
bool uses_shadow(const leea_config* cfg, const NetDesc& nd) {
  return cfg->eval_dtype == LEEA_DT_BF16 && (int64_t)nd.w[0] * nd.w[1] < (1 << 24);
}
int64_t shadow_net(const NetDesc& nd) {
  return (int64_t)padded_k(nd.w[0]) * ((nd.w[1] + 15) & ~15);
}

// FP8 copy of W_1: kept with an FP8 first layer when W_1 has fewer than 2^24
// genes; rows padded to 16, K to 64 (one byte per element)
bool uses_fp8_copy(const leea_config* cfg, const NetDesc& nd) {
  return cfg->eval_dtype == LEEA_DT_FP8 && (int64_t)nd.w[0] * nd.w[1] < (1 << 24);
}
int fp8_kp(int n0) { return (n0 + 63) & ~63; }
int64_t fp8_net(const NetDesc& nd) { return (int64_t)fp8_kp(nd.w[0]) * ((nd.w[1] + 15) & ~15); }

Carve carve(const leea_config* cfg, const NetDesc& nd) {
  Carve c;
  const size_t P = (size_t)cfg->pop;
  const int n_mt = (cfg->max_batch + 63) / 64;
  c.genomes = align256(P * (size_t)nd.stride * 4);
  c.scalars = align256(P * 4);
  c.plan = align256(P * 16);
  c.order = align256(P * 4);
  c.partial = align256(P * (size_t)n_mt * 8);
  c.xq = 0;
  c.wsh = 0;
  c.w8 = 0;
  c.tail = 0;
  if (cfg->eval_dtype != LEEA_DT_F32) {
    const size_t kp = (size_t)padded_k(nd.w[0]);
    const size_t row = (size_t)nd.w[0] * 4 > kp * 2 ? (size_t)nd.w[0] * 4 : kp * 2;
    const size_t chunked = (size_t)round128(cfg->max_batch) * kp * 2;
    const size_t q = (size_t)cfg->max_batch * row > chunked ? (size_t)cfg->max_batch * row
                                                            : chunked;
    c.xq = align256(q) + 256;  // + the batch amax
    if (uses_shadow(cfg, nd)) c.wsh = align256(P * (size_t)shadow_net(nd) * 2);
    if (uses_fp8_copy(cfg, nd)) c.w8 = align256(P * (size_t)fp8_net(nd));
    if (cfg->eval_dtype == LEEA_DT_FP8) c.tail = align256(P * (size_t)kTailScales * 4);
  }
  c.total = 2 * c.genomes + 10 * c.scalars + c.plan + c.order + c.partial + c.xq + c.wsh + c.w8 +
            c.tail;
  return c;
}

Key key_of(const leea_ctx* c) {
  Key k;
  k.k0 = (uint32_t)c->cfg.seed;
  k.k1 = (uint32_t)(c->cfg.seed >> 32);
  k.run = c->cfg.run;
  return k;
}

leea_status check_batch(leea_ctx* c, const float* x, const int32_t* y, int32_t b) {
  if (!x || !y) return fail(c, LEEA_EINVAL, "x and y must be device pointers");
  if (!aligned16(x)) return fail(c, LEEA_EINVAL, "x must be 16-byte aligned");
  if (b < 1 || b > c->cfg.max_batch) return fail(c, LEEA_EINVAL, "b must be in 1..max_batch");
  return LEEA_OK;
}

// The bfloat16 copy of W_1, rebuilt first if the population changed other
// than through the variation kernel.
leea_status shadow_ready(leea_ctx* c) {
  if (!c->wsh.p || c->wsh_ok) return LEEA_OK;
  leea_status st = dev(c, launch_shadow_w1(c->genomes[c->cur], c->nd, c->cfg.pop, c->wsh,
                                           c->stream),
                       "W1 copy launch");
  if (!st) c->wsh_ok = 1;
  return st;
}

// FP8: the exact largest |W_1| of every network of the current population,
// the scale bounds (equal to it) and the FP8 copy, rebuilt when the
// population changed other than through the variation kernel (which keeps
// all three in step for the children it makes).
leea_status fp8_ready(leea_ctx* c) {
  if (c->dt != LEEA_DT_FP8 || c->w8_ok) return LEEA_OK;
  leea_status st = dev(c, launch_amax_w1(c->genomes[c->cur], c->nd, c->cfg.pop,
                                         c->w_amax[c->cur], c->stream),
                       "amax launch");
  if (!st)
    st = dev(c, hipMemcpyAsync(c->w_bound, c->w_amax[c->cur], (size_t)c->cfg.pop * 4,
                               hipMemcpyDeviceToDevice, c->stream),
             "bound copy");
  if (!st && c->w8.p)
    st = dev(c, launch_fp8_copy(c->genomes[c->cur], c->nd, c->cfg.pop, c->w8, c->stream),
             "FP8 copy launch");
  if (!st) c->w8_ok = 1;
  return st;
}

// Reduced-precision forward pass: FP8 scales, the quantised batch, then
// the small-batch kernel on quantised values (b <= 16) or the bf16 / FP8
// matrix-core kernel.  Returns the number of partial row tiles.
leea_status run_eval_lp(leea_ctx* c, const float* x, const int32_t* y, int32_t b, int* n_mt) {
  const int n0 = c->nd.w[0];
  leea_status st = fp8_ready(c);
  if (st) return st;
  if (c->dt == LEEA_DT_FP8) {
    // the batch amax and the later layers' largest magnitudes in one launch
    st = dev(c, launch_fp8_scales(x, (int64_t)b * n0, c->x_amax, c->genomes[c->cur], c->nd,
                                  c->cfg.pop, c->tail_amax, c->stream),
             "FP8 scales launch");
    if (st) return st;
  }
  const bool small = b <= 16;
  if (!small && c->wsh.p && eval_lpw_supported(c->nd, b)) {
    // large batch from the bfloat16 W_1 copy
    st = shadow_ready(c);
    if (st) return st;
    const int bpad = round128(b);
    st = dev(c, launch_quantize_x_chunks(x, b, n0, c->kp, bpad, (uint16_t*)c->xq, c->stream),
             "quantize launch");
    if (st) return st;
    *n_mt = eval_lpw_ptiles(c->nd, b);
    return dev(c, launch_evaluate_lpw(c->genomes[c->cur], c->nd, c->cfg.pop, c->wsh,
                                      (const uint16_t*)c->xq, c->kp, bpad, y, b, c->partial,
                                      c->stream),
               "evaluate launch");
  }
  if (!small && c->w8.p && eval_lpw_supported(c->nd, b)) {
    // large batch from the FP8 copy of W_1 (fp8_ready above rebuilt it if
    // needed; the batch amax is computed above)
    const int bpad = round128(b);
    st = dev(c, launch_quantize_x_chunks8(x, b, n0, c->w8.kp, bpad, c->x_amax,
                                          (uint8_t*)c->xq, c->stream),
             "quantize launch");
    if (st) return st;
    *n_mt = eval_lpw_ptiles(c->nd, b);
    return dev(c, launch_evaluate_lpw8(c->genomes[c->cur], c->nd, c->cfg.pop, c->w8,
                                       (const uint8_t*)c->xq, bpad, c->x_amax, y, b, c->partial,
                                       c->stream),
               "evaluate launch");
  }
  if (!small && !eval_lp_supported(c->nd, b, c->dt))
    return fail(c, LEEA_EINVAL, "reduced-precision evaluation does not fit this batch");
  st = dev(c, launch_quantize_x(c->dt, !small, x, b, n0, c->kp, c->x_amax, c->xq, c->stream),
           "quantize launch");
  if (st) return st;
  if (small) {
    *n_mt = 1;
    return dev(c, launch_evaluate_small_lp(c->dt, c->genomes[c->cur], c->nd, c->cfg.pop,
                                           (const float*)c->xq, y, b, c->partial,
                                           c->w_bound, c->x_amax, c->stream),
               "evaluate launch");
  }
  *n_mt = eval_lp_ptiles(c->nd, b, c->dt);
  return dev(c, launch_evaluate_lp(c->dt, c->genomes[c->cur], c->nd, c->cfg.pop, c->xq, c->kp,
                                   c->w_bound, c->x_amax, y, b, c->partial, c->stream),
             "evaluate launch");
}

leea_status run_eval(leea_ctx* c, const float* x, const int32_t* y, int32_t b, bool update,
                     float* f_adj, float* f_raw, float* acc) {
  int n_mt = 1;
  leea_status st;
  const int use_inh = update && c->has_inh && c->cfg.alpha != 1.0f;
  // batches of up to 16 rows: the evaluation kernel finishes each network
  // itself (no finalize launch)
  const FinArgs fin{c->f_inh, update ? c->f_adj : nullptr, update ? c->f_raw : nullptr,
                    update ? c->acc : nullptr, f_adj, f_raw, acc, c->cfg.alpha, use_inh, 1};
  if (c->dt == LEEA_DT_BF16 && b <= 16) {
    st = shadow_ready(c);
    if (st) return st;
    return dev(c, launch_evaluate_small_bf16(c->genomes[c->cur], c->nd, c->cfg.pop, c->wsh, x, y,
                                             b, c->partial, c->stream, fin),
               "evaluate launch");
  }
  if (c->dt == LEEA_DT_FP8 && b <= 16 && c->w8.p) {
    st = fp8_ready(c);
    if (!st)
      st = dev(c, launch_fp8_scales(x, (int64_t)b * c->nd.w[0], c->x_amax, c->genomes[c->cur],
                                    c->nd, c->cfg.pop, c->tail_amax, c->stream),
               "FP8 scales launch");
    if (st) return st;
    return dev(c, launch_evaluate_small_fp8(c->genomes[c->cur], c->nd, c->cfg.pop, c->w8, x,
                                            c->x_amax, y, b, c->partial, c->stream, fin),
               "evaluate launch");
  }
  if (c->dt == LEEA_DT_F32) {
    bool finalized = false;
    st = dev(c, launch_evaluate(c->genomes[c->cur], c->nd, c->cfg.pop, x, y, b, c->partial,
                                c->stream, &fin, &finalized),
             "evaluate launch");
    if (st || finalized) return st;
    n_mt = eval_mtiles(c->nd, b);
  } else {
    st = run_eval_lp(c, x, y, b, &n_mt);
  }
  if (st) return st;
  st = dev(c, launch_finalize(c->partial, c->cfg.pop, n_mt, b, c->f_inh, use_inh, c->cfg.alpha,
                              update ? c->f_adj : nullptr, update ? c->f_raw : nullptr,
                              update ? c->acc : nullptr, f_adj, f_raw, acc, c->stream),
           "finalize launch");
  return st;
}

}  // namespace

extern "C" {

leea_status leea_param_count(const leea_config* cfg, int64_t* genes, int64_t* stride) {
  NetDesc nd;
  leea_status st = validate(cfg, &nd);
  if (st) return st;
  if (genes) *genes = nd.genes;
  if (stride) *stride = nd.stride;
  return LEEA_OK;
}

leea_status leea_config_from_fractions(leea_config* cfg, double p_elite, double p_cross,
                                       double p_mut, double rho, double p_gene) {
  if (!cfg) return fail(nullptr, LEEA_EINVAL, "config is NULL");
  const int L = cfg->n_layers;
  if (L < 1 || L > LEEA_MAX_LAYERS) return fail(nullptr, LEEA_EINVAL, "n_layers must be 1..8");
  if (cfg->pop < 1) return fail(nullptr, LEEA_EINVAL, "pop must be positive");
  if (!(p_elite >= 0.0 && p_cross >= 0.0 && p_mut >= 0.0 && rho >= 0.0 && rho <= 1.0))
    return fail(nullptr, LEEA_EINVAL, "fractions must be in [0, 1]");
  if (fabs(p_elite + p_cross + p_mut - 1.0) > 1e-9)
    return fail(nullptr, LEEA_EINVAL, "p_elite + p_cross + p_mut must equal 1");
  if (!(p_gene >= 0.0 && p_gene <= 1.0)) return fail(nullptr, LEEA_EINVAL, "p_gene must be in [0, 1]");
  const double pop = (double)cfg->pop;
  const int64_t n_e = (int64_t)floor(p_elite * pop + 0.5);
  const int64_t n_c = (int64_t)floor(p_cross * pop + 0.5);
  const int64_t n_m = cfg->pop - n_e - n_c;
  if (n_e < 0 || n_c < 0 || n_m < 0)
    return fail(nullptr, LEEA_EINVAL, "counts do not fit the population");
  int64_t n_r = (int64_t)floor(rho * pop + 0.5);
  n_r = n_r < 1 ? 1 : (n_r > cfg->pop ? cfg->pop : n_r);
  cfg->n_elite = (int32_t)n_e;
  cfg->n_cross = (int32_t)n_c;
  cfg->n_mut = (int32_t)n_m;
  cfg->n_trunc = (int32_t)n_r;
  // p * 2^32 is exact in double (a power-of-two scaling), so the floor is too
  const double t = floor(p_gene * 4294967296.0);
  cfg->mut_threshold = t >= 4294967296.0 ? (1ull << 32) : (uint64_t)t;
  // widths are checked by every call that takes cfg; a bound whose fan sum
  // is not positive is left at zero
  for (int l = 0; l < LEEA_MAX_LAYERS; ++l) {
    const double fan = l < L ? (double)cfg->widths[l] + (double)cfg->widths[l + 1] : 0.0;
    cfg->glorot_a[l] = fan > 0.0 ? (float)sqrt(6.0 / fan) : 0.0f;
  }
  return LEEA_OK;
}

leea_status leea_workspace_bytes(const leea_config* cfg, size_t* bytes) {
  NetDesc nd;
  leea_status st = validate(cfg, &nd);
  if (st) return st;
  if (!bytes) return fail(nullptr, LEEA_EINVAL, "bytes is NULL");
  *bytes = carve(cfg, nd).total;
  return LEEA_OK;
}

leea_status leea_init_population(const leea_config* cfg, void* workspace, size_t bytes,
                                 void* hip_stream, leea_ctx** out) {
  NetDesc nd;
  leea_status st = validate(cfg, &nd);
  if (st) return st;
  if (!out) return fail(nullptr, LEEA_EINVAL, "out is NULL");
  *out = nullptr;
  if (!workspace) return fail(nullptr, LEEA_EINVAL, "workspace is NULL");
  if ((uintptr_t)workspace & 255u) return fail(nullptr, LEEA_EINVAL, "workspace must be 256-byte aligned");
  const Carve cv = carve(cfg, nd);
  if (bytes < cv.total) return fail(nullptr, LEEA_ENOMEM, "workspace smaller than leea_workspace_bytes");
  leea_ctx* c = new (std::nothrow) leea_ctx();
  if (!c) return fail(nullptr, LEEA_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->nd = nd;
  c->stream = (hipStream_t)hip_stream;
  char* p = (char*)workspace;
  c->genomes[0] = (float*)p;
  p += cv.genomes;
  c->genomes[1] = (float*)p;
  p += cv.genomes;
  c->f_adj = (float*)p;
  p += cv.scalars;
  c->f_raw = (float*)p;
  p += cv.scalars;
  c->acc = (float*)p;
  p += cv.scalars;
  c->f_inh = (float*)p;
  p += cv.scalars;
  c->f_inh_next = (float*)p;
  p += cv.scalars;
  c->plan = (int4*)p;
  p += cv.plan;
  c->order = (int32_t*)p;
  p += cv.order;
  c->partial = (float2*)p;
  p += cv.partial;
  c->sig[0] = (float*)p;
  p += cv.scalars;
  c->sig[1] = (float*)p;
  p += cv.scalars;
  c->w_amax[0] = (uint32_t*)p;
  p += cv.scalars;
  c->w_amax[1] = (uint32_t*)p;
  p += cv.scalars;
  c->x_amax = cv.xq ? (uint32_t*)p : nullptr;
  c->xq = cv.xq ? (void*)(p + 256) : nullptr;
  p += cv.xq;
  c->wsh.p = cv.wsh ? (uint16_t*)p : nullptr;
  c->wsh.net = shadow_net(nd);
  c->wsh.n0 = nd.w[0];
  c->wsh.nrp = (nd.w[1] + 15) & ~15;
  c->wsh.kp = padded_k(nd.w[0]);
  c->wsh.rcp_n0 = 1.0f / (float)nd.w[0];
  c->wsh_ok = 0;
  p += cv.wsh;
  c->w_bound = (uint32_t*)p;
  p += cv.scalars;
  c->w8.p = cv.w8 ? (uint8_t*)p : nullptr;
  c->w8.net = fp8_net(nd);
  c->w8.n0 = nd.w[0];
  c->w8.nrp = (nd.w[1] + 15) & ~15;
  c->w8.kp = fp8_kp(nd.w[0]);
  c->w8.rcp_n0 = 1.0f / (float)nd.w[0];
  c->w8.amax_par = nullptr;
  c->w8.bound = c->w_bound;
  c->w8_ok = 0;
  p += cv.w8;
  c->tail_amax = cv.tail ? (uint32_t*)p : nullptr;
  c->w8.tail = c->tail_amax;
  p += cv.tail;
  c->dt = cfg->eval_dtype;
  c->kp = padded_k(nd.w[0]);
  c->n_mt_max = (cfg->max_batch + 63) / 64;
  c->side = 0;
  if (cfg->input_pool == 2) {
    int side = 2;
    while ((int64_t)side * side < 4ll * cfg->widths[0]) side += 2;
    c->side = side;
  }
  c->tau = cfg->tau > 0.0f ? cfg->tau : (float)(1.0 / sqrt((double)nd.genes));
  c->cur = 0;
  c->gen = 0;
  c->state = kNeedEval;
  c->has_inh = 0;
  c->sigma = cfg->sigma;
  c->fused = 0;
  c->sur = 0;
  Glorot ga;
  for (int l = 0; l < LEEA_MAX_LAYERS; ++l) ga.a[l] = l < nd.L ? cfg->glorot_a[l] : 0.0f;
  st = dev(nullptr, launch_init(c->genomes[0], nd, ga, cfg->pop, key_of(c), c->stream),
           "init launch");
  if (!st && cfg->sigma_mode == LEEA_SIGMA_SELF_ADAPTIVE)
    st = dev(nullptr, launch_fill(c->sig[0], cfg->pop, cfg->sigma, c->stream), "sigma fill");
  if (!st && c->dt == LEEA_DT_FP8) {
    st = fp8_ready(c);
    if (st) fail(nullptr, st, "%s", c->err.c_str());
  }
  // the whole copy, padding included (the variation writes only W_1 itself)
  if (!st && c->wsh.p)
    st = dev(nullptr, launch_shadow_w1(c->genomes[0], nd, cfg->pop, c->wsh, c->stream),
             "W1 copy launch");
  c->wsh_ok = c->wsh.p ? 1 : 0;
  if (st) {
    delete c;
    return st;
  }
  *out = c;
  return LEEA_OK;
}

leea_status leea_draw_batch(leea_ctx* c, uint32_t gen, const float* x_train,
                            const int32_t* y_train, int64_t n_train, int32_t b, float* x_out,
                            int32_t* y_out) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (!x_train || !y_train || !x_out || !y_out)
    return fail(c, LEEA_EINVAL, "training and output arrays must be device pointers");
  if (!aligned16(x_train) || !aligned16(x_out))
    return fail(c, LEEA_EINVAL, "x arrays must be 16-byte aligned");
  if (n_train < 1 || n_train > 0xFFFFFFFFll) return fail(c, LEEA_EINVAL, "n_train out of range");
  if (b < 1 || b > LEEA_MAX_BATCH) return fail(c, LEEA_EINVAL, "b out of range");
  return dev(c, launch_draw_batch(x_train, y_train, n_train, c->nd.w[0], c->side, b, x_out,
                                  y_out, key_of(c), gen, c->stream),
             "draw_batch launch");
}

leea_status leea_evaluate(leea_ctx* c, const float* x, const int32_t* y, int32_t b,
                          float* f_adj, float* f_raw, float* acc) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (c->state == kSelected)
    return fail(c, LEEA_ESTATE, "evaluate after select: call crossover_mutate first");
  leea_status st = check_batch(c, x, y, b);
  if (st) return st;
  st = run_eval(c, x, y, b, true, f_adj, f_raw, acc);
  if (st) return st;
  c->state = kEvaluated;
  return LEEA_OK;
}

leea_status leea_score(leea_ctx* c, const float* x, const int32_t* y, int32_t n, float* f_raw,
                       float* acc) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  leea_status st = check_batch(c, x, y, n);
  if (st) return st;
  return run_eval(c, x, y, n, false, nullptr, f_raw, acc);
}

leea_status leea_select(leea_ctx* c, int32_t* plan_out, float* f_inh_out, int32_t* order_out) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (c->state != kEvaluated) return fail(c, LEEA_ESTATE, "select needs an evaluated population");
  const leea_config& g = c->cfg;
  leea_status st = dev(c,
                       launch_select(c->f_adj, g.pop, g.n_elite, g.n_cross, g.n_trunc,
                                     g.selection, g.tournament_k, key_of(c), c->gen + 1, c->plan,
                                     c->f_inh_next, c->order, c->stream),
                       "select launch");
  if (st) return st;
  if (plan_out)
    st = dev(c, hipMemcpyAsync(plan_out, c->plan, (size_t)g.pop * 16, hipMemcpyDeviceToDevice,
                               c->stream), "plan copy");
  if (!st && f_inh_out)
    st = dev(c, hipMemcpyAsync(f_inh_out, c->f_inh_next, (size_t)g.pop * 4,
                               hipMemcpyDeviceToDevice, c->stream), "f_inh copy");
  if (!st && order_out)
    st = dev(c, hipMemcpyAsync(order_out, c->order, (size_t)g.pop * 4, hipMemcpyDeviceToDevice,
                               c->stream), "order copy");
  if (st) return st;
  c->state = kSelected;
  return LEEA_OK;
}

}  // extern "C"

namespace {

// Mutation strength of the variation that creates generation g (constant,
// decayed, or NULL sigma arrays unless self-adaptive).
void vary_sigma(const leea_ctx* c, uint32_t g, float* sigma, const float** sig_cur,
                float** sig_next) {
  *sigma = c->sigma;
  if (c->cfg.sigma_mode == LEEA_SIGMA_DECAY)
    *sigma = (float)((double)c->sigma * pow(0.99, (double)g / (double)c->cfg.sigma_decay_k));
  const bool adaptive = c->cfg.sigma_mode == LEEA_SIGMA_SELF_ADAPTIVE;
  *sig_cur = adaptive ? c->sig[c->cur] : nullptr;
  *sig_next = adaptive ? c->sig[c->cur ^ 1] : nullptr;
}

// The new population becomes current: buffers swap, inherited fitness of
// the plan takes effect, the generation advances.
void advance(leea_ctx* c) {
  c->cur ^= 1;
  float* t = c->f_inh;
  c->f_inh = c->f_inh_next;
  c->f_inh_next = t;
  c->has_inh = 1;
  c->gen += 1;
  c->state = kNeedEval;
}

}  // namespace

extern "C" {

leea_status leea_crossover_mutate(leea_ctx* c) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (c->state != kSelected) return fail(c, LEEA_ESTATE, "crossover_mutate needs a select first");
  const uint32_t g = c->gen + 1;
  float sigma;
  const float* sig_cur;
  float* sig_next;
  vary_sigma(c, g, &sigma, &sig_cur, &sig_next);
  uint32_t* amax = c->dt == LEEA_DT_FP8 ? c->w_amax[c->cur ^ 1] : nullptr;
  leea_status st = fp8_ready(c);  // the parents' largest magnitudes
  if (!st && amax) st = dev(c, launch_fill((float*)amax, c->cfg.pop, 0.0f, c->stream), "amax clear");
  if (st) return st;
  W1Fp8 w8 = c->w8;
  if (c->dt == LEEA_DT_FP8) {
    w8.amax_par = c->w_amax[c->cur];
    w8.bound = c->w_bound;
  } else {
    w8.bound = nullptr;
  }
  st = dev(c,
           launch_vary(c->genomes[c->cur], c->genomes[c->cur ^ 1], c->plan, c->nd, c->cfg.pop,
                       c->cfg.crossover, sigma, c->cfg.mut_threshold, key_of(c), g, sig_cur,
                       sig_next, c->tau, amax, c->wsh, w8, c->stream),
           "vary launch");
  if (st) return st;
  c->wsh_ok = c->wsh.p ? 1 : 0;  // the variation wrote the children's copies
  advance(c);
  return LEEA_OK;
}

leea_status leea_crossover_mutate_evaluate(leea_ctx* c, const float* x, const int32_t* y,
                                          int32_t b, float* f_adj, float* f_raw, float* acc) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (c->state != kSelected)
    return fail(c, LEEA_ESTATE, "crossover_mutate_evaluate needs a select first");
  leea_status st = check_batch(c, x, y, b);
  if (st) return st;
  // the fused kernel multiplies on the matrix cores like the small-batch
  // kernel; batches the row-streaming or 1 KiB-row kernels take keep the
  // separate calls (their sums are grouped differently)
  if (!(c->fused && c->dt == LEEA_DT_F32 && fused_supported(c->nd, b) &&
        !eval_stream_supported(c->nd, b) && !eval_rows_supported(c->nd, b))) {
    st = leea_crossover_mutate(c);
    if (st) return st;
    return leea_evaluate(c, x, y, b, f_adj, f_raw, acc);
  }
  // small batch: variation and evaluation in one pass over the parents
  const uint32_t g = c->gen + 1;
  float sigma;
  const float* sig_cur;
  float* sig_next;
  vary_sigma(c, g, &sigma, &sig_cur, &sig_next);
  st = dev(c,
           launch_vary_eval(c->genomes[c->cur], c->genomes[c->cur ^ 1], c->plan, c->nd,
                            c->cfg.pop, c->cfg.crossover, sigma, c->cfg.mut_threshold, key_of(c),
                            g, sig_cur, sig_next, c->tau, x, y, b, c->partial, c->stream),
           "fused vary+evaluate launch");
  if (st) return st;
  advance(c);
  const int use_inh = c->cfg.alpha != 1.0f;
  st = dev(c, launch_finalize(c->partial, c->cfg.pop, 1, b, c->f_inh, use_inh, c->cfg.alpha,
                              c->f_adj, c->f_raw, c->acc, f_adj, f_raw, acc, c->stream),
           "finalize launch");
  if (st) return st;
  c->state = kEvaluated;
  return LEEA_OK;
}

leea_status leea_step(leea_ctx* c, const float* x, const int32_t* y, int32_t b, float* f_adj,
                      float* f_raw, float* acc) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (c->state != kEvaluated) return fail(c, LEEA_ESTATE, "step needs an evaluated population");
  leea_status st = check_batch(c, x, y, b);
  if (st) return st;
  st = leea_select(c, nullptr, nullptr, nullptr);
  if (st) return st;
  return leea_crossover_mutate_evaluate(c, x, y, b, f_adj, f_raw, acc);
}

leea_status leea_set_fused_step(leea_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  c->fused = enable ? 1 : 0;
  return LEEA_OK;
}

leea_status leea_set_sigma(leea_ctx* c, float sigma) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (!(sigma >= 0.0f) || sigma == __builtin_inff())
    return fail(c, LEEA_EINVAL, "sigma must be finite and >= 0");
  c->sigma = sigma;
  if (c->cfg.sigma_mode == LEEA_SIGMA_SELF_ADAPTIVE)
    return dev(c, launch_fill(c->sig[c->cur], c->cfg.pop, sigma, c->stream), "sigma fill");
  return LEEA_OK;
}

leea_status leea_sigmas(leea_ctx* c, float** sigmas) {
  if (!c || !sigmas) return fail(nullptr, LEEA_EINVAL, "NULL argument");
  *sigmas = c->cfg.sigma_mode == LEEA_SIGMA_SELF_ADAPTIVE ? c->sig[c->cur] : nullptr;
  return LEEA_OK;
}

leea_status leea_set_sigmas(leea_ctx* c, const float* sigmas) {
  if (!c || !sigmas) return fail(nullptr, LEEA_EINVAL, "NULL argument");
  if (c->cfg.sigma_mode != LEEA_SIGMA_SELF_ADAPTIVE)
    return fail(c, LEEA_ESTATE, "sigma genes exist only with self-adaptive sigma");
  return dev(c, hipMemcpyAsync(c->sig[c->cur], sigmas, (size_t)c->cfg.pop * 4,
                               hipMemcpyDeviceToDevice, c->stream), "sigma copy");
}

leea_status leea_generation(const leea_ctx* c, uint32_t* gen) {
  if (!c || !gen) return fail(nullptr, LEEA_EINVAL, "NULL argument");
  *gen = c->gen;
  return LEEA_OK;
}

leea_status leea_population(leea_ctx* c, float** genomes, int64_t* stride, float** f_adj) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (genomes) *genomes = c->genomes[c->cur];
  if (stride) *stride = c->nd.stride;
  if (f_adj) *f_adj = c->f_adj;
  return LEEA_OK;
}

leea_status leea_set_state(leea_ctx* c, const float* src, const float* f_adj,
                           const float* f_inh) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  const size_t gbytes = (size_t)c->cfg.pop * c->nd.stride * 4;
  const size_t sbytes = (size_t)c->cfg.pop * 4;
  leea_status st = LEEA_OK;
  if (src)
    st = dev(c, hipMemcpyAsync(c->genomes[c->cur], src, gbytes, hipMemcpyDeviceToDevice,
                               c->stream), "population copy");
  if (!st && f_adj)
    st = dev(c, hipMemcpyAsync(c->f_adj, f_adj, sbytes, hipMemcpyDeviceToDevice, c->stream),
             "f_adj copy");
  if (!st && f_inh)
    st = dev(c, hipMemcpyAsync(c->f_inh, f_inh, sbytes, hipMemcpyDeviceToDevice, c->stream),
             "f_inh copy");
  if (st) return st;
  if (src) {
    c->wsh_ok = 0;
    c->w8_ok = 0;
  }
  c->has_inh = f_inh ? 1 : 0;
  c->state = f_adj ? kEvaluated : kNeedEval;
  return LEEA_OK;
}

// Checkpoint: header {magic, version, gen, state, has_inh, cur=0, sigma,
// pop, stride} then genomes, f_adj, f_raw, acc, f_inh.
struct CkptHeader {
  uint32_t magic, version, gen, state, has_inh;
  float sigma;
  int64_t pop, stride;
  uint64_t seed;
};

leea_status leea_state_bytes(const leea_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(nullptr, LEEA_EINVAL, "NULL argument");
  *bytes = sizeof(CkptHeader) + (size_t)c->cfg.pop * c->nd.stride * 4 + 5 * (size_t)c->cfg.pop * 4;
  return LEEA_OK;
}

leea_status leea_save(leea_ctx* c, void* host_buf, size_t bytes) {
  if (!c || !host_buf) return fail(c, LEEA_EINVAL, "NULL argument");
  size_t need;
  leea_state_bytes(c, &need);
  if (bytes < need) return fail(c, LEEA_ENOMEM, "checkpoint buffer too small");
  CkptHeader h;
  h.magic = kStateMagic;
  h.version = kStateVersion;
  h.gen = c->gen;
  h.state = (uint32_t)c->state;
  h.has_inh = (uint32_t)c->has_inh;
  h.sigma = c->sigma;
  h.pop = c->cfg.pop;
  h.stride = c->nd.stride;
  h.seed = c->cfg.seed;
  char* p = (char*)host_buf;
  memcpy(p, &h, sizeof h);
  p += sizeof h;
  const size_t gbytes = (size_t)c->cfg.pop * c->nd.stride * 4;
  const size_t sbytes = (size_t)c->cfg.pop * 4;
  leea_status st = dev(c, hipStreamSynchronize(c->stream), "sync before save");
  if (!st) st = dev(c, hipMemcpy(p, c->genomes[c->cur], gbytes, hipMemcpyDeviceToHost), "save");
  p += gbytes;
  const float* arr[5] = {c->f_adj, c->f_raw, c->acc, c->f_inh, c->sig[c->cur]};
  for (int i = 0; i < 5 && !st; ++i) {
    st = dev(c, hipMemcpy(p, arr[i], sbytes, hipMemcpyDeviceToHost), "save");
    p += sbytes;
  }
  return st;
}

leea_status leea_load(leea_ctx* c, const void* host_buf, size_t bytes) {
  if (!c || !host_buf) return fail(c, LEEA_EINVAL, "NULL argument");
  size_t need;
  leea_state_bytes(c, &need);
  if (bytes < need) return fail(c, LEEA_EINVAL, "checkpoint buffer too small");
  CkptHeader h;
  memcpy(&h, host_buf, sizeof h);
  if (h.magic != kStateMagic || h.version != kStateVersion)
    return fail(c, LEEA_EINVAL, "not a LEEA checkpoint");
  if (h.pop != c->cfg.pop || h.stride != c->nd.stride || h.seed != c->cfg.seed)
    return fail(c, LEEA_EINVAL, "checkpoint does not match this configuration");
  if (h.state > kSelected) return fail(c, LEEA_EINVAL, "corrupt checkpoint state");
  const char* p = (const char*)host_buf + sizeof h;
  const size_t gbytes = (size_t)c->cfg.pop * c->nd.stride * 4;
  const size_t sbytes = (size_t)c->cfg.pop * 4;
  leea_status st = dev(c, hipStreamSynchronize(c->stream), "sync before load");
  if (!st) st = dev(c, hipMemcpy(c->genomes[c->cur], p, gbytes, hipMemcpyHostToDevice), "load");
  p += gbytes;
  float* arr[5] = {c->f_adj, c->f_raw, c->acc, c->f_inh, c->sig[c->cur]};
  for (int i = 0; i < 5 && !st; ++i) {
    st = dev(c, hipMemcpy(arr[i], p, sbytes, hipMemcpyHostToDevice), "load");
    p += sbytes;
  }
  if (st) return st;
  c->wsh_ok = 0;
  c->w8_ok = 0;
  c->gen = h.gen;
  // a checkpoint taken between select and crossover_mutate resumes at select
  c->state = h.state == kSelected ? kEvaluated : (int)h.state;
  c->has_inh = (int)h.has_inh;
  c->sigma = h.sigma;
  return LEEA_OK;
}

const char* leea_last_error(const leea_ctx* c) { return c ? c->err.c_str() : g_err; }

void leea_destroy(leea_ctx* c) { delete c; }

leea_status leea_pool2x2(const float* x, int64_t n, int32_t side, float* out, void* hip_stream) {
  if (!x || !out || n < 0 || side < 2 || side % 2 != 0 || side > 4096)
    return fail(nullptr, LEEA_EINVAL, "bad arguments");
  if (n == 0) return LEEA_OK;
  return dev(nullptr, launch_pool2x2(x, n, side, out, (hipStream_t)hip_stream), "pool2x2");
}

leea_status leea_rng_philox(const uint32_t* ctr, uint64_t key, uint32_t* out, int64_t n,
                            void* hip_stream) {
  if (!ctr || !out || n < 0) return fail(nullptr, LEEA_EINVAL, "bad arguments");
  if (n == 0) return LEEA_OK;
  return dev(nullptr, launch_rng_philox(ctr, key, out, n, (hipStream_t)hip_stream), "philox");
}

leea_status leea_rng_ln32(const float* u, float* out, int64_t n, void* hip_stream) {
  if (!u || !out || n < 0) return fail(nullptr, LEEA_EINVAL, "bad arguments");
  if (n == 0) return LEEA_OK;
  return dev(nullptr, launch_rng_ln32(u, out, n, (hipStream_t)hip_stream), "ln32");
}

leea_status leea_rng_normal_pairs(const uint32_t* ab, float* z, int64_t n, void* hip_stream) {
  if (!ab || !z || n < 0) return fail(nullptr, LEEA_EINVAL, "bad arguments");
  if (n == 0) return LEEA_OK;
  return dev(nullptr, launch_rng_normal_pairs(ab, z, n, (hipStream_t)hip_stream), "normal");
}

// ------------------------------------------------------ fitness surrogate --

}  // extern "C"

namespace {

constexpr int kSurFeat = 256, kSurHid = 64, kSurIn = 259, kSurLd = 260;
constexpr int kSurParams = kSurHid * kSurIn + 2 * kSurHid + 1;

struct SurCarve {
  int M, N, kc, nc, ngroups, nchunks, splits;
  size_t cand, cplan, m4, nu, part, feat, n4, bits, prm, grad, pre, st, total;
};

leea_status sur_carve(const leea_config* cfg, const leea_surrogate_config* sc, const NetDesc& nd,
                      SurCarve* o) {
  if (!sc) return fail(nullptr, LEEA_EINVAL, "surrogate config is NULL");
  if (sc->oversample < 1 || sc->oversample > 64)
    return fail(nullptr, LEEA_EINVAL, "oversample must be in 1..64");
  if (sc->steps < 0 || sc->steps > 1000) return fail(nullptr, LEEA_EINVAL, "steps must be in 0..1000");
  if (!(sc->lr >= 0.0f && sc->lr < 1e6f)) return fail(nullptr, LEEA_EINVAL, "lr must be finite, >= 0");
  if (sc->warmup < 0) return fail(nullptr, LEEA_EINVAL, "warmup must be >= 0");
  if (!(sc->tau_min >= -1.0f && sc->tau_min <= 1.0f))
    return fail(nullptr, LEEA_EINVAL, "tau_min must be in [-1, 1]");
  if (cfg->sigma_mode == LEEA_SIGMA_SELF_ADAPTIVE)
    return fail(nullptr, LEEA_EINVAL, "the surrogate does not support self-adaptive sigma");
  SurCarve c;
  c.N = cfg->pop - cfg->n_elite;
  c.nc = cfg->n_cross;
  c.kc = sc->oversample * cfg->n_cross;
  c.M = sc->oversample * c.N;
  if (c.N < 1) return fail(nullptr, LEEA_EINVAL, "the surrogate needs non-elite slots");
  if (c.M > 8192) return fail(nullptr, LEEA_EINVAL, "oversample * (pop - n_elite) must be <= 8192");
  c.ngroups = (int)((nd.stride + 8191) / 8192);
  c.nchunks = (int)((nd.genes + 31) / 32);
  const int tiles = (c.M + 63) / 64;
  c.splits = (512 + tiles - 1) / tiles;
  if (c.splits > c.nchunks) c.splits = c.nchunks;
  if (c.splits < 1) c.splits = 1;
  c.cand = align256((size_t)c.M * nd.stride * 4);
  c.cplan = align256((size_t)c.M * 16);
  c.m4 = align256((size_t)c.M * 4);
  c.nu = align256((size_t)c.M * c.ngroups * 4);
  c.part = align256((size_t)c.splits * c.M * kSurFeat * 4);
  c.feat = align256((size_t)c.M * kSurLd * 4);
  c.n4 = align256((size_t)c.N * 4);
  c.bits = align256((size_t)c.nchunks * kSurFeat * 4);
  c.prm = align256((size_t)kSurParams * 4);
  c.grad = align256((size_t)mlp_grad_blocks(c.N) * (kSurParams + 1) * 4);
  c.pre = align256((size_t)c.N * kSurHid * 4);
  c.st = 256;
  c.total = c.cand + c.cplan + 2 * c.m4 + c.nu + c.part + 2 * c.feat + 4 * c.n4 + c.bits + c.prm +
            c.grad + c.pre + 2 * c.st;
  *o = c;
  return LEEA_OK;
}

}  // namespace

extern "C" {

leea_status leea_surrogate_workspace_bytes(const leea_config* cfg,
                                           const leea_surrogate_config* sc, size_t* bytes) {
  NetDesc nd;
  leea_status st = validate(cfg, &nd);
  if (st) return st;
  if (!bytes) return fail(nullptr, LEEA_EINVAL, "bytes is NULL");
  SurCarve c;
  st = sur_carve(cfg, sc, nd, &c);
  if (st) return st;
  *bytes = c.total;
  return LEEA_OK;
}

leea_status leea_surrogate_attach(leea_ctx* c, const leea_surrogate_config* sc, void* workspace,
                                  size_t bytes) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  SurCarve v;
  leea_status st = sur_carve(&c->cfg, sc, c->nd, &v);
  if (st) return fail(c, st, "%s", leea_last_error(nullptr));
  if (!workspace || ((uintptr_t)workspace & 255u))
    return fail(c, LEEA_EINVAL, "workspace must be a 256-byte aligned device pointer");
  if (bytes < v.total) return fail(c, LEEA_ENOMEM, "workspace smaller than leea_surrogate_workspace_bytes");
  char* p = (char*)workspace;
  c->sc = *sc;
  c->sM = v.M;
  c->sN = v.N;
  c->skc = v.kc;
  c->snc = v.nc;
  c->sngroups = v.ngroups;
  c->snchunks = v.nchunks;
  c->ssplits = v.splits;
  c->scand = (float*)p;
  p += v.cand;
  c->scplan = (int4*)p;
  p += v.cplan;
  c->scf_inh = (float*)p;
  p += v.m4;
  c->spred = (float*)p;
  p += v.m4;
  c->snu = (float*)p;
  p += v.nu;
  c->spart = (float*)p;
  p += v.part;
  c->sfeat = (float*)p;
  p += v.feat;
  c->szfeat = (float*)p;
  p += v.feat;
  c->sytgt = (float*)p;
  p += v.n4;
  c->schosen = (int32_t*)p;
  p += v.n4;
  c->schosen_pred = (float*)p;
  p += v.n4;
  c->spred_t = (float*)p;
  p += v.n4;
  c->sbits = (uint32_t*)p;
  p += v.bits;
  c->sprm = (float*)p;
  p += v.prm;
  c->sgrad = (float*)p;
  p += v.grad;
  c->spre = (float*)p;
  p += v.pre;
  c->sstate = (int32_t*)p;
  p += v.st;
  c->sstats = (float*)p;
  const float a1 = (float)sqrt(6.0 / (kSurIn + kSurHid));
  const float a2 = (float)sqrt(6.0 / (kSurHid + 1));
  st = dev(c, launch_proj_bits(c->sbits, v.nchunks, key_of(c), c->stream), "projection bits");
  if (!st) st = dev(c, launch_mlp_init(c->sprm, key_of(c), a1, a2, c->stream), "surrogate init");
  if (!st) st = dev(c, launch_fill((float*)c->sstate, 64, 0.0f, c->stream), "surrogate state");
  if (!st) st = dev(c, launch_fill(c->sstats, 64, 0.0f, c->stream), "surrogate stats");
  if (st) return st;
  c->sur = 1;
  return LEEA_OK;
}

leea_status leea_surrogate_step(leea_ctx* c, const float* x, const int32_t* y, int32_t b,
                                float* f_adj, float* f_raw, float* acc, float* stats) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (!c->sur) return fail(c, LEEA_ESTATE, "no surrogate attached");
  if (c->state != kEvaluated) return fail(c, LEEA_ESTATE, "surrogate step needs an evaluated population");
  leea_status st = check_batch(c, x, y, b);
  if (st) return st;
  st = leea_select(c, nullptr, nullptr, nullptr);
  if (st) return st;
  const leea_config& g = c->cfg;
  const uint32_t gen = c->gen + 1;
  float sigma;
  const float* sig_cur;
  float* sig_next;
  vary_sigma(c, gen, &sigma, &sig_cur, &sig_next);
  const float scale = (float)(1.0 / sqrt((double)c->nd.genes));
  hipStream_t s = c->stream;
  st = dev(c, launch_cand_plan(c->order, c->f_adj, c->sM, c->skc, g.pop, g.n_trunc, g.selection,
                               g.tournament_k, key_of(c), gen, c->scplan, c->scf_inh, s),
           "candidate plan");
  if (!st)
    st = dev(c, launch_vary_cand(c->genomes[c->cur], c->scand, c->scplan, c->nd, c->sM,
                                 g.crossover, sigma, g.mut_threshold, key_of(c), gen,
                                 (uint32_t)g.pop, c->snu, s),
             "candidate variation");
  if (!st)
    st = dev(c, launch_proj(c->scand, c->nd.stride, c->sM, c->sbits, c->snchunks, c->ssplits,
                            c->spart, s),
             "projection");
  if (!st)
    st = dev(c, launch_features(c->spart, c->ssplits, c->sM, c->snu, c->sngroups, c->scplan,
                                c->f_adj, scale, c->sfeat, s),
             "features");
  if (!st) st = dev(c, launch_standardize(c->sfeat, c->sM, c->szfeat, s), "standardise");
  if (!st)
    st = dev(c, launch_mlp_forward(c->sprm, c->szfeat, nullptr, c->sM, nullptr, c->spred, s),
             "prediction");
  if (!st)
    st = dev(c, launch_screen(c->spred, c->sM, c->sN, c->snc, c->skc, c->sstate, c->schosen,
                              c->schosen_pred, s),
             "screening");
  if (!st)
    st = dev(c, launch_gather(c->genomes[c->cur], c->scand, c->genomes[c->cur ^ 1], c->nd.stride,
                              g.pop, g.n_elite, c->plan, c->schosen, c->f_adj, c->scf_inh,
                              c->f_inh_next, s),
             "gather");
  if (st) return st;
  c->wsh_ok = 0;  // the new population came from the candidates
  c->w8_ok = 0;
  advance(c);
  st = run_eval(c, x, y, b, true, f_adj, f_raw, acc);
  if (st) return st;
  c->state = kEvaluated;
  const float* yk = c->f_raw + g.n_elite;
  st = dev(c, launch_targets(yk, c->sN, c->sytgt, s), "training targets");
  if (!st)
    st = dev(c, launch_surrogate_judge(c->schosen_pred, yk, c->sytgt, c->sN, c->sc.warmup,
                                       c->sc.tau_min, c->sstate, c->sstats, stats, s),
             "surrogate judge");
  for (int k = 0; k < c->sc.steps && !st; ++k)
    st = dev(c, launch_mlp_train_step(c->sprm, c->szfeat, c->schosen, c->sN, c->sytgt, c->spre,
                                      c->spred_t, c->sgrad, c->sc.lr, s),
             "surrogate training");
  return st;
}

leea_status leea_surrogate_views(leea_ctx* c, float** candidates, int32_t** plan,
                                 float** features, float** inputs, float** pred, int32_t** chosen,
                                 float** chosen_pred, float** params, int32_t* n_candidates) {
  if (!c) return fail(nullptr, LEEA_EINVAL, "ctx is NULL");
  if (!c->sur) return fail(c, LEEA_ESTATE, "no surrogate attached");
  if (candidates) *candidates = c->scand;
  if (plan) *plan = (int32_t*)c->scplan;
  if (features) *features = c->sfeat;
  if (inputs) *inputs = c->szfeat;
  if (pred) *pred = c->spred;
  if (chosen) *chosen = c->schosen;
  if (chosen_pred) *chosen_pred = c->schosen_pred;
  if (params) *params = c->sprm;
  if (n_candidates) *n_candidates = c->sM;
  return LEEA_OK;
}

}  // extern "C"

// ------------------------------------------- scoring without allocation --
// leea_score_noalloc keeps the per-network partial sums of the evaluation in
// this array instead of a workspace.  Each device holds its own copy; host
// code reaches it only through the address hipGetSymbolAddress returns for
// that device (the array's name is not a device address on the host side).

namespace {

constexpr size_t kScratchPartials = LEEA_NOALLOC_SCRATCH_BYTES / sizeof(float2);
constexpr int kScratchDevices = 64;

std::mutex g_scratch_mu;
float2* g_scratch_ptr[kScratchDevices];  // per device, filled on first use

}  // namespace

static __device__ __align__(256) float2 scratch[kScratchPartials];

namespace {

// Device address of the current device's scratch array (looked up once per
// device, with that device current).
leea_status current_scratch(float2** out) {
  int d = -1;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return dev(nullptr, e, "hipGetDevice");
  if (d < 0 || d >= kScratchDevices) return fail(nullptr, LEEA_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[d]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return dev(nullptr, e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(nullptr, LEEA_EDEVICE, "scratch array has no device address");
    g_scratch_ptr[d] = (float2*)p;
  }
  *out = g_scratch_ptr[d];
  return LEEA_OK;
}

}  // namespace

extern "C" leea_status leea_score_noalloc(const leea_config* cfg, const float* genomes,
                                          int64_t stride, const float* x, const int32_t* y,
                                          int32_t n, float* f_raw, float* acc,
                                          void* hip_stream) {
  NetDesc nd;
  leea_status st = validate(cfg, &nd);
  if (st) return st;
  if (cfg->eval_dtype != LEEA_DT_F32)
    return fail(nullptr, LEEA_EINVAL, "leea_score_noalloc evaluates a float32 first layer only");
  if (!genomes || !aligned16(genomes))
    return fail(nullptr, LEEA_EINVAL, "genomes must be a 16-byte aligned device pointer");
  if (stride != nd.stride) return fail(nullptr, LEEA_EINVAL, "stride does not match the widths");
  if (!x || !y) return fail(nullptr, LEEA_EINVAL, "x and y must be device pointers");
  if (!aligned16(x)) return fail(nullptr, LEEA_EINVAL, "x must be 16-byte aligned");
  if (n < 1 || n > LEEA_MAX_BATCH) return fail(nullptr, LEEA_EINVAL, "n must be in 1..65536");
  const int n_mt = eval_mtiles(nd, n);
  if ((size_t)cfg->pop * (size_t)n_mt > kScratchPartials)
    return fail(nullptr, LEEA_EINVAL,
                "pop * ceil(n / 64) exceeds the scratch of leea_score_noalloc (131072 partials)");
  float2* part = nullptr;
  st = current_scratch(&part);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  // every partial the finish reads is written by this call's evaluation
  // first, so nothing needs clearing
  const FinArgs fin{nullptr, nullptr, nullptr, nullptr, nullptr, f_raw, acc, 1.0f, 0, 1};
  bool finalized = false;
  st = dev(nullptr, launch_evaluate(genomes, nd, cfg->pop, x, y, n, part, s, &fin, &finalized),
           "evaluate launch");
  if (st || finalized) return st;
  return dev(nullptr, launch_finalize(part, cfg->pop, n_mt, n, nullptr, 0, 1.0f, nullptr, nullptr,
                                      nullptr, nullptr, f_raw, acc, s),
             "finalize launch");
}
