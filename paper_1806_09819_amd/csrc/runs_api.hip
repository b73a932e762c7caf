// C ABI of many independent EA runs driven together (leea_runs_*; contract
// in include/leea.h).  Every phase of a generation is one grouped launch
// over all runs (evaluation: one launch per kernel class), the per-run
// descriptors and the shared generation state live in device memory, and
// the whole generation is captured once into a hipGraph that every later
// generation replays.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/leea.h"
#include "runs.hpp"

using namespace leea;

namespace {

thread_local std::string g_runs_err;

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// Host copy of one run's layout (offsets into the workspace).
struct RunHost {
  leea_config cfg;
  NetDesc nd;
  size_t base;   // workspace offset of the run's region
  size_t bytes;  // region size
};

struct EvalClass {
  int kind, nt, mw, dt, rt;
  std::vector<int> runs;
};

// The large-batch kernels' tail and staging for one run: 0 the LDS-tile
// epilogue, 1 the register tail, 2 the register tail on the float32 kernel
// with global -> LDS staging (bitwise equal to 1 with register staging).
int eval_tail_kind(int kind, int dt, const NetDesc& nd, int b, int mw, const float* xb) {
  if ((kind != 1 && kind != 2) || !large_reg_tail(nd)) return 0;
  return kind == 1 && dt == 0 && eval_lfw_supported(nd, b, mw, xb) ? 2 : 1;
}

}  // namespace

struct leea_runs {
  int n;
  hipStream_t stream;
  char* ws;
  std::vector<RunHost> host;
  std::vector<RunDesc> desc;     // host mirror of the device descriptors
  RunDesc* d_desc;
  BatchState* d_state;
  int* d_tables;                 // group offsets and ids
  size_t table_ints;
  // groups
  Group g_draw, g_select, g_vary, g_quant, g_final;
  std::vector<EvalClass> classes;
  std::vector<Group> g_eval;
  bool any_lp;
  // generation bookkeeping (all runs advance together)
  uint32_t gen;
  bool evaluated;
  // graphs
  bool use_graph;
  hipGraphExec_t exec0, exec1;
  const void* gx_train;
  const void* gy_train;
  int64_t gn_train;
  std::string err;
};

namespace {

leea_status rfail(leea_runs* m, leea_status st, const std::string& msg) {
  if (m)
    m->err = msg;
  else
    g_runs_err = msg;
  return st;
}

leea_status rdev(leea_runs* m, hipError_t e, const char* what) {
  if (e == hipSuccess) return LEEA_OK;
  return rfail(m, LEEA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

uint32_t multiplier(int pop) {
  if (pop <= 1) return 1u;
  uint32_t mul = (uint32_t)(pop * 0.6180339887) | 1u;
  auto gcd = [](uint32_t a, uint32_t b) {
    while (b) {
      const uint32_t t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  while (gcd(mul, (uint32_t)pop) != 1u) ++mul;
  return mul;
}

// Validation of one run's config through the single-run entry point, plus
// the restrictions of grouped runs.
leea_status check_run(const leea_config* c, NetDesc* nd) {
  int64_t genes = 0, stride = 0;
  leea_status st = leea_param_count(c, &genes, &stride);
  if (st) return rfail(nullptr, st, std::string("run config: ") + leea_last_error(nullptr));
  if (c->sigma_mode != LEEA_SIGMA_CONSTANT)
    return rfail(nullptr, LEEA_EINVAL, "grouped runs use a constant sigma");
  if (c->eval_dtype == LEEA_DT_FP8)
    return rfail(nullptr, LEEA_EINVAL, "grouped runs evaluate in float32 or bfloat16");
  if (c->input_pool != 0) return rfail(nullptr, LEEA_EINVAL, "grouped runs do not pool inputs");
  memset(nd, 0, sizeof *nd);
  nd->L = c->n_layers;
  int64_t off = 0;
  for (int l = 0; l <= nd->L; ++l) nd->w[l] = c->widths[l];
  for (int l = 0; l < nd->L; ++l) {
    nd->woff[l] = off;
    off += (int64_t)nd->w[l + 1] * nd->w[l];
    nd->boff[l] = off;
    off += nd->w[l + 1];
  }
  nd->genes = off;
  nd->stride = stride;
  return LEEA_OK;
}

// Region of one run: genomes x2, f_adj, f_raw, acc, f_inh x2, plan,
// partial, batch x / y, quantised batch.
size_t run_bytes(const leea_config& c, const NetDesc& nd) {
  const size_t P = (size_t)c.pop;
  const int b = c.max_batch;
  const int kp = (nd.w[0] + 31) & ~31;
  size_t s = 2 * a256(P * (size_t)nd.stride * 4);
  s += 5 * a256(P * 4);
  s += a256(P * 16);
  s += a256(P * (size_t)((b + 15) / 16) * 8);
  s += a256((size_t)b * nd.w[0] * 4) + a256((size_t)b * 4);
  const size_t qrow = std::max((size_t)nd.w[0] * 4, (size_t)kp * 2);
  s += a256((size_t)b * qrow);
  return s;
}

constexpr size_t kTableInts = 1 << 16;

size_t total_bytes(const std::vector<RunHost>& h) {
  size_t s = 0;
  for (const auto& r : h) s += r.bytes;
  s += a256(sizeof(RunDesc) * h.size()) + a256(sizeof(BatchState)) + a256(kTableInts * 4);
  return s;
}

bool shape_of(const RunHost& h, int kind, int mw, EvalShape* sh) {
  if (h.cfg.eval_dtype == LEEA_DT_F32) return eval_shape_f32(h.nd, h.cfg.max_batch, kind, mw, sh);
  return eval_shape_lp(h.nd, h.cfg.max_batch, h.cfg.eval_dtype, kind, mw, sh);
}

void apply_shape(RunDesc& d, const EvalShape& sh) {
  d.ekind = sh.kind;
  d.emw = sh.mw;
  d.n_wt = sh.n_wt;
  d.n_pt = sh.n_pt;
  d.pass_rows = sh.pass_rows;
  d.tail_vec = sh.tail_vec;
  d.lo = sh.lo;
}

// Rebuild every launch group (block offsets, run ids, LDS) and upload the
// descriptors and tables.  Invalidates captured graphs.
leea_status build_groups(leea_runs* m) {
  std::vector<int> tab;
  auto add_group = [&](const std::vector<int>& ids, const std::vector<int>& blocks, size_t lds,
                       Group* g) {
    const size_t o = tab.size();
    int acc = 0;
    for (size_t i = 0; i < ids.size(); ++i) {
      tab.push_back(acc);
      acc += blocks[i];
    }
    tab.push_back(acc);
    const size_t o_ids = tab.size();
    for (int id : ids) tab.push_back(id);
    g->off = m->d_tables + o;
    g->ids = m->d_tables + o_ids;
    g->n = (int)ids.size();
    g->blocks = acc;
    g->lds = lds;
  };
  std::vector<int> all(m->n), b_draw(m->n), b_vary(m->n), b_fin(m->n);
  size_t sel_lds = 16;
  std::vector<int> q_ids, q_blocks;
  for (int r = 0; r < m->n; ++r) {
    const RunDesc& d = m->desc[r];
    all[r] = r;
    b_draw[r] = d.b;
    b_vary[r] = d.vgx * d.pop;
    b_fin[r] = (d.pop + 255) / 256;
    sel_lds = std::max(sel_lds, (size_t)d.n2 * 8);
    if (d.dt == LEEA_DT_BF16) {
      const int64_t items = (d.ekind == 0 || d.ekind == 4) ? (int64_t)d.b * d.nd.w[0] : (int64_t)d.b * (d.kp >> 3);
      q_ids.push_back(r);
      q_blocks.push_back((int)((items + 255) / 256));
    }
  }
  add_group(all, b_draw, 0, &m->g_draw);
  add_group(all, std::vector<int>(m->n, 1), sel_lds, &m->g_select);
  add_group(all, b_vary, 0, &m->g_vary);
  add_group(all, b_fin, 0, &m->g_final);
  m->any_lp = !q_ids.empty();
  if (m->any_lp) add_group(q_ids, q_blocks, 0, &m->g_quant);
  // evaluation classes
  std::map<std::tuple<int, int, int, int, int>, std::vector<int>> cls;
  for (int r = 0; r < m->n; ++r) {
    const RunDesc& d = m->desc[r];
    const int nt = (d.nd.w[1] + 15) / 16;
    const int mw = d.ekind == 0 ? 1 : d.emw;
    const int rt = eval_tail_kind(d.ekind, d.dt, d.nd, d.b, mw, d.xb);
    cls[std::make_tuple(d.ekind, nt, mw, d.dt, rt)].push_back(r);
  }
  m->classes.clear();
  m->g_eval.clear();
  for (auto& kv : cls) {
    EvalClass ec;
    std::tie(ec.kind, ec.nt, ec.mw, ec.dt, ec.rt) = kv.first;
    ec.runs = kv.second;
    std::vector<int> blocks;
    size_t lds = 0;
    for (int r : ec.runs) {
      const RunDesc& d = m->desc[r];
      blocks.push_back(d.ekind == 0 ? d.pop : d.n_wt * d.pop);
      EvalShape sh;
      shape_of(m->host[r], d.ekind, d.emw, &sh);
      lds = std::max(lds, sh.lds);
    }
    Group g;
    add_group(ec.runs, blocks, lds, &g);
    m->classes.push_back(ec);
    m->g_eval.push_back(g);
  }
  if (tab.size() > kTableInts - 8)  // the last 8 entries are the autotuner's
    return rfail(m, LEEA_EINVAL, "too many runs for the launch tables");
  leea_status st = rdev(m, hipMemcpyAsync(m->d_tables, tab.data(), tab.size() * 4,
                                          hipMemcpyHostToDevice, m->stream), "table upload");
  if (!st)
    st = rdev(m, hipMemcpyAsync(m->d_desc, m->desc.data(), sizeof(RunDesc) * m->n,
                                hipMemcpyHostToDevice, m->stream), "descriptor upload");
  if (!st) st = rdev(m, hipStreamSynchronize(m->stream), "upload sync");
  if (m->exec0) hipGraphExecDestroy(m->exec0);
  if (m->exec1) hipGraphExecDestroy(m->exec1);
  m->exec0 = m->exec1 = nullptr;
  return st;
}

// The launches of one generation (step = 0: initial evaluation; 1: select,
// vary, advance, evaluate).
leea_status enqueue(leea_runs* m, int step, const float* x, const int32_t* y, int64_t n_train) {
  hipStream_t s = m->stream;
  leea_status st = rdev(m, launch_runs_draw(m->d_desc, m->d_state, m->g_draw, x, y, n_train, step, s),
                        "grouped draw");
  if (!st && step) {
    st = rdev(m, launch_runs_select(m->d_desc, m->d_state, m->g_select, s), "grouped select");
    if (!st) st = rdev(m, launch_runs_vary(m->d_desc, m->d_state, m->g_vary, s), "grouped vary");
    if (!st) st = rdev(m, launch_runs_advance(m->d_state, s), "advance");
  }
  if (!st && m->any_lp)
    st = rdev(m, launch_runs_quantize(m->d_desc, m->g_quant, s), "grouped quantize");
  for (size_t c = 0; c < m->classes.size() && !st; ++c) {
    const EvalClass& ec = m->classes[c];
    st = rdev(m, launch_runs_eval(ec.kind, ec.nt, ec.mw, ec.dt, ec.rt, m->d_desc, m->d_state,
                                  m->g_eval[c], s),
              "grouped evaluate");
  }
  if (!st) st = rdev(m, launch_runs_finalize(m->d_desc, m->d_state, m->g_final, s), "grouped finalize");
  return st;
}

leea_status capture(leea_runs* m, int step, const float* x, const int32_t* y, int64_t n_train,
                    hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  leea_status st = rdev(m, hipStreamBeginCapture(m->stream, hipStreamCaptureModeRelaxed),
                        "begin capture");
  if (st) return st;
  leea_status st2 = enqueue(m, step, x, y, n_train);
  hipError_t e = hipStreamEndCapture(m->stream, &graph);
  if (st2) {
    if (graph) hipGraphDestroy(graph);
    return st2;
  }
  st = rdev(m, e, "end capture");
  if (st) return st;
  st = rdev(m, hipGraphInstantiate(out, graph, nullptr, nullptr, 0), "graph instantiate");
  hipGraphDestroy(graph);
  return st;
}

}  // namespace

extern "C" {

leea_status leea_runs_workspace_bytes(const leea_config* cfgs, int32_t n, size_t* bytes) {
  if (!cfgs || !bytes || n < 1 || n > LEEA_MAX_RUNS)
    return rfail(nullptr, LEEA_EINVAL, "need 1..LEEA_MAX_RUNS configs and an output");
  std::vector<RunHost> h(n);
  for (int r = 0; r < n; ++r) {
    leea_status st = check_run(&cfgs[r], &h[r].nd);
    if (st) return st;
    h[r].cfg = cfgs[r];
    h[r].bytes = run_bytes(cfgs[r], h[r].nd);
  }
  *bytes = total_bytes(h);
  return LEEA_OK;
}

leea_status leea_runs_create(const leea_config* cfgs, int32_t n, void* workspace, size_t bytes,
                             void* hip_stream, leea_runs** out) {
  if (!out) return rfail(nullptr, LEEA_EINVAL, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  leea_status st = leea_runs_workspace_bytes(cfgs, n, &need);
  if (st) return st;
  if (!workspace || ((uintptr_t)workspace & 255u))
    return rfail(nullptr, LEEA_EINVAL, "workspace must be a 256-byte aligned device pointer");
  if (bytes < need) return rfail(nullptr, LEEA_ENOMEM, "workspace smaller than leea_runs_workspace_bytes");
  if (!hip_stream) return rfail(nullptr, LEEA_EINVAL, "grouped runs need a non-default stream");
  leea_runs* m = new (std::nothrow) leea_runs();
  if (!m) return rfail(nullptr, LEEA_ENOMEM, "host allocation failed");
  m->n = n;
  m->stream = (hipStream_t)hip_stream;
  m->ws = (char*)workspace;
  m->host.resize(n);
  m->desc.resize(n);
  m->exec0 = m->exec1 = nullptr;
  m->use_graph = true;
  m->gen = 0;
  m->evaluated = false;
  m->gx_train = m->gy_train = nullptr;
  m->gn_train = 0;
  size_t off = 0;
  for (int r = 0; r < n; ++r) {
    RunHost& h = m->host[r];
    check_run(&cfgs[r], &h.nd);
    h.cfg = cfgs[r];
    h.bytes = run_bytes(cfgs[r], h.nd);
    h.base = off;
    off += h.bytes;
    const leea_config& c = h.cfg;
    const size_t P = (size_t)c.pop;
    char* p = m->ws + h.base;
    RunDesc& d = m->desc[r];
    memset(&d, 0, sizeof d);
    d.nd = h.nd;
    d.genomes[0] = (float*)p;
    p += a256(P * (size_t)h.nd.stride * 4);
    d.genomes[1] = (float*)p;
    p += a256(P * (size_t)h.nd.stride * 4);
    d.f_adj = (float*)p;
    p += a256(P * 4);
    d.f_raw = (float*)p;
    p += a256(P * 4);
    d.acc = (float*)p;
    p += a256(P * 4);
    d.f_inh[0] = (float*)p;
    p += a256(P * 4);
    d.f_inh[1] = (float*)p;
    p += a256(P * 4);
    d.plan = (int4*)p;
    p += a256(P * 16);
    d.partial = (float2*)p;
    p += a256(P * (size_t)((c.max_batch + 15) / 16) * 8);
    d.xb = (float*)p;
    p += a256((size_t)c.max_batch * h.nd.w[0] * 4);
    d.yb = (int32_t*)p;
    p += a256((size_t)c.max_batch * 4);
    d.xq = p;
    d.key.k0 = (uint32_t)c.seed;
    d.key.k1 = (uint32_t)(c.seed >> 32);
    d.key.run = c.run;
    d.thr = c.mut_threshold;
    d.sigma = c.sigma;
    d.alpha = c.alpha;
    d.pop = c.pop;
    d.n_elite = c.n_elite;
    d.n_cross = c.n_cross;
    d.n_trunc = c.n_trunc;
    d.selection = c.selection;
    d.tk = c.tournament_k;
    d.crossover = c.crossover;
    d.b = c.max_batch;
    d.dt = c.eval_dtype;
    d.kp = (h.nd.w[0] + 31) & ~31;
    d.side = 0;
    d.mul = multiplier(c.pop);
    int n2 = 1;
    while (n2 < c.pop) n2 <<= 1;
    d.n2 = n2 < 2 ? 2 : n2;
    d.vgx = (int)((((h.nd.stride + 8191) / 8192) + 3) / 4);
    EvalShape sh;
    if (!shape_of(h, -1, 0, &sh)) {
      delete m;
      return rfail(nullptr, LEEA_EINVAL, "no evaluation shape for a run's widths and batch");
    }
    apply_shape(d, sh);
  }
  m->d_desc = (RunDesc*)(m->ws + off);
  off += a256(sizeof(RunDesc) * n);
  m->d_state = (BatchState*)(m->ws + off);
  off += a256(sizeof(BatchState));
  m->d_tables = (int*)(m->ws + off);
  BatchState s0 = {0u, 0, 0, 0};
  st = rdev(m, hipMemcpyAsync(m->d_state, &s0, sizeof s0, hipMemcpyHostToDevice, m->stream),
            "state upload");
  for (int r = 0; r < n && !st; ++r) {
    const leea_config& c = m->host[r].cfg;
    Glorot ga;
    for (int l = 0; l < LEEA_MAX_LAYERS; ++l) ga.a[l] = l < c.n_layers ? c.glorot_a[l] : 0.0f;
    st = rdev(m, launch_init(m->desc[r].genomes[0], m->host[r].nd, ga, c.pop, m->desc[r].key,
                             m->stream),
              "init launch");
  }
  if (!st) st = build_groups(m);
  if (st) {
    g_runs_err = m->err;
    delete m;
    return st;
  }
  *out = m;
  return LEEA_OK;
}

leea_status leea_runs_generation(leea_runs* m, const float* x_train, const int32_t* y_train,
                                 int64_t n_train) {
  if (!m) return rfail(nullptr, LEEA_EINVAL, "runs is NULL");
  if (!x_train || !y_train || ((uintptr_t)x_train & 15u))
    return rfail(m, LEEA_EINVAL, "x_train / y_train must be device pointers (x 16-byte aligned)");
  if (n_train < 1 || n_train > 0xFFFFFFFFll) return rfail(m, LEEA_EINVAL, "n_train out of range");
  const int step = m->evaluated ? 1 : 0;
  leea_status st;
  if (!m->use_graph) {
    st = enqueue(m, step, x_train, y_train, n_train);
  } else {
    if (m->gx_train != x_train || m->gy_train != y_train || m->gn_train != n_train) {
      if (m->exec0) hipGraphExecDestroy(m->exec0);
      if (m->exec1) hipGraphExecDestroy(m->exec1);
      m->exec0 = m->exec1 = nullptr;
      m->gx_train = x_train;
      m->gy_train = y_train;
      m->gn_train = n_train;
    }
    hipGraphExec_t* ex = step ? &m->exec1 : &m->exec0;
    st = LEEA_OK;
    if (!*ex) st = capture(m, step, x_train, y_train, n_train, ex);
    if (!st) st = rdev(m, hipGraphLaunch(*ex, m->stream), "graph launch");
  }
  if (st) return st;
  if (step) m->gen += 1;
  m->evaluated = true;
  return LEEA_OK;
}

leea_status leea_runs_set_graph(leea_runs* m, int32_t enable) {
  if (!m) return rfail(nullptr, LEEA_EINVAL, "runs is NULL");
  m->use_graph = enable != 0;
  return LEEA_OK;
}

leea_status leea_runs_generation_count(const leea_runs* m, uint32_t* gen) {
  if (!m || !gen) return rfail(nullptr, LEEA_EINVAL, "NULL argument");
  *gen = m->gen;
  return LEEA_OK;
}

leea_status leea_runs_population(leea_runs* m, int32_t r, float** genomes, int64_t* stride,
                                 float** f_adj, float** f_raw, float** acc) {
  if (!m) return rfail(nullptr, LEEA_EINVAL, "runs is NULL");
  if (r < 0 || r >= m->n) return rfail(m, LEEA_EINVAL, "run index out of range");
  const RunDesc& d = m->desc[r];
  const int cur = (int)(m->gen & 1u);
  if (genomes) *genomes = d.genomes[cur];
  if (stride) *stride = d.nd.stride;
  if (f_adj) *f_adj = d.f_adj;
  if (f_raw) *f_raw = d.f_raw;
  if (acc) *acc = d.acc;
  return LEEA_OK;
}

leea_status leea_runs_shape(const leea_runs* m, int32_t r, int32_t* kind, int32_t* mw) {
  if (!m || r < 0 || r >= m->n) return rfail(nullptr, LEEA_EINVAL, "bad arguments");
  if (kind) *kind = m->desc[r].ekind;
  if (mw) *mw = m->desc[r].emw;
  return LEEA_OK;
}

leea_status leea_runs_set_shape(leea_runs* m, int32_t r, int32_t kind, int32_t mw) {
  if (!m || r < 0 || r >= m->n) return rfail(nullptr, LEEA_EINVAL, "bad arguments");
  EvalShape sh;
  if (!shape_of(m->host[r], kind, mw, &sh))
    return rfail(m, LEEA_EINVAL, "that evaluation shape does not exist for this run");
  apply_shape(m->desc[r], sh);
  return build_groups(m);
}

// Autotuner: for every distinct (population, widths, batch, dtype) among
// the runs, time each evaluation shape that exists for it on that run's own
// batch (5 launches after 2 warm-ups, HIP events on the runs' stream) and
// give every run with that key the fastest.
leea_status leea_runs_autotune(leea_runs* m, const float* x_train, const int32_t* y_train,
                               int64_t n_train, int32_t* kind_out, int32_t* mw_out,
                               float* us_out) {
  if (!m) return rfail(nullptr, LEEA_EINVAL, "runs is NULL");
  if (!x_train || !y_train || n_train < 1) return rfail(m, LEEA_EINVAL, "bad training set");
  // a batch for every run (generation of the last draw; timing only)
  leea_status st = rdev(m, launch_runs_draw(m->d_desc, m->d_state, m->g_draw, x_train, y_train,
                                            n_train, 0, m->stream),
                        "grouped draw");
  if (st) return st;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return rfail(m, LEEA_EDEVICE, "event creation failed");
  std::map<std::vector<int64_t>, std::pair<EvalShape, float>> best;
  const int cands[7][2] = {{0, 1}, {3, 1}, {4, 1}, {1, 1}, {1, 2}, {2, 1}, {2, 2}};
  for (int r = 0; r < m->n && !st; ++r) {
    const RunHost& h = m->host[r];
    std::vector<int64_t> key = {h.cfg.pop, h.cfg.max_batch, h.cfg.eval_dtype, h.nd.L};
    for (int l = 0; l <= h.nd.L; ++l) key.push_back(h.nd.w[l]);
    auto it = best.find(key);
    if (it == best.end()) {
      EvalShape bsh;
      float bus = 1e30f;
      bool any = false;
      for (const auto& c : cands) {
        if (h.cfg.eval_dtype == LEEA_DT_F32 && c[0] == 2) continue;
        if (h.cfg.eval_dtype != LEEA_DT_F32 && (c[0] == 1 || c[0] == 3)) continue;
        if (h.cfg.eval_dtype == LEEA_DT_FP8 && c[0] == 4) continue;
        EvalShape sh;
        if (!shape_of(h, c[0], c[1], &sh)) continue;
        // a one-run group in this shape
        RunDesc d = m->desc[r];
        apply_shape(d, sh);
        st = rdev(m, hipMemcpyAsync(m->d_desc + r, &d, sizeof d, hipMemcpyHostToDevice, m->stream),
                  "descriptor upload");
        std::vector<int> tab = {0, sh.kind == 0 ? d.pop : d.n_wt * d.pop, r};
        if (!st)
          st = rdev(m, hipMemcpyAsync(m->d_tables + kTableInts - 3, tab.data(), 12,
                                      hipMemcpyHostToDevice, m->stream),
                    "table upload");
        if (st) break;
        Group g;
        g.off = m->d_tables + kTableInts - 3;
        g.ids = m->d_tables + kTableInts - 1;
        g.n = 1;
        g.blocks = tab[1];
        g.lds = sh.lds;
        if (d.dt == LEEA_DT_BF16) {
          const int64_t items = (sh.kind == 0 || sh.kind == 4) ? (int64_t)d.b * d.nd.w[0] : (int64_t)d.b * (d.kp >> 3);
          Group q = g;
          q.blocks = (int)((items + 255) / 256);
          std::vector<int> qt = {0, q.blocks};
          st = rdev(m, hipMemcpyAsync(m->d_tables + kTableInts - 3, qt.data(), 8,
                                      hipMemcpyHostToDevice, m->stream), "table upload");
          if (!st) st = rdev(m, launch_runs_quantize(m->d_desc, q, m->stream), "quantize");
          if (!st)
            st = rdev(m, hipMemcpyAsync(m->d_tables + kTableInts - 3, tab.data(), 8,
                                        hipMemcpyHostToDevice, m->stream), "table upload");
        }
        const int nt = (h.nd.w[1] + 15) / 16;
        for (int k = 0; k < 7 && !st; ++k) {
          if (k == 2) hipEventRecord(e0, m->stream);
          const int rt = eval_tail_kind(sh.kind, d.dt, h.nd, d.b, sh.kind == 0 ? 1 : sh.mw, d.xb);
          st = rdev(m, launch_runs_eval(sh.kind, nt, sh.kind == 0 ? 1 : sh.mw, d.dt, rt,
                                        m->d_desc, m->d_state, g, m->stream),
                    "evaluate");
        }
        hipEventRecord(e1, m->stream);
        if (!st) st = rdev(m, hipEventSynchronize(e1), "event sync");
        if (st) break;
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        const float us = ms * 1000.0f / 5.0f;
        if (us < bus) {
          bus = us;
          bsh = sh;
          any = true;
        }
      }
      if (st) break;
      if (!any) {
        st = rfail(m, LEEA_EINVAL, "no evaluation shape could be timed");
        break;
      }
      it = best.emplace(key, std::make_pair(bsh, bus)).first;
    }
    apply_shape(m->desc[r], it->second.first);
    if (kind_out) kind_out[r] = it->second.first.kind;
    if (mw_out) mw_out[r] = it->second.first.mw;
    if (us_out) us_out[r] = it->second.second;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  return build_groups(m);
}

const char* leea_runs_last_error(const leea_runs* m) {
  return m ? m->err.c_str() : g_runs_err.c_str();
}

void leea_runs_destroy(leea_runs* m) {
  if (!m) return;
  if (m->exec0) hipGraphExecDestroy(m->exec0);
  if (m->exec1) hipGraphExecDestroy(m->exec1);
  delete m;
}

}  // extern "C"
