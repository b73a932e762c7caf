/*
 * leea.h -- C ABI of the MI355X (gfx950) limited-evaluation evolutionary
 * algorithm library, libleea.so.
 *
 * The library runs one generation of the EA of Prellberg & Kramer,
 * "Limited Evaluation Evolutionary Optimization of Large Neural Networks"
 * (arXiv 1806.09819), Algorithm 1 of section 3.1, entirely on one GPU:
 * population-batched forward pass of P directly encoded MLPs on a shared
 * minibatch (section 3.3), softmax-cross-entropy fitness (Eq. 1) and accuracy,
 * fitness inheritance (section 3.1), rank + truncation or tournament
 * selection, uniform or arithmetic crossover and Gaussian mutation
 * (section 3.2).
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory.  Every pointer named "device" is caller-owned device memory (for
 *   example a torch tensor's data_ptr()).  The workspace given to
 *   leea_init_population holds the population and all per-individual state
 *   and must stay allocated until leea_destroy.  The ctx is a host object
 *   owned by the library.
 * Streams.  Every call enqueues work on the HIP stream given at init (a
 *   hipStream_t cast to void*, e.g. torch.cuda.current_stream().cuda_stream;
 *   NULL is the legacy default stream) and returns without synchronising,
 *   except leea_save / leea_load which synchronise that stream.
 * Errors.  Every call returns a leea_status and never aborts.  Argument and
 *   call-order checks happen on the host before anything is enqueued; a
 *   failed check leaves the state unchanged.  A launch failure or sticky
 *   device error returns LEEA_EDEVICE.  leea_last_error(ctx) gives a
 *   human-readable message of the last failure on that ctx;
 *   leea_last_error(NULL) that of the last failure of a call without a ctx.
 * Threads.  A ctx must not be used by two host threads at once; different
 *   ctxs are independent.
 * Call order.  init -> evaluate (generation 0) -> { select ->
 *   crossover_mutate -> evaluate }*, or step in place of the braces.
 *   Out-of-order calls return LEEA_ESTATE.
 * Genome layout.  Logical gene i of a network with widths n0..nL runs layer
 *   by layer: W_l as [n_l][n_{l-1}] row-major, then b_l.  The device stores
 *   individual j's genome at genomes + j*stride (floats), stride = the gene
 *   count rounded up to a multiple of 64; padding genes are zero.
 * Random numbers.  Philox4x32-10 (Salmon et al., SC'11) with key = seed and
 *   counter = (block, slot, generation, run << 8 | purpose); every draw of
 *   the method is a pure function of that counter, so results do not depend
 *   on launch shapes.
 */
#ifndef LEEA_H
#define LEEA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LEEA_MAX_LAYERS 8       /* weight layers */
#define LEEA_MAX_WIDTH 256      /* widest hidden or output layer */
#define LEEA_MAX_POP 8192       /* lambda; the rank kernel sorts in one workgroup */
#define LEEA_MAX_BATCH 65536

typedef struct leea_ctx leea_ctx;

typedef enum {
  LEEA_OK = 0,
  LEEA_EINVAL = 1,   /* bad argument or configuration */
  LEEA_ENOMEM = 2,   /* workspace too small, or host allocation failed */
  LEEA_EDEVICE = 3,  /* HIP launch or runtime error */
  LEEA_ESTATE = 4    /* call out of order */
} leea_status;

enum { LEEA_SEL_TRUNCATION = 0, LEEA_SEL_TOURNAMENT = 1 };
enum { LEEA_XO_UNIFORM = 0, LEEA_XO_ARITHMETIC = 1 };
enum { LEEA_OP_ELITE = 0, LEEA_OP_CROSSOVER = 1, LEEA_OP_MUTATION = 2 };
/* Mutation-strength control (section 3.2): constant; exponential decay
 * sigma_i = sigma * 0.99^(i/k) for the mutation that creates generation i
 * (computed on the host in double precision, rounded once to float); or
 * self-adaptive, where every individual carries a sigma gene (see
 * leea_crossover_mutate). */
enum { LEEA_SIGMA_CONSTANT = 0, LEEA_SIGMA_DECAY = 1, LEEA_SIGMA_SELF_ADAPTIVE = 2 };
/* Arithmetic of the forward pass (section 3.3): the weights of every layer
 * and the network's input, the batch, in the given format; the products
 * are summed in float32; biases, hidden activations, the fitness (Eq. 1)
 * and the genomes stay float32.  (Hidden activations are not rounded: they
 * are float32 sums whose last bits depend on the summation order.)
 * F32:  float32 operands (the paper's arithmetic).
 * BF16: X and every W_l rounded to bfloat16 (nearest, ties to even); the
 *       first layer on the bf16 matrix cores.
 * FP8:  OCP FP8 E4M3 with power-of-two scales, one per network and layer:
 *       X / 2^e_x and W_l / 2^e_l rounded to E4M3 (nearest, ties to even), e
 *       the smallest integer with B <= 448 * 2^e, each layer's sums
 *       multiplied by 2^(e_x + e_1) (first layer) or 2^e_l.  For the batch
 *       and for W_2 .. W_L, B is the largest |value|.  For each network's W_1
 *       B is its largest |value| after initialisation, leea_set_state,
 *       leea_load or a surrogate step, and for a child of crossover_mutate
 *       the bound its parents give (elite: the parent's largest |W_1|;
 *       crossover: the larger parent's; mutant: fl(fl(a * (1 + 2^-20)) +
 *       fl(6 * sigma)), a the parent's), which is known before the child is
 *       written, so that the variation kernel writes the child's FP8 copy of
 *       W_1 with it.  A batch holding NaN or an infinity gives every network a
 *       NaN fitness; such a weight gives its network a NaN fitness. */
enum { LEEA_DT_F32 = 0, LEEA_DT_BF16 = 1, LEEA_DT_FP8 = 2 };

/* Hyperparameters of one EA run.  Counts are integers: the paper's
 * fractions p_E*lambda, p_C*lambda, p_M*lambda and rho*lambda (Algorithm 1)
 * are rounded by leea_config_from_fractions (or by the caller);
 * n_elite + n_cross + n_mut must equal pop. */
typedef struct {
  int32_t n_layers;                       /* L >= 1 weight layers */
  int32_t widths[LEEA_MAX_LAYERS + 1];    /* widths[0] = input dim (multiple of 4),
                                             widths[L] = classes d; widths[1..L] <= 256 */
  int32_t pop;                            /* lambda, 1..LEEA_MAX_POP */
  int32_t n_elite, n_cross, n_mut;        /* offspring made by each operator */
  int32_t n_trunc;                        /* rho*lambda, 1..pop (truncation selection) */
  int32_t selection;                      /* LEEA_SEL_* */
  int32_t tournament_k;                   /* contestants, 1..16 (tournament only) */
  int32_t crossover;                      /* LEEA_XO_* */
  float sigma;                            /* mutation strength (section 3.2), >= 0 */
  float alpha;                            /* inheritance weight in [0,1]; 1 = off */
  uint64_t mut_threshold;                 /* gene mutated iff its 32-bit draw < this;
                                             4294967296 = every gene (the paper) */
  float glorot_a[LEEA_MAX_LAYERS];        /* Glorot-uniform bound of each layer (section 4.1) */
  uint64_t seed;                          /* Philox key */
  uint32_t run;                           /* run index in the Philox counter */
  int32_t max_batch;                      /* largest b passed to evaluate/step, 1..LEEA_MAX_BATCH */
  int32_t sigma_mode;                     /* LEEA_SIGMA_* */
  float sigma_decay_k;                    /* k > 0 of the decay schedule */
  float tau;                              /* self-adaptation rate in [0, 10]; 0 = 1/sqrt(genes) */
  int32_t input_pool;                     /* 0, or 2: draw_batch max-pools 2x2 from square images
                                             of 4*widths[0] pixels (section 4.1) */
  int32_t eval_dtype;                     /* LEEA_DT_*: arithmetic of the weights (BF16
                                             adds a bfloat16 copy of every W_1 to the
                                             workspace, FP8 an FP8 copy) */
} leea_config;

/* Host helper: fill the integer fields of cfg that Algorithm 1 writes as
 * fractions of lambda (section 3.1), from cfg->pop, cfg->n_layers and
 * cfg->widths, which the caller sets first:
 *   n_elite = floor(p_elite*pop + 1/2), n_cross = floor(p_cross*pop + 1/2),
 *   n_mut = pop - n_elite - n_cross (the three always sum to pop),
 *   n_trunc = floor(rho*pop + 1/2) clamped to [1, pop] (truncation, rho*lambda);
 * mut_threshold = floor(p_gene * 2^32) (a gene mutates iff its 32-bit draw is
 * below it; p_gene = 1 mutates every gene, the paper's operator); and each
 * layer's Glorot-uniform bound glorot_a[l] = sqrt(6 / (n_l + n_{l+1})) in
 * double, rounded once to float (section 4.1); glorot_a past the last layer
 * is zeroed.  All arithmetic is double precision on the host.  Fractions
 * outside [0, 1] or p_elite + p_cross + p_mut further than 1e-9 from 1 give
 * LEEA_EINVAL and leave cfg unchanged.  Touches no device. */
leea_status leea_config_from_fractions(leea_config* cfg, double p_elite, double p_cross,
                                       double p_mut, double rho, double p_gene);

/* Genes per network (c) and the padded per-individual stride in floats. */
leea_status leea_param_count(const leea_config* cfg, int64_t* genes, int64_t* stride);

/* Bytes of device workspace leea_init_population needs for cfg. */
leea_status leea_workspace_bytes(const leea_config* cfg, size_t* bytes);

/* Validate cfg, carve the workspace (device, >= leea_workspace_bytes, 256-byte
 * aligned) and write the initial population (Algorithm 1, first line):
 * Glorot-uniform weights, zero biases.  On success *out is a new ctx at
 * generation 0 that still needs its first evaluate. */
leea_status leea_init_population(const leea_config* cfg, void* workspace, size_t bytes,
                                 void* hip_stream, leea_ctx** out);

/* Draw generation gen's minibatch (Algorithm 1, "select random batch"): b
 * examples with replacement from x_train [n_train][row] / y_train
 * [n_train] (device) into x_out [b][widths[0]] / y_out [b] (device), where
 * row = widths[0], or 4*widths[0] pixels of a square image that is 2x2
 * max-pooled on the way when input_pool = 2 (NaN if any pooled pixel is NaN).
 * Example k is index floor(w * n_train / 2^32), w = word k&3 of Philox block
 * (BATCH, gen, slot 0, k>>2).  Valid in any state. */
leea_status leea_draw_batch(leea_ctx* ctx, uint32_t gen, const float* x_train,
                            const int32_t* y_train, int64_t n_train, int32_t b,
                            float* x_out, int32_t* y_out);

/* Evaluate the current population on the batch x [b][widths[0]], y [b]
 * (device; labels in [0, d)) (Algorithm 1, last line): logits through every
 * layer (ReLU on all but the last, section 4.1), fitness = mean log-softmax
 * of the true class (Eq. 1, left side), accuracy = share of argmax == y
 * (lowest class wins ties), then f_adj = (1-alpha) f_inh + alpha fitness
 * (section 3.1) once a selection has produced inherited values.  The three
 * outputs (device, [pop] floats each) may be NULL.  Labels outside [0, d)
 * give a NaN fitness for that network.  1 <= b <= max_batch; x must be
 * 16-byte aligned (LEEA_EINVAL otherwise: the kernels read it in 16-byte
 * pieces). */
leea_status leea_evaluate(leea_ctx* ctx, const float* x, const int32_t* y, int32_t b,
                          float* f_adj, float* f_raw, float* acc);

/* Fitness and accuracy of the current population on n examples without
 * touching the EA state (validation / test scoring).  1 <= n <= max_batch;
 * x 16-byte aligned as for leea_evaluate. */
leea_status leea_score(leea_ctx* ctx, const float* x, const int32_t* y, int32_t n,
                       float* f_raw, float* acc);

/* For callers that cannot allocate device memory or bring a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): leea_score without a ctx.  Fitness and accuracy (as
 * leea_score computes them, bit for bit) of the cfg->pop networks in genomes
 * (device, [pop][stride] floats in the layout above, 16-byte aligned; stride
 * must be the one leea_param_count gives; padding genes are not read) on n
 * examples x [n][widths[0]] (device, 16-byte aligned) and y [n] (device),
 * into f_raw and acc (device [pop], either may be NULL), enqueued on
 * hip_stream, which must belong to the current device.  Float32 first layer
 * only (cfg->eval_dtype = LEEA_DT_F32).
 * The per-network partial sums live in a static device array of
 * LEEA_NOALLOC_SCRATCH_BYTES per device (131072 float pairs), held by every
 * device the library runs on until the process ends: pop * ceil(n / 64)
 * must not exceed 131072 (pop * 1 for n <= 16), else LEEA_EINVAL.  The call
 * allocates nothing (the array's device address is looked up once per
 * device, on the first call with that device current).  Every call on a
 * device shares that device's array, so calls that overlap on one device
 * (different streams or host threads) race; calls ordered on one stream do
 * not.  Errors: leea_last_error(NULL). */
#define LEEA_NOALLOC_SCRATCH_BYTES (1 << 20)
leea_status leea_score_noalloc(const leea_config* cfg, const float* genomes, int64_t stride,
                               const float* x, const int32_t* y, int32_t n, float* f_raw,
                               float* acc, void* hip_stream);

/* Sort by adjusted fitness (descending; ties by slot, -0 == +0, NaN last)
 * and plan the next generation (Algorithm 1, sort / elites / parent pairs /
 * mutation parents): slot j < n_elite copies rank j; the next n_cross slots
 * are crossover children and the rest mutants, with parents drawn from the
 * top n_trunc (truncation) or by k-tournament.  Optional outputs (device):
 * plan_out [pop][4] int32 {op, parent1, parent2, 0}, f_inh_out [pop] float,
 * order_out [pop] int32 (slot of each rank).  Requires a preceding evaluate. */
leea_status leea_select(leea_ctx* ctx, int32_t* plan_out, float* f_inh_out,
                        int32_t* order_out);

/* Build the next population from the plan (Algorithm 1, crossover / mutation
 * / union): elites copied, crossover children not mutated, mutants get
 * theta + sigma*N(0,1) on each gene selected by mut_threshold.  With
 * self-adaptive sigma (section 3.2) elites keep their sigma gene, crossover
 * children take the parents' mean fl(fl(s1+s2)*0.5), and mutants take
 * fl(s * exp(fl(tau*z))) (z = first normal of Philox block (SIGMA, gen,
 * slot, 0), exp the library's float32 exp) and are mutated with that new
 * sigma.  Advances the generation counter.  Requires a preceding select. */
leea_status leea_crossover_mutate(leea_ctx* ctx);

/* select -> crossover_mutate -> evaluate, one generation.  With the fused
 * path allowed (leea_set_fused_step), for float32 batches of 5..16 rows that
 * the 1 KiB-row evaluation kernel does not take (and hidden widths that are
 * multiples of 4, with the genes after layer 1's weights small enough for
 * LDS) the variation and the evaluation run as one
 * kernel that builds each child from its parents in registers and evaluates
 * it as it is written (the children are not streamed back from HBM); the
 * results are bitwise identical to the three separate calls. */
leea_status leea_step(leea_ctx* ctx, const float* x, const int32_t* y, int32_t b,
                      float* f_adj, float* f_raw, float* acc);

/* crossover_mutate followed by evaluate (the second half of leea_step, with
 * the same fused small-batch path).  Requires a preceding select. */
leea_status leea_crossover_mutate_evaluate(leea_ctx* ctx, const float* x, const int32_t* y,
                                          int32_t b, float* f_adj, float* f_raw, float* acc);

/* Allow (enable != 0) or forbid (the default) the fused small-batch path of
 * leea_step and leea_crossover_mutate_evaluate: one kernel that builds each
 * child from its parents and evaluates it without writing and re-reading it
 * (float32 batches of 5..16 rows, hidden widths multiples of 4; batches of at
 * most 4, and of at most 8 where the 1 KiB-row evaluation kernel applies
 * (n0 a multiple of 4, at most 1024), always take the separate calls).
 * Results are bit-identical either way; it is off by default because the
 * separate variation and evaluation kernels measured faster. */
leea_status leea_set_fused_step(leea_ctx* ctx, int32_t enable);

/* Base mutation strength for the following crossover_mutate calls; with
 * self-adaptive sigma it resets every individual's sigma gene to sigma. */
leea_status leea_set_sigma(leea_ctx* ctx, float sigma);

/* Self-adaptive sigma genes of the current population (device [pop],
 * borrowed, valid until the next crossover_mutate); NULL in other modes. */
leea_status leea_sigmas(leea_ctx* ctx, float** sigmas);

/* Replace the sigma genes (device [pop]); LEEA_ESTATE unless self-adaptive. */
leea_status leea_set_sigmas(leea_ctx* ctx, const float* sigmas);

/* Current generation index (0 after init). */
leea_status leea_generation(const leea_ctx* ctx, uint32_t* gen);

/* Borrowed device pointers, valid until the next crossover_mutate/step:
 * the current population ([pop][stride] floats) and its f_adj [pop].  Read
 * only: replace a population with leea_set_state, which keeps the data the
 * reduced-precision paths derive from it (FP8 scales, the bfloat16 copy of
 * W_1 kept for batches above 16) in step. */
leea_status leea_population(leea_ctx* ctx, float** genomes, int64_t* stride,
                            float** f_adj);

/* Replace the current population with src (device, [pop][stride] floats,
 * padding genes zero) and, if f_adj is not NULL, its adjusted fitness
 * (device [pop]), which makes the ctx ready for select.  f_inh (device, may be
 * NULL) gives inherited values for the next evaluate (else none).  Used for
 * checkpoint restore and for feeding identical inputs to tests. */
leea_status leea_set_state(leea_ctx* ctx, const float* src, const float* f_adj,
                           const float* f_inh);

/* Host checkpoint: bytes needed, save (synchronises the stream) and load. */
leea_status leea_state_bytes(const leea_ctx* ctx, size_t* bytes);
leea_status leea_save(leea_ctx* ctx, void* host_buf, size_t bytes);
leea_status leea_load(leea_ctx* ctx, const void* host_buf, size_t bytes);

const char* leea_last_error(const leea_ctx* ctx);
void leea_destroy(leea_ctx* ctx);

/* ---- Learned fitness surrogate -------------------------------------------
 * A variant of the generation (not in the paper) that pre-screens
 * over-generated offspring: the n_elite elites are kept; k * (pop - n_elite)
 * candidate children are made (the first k * n_cross by crossover, the rest
 * by mutation, candidate c drawing from slot pop + c of the generation's
 * streams, section 3.2 operators); each is described by 256 +-1 random
 * projections of its bfloat16-rounded genome (times 1/sqrt(genes)), its
 * parents' adjusted fitness and its distance to parent 1 (times
 * 1/sqrt(genes)); every feature is standardised over the generation's
 * candidates (minus its mean, divided by its standard deviation, 0 where it
 * does not vary) and the 256 projections are scaled by 1/16, so that the
 * projection weighs as much as one scalar feature; a 259-64-1 MLP predicts
 * each candidate's standardised
 * fitness and the best pop - n_elite predictions fill the other slots.  The
 * new population is evaluated as usual (Eq. 1), which judges the MLP
 * (Kendall tau-a of its predictions for the kept candidates against their
 * fitness, RMSE against the training targets) and trains it (`steps`
 * full-batch gradient steps on the squared error against the kept
 * candidates' raw fitness standardised over them).  Until the MLP has
 * trained for `warmup` generations and the previous generation's tau reached
 * tau_min, the first n_cross crossover and n_mut mutation candidates are
 * kept instead (plain LEEA's mix). */
typedef struct {
  int32_t oversample;  /* k, 1..64; k * (pop - n_elite) <= 8192 */
  int32_t steps;       /* gradient steps per generation, 0..1000 */
  float lr;            /* learning rate, >= 0 */
  int32_t warmup;      /* trained generations before screening may start, >= 0 */
  float tau_min;       /* in [-1, 1] */
} leea_surrogate_config;

/* Device workspace bytes of the surrogate for this run. */
leea_status leea_surrogate_workspace_bytes(const leea_config* cfg,
                                           const leea_surrogate_config* sc, size_t* bytes);

/* Attach a surrogate (workspace: device, 256-byte aligned, caller-owned)
 * to ctx: writes the projection's sign bits and the MLP's initial
 * weights.  Not with self-adaptive sigma. */
leea_status leea_surrogate_attach(leea_ctx* ctx, const leea_surrogate_config* sc,
                                  void* workspace, size_t bytes);

/* One generation with pre-screening (in place of leea_step; same state
 * rules and outputs).  stats (device, 4 floats, may be NULL): {1 if the
 * surrogate screened this generation, tau, rmse, trained generations}. */
leea_status leea_surrogate_step(leea_ctx* ctx, const float* x, const int32_t* y, int32_t b,
                                float* f_adj, float* f_raw, float* acc, float* stats);

/* Borrowed device views of the last surrogate step (any may be NULL):
 * candidates [n][stride], their plan [n][4] {op, parent 1, parent 2, 0},
 * features [n][260] (259 used), the MLP's standardised inputs [n][260],
 * predictions [n], kept candidate indices [pop - n_elite] and their
 * predictions, MLP parameters (W1 [64][259], b1 [64], w2 [64], b2);
 * *n_candidates = n. */
leea_status leea_surrogate_views(leea_ctx* ctx, float** candidates, int32_t** plan,
                                 float** features, float** inputs, float** pred, int32_t** chosen,
                                 float** chosen_pred, float** params, int32_t* n_candidates);

/* ---- Many independent runs driven together -----------------------------
 * n EA runs, each with its own configuration (population, widths,
 * selection, crossover, seed and run index; batch size = max_batch), share one
 * training set and advance one generation per leea_runs_generation call.
 * Every phase of a generation is a single grouped launch over all runs
 * (evaluation: one launch per kernel class), and the generation is captured
 * once into a HIP graph that later calls replay, so the host cost does not
 * grow with the number of runs.  Each run computes exactly what it computes
 * alone through leea_step with the same config and the same evaluation
 * shape.  Restrictions: constant sigma, no input pooling, first layer in
 * float32 or bfloat16.  The stream must not be the null stream (graph
 * capture).  Calls on one leea_runs object must not overlap. */
#define LEEA_MAX_RUNS 1024
typedef struct leea_runs leea_runs;

/* Device workspace bytes for these n configs (1 <= n <= LEEA_MAX_RUNS). */
leea_status leea_runs_workspace_bytes(const leea_config* cfgs, int32_t n, size_t* bytes);

/* Carve the workspace (device, 256-byte aligned, caller-owned) and write
 * every run's initial population (Algorithm 1, first line).  *out is
 * host memory owned by the library (leea_runs_destroy). */
leea_status leea_runs_create(const leea_config* cfgs, int32_t n, void* workspace, size_t bytes,
                             void* hip_stream, leea_runs** out);

/* First call: draw generation 0's batch of every run and evaluate the
 * initial populations.  Later calls: one whole generation of every run
 * (draw, rank + plan, crossover / mutation, evaluate + inheritance).
 * x_train [n_train][widths[0]] (16-byte aligned) and y_train [n_train] are
 * device arrays shared by all runs (every run needs the same widths[0]). */
leea_status leea_runs_generation(leea_runs* m, const float* x_train, const int32_t* y_train,
                                 int64_t n_train);

/* Replay captured graphs (enable != 0, the default) or launch eagerly. */
leea_status leea_runs_set_graph(leea_runs* m, int32_t enable);

/* Completed generations (the same for every run). */
leea_status leea_runs_generation_count(const leea_runs* m, uint32_t* gen);

/* Borrowed device views of run r: current genomes [pop][stride] and its
 * adjusted / raw fitness and accuracy [pop] (any output may be NULL);
 * valid until the next generation. */
leea_status leea_runs_population(leea_runs* m, int32_t r, float** genomes, int64_t* stride,
                                 float** f_adj, float** f_raw, float** acc);

/* Evaluation shape of run r: kind 0 small-batch kernel (b <= 16), 1 float32
 * large-batch, 2 bfloat16 large-batch, 3 float32 row-streaming (b <= 4, the
 * float32 default there), 4 1 KiB-row kernel, float32 or bfloat16 (b <= 8,
 * n0 a multiple of 4 and at most 1024; the default for b <= 8 where kind 3
 * does not apply); mw = row tiles of 16 rows per wave (1 for kinds 0, 3, 4).
 * set_shape fails with LEEA_EINVAL for a shape that does not exist there.
 * A different shape may change the last bits of the fitness (the per-row
 * sums are grouped differently). */
leea_status leea_runs_shape(const leea_runs* m, int32_t r, int32_t* kind, int32_t* mw);
leea_status leea_runs_set_shape(leea_runs* m, int32_t r, int32_t kind, int32_t mw);

/* Autotuner: for each distinct (population, widths, batch, dtype) among the
 * runs, time every evaluation shape that exists for it (HIP events, 5
 * launches after 2 warm-ups, on a batch drawn from the training set) and
 * give all runs with that key the fastest.  Optional outputs per run
 * (host arrays of n): chosen kind, mw, and its time in microseconds. */
leea_status leea_runs_autotune(leea_runs* m, const float* x_train, const int32_t* y_train,
                               int64_t n_train, int32_t* kind_out, int32_t* mw_out,
                               float* us_out);

/* Text of the last error of m (of the last failed create if m is NULL). */
const char* leea_runs_last_error(const leea_runs* m);
void leea_runs_destroy(leea_runs* m);

/* 2x2 max-pooling (section 4.1) of n square side x side images x [n][side*side]
 * (device) into out [n][(side/2)^2] (device); side even.  NaN if any pooled
 * pixel is NaN.  Enqueues on hip_stream. */
leea_status leea_pool2x2(const float* x, int64_t n, int32_t side, float* out, void* hip_stream);

/* ---- generator entry points (bit-exactness checks of the random streams) ----
 * Each enqueues on hip_stream and returns without synchronising. */

/* out[i][0..3] = Philox4x32-10(ctr[i][0..3], key) for i < n (device arrays). */
leea_status leea_rng_philox(const uint32_t* ctr, uint64_t key, uint32_t* out, int64_t n,
                            void* hip_stream);
/* out[i] = float32 natural log of u[i] in (0, 1] (the mutation sampler's ln). */
leea_status leea_rng_ln32(const float* u, float* out, int64_t n, void* hip_stream);
/* Box-Muller: z[i][0..1] from words ab[i][0..1] (device). */
leea_status leea_rng_normal_pairs(const uint32_t* ab, float* z, int64_t n, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* LEEA_H */
