/*
 * metade.h -- C ABI of the MetaDE inner-DE library for AMD Instinct MI355X (gfx950).
 *
 * What it computes (paper: "MetaDE: Evolving Differential Evolution by
 * Differential Evolution", arXiv 2502.10470):
 *   - many Parameterized DE executors (Sec. III-A, Alg. 2) side by side, each
 *     with its own hyperparameter vector theta = (F, CR, bl, br, dn, cs);
 *     per generation: ranking (best / top-p), index sampling, mutation
 *     (Eq. 12), crossover (Eqs. 8-10), clipping to the search box, fitness,
 *     greedy selection (Alg. 1 selection rule);
 *   - the evolver of MetaDE (Alg. 3): DE/rand/1/bin over theta with one-shot
 *     evaluation (Sec. III-C) and the power-up schedule (Sec. III-D).
 *
 * Conventions shared by every entry point:
 *   - All device pointers are plain HIP device addresses owned by the caller
 *     unless stated otherwise; the context keeps them (non-owning) and they
 *     must outlive it.  The context owns only its internal scratch memory.
 *   - Work is enqueued on the caller's HIP stream (metade_config.stream) and
 *     is asynchronous unless an entry point says it synchronises.
 *   - Errors are returned as metade_status; nothing is thrown across the ABI.
 *     Device errors of asynchronous work surface as METADE_EDEVICE at the next
 *     synchronising call.  metade_last_error() gives a readable message.
 *   - A context is not thread-safe; use one context per stream.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with
 *     key = (seed & 0xffffffff, seed >> 32) and
 *     counter = (block, individual, phase, stream); phase is the generation
 *     number, 0xffffffff for the initial population; the evolver uses
 *     stream | 0x80000000.  Word w of an individual is word w % 4 of block
 *     w / 4: words 0..8 index draws, 9 pbest pick, 10 j_rand or start n,
 *     11 K, 12 + t crossover uniform t.
 *
 * Memory layouts (device, caller-owned):
 *   pop    float32, runs packed in order; run r occupies N_r * D_r floats
 *          starting at float offset sum_{s<r} N_s D_s, individual-major
 *          (individual i, gene j at i * D_r + j).
 *   fit    float32 [sum_r N_r], same run packing; fitness in the precision
 *          selection decisions are taken in.
 *   best_y float64 [n_runs]: y* of each run (fitness of its best individual,
 *          evaluated in float64 on the GPU).
 *   best_x float32 [sum_r D_r]: that individual.
 */
#ifndef METADE_H
#define METADE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct metade_ctx metade_ctx;

typedef enum {
  METADE_OK = 0,
  METADE_EINVAL = -1,   /* invalid argument or configuration */
  METADE_ENOMEM = -2,   /* device allocation of internal scratch failed */
  METADE_EDEVICE = -3,  /* a HIP call or an earlier asynchronous launch failed */
  METADE_ESTATE = -4    /* call out of order (e.g. outer step before outer reset) */
} metade_status;

/* Precision of the rotation z = R (u - o) of the shifted-rotated kinds.  The
 * control kind ignores it (its rollout is always float64).
 *   FP32: z accumulated in float64 (exact products), rounded once to float32;
 *         fitness terms in float32, sums in float64.
 *   BF16_REFINE: z from bf16 splits on the matrix cores with float32
 *         accumulation and a certified bound E on the fitness error; a trial
 *         whose approximate fitness minus E exceeds its target's is rejected
 *         at once, every other trial is re-evaluated as in FP32 and decided
 *         from that value, so decisions equal those of FP32. */
typedef enum {
  METADE_FP32 = 0,
  METADE_BF16_REFINE = 1
} metade_precision;

/* Evolver of the outer loop.
 *   DE:  DE/rand/1/bin with F = 0.5, CR = 0.9 (Alg. 3).
 *   PSO: particle swarm with inertia 0.729 and acceleration 1.49 + 1.49, the
 *        alternative evolver of the paper's supplement (S.III).  Positions
 *        start at the DE evolver's initial population with zero velocity; outer
 *        generation 0 scores them, later generations first move every particle
 *        (v = w v + c1 r1 (p - x) + c2 r2 (g - x), x = clip(x + v), float32 in
 *        that order; r1, r2 from Philox words k and 6 + k of (particle, outer
 *        generation) on the evolver's stream), then score; a personal best is
 *        replaced iff the new score <= its score.  In metade_get_outer, X and y
 *        are the personal bests, U and y_trial the current positions and scores.
 *   CSO: competitive swarm (Cheng and Jin's optimiser, also in S.III) without
 *        the mean-position term; at most 1024 particles.  Same start as PSO;
 *        from outer generation 1 on the particles are paired by sorting
 *        Philox word 12 of (particle, outer generation) (index breaks ties);
 *        in each pair the particle first in (score, index) order stays, the
 *        other moves v = r1 v + r2 (x_w - x_l), x = clip(x + v) (r1, r2 as for
 *        PSO); every particle is then scored and takes that score.  X and y
 *        are the swarm, U and y_trial the positions just scored (the same).
 *   NES: separable natural evolution strategy (Schaul et al.'s SNES, also in
 *        S.III); at most 1024 samples.  A Gaussian N(mu, diag sigma^2) starts
 *        at the centre of the theta box with sigma a quarter of its width;
 *        every outer generation draws n_runs samples z = mu + sigma s (s by
 *        Box-Muller from Philox words 2m, 2m + 1 of (sample, outer generation)
 *        on the evolver's stream, float64; z rounded once to float32 and
 *        clipped), scores them and moves mu += sigma sum_r u_r s_(r), sigma *=
 *        exp(eta_sigma / 2 sum_r u_r (s^2 - 1)) with rank utilities u_r and
 *        eta_sigma = (3 + ln 6) / (5 sqrt 6).  X, y, U and y_trial are the
 *        generation's samples and scores. */
typedef enum {
  METADE_EVOLVER_DE = 0,
  METADE_EVOLVER_PSO = 1,
  METADE_EVOLVER_CSO = 2,
  METADE_EVOLVER_NES = 3
} metade_evolver;

/* Objective functions: z = R (u - o) [+ c], f = g(z) + bias (textbook base
 * functions standing in for the paper's CEC2022 suite, Sec. IV-A). */
typedef enum {
  METADE_FN_RASTRIGIN = 1,
  METADE_FN_ROSENBROCK = 2,  /* c = 1 */
  METADE_FN_ACKLEY = 3,
  METADE_FN_ELLIPTIC = 4,    /* weights cond^(j/(D-1)) */
  METADE_FN_SCHWEFEL = 5,    /* c = 420.96875 */
  METADE_FN_HYBRID = 6,      /* permuted blocks: Schwefel | Rastrigin | elliptic */
  METADE_FN_LQR_MLP = 7      /* tanh policy scored by a linear-system rollout */
} metade_fn;

/* One problem instance.  Device pointers are caller-owned. */
typedef struct {
  uint32_t kind;         /* metade_fn */
  uint32_t D;            /* decision dimension */
  float bias;            /* added to g(z) */
  float cond;            /* elliptic condition number (elliptic and hybrid) */
  const float *o;        /* device [D] shift (not used by LQR_MLP) */
  const float *R;        /* device [D*D] row-major orthogonal rotation, z_j = sum_k R[j*D+k] y_k */
  const uint32_t *perm;  /* device [D] hybrid permutation (HYBRID only, else NULL) */
  uint32_t split[3];     /* hybrid block sizes, sum = D */
  /* control workload (LQR_MLP): policy obs -> hidden1 -> hidden2 -> act with
   * tanh on every layer, weights flattened W1 (hidden1 x obs, row-major), b1,
   * W2, b2, W3, b3; cost sum_{t<steps} |x_t|^2 + ctrl_weight |u_t|^2 averaged
   * over n_rollouts initial states; x_{t+1} = A x_t + B u_t.  The hidden
   * layers are both 32 wide (the policy MLPs of Sec. IV-D, Table VII) or both
   * 64 wide, and all control problems of one context share that width.  When
   * every control problem of a context has a multiple of 16 rollouts, each
   * policy is evaluated on the float64 matrix cores (16 rollouts per product);
   * otherwise the rollouts run one after another on the vector units. */
  uint32_t obs, act, hidden1, hidden2, steps, n_rollouts;
  float ctrl_weight;
  const float *A;        /* device [obs*obs] row-major */
  const float *B;        /* device [obs*act] row-major */
  const float *x0;       /* device [n_rollouts*obs] */
} metade_problem;

typedef struct {
  uint32_t n_runs;                 /* number of executors (>= 1) */
  const uint32_t *N;               /* host [n_runs] population sizes */
  const uint32_t *problem;         /* host [n_runs] index into problems */
  const uint32_t *stream_id;       /* host [n_runs] Philox stream; equal streams give the
                                      one-shot common seed of Sec. III-C */
  uint32_t n_problems;
  const metade_problem *problems;  /* host [n_problems]; copied at init */
  uint64_t seed;                   /* Philox key */
  float lb, ub;                    /* search box of every gene, lb < ub */
  uint32_t n_cs;                   /* crossover schemes in the theta space: 2 (bin, exp) or 3 (+arith) */
  uint32_t precision;              /* metade_precision */
  float *pop;                      /* device, caller-owned, see layouts above */
  float *fit;
  double *best_y;
  float *best_x;
  void *stream;                    /* hipStream_t (NULL = default stream) */
  uint32_t evolver;                /* metade_evolver */
  uint32_t graph;                  /* nonzero: the generation loop of control runs (four
                                      launches per generation) is captured once per
                                      sequence length as a HIP graph on a private stream
                                      and replayed on `stream`; traced steps always launch
                                      directly.  Results are identical either way. */
} metade_config;

/* Sizes in bytes of the caller-owned buffers and of the library's internal
 * scratch for this configuration.  Validates the configuration (see
 * metade_init).  Any output pointer may be NULL. */
metade_status metade_query_sizes(const metade_config *cfg, size_t *pop_bytes, size_t *fit_bytes,
                                 size_t *best_y_bytes, size_t *best_x_bytes, size_t *scratch_bytes);

/* Validate cfg, allocate internal scratch, copy the run and problem tables to
 * the device, set every run's theta to DE/rand/1/bin with F = 0.5, CR = 0.9,
 * and initialise every population (Alg. 2 initialisation and first
 * evaluation; x = lb + (ub - lb) (w >> 8) 2^-24 in float64, rounded once).
 * Rejected with METADE_EINVAL: n_runs = 0, N_r < 10 (the largest index draw,
 * 1 + 2 * 4 distinct indices plus the target), N_r > 256 or D_r > 128 for the
 * shifted-rotated kinds, lb >= ub, |lb| or |ub| > 1e30, n_cs not in {2, 3},
 * a precision not in metade_precision, a problem index out of range, a
 * missing device pointer, a hybrid permutation that is not one, an unknown
 * kind; for LQR_MLP: N_r > 1024, hidden1 != hidden2, a hidden width other
 * than 32 or 64 or two widths in one context, obs not in 1..20,
 * act not in 1..8, steps or n_rollouts = 0, a non-finite ctrl_weight, D not
 * equal to the policy's weight count.  A run is also rejected when its
 * population and draws do not fit in the 160 KB of LDS of its generation
 * kernel.  On success *out owns the context. */
metade_status metade_init(const metade_config *cfg, metade_ctx **out);

/* Re-run the initialisation and first evaluation of every run and reset the
 * generation counter to 0 (a fresh executor run with the same streams). */
metade_status metade_reset(metade_ctx *ctx);

/* Set every run's theta from host memory theta[n_runs][6] = (F, CR, bl, br,
 * dn, cs) in the continuous encoding.  On the device each vector is clipped
 * to the box [0,1]^2 x [1,5]^3 x [1, 1 + n_cs] (NaN -> lower bound) and
 * decoded as in Alg. 3: F, CR as is, categorical parts by floor with the box
 * end mapped to the last category (bl, br: 1 rand, 2 best, 3 pbest,
 * 4 current; dn 1..4; cs: 1 bin, 2 exp, 3 arith). */
metade_status metade_set_theta(metade_ctx *ctx, const float *theta);

/* Advance every run by n_generations generations of Alg. 2 (ranking, index
 * sampling, Eq. 12 mutation, Eq. 8-10 crossover, clip, fitness, greedy
 * selection), then refresh the best record (best_y in float64, best_x).
 * Asynchronous.  n_generations = 0 only refreshes the record. */
metade_status metade_inner_step(metade_ctx *ctx, uint32_t n_generations);

/* Size of the library's static device workspace (one copy per GPU the
 * library runs on, held until the process ends). */
#define METADE_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): exactly
 * metade_inner_step(ctx, n_generations), same kernels and same results, but
 * the matrix-core kernel's trial rows live in the library's static workspace
 * instead of the context's scratch, and the call allocates nothing: no
 * hipMalloc, no events (it is not timed by metade_kernel_timing), no graphs.  Asynchronous on the context's stream.
 * The workspace is shared by every call on a GPU and keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one
 * GPU -- from contexts on different streams or threads -- race and must be
 * serialised by the caller.  METADE_EINVAL if the context has control runs,
 * if its trial rows need more than METADE_STATIC_SCRATCH_BYTES (sum over the
 * matrix-core runs of N * Dk * 4 bytes, Dk = D rounded up to 32), or if the
 * current device is not the one the context was created on. */
metade_status metade_inner_step_static(metade_ctx *ctx, uint32_t n_generations);

/* Sizes of the trace buffers of metade_inner_step_trace, in bytes. */
metade_status metade_trace_sizes(metade_ctx *ctx, size_t *u_bytes, size_t *fu_bytes,
                                 size_t *desc_bytes);

/* One generation exactly like metade_inner_step(ctx, 1), additionally writing
 * per trial (device buffers, caller-owned, packed like pop / fit):
 *   u    float32 trial vector after crossover and clipping;
 *   fu   float32 its fitness as used by selection;
 *   desc int32 [sum_r N_r][16]: 0 base-left index, 1 base-right index,
 *        2..9 difference pairs (a1,b1,..,a4,b4; -1 unused), 10 j_rand or n,
 *        11 L (exponential) or -1, 12 pbest rank, 13 rand index or -1,
 *        14 K bits (float32) , 15 accept flag.
 * In a METADE_BF16_REFINE context a traced generation re-evaluates every
 * trial with the plain evaluation (fu is that value; the decisions are the
 * mode's, which equal the plain ones) and checks each trial's bf16 value
 * against its bound (see metade_get_bound_check). */
metade_status metade_inner_step_trace(metade_ctx *ctx, float *u, float *fu, int32_t *desc);

/* Totals since metade_init of the bound check that traced generations of a
 * METADE_BF16_REFINE context carry out (synchronises; any pointer may be
 * NULL; all zero in other contexts): trials checked; trials whose bf16
 * fitness lies farther than its bound from the plain value (a bound
 * violation: must stay 0); trials the screen alone would have rejected
 * without re-evaluation; of those, the ones the plain value accepts (a wrong
 * decision: must stay 0); the largest |f_bf16 - f_plain| / bound seen. */
metade_status metade_get_bound_check(metade_ctx *ctx, uint64_t *checked, uint64_t *outside,
                                     uint64_t *screened, uint64_t *screen_wrong,
                                     double *max_ratio);

/* Evolver (Alg. 3; metade_config.evolver selects DE or PSO).  The context's
 * runs are the P = n_runs executors of one outer population.
 * metade_outer_reset draws the initial population in the theta box on the
 * device and sets every fitness to +inf (PSO: positions = that population,
 * velocities 0). */
metade_status metade_outer_reset(metade_ctx *ctx);

/* One outer generation: DE/rand/1/bin trial vectors (F = 0.5, CR = 0.9) --
 * or, for PSO, the moved particle positions (none moved in generation 0) --
 * clipped and decoded into the runs' theta; all executors re-initialised
 * (same streams: one-shot evaluation) and run for G_inner generations
 * (G_inner * power_up if power_up > 1: Sec. III-D); y* of each run; the
 * trial replaces its target (PSO: the position replaces the personal best)
 * iff y*(trial) <= y(target).  METADE_EINVAL if G_inner * power_up does not
 * fit in 32 bits.  Asynchronous. */
metade_status metade_outer_step(metade_ctx *ctx, uint32_t G_inner, uint32_t power_up);

/* Copy the evolver state to host memory (synchronises): X[n_runs][6],
 * y[n_runs], the last trial vectors U[n_runs][6] and their scores
 * y_trial[n_runs]; any pointer may be NULL. */
metade_status metade_get_outer(metade_ctx *ctx, float *X, double *y, float *U, double *y_trial);

/* Set the evolver state from host memory (X[n_runs][6], y[n_runs]) and the
 * outer generation counter.  For the PSO, CSO and NES evolvers, whose other
 * state (positions and velocities, the search distribution) X and y do not
 * carry, metade_outer_reset must have been called on the context first
 * (METADE_ESTATE otherwise); that state is left as it is. */
metade_status metade_set_outer(metade_ctx *ctx, const float *X, const double *y, uint32_t gen);

/* Whole MetaDE run (synchronises): outer reset, outer_gens outer generations
 * of G_inner inner generations, the last multiplied by power_up, then the
 * best evolver individual: its score, theta, and the best x of the executor
 * run that produced it.  Host outputs; best_x has D of that run's problem. */
metade_status metade_run(metade_ctx *ctx, uint32_t outer_gens, uint32_t G_inner, uint32_t power_up,
                         double *best_y, float *best_theta, float *best_x);

/* Copy best_y[n_runs] to host memory (synchronises). */
metade_status metade_get_best(metade_ctx *ctx, double *y);

/* Checkpoint: all state that determines future results (populations,
 * fitness, decoded theta, generation counters, evolver state, best records)
 * as an opaque host blob.  With blob == NULL only *bytes is set.
 * Synchronises.  metade_set_state accepts a blob from any context with the
 * same runs (sizes, packing) and n_cs, whatever its precision: the run layout
 * always comes from the receiving context.  METADE_EINVAL for a blob of
 * another size or configuration, or one whose theta lies outside the decoded
 * domain (F, CR in [0, 1], bl, br, dn in 1..4, cs in 1..n_cs). */
metade_status metade_get_state(metade_ctx *ctx, void *blob, size_t *bytes);
metade_status metade_set_state(metade_ctx *ctx, const void *blob, size_t bytes);

/* Timing of the generation kernel: when enabled, every launch of it is
 * bracketed by HIP events on the context's stream; metade_kernel_time
 * synchronises and returns the summed milliseconds and launch count since
 * the last enable. */
metade_status metade_kernel_timing(metade_ctx *ctx, int enable);
metade_status metade_kernel_time(metade_ctx *ctx, double *ms, uint64_t *launches);

/* Counters since metade_init (synchronises): trials evaluated, and trials
 * re-evaluated exactly by the BF16_REFINE mode (0 otherwise). */
metade_status metade_get_counters(metade_ctx *ctx, uint64_t *trials, uint64_t *refined);

/* Launch-shape choices of the generation kernels.  Results do not depend on
 * mfma_rows; lane_parts regroups the float64 sums of a trial's terms, which
 * can move a float32 fitness by one unit in the last place.
 *   lane_parts: parts per trial in the lane kernel's fitness stage (each
 *               part a whole number of waves covering the population): 0 =
 *               as many as fit the consumer lanes (at most 8), else 1, 2, 4
 *               or 8, capped at that number;
 *   mfma_rows:  row tiles (16 trials each) per rotation item of the
 *               matrix-core kernel's plain evaluation: 2 or 4 (0 = 4). */
typedef struct {
  uint32_t lane_parts;
  uint32_t mfma_rows;
} metade_tuning;

/* Read or set the context's tuning (set: METADE_EINVAL for values outside
 * the lists above; synchronises). */
metade_status metade_get_tuning(metade_ctx *ctx, metade_tuning *t);
metade_status metade_set_tuning(metade_ctx *ctx, const metade_tuning *t);

/* Autotuner: time n_generations of the context's own runs under every
 * candidate tuning of the kernels it uses (lane_parts 0/4/2/1 when it has
 * lane-kernel runs; mfma_rows 4/2 when it has matrix-core runs in float32
 * precision), each from the same checkpoint, fastest of two timed passes
 * after a warm-up, and keep the fastest.  The context's state (populations,
 * counters, records) is restored afterwards, so results do not depend on
 * the search itself.  With cache_path != NULL the choice is looked up first
 * in that text file, one line per key "<16 hex digits> <lane_parts>
 * <mfma_rows> <ms>", the key hashing the runs' (N, D, kind) multiset, the
 * precision and n_generations; a measured choice is appended to it.
 * chosen and best_ms (the chosen tuning's time for n_generations) may be
 * NULL.  Synchronises.  On an error during the search the
 * context is put back, as far as the device allows, to the tuning and the
 * state it had before the call, and metade_last_error names the failure. */
metade_status metade_autotune(metade_ctx *ctx, uint32_t n_generations, const char *cache_path,
                              metade_tuning *chosen, double *best_ms);

/* Readable message of the last error on ctx (or of the last failed
 * metade_init when ctx is NULL).  Never NULL. */
const char *metade_last_error(const metade_ctx *ctx);

/* Release the context's scratch.  Safe on NULL. */
void metade_destroy(metade_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* METADE_H */
