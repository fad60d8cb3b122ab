/*
 * psgld.h -- C ABI of an MI355X (gfx950) library for Parallel SGLD (PSGLD)
 * matrix factorisation, after Simsekli et al., "Parallel Stochastic Gradient
 * Markov Chain Monte Carlo for Matrix Factorisation Models" (arXiv:1506.01418).
 *
 * Model (Section 2, Eq. (1); Section 4, Eq. (13)): V (I x J) ~ W H with W
 * (I x K) and H (K x J); v_ij ~ Tweedie(mean sum_k w_ik h_kj, dispersion phi,
 * power parameter beta), whose log density is -d_beta(v||mu)/phi up to a
 * constant; iid exponential or Gaussian priors on every factor element.
 *
 * Sampler (Section 3, Eq. (7)-(9), Algorithm 1): [I] and [J] are each cut
 * into B pieces; block (b, c) is the cross product of row piece b and column
 * piece c (Definition 1); iteration t uses part p = t mod B, made of blocks
 * (b, (b + p) mod B) for b = 0..B-1 (Definition 2, cyclic order as in the
 * experiments of Section 4.2.1).  Every element x of W and H moves by
 *     x <- x + eps_t (N/|Pi_t| * sum over its block's entries of
 *                     d log p(v_ij | .)/dx + d log p(x)/dx) + sqrt(2 eps_t) z
 * with both gradients at the previous state, z ~ N(0,1), then x <- |x| when
 * mirroring is on (Section 3.2).  N is the number of observed training
 * entries and |Pi_t| the number of them in the part.
 *
 * Conventions of the whole ABI:
 *  - Every call returns a psgld_status (0 = OK, negative = error) except
 *    psgld_last_error, psgld_destroy and psgld_default_options.  No exception
 *    crosses the ABI.  After an error, psgld_last_error(ctx) describes it
 *    until the next call on that ctx.
 *  - All array arguments are HOST pointers owned by the caller; the library
 *    copies what it needs during the call and never keeps the pointer.
 *    Output arrays are caller-allocated with the sizes stated below.
 *  - W is exchanged as I x K row-major and H as K x J row-major (the paper's
 *    orientation), in the precision named in each signature.
 *  - The library owns the context and all device memory it allocates,
 *    through the caller's allocator hooks when options give them.
 *  - A context is used by one host thread at a time.  Stepping is
 *    asynchronous on the context's stream; getters synchronise it.
 */
#ifndef PSGLD_H
#define PSGLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSGLD_OK = 0,
    PSGLD_E_ARG = -1,         /* invalid argument or data (message says which) */
    PSGLD_E_STATE = -2,       /* call not valid in the context's current state */
    PSGLD_E_NOMEM = -3,       /* host or device allocation failed */
    PSGLD_E_DEVICE = -4,      /* HIP runtime error, or no gfx950 device */
    PSGLD_E_NUMERIC = -5,     /* a non-finite value appeared in W or H */
    PSGLD_E_UNSUPPORTED = -6  /* valid request the library does not implement */
} psgld_status;

typedef struct psgld_ctx psgld_ctx;

/* Tweedie likelihood, Section 4: beta = 2 Gaussian, 1 Poisson, 0 < beta < 1
 * compound Poisson, 0 gamma.  phi > 0.  For beta < 2 the mean is floored at
 * options.mu_floor before the residual (v - mu) mu^(beta-2) / phi. */
typedef struct {
    double beta;
    double phi;
} psgld_likelihood;

typedef enum {
    PSGLD_PRIOR_EXPONENTIAL = 0,  /* rate lambda, density on |x| (Eq. (13)) */
    PSGLD_PRIOR_GAUSSIAN = 1      /* mean 0, precision lambda */
} psgld_prior_kind;

typedef struct {
    int32_t kind;       /* psgld_prior_kind */
    double lambda_w;    /* > 0 */
    double lambda_h;    /* > 0 */
    int32_t mirror;     /* 1: x <- |x| after each update (Algorithm 1) */
} psgld_prior;

/* Step size eps_t = a * (t0 + t)^(-gamma) at the 0-based global iteration t
 * (the paper's (a/t)^b is a = a^b, t0 = 1, gamma = b).  Eq. (4) asks for
 * gamma in (0.5, 1]; gamma = 0 (a constant step) is accepted too. */
typedef struct {
    double a;
    double t0;
    double gamma;
} psgld_eps_schedule;

/* Precision of the dense-block kernels (coordinate entries are always FP32).
 * PSGLD_BF16_DENSE: the three products of Eq. (8)-(9) on a dense block take
 * W, H and E rounded to BF16 (nearest even), accumulating in FP32.
 * PSGLD_BF16_DENSE_VALUES: the same, and the dense blocks' training values
 * are also stored in BF16, rounded to nearest even once when loaded: the
 * chain then samples the posterior of those rounded values (relative change
 * at most 2^-9 per value; integers up to 256 are unchanged), and an
 * iteration reads 2 instead of 4 bytes per cell. */
enum { PSGLD_FP32 = 0, PSGLD_BF16_DENSE = 1, PSGLD_BF16_DENSE_VALUES = 2 };
/* Part order: cyclic, p_t = t mod B (Section 4.2.1), or drawn at every
 * iteration with probability |part| / N (Condition 2) from the Philox stream
 * PART = 4: counter (0, 0, t, 4), u = (2 (r0 >> 9) + 1) 2^-24, part = the
 * first p with u N < n_0 + ... + n_p (compared exactly on integers scaled by
 * 2^24); cyclic when there are no entries. */
enum { PSGLD_PART_CYCLIC = 0, PSGLD_PART_RANDOM = 1 };
enum {
    PSGLD_TEST_NOISE_OFF = 1u,  /* z = 0: the chain becomes parallel SGD */
    PSGLD_TEST_FREEZE_W = 2u,   /* W is not updated */
    PSGLD_TEST_FREEZE_H = 4u    /* H is not updated */
};

typedef struct {
    uint64_t seed;            /* Philox key of the Langevin noise */
    int64_t burn_in;          /* moments and held-out sums start at t >= burn_in */
    int32_t thin;             /* moments kept at t - burn_in = 0, thin, 2 thin, ... */
    int32_t precision;        /* PSGLD_FP32, PSGLD_BF16_DENSE or PSGLD_BF16_DENSE_VALUES (dense blocks only) */
    double dense_threshold;   /* blocks denser than this use the dense kernel */
    double mu_floor;          /* floor of the Tweedie mean when beta < 2 */
    const int32_t *row_piece; /* optional, length I: piece of each row; NULL = contiguous split */
    const int32_t *col_piece; /* optional, length J: piece of each column */
    void *stream;             /* hipStream_t to run on; NULL = the library's own stream */
    uint32_t test_flags;      /* PSGLD_TEST_* (test use only) */
    int32_t device;           /* HIP device ordinal */
    int32_t graph_iters;      /* iterations per captured HIP graph in psgld_step:
                                 < 0 = never capture, one launch sequence per
                                 iteration (the default: on MI355X graph replay
                                 measured no faster); 0 = one cycle of B
                                 parts repeated to at least 32 iterations;
                                 > 0 = that many iterations */
    int32_t persistent;       /* 1: contexts without dense blocks run their
                                 iterations in cooperative single launches of up
                                 to 256 iterations (grid-wide barrier between
                                 iterations; no graph); 0 = off */
    int32_t part_order;       /* PSGLD_PART_CYCLIC (default) or PSGLD_PART_RANDOM;
                                 random order is never captured into graphs */
    int32_t dense_min_cols;   /* blocks narrower than this run as coordinates
                                 even when dense (default 256: one dense
                                 work-group's width; narrower tiles measured
                                 slower than the coordinate kernel) */
    int32_t persistent_grid;  /* work-groups of a persistent launch; 0 = as many
                                 as the device holds at once (capped by the
                                 work).  Fewer make each work-group run several
                                 tasks of an iteration in turn. */
    /* Device memory of the context (Algorithm 1's inputs and outputs held on
     * the GPU: factors, entries, moment sums, schedules, scratch).  With both
     * hooks NULL the library calls hipMalloc / hipFree itself; with both set
     * every device allocation of the context goes through them instead (the
     * Python binding passes PyTorch's caching allocator), so the caller sees
     * and accounts for all of it.  dev_alloc(bytes, alloc_user) returns device
     * memory of options.device aligned to 256 bytes, or NULL (the calling
     * function then fails with PSGLD_E_NOMEM); it is called with that device
     * current, on the host thread that called the library.  dev_free(ptr,
     * bytes, alloc_user) returns a block with the size it was asked for; the
     * library calls it only once the context's stream has finished every
     * use of the block.  Setting only one hook is PSGLD_E_ARG. */
    void *(*dev_alloc)(size_t bytes, void *user);
    void (*dev_free)(void *ptr, size_t bytes, void *user);
    void *alloc_user;
} psgld_options;

/* Fills *opt with the defaults: seed 0, burn_in 0, thin 1, FP32,
 * dense_threshold 0.3, mu_floor 1e-6, contiguous pieces, own stream,
 * no test flags, device 0, graph_iters -1, persistent 0, cyclic part order,
 * dense_min_cols 256, persistent_grid 0, no allocator hooks (hipMalloc). */
void psgld_default_options(psgld_options *opt);

/* Creates a context for an I x J matrix, rank K (1..256), B x B blocks
 * (1 <= B <= min(I, J)).  opt may be NULL for the defaults; it is copied.
 * Pieces given in opt must be non-empty for every b (Section 3, P_B).
 * E_ARG on invalid sizes or parameters (phi, lambda > 0, thin >= 1).
 * No device memory is allocated until data is loaded. */
psgld_status psgld_create(int64_t I, int64_t J, int32_t K, int32_t B,
                          const psgld_likelihood *lik, const psgld_prior *prior,
                          const psgld_options *opt, psgld_ctx **out);

/* Loads the observed TRAINING entries (Algorithm 1 input V) as coordinates:
 * row[n] in [0, I), col[n] in [0, J), val[n] finite, with val >= 0 when
 * beta <= 1 and val > 0 when beta <= 0.  Cells absent from the list are
 * missing (not zero).  Duplicated (row, col) pairs are E_ARG.  Builds the
 * block-sorted layout on the host and uploads it.  Once per context
 * (E_STATE on a second load).  0 <= nnz <= 2^31 - 64. */
psgld_status psgld_load_coo(psgld_ctx *ctx, int64_t nnz, const int32_t *row,
                            const int32_t *col, const float *val);

/* Loads a dense I x J row-major value matrix V with a training mask
 * (1 = observed training cell, 0 = missing; NULL = every cell observed).
 * Blocks whose training density exceeds options.dense_threshold are run by
 * the dense kernel, the rest as coordinates (E_ARG if those exceed 2^31 - 64
 * cells).  Same value rules as load_coo.  With options.precision =
 * PSGLD_BF16_DENSE_VALUES the values of the dense-kernel blocks are kept in
 * BF16 (rounded to nearest even here, once); coordinate blocks keep FP32. */
psgld_status psgld_load_dense(psgld_ctx *ctx, const float *V, const uint8_t *train_mask);

/* Held-out cells whose posterior-mean prediction is tracked: at every
 * iteration t >= burn_in whose part contains the cell's block, mu_ij of the
 * state entering that iteration is added to the cell's FP64 sum.  Cells
 * must be distinct and must not be training entries (E_STATE).  Call after
 * a load and before the first step.  val may be NULL (then heldout_rmse is
 * unavailable). */
psgld_status psgld_load_heldout(psgld_ctx *ctx, int64_t n, const int32_t *row,
                                const int32_t *col, const float *val);

/* Sets the current sample: W is I x K, H is K x J, finite.  With mirroring
 * on, |W| and |H| are stored.  Required before the first step (Algorithm 1
 * takes W(0), H(0) as inputs). */
psgld_status psgld_set_factors(psgld_ctx *ctx, const float *W, const float *H);

/* Runs n_iter >= 0 iterations of Algorithm 1, asynchronously on the
 * context's stream, continuing from the context's iteration counter t.
 * Runs of graph_iters iterations are captured once into a HIP graph (per
 * starting part and ping-pong phase) and replayed; the graph reads the
 * iteration from a device counter and the step sizes from a device table,
 * so replays are bitwise identical to launching the iterations one by one.
 * E_STATE before data and factors are set.  A non-finite value produced by
 * these iterations is reported as E_NUMERIC by the next synchronising call. */
psgld_status psgld_step(psgld_ctx *ctx, int64_t n_iter, const psgld_eps_schedule *sched);

/* Runs n_iter[j] >= 0 iterations of context ctxs[j] with schedule
 * scheds[j], for j < n, interleaved iteration by iteration.  Contexts with
 * only coordinate-stored blocks are grouped by kernel variant (rank class and
 * likelihood branch) and up to 64 of them share one launch per iteration: the
 * launch reads a device table of the contexts, and each context's iteration
 * from its device clock.  With more than one variant, each variant's launches
 * go to an auxiliary stream of the library (a pool per device, kept for the
 * life of the process), forked from the contexts' stream and joined back
 * into it before the call returns, so the variants overlap on the device;
 * work enqueued on the contexts' stream afterwards sees all of it.  Contexts
 * with dense blocks are launched one by one
 * inside the same loop.  Each context's results are bitwise those of
 * psgld_step on it alone: the contexts share no memory.  All contexts must be
 * distinct and share one device and one stream (options.stream), else E_ARG;
 * each needs data and factors (E_STATE).  When every coordinate-stored
 * context has options.persistent set, each group of contexts with the same
 * variant and iteration count runs all its iterations in one cooperative
 * launch instead.  Asynchronous like psgld_step. */
psgld_status psgld_step_batch(psgld_ctx *const *ctxs, int32_t n, const int64_t *n_iter,
                              const psgld_eps_schedule *scheds);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, e.g. a tight serving loop or a harness that forbids it): the
 * same iterations as psgld_step, from the same kernels and bitwise the same
 * results, with no device or host allocation in the call.  The scratch those
 * kernels use beside the context's own arrays -- the partial gradients and
 * arrival counters of items cut over several work-groups, and this call's
 * step sizes -- lives in one static 16 MiB device array per GPU, held until
 * the process ends.  Per call at most 65536 iterations (E_ARG beyond); only
 * contexts without dense blocks (E_UNSUPPORTED), whose schedule's split
 * shares fit the array: at most 65536 shares of Kp floats within 15.25 MiB
 * (E_UNSUPPORTED beyond).  Waits for the context's queued work before it
 * overwrites the step sizes, then runs asynchronously on the context's
 * stream like psgld_step (per-iteration launches; no graph, no persistent
 * launch).  Calls on one GPU share the array: two calls whose work overlaps
 * on the device (different streams or threads) race and give wrong results,
 * so callers serialise them.  The context itself is created and loaded as
 * usual beforehand. */
psgld_status psgld_step_static(psgld_ctx *ctx, int64_t n_iter, const psgld_eps_schedule *sched);

/* Tunes the work schedule of the coordinate-stored blocks on this context's
 * own data: how many entries one lane group takes before an item is spread
 * over more groups (the candidates), and the kernel variant -- how many
 * 4-element pieces of a row each lane holds (1, 2 or 4), which sets how many
 * lanes share an item.  With n > 1, each candidate in candidates[0..n) is
 * timed with every variant built for this rank, over `iters` iterations
 * (iters < 1: one cycle of B parts) from the current state with schedule
 * `sched`; the state is restored afterwards, so the chain is unchanged, and
 * the fastest pair is kept and remembered for this shape (in-process, and in
 * the file named by the environment variable PSGLD_TUNE_CACHE if set, which
 * later contexts of the same shape read at load).  With n == 1 the candidate
 * is applied with the current variant.  Results are bitwise reproducible for
 * a fixed choice; different choices change the FP32 summation order.
 * *chosen (may be NULL) receives the entries per group kept.  Syncs. */
psgld_status psgld_tune(psgld_ctx *ctx, const int32_t *candidates, int32_t n, int32_t iters,
                        const psgld_eps_schedule *sched, int32_t *chosen);

/* Sets the sparse schedule directly (what psgld_tune chooses): entries per
 * lane group >= 1 and quads per lane 1, 2 or 4 (0: the default for the rank);
 * E_ARG if no kernel variant covers the rank with that many quads per lane.
 * Needs loaded data (E_STATE).  Waits for queued work. */
psgld_status psgld_set_schedule(psgld_ctx *ctx, int32_t entries_per_group, int32_t quads_per_lane);

/* The sparse schedule in use: entries per lane group, quads per lane and
 * lanes per item group (any output may be NULL). */
psgld_status psgld_schedule_info(psgld_ctx *ctx, int32_t *entries_per_group, int32_t *quads_per_lane,
                                 int32_t *lanes_per_group);

/* Blocks until the context's queued work is done.  E_NUMERIC (with the
 * first iteration index in the message) if a non-finite value appeared. */
psgld_status psgld_sync(psgld_ctx *ctx);

/* Copies the current sample out (FP32): W is I x K, H is K x J.  Syncs. */
psgld_status psgld_get_factors(psgld_ctx *ctx, float *W, float *H);

/* Posterior mean and plug-in variance sum(x^2)/S - mean^2 over the S kept
 * samples (FP64 sums kept on the device).  E_STATE if S = 0.  Syncs. */
psgld_status psgld_posterior_mean(psgld_ctx *ctx, double *W, double *H);
psgld_status psgld_posterior_var(psgld_ctx *ctx, double *W, double *H);

/* Number of kept samples S so far. */
psgld_status psgld_num_samples(psgld_ctx *ctx, int64_t *S);

/* Posterior-mean prediction of each held-out cell, in load order (n values):
 * the average of mu_ij over the iterations that visited its block after
 * burn-in.  Cells not visited yet give NaN.  Syncs. */
psgld_status psgld_heldout_predictions(psgld_ctx *ctx, double *pred);

/* Root mean squared error of those predictions against the held-out values,
 * unclipped.  E_STATE if no held-out values were given or none visited. */
psgld_status psgld_heldout_rmse(psgld_ctx *ctx, double *rmse);

/* Training log-likelihood of the current sample, -sum d_beta(v||mu)/phi over
 * the training entries (the Tweedie normaliser, free of W and H, dropped),
 * reduced in FP64 on the device.  Syncs. */
psgld_status psgld_log_likelihood(psgld_ctx *ctx, double *ll);

/* Iteration counter t (number of iterations run so far). */
psgld_status psgld_iteration(psgld_ctx *ctx, int64_t *t);

/* |Pi_p| for p = 0..B-1 (training entries in each part), and N. */
psgld_status psgld_part_sizes(psgld_ctx *ctx, int64_t *n_p, int64_t *N);

/* Checkpoint.  get_state with buf == NULL stores the needed size in *size;
 * otherwise writes the chain state (t, W, H, moments, held-out sums) into
 * buf of *size bytes.  set_state restores it into a context created and
 * loaded identically; since the noise is keyed by (seed, t, index), a
 * restored chain continues bit for bit. */
psgld_status psgld_get_state(psgld_ctx *ctx, void *buf, size_t *size);
psgld_status psgld_set_state(psgld_ctx *ctx, const void *buf, size_t size);

/* Device memory held by the context, in bytes. */
psgld_status psgld_memory_bytes(psgld_ctx *ctx, int64_t *bytes);

/* The hipStream_t the context runs on. */
psgld_status psgld_get_stream(psgld_ctx *ctx, void **stream);

/* Message of the context's last error ("" if none).  ctx may be NULL, then
 * the message of the last failed psgld_create on this thread. */
const char *psgld_last_error(const psgld_ctx *ctx);

/* Frees the context and its device memory.  NULL is ignored. */
void psgld_destroy(psgld_ctx *ctx);

/* ---- noise stream (Section 2: noise N(0, 2 eps) per parameter) ----------
 * The Langevin noise of parameter k of row i of W (stream 0) or column j of
 * H (stream 1) at iteration t is z = Box-Muller(Philox4x32-10(counter =
 * (k/4, index, t, stream), key = (seed lo, seed hi))) component k mod 4,
 * uniforms u = (2 (r >> 9) + 1) 2^-24.  These two calls evaluate the stream
 * on the device for n counters given on the host, so tests can compare it
 * with an independent implementation. */

/* out[4n]: raw Philox4x32-10 blocks of ctr[4n] under key[2n]. */
psgld_status psgld_philox_blocks(int64_t n, const uint32_t *ctr, const uint32_t *key,
                                 uint32_t *out, int32_t device);

/* z[K n], radius[K n]: the K normals of rows/columns index[n] of stream
 * stream[n] at iteration t[n] under `seed`, as the sampler draws them. */
psgld_status psgld_normals(int64_t n, uint64_t seed, const int64_t *t, const uint32_t *stream,
                           const int64_t *index, int32_t K, float *z, float *radius,
                           int32_t device);

/* The part (0 .. B-1) iteration t uses under the context's part order.
 * Needs loaded data (E_STATE). */
psgld_status psgld_part_at(psgld_ctx *ctx, int64_t t, int32_t *part);

/* Data-dependent pieces (Section 3 lets the pieces be any partition): each
 * of the n elements (rows or columns) with weight[m] >= 0 (e.g. its number
 * of training entries plus one for its own update) is put into one of B
 * pieces, heaviest first, each into the piece with the least weight so far
 * (lowest index on ties), so no piece is empty when n >= B and the heaviest
 * piece exceeds the lightest by at most the largest single weight.
 * Deterministic.  piece[n] is written.  Host only; E_ARG if n < B, B < 1 or
 * a weight is negative.  Use the result as options.row_piece / col_piece. */
psgld_status psgld_balanced_pieces(int64_t n, const int64_t *weight, int32_t B, int32_t *piece);

/* ---------------------------------------------------------------------
 * Serving: many independent PSGLD runs ("jobs") on one device.
 *
 * Jobs wait in a FIFO queue.  A job is admitted when fewer than max_active
 * jobs run and the device bytes it will need (an upper estimate before it is
 * loaded, its context's actual allocation afterwards) fit in hbm_budget
 * beside the running jobs; the queue head blocks those behind it, so jobs
 * start in submission order.  Each tick admits what fits, advances every
 * running job by up to iters_per_tick iterations with psgld_step_batch (one
 * launch per kernel variant for all coordinate-stored jobs), waits for the
 * device, and retires jobs that reached their n_iter: their FP64 posterior
 * moments and held-out RMSE are copied to host memory and their device
 * memory is freed.  A job's results are bitwise those of the same run on a
 * context of its own.  A server is used by one host thread at a time.
 * --------------------------------------------------------------------- */
typedef struct psgld_server psgld_server;

typedef struct {
    int64_t hbm_budget;       /* device bytes the running jobs may hold; > 0 */
    int32_t max_active;       /* running jobs at most; >= 1 */
    int32_t iters_per_tick;   /* iterations per job per tick; >= 1 */
    int32_t device;           /* HIP device ordinal */
    int32_t persistent;       /* 1: a tick runs in cooperative launches (options.persistent of the jobs) */
    /* Allocator hooks handed to every job's context (as in psgld_options);
     * a job's device bytes are what its context asked of them. */
    void *(*dev_alloc)(size_t bytes, void *user);
    void (*dev_free)(void *ptr, size_t bytes, void *user);
    void *alloc_user;
} psgld_server_options;

/* One complete run.  Data as for psgld_load_coo (row != NULL) or
 * psgld_load_dense (row == NULL, dense != NULL, mask may be NULL); held-out
 * cells as for psgld_load_heldout (n_heldout may be 0); W0 (I x K) and H0
 * (K x J) as for psgld_set_factors.  The job runs n_iter >= 1 iterations of
 * schedule sched with the given seed, burn-in, thinning, precision, dense
 * threshold and dense width (other options at their defaults). */
typedef struct {
    int64_t I, J;
    int32_t K, B;
    psgld_likelihood lik;
    psgld_prior prior;
    uint64_t seed;
    int64_t burn_in;
    int32_t thin;
    int32_t precision;
    double dense_threshold;
    int32_t dense_min_cols;   /* as options.dense_min_cols; 0 = its default */
    psgld_eps_schedule sched;
    int64_t n_iter;
    int64_t nnz;
    const int32_t *row, *col;
    const float *val;
    const float *dense;
    const uint8_t *mask;
    int64_t n_heldout;
    const int32_t *hrow, *hcol;
    const float *hval;
    const float *W0, *H0;
} psgld_job;

enum { PSGLD_JOB_QUEUED = 0, PSGLD_JOB_RUNNING = 1, PSGLD_JOB_DONE = 2, PSGLD_JOB_FAILED = 3 };

psgld_status psgld_server_create(const psgld_server_options *opt, psgld_server **out);

/* Upper estimate of the device bytes a job's context allocates. */
psgld_status psgld_server_estimate_bytes(const psgld_job *job, int64_t *bytes);

/* Copies the job's inputs and queues it; *id receives its handle.  E_ARG if
 * the job is malformed or its estimate exceeds the whole budget. */
psgld_status psgld_server_submit(psgld_server *srv, const psgld_job *job, int64_t *id);

/* One tick (see above).  Outputs (each may be NULL): jobs running after the
 * tick, jobs still queued, jobs retired by this tick.  A job whose load or
 * run fails is marked FAILED (its message in psgld_server_job_error) and the
 * tick goes on; only device errors of the shared stream fail the tick. */
psgld_status psgld_server_tick(psgld_server *srv, int32_t *n_running, int32_t *n_queued, int32_t *n_retired);

/* State, iterations done, estimated and actual device bytes (actual is 0
 * until admitted) of a job.  Any output may be NULL. */
psgld_status psgld_server_job_info(psgld_server *srv, int64_t id, int32_t *state, int64_t *iterations,
                                   int64_t *est_bytes, int64_t *bytes);

/* Results of a DONE job: posterior means and variances (I x K and K x J,
 * FP64, as psgld_posterior_mean/var) and held-out RMSE (NaN without held-out
 * values).  Any output may be NULL.  E_STATE unless the job is DONE. */
psgld_status psgld_server_job_result(psgld_server *srv, int64_t id, double *W_mean, double *H_mean,
                                     double *W_var, double *H_var, double *heldout_rmse);

/* Forgets a finished (DONE or FAILED) job and its results. */
psgld_status psgld_server_release(psgld_server *srv, int64_t id);

/* Message of the last failing call on srv (or of a FAILED job). */
const char *psgld_server_last_error(const psgld_server *srv);
const char *psgld_server_job_error(const psgld_server *srv, int64_t id);

/* Waits for the device and frees every job and the server. */
void psgld_server_destroy(psgld_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* PSGLD_H */
