/*
 * fsmmc.h -- C ABI of libfsmmc: FSM-scheduled multi-chain MCMC on AMD
 * MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem (Dance et al.,
 * "Efficiently Vectorized MCMC on Modern Accelerators", ICML 2025):
 *   - a sampler is a map sample: R^d x N -> R^d x N from a state and a
 *     random state to the next state (Sec. 2.1); m chains are the batched
 *     map R^{d x m} x N^m -> R^{d x m} x N^m;
 *   - the FSM runtime advances every chain by FSM steps and collects a draw
 *     whenever a chain passes its final state (Sec. 3.2, Alg. "step function
 *     for FSM", Alg. "FSM MCMC algorithm"; Appendix, Alg. "Vectorized FSM
 *     MCMC algorithm");
 *   - the synchronized runtime draws sample i of every chain before any
 *     chain starts sample i+1 (Appendix, Alg. "Vectorized MCMC algorithm
 *     with vmap(sample)"; Sec. 2.2).
 *
 * Conventions for every call:
 *   - Pointers named "device" are HIP device pointers on the context's
 *     device; "host" pointers are ordinary CPU memory.
 *   - Arrays are dense, row-major, in the job's dtype (FP32 or FP64) unless
 *     stated otherwise.
 *   - Calls return FSMMC_OK or an error code; no exception crosses the ABI.
 *     After an error the message is in fsmmc_last_error() (per thread) and
 *     the job is unchanged unless the text says otherwise.
 *   - Work is queued on the job's stream; a call returns before the device
 *     finishes unless it reports completion (an all_done out-argument) or
 *     says it synchronises.
 *   - Given (target, sampler, seed, x0), the draws are bit-identical whether
 *     produced by fsmmc_step_fsm or fsmmc_step_synchronized, for any split of
 *     the work into calls and for any launch tuning.
 */
#ifndef FSMMC_H
#define FSMMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSMMC_OK = 0,
    FSMMC_EINVAL = 1,   /* bad argument: null pointer, size, kind or dtype        */
    FSMMC_ENOMEM = 2,   /* device allocation failed                               */
    FSMMC_EBUDGET = 3,  /* the job would exceed the context's HBM budget          */
    FSMMC_EDEVICE = 4,  /* a HIP runtime call failed                              */
    FSMMC_EBUSY = 5,    /* the request conflicts with work in flight              */
    FSMMC_ENOTDONE = 6, /* the requested draws are not produced yet               */
    FSMMC_ENOTSUP = 7   /* valid request this build does not implement            */
} fsmmc_status;

/* Targets: the density each chain samples. */
typedef enum {
    FSMMC_GP_GAUSS = 0,    /* latent GP, prior N(0, L L^T), y_i ~ N(f_i, noise_sd^2) */
    FSMMC_GP_LOGISTIC = 1, /* latent GP, prior N(0, L L^T), y_i ~ Bern(sigmoid f_i)   */
    FSMMC_LOGREG = 2,      /* Bayesian logistic regression, prior N(0, I)            */
    FSMMC_FUNNEL = 3,      /* Neal's funnel: v ~ N(0, 9), x_i | v ~ N(0, e^v)        */
    FSMMC_GAUSS_DIAG = 4,  /* N(0, diag(prec)^-1)                                    */
    FSMMC_MOG = 5,         /* mixture of K Gaussians sharing one covariance (Sec. 7.3):
                              pi(x) ∝ sum_k w_k exp(-(x - mu_k)^T P (x - mu_k) / 2)  */
    FSMMC_GP_HYPER = 6     /* GP-regression hyperparameters theta = (tau, lambda, sigma),
                              prior N(0, I), likelihood N(y; 0, tau^2 exp(-lambda^2
                              |x_i - x_k|^2) + (sigma^2 + jitter) I) (Sec. 7.2); ESS, FP64 */
} fsmmc_target_kind;

/* Samplers (Sec. 3.1, Fig. "Finite state machines for the sample function"). */
typedef enum {
    FSMMC_ESS = 0,  /* elliptical slice sampling: INIT, SHRINK, DONE                  */
    FSMMC_NUTS = 1, /* no-U-turn HMC: INIT, DOUBLE, INTEGRATE, CHECK, DONE            */
    FSMMC_DRMH = 2, /* delayed-rejection MH: INIT, PROPOSE, DONE                      */
    FSMMC_DRSYM = 3, /* symmetric delayed rejection (Mira 2001; Sec. 7.1): up to n_stages
                       tries, each proposal N(previous rejected proposal, scales[0]^2 I),
                       accepted with probability min(1, max(0, pi(y) - pi*) / (pi(x) - pi*)),
                       pi* the largest density rejected so far in the draw            */
    FSMMC_SLICE = 4 /* slice sampling along a random direction (Neal 2003): INIT E,
                       EXPAND, INIT S, SHRINK, DONE (Sec. 3.1); scales[0] is the
                       stepping-out width w                                           */
} fsmmc_sampler_kind;

typedef enum { FSMMC_F32 = 0, FSMMC_F64 = 1 } fsmmc_dtype;

/* Synchronized runtime flavours. */
typedef enum {
    FSMMC_SYNC_VMAP = 0,   /* every chain runs max_j N_j loop bodies per draw; the
                              bodies after a chain's own exit are computed and
                              discarded, as a batched while loop does (Sec. 2.2)  */
    FSMMC_SYNC_COMPACT = 1 /* finished chains idle until the draw's barrier        */
} fsmmc_sync_mode;

/* Target description.  All arrays are device pointers in the sampler's dtype;
 * init_chains copies what it needs, so the caller may free them afterwards. */
typedef struct {
    int32_t kind;     /* fsmmc_target_kind                                         */
    int32_t dim;      /* d >= 1                                                    */
    int32_t n_data;   /* LOGREG: number of rows of X; MOG: components K in [1, 8];
                         GP_HYPER: observations n in [1, 512]                     */
    int32_t aux;      /* GP_HYPER: input dimension p in [1, 16]; otherwise 0       */
    const void* X;    /* LOGREG: n_data x dim design matrix; MOG: K x dim means mu_k;
                         GP_HYPER: n_data x aux inputs                            */
    const void* y;    /* GP: dim observations (GAUSS) or labels in {0,1} (LOGISTIC);
                         LOGREG: n_data labels in {0,1}; MOG: K log weights log w_k;
                         GP_HYPER: n_data outputs                                */
    const void* chol_L; /* GP: dim x dim lower Cholesky factor of the prior covariance
                           (entries above the diagonal are ignored)                */
    const void* prec; /* GAUSS_DIAG: dim precisions; MOG: dim x dim precision
                         matrix P (symmetric positive definite), shared by all
                         components                                            */
    double noise_sd;  /* GP_GAUSS: observation noise standard deviation;
                         GP_HYPER: jitter added to the diagonal (>= 0)            */
} fsmmc_target_spec;

/* Sampler description. */
typedef struct {
    int32_t kind;      /* fsmmc_sampler_kind                                        */
    int32_t dtype;     /* fsmmc_dtype                                               */
    int32_t max_depth; /* NUTS: maximum tree depth J in [1, 15] (<= 2^J - 1 leapfrogs) */
    int32_t n_stages;  /* DRMH: number of proposal stages in [1, 3]; DRSYM: maximum
                          number of tries M in [1, 2^20]                          */
    double step_size;  /* NUTS: leapfrog step size > 0                              */
    double scales[4];  /* DRMH: proposal standard deviation of each stage > 0;
                          DRSYM: scales[0] is the proposal standard deviation;
                          SLICE: scales[0] is the stepping-out width > 0         */
} fsmmc_sampler_spec;

/* Launch tuning (0 = library default).  Tuning never changes the draws. */
typedef struct {
    int32_t window;        /* ESS: draws of ellipse directions precomputed per chain */
    int32_t timing;        /* 1: time every kernel launch with HIP events on the job's
                              stream (reported by fsmmc_job_stats)                   */
    int32_t fsm_states;    /* DRSYM: 0 or 1 = condensed FSM (the loop body is one state,
                              one try per step); 4 = the loop body split into four
                              states PROPOSE, EVAL, TEST, NEXT, one per step (Sec.
                              7.1's ablation of bundling); same draws either way  */
    int32_t reserved[5];
} fsmmc_tune;

#define FSMMC_HIST_BINS 1025

typedef struct {
    int64_t steps;        /* FSM steps executed, summed over chains (one step = one
                             evaluation of the expensive quantity g: a log-likelihood,
                             a gradient or a density)                               */
    int64_t padded_steps; /* loop bodies executed and discarded (SYNC_VMAP only)    */
    int64_t draws;        /* draws produced, summed over chains                     */
    int32_t chains_done;  /* chains with all n_draws draws                          */
    int32_t guard_trips;  /* ESS draws stopped by the evaluation guard (expected 0) */
    int32_t launches;     /* kernel launches issued for this job                    */
    int32_t reserved;
    /* With tune.timing = 1: device time (ms) and launch count per kernel class:
     * [0] batched g (ESS ellipse GEMM, NUTS gradient), [1] FSM transition
     * kernels, [2] synchronized-runtime kernels, [3] padding kernels.        */
    double kernel_ms[4];
    int32_t kernel_launches[4];
    /* Loop counts N_ij (Sec. 2.2; Sec. 4, R(m)) over the draws produced so far:
     * hist[b] counts draws with N_ij = b for b < FSMMC_HIST_BINS - 1, the last
     * bin those with N_ij >= FSMMC_HIST_BINS - 1; mean_loops is the mean of
     * N_ij; over the draws i every chain has produced, mean_max_loops is the
     * mean of max_j N_ij and r_hat = mean_max_loops / (the mean of N_ij over
     * those draws): the measured ratio R(m) that bounds the FSM's gain. */
    double mean_loops;
    double mean_max_loops;
    double r_hat;
    /* Lane occupancy.  Lane-per-chain kernels (DRMH, alone or in a batch)
     * count in the kernel: a wave runs its loop body as often as its busiest
     * lane, so it spends 64 lane slots per iteration, of which the lanes whose
     * chain still had work are active.  Wave-per-chain kernels (ESS, NUTS)
     * keep all of a running chain's lanes on its dim coordinates: active =
     * steps * dim, slots = (steps + padded_steps) * dim rounded up to 64. */
    int64_t active_lanes;
    int64_t lane_slots;
    /* NUTS: sum over every leapfrog so far of min(1, exp(H0 - H)) (a
     * divergent or undefined energy counts 0); divided by steps it is the
     * mean acceptance statistic that step-size tuning targets. */
    double accept_sum;
    int64_t hist[FSMMC_HIST_BINS];
} fsmmc_stats;

typedef struct fsmmc_ctx fsmmc_ctx;
typedef struct fsmmc_job fsmmc_job;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory all of its jobs may hold (0 = no bound).  *out receives the
 * context.  Errors: EINVAL (null out, bad device), EDEVICE. */
fsmmc_status fsmmc_ctx_create(int device, size_t hbm_budget_bytes, fsmmc_ctx** out);

/* Destroy a context; every job of it must have been freed (else EBUSY). */
fsmmc_status fsmmc_ctx_destroy(fsmmc_ctx* ctx);

/* Bytes of device memory the context's jobs hold now. */
size_t fsmmc_ctx_bytes_in_use(const fsmmc_ctx* ctx);

/* Create a job of n_chains chains that will each produce n_draws draws, and
 * initialise every chain (Alg. "FSM MCMC algorithm", initialisation: z =
 * init(x0), t = 0, k = S_1).
 *   x0:          device, n_chains x dim initial states, or NULL for the default
 *                start (ESS: a prior draw L z; DRMH on FUNNEL: an exact funnel
 *                draw; otherwise a standard normal draw), keyed by seed.
 *   out_samples: device, n_chains x n_draws x dim buffer the draws are written
 *                to (caller-owned, must outlive the job), or NULL to let the
 *                library allocate it (counted against the budget).
 *   stream:      hipStream_t the job's work is queued on (NULL = default stream).
 *   tune:        launch tuning or NULL.
 * Chain j's random stream is keyed by (seed, j) only.  The call queues the
 * initialisation and returns.  Errors: EINVAL, ENOMEM, EBUDGET, EDEVICE, ENOTSUP. */
fsmmc_status fsmmc_init_chains(fsmmc_ctx* ctx, const fsmmc_target_spec* target,
                               const fsmmc_sampler_spec* sampler, int32_t n_chains,
                               int32_t n_draws, uint64_t seed, const void* x0,
                               void* out_samples, void* stream, const fsmmc_tune* tune,
                               fsmmc_job** out);

/* Advance every unfinished chain by FSM steps (Alg. "Vectorized FSM MCMC
 * algorithm").  A chain stops when it holds n_draws draws or has taken
 * max_steps steps in this call; max_steps <= 0 means run every chain to
 * n_draws.  Each step runs the chain's cheap states back to back until the
 * next evaluation of g and then evaluates g once (Appendix, Alg. "bundled
 * step as input to amortized step"); chains never wait for each other inside
 * the call.  Synchronises the job's stream before returning.  If all_done is
 * not NULL it receives 1 when every chain has n_draws draws, else 0. */
fsmmc_status fsmmc_step_fsm(fsmmc_job* job, int64_t max_steps, int32_t* all_done);

/* fsmmc_step_fsm without waiting: the steps are queued on the job's stream
 * and the call returns; nothing is read back from the device (chains meet
 * only at their n-th draw, Sec. 3.2, so the host need not watch them).  When
 * the queued work has run, *done holds 1 if every chain has n_draws draws,
 * else 0; done must be device memory or pinned host memory (hipHostMalloc),
 * read after fsmmc_job_sync or after an event recorded on the job's stream.
 * The draws are those of fsmmc_step_fsm.  max_steps as there; for NUTS on
 * logistic regression max_steps must be > 0 (the number of runtime steps to
 * the last draw is not known ahead), and the call queues max_steps + 1 of
 * them.  Errors: EINVAL (NULL or pageable done, NUTS without a budget),
 * EBUSY (the job belongs to a batch), EDEVICE. */
fsmmc_status fsmmc_step_fsm_async(fsmmc_job* job, int64_t max_steps, int32_t* done);

/* Produce the next n_draws draws of every chain in lock step: draw i of all
 * chains completes before any chain starts draw i+1 (Appendix, Alg.
 * "Vectorized MCMC algorithm with vmap(sample)").  mode is an
 * fsmmc_sync_mode.  All chains must be at the same draw index and at a draw
 * boundary (EINVAL otherwise).  Synchronises the job's stream.  all_done as
 * for fsmmc_step_fsm. */
fsmmc_status fsmmc_step_synchronized(fsmmc_job* job, int32_t n_draws, int32_t mode,
                                     int32_t* all_done);

/* Copy draws [draw_begin, draw_end) of every chain to dst, laid out
 * n_chains x (draw_end - draw_begin) x dim; dst is host memory if dst_is_host
 * is non-zero, else device memory.  Synchronises the job's stream.  Errors:
 * EINVAL (range), ENOTDONE (a chain has not produced draw_end - 1 yet). */
fsmmc_status fsmmc_collect_samples(fsmmc_job* job, int32_t draw_begin, int32_t draw_end,
                                   void* dst, int32_t dst_is_host);

/* Copy the per-draw loop counts N_ij (ESS: log-likelihood evaluations; NUTS:
 * leapfrog steps; DRMH: stages) to host memory dst, n_chains x n_draws int32
 * (Sec. 2.2, "Formalizing the problem").  Synchronises the job's stream. */
fsmmc_status fsmmc_collect_counts(fsmmc_job* job, int32_t* dst);

/* Evaluate the job's target at n_points positions with the same kernels the
 * sampler uses (NUTS jobs: the potential U = -log pi and its gradient).
 *   theta: device, n_points x dim positions (n_points <= n_chains);
 *   grad:  device, n_points x dim output, or NULL;
 *   U:     device, n_points output.
 * Uses the job's scratch buffers: call it only between stepping calls.
 * Synchronises the job's stream.  Errors: EINVAL, ENOTSUP (ESS jobs). */
fsmmc_status fsmmc_eval_potential(fsmmc_job* job, int32_t n_points, const void* theta, void* grad,
                                  void* U);

/* Size of the device workspace of fsmmc_eval_potential_noalloc: one fixed
 * array per device, held from the first context on that device until the
 * process ends. */
#define FSMMC_NOALLOC_SCRATCH_BYTES (8u << 20)

/* fsmmc_eval_potential for callers that cannot allocate device memory (code
 * under stream or graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same bits, but the padded results go
 * through the library's fixed per-device workspace instead of buffers
 * allocated per call, and the call does not synchronise.
 *   theta: device, n_points x dim positions (n_points <= n_chains);
 *   grad:  device, n_points x dim output, or NULL;
 *   U:     device, n_points output.
 * Everything is queued on the job's stream; the outputs are ready when that
 * stream reaches this point (fsmmc_job_sync).  Calls no hipMalloc, hipFree,
 * memset or allocating routine.  Limit: n_points * (dim rounded up to 64, + 1)
 * * 4 bytes <= FSMMC_NOALLOC_SCRATCH_BYTES (16256 points at dim 100), else
 * EINVAL.  Every call on one GPU shares the workspace (and uses the job's
 * request and partial buffers, like fsmmc_eval_potential), so calls that may
 * overlap on one GPU -- other streams, other threads -- race and must be
 * ordered by the caller.  Nothing in the workspace needs to start at zero:
 * each call writes every entry it reads.  Errors: EINVAL, ENOTSUP (not a
 * NUTS job), EBUSY (job in a batch or server), EDEVICE. */
fsmmc_status fsmmc_eval_potential_noalloc(fsmmc_job* job, int32_t n_points, const void* theta,
                                          void* grad, void* U);

/* Per-chain draw counters t_j (host dst, n_chains uint32).  Synchronises. */
fsmmc_status fsmmc_chain_progress(fsmmc_job* job, uint32_t* dst);

/* Counters of the job so far.  Synchronises the job's stream. */
fsmmc_status fsmmc_job_stats(fsmmc_job* job, fsmmc_stats* out);

/* Block until the job's queued work has finished. */
fsmmc_status fsmmc_job_sync(fsmmc_job* job);

/* Release a job and its device memory (waits for its queued work first). */
fsmmc_status fsmmc_job_free(fsmmc_job* job);

/* ---------------------------------------------------------------- batching
 * A batch steps several jobs together, possibly of different samplers,
 * targets, dimensions, chain counts and draw counts (FP32 jobs of any
 * sampler).  One round is one replay of a captured hipGraph whose kernels
 * serve every job at once:
 *   - a grouped ellipse GEMM: the next `window` directions nu = L z of every
 *     ESS chain, all jobs' column blocks in one launch per tile shape;
 *   - one persistent FSM kernel: its wavefronts take work items from a
 *     device queue, longest first -- one ESS chain for `window` draws, or 64
 *     DRMH chains (one per lane) for `dr_chunk` draws -- and run the chains'
 *     FSM steps (Sec. 3.2, Alg. "Vectorized FSM MCMC algorithm") without
 *     waiting for any other chain or job;
 *   - `nuts_steps` NUTS runtime steps of every NUTS job: grouped transition
 *     (which adds up the gradient's row-slice partials it consumes), per-job
 *     request compaction and grouped gradient tiles.
 * Chains of a job never synchronise with other jobs, and a job's draws are
 * bit-identical to running it alone with fsmmc_step_fsm.  While a job
 * belongs to a batch, the per-job stepping calls and fsmmc_job_free return
 * EBUSY. */
typedef struct fsmmc_batch fsmmc_batch;

typedef struct {
    int32_t autotune;        /* 1: choose window, dr_chunk and gemm_cols from measured
                                rounds (the tuning rounds do real work)              */
    int32_t window;          /* ESS draws per chain per round (0 = 16), capped by the
                                direction buffer each job was created with           */
    int32_t dr_chunk;        /* DRMH draws per chain per round (0 = 16)              */
    int32_t gemm_cols;       /* ellipse GEMM columns per block, 64 or 128 (0 = 64;
                                128 applies to FP32 jobs with dim <= 256)            */
    int32_t rounds_per_sync; /* graph replays between progress reads (0 = 4)         */
    int32_t nuts_steps;      /* NUTS runtime steps per round (0 = 16)                */
    int32_t reserved[2];
} fsmmc_batch_tune;

typedef struct {
    int64_t rounds;      /* graph replays                                           */
    int64_t captures;    /* graphs captured (start, after jobs finish, tuning)      */
    int64_t draws;       /* draws produced by the batch, summed over jobs and chains */
    int32_t window;      /* configuration in use                                     */
    int32_t dr_chunk;
    int32_t gemm_cols;
    int32_t live_jobs;   /* jobs with a chain short of its n_draws                  */
    double gpu_ms;       /* device time of all replays (HIP events on the stream)   */
    double tune_ms;      /* part of gpu_ms spent in autotuning rounds               */
    int32_t tune_trials; /* configurations the autotuner measured                   */
    int32_t fsm_blocks;  /* workgroups of the persistent FSM kernel                 */
} fsmmc_batch_counters;

/* Group n_jobs jobs of context ctx into a batch stepped on `stream`
 * (hipStream_t; NULL = a stream the batch creates).  The jobs must be FP32
 * jobs not already in a batch; their queued initialisation is waited for.
 * Errors: EINVAL (null or repeated job, other context, bad tuning value),
 * ENOTSUP (FP64 job), EBUSY (job in another batch), EDEVICE. */
fsmmc_status fsmmc_batch_create(fsmmc_ctx* ctx, fsmmc_job* const* jobs, int32_t n_jobs,
                                void* stream, const fsmmc_batch_tune* tune,
                                fsmmc_batch** out);

/* Replay rounds until every chain of every job has its n_draws draws, or
 * max_rounds rounds have run (max_rounds <= 0: no limit).  Synchronises the
 * batch's stream.  all_done (may be NULL) receives 1 when every job is
 * complete. */
fsmmc_status fsmmc_batch_run(fsmmc_batch* batch, int64_t max_rounds, int32_t* all_done);

/* Counters and the configuration in use. */
fsmmc_status fsmmc_batch_stats(fsmmc_batch* batch, fsmmc_batch_counters* out);

/* Release the batch (not its jobs, which become free-standing again). */
fsmmc_status fsmmc_batch_free(fsmmc_batch* batch);

/* ---------------------------------------------------------------- serving
 * A server runs sampling jobs submitted at any time, with continuous
 * batching: a request loop in a thread of its own admits submitted jobs in
 * arrival order as the context's HBM budget allows (their chain state is
 * allocated on the device at admission and stays there), steps every
 * admitted job together in the rounds of one shared batch, and retires a
 * job as soon as its last chain has its last draw -- in the middle of the
 * stream, while other jobs keep running -- which frees its memory for the
 * next admission.  Because chains only meet their own job at its n-th draw
 * (Sec. 3.2), retiring a job never waits for any other job.  A job's draws
 * are bit-identical to running it alone with fsmmc_step_fsm. */
typedef struct fsmmc_server fsmmc_server;

typedef struct {
    fsmmc_batch_tune batch; /* round shape of the shared batch (autotune is ignored)  */
    int32_t ess_window;     /* direction buffer of an admitted ESS job, in draws per
                               chain (0 = 16); bounds its memory to chains x window x
                               dim floats                                             */
    int32_t reserved[7];
} fsmmc_server_config;

/* One finished job, as reported by fsmmc_server_poll. */
typedef struct {
    uint64_t job_id;
    int32_t status;   /* FSMMC_OK, or the error that ended the job (EBUDGET: the job
                         alone exceeds the context's budget)                         */
    int32_t reserved;
    double t_submit;  /* fsmmc_clock() at submission, admission and completion        */
    double t_admit;
    double t_done;
} fsmmc_server_done;

typedef struct {
    int64_t submitted, admitted, completed, failed;
    int64_t rounds;      /* graph replays                                          */
    int64_t draws;       /* draws produced, all jobs                               */
    int32_t live_jobs;   /* admitted, not yet retired                              */
    int32_t pending_jobs;/* submitted, waiting for admission                       */
    int32_t peak_live_jobs;
    int32_t reserved;
    uint64_t peak_bytes; /* peak device bytes held by admitted jobs                */
    double gpu_ms;       /* device time of the rounds                              */
} fsmmc_server_counters;

/* Monotonic host clock (seconds) the server stamps its records with. */
double fsmmc_clock(void);

/* Start a server on context ctx (its HBM budget bounds the admitted jobs'
 * state).  cfg may be NULL.  Errors: EINVAL, EDEVICE. */
fsmmc_status fsmmc_server_create(fsmmc_ctx* ctx, const fsmmc_server_config* cfg, fsmmc_server** out);

/* Queue a job (same arguments as fsmmc_init_chains; FP32 only).  Returns at
 * once with *job_id.  The target arrays and x0 must stay valid, and
 * out_samples (device, n_chains x n_draws x dim, required) and out_counts
 * (device, n_chains x n_draws int32 loop counts, or NULL) untouched, until
 * the job is reported finished.  Errors: EINVAL, ENOTSUP (checked at once),
 * EDEVICE (the server stopped after a device error). */
fsmmc_status fsmmc_server_submit(fsmmc_server* srv, const fsmmc_target_spec* target,
                                 const fsmmc_sampler_spec* sampler, int32_t n_chains,
                                 int32_t n_draws, uint64_t seed, const void* x0,
                                 void* out_samples, int32_t* out_counts, uint64_t* job_id);

/* Move up to cap finished-job records into out (host array); *n_out
 * receives how many.  Records are returned once, in completion order. */
fsmmc_status fsmmc_server_poll(fsmmc_server* srv, fsmmc_server_done* out, int32_t cap,
                               int32_t* n_out);

/* Block until every submitted job has finished or timeout_s seconds have
 * passed (timeout_s < 0: no limit); *idle (may be NULL) receives 1 if no
 * job is pending or running. */
fsmmc_status fsmmc_server_wait(fsmmc_server* srv, double timeout_s, int32_t* idle);

fsmmc_status fsmmc_server_stats(fsmmc_server* srv, fsmmc_server_counters* out);

/* Finish every submitted job, stop the request loop and release the server. */
fsmmc_status fsmmc_server_destroy(fsmmc_server* srv);

/* Message of the last error on the calling thread ("" if none). */
const char* fsmmc_last_error(void);

/* Library version string. */
const char* fsmmc_version(void);

/* ---------------------------------------------------------------- ceilings
 * Measured rates of the units the hot path runs on, to set beside the
 * spec-sheet peaks its rooflines are quoted against (the paper reports
 * throughput only; these are the denominators of the roofline fractions).  */
typedef struct {
    double hbm_copy_gbps;    /* device-to-device copy: (read + write bytes) / s, 1e9 units      */
    double mfma_bf16_tflops; /* v_mfma_f32_32x32x16_bf16 with independent accumulators          */
    double mfma_f32_tflops;  /* v_mfma_f32_32x32x2_f32                                           */
    double valu_f32_tflops;  /* vector FP32 FMA, unpacked (this library never emits packed FP32) */
    double valu_f64_tflops;  /* vector FP64 FMA                                                  */
    double exp_f32_gops;     /* hardware exp2 results per second, 1e9 units                      */
    int32_t cus;             /* compute units                                                    */
    int32_t clock_mhz;       /* peak engine clock reported by the runtime                        */
} fsmmc_ceilings;

/* Run the measurement kernels on `device` (about a second) and fill *out.
 * copy_bytes: size of each of the two copy buffers (>= 64 MiB, a multiple of
 * 16); the call allocates and frees them and a small result buffer, and
 * synchronises the device.  Errors: EINVAL, EDEVICE (including out of memory). */
fsmmc_status fsmmc_measure_ceilings(int device, size_t copy_bytes, fsmmc_ceilings* out);

#ifdef __cplusplus
}
#endif

#endif /* FSMMC_H */
