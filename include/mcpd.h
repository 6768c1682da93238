/*
 * mcpd.h -- C ABI of the MI355X unbiased Markov chain pool decoder.
 *
 * The library estimates every clone's posterior positive probability
 * p_i = E_pi[Z_i] under the pooled-test posterior
 *   pi(z | y) ~ prod_i q^{z_i} (1-q)^{1-z_i} prod_j Pr{y_j | xi_j(z)}
 * (paper, Section "Knill's Method") with lag-1 coupled pairs of the
 * score-weighted random-scan Gibbs sampler (Section "Coupled Score-Weighted
 * Update Gibbs Sampler", Algorithm 3), the time-averaged estimator H_{k:l}
 * (Section "Coupled Estimator and Fixed-Budget GPU Execution"), and
 * fixed-budget logical slots with refill and the completion-time-corrected
 * equal-weight aggregate (Algorithm 4, Theorem 2).
 *
 * Conventions for every entry point:
 *   - Plain C types only.  Pointers marked "host" are read or written by the
 *     CPU; the library copies inputs at the call and never keeps caller
 *     pointers.  Outputs are caller-allocated.
 *   - Return value 0 (MCPD_OK) on success, a negative MCPD_E* code otherwise;
 *     mcpd_strerror() names the code and mcpd_last_error() gives the detail
 *     of the last failure on the calling thread.  No C++ exception crosses
 *     the ABI.  On error, outputs are unspecified.
 *   - One instance is not thread-safe; separate instances may be used from
 *     separate threads on separate streams.
 *   - Results are a pure function of (instance, weights, budget, slots, k, m,
 *     seed, options): they do not depend on launch geometry or timing.
 */
#ifndef MCPD_H
#define MCPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCPD_OK 0
#define MCPD_EINVAL (-1)   /* invalid argument (see each function)              */
#define MCPD_ENOMEM (-2)   /* host or device allocation failed                   */
#define MCPD_EDEVICE (-3)  /* HIP runtime error or no usable gfx950 device       */
#define MCPD_ECAP (-4)     /* strict_cap set and a retained pair hit the cap     */

#define MCPD_MAX_DEGREE 12          /* pools per clone                          */
#define MCPD_MAX_POOL_SIZE 255      /* clones per pool                          */
#define MCPD_MAX_CLONES (1 << 24)

typedef struct mcpd_instance mcpd_instance;
typedef struct mcpd_batch mcpd_batch;

/* Run options.  Initialise with mcpd_run_opts_init() and override fields. */
typedef struct mcpd_run_opts {
    uint64_t max_steps;     /* meeting cap: 0 = none (hard limit 2^32-1 draws);
                               else >= max(m,1): a pair not met after
                               max(max_steps, m) draws stops with the truncated
                               estimator and counts in cap_hits               */
    uint32_t refill;        /* 1 = slot refill (default); 0 = one pair per slot */
    uint32_t strict_cap;    /* 1 = return MCPD_ECAP if a retained pair was capped */
    uint32_t hist_bins;     /* meeting-time histogram bins (default 64)       */
    uint32_t hist_width;    /* draws per bin (default 0 = n, one sweep)        */
    uint32_t u_hi_bits;     /* bits of U taken from the main random block
                               (default 32; 1..32; lower values only serve to
                               exercise the low-bit refinement in tests)      */
    uint32_t instance_id;   /* g of the random-number counter (< 2^24), default
                               0; in a batch, instance i uses instance_id + i */
    uint32_t plan;          /* placement (results never depend on it): 0 = auto
                               per instance, 1 = chain state and tables in LDS,
                               2 = state in LDS and tables in global memory,
                               3 = state in global memory and tables in LDS,
                               4 = both global; a plan that does not fit returns
                               MCPD_EINVAL                                    */
    uint32_t wg_per_cu;     /* workgroups of 256 lanes per compute unit (0 = auto,
                               at most 8)                                       */
    uint32_t ticket_slots;  /* slots per lane that one work ticket stands for
                               (0 = auto; a ticket sends one workgroup to one
                               instance)                                      */
    uint32_t use_graph;     /* batches: 1 = replay a captured HIP graph
                               (default), 0 = plain stream launches           */
    uint32_t keep_slot_records; /* batches: keep N*_p and S_p of every slot on
                               the device for mcpd_batch_slot_records         */
    uint32_t narrow_lanes;  /* least lanes of a narrow LDS layout, in which a
                               workgroup runs only as many slots as fit their
                               chain state in LDS: 0 = default (8), 256 = wide
                               layouts only (state in LDS for 256 lanes or in
                               global memory)                                 */
    uint32_t bucket_rows;   /* rows provided in bucket_sum / bucket_sumsq; must
                               be >= the largest N*                            */
    uint32_t kernel;        /* 0 = auto: the cooperative kernel when every
                               instance's chain states fit it, else the lane
                               kernel; 1 = lane kernel (one slot per lane);
                               2 = cooperative kernel (one slot per group of
                               lanes, one speculative draw per lane and step),
                               MCPD_EINVAL if the states do not fit           */
    uint32_t group_lanes;   /* cooperative kernel: lanes per slot, 8, 16, 32 or
                               64 for every instance; 0 = each instance its
                               own: the least of 16, 32 and 64 whose layout
                               keeps the instance's tables in LDS, else the
                               least whose chain states fit               */
    uint32_t init_mode;     /* initial distribution nu of every pair (Algorithm
                               3: Z_0 ~ nu, X_0 = Y_0 = Z_0): 0 = all-negative
                               state (default); 1 = the prior, clones
                               independent with Pr{Z_0,i = 1} = floor(q 2^32)
                               / 2^32, clone i drawn from word i mod 4 of the
                               Philox block with counter (floor(i/4), r, p,
                               g + 2^25); MCPD_EINVAL otherwise               */
    uint32_t cap_sweeps;    /* meeting cap in sweeps of each instance: a pair not
                               met after max(cap_sweeps * n, m) draws stops as
                               with max_steps (the paper's runs cap at 20
                               sweeps); 0 = none; MCPD_EINVAL together with
                               max_steps or when cap_sweeps * n >= 2^32     */
    uint32_t first_slot;    /* global index of the run's first slot in the
                               random-number counter (default 0): the run
                               covers slots first_slot .. first_slot+slots-1
                               of a larger run at the same horizon B, so a run
                               split into such shares (say one per GPU) has
                               integer sums, histogram and counters that add
                               up exactly to the whole run's; slot records
                               are indexed from the first slot;
                               MCPD_EINVAL if first_slot + slots > 2^32     */
    uint32_t keep_mismatch; /* batches: count the mismatch times of every
                               instance for mcpd_batch_mismatch (single runs
                               count them when `mismatch` is given); off by
                               default, since their events cost device-wide
                               atomics on the few clones most pairs disagree on */
    uint32_t reserved0;     /* set to 0                                        */
    /* Optional host outputs of mcpd_run_unbiased (NULL = not wanted; must be
       NULL for batches). */
    uint32_t *slot_nstar;   /* [slots] N*_p(B)                                 */
    uint64_t *slot_units;   /* [slots] S_p(N*): progress units of the retained  */
    int64_t *bucket_sum;    /* [bucket_rows * n] sum of V_pj over slots with
                               N*_p = row+1 (V = W * slot numerator, exact)     */
    uint64_t *bucket_sumsq; /* [bucket_rows * n * 2] (low, high) words of the
                               128-bit sum of V_pj^2, same grouping            */
    uint64_t *mismatch;     /* host, [n] or NULL (mcpd_run_unbiased only): the
                               mismatch time of every clone, summed over the
                               retained replications of every slot: the number
                               of time indices s = 1..C at which
                               x_j(s) != y_j(s-1), i.e. how long the pair spent
                               apart at clone j before it met (Algorithm 3);
                               for batches see mcpd_batch_mismatch             */
} mcpd_run_opts;

/* Run statistics of one instance (all integers exact). */
typedef struct mcpd_run_stats {
    uint64_t progress_units;      /* draws executed on the device, including
                                     the replayed draws of rolled-back pairs   */
    uint64_t retained_units;      /* sum of C over retained pairs               */
    uint64_t single_site_updates; /* over retained pairs                        */
    uint64_t reps_started;        /* pairs started (retained + aborted)         */
    uint64_t reps_retained;
    uint64_t reps_aborted;        /* started pairs stopped because they could no
                                     longer be retained (then rolled back)      */
    uint64_t cap_hits;            /* retained pairs stopped by the cap          */
    uint64_t zero_completion_slots; /* slots whose first pair ended beyond B   */
    uint64_t tau_sum;             /* over retained, met pairs                   */
    uint64_t tau_max;
    uint64_t nstar_max;           /* largest N*_p                               */
    uint64_t rollback_units;      /* draws replayed to roll back aborted pairs  */
    uint64_t list_overflows;      /* slots whose touched-clone list overflowed
                                     (their numerators were flushed by a scan)  */
    uint64_t lanes;               /* persistent lanes of the launch             */
    uint32_t placement;           /* bit 0: chain state in LDS; bit 1: tables in
                                     LDS; bit 2: cooperative kernel; bit 3:
                                     threshold table alone in LDS (alias table
                                     and rows in global memory)                 */
    uint32_t wg_per_cu;           /* workgroups per CU of the launch            */
    uint32_t wg_slots;            /* slots a workgroup runs at once for this
                                     instance: 256 lanes (fewer in a narrow
                                     layout), or 256 / group_lanes groups
                                     (cooperative)                              */
    uint32_t kernel;              /* 1 = lane kernel, 2 = cooperative kernel    */
    uint32_t group_lanes;         /* lanes per slot (1 for the lane kernel)     */
    uint32_t reserved;
    double kernel_ms;             /* device time: the sampler launch, or for a
                                     batch replayed as a graph the whole replay
                                     (key copy, zeroing, sampler, copy back)   */
} mcpd_run_stats;

/* One measured configuration of mcpd_batch_tune. */
typedef struct mcpd_tune_entry {
    uint32_t wg_per_cu;
    uint32_t ticket_slots;
    uint32_t narrow_lanes;        /* least lanes of a narrow LDS layout (0 = wide
                                     layouts only)                              */
    uint32_t kernel;              /* 1 = lane kernel, 2 = cooperative kernel    */
    uint32_t group_lanes;         /* lanes per slot (1 for the lane kernel), or
                                     with per_instance the least an instance
                                     may take                                   */
    uint32_t per_instance;        /* 1 = group sizes chosen per instance (as
                                     group_lanes = 0 of mcpd_run_opts does)     */
    double ms;                    /* sampler time of one full run               */
} mcpd_tune_entry;

/* Defaults: no cap, refill on, 64 bins of n draws, u_hi_bits 32, id 0,
 * automatic placement and launch shape, graphs on for batches. */
void mcpd_run_opts_init(mcpd_run_opts *opts);

/* Score weights of the paper (Section "Score-Weighted Update Gibbs Sampler"):
 * d_j pool sizes, a_j = log Pr{y_j|xi=1} - log Pr{y_j|xi=0},
 * s_i = sum_{j in P(i)} d_j a_j, gamma = 100 n,
 * tau_w = log gamma / (s_max - s_min) (0 if equal),
 * w_i = (1/2) softmax(tau_w s)_i + 1/(2n).
 * Host-only, needs no device.  Arguments as for mcpd_create; s_out may be
 * NULL; w_out [n] host.  Errors: MCPD_EINVAL for an invalid design. */
int mcpd_score_weights(int32_t n_clones, int32_t n_pools, const int32_t *row_ptr,
                       const int32_t *pool_idx, const uint8_t *outcomes, double fp,
                       double fn, double prior, double *s_out, double *w_out);

/* Pruning by the naive ranking (Section "Knill's Method": R_i, the product
 * over the clone's pools of Pr{y_j|xi=1} / Pr{y_j|xi=0}; Section
 * "Score-Weighted Update Gibbs Sampler": eta_i = log{q/(1-q)} + log R_i).
 * Clones are ranked by log R_i, evaluated as n+_i a+ + n-_i a- in FP64
 * (n+_i, n-_i: the clone's pools with y = 1 and y = 0; a+, a- as in
 * mcpd_score_weights), so clones with equal counts tie exactly; ties go to
 * the lower index.  The top n_active clones are retained; every other clone
 * is fixed to 0, which makes the pruned posterior the posterior of the
 * design restricted to the retained clones (all pools kept, prior
 * unchanged): build that instance with mcpd_create.
 *   design arguments as for mcpd_create (prior is not needed)
 *   n_active  1..n_clones
 *   active    host [n_active] out: the retained clones in ascending order
 * Host-only, needs no device.  Errors: MCPD_EINVAL. */
int mcpd_prune(int32_t n_clones, int32_t n_pools, const int32_t *row_ptr,
               const int32_t *pool_idx, const uint8_t *outcomes, double fp, double fn,
               int32_t n_active, int32_t *active);

/* Create an instance: the pooling design A as a clone->pool CSR and the
 * observed pool outcomes y (Section "Knill's Method").
 *   n_clones, n_pools  > 0 (n_clones <= MCPD_MAX_CLONES, n_pools <= 32767)
 *   row_ptr   host [n_clones+1], row_ptr[0] = 0, non-decreasing
 *   pool_idx  host [row_ptr[n]], strictly ascending within each row, in
 *             [0, n_pools); at most MCPD_MAX_DEGREE per clone and at most
 *             MCPD_MAX_POOL_SIZE clones per pool
 *   outcomes  host [n_pools], each 0 or 1
 *   fp, fn, prior in (0,1) (Assumption 1 needs 0 < q, alpha, beta < 1)
 *   hip_stream  hipStream_t to order all device work, NULL = default stream
 *   out       receives the handle
 * The instance starts with the paper's score weights, copies its inputs to
 * device memory and owns them until mcpd_destroy.  Errors: MCPD_EINVAL,
 * MCPD_ENOMEM, MCPD_EDEVICE. */
int mcpd_create(int32_t n_clones, int32_t n_pools, const int32_t *row_ptr,
                const int32_t *pool_idx, const uint8_t *outcomes, double fp, double fn,
                double prior, void *hip_stream, mcpd_instance **out);

/* Replace the selection weights (Assumption 1: fixed before the chains
 * start, positive).  w: host [n], finite and > 0 (normalised internally);
 * NULL restores the score weights.  The sampled weights are the integer
 * masses M_i / 2^32 with sum M_i = 2^32 (see mcpd_get_weights).
 * Errors: MCPD_EINVAL (non-positive or non-finite weight), MCPD_EDEVICE. */
int mcpd_set_weights(mcpd_instance *inst, const double *w);

/* The weights actually sampled: w_exact [n] host = M_i / 2^32 (may be NULL),
 * mass [n] host = M_i (may be NULL; M_i >= 1, sum 2^32). */
int mcpd_get_weights(const mcpd_instance *inst, double *w_exact, uint64_t *mass);

/* Run the fixed-budget unbiased estimator (Algorithm 4 over Algorithm 3).
 *   budget   total progress units (one coupled draw = one unit); the per-slot
 *            horizon is B = floor(budget / slots); 0 = one pair per slot
 *   slots    P >= 1 logical slots
 *   k, m     averaging window k:m (the paper's k:l), 0 <= k <= m <= 2^31
 *   seed     64-bit key of the counter-based random numbers
 *   opts     NULL = defaults
 *   marginals host [n]: (1/P) sum_p A_p (the completion-time-corrected
 *            aggregate); stderr_out host [n]: sd_p(A_p)/sqrt(P) (NaN if P=1);
 *   hist     host [opts->hist_bins] meeting-time histogram of retained pairs
 *            (may be NULL); stats may be NULL.
 * Errors: MCPD_EINVAL, MCPD_ENOMEM, MCPD_EDEVICE, MCPD_ECAP. */
int mcpd_run_unbiased(mcpd_instance *inst, uint64_t budget, uint32_t slots, uint32_t k,
                      uint32_t m, uint64_t seed, const mcpd_run_opts *opts, double *marginals,
                      double *stderr_out, uint64_t *hist, mcpd_run_stats *stats);

/* mcpd_run_unbiased with the outputs left in device memory (the same
 * estimator, Algorithm 4 over Algorithm 3; the aggregate of Section
 * "Coupled Estimator and Fixed-Budget GPU Execution"): the marginals and
 * standard errors are formed on the device in FP64 from the same integer
 * sums (mcpd_run_unbiased forms them on the host in extended precision, so
 * the two agree to rounding), the histogram is copied device to device.
 *   marginals_dev  device [n] (required), stderr_dev device [n] or NULL,
 *   hist_dev       device [hist_bins] or NULL; all on the instance's device,
 *                  owned by the caller, written in order on the instance's
 *                  stream
 *   stats          host, may be NULL
 * Returns once the outputs are written.  Slot records and buckets (host
 * outputs) are not accepted here.  Errors as mcpd_run_unbiased. */
int mcpd_run_unbiased_dev(mcpd_instance *inst, uint64_t budget, uint32_t slots, uint32_t k,
                          uint32_t m, uint64_t seed, const mcpd_run_opts *opts, double *marginals_dev,
                          double *stderr_dev, uint64_t *hist_dev, mcpd_run_stats *stats);

/* Release the instance and its device memory (NULL is a no-op).  Destroy
 * every batch that holds the instance first. */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the run of
 * mcpd_run_unbiased_dev with every device buffer it needs carved from one
 * static device array of MCPD_NOALLOC_SCRATCH_BYTES per device, which the
 * library holds until the process ends; the call itself allocates nothing
 * (no hipMalloc, hipHostMalloc or event creation).  Same arguments, outputs
 * and errors as mcpd_run_unbiased_dev; results are bit-identical to it
 * (the grid shrinks to what the array holds, and results never depend on
 * the grid).  stats->kernel_ms is 0 (the call keeps no timing events).
 * The first call on a device looks up the array's address there.  Every
 * call on one device shares that device's array: calls that overlap in
 * time on one device race and must be serialised by the caller.  A run
 * whose buffers for a single workgroup exceed the array (for example
 * n_clones x 8 bytes of numerator row per group of lanes, roughly above
 * 10^6 clones) returns MCPD_EINVAL naming the size it needs. */
#define MCPD_NOALLOC_SCRATCH_BYTES (256u << 20)
int mcpd_run_unbiased_dev_noalloc(mcpd_instance *inst, uint64_t budget, uint32_t slots, uint32_t k,
                                  uint32_t m, uint64_t seed, const mcpd_run_opts *opts, double *marginals_dev,
                                  double *stderr_dev, uint64_t *hist_dev, mcpd_run_stats *stats);

void mcpd_destroy(mcpd_instance *inst);

/* Batches: many instances, each with its own run parameters, in ONE
 * persistent launch (Algorithm 4 for every instance; slots of different
 * instances are independent, so they share the device freely).
 *   insts    host [count] instances (kept by the caller, not copied; they
 *            must outlive the batch and keep their weights while it runs)
 *   budget, slots, k, m   host [count] per-instance run parameters, as in
 *            mcpd_run_unbiased
 *   opts     shared options (NULL = defaults); instance i draws its random
 *            numbers with g = opts->instance_id + i, so it gives exactly what
 *            mcpd_run_unbiased gives with instance_id = opts->instance_id + i
 *   hip_stream  stream of the batch's device work (NULL = a stream the batch
 *            creates; graphs cannot be captured on the legacy default stream)
 * Creation plans the launch: the kernel, the row format, each instance's
 * placement in LDS, the work tickets (longest slots first) and the
 * workspace; the first
 * run captures the device work of a run in a HIP graph (use_graph = 1) that
 * later runs replay.  Errors: MCPD_EINVAL, MCPD_ENOMEM, MCPD_EDEVICE. */
int mcpd_batch_create(mcpd_instance *const *insts, int32_t count, const uint64_t *budget,
                      const uint32_t *slots, const uint32_t *k, const uint32_t *m,
                      const mcpd_run_opts *opts, void *hip_stream, mcpd_batch **out);

/* Run every instance of the batch with key `seed`.  marginals, stderr_out,
 * hist: host arrays of count pointers (each as in mcpd_run_unbiased; the
 * arrays, or any of their entries, may be NULL); stats: host [count] or NULL.
 * Errors: MCPD_EINVAL, MCPD_EDEVICE, MCPD_ECAP (strict_cap). */
int mcpd_batch_run(mcpd_batch *batch, uint64_t seed, double *const *marginals,
                   double *const *stderr_out, uint64_t *const *hist, mcpd_run_stats *stats);

/* Autotuner: run the batch twice (seeds seed and seed + 1) per candidate
 * launch shape (kernel x workgroups per CU x slots per ticket x LDS layout,
 * within opts' fixed values), time the sampler, keep the fastest mean (the
 * entries' ms is that mean).  Lane kernel layouts: wide
 * only (chain state in LDS for 256 lanes when it fits, else in global
 * memory), or also narrow (a workgroup runs only as many lanes as fit the
 * state in LDS, at least 8); cooperative kernel: one state per group of 8,
 * 16, 32 or 64 lanes.
 * The results do not depend on the shape.  entries: host [cap] or NULL;
 * count receives the number of candidates measured. */
int mcpd_batch_tune(mcpd_batch *batch, uint64_t seed, mcpd_tune_entry *entries, uint32_t cap,
                    uint32_t *count);

/* The batch's current launch shape; placement and wg_slots: host [count] or
 * NULL (as in mcpd_run_stats). */
int mcpd_batch_config(const mcpd_batch *batch, uint32_t *wg_per_cu, uint32_t *ticket_slots,
                      uint32_t *lanes, uint32_t *placement, uint32_t *wg_slots);

/* Integer bucket sums of instance `index` from the last run, laid out as
 * opts.bucket_sum / bucket_sumsq of mcpd_run_unbiased (host [rows * n] and
 * [rows * n * 2]; either may be NULL). */
int mcpd_batch_buckets(const mcpd_batch *batch, int32_t index, uint32_t rows, int64_t *sum,
                       uint64_t *sumsq);

/* N*_p and S_p of every slot of instance `index` from the last run (host
 * [slots]; either may be NULL).  Needs opts.keep_slot_records at creation. */
int mcpd_batch_slot_records(mcpd_batch *batch, int32_t index, uint32_t *nstar, uint64_t *units);

/* Mismatch times of instance `index` of the last batch run (host, n values;
 * as mcpd_run_opts.mismatch).  Needs opts.keep_mismatch at creation.
 * Errors: MCPD_EINVAL (null, index out of range, not kept). */
int mcpd_batch_mismatch(const mcpd_batch *batch, int32_t index, uint64_t *out);

/* Release a batch (NULL is a no-op); the instances stay. */
void mcpd_batch_destroy(mcpd_batch *batch);

/* One-shot batch: create, run once, destroy. */
int mcpd_run_batch(mcpd_instance *const *insts, int32_t count, const uint64_t *budget,
                   const uint32_t *slots, const uint32_t *k, const uint32_t *m, uint64_t seed,
                   const mcpd_run_opts *opts, double *const *marginals, double *const *stderr_out,
                   uint64_t *const *hist, mcpd_run_stats *stats);

/* ------------------------------------------------------------------------
 * Learned selection weights.  Any positive weights fixed before the chains
 * start keep pi invariant (Proposition 1) and the estimator unbiased
 * (Theorem 1), so they may be chosen by a small network from per-clone
 * features; the score weights stay the fallback.
 *
 * Base logits: c_i = tau_w (s_i - s_max), the log-weights of the softmax
 * part of the score weights (s, tau_w as in mcpd_score_weights; c = 0 if all
 * scores are equal).
 * Features (8 per clone, FP32): #positive pools / 8, #negative pools / 8,
 * mean size of the positive pools / 64, mean size of the negative pools / 64,
 * smallest positive pool / 64 (the three are 0 without such pools), c_i / 16,
 * 10 fp, 10 fn.
 * Network: f = W3 relu(W2 relu(W1 x + b1) + b2) + b3, widths 8-64-64-1,
 * MCPD_MLP_PARAMS parameters laid out flat as W1 [64][8] (out, in), b1 [64],
 * W2 [64][64], b2 [64], W3 [64], b3.  An FP32 master copy is trained; the
 * kernels compute in FP32 with its BF16 rounding (nearest, ties to even).
 * Weights: w = (1 - alpha) softmax(c + f) + alpha / n (FP64 softmax on the
 * host): a network that outputs 0 gives back the score weights.
 * Training target of an instance: t_i ~ exp(beta c_i) (u_i + eps)^gamma,
 * u = clip(v, 0, 1) for a per-clone signal v from the method's own outputs
 * (for instance its marginals, or the per-update scales SE_j sqrt(w_j) of
 * its standard errors over their maximum); loss = mean over
 * instances of KL(t || softmax(c + f)); optimiser AdamW (decoupled weight
 * decay on every parameter).
 * ------------------------------------------------------------------------ */
#define MCPD_MLP_FEATURES 8
#define MCPD_MLP_HIDDEN 64
#define MCPD_MLP_PARAMS 4801

typedef struct mcpd_mlp mcpd_mlp;

typedef struct mcpd_adamw {
    float lr, beta1, beta2, eps, weight_decay;
} mcpd_adamw;

/* Features of every clone: out host [n * 8] (row-major) and base logits
 * base_out host [n] (may be NULL), computed on the device.
 * Errors: MCPD_EINVAL, MCPD_ENOMEM, MCPD_EDEVICE. */
int mcpd_features(mcpd_instance *inst, float *out, double *base_out);

/* Create a network from FP32 master parameters (host [MCPD_MLP_PARAMS]).
 * hip_stream as in mcpd_create.  Errors: MCPD_EINVAL (null or non-finite
 * parameter), MCPD_ENOMEM, MCPD_EDEVICE. */
int mcpd_mlp_create(const float *params, void *hip_stream, mcpd_mlp **out);

/* Read the FP32 master copy and/or its BF16 rounding (host arrays of
 * MCPD_MLP_PARAMS, either may be NULL). */
int mcpd_mlp_get_params(const mcpd_mlp *mlp, float *master, uint16_t *bf16);

/* Replace the master copy (host [MCPD_MLP_PARAMS]); resets the optimiser. */
int mcpd_mlp_set_params(mcpd_mlp *mlp, const float *master);

/* Network outputs f of `rows` feature rows: x host [rows * 8], g host [rows]. */
int mcpd_mlp_forward(mcpd_mlp *mlp, const float *x, int64_t rows, float *g);

/* Training set from raw rows: x host [rows * 8], base host [rows] (base
 * logits, finite and <= 0), signal host [rows] (the per-clone signal v),
 * seg_ptr host [nseg + 1] with seg_ptr[0] = 0 and seg_ptr[nseg] = rows,
 * increasing (one non-empty segment per instance); beta, gamma >= 0,
 * eps > 0.  Copied to the device. */
int mcpd_mlp_set_training_rows(mcpd_mlp *mlp, const float *x, const double *base, const double *signal,
                               int64_t rows, const int64_t *seg_ptr, int32_t nseg, double beta, double gamma,
                               double eps);

/* Training set from instances: their features (computed on the device) and
 * signal[i] host [n_i] (the signal v) for instance i. */
int mcpd_mlp_set_training_data(mcpd_mlp *mlp, mcpd_instance *const *insts, const double *const *signal,
                               int32_t count, double beta, double gamma, double eps);

/* Loss over the training set and its gradient in the parameters (host
 * [MCPD_MLP_PARAMS] or NULL), for the current parameters. */
int mcpd_mlp_loss_grad(mcpd_mlp *mlp, double *loss, float *grad);

/* `steps` full-batch AdamW steps, every step (forward, loss, backward,
 * update) on the device; loss_history host [steps] or NULL receives the
 * loss before each step.  The step counter of the bias corrections
 * continues across calls until mcpd_mlp_set_params. */
int mcpd_mlp_train(mcpd_mlp *mlp, int32_t steps, const mcpd_adamw *hp, double *loss_history);

/* Gradient in the parameters (host [MCPD_MLP_PARAMS]) of sum_r dg[r] g_r
 * over `rows` rows of features x (host [rows * 8]) with the upstream
 * derivatives dg (host [rows]), through the BF16 working copy (the
 * straight-through gradient the FP32 master receives): the backward pass
 * alone, on the device.  Errors: MCPD_EINVAL, MCPD_ENOMEM, MCPD_EDEVICE. */
int mcpd_mlp_backward(mcpd_mlp *mlp, const float *x, int64_t rows, const float *dg, float *grad);

/* One AdamW step with decoupled weight decay on every parameter, with the
 * given gradient (host [MCPD_MLP_PARAMS], finite), on the device: moments,
 * bias corrections from the step counter (which it advances), FP32 master
 * update and the BF16 copy.  Errors: MCPD_EINVAL, MCPD_EDEVICE. */
int mcpd_mlp_adamw_step(mcpd_mlp *mlp, const float *grad, const mcpd_adamw *hp);

/* Optimiser state for checkpoints: FP32 master parameters, their BF16 copy,
 * the AdamW first and second moments (host [MCPD_MLP_PARAMS] each; any may be
 * NULL) and the step counter.  set_state restores master, moments and step
 * and rebuilds the BF16 copy from the master (round to nearest even), so a
 * restored network continues training exactly as the saved one would.
 * Errors: MCPD_EINVAL (null or non-finite state, negative second moment or
 * step), MCPD_EDEVICE. */
int mcpd_mlp_get_state(const mcpd_mlp *mlp, float *master, uint16_t *bf16, float *adam_m, float *adam_v,
                       int64_t *step);
int mcpd_mlp_set_state(mcpd_mlp *mlp, const float *master, const float *adam_m, const float *adam_v, int64_t step);

/* Set an instance's selection weights from the network: features, base
 * logits and network outputs on the device, then w = (1 - alpha)
 * softmax(c + f) + alpha / n, 0 < alpha <= 1, passed to mcpd_set_weights.
 * w_out host [n] or NULL receives w. */
int mcpd_set_learned_weights(mcpd_instance *inst, mcpd_mlp *mlp, double alpha, double *w_out);

/* Release a network (NULL is a no-op). */
void mcpd_mlp_destroy(mcpd_mlp *mlp);

/* Static name of an error code. */
/* ---- Peak-rate probes (measurement support) ----------------------------
 * The benchmark's roofline divides achieved rates by peaks measured on the
 * device by these probes, not by figures assumed from other chips.  Each
 * probe launches eight workgroups of 256 lanes per compute unit that run
 * `iters` iterations of one kind of independent operation:
 *   LDS_B32, LDS_B64, LDS_B128: conflict-free streaming LDS reads of 4, 8 or
 *     16 bytes per lane (the 64 lanes of a read touch consecutive words);
 *   LDS_B32_RANDOM: 4-byte LDS reads at fixed pseudo-random addresses;
 *   VALU_ADD, VALU_MUL_LO, VALU_MUL_HI, VALU_BITOP3, VALU_MUL64: 32-bit
 *     add, low and high 32x32 products, three-input xor, and the full 64-bit
 *     product of two 32-bit words (one lane operation each);
 *   PHILOX10: whole Philox4x32-10 blocks as the sampler computes them.
 * Results: per_second for the whole device (the launch's work over its
 * event-timed duration), the shader clock the probe ran at (in-kernel clock
 * counters), per_cu_per_clock = per_second / (clock x compute units) in
 * bytes, lane operations or blocks, and the kernel time.  Uses the current device; allocates and frees
 * a few MB.  Errors: MCPD_EINVAL (kind out of range, iters = 0, out null),
 * MCPD_ENOMEM, MCPD_EDEVICE. */
enum {
    MCPD_PROBE_LDS_B32 = 0,
    MCPD_PROBE_LDS_B64 = 1,
    MCPD_PROBE_LDS_B128 = 2,
    MCPD_PROBE_LDS_B32_RANDOM = 3,
    MCPD_PROBE_VALU_ADD = 4,
    MCPD_PROBE_VALU_MUL_LO = 5,
    MCPD_PROBE_VALU_MUL_HI = 6,
    MCPD_PROBE_VALU_BITOP3 = 7,
    MCPD_PROBE_VALU_MUL64 = 8,
    MCPD_PROBE_PHILOX10 = 9,
    MCPD_PROBE_COUNT = 10
};

typedef struct mcpd_probe_result {
    double per_cu_per_clock;
    double per_second;
    double clock_hz;
    double ms;
    uint32_t cus;
    uint32_t reserved;
} mcpd_probe_result;

int mcpd_probe(int kind, uint32_t iters, mcpd_probe_result *out);

const char *mcpd_strerror(int code);

/* Detail of the last error on the calling thread ("" if none). */
const char *mcpd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCPD_H */
