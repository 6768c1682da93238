/*
 * mcpd_oracle.h -- the CPU oracle's entry points in the shape of the
 * library's C ABI (mcpd_create / mcpd_set_weights / mcpd_get_weights /
 * mcpd_run_unbiased / mcpd_destroy), plus mcpd_oracle_trace.
 *
 * TEST INFRASTRUCTURE ONLY (see mcpd_oracle.c).  The oracle shares no code,
 * header or type with the HIP library: the types below are its own, with
 * the fields the oracle implements.  All pointers are host pointers; inputs
 * are copied at the call; outputs are caller-allocated.  Return value 0 on
 * success, -1 for an invalid argument (the same rules as the library:
 * Section "Knill's Method" for the design, 0 < fp, fn, prior < 1, k <= m,
 * slots >= 1, positive finite weights), -2 when memory runs out, -5 when a
 * trace does not fit max_len.
 */
#ifndef MCPD_ORACLE_H
#define MCPD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mo_model mcpd_oracle_instance;

/* Run options (mcpd_oracle_opts_init sets the defaults: no cap, refill on,
 * 64 histogram bins of one sweep, 32 high bits of U, instance id 0, the
 * all-negative start, all threads, no optional outputs). */
typedef struct mcpd_oracle_opts {
    uint64_t max_steps;     /* meeting cap in draws, 0 = none (>= max(m, 1) otherwise) */
    uint32_t refill;        /* 1 = slot refill, 0 = one pair per slot */
    uint32_t hist_bins;     /* meeting-time histogram bins */
    uint32_t hist_width;    /* draws per bin, 0 = n (one sweep) */
    uint32_t u_hi_bits;     /* bits of U from the main block, 1..32 */
    uint32_t instance_id;   /* g of the random-number counter, < 2^24 */
    uint32_t init_mode;     /* 0 = all-negative start, 1 = drawn from the prior */
    int32_t nthreads;       /* OpenMP threads, 0 = all */
    uint32_t bucket_rows;   /* rows of bucket_sum / bucket_sumsq */
    uint32_t *slot_nstar;   /* [slots] N*_p, or NULL */
    uint64_t *slot_units;   /* [slots] S_p(N*_p), or NULL */
    int64_t *bucket_sum;    /* [bucket_rows * n] sum of V_pj over slots with N*_p = row + 1, or NULL */
    uint64_t *bucket_sumsq; /* [bucket_rows * n * 2] (low, high) words of the sum of V_pj^2, or NULL */
    uint64_t *mismatch;     /* [n] mismatch time of each clone over retained replications, or NULL */
} mcpd_oracle_opts;

/* Statistics of a run (as the library's, for the counters the oracle keeps). */
typedef struct mcpd_oracle_stats {
    uint64_t retained_units, single_site_updates, reps_retained, cap_hits, zero_completion_slots,
             tau_sum, tau_max, reps_discarded, discarded_units, nstar_max;
} mcpd_oracle_stats;

void mcpd_oracle_opts_init(mcpd_oracle_opts *opts);
int mcpd_oracle_create(int32_t n_clones, int32_t n_pools, const int32_t *row_ptr, const int32_t *pool_idx,
                       const uint8_t *outcomes, double fp, double fn, double prior, mcpd_oracle_instance **out);
/* w: n weights (positive, finite), or NULL for the paper's score weights. */
int mcpd_oracle_set_weights(mcpd_oracle_instance *inst, const double *w);
/* The exact sampled weights M_i / 2^32 and the integer masses (either may be NULL). */
int mcpd_oracle_get_weights(const mcpd_oracle_instance *inst, double *w_exact, uint64_t *mass);
int mcpd_oracle_run_unbiased(mcpd_oracle_instance *inst, uint64_t budget, uint32_t slots, uint32_t k, uint32_t m,
                             uint64_t seed, const mcpd_oracle_opts *opts, double *marginals, double *stderr_out,
                             uint64_t *hist, mcpd_oracle_stats *stats);
/* One replication r (>= 1) of slot `slot`, every step recorded: X [(max_len+1) x n] holds X_0..X_C,
 * Y [max_len x n] Y_0..Y_{C-1}, I and U the sites and 53-bit uniforms of draws 0..C-1; numer the
 * numerators W H_{k:m}, mismatch the clone mismatch times (either may be NULL); out = (C, tau, capped).
 * opts supplies max_steps, u_hi_bits, instance_id and init_mode (NULL = defaults). */
int mcpd_oracle_trace(mcpd_oracle_instance *inst, uint32_t slot, uint32_t r, uint64_t seed, uint32_t k, uint32_t m,
                      const mcpd_oracle_opts *opts, uint64_t max_len, uint8_t *X, uint8_t *Y, int32_t *I, uint64_t *U,
                      int64_t *numer, int64_t *mismatch, uint64_t out[3]);
void mcpd_oracle_destroy(mcpd_oracle_instance *inst);

#ifdef __cplusplus
}
#endif

#endif
