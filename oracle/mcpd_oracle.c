/*
 * mcpd_oracle.c -- plain, slow, FP64 CPU oracle for unbiased Markov chain
 * pool decoding (coupled score-weighted random-scan Gibbs sampler, the
 * time-averaged H_{k:l} estimator, fixed-budget slots with refill and the
 * completion-time-corrected aggregate).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library: both follow the same written reading of
 * the paper independently.
 *
 * Every function cites the passage of the paper it follows.  Where the paper
 * leaves a choice open (precision, random-number generator, site sampler,
 * initial distribution, summation order) the reading used here is stated at
 * the function.  Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).
 *
 * Pinning status, per function (what fixes it independently of itself):
 *   philox4x32_10 ......... rocRAND's own Philox4x32-10 engine (header source)
 *   log-odds terms ......... brute-force posterior ratios (exact enumeration)
 *   score_weights .......... sum to one, uniform floor, max/min ratio = gamma
 *   quantize / alias ....... exact mass identities of the table; chi-square of draws
 *   cond_p1 (full cond.) ... brute-force pi(x^{i<-1}) / (pi(x^{i<-1}) + pi(x^{i<-0}))
 *   gibbs update + draw .... pi P_w = pi, detailed balance; chi-square vs P_w rows
 *   replication ............ literal H_r sums from the trace; faithfulness;
 *                            cost C = max(l, tau); identity-design tau law
 *   slot scheduler ......... per-slot refill/retention rules from the records
 *   aggregate .............. mean over slots vs exact posterior marginals (CI)
 *   mismatch time .......... literal count of x_j(s) != y_j(s-1) on the trace;
 *                            run totals = sums over retained replications
 * Trajectory bits themselves have no printed worked example in the paper:
 * beyond the pins above they are parity unpinned.
 */
#include "mcpd_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MO_OK 0
#define MO_EINVAL (-1)
#define MO_ENOMEM (-2)
#define MO_ETOOLONG (-5)

/* Hard safety bound on draws per replication when no cap is requested:
 * the Philox counter word for the draw index is 32 bits wide. */
#define MO_MAX_DRAWS 4294967295ULL

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  The paper asks only for an i.i.d. ideal random
 * stream per pair (Assumption 2); this counter-based generator is our
 * reading.  Round function: with the two 32x32->64 products
 * M0*c0 = (hi0,lo0) and M1*c2 = (hi1,lo1), the new counter is
 * (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key is bumped by the Weyl constants
 * between rounds.
 * ---------------------------------------------------------------------- */
void mo_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------
 * Random numbers of one draw (reading of "draw I_t with Pr{I_t=i}=w_i and
 * U_t ~ Unif(0,1)", Algorithm 3).  Key = (seed low word, seed high word).
 * Draw t of replication r in slot p of instance g reads
 *   main block  ctr = (floor(t/2), r, p, g)            words 2(t mod 2), 2(t mod 2)+1
 *   low block   ctr = (t,          r, p, g | 1 << 24)   words 0, 1
 * The first main word selects the site; U has 53 bits: the top b bits of the
 * second main word followed by the top 53-b bits of the 64-bit low block.
 * U = U53 * 2^-53.  b = 32 unless a test asks for fewer.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t site_word;
    uint64_t u53;
} mo_draw_t;

static mo_draw_t draw_numbers(uint64_t seed, uint32_t g, uint32_t p, uint32_t r,
                              uint64_t t, uint32_t b)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)(t >> 1), r, p, g};
    uint32_t w[4];
    mo_philox4x32_10(ctr, key, w);
    unsigned o = 2u * (unsigned)(t & 1u);
    mo_draw_t d;
    d.site_word = w[o];
    uint64_t hi = (uint64_t)w[o + 1] >> (32u - b);
    uint32_t ctr2[4] = {(uint32_t)t, r, p, g | (1u << 24)};
    uint32_t v[4];
    mo_philox4x32_10(ctr2, key, v);
    uint64_t low64 = ((uint64_t)v[0] << 32) | (uint64_t)v[1];
    uint64_t lo = low64 >> (11u + b);
    d.u53 = (hi << (53u - b)) | lo;
    return d;
}

void mo_draw(uint64_t seed, uint32_t g, uint32_t p, uint32_t r, uint64_t t, uint32_t b,
             uint32_t *site_word, uint64_t *u53)
{
    mo_draw_t d = draw_numbers(seed, g, p, r, t, b);
    *site_word = d.site_word;
    *u53 = d.u53;
}

/* ------------------------------------------------------------------------
 * Model (Section "Knill's Method"): posterior
 *   pi(z|y) ~ prod_i q^{z_i}(1-q)^{1-z_i} prod_j Pr{y_j | xi_j(z)},
 * xi_j(z) = 1{sum_i A_ji z_i > 0}.  Observation channel (reading; the paper
 * names only the two rates): Pr{y=1|xi=1} = 1-fn, Pr{y=1|xi=0} = fp.
 * ---------------------------------------------------------------------- */
typedef struct mo_model {
    int32_t n, m;
    int32_t *row_ptr;   /* n+1 */
    int32_t *pool_idx;  /* nnz, ascending per row */
    uint8_t *y;         /* m */
    double fp, fn, q;
    double lq;          /* log{q/(1-q)} */
    double a_pos;       /* a_j for y_j = 1 */
    double a_neg;       /* a_j for y_j = 0 */
    double *w;          /* selection weights as given or the score weights */
    uint64_t *mass;     /* quantized integer masses, sum 2^32 */
    int32_t abits;      /* a: the alias table has 2^a columns, 2^a >= n */
    uint32_t *athr;     /* [2^a] column threshold T_c in [0, 2^(32-a)] */
    uint32_t *alias;    /* [2^a] column alias A_c */
} mo_model;

/* a_j = log Pr{y_j|xi=1} - log Pr{y_j|xi=0} (Section "Score-Weighted Update
 * Gibbs Sampler"); logit of the prior as in eta_i = log{q/(1-q)} + log R_i. */
void mo_log_odds_terms(double fp, double fn, double q, double out[3])
{
    out[0] = log(q / (1.0 - q));
    out[1] = log(1.0 - fn) - log(fp);   /* y = 1 */
    out[2] = log(fn) - log(1.0 - fp);   /* y = 0 */
}

static int validate_design(int32_t n, int32_t m, const int32_t *row_ptr,
                           const int32_t *pool_idx, const uint8_t *y,
                           double fp, double fn, double q)
{
    if (n <= 0 || m <= 0) return MO_EINVAL;
    if (!(fp > 0.0 && fp < 1.0 && fn > 0.0 && fn < 1.0 && q > 0.0 && q < 1.0)) return MO_EINVAL;
    if (row_ptr[0] != 0) return MO_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return MO_EINVAL;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (pool_idx[e] < 0 || pool_idx[e] >= m) return MO_EINVAL;
            if (e > row_ptr[i] && pool_idx[e] <= pool_idx[e - 1]) return MO_EINVAL;
        }
    }
    for (int32_t j = 0; j < m; ++j)
        if (y[j] > 1) return MO_EINVAL;
    return MO_OK;
}

/* Score weights (Section "Score-Weighted Update Gibbs Sampler"):
 * d_j = active pool size, s_i = sum_{j: A_ji = 1} d_j a_j, gamma = 100 n,
 * tau_w = log(gamma)/(s_max - s_min) (0 when all scores are equal),
 * w_i = (1 - alpha_w) softmax(tau_w s)_i + alpha_w / n, alpha_w = 1/2.
 * Reading: the softmax is evaluated as exp(tau_w (s_i - s_max)) / sum, which
 * is the same function written so that exp cannot overflow; sums run in
 * ascending index order. */
int mo_score_weights(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx,
                     const uint8_t *y, double fp, double fn, double q,
                     double *s_out, double *w_out)
{
    int rc = validate_design(n, m, row_ptr, pool_idx, y, fp, fn, q);
    if (rc) return rc;
    double lo[3];
    mo_log_odds_terms(fp, fn, q, lo);
    int64_t *d = (int64_t *)calloc((size_t)m, sizeof(int64_t));
    double *e = (double *)malloc((size_t)n * sizeof(double));
    if (!d || !e) { free(d); free(e); return MO_ENOMEM; }
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) d[pool_idx[k]] += 1;
    double smax = -INFINITY, smin = INFINITY;
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t j = pool_idx[k];
            double aj = y[j] ? lo[1] : lo[2];
            s = s + (double)d[j] * aj;
        }
        s_out[i] = s;
        if (s > smax) smax = s;
        if (s < smin) smin = s;
    }
    double gamma = 100.0 * (double)n;
    double tau = (smax > smin) ? log(gamma) / (smax - smin) : 0.0;
    double esum = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        e[i] = exp(tau * (s_out[i] - smax));
        esum = esum + e[i];
    }
    for (int32_t i = 0; i < n; ++i)
        w_out[i] = 0.5 * (e[i] / esum) + 0.5 / (double)n;
    free(d);
    free(e);
    return MO_OK;
}

/* Integer site masses (reading; the paper only requires Pr{I_t=i} = w_i with
 * fixed positive weights, Assumption 1).  v_i = w_i / sum(w); with
 * S = 2^32 - n, M_i = 1 + floor(v_i S); the D = 2^32 - sum M_i units left go
 * one each to the D clones of largest remainder v_i S - floor(v_i S), ties to
 * the lower index.  Every M_i >= 1, sum M_i = 2^32, and the sampled weight
 * is exactly M_i / 2^32. */
typedef struct { double rem; int32_t idx; } rem_t;

static int rem_cmp(const void *a, const void *b)
{
    const rem_t *x = (const rem_t *)a, *y = (const rem_t *)b;
    if (x->rem > y->rem) return -1;
    if (x->rem < y->rem) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

int mo_quantize(int32_t n, const double *w, uint64_t *mass)
{
    if (n <= 0 || n > (1 << 24)) return MO_EINVAL;
    double wsum = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (!(w[i] > 0.0) || !isfinite(w[i])) return MO_EINVAL;
        wsum = wsum + w[i];
    }
    if (!isfinite(wsum)) return MO_EINVAL;
    double S = 4294967296.0 - (double)n;
    rem_t *r = (rem_t *)malloc((size_t)n * sizeof(rem_t));
    if (!r) return MO_ENOMEM;
    uint64_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
        double f = (w[i] / wsum) * S;
        double fl = floor(f);
        uint64_t mi = 1u + (uint64_t)fl;
        if (mi > 4294967296ull) { free(r); return MO_EINVAL; }
        mass[i] = mi;
        total += mi;
        r[i].rem = f - fl;
        r[i].idx = i;
    }
    int64_t D = (int64_t)4294967296LL - (int64_t)total;
    if (D < 0 || D > n) { free(r); return MO_EINVAL; }
    qsort(r, (size_t)n, sizeof(rem_t), rem_cmp);
    for (int64_t t = 0; t < D; ++t) mass[r[t].idx] += 1u;
    free(r);
    return MO_OK;
}

/* Site sampler (reading; the paper only requires Pr{I_t = i} = w_i with
 * fixed weights): a Walker alias table (Walker 1977) built by Vose's
 * procedure (Vose 1991) on the integer masses.  With a = max(1, ceil(log2 n))
 * there are 2^a columns of capacity K = 2^(32-a); column c < n starts with
 * mass M_c, columns c >= n with 0.  Columns with mass < K are pushed on the
 * "small" stack, the others on the "large" stack, in ascending c; then, while
 * both are non-empty, pop l from small and g from large, set T_l = mass_l,
 * A_l = g, mass_g -= K - mass_l, and push g back on small (mass_g < K) or
 * large.  Columns left on either stack get T = K, A = self.  The draw takes
 * the top a bits of the site word as the column c and the low 32-a bits as r:
 * I = c if r < T_c, else A_c.  Every step is exact integer arithmetic, so
 * Pr{I = i} = M_i / 2^32 exactly. */
static int build_alias(mo_model *M)
{
    int32_t a = 1;
    while (((int64_t)1 << a) < M->n) ++a;
    const int64_t N = (int64_t)1 << a;
    const uint64_t K = (uint64_t)1 << (32 - a);
    uint64_t *mass = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    int64_t *small = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int64_t *large = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    M->athr = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    M->alias = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    if (!mass || !small || !large || !M->athr || !M->alias) {
        free(mass); free(small); free(large);
        return MO_ENOMEM;
    }
    int64_t ns = 0, nl = 0;
    for (int64_t c = 0; c < N; ++c) {
        mass[c] = c < M->n ? M->mass[c] : 0u;
        if (mass[c] < K) small[ns++] = c; else large[nl++] = c;
    }
    while (ns > 0 && nl > 0) {
        const int64_t l = small[--ns];
        const int64_t g = large[--nl];
        M->athr[l] = (uint32_t)mass[l];
        M->alias[l] = (uint32_t)g;
        mass[g] -= K - mass[l];
        if (mass[g] < K) small[ns++] = g; else large[nl++] = g;
    }
    while (nl > 0) { const int64_t g = large[--nl]; M->athr[g] = (uint32_t)K; M->alias[g] = (uint32_t)g; }
    while (ns > 0) { const int64_t l = small[--ns]; M->athr[l] = (uint32_t)K; M->alias[l] = (uint32_t)l; }
    M->abits = a;
    free(mass); free(small); free(large);
    return MO_OK;
}

mo_model *mo_model_create(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx,
                          const uint8_t *y, double fp, double fn, double q, const double *w)
{
    if (validate_design(n, m, row_ptr, pool_idx, y, fp, fn, q)) return NULL;
    mo_model *M = (mo_model *)calloc(1, sizeof(mo_model));
    if (!M) return NULL;
    int32_t nnz = row_ptr[n];
    M->n = n; M->m = m; M->fp = fp; M->fn = fn; M->q = q;
    M->row_ptr = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    M->pool_idx = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    M->y = (uint8_t *)malloc((size_t)m);
    M->w = (double *)malloc((size_t)n * sizeof(double));
    M->mass = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    double *s = (double *)malloc((size_t)n * sizeof(double));
    if (!M->row_ptr || !M->pool_idx || !M->y || !M->w || !M->mass || !s) goto fail;
    memcpy(M->row_ptr, row_ptr, (size_t)(n + 1) * sizeof(int32_t));
    if (nnz) memcpy(M->pool_idx, pool_idx, (size_t)nnz * sizeof(int32_t));
    memcpy(M->y, y, (size_t)m);
    double lo[3];
    mo_log_odds_terms(fp, fn, q, lo);
    M->lq = lo[0]; M->a_pos = lo[1]; M->a_neg = lo[2];
    if (w) {
        memcpy(M->w, w, (size_t)n * sizeof(double));
    } else if (mo_score_weights(n, m, row_ptr, pool_idx, y, fp, fn, q, s, M->w)) {
        goto fail;
    }
    if (mo_quantize(n, M->w, M->mass)) goto fail;
    if (build_alias(M)) goto fail;
    free(s);
    return M;
fail:
    free(s);
    free(M->row_ptr); free(M->pool_idx); free(M->y); free(M->w); free(M->mass);
    free(M->athr); free(M->alias);
    free(M);
    return NULL;
}

void mo_model_free(mo_model *M)
{
    if (!M) return;
    free(M->row_ptr); free(M->pool_idx); free(M->y); free(M->w); free(M->mass);
    free(M->athr); free(M->alias);
    free(M);
}

void mo_model_masses(const mo_model *M, uint64_t *mass)
{
    memcpy(mass, M->mass, (size_t)M->n * sizeof(uint64_t));
}

/* Site draw from the alias table (see build_alias). */
static int32_t site_of(const mo_model *M, uint32_t s)
{
    const int32_t a = M->abits;
    const uint32_t c = s >> (32 - a);
    const uint32_t r = s & (uint32_t)((((uint64_t)1) << (32 - a)) - 1u);
    return (int32_t)(r < M->athr[c] ? c : M->alias[c]);
}

/* The alias table (tests): 2^a thresholds and aliases; returns a. */
int32_t mo_model_alias(const mo_model *M, uint32_t *thr, uint32_t *alias)
{
    const int64_t N = (int64_t)1 << M->abits;
    if (thr) memcpy(thr, M->athr, (size_t)N * sizeof(uint32_t));
    if (alias) memcpy(alias, M->alias, (size_t)N * sizeof(uint32_t));
    return M->abits;
}

int32_t mo_site(const mo_model *M, uint32_t site_word) { return site_of(M, site_word); }

/* ------------------------------------------------------------------------
 * Chain state and the full conditional.  c_j = sum_i A_ji x_i.  For pools
 * j in P(i): xi_j(x^{i<-1}) = 1 and xi_j(x^{i<-0}) = 1{c_j - x_i > 0}; all
 * other pools cancel in the ratio pi(x^{i<-1}) / pi(x^{i<-0}), so
 *   logit p_i(1|x_{-i}) = log{q/(1-q)} + sum_{j in P(i), c_j - x_i = 0} a_j.
 * Reading: the FP64 sum adds the terms in ascending pool index starting
 * from log{q/(1-q)}; p = 1/(1 + exp(-L)).
 * ---------------------------------------------------------------------- */
typedef struct {
    uint8_t *x;       /* n */
    int32_t *c;       /* m */
    int32_t *pos;     /* list of clones with x = 1 */
    int32_t *where;   /* position in pos, -1 if absent */
    int32_t npos;
} chain_t;

static double cond_p1(const mo_model *M, const chain_t *ch, int32_t i)
{
    double L = M->lq;
    for (int32_t e = M->row_ptr[i]; e < M->row_ptr[i + 1]; ++e) {
        int32_t j = M->pool_idx[e];
        if (ch->c[j] - (int32_t)ch->x[i] == 0) L = L + (M->y[j] ? M->a_pos : M->a_neg);
    }
    return 1.0 / (1.0 + exp(-L));
}

static void chain_set(const mo_model *M, chain_t *ch, int32_t i, uint8_t v)
{
    if (ch->x[i] == v) return;
    int delta = v ? 1 : -1;
    for (int32_t e = M->row_ptr[i]; e < M->row_ptr[i + 1]; ++e) ch->c[M->pool_idx[e]] += delta;
    ch->x[i] = v;
    if (v) {
        ch->where[i] = ch->npos;
        ch->pos[ch->npos++] = i;
    } else {
        int32_t at = ch->where[i];
        int32_t last = ch->pos[--ch->npos];
        ch->pos[at] = last;
        ch->where[last] = at;
        ch->where[i] = -1;
    }
}

/* Phi_i(x, u): coordinate i becomes 1{u <= p_i(1|x_{-i})} (Section
 * "Knill's Method", single-site update map).  Returns the new value. */
static uint8_t gibbs_value(const mo_model *M, const chain_t *ch, int32_t i, uint64_t u53)
{
    double p = cond_p1(M, ch, i);
    double u = (double)u53 * 0x1p-53;
    return (uint8_t)(u <= p);
}

static int chain_alloc(chain_t *ch, int32_t n, int32_t m)
{
    ch->x = (uint8_t *)calloc((size_t)n, 1);
    ch->c = (int32_t *)calloc((size_t)m, sizeof(int32_t));
    ch->pos = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    ch->where = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    ch->npos = 0;
    if (!ch->x || !ch->c || !ch->pos || !ch->where) return MO_ENOMEM;
    for (int32_t i = 0; i < n; ++i) ch->where[i] = -1;
    return MO_OK;
}

static void chain_free(chain_t *ch)
{
    free(ch->x); free(ch->c); free(ch->pos); free(ch->where);
}

/* Initial distribution nu (reading; never specified in the paper, and the
 * estimator is unbiased for any nu): the all-negative state. */
static void chain_reset(const mo_model *M, chain_t *ch)
{
    while (ch->npos > 0) chain_set(M, ch, ch->pos[ch->npos - 1], 0);
}

/* Full conditional p_i(1 | x_{-i}) of an arbitrary state (tests). */
double mo_conditional(const mo_model *M, const uint8_t *x, int32_t i)
{
    chain_t ch;
    if (chain_alloc(&ch, M->n, M->m)) { chain_free(&ch); return NAN; }
    for (int32_t l = 0; l < M->n; ++l) if (x[l]) chain_set(M, &ch, l, 1);
    double p = cond_p1(M, &ch, i);
    chain_free(&ch);
    return p;
}

/* One single-site Gibbs update Phi_I(x, U) driven by the random numbers of
 * draw (g, p, r, t): x_out = Phi_{I_t}(x_in, U_t) (tests). */
int mo_gibbs_step(const mo_model *M, const uint8_t *x_in, uint64_t seed, uint32_t g,
                  uint32_t p, uint32_t r, uint64_t t, uint32_t b, uint8_t *x_out, int32_t *site)
{
    if (b < 1 || b > 32) return MO_EINVAL;
    chain_t ch;
    if (chain_alloc(&ch, M->n, M->m)) { chain_free(&ch); return MO_ENOMEM; }
    for (int32_t l = 0; l < M->n; ++l) if (x_in[l]) chain_set(M, &ch, l, 1);
    mo_draw_t d = draw_numbers(seed, g, p, r, t, b);
    int32_t I = site_of(M, d.site_word);
    chain_set(M, &ch, I, gibbs_value(M, &ch, I, d.u53));
    memcpy(x_out, ch.x, (size_t)M->n);
    *site = I;
    chain_free(&ch);
    return MO_OK;
}

/* ------------------------------------------------------------------------
 * Run parameters (all 64-bit so the Python side can pass one array).
 * ---------------------------------------------------------------------- */
typedef struct {
    uint64_t budget;      /* total progress units; B = floor(budget / slots) */
    uint64_t slots;       /* P */
    uint64_t k;           /* window start */
    uint64_t ell;         /* window end l (Jacob's m) */
    uint64_t seed;
    uint64_t max_steps;   /* 0: no cap; else draws per replication are capped at
                             max(max_steps, l) when the pair has not met */
    uint64_t refill;      /* 1: slot refill; 0: one replication per slot */
    uint64_t hist_bins;
    uint64_t hist_width;
    uint64_t u_hi_bits;   /* b of draw_numbers, 1..32 */
    uint64_t instance_id; /* g, < 2^24 */
    uint64_t init_mode;   /* nu: 0 = all-negative state, 1 = the prior */
} mo_params;

/* Sparse numerator accumulator: dense int64 values plus a touched list. */
typedef struct {
    int64_t *v;
    uint8_t *mark;
    int32_t *list;
    int32_t nlist;
} acc_t;

static int acc_alloc(acc_t *a, int32_t n)
{
    a->v = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    a->mark = (uint8_t *)calloc((size_t)n, 1);
    a->list = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    a->nlist = 0;
    return (a->v && a->mark && a->list) ? MO_OK : MO_ENOMEM;
}

static void acc_free(acc_t *a) { free(a->v); free(a->mark); free(a->list); }

/* Values are summed modulo 2^64: intermediate sums may leave int64 range
 * even though every final numerator is bounded by W (1 + 2 C). */
static void acc_add(acc_t *a, int32_t j, int64_t val)
{
    if (!a->mark[j]) { a->mark[j] = 1; a->list[a->nlist++] = j; }
    a->v[j] = (int64_t)((uint64_t)a->v[j] + (uint64_t)val);
}

static void acc_clear(acc_t *a)
{
    for (int32_t t = 0; t < a->nlist; ++t) { a->v[a->list[t]] = 0; a->mark[a->list[t]] = 0; }
    a->nlist = 0;
}

static void acc_merge(acc_t *dst, const acc_t *src)
{
    for (int32_t t = 0; t < src->nlist; ++t) acc_add(dst, src->list[t], src->v[src->list[t]]);
}

/* Per-replication scratch. */
typedef struct {
    chain_t X, Y;
    int32_t *mis;      /* clones with x_j(s) != y_j(s-1) */
    int32_t *mwhere;
    int32_t nmis;
    acc_t rep;         /* numerators of the current replication */
    acc_t rmis;        /* its mismatch time per clone: #{s >= 1 : x_j(s) != y_j(s-1)} */
    acc_t slot;        /* numerators summed over retained replications */
} scratch_t;

static int scratch_alloc(scratch_t *s, int32_t n, int32_t m)
{
    memset(s, 0, sizeof(*s));
    int rc = chain_alloc(&s->X, n, m) | chain_alloc(&s->Y, n, m);
    s->mis = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    s->mwhere = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!s->mis || !s->mwhere) rc = MO_ENOMEM;
    else for (int32_t i = 0; i < n; ++i) s->mwhere[i] = -1;
    s->nmis = 0;
    rc |= acc_alloc(&s->rep, n) | acc_alloc(&s->slot, n) | acc_alloc(&s->rmis, n);
    return rc ? MO_ENOMEM : MO_OK;
}

static void scratch_free(scratch_t *s)
{
    chain_free(&s->X); chain_free(&s->Y);
    free(s->mis); free(s->mwhere);
    acc_free(&s->rep); acc_free(&s->slot); acc_free(&s->rmis);
}

static void mis_update(scratch_t *s, int32_t i)
{
    int differ = s->X.x[i] != s->Y.x[i];
    int listed = s->mwhere[i] >= 0;
    if (differ && !listed) {
        s->mwhere[i] = s->nmis;
        s->mis[s->nmis++] = i;
    } else if (!differ && listed) {
        int32_t at = s->mwhere[i];
        int32_t last = s->mis[--s->nmis];
        s->mis[at] = last;
        s->mwhere[last] = at;
        s->mwhere[i] = -1;
    }
}

typedef struct {
    uint64_t C;        /* progress units = draws made = max(l, tau) (or the cap) */
    uint64_t tau;      /* meeting time, 0 if capped */
    int capped;
} rep_out_t;

/* Optional per-step trace for small instances. */
typedef struct {
    uint64_t max_len;
    uint8_t *X;        /* (max_len+1) x n : X_0 .. X_C */
    uint8_t *Y;        /* max_len x n     : Y_0 .. Y_{C-1} */
    int32_t *I;        /* max_len */
    uint64_t *U;       /* max_len */
    int overflow;
} trace_t;

/* Contributions of time index s to the numerator of H_{k:l} (Section
 * "Coupled Estimator and Fixed-Budget GPU Execution"):
 *   W H_{k:l}(h_j) = sum_{r=k}^{l} [ x_j(r) + sum_{s>r} (x_j(s) - y_j(s-1)) ]
 *                  = sum_{s=k}^{l} x_j(s) + sum_{s>=k+1} min(s-k, W) (x_j(s) - y_j(s-1)),
 * exchanging the two finite sums (time index s is counted once for every
 * r in [k, min(l, s-1)]).  Terms with x_j(s) = 0, or with x_j(s) = y_j(s-1),
 * are zero and skipped.  After the meeting time every difference vanishes
 * (Theorem 1 (d)), so the correction sum is finite; a replication stopped by
 * a cap keeps the terms up to its last time index (the truncated H^{(R)}). */
static void add_time_index(scratch_t *s, uint64_t tidx, uint64_t k, uint64_t ell, uint64_t W)
{
    /* mismatch time: every time index s >= 1 at which x_j(s) != y_j(s-1)
     * counts once for clone j (the per-clone share of the time the pair
     * spends apart before it meets, Algorithm 3; zero after the meeting) */
    if (tidx >= 1)
        for (int32_t e = 0; e < s->nmis; ++e) acc_add(&s->rmis, s->mis[e], 1);
    if (tidx >= k && tidx <= ell)
        for (int32_t e = 0; e < s->X.npos; ++e) acc_add(&s->rep, s->X.pos[e], 1);
    if (tidx >= k + 1 && s->nmis > 0) {
        uint64_t g = tidx - k < W ? tidx - k : W;
        for (int32_t e = 0; e < s->nmis; ++e) {
            int32_t j = s->mis[e];
            int64_t diff = (int64_t)s->X.x[j] - (int64_t)s->Y.x[j];
            acc_add(&s->rep, j, (int64_t)((uint64_t)diff * g));
        }
    }
}

static void trace_state(trace_t *tr, const scratch_t *s, int32_t n, uint64_t xt, int with_y, uint64_t yt)
{
    if (!tr) return;
    if (xt > tr->max_len || (with_y && yt >= tr->max_len)) { tr->overflow = 1; return; }
    memcpy(tr->X + xt * (uint64_t)n, s->X.x, (size_t)n);
    if (with_y) memcpy(tr->Y + yt * (uint64_t)n, s->Y.x, (size_t)n);
}

/* Z_0 ~ nu for nu = the prior (reading; the paper leaves nu open): clones
 * independent, Pr{Z_0,i = 1} = floor(q 2^32) / 2^32, clone i positive when
 * its 32-bit uniform is below floor(q 2^32); the uniform of clone i is word
 * i mod 4 of the Philox block with counter (floor(i/4), r, p, g + 2^25).
 * X_0 = Y_0 = Z_0 (Algorithm 3). */
static void draw_prior_state(const mo_model *M, const mo_params *P, uint32_t p, uint32_t r, scratch_t *s)
{
    const uint64_t Q = (uint64_t)floor(ldexp(M->q, 32));
    const uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
    for (int32_t i = 0; i < M->n; ++i) {
        uint32_t ctr[4] = {(uint32_t)(i / 4), r, p, (uint32_t)P->instance_id + (1u << 25)};
        uint32_t w[4];
        mo_philox4x32_10(ctr, key, w);
        if ((uint64_t)w[i % 4] < Q) {
            chain_set(M, &s->X, i, 1);
            chain_set(M, &s->Y, i, 1);
        }
    }
}

/* One coupled replication (Algorithm 3): X_0 = Y_0 = Z_0 ~ nu; the pre-lag
 * draw moves X only; every later draw (I_t, U_t) moves X_t -> X_{t+1} and
 * Y_{t-1} -> Y_t with the same numbers; tau_1 = inf{t >= 1 : X_t = Y_{t-1}};
 * the loop runs while t < l or X_t != Y_{t-1}.  Both chains keep moving
 * after the meeting, literally as written (they stay together by
 * Theorem 1 (d)). */
static int run_replication(const mo_model *M, const mo_params *P, uint32_t p, uint32_t r,
                           scratch_t *s, rep_out_t *out, trace_t *tr)
{
    const uint64_t k = P->k, ell = P->ell, W = P->ell - P->k + 1;
    const uint32_t g = (uint32_t)P->instance_id, b = (uint32_t)P->u_hi_bits;
    uint64_t cap = MO_MAX_DRAWS;
    if (P->max_steps) cap = P->max_steps > ell ? P->max_steps : ell;

    chain_reset(M, &s->X);
    chain_reset(M, &s->Y);
    while (s->nmis > 0) { s->mwhere[s->mis[s->nmis - 1]] = -1; s->nmis--; }
    acc_clear(&s->rep);
    acc_clear(&s->rmis);
    if (P->init_mode == 1) draw_prior_state(M, P, p, r, s);

    /* time index 0 */
    trace_state(tr, s, M->n, 0, 1, 0);
    add_time_index(s, 0, k, ell, W);

    /* pre-lag draw t = 0 */
    mo_draw_t d = draw_numbers(P->seed, g, p, r, 0, b);
    int32_t I = site_of(M, d.site_word);
    if (tr && 0 < tr->max_len) { tr->I[0] = I; tr->U[0] = d.u53; }
    chain_set(M, &s->X, I, gibbs_value(M, &s->X, I, d.u53));
    mis_update(s, I);
    uint64_t draws = 1;
    trace_state(tr, s, M->n, 1, 0, 0);
    add_time_index(s, 1, k, ell, W);
    int met = (s->nmis == 0);
    uint64_t tau = met ? 1 : 0;
    int capped = 0;

    while (draws < ell || !met) {
        if (!met && draws >= cap) { capped = 1; break; }
        uint64_t t = draws;
        d = draw_numbers(P->seed, g, p, r, t, b);
        I = site_of(M, d.site_word);
        if (tr && t < tr->max_len) { tr->I[t] = I; tr->U[t] = d.u53; }
        uint8_t xn = gibbs_value(M, &s->X, I, d.u53);
        uint8_t yn = gibbs_value(M, &s->Y, I, d.u53);
        chain_set(M, &s->X, I, xn);
        chain_set(M, &s->Y, I, yn);
        mis_update(s, I);
        draws = t + 1;
        trace_state(tr, s, M->n, draws, 1, t);
        add_time_index(s, draws, k, ell, W);
        if (!met && s->nmis == 0) { met = 1; tau = draws; }
        if (met && s->nmis != 0) return MO_EINVAL;  /* faithfulness violated: cannot happen */
    }
    out->C = draws;
    out->tau = capped ? 0 : tau;
    out->capped = capped;
    return MO_OK;
}

/* Trace of one replication (tests; small n). */
int mo_trace(const mo_model *M, const mo_params *P, uint32_t p, uint32_t r, uint64_t max_len,
             uint8_t *X, uint8_t *Y, int32_t *I, uint64_t *U, int64_t *numer, int64_t *mismatch, uint64_t out[3])
{
    if (P->k > P->ell || P->u_hi_bits < 1 || P->u_hi_bits > 32 || P->init_mode > 1) return MO_EINVAL;
    scratch_t s;
    if (scratch_alloc(&s, M->n, M->m)) { scratch_free(&s); return MO_ENOMEM; }
    trace_t tr = {max_len, X, Y, I, U, 0};
    rep_out_t ro;
    int rc = run_replication(M, P, p, r, &s, &ro, &tr);
    if (!rc) {
        for (int32_t j = 0; j < M->n; ++j) numer[j] = s.rep.v[j];
        if (mismatch) for (int32_t j = 0; j < M->n; ++j) mismatch[j] = s.rmis.v[j];
        out[0] = ro.C; out[1] = ro.tau; out[2] = (uint64_t)ro.capped;
        if (tr.overflow) rc = MO_ETOOLONG;
    }
    scratch_free(&s);
    return rc;
}

/* ------------------------------------------------------------------------
 * Fixed-budget slots (Algorithm 4; supplementary "Fixed-Budget GPU
 * Execution and Parallel Aggregation"): C_{p,r} = max{l, tau_{p,r}},
 * S_p(r) = sum_{u<=r} C_{p,u}.  Replication r+1 starts iff S_p(r) < B.
 * Replications with S_p(r) <= B are retained; if none is (N_p(B) = 0) the
 * first one is retained; later ones completing beyond B are discarded.
 * Literal: a started replication always runs to its end, even one that is
 * certain to be discarded.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint32_t nstar;        /* N*_p(B) */
    uint64_t s_ret;        /* S_p(N*) */
    uint64_t disc_C;       /* C of the discarded replication, 0 if none */
    int32_t nent;          /* sparse slot numerator */
    int32_t *ent_j;
    int64_t *ent_v;
} slot_rec_t;

typedef struct {
    uint64_t retained_units, single_site, reps_retained, cap_hits, zero_completion,
             tau_sum, tau_max, reps_discarded, discarded_units, nstar_max;
} stats_t;

enum {
    ST_RETAINED_UNITS = 0, ST_SINGLE_SITE, ST_REPS_RETAINED, ST_CAP_HITS, ST_ZERO_COMPLETION,
    ST_TAU_SUM, ST_TAU_MAX, ST_REPS_DISCARDED, ST_DISCARDED_UNITS, ST_NSTAR_MAX, ST_COUNT
};

static int run_slot(const mo_model *M, const mo_params *P, uint64_t B, uint32_t p,
                    scratch_t *s, slot_rec_t *rec, stats_t *st, uint64_t *hist, uint64_t *mis_tot)
{
    acc_clear(&s->slot);
    uint64_t S = 0;
    uint32_t nret = 0;
    rec->disc_C = 0;
    for (uint32_t r = 1;; ++r) {
        if (r >= 2 && (!P->refill || S >= B)) break;
        rep_out_t ro;
        int rc = run_replication(M, P, p, r, s, &ro, NULL);
        if (rc) return rc;
        int retained = (r == 1) || (S + ro.C <= B);
        S += ro.C;
        if (!retained) {
            rec->disc_C = ro.C;
            st->reps_discarded += 1;
            st->discarded_units += ro.C;
            break;
        }
        nret += 1;
        acc_merge(&s->slot, &s->rep);
        if (mis_tot)
            for (int32_t e = 0; e < s->rmis.nlist; ++e)
                mis_tot[s->rmis.list[e]] += (uint64_t)s->rmis.v[s->rmis.list[e]];
        st->retained_units += ro.C;
        st->reps_retained += 1;
        if (ro.capped) {
            st->cap_hits += 1;
            st->single_site += 1 + 2 * (ro.C - 1);
        } else {
            uint64_t mt = ro.tau < ro.C ? ro.tau : ro.C;
            st->single_site += 1 + 2 * (mt - 1) + (ro.C - mt);
            st->tau_sum += ro.tau;
            if (ro.tau > st->tau_max) st->tau_max = ro.tau;
            uint64_t bin = ro.tau / P->hist_width;
            if (bin >= P->hist_bins) bin = P->hist_bins - 1;
            hist[bin] += 1;
        }
        if (r == 1 && ro.C > B) st->zero_completion += 1;
    }
    rec->nstar = nret;
    rec->s_ret = 0;
    /* S_p(N*): cumulative cost of the retained replications */
    rec->s_ret = S - rec->disc_C;
    if (nret > st->nstar_max) st->nstar_max = nret;
    rec->nent = s->slot.nlist;
    rec->ent_j = (int32_t *)malloc((size_t)(rec->nent > 0 ? rec->nent : 1) * sizeof(int32_t));
    rec->ent_v = (int64_t *)malloc((size_t)(rec->nent > 0 ? rec->nent : 1) * sizeof(int64_t));
    if (!rec->ent_j || !rec->ent_v) return MO_ENOMEM;
    for (int32_t t = 0; t < rec->nent; ++t) {
        rec->ent_j[t] = s->slot.list[t];
        rec->ent_v[t] = s->slot.v[s->slot.list[t]];
    }
    return MO_OK;
}

/* Full run.  Outputs (Section "Coupled Estimator and Fixed-Budget GPU
 * Execution", the aggregate p_CT):
 *   A_pj = (1/N*_p) sum_{r<=N*_p} H^{(p,r)}_{k:l}(h_j) = V_pj / (W N*_p),
 *   marginal_j = (1/P) sum_p A_pj  (FP64, slots in ascending order),
 *   stderr_j = sqrt( sum_p (A_pj - marginal_j)^2 / (P-1) / P )  (reading:
 *   slots are i.i.d. by Assumption 2; NaN when P = 1).
 * Optional outputs: per-slot N*, S_p(N*), discarded C; integer buckets
 * bucket[n-1][j] = sum_{p: N*_p = n} V_pj and the 128-bit sums of V_pj^2;
 * mismatch[j] = the mismatch time of clone j summed over every retained
 * replication of every slot. */
int mo_run(const mo_model *M, const mo_params *P, double *marginals, double *stderr_out,
           uint64_t *hist, uint64_t *stats_out, uint32_t *slot_nstar, uint64_t *slot_sret,
           uint64_t *slot_disc, int64_t *bucket1, uint64_t *bucket2, uint64_t nbuckets,
           uint64_t *mismatch, int32_t nthreads)
{
    if (P->slots == 0 || P->slots > 0xFFFFFFFFull) return MO_EINVAL;
    if (P->k > P->ell || P->ell > (1ull << 31)) return MO_EINVAL;
    if (P->hist_bins == 0 || P->hist_width == 0) return MO_EINVAL;
    if (P->u_hi_bits < 1 || P->u_hi_bits > 32 || P->init_mode > 1) return MO_EINVAL;
    if (P->instance_id >= (1ull << 24)) return MO_EINVAL;
    if (P->max_steps && P->max_steps < (P->ell > 1 ? P->ell : 1)) return MO_EINVAL;
    const int32_t n = M->n;
    const uint64_t Pn = P->slots, B = P->budget / P->slots, W = P->ell - P->k + 1;
    slot_rec_t *recs = (slot_rec_t *)calloc((size_t)Pn, sizeof(slot_rec_t));
    if (!recs) return MO_ENOMEM;
    int rc = MO_OK;
    stats_t total;
    memset(&total, 0, sizeof(total));
    uint64_t *hist_total = (uint64_t *)calloc((size_t)P->hist_bins, sizeof(uint64_t));
    uint64_t *mis_total = (uint64_t *)calloc((size_t)n, sizeof(uint64_t));
    if (!hist_total || !mis_total) { free(recs); free(hist_total); free(mis_total); return MO_ENOMEM; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        scratch_t s;
        stats_t st;
        memset(&st, 0, sizeof(st));
        uint64_t *h = (uint64_t *)calloc((size_t)P->hist_bins, sizeof(uint64_t));
        uint64_t *dm = mismatch ? (uint64_t *)calloc((size_t)n, sizeof(uint64_t)) : NULL;
        int lrc = scratch_alloc(&s, n, M->m);
        if (!h || (mismatch && !dm)) lrc = MO_ENOMEM;
#pragma omp for schedule(dynamic, 8)
        for (int64_t p = 0; p < (int64_t)Pn; ++p) {
            if (lrc) continue;
            lrc = run_slot(M, P, B, (uint32_t)p, &s, &recs[p], &st, h, dm);
        }
#pragma omp critical
        {
            if (lrc && !rc) rc = lrc;
            total.retained_units += st.retained_units;
            total.single_site += st.single_site;
            total.reps_retained += st.reps_retained;
            total.cap_hits += st.cap_hits;
            total.zero_completion += st.zero_completion;
            total.tau_sum += st.tau_sum;
            if (st.tau_max > total.tau_max) total.tau_max = st.tau_max;
            total.reps_discarded += st.reps_discarded;
            total.discarded_units += st.discarded_units;
            if (st.nstar_max > total.nstar_max) total.nstar_max = st.nstar_max;
            if (h) for (uint64_t b = 0; b < P->hist_bins; ++b) hist_total[b] += h[b];
            if (dm) for (int32_t j = 0; j < n; ++j) mis_total[j] += dm[j];
        }
        free(h);
        free(dm);
        scratch_free(&s);
    }
    if (rc) goto done;

    /* Aggregate in slot order. */
    double *theta = (double *)calloc((size_t)n, sizeof(double));
    double *arow = (double *)calloc((size_t)n, sizeof(double));
    double *ss = (double *)calloc((size_t)n, sizeof(double));
    if (!theta || !arow || !ss) { free(theta); free(arow); free(ss); rc = MO_ENOMEM; goto done; }
    for (uint64_t p = 0; p < Pn; ++p) {
        double den = (double)(W * (uint64_t)recs[p].nstar);
        for (int32_t e = 0; e < recs[p].nent; ++e)
            theta[recs[p].ent_j[e]] += (double)recs[p].ent_v[e] / den;
    }
    for (int32_t j = 0; j < n; ++j) theta[j] = theta[j] / (double)Pn;
    for (uint64_t p = 0; p < Pn; ++p) {
        double den = (double)(W * (uint64_t)recs[p].nstar);
        for (int32_t e = 0; e < recs[p].nent; ++e)
            arow[recs[p].ent_j[e]] = (double)recs[p].ent_v[e] / den;
        for (int32_t j = 0; j < n; ++j) {
            double dv = arow[j] - theta[j];
            ss[j] += dv * dv;
        }
        for (int32_t e = 0; e < recs[p].nent; ++e) arow[recs[p].ent_j[e]] = 0.0;
    }
    for (int32_t j = 0; j < n; ++j) {
        marginals[j] = theta[j];
        stderr_out[j] = (Pn > 1) ? sqrt(ss[j] / (double)(Pn - 1) / (double)Pn) : NAN;
    }
    free(theta); free(arow); free(ss);

    if (bucket1 || bucket2) {
        if (total.nstar_max > nbuckets) { rc = MO_EINVAL; goto done; }
        for (uint64_t p = 0; p < Pn; ++p) {
            uint64_t row = (uint64_t)(recs[p].nstar - 1) * (uint64_t)n;
            for (int32_t e = 0; e < recs[p].nent; ++e) {
                int32_t j = recs[p].ent_j[e];
                int64_t v = recs[p].ent_v[e];
                if (bucket1) bucket1[row + j] = (int64_t)((uint64_t)bucket1[row + j] + (uint64_t)v);
                if (bucket2) {
                    unsigned __int128 sq = (unsigned __int128)((__int128)v * (__int128)v);
                    unsigned __int128 cur = ((unsigned __int128)bucket2[2 * (row + j) + 1] << 64) |
                                            bucket2[2 * (row + j)];
                    cur += sq;
                    bucket2[2 * (row + j)] = (uint64_t)cur;
                    bucket2[2 * (row + j) + 1] = (uint64_t)(cur >> 64);
                }
            }
        }
    }
    for (uint64_t b = 0; b < P->hist_bins; ++b) hist[b] = hist_total[b];
    if (mismatch) memcpy(mismatch, mis_total, (size_t)n * sizeof(uint64_t));
    stats_out[ST_RETAINED_UNITS] = total.retained_units;
    stats_out[ST_SINGLE_SITE] = total.single_site;
    stats_out[ST_REPS_RETAINED] = total.reps_retained;
    stats_out[ST_CAP_HITS] = total.cap_hits;
    stats_out[ST_ZERO_COMPLETION] = total.zero_completion;
    stats_out[ST_TAU_SUM] = total.tau_sum;
    stats_out[ST_TAU_MAX] = total.tau_max;
    stats_out[ST_REPS_DISCARDED] = total.reps_discarded;
    stats_out[ST_DISCARDED_UNITS] = total.discarded_units;
    stats_out[ST_NSTAR_MAX] = total.nstar_max;
    for (uint64_t p = 0; p < Pn; ++p) {
        if (slot_nstar) slot_nstar[p] = recs[p].nstar;
        if (slot_sret) slot_sret[p] = recs[p].s_ret;
        if (slot_disc) slot_disc[p] = recs[p].disc_C;
    }
done:
    for (uint64_t p = 0; p < Pn; ++p) { free(recs[p].ent_j); free(recs[p].ent_v); }
    free(recs);
    free(hist_total);
    free(mis_total);
    return rc;
}

/* Numerator of one slot, dense (tests: sampled slots at full size). */
int mo_slot(const mo_model *M, const mo_params *P, uint32_t p, int64_t *numer, uint64_t out[3])
{
    if (P->k > P->ell || P->u_hi_bits < 1 || P->u_hi_bits > 32 || P->slots == 0 || P->init_mode > 1) return MO_EINVAL;
    if (P->hist_bins == 0 || P->hist_width == 0) return MO_EINVAL;
    scratch_t s;
    if (scratch_alloc(&s, M->n, M->m)) { scratch_free(&s); return MO_ENOMEM; }
    stats_t st;
    memset(&st, 0, sizeof(st));
    uint64_t *h = (uint64_t *)calloc((size_t)P->hist_bins, sizeof(uint64_t));
    slot_rec_t rec;
    memset(&rec, 0, sizeof(rec));
    int rc = h ? run_slot(M, P, P->budget / P->slots, p, &s, &rec, &st, h, NULL) : MO_ENOMEM;
    if (!rc) {
        memset(numer, 0, (size_t)M->n * sizeof(int64_t));
        for (int32_t e = 0; e < rec.nent; ++e) numer[rec.ent_j[e]] = rec.ent_v[e];
        out[0] = rec.nstar; out[1] = rec.s_ret; out[2] = rec.disc_C;
    }
    free(rec.ent_j); free(rec.ent_v); free(h);
    scratch_free(&s);
    return rc;
}


/* ------------------------------------------------------------------------
 * The same entry points in the shape of the library's C ABI (declared in
 * mcpd_oracle.h): thin wrappers over the functions above.
 * ---------------------------------------------------------------------- */
void mcpd_oracle_opts_init(mcpd_oracle_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->refill = 1;
    o->hist_bins = 64;
    o->u_hi_bits = 32;
}

int mcpd_oracle_create(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx, const uint8_t *y,
                       double fp, double fn, double prior, mcpd_oracle_instance **out)
{
    if (!out) return MO_EINVAL;
    *out = NULL;
    if (!row_ptr || !pool_idx || !y) return MO_EINVAL;
    mo_model *M = mo_model_create(n, m, row_ptr, pool_idx, y, fp, fn, prior, NULL);
    if (!M) return MO_EINVAL;
    *out = M;
    return MO_OK;
}

int mcpd_oracle_set_weights(mcpd_oracle_instance *M, const double *w)
{
    if (!M) return MO_EINVAL;
    double *nw = (double *)malloc((size_t)M->n * sizeof(double));
    double *s = (double *)malloc((size_t)M->n * sizeof(double));
    uint64_t *mass = (uint64_t *)malloc((size_t)M->n * sizeof(uint64_t));
    int rc = (nw && s && mass) ? MO_OK : MO_ENOMEM;
    if (!rc) {
        if (w) memcpy(nw, w, (size_t)M->n * sizeof(double));
        else rc = mo_score_weights(M->n, M->m, M->row_ptr, M->pool_idx, M->y, M->fp, M->fn, M->q, s, nw);
    }
    if (!rc) rc = mo_quantize(M->n, nw, mass);
    if (!rc) {
        memcpy(M->w, nw, (size_t)M->n * sizeof(double));
        memcpy(M->mass, mass, (size_t)M->n * sizeof(uint64_t));
        free(M->athr);
        free(M->alias);
        M->athr = NULL;
        M->alias = NULL;
        rc = build_alias(M);
    }
    free(nw); free(s); free(mass);
    return rc;
}

int mcpd_oracle_get_weights(const mcpd_oracle_instance *M, double *w_exact, uint64_t *mass)
{
    if (!M) return MO_EINVAL;
    for (int32_t i = 0; i < M->n; ++i) {
        if (w_exact) w_exact[i] = (double)M->mass[i] / 4294967296.0;
        if (mass) mass[i] = M->mass[i];
    }
    return MO_OK;
}

static void params_from(const mcpd_oracle_instance *M, const mcpd_oracle_opts *o, uint64_t budget, uint32_t slots,
                        uint32_t k, uint32_t m, uint64_t seed, mo_params *P)
{
    mcpd_oracle_opts d;
    if (!o) { mcpd_oracle_opts_init(&d); o = &d; }
    P->budget = budget; P->slots = slots; P->k = k; P->ell = m; P->seed = seed;
    P->max_steps = o->max_steps; P->refill = o->refill; P->hist_bins = o->hist_bins;
    P->hist_width = o->hist_width ? o->hist_width : (uint64_t)M->n;
    P->u_hi_bits = o->u_hi_bits; P->instance_id = o->instance_id; P->init_mode = o->init_mode;
}

int mcpd_oracle_run_unbiased(mcpd_oracle_instance *M, uint64_t budget, uint32_t slots, uint32_t k, uint32_t m,
                             uint64_t seed, const mcpd_oracle_opts *o, double *marginals, double *stderr_out,
                             uint64_t *hist, mcpd_oracle_stats *stats)
{
    if (!M || !marginals || !stderr_out || !hist) return MO_EINVAL;
    mo_params P;
    params_from(M, o, budget, slots, k, m, seed, &P);
    uint64_t st[ST_COUNT];
    int rc = mo_run(M, &P, marginals, stderr_out, hist, st, o ? o->slot_nstar : NULL, o ? o->slot_units : NULL, NULL,
                    o ? o->bucket_sum : NULL, o ? o->bucket_sumsq : NULL, o ? o->bucket_rows : 0,
                    o ? o->mismatch : NULL, o ? o->nthreads : 0);
    if (!rc && stats) {
        stats->retained_units = st[ST_RETAINED_UNITS];
        stats->single_site_updates = st[ST_SINGLE_SITE];
        stats->reps_retained = st[ST_REPS_RETAINED];
        stats->cap_hits = st[ST_CAP_HITS];
        stats->zero_completion_slots = st[ST_ZERO_COMPLETION];
        stats->tau_sum = st[ST_TAU_SUM];
        stats->tau_max = st[ST_TAU_MAX];
        stats->reps_discarded = st[ST_REPS_DISCARDED];
        stats->discarded_units = st[ST_DISCARDED_UNITS];
        stats->nstar_max = st[ST_NSTAR_MAX];
    }
    return rc;
}

int mcpd_oracle_trace(mcpd_oracle_instance *M, uint32_t slot, uint32_t r, uint64_t seed, uint32_t k, uint32_t m,
                      const mcpd_oracle_opts *o, uint64_t max_len, uint8_t *X, uint8_t *Y, int32_t *I, uint64_t *U,
                      int64_t *numer, int64_t *mismatch, uint64_t out[3])
{
    if (!M || !X || !Y || !I || !U || !out || r < 1) return MO_EINVAL;
    mo_params P;
    params_from(M, o, 0, 1, k, m, seed, &P);
    int64_t *nbuf = numer ? numer : (int64_t *)malloc((size_t)M->n * sizeof(int64_t));
    if (!nbuf) return MO_ENOMEM;
    int rc = mo_trace(M, &P, slot, r, max_len, X, Y, I, U, nbuf, mismatch, out);
    if (!numer) free(nbuf);
    return rc;
}

void mcpd_oracle_destroy(mcpd_oracle_instance *M) { mo_model_free(M); }
