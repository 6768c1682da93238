// Host side of the C ABI (include/mcpd.h): validation, instance tables,
// launch planning and the final FP64 reduction of the integer buckets.
//
// Instance tables built here, once per instance (the paper computes the
// score weights "only once, before the chain starts", Section
// "Score-Weighted Update Gibbs Sampler"):
//   * score weights w (or caller weights) -> integer masses M_i, sum 2^32
//   * the alias table of the site draw
//   * clone rows: pool index | outcome << top bit, ascending
//   * the decision thresholds floor(p * 2^53) for every ordered pattern of
//     free-pool outcomes (at most 2^(dmax+1) - 1 values of the FP64 log-odds)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mcpd.h"
#include "mcpd_device.h"

struct mcpd_instance {
    int32_t n = 0, m = 0, dmax = 0, fmt = 0, abits = 1;
    uint32_t row_bytes = 8, thr_len = 1;
    double fp = 0, fn = 0, q = 0;
    std::vector<int32_t> row_ptr, pool_idx;
    std::vector<uint8_t> y;
    std::vector<uint64_t> mass;
    hipStream_t stream = nullptr;
    int device = 0;
    int cus = 0;
    // device tables
    uint32_t *d_alias = nullptr, *d_rows = nullptr;
    uint64_t *d_thr = nullptr;
    // workspace reused across runs
    int64_t *d_acc = nullptr;
    size_t acc_lanes = 0;
    uint32_t *d_lists = nullptr;
    uint32_t *d_gstate = nullptr;
    size_t gstate_words = 0;
    uint64_t *d_lane_stats = nullptr;
    size_t lane_stats_cap = 0;
    int64_t *d_S1 = nullptr;
    uint64_t *d_S2 = nullptr;
    size_t bucket_cap = 0, bucket2_cap = 0;
    uint64_t *d_small = nullptr;   // hist + stats + ctrl
    size_t small_cap = 0;
    uint32_t *d_slot_nstar = nullptr;
    uint64_t *d_slot_units = nullptr;
    size_t slot_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(MCPD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

constexpr uint32_t LIST_CAP = 64;

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS bytes of the table copy: thresholds, alias table, clone rows.
size_t table_bytes(size_t thr_len, int abits, size_t n, size_t row_bytes)
{
    return align16(align16(align16(thr_len * 8) + ((size_t)4 << abits)) + n * row_bytes);
}
constexpr size_t LDS_BYTES = 160 * 1024;

int validate_design(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx,
                    const uint8_t *y, double fp, double fn, double q, int32_t *dmax_out)
{
    if (n <= 0 || n > MCPD_MAX_CLONES) return fail(MCPD_EINVAL, "n_clones out of range");
    if (m <= 0 || m > 32767) return fail(MCPD_EINVAL, "n_pools out of range");
    if (!row_ptr || !pool_idx || !y) return fail(MCPD_EINVAL, "null design pointer");
    if (!(fp > 0.0 && fp < 1.0 && fn > 0.0 && fn < 1.0 && q > 0.0 && q < 1.0))
        return fail(MCPD_EINVAL, "fp, fn and prior must lie in (0,1)");
    if (row_ptr[0] != 0) return fail(MCPD_EINVAL, "row_ptr[0] != 0");
    std::vector<int32_t> size(m, 0);
    int32_t dmax = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return fail(MCPD_EINVAL, "row_ptr decreasing");
        const int32_t d = row_ptr[i + 1] - row_ptr[i];
        if (d > MCPD_MAX_DEGREE) return fail(MCPD_EINVAL, "clone degree above MCPD_MAX_DEGREE");
        dmax = std::max(dmax, d);
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = pool_idx[e];
            if (j < 0 || j >= m) return fail(MCPD_EINVAL, "pool index out of range");
            if (e > row_ptr[i] && j <= pool_idx[e - 1])
                return fail(MCPD_EINVAL, "pool indices not strictly ascending in a row");
            if (++size[j] > MCPD_MAX_POOL_SIZE) return fail(MCPD_EINVAL, "pool size above MCPD_MAX_POOL_SIZE");
        }
    }
    for (int32_t j = 0; j < m; ++j)
        if (y[j] > 1) return fail(MCPD_EINVAL, "outcome not 0/1");
    if (dmax_out) *dmax_out = dmax;
    return MCPD_OK;
}

// Score weights, Section "Score-Weighted Update Gibbs Sampler" (see header).
void score_weights(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx,
                   const uint8_t *y, double fp, double fn, double q, double *s, double *w)
{
    (void)q;
    const double a_pos = std::log(1.0 - fn) - std::log(fp);
    const double a_neg = std::log(fn) - std::log(1.0 - fp);
    std::vector<int64_t> d(m, 0);
    for (int32_t e = 0; e < row_ptr[n]; ++e) d[pool_idx[e]] += 1;
    double smax = -INFINITY, smin = INFINITY;
    for (int32_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = pool_idx[e];
            acc = acc + (double)d[j] * (y[j] ? a_pos : a_neg);
        }
        s[i] = acc;
        smax = std::max(smax, acc);
        smin = std::min(smin, acc);
    }
    const double gamma = 100.0 * (double)n;
    const double tau = smax > smin ? std::log(gamma) / (smax - smin) : 0.0;
    std::vector<double> e(n);
    double esum = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        e[i] = std::exp(tau * (s[i] - smax));
        esum = esum + e[i];
    }
    for (int32_t i = 0; i < n; ++i) w[i] = 0.5 * (e[i] / esum) + 0.5 / (double)n;
}

// Integer masses M_i >= 1 with sum 2^32: 1 + floor(v_i (2^32 - n)), the
// leftover units to the largest remainders (ties to the lower index).
int quantize(int32_t n, const double *w, std::vector<uint64_t> &mass)
{
    double wsum = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (!(w[i] > 0.0) || !std::isfinite(w[i])) return fail(MCPD_EINVAL, "weights must be finite and > 0");
        wsum = wsum + w[i];
    }
    if (!std::isfinite(wsum)) return fail(MCPD_EINVAL, "weights sum is not finite");
    const double S = 4294967296.0 - (double)n;
    mass.assign(n, 0);
    std::vector<std::pair<double, int32_t>> rem(n);
    uint64_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
        const double f = (w[i] / wsum) * S;
        const double fl = std::floor(f);
        const uint64_t mi = 1u + (uint64_t)fl;
        if (mi > 4294967296ull) return fail(MCPD_EINVAL, "weight quantization overflow");
        mass[i] = mi;
        total += mi;
        rem[i] = {f - fl, i};
    }
    const int64_t D = (int64_t)4294967296LL - (int64_t)total;
    if (D < 0 || D > n) return fail(MCPD_EINVAL, "weight quantization failed");
    std::sort(rem.begin(), rem.end(), [](const auto &x, const auto &y_) {
        return x.first != y_.first ? x.first > y_.first : x.second < y_.second;
    });
    for (int64_t t = 0; t < D; ++t) mass[rem[t].second] += 1u;
    return MCPD_OK;
}

template <typename T>
int upload(T **dptr, const std::vector<T> &h, hipStream_t s)
{
    if (*dptr) { (void)hipFree(*dptr); *dptr = nullptr; }
    HIP_TRY(hipMalloc(reinterpret_cast<void **>(dptr), std::max<size_t>(1, h.size()) * sizeof(T)));
    if (!h.empty()) HIP_TRY(hipMemcpyAsync(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return MCPD_OK;
}

// Alias table of the site draw from the integer masses (Walker's method,
// built by Vose's procedure): 2^a >= n columns of capacity K = 2^(32-a);
// columns under capacity go on the "small" stack and the others on the
// "large" stack in ascending order; pairs are popped from the tops, the
// small column keeps its mass as threshold and the large one as alias, and
// the large one returns to whichever stack its remaining mass belongs.
// Integer arithmetic keeps Pr{I = i} = M_i / 2^32 exact.  Packed words:
// T_c | A_c << (32 - a), a column that always keeps its clone as 0 | c << (32 - a).
int upload_site_tables(mcpd_instance *I)
{
    const int a = I->abits;
    const size_t N = (size_t)1 << a;
    const uint64_t K = (uint64_t)1 << (32 - a);
    std::vector<uint64_t> mass(N, 0);
    for (int32_t i = 0; i < I->n; ++i) mass[i] = I->mass[i];
    std::vector<size_t> small, large;
    small.reserve(N);
    large.reserve(N);
    for (size_t c = 0; c < N; ++c) (mass[c] < K ? small : large).push_back(c);
    std::vector<uint32_t> words(N);
    const uint32_t sh = 32u - (uint32_t)a;
    while (!small.empty() && !large.empty()) {
        const size_t l = small.back();
        small.pop_back();
        const size_t g = large.back();
        large.pop_back();
        words[l] = (uint32_t)mass[l] | ((uint32_t)g << sh);
        mass[g] -= K - mass[l];
        (mass[g] < K ? small : large).push_back(g);
    }
    for (size_t c : large) words[c] = (uint32_t)c << sh;
    for (size_t c : small) words[c] = (uint32_t)c << sh;
    // Every draw must land on a real clone: aliases below n, and columns
    // past n (mass 0) never keep themselves.
    const uint32_t tmask = (uint32_t)(K - 1);
    for (size_t c = 0; c < N; ++c) {
        const uint32_t A = words[c] >> sh, T = words[c] & tmask;
        if (A >= (uint32_t)I->n || (c >= (size_t)I->n && T != 0))
            return fail(MCPD_EINVAL, "internal: alias table maps outside the clones");
    }
    return upload(&I->d_alias, words, I->stream);
}

void free_ptr(void *p)
{
    if (p) (void)hipFree(p);
}

void release(mcpd_instance *I)
{
    free_ptr(I->d_alias); free_ptr(I->d_rows); free_ptr(I->d_thr); free_ptr(I->d_lane_stats);
    free_ptr(I->d_acc); free_ptr(I->d_lists); free_ptr(I->d_gstate);
    free_ptr(I->d_S1); free_ptr(I->d_S2); free_ptr(I->d_small);
    free_ptr(I->d_slot_nstar); free_ptr(I->d_slot_units);
    if (I->ev0) (void)hipEventDestroy(I->ev0);
    if (I->ev1) (void)hipEventDestroy(I->ev1);
}

template <typename T>
int ensure(T **p, size_t &cap, size_t want)
{
    if (cap >= want && *p) return MCPD_OK;
    free_ptr(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(want, 1) * sizeof(T));
    if (e == hipErrorOutOfMemory) return fail(MCPD_ENOMEM, "device allocation failed");
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    cap = want;
    return MCPD_OK;
}

}  // namespace

extern "C" {

void mcpd_run_opts_init(mcpd_run_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->refill = 1;
    o->hist_bins = 64;
    o->hist_width = 0;
    o->u_hi_bits = 32;
}

const char *mcpd_strerror(int code)
{
    switch (code) {
    case MCPD_OK: return "ok";
    case MCPD_EINVAL: return "invalid argument";
    case MCPD_ENOMEM: return "out of memory";
    case MCPD_EDEVICE: return "device error";
    case MCPD_ECAP: return "a retained pair hit the meeting cap";
    default: return "unknown error";
    }
}

const char *mcpd_last_error(void) { return g_last_error.c_str(); }

int mcpd_score_weights(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx,
                       const uint8_t *y, double fp, double fn, double q, double *s_out, double *w_out)
{
    int rc = validate_design(n, m, row_ptr, pool_idx, y, fp, fn, q, nullptr);
    if (rc) return rc;
    if (!w_out) return fail(MCPD_EINVAL, "w_out is null");
    std::vector<double> s(n);
    score_weights(n, m, row_ptr, pool_idx, y, fp, fn, q, s.data(), w_out);
    if (s_out) std::memcpy(s_out, s.data(), sizeof(double) * n);
    return MCPD_OK;
}

int mcpd_create(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx,
                const uint8_t *y, double fp, double fn, double q, void *hip_stream, mcpd_instance **out)
{
    if (!out) return fail(MCPD_EINVAL, "out is null");
    *out = nullptr;
    int32_t dmax = 0;
    int rc = validate_design(n, m, row_ptr, pool_idx, y, fp, fn, q, &dmax);
    if (rc) return rc;
    mcpd_instance *I = new (std::nothrow) mcpd_instance();
    if (!I) return fail(MCPD_ENOMEM, "host allocation failed");
    I->n = n; I->m = m; I->dmax = dmax; I->fp = fp; I->fn = fn; I->q = q;
    // record format: narrowest entries, shortest compile-time loop >= dmax
    if (m <= 127) {
        I->fmt = dmax <= 4 ? mcpd::FMT_U8_4 : dmax <= 5 ? mcpd::FMT_U8_5 : dmax <= 8 ? mcpd::FMT_U8_8 : mcpd::FMT_U8_12;
    } else {
        I->fmt = dmax <= 4 ? mcpd::FMT_U16_4 : dmax <= 8 ? mcpd::FMT_U16_8 : mcpd::FMT_U16_12;
    }
    I->row_bytes = (uint32_t)mcpd::fmt_row_bytes(I->fmt);
    int ab = 1;
    while ((1 << ab) < n) ++ab;
    I->abits = ab;
    I->row_ptr.assign(row_ptr, row_ptr + n + 1);
    I->pool_idx.assign(pool_idx, pool_idx + row_ptr[n]);
    I->y.assign(y, y + m);
    I->stream = reinterpret_cast<hipStream_t>(hip_stream);

    // weights -> masses (host only; no device needed yet)
    std::vector<double> s(n), w(n);
    score_weights(n, m, row_ptr, pool_idx, y, fp, fn, q, s.data(), w.data());
    rc = quantize(n, w.data(), I->mass);
    if (rc) { delete I; return rc; }

    // rows: entry = pool | outcome << (top bit), ascending, padded with all-ones
    std::vector<uint8_t> rowb((size_t)n * I->row_bytes, 0xFFu);
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const uint32_t j = (uint32_t)pool_idx[e], yj = y[pool_idx[e]];
            const size_t at = (size_t)i * I->row_bytes;
            const int32_t pos = e - row_ptr[i];
            if (!mcpd::fmt_wide(I->fmt)) {
                rowb[at + pos] = (uint8_t)(j | (yj << 7));
            } else {
                const uint16_t v = (uint16_t)(j | (yj << 15));
                std::memcpy(&rowb[at + 2 * pos], &v, 2);
            }
        }
    }
    std::vector<uint32_t> rows(rowb.size() / 4);
    std::memcpy(rows.data(), rowb.data(), rowb.size());

    // thresholds for every ordered pattern of free-pool outcomes: the FP64
    // sum lq + a_{1st} + a_{2nd} + ... in ascending pool order
    const double lq = std::log(q / (1.0 - q));
    const double a_pos = std::log(1.0 - fn) - std::log(fp);
    const double a_neg = std::log(fn) - std::log(1.0 - fp);
    std::vector<uint64_t> thr(((size_t)2 << dmax) - 1);
    I->thr_len = (uint32_t)thr.size();
    for (int len = 0; len <= dmax; ++len) {
        for (uint32_t pat = 0; pat < (1u << len); ++pat) {
            double L = lq;
            for (int b = len - 1; b >= 0; --b) L = L + (((pat >> b) & 1u) ? a_pos : a_neg);
            const double p = 1.0 / (1.0 + std::exp(-L));
            uint64_t T = (uint64_t)(p * 9007199254740992.0);
            if (T > 9007199254740991ull) T = 9007199254740991ull;
            thr[((size_t)1 << len) - 1 + pat] = T;
        }
    }

    hipError_t e = hipGetDevice(&I->device);
    if (e != hipSuccess) { delete I; return hip_fail(e, "hipGetDevice"); }
    e = hipDeviceGetAttribute(&I->cus, hipDeviceAttributeMultiprocessorCount, I->device);
    if (e != hipSuccess) { delete I; return hip_fail(e, "hipDeviceGetAttribute"); }
    if ((rc = upload(&I->d_thr, thr, I->stream)) || (rc = upload(&I->d_rows, rows, I->stream)) ||
        (rc = upload_site_tables(I))) {
        release(I);
        delete I;
        return rc;
    }
    if ((e = hipEventCreate(&I->ev0)) != hipSuccess || (e = hipEventCreate(&I->ev1)) != hipSuccess) {
        release(I);
        delete I;
        return hip_fail(e, "hipEventCreate");
    }
    e = hipStreamSynchronize(I->stream);
    if (e != hipSuccess) { release(I); delete I; return hip_fail(e, "hipStreamSynchronize"); }
    *out = I;
    return MCPD_OK;
}

int mcpd_set_weights(mcpd_instance *I, const double *w)
{
    if (!I) return fail(MCPD_EINVAL, "null instance");
    std::vector<uint64_t> mass;
    int rc;
    if (w) {
        rc = quantize(I->n, w, mass);
    } else {
        std::vector<double> s(I->n), ws(I->n);
        score_weights(I->n, I->m, I->row_ptr.data(), I->pool_idx.data(), I->y.data(), I->fp, I->fn,
                      I->q, s.data(), ws.data());
        rc = quantize(I->n, ws.data(), mass);
    }
    if (rc) return rc;
    I->mass.swap(mass);
    rc = upload_site_tables(I);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(I->stream));
    return MCPD_OK;
}

int mcpd_get_weights(const mcpd_instance *I, double *w_exact, uint64_t *mass)
{
    if (!I) return fail(MCPD_EINVAL, "null instance");
    for (int32_t i = 0; i < I->n; ++i) {
        if (w_exact) w_exact[i] = (double)I->mass[i] / 4294967296.0;
        if (mass) mass[i] = I->mass[i];
    }
    return MCPD_OK;
}

int mcpd_run_unbiased(mcpd_instance *I, uint64_t budget, uint32_t slots, uint32_t k, uint32_t m,
                      uint64_t seed, const mcpd_run_opts *opts_in, double *marginals, double *stderr_out,
                      uint64_t *hist, mcpd_run_stats *stats)
{
    if (!I) return fail(MCPD_EINVAL, "null instance");
    if (!marginals || !stderr_out) return fail(MCPD_EINVAL, "null output");
    mcpd_run_opts opts;
    if (opts_in) opts = *opts_in; else mcpd_run_opts_init(&opts);
    if (slots == 0) return fail(MCPD_EINVAL, "slots must be >= 1");
    if (k > m || m > (1u << 31)) return fail(MCPD_EINVAL, "need 0 <= k <= m <= 2^31");
    if (opts.hist_bins == 0) return fail(MCPD_EINVAL, "hist_bins must be >= 1");
    if (opts.u_hi_bits < 1 || opts.u_hi_bits > 32) return fail(MCPD_EINVAL, "u_hi_bits must be in 1..32");
    if (opts.instance_id >= (1u << 24)) return fail(MCPD_EINVAL, "instance_id must be < 2^24");
    const uint32_t cmin = std::max<uint32_t>(m, 1u);
    if (opts.max_steps && (opts.max_steps < cmin || opts.max_steps > 0xFFFFFFFFull))
        return fail(MCPD_EINVAL, "max_steps must be 0 or in [max(m,1), 2^32-1]");
    const int32_t n = I->n;
    const uint64_t B = budget / slots;
    const uint64_t nb64 = std::max<uint64_t>(1, B / cmin);
    if (nb64 * (uint64_t)n > (1ull << 27)) return fail(MCPD_EINVAL, "budget/slots/m give too many N* buckets");
    const uint32_t nbuckets = (uint32_t)nb64;

    mcpd::RunArgs a;
    std::memset(&a, 0, sizeof(a));
    a.T.alias = I->d_alias; a.T.rows = I->d_rows; a.T.thr = I->d_thr;
    a.T.n = n; a.T.m = I->m; a.T.dmax = I->dmax; a.T.fmt = I->fmt;
    a.T.abits = (uint32_t)I->abits;
    a.T.row_bytes = I->row_bytes;
    a.T.thr_len = I->thr_len;
    a.B = B;
    a.capmax = opts.max_steps ? (uint32_t)std::max<uint64_t>(opts.max_steps, m) : 0xFFFFFFFFu;
    a.seed = seed;
    a.P = slots;
    a.k = k; a.ell = m; a.W = m - k + 1; a.cmin = cmin;
    a.g = opts.instance_id;
    a.refill = opts.refill ? 1u : 0u;
    a.ubits = opts.u_hi_bits;
    a.hist_bins = opts.hist_bins;
    a.hist_width = opts.hist_width ? opts.hist_width : (uint32_t)n;
    a.words_bits = (uint32_t)((n + 15) / 16);
    a.words_cnt = (uint32_t)((I->m + 1) / 2);
    a.list_cap = LIST_CAP;
    a.nbuckets = nbuckets;

    // LDS copy of the read-only tables: thresholds, alias table, clone rows.
    a.tab_off_thr = 0;
    a.tab_off_alias = (uint32_t)align16((size_t)I->thr_len * 8);
    a.tab_off_rows = (uint32_t)align16(a.tab_off_alias + ((size_t)4 << I->abits));
    const size_t tab_bytes = table_bytes(I->thr_len, I->abits, n, I->row_bytes);
    a.tab_bytes = tab_bytes > LDS_BYTES ? 0u : (uint32_t)tab_bytes;

    // Launch plan.  Chain state in LDS needs at least one full wave per SIMD
    // (256 lanes per CU) to be worth it; otherwise the state goes to global
    // memory and more waves hide its latency.  Tables go to LDS when they fit
    // next to whatever else the workgroup keeps there.
    int block = 256;
    bool lds_state = false, lds_tables = false;
    size_t wg_per_cu = 1;
    auto fits = [&](int L, bool sl, bool tl) {
        if (tl && !a.tab_bytes) return false;
        return mcpd::sampler_lds_bytes(a, L, sl, tl) <= LDS_BYTES;
    };
    if (opts.plan > 4) return fail(MCPD_EINVAL, "plan must be 0..4");
    if (opts.plan == 0) {
        if (fits(256, true, true)) { lds_state = lds_tables = true; }
        else if (fits(256, true, false)) { lds_state = true; }
        else { lds_tables = fits(256, false, true); }
    } else {
        lds_state = opts.plan <= 2;
        lds_tables = opts.plan == 1 || opts.plan == 3;
        if (!fits(256, lds_state, lds_tables)) return fail(MCPD_EINVAL, "requested plan does not fit in LDS");
    }
    {
        const size_t per_wg = mcpd::sampler_lds_bytes(a, block, lds_state, lds_tables);
        const size_t by_lds = per_wg ? LDS_BYTES / per_wg : 8;
        const size_t by_waves = lds_state ? 2048 / block : 1024 / block;
        wg_per_cu = std::max<size_t>(1, std::min(by_lds, by_waves));
        if (opts.wg_per_cu) {
            if (opts.wg_per_cu > 8 || opts.wg_per_cu > by_lds)
                return fail(MCPD_EINVAL, "wg_per_cu does not fit");
            wg_per_cu = opts.wg_per_cu;
        }
    }
    const size_t max_lanes = (size_t)I->cus * wg_per_cu * (size_t)block;
    const size_t want_lanes = std::min<size_t>(((size_t)slots + block - 1) / block * block, max_lanes);
    const int grid = (int)(want_lanes / block);
    const size_t lanes = (size_t)grid * block;
    // Workspace.  Numerator rows are kept zero between runs by the kernel.
    int rc;
    if (I->acc_lanes < lanes || !I->d_acc) {
        size_t cap = 0;
        free_ptr(I->d_acc); I->d_acc = nullptr;
        free_ptr(I->d_lists); I->d_lists = nullptr;
        I->acc_lanes = 0;
        if ((rc = ensure(&I->d_acc, cap, lanes * (size_t)n))) return rc;
        HIP_TRY(hipMemsetAsync(I->d_acc, 0, lanes * (size_t)n * sizeof(int64_t), I->stream));
        cap = 0;
        if ((rc = ensure(&I->d_lists, cap, lanes * LIST_CAP))) return rc;
        I->acc_lanes = lanes;
    }
    const size_t words = (size_t)a.words_bits + a.words_cnt;
    if (!lds_state) {
        if ((rc = ensure(&I->d_gstate, I->gstate_words, lanes * words))) return rc;
    }
    if ((rc = ensure(&I->d_S1, I->bucket_cap, (size_t)nbuckets * n))) return rc;
    if ((rc = ensure(&I->d_S2, I->bucket2_cap, (size_t)nbuckets * n * 2))) return rc;
    const size_t small_words = opts.hist_bins + mcpd::ST_COUNT + 2;
    if ((rc = ensure(&I->d_small, I->small_cap, small_words))) return rc;
    if (opts.slot_nstar || opts.slot_units) {
        if (I->slot_cap < slots) {
            free_ptr(I->d_slot_nstar); free_ptr(I->d_slot_units);
            I->d_slot_nstar = nullptr; I->d_slot_units = nullptr;
            size_t c1 = 0, c2 = 0;
            if ((rc = ensure(&I->d_slot_nstar, c1, slots)) || (rc = ensure(&I->d_slot_units, c2, slots))) {
                I->slot_cap = 0;
                return rc;
            }
            I->slot_cap = slots;
        }
    }
    if ((rc = ensure(&I->d_lane_stats, I->lane_stats_cap, lanes * mcpd::ST_COUNT))) return rc;
    a.lane_stats = I->d_lane_stats;
    a.acc = I->d_acc;
    a.lists = I->d_lists;
    a.gstate = lds_state ? nullptr : I->d_gstate;
    a.S1 = I->d_S1;
    a.S2 = I->d_S2;
    a.hist = I->d_small;
    a.stats = I->d_small + opts.hist_bins;
    a.ctrl = reinterpret_cast<uint32_t *>(I->d_small + opts.hist_bins + mcpd::ST_COUNT);
    a.slot_nstar = opts.slot_nstar ? I->d_slot_nstar : nullptr;
    a.slot_units = opts.slot_units ? I->d_slot_units : nullptr;

    HIP_TRY(hipMemsetAsync(I->d_S1, 0, (size_t)nbuckets * n * sizeof(int64_t), I->stream));
    HIP_TRY(hipMemsetAsync(I->d_S2, 0, (size_t)nbuckets * n * 2 * sizeof(uint64_t), I->stream));
    HIP_TRY(hipMemsetAsync(I->d_small, 0, small_words * sizeof(uint64_t), I->stream));

    HIP_TRY(hipEventRecord(I->ev0, I->stream));
    int e = mcpd::launch_sampler(a, grid, block, lds_state, lds_tables, I->stream);
    if (e != hipSuccess) return hip_fail((hipError_t)e, "sampler launch");
    HIP_TRY(hipEventRecord(I->ev1, I->stream));

    std::vector<int64_t> S1((size_t)nbuckets * n);
    std::vector<uint64_t> S2((size_t)nbuckets * n * 2);
    std::vector<uint64_t> small(small_words);
    HIP_TRY(hipMemcpyAsync(S1.data(), I->d_S1, S1.size() * sizeof(int64_t), hipMemcpyDeviceToHost, I->stream));
    HIP_TRY(hipMemcpyAsync(S2.data(), I->d_S2, S2.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, I->stream));
    HIP_TRY(hipMemcpyAsync(small.data(), I->d_small, small_words * sizeof(uint64_t), hipMemcpyDeviceToHost,
                           I->stream));
    if (opts.slot_nstar)
        HIP_TRY(hipMemcpyAsync(opts.slot_nstar, I->d_slot_nstar, (size_t)slots * 4, hipMemcpyDeviceToHost, I->stream));
    if (opts.slot_units)
        HIP_TRY(hipMemcpyAsync(opts.slot_units, I->d_slot_units, (size_t)slots * 8, hipMemcpyDeviceToHost, I->stream));
    HIP_TRY(hipStreamSynchronize(I->stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, I->ev0, I->ev1));

    const uint32_t *ctrl = reinterpret_cast<const uint32_t *>(small.data() + opts.hist_bins + mcpd::ST_COUNT);
    if (ctrl[1] & mcpd::ERR_BUCKETS) return fail(MCPD_EINVAL, "internal: N* above bucket count");
    const uint64_t *st = small.data() + opts.hist_bins;

    // marginal_j = (1/(P W)) sum_n S1[n][j] / n ;  SE from the sums of squares.
    const long double PW = (long double)slots * (long double)a.W;
    const long double W = (long double)a.W;
    for (int32_t j = 0; j < n; ++j) {
        long double sa = 0.0L, sq = 0.0L;
        for (uint32_t r = 0; r < nbuckets; ++r) {
            const size_t idx = (size_t)r * n + j;
            const long double nn = (long double)(r + 1);
            sa += (long double)S1[idx] / nn;
            const long double v2 = (long double)S2[2 * idx + 1] * 18446744073709551616.0L + (long double)S2[2 * idx];
            sq += v2 / (nn * nn);
        }
        marginals[j] = (double)(sa / PW);
        if (slots > 1) {
            const long double sumA = sa / W, sumA2 = sq / (W * W);
            long double var = (sumA2 - sumA * sumA / (long double)slots) / (long double)(slots - 1);
            if (var < 0) var = 0;
            stderr_out[j] = (double)std::sqrt(var / (long double)slots);
        } else {
            stderr_out[j] = NAN;
        }
    }
    if (hist) std::memcpy(hist, small.data(), sizeof(uint64_t) * opts.hist_bins);
    if (opts.bucket_sum || opts.bucket_sumsq) {
        if (st[mcpd::ST_NSTAR_MAX] > opts.bucket_rows) return fail(MCPD_EINVAL, "bucket_rows below N*");
        const size_t rows = std::min<size_t>(opts.bucket_rows, nbuckets);
        if (opts.bucket_sum) {
            std::memset(opts.bucket_sum, 0, sizeof(int64_t) * (size_t)opts.bucket_rows * n);
            std::memcpy(opts.bucket_sum, S1.data(), sizeof(int64_t) * rows * n);
        }
        if (opts.bucket_sumsq) {
            std::memset(opts.bucket_sumsq, 0, sizeof(uint64_t) * 2 * (size_t)opts.bucket_rows * n);
            std::memcpy(opts.bucket_sumsq, S2.data(), sizeof(uint64_t) * 2 * rows * n);
        }
    }
    if (stats) {
        stats->progress_units = st[mcpd::ST_PROGRESS];
        stats->retained_units = st[mcpd::ST_RETAINED_UNITS];
        stats->single_site_updates = st[mcpd::ST_SINGLE_SITE];
        stats->reps_started = st[mcpd::ST_REPS_STARTED];
        stats->reps_retained = st[mcpd::ST_REPS_RETAINED];
        stats->reps_aborted = st[mcpd::ST_REPS_ABORTED];
        stats->cap_hits = st[mcpd::ST_CAP_HITS];
        stats->zero_completion_slots = st[mcpd::ST_ZERO_COMPLETION];
        stats->tau_sum = st[mcpd::ST_TAU_SUM];
        stats->tau_max = st[mcpd::ST_TAU_MAX];
        stats->nstar_max = st[mcpd::ST_NSTAR_MAX];
        stats->rollback_units = st[mcpd::ST_ROLLBACK_UNITS];
        stats->kernel_ms = ms;
        stats->lanes = (uint64_t)lanes;
        stats->lds_state = (lds_state ? 1u : 0u) | (lds_tables ? 2u : 0u);
    }
    if (opts.strict_cap && st[mcpd::ST_CAP_HITS]) return fail(MCPD_ECAP, "a retained pair hit the meeting cap");
    return MCPD_OK;
}

void mcpd_destroy(mcpd_instance *I)
{
    if (!I) return;
    (void)hipStreamSynchronize(I->stream);
    release(I);
    delete I;
}

}  // extern "C"
