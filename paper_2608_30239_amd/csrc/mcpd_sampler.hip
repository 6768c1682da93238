// Persistent slot-refill sampler for unbiased Markov chain pool decoding on
// gfx950.
//
// One lane (lane kernel) or one group of lanes (cooperative kernel) owns one
// logical slot at a time and runs its i.i.d. coupled replications
// (Algorithm 3) one after the other, as the fixed-budget scheduler of
// Algorithm 4 prescribes for a persistent worker.  Slots are handed
// out dynamically from a per-instance counter; the result does not depend on
// which lane runs which slot because every random number is keyed by
// (instance, slot, replication, draw).
//
// One launch serves a batch of instances of any sizes.  A workgroup takes a
// ticket from a global queue, which names the instance it joins; it places
// that instance's tables (and chain state, if it fits) in LDS, its lanes take
// the instance's slots until none is left, and the workgroup takes the next
// ticket.  The host orders the tickets (longest slots first) and sizes them.
//
// Per-lane chain state (both chains X and Y):
//   bit words   : 16 clones per dword, clone i at bits 2(i mod 16) (x) and
//                 2(i mod 16)+1 (y)
//   count words : 2 pools per dword, pool j at byte 2(j mod 2) (c^X_j) and
//                 2(j mod 2)+1 (c^Y_j), c_j = sum_i A_ji x_i
// laid out structure-of-arrays with the lane index fastest, so that the 64
// lanes of a wave touching any word index hit 64 distinct banks.  The state
// lives in LDS when the instance fits, otherwise in global memory with the
// same layout.  The read-only instance tables (thresholds, the alias table
// of the site draw and the clone rows) are copied into LDS when they fit, so
// that a draw touches no global memory.
//
// A draw is a short chain of LDS round trips: alias column (site in O(1),
// no search) -> clone row -> all count words of the clone at once -> the
// threshold of the free-pool pattern.  Control flow inside a draw is
// branch-free except for the rare flip, event and bookkeeping paths.
//
// Estimator: the numerator V_j = W H_{k:l}(h_j) (Section "Coupled Estimator
// and Fixed-Budget GPU Execution") is accumulated exactly in 64-bit integers
// from flip events only.  With Delta_j(s) = x_j(s) - y_j(s-1) and
// G(t) = sum_{s=k+1}^{t} min(s-k, W), exchanging the sums gives
//   V_j = sum_{flips of x_j at time s} dx (l - max(s,k) + 1)^+
//       - sum_{changes c of Delta_j at time s} c G(s-1)
//       (+ G(C) Delta_j(C) for a pair stopped by the cap),
// using sum_s c = Delta_j(C) (= 0 once the pair has met, Theorem 1 (d)).
// A draw at t changes Delta at time t+1 by dx - dy.  Each lane keeps the
// numerators of up to CACHE clones of its slot in registers and spills any
// further clone to its own int64 row in global memory (no-return atomics,
// recorded in a touched list).  A replication that can no longer be retained
// (it would complete beyond B) is stopped and rolled back by replaying its
// draws with negated contributions.  At the end of a slot its numerators are
// added to integer buckets keyed by N*_p, which makes the
// completion-time-corrected aggregate exact and order-independent.
//
// Mismatch time: for each clone, D_j = #{s = 1..C : x_j(s) != y_j(s-1)},
// summed over retained replications (where a pair's time apart goes, clone
// by clone).  By summation by parts D_j = (C+1)|Delta_j(C)| - sum_u u e_u,
// with e_u = |Delta_j(u)| - |Delta_j(u-1)| the change at time index u, so a
// draw at t that changes |Delta_I| by e adds -(t+1) e, and a pair stopped by
// the cap adds C+1 for every clone still apart.  The events only happen
// before the meeting and go straight to the instance's output with
// device-scope atomics (a rolled-back replication's replay cancels them);
// they are counted only when a run asks for them, since most pairs disagree
// on the same few clones and those atomics then contend.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mcpd_device.h"

namespace mcpd {

#if defined(MCPD_FMT)
namespace {

constexpr uint32_t MODE_NEED_SLOT = 0;
constexpr uint32_t MODE_NEED_REP = 1;
constexpr uint32_t MODE_RUN = 2;
constexpr uint32_t MODE_DONE = 3;
constexpr uint32_t NO_TAG = 0xFFFFFFFFu;
constexpr int CACHE = 8;
constexpr uint32_t WG = WG_LANES;   // lanes per workgroup (state stride), fixed at launch

// The instance descriptors are read-only for the whole launch: reading them
// through the constant address space lets the compiler use scalar loads and
// reload them instead of keeping every field live.
using DescPtr = const __attribute__((address_space(4))) InstDesc *;

// Philox4x32-10 (Salmon et al., SC'11).  The key is wave-uniform, so its
// schedule stays on the scalar unit.
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // three-input xors (truth table 0x96) in one instruction each
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// sum_{s=k+1}^{t} min(s-k, W) for t >= k, modulo 2^64.
__device__ __forceinline__ uint64_t gsum(uint32_t t, uint32_t k, uint32_t ell, uint32_t W)
{
    if (t <= ell + 1u) {
        const uint64_t tk = (uint64_t)(t - k);
        return tk * (tk + 1) / 2;
    }
    return (uint64_t)W * (uint64_t)(W + 1u) / 2 + (uint64_t)(t - ell - 1u) * (uint64_t)W;
}

struct Lane {
    uint32_t mode, p, r, t, nret, tau, target, lim;
    int32_t mu, sgn;
    uint64_t S;
    uint32_t lc, f0, f1;
    uint32_t ctag[CACHE];
    uint64_t cval[CACHE];
};

template <int F>
struct Row {
    static constexpr int NE = fmt_entries(F);
    static constexpr bool WIDE = fmt_wide(F);
    static constexpr int WORDS = fmt_row_bytes(F) / 4;
    uint32_t w[WORDS];

    __device__ __forceinline__ void load(const uint32_t *base, uint32_t I)
    {
        const uint32_t *src = base + (size_t)I * WORDS;
        if constexpr (WORDS == 1) {
            w[0] = *src;
        } else if constexpr (WORDS == 2) {
            const uint2 v = *reinterpret_cast<const uint2 *>(src);
            w[0] = v.x; w[1] = v.y;
        } else if constexpr (WORDS == 4) {
            const uint4 v = *reinterpret_cast<const uint4 *>(src);
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
        } else {
            const uint4 v = *reinterpret_cast<const uint4 *>(src);
            const uint4 u = *reinterpret_cast<const uint4 *>(src + 4);
            w[0] = v.x; w[1] = v.y; w[2] = v.z; w[3] = v.w;
            w[4] = u.x; w[5] = u.y; w[6] = u.z; w[7] = u.w;
        }
    }
    __device__ __forceinline__ uint32_t raw(int e) const
    {
        if constexpr (WIDE) return (w[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu;
        else return (w[e >> 2] >> ((e & 3) * 8)) & 0xFFu;
    }
    // Padding entries name pool m, one past the last pool (whose counts are a
    // sentinel in the cooperative kernel's layout).
    __device__ __forceinline__ static bool valid(uint32_t v, uint32_t m) { return pool(v) != m; }
    __device__ __forceinline__ static uint32_t pool(uint32_t v) { return WIDE ? (v & 0x7FFFu) : (v & 0x7Fu); }
    __device__ __forceinline__ static uint32_t outcome(uint32_t v) { return WIDE ? (v >> 15) : (v >> 7); }
};

template <bool SL, bool TL, int F>
struct Sampler {
    const LaunchArgs &a;
    DescPtr D;
    uint32_t k0, k1;        // the key of the random numbers
    uint32_t *st;           // this workgroup's state base (LDS or global): bit words
    uint32_t *cst;          // its count words (st + words_bits * stride)
    uint32_t stride;        // state words of one index for all lanes (lane-fastest)
    const uint64_t *thr;    // tables (LDS copies or global)
    const uint32_t *alias;
    const uint32_t *rows;
    uint32_t lane;          // lane within the workgroup
    int64_t *acc;           // this lane's spill row
    uint32_t *list;         // this lane's touched list
    uint64_t *ls;           // this lane's statistics
    uint32_t *hist_lds;

    __device__ __forceinline__ uint32_t &bits(uint32_t w) const { return st[w * stride + lane]; }
    __device__ __forceinline__ uint32_t &cnt(uint32_t q) const { return cst[q * stride + lane]; }

    // Statistic slots and spill rows belong to one lane: workgroup-scope
    // atomics keep them in the L2 of the lane's XCD instead of memory.
    __device__ __forceinline__ void stat_add(int i, uint64_t v) const
    {
        __hip_atomic_fetch_add(ls + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ __forceinline__ void stat_max(int i, uint64_t v) const
    {
        __hip_atomic_fetch_max(ls + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    __device__ __forceinline__ void reset_state() const
    {
        const uint32_t nw = D->words_bits + D->words_cnt;
        for (uint32_t w = 0; w < nw; ++w) st[w * stride + lane] = 0u;
    }

    // Initial state drawn from the prior (init_mode 1): clone i starts
    // positive in both chains when word i mod 4 of the block (floor(i/4), r,
    // p, g + 2^25) is below floor(q 2^32).  A positive start adds the W terms
    // x_i(s) = 1, s = k..l, to the clone's numerator; later changes are
    // events like any other.
    __device__ __forceinline__ void init_prior(Lane &s) const
    {
        const uint32_t n = (uint32_t)D->n, nb = (n + 3u) >> 2;
        const uint32_t q = D->qthr;
        const uint64_t W = D->W;
        for (uint32_t b = 0; b < nb; ++b) {
            uint32_t w[4];
            philox10(b, s.r, s.p, D->g | (1u << 25), k0, k1, w);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t i = 4u * b + (uint32_t)e;
                if (i >= n || w[e] >= q) continue;
                bits(i >> 4) |= 3u << ((i & 15u) << 1);
                Row<F> rr;
                rr.load(rows, i);
#pragma unroll
                for (int x = 0; x < Row<F>::NE; ++x) {
                    const uint32_t v = rr.raw(x);
                    if (!Row<F>::valid(v, (uint32_t)D->m)) continue;
                    const uint32_t j = Row<F>::pool(v);
                    cnt(j >> 1) += 0x0101u << ((j & 1u) << 4);
                }
                event(s, i, s.sgn > 0 ? W : (uint64_t)0 - W);
            }
        }
    }

    // First draw count at which after_step has anything to decide: the end of
    // the window, the cap, the end of a replay, or the abort point.
    __device__ __forceinline__ void set_limit(Lane &s) const
    {
        uint32_t lim = D->ell < D->capmax ? D->ell : D->capmax;
        if (s.sgn < 0 && s.target < lim) lim = s.target;
        if (s.r >= 2u) {
            const uint64_t ab = D->B - s.S + 1u;
            if (ab < (uint64_t)lim) lim = (uint32_t)ab;
        }
        s.lim = lim;
    }

    // Mismatch-time event of clone j (sign of the replication applied).
    __device__ __forceinline__ void mismatch_event(int32_t sgn, uint32_t j, uint64_t v) const
    {
        atomicAdd(reinterpret_cast<unsigned long long *>(D->Dmis + j), (unsigned long long)(sgn > 0 ? v : (uint64_t)0 - v));
    }

    __device__ __forceinline__ void spill(Lane &s, uint32_t j, uint64_t v) const
    {
        __hip_atomic_fetch_add(reinterpret_cast<uint64_t *>(acc + j), v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        if (j != s.f0 && j != s.f1) {
            if (s.lc < a.list_cap) list[s.lc] = j;
            s.lc += 1;
            s.f1 = s.f0;
            s.f0 = j;
        }
    }

    // Add v to clone j's numerator.  A clone holds a register entry for the
    // rest of the slot once it has one; entries are never evicted, so a
    // clone is either cached or spilled, never both.
    __device__ __forceinline__ void event(Lane &s, uint32_t j, uint64_t v) const
    {
        bool hit = false;
#pragma unroll
        for (int e = 0; e < CACHE; ++e) {
            const bool m = s.ctag[e] == j;
            s.cval[e] += m ? v : 0ull;
            hit |= m;
        }
        if (!hit) {
            bool placed = false;
#pragma unroll
            for (int e = 0; e < CACHE; ++e) {
                if (!placed && s.ctag[e] == NO_TAG) {
                    s.ctag[e] = j;
                    s.cval[e] = v;
                    placed = true;
                }
            }
            if (!placed) spill(s, j, v);
        }
    }

    // Low 53-b bits of U of draw t (block (t, r, p, g | 2^24)).
    __device__ __forceinline__ uint64_t low_bits(const Lane &s, uint32_t t) const
    {
        uint32_t o[4];
        philox10(t, s.r, s.p, D->g | (1u << 24), k0, k1, o);
        const uint64_t v = ((uint64_t)o[0] << 32) | (uint64_t)o[1];
        return v >> (11u + a.ubits);
    }

    // 1{U53 <= T}, U53 = (hw >> (32-b)) << (53-b) | low; both high parts
    // have b bits, so they compare as 32-bit words.
    __device__ __forceinline__ uint32_t decide(const Lane &s, uint32_t t, uint32_t hw, uint64_t T,
                                               bool &have_lo, uint64_t &lo) const
    {
        const uint32_t b = a.ubits;
        const uint32_t hb = hw >> (32u - b);
        const uint32_t th = (uint32_t)(T >> (53u - b));
        if (hb != th) return hb < th ? 1u : 0u;
        if (!have_lo) { lo = low_bits(s, t); have_lo = true; }
        return lo <= (T & ((1ull << (53u - b)) - 1ull)) ? 1u : 0u;
    }

    // Site of a draw from its site word: alias column from the top bits,
    // coin from the low bits (one LDS read, no search).
    __device__ __forceinline__ uint32_t site(uint32_t sw) const
    {
        const uint32_t cb = 32u - D->abits;
        const uint32_t col = sw >> cb;
        const uint32_t aw = alias[col];
        const uint32_t kmask = (1u << cb) - 1u;
        return (sw & kmask) < (aw & kmask) ? col : (aw >> cb);
    }

    // State words a draw at clone I reads: its bit word and one count word
    // per pool, issued back to back.
    struct Loads {
        uint32_t bw;
        uint32_t cw[Row<F>::NE];
    };
    __device__ __forceinline__ Loads issue(uint32_t I, const Row<F> &rc) const
    {
        using R = Row<F>;
        Loads ld;
        ld.bw = bits(I >> 4);
#pragma unroll
        for (int e = 0; e < R::NE; ++e) {
            const uint32_t v = rc.raw(e);
            ld.cw[e] = cnt((R::valid(v, (uint32_t)D->m) ? R::pool(v) : 0u) >> 1);
        }
        return ld;
    }

    // The rest of draw t at clone I with U word hw: both chains' free-pool
    // patterns, thresholds, decisions, state update and estimator events.
    __device__ __forceinline__ void finish(Lane &s, uint32_t I, const Row<F> &rc, const Loads &ld,
                                           uint32_t hw) const
    {
        using R = Row<F>;
        const uint32_t t = s.t;
        const uint32_t bw_idx = I >> 4;
        const uint32_t bw = ld.bw;
        const uint32_t sh = (I & 15u) << 1;
        const uint32_t xi = (bw >> sh) & 1u;
        const uint32_t yi = (bw >> (sh + 1u)) & 1u;
        const bool updY = (s.tau == 0u) && (t > 0u);

        // free-pool patterns of both chains from the same count words
        uint32_t patX = 0, lenX = 0, patY = 0, lenY = 0;
#pragma unroll
        for (int e = 0; e < R::NE; ++e) {
            const uint32_t v = rc.raw(e);
            const bool ok = R::valid(v, (uint32_t)D->m);
            const uint32_t o = R::outcome(v);
            const uint32_t c = ld.cw[e] >> ((R::pool(v) & 1u) << 4);
            const bool fx = ok && (c & 0xFFu) == xi;
            const bool fy = ok && ((c >> 8) & 0xFFu) == yi;
            patX = fx ? ((patX << 1) | o) : patX;
            lenX += fx ? 1u : 0u;
            patY = fy ? ((patY << 1) | o) : patY;
            lenY += fy ? 1u : 0u;
        }
        bool have_lo = false;
        uint64_t lo = 0;
        const uint32_t ix = (1u << lenX) - 1u + patX;
        const uint32_t xn = decide(s, t, hw, thr[ix], have_lo, lo);
        uint32_t yn = yi;
        if (updY) {
            // the same pattern gives the same threshold, hence the same value
            const uint32_t iy = (1u << lenY) - 1u + patY;
            yn = (iy == ix) ? xn : decide(s, t, hw, thr[iy], have_lo, lo);
        }
        const int dx = (int)xn - (int)xi;
        const int dy = (int)yn - (int)yi;
        if (dx | dy) {
            bits(bw_idx) = bw ^ ((uint32_t)(dx != 0) << sh) ^ ((uint32_t)(dy != 0) << (sh + 1u));
#pragma unroll
            for (int e = 0; e < R::NE; ++e) {
                const uint32_t v = rc.raw(e);
                if (!R::valid(v, (uint32_t)D->m)) continue;
                const uint32_t j = R::pool(v);
                const uint32_t cs = (j & 1u) << 4;
                const uint32_t delta = ((uint32_t)dx << cs) + ((uint32_t)dy << (cs + 8u));
                if constexpr (SL) atomicAdd(&cnt(j >> 1), delta);   // LDS, no return
                else cnt(j >> 1) += delta;
            }
            if (s.tau == 0u) {
                const int dmu = (int)(xn != yn) - (int)(xi != yi);
                s.mu += dmu;
                if (a.mismatch && dmu != 0) mismatch_event(s.sgn, I, (uint64_t)(int64_t)(-dmu) * (uint64_t)(t + 1u));
            }
            // estimator events at time te = t + 1
            uint64_t val = 0;
            const uint32_t te = t + 1u;
            if (dx != 0 && te <= D->ell) {
                const uint32_t from = te > D->k ? te : D->k;
                val += (uint64_t)(int64_t)dx * (uint64_t)(D->ell - from + 1u);
            }
            if (updY && t >= D->k + 1u && dx != dy)
                val -= (uint64_t)(int64_t)(dx - dy) * gsum(t, D->k, D->ell, D->W);
            if (val != 0) event(s, I, s.sgn > 0 ? val : (uint64_t)0 - val);
        }
        if (s.tau == 0u && s.mu == 0) s.tau = t + 1u;
        s.t = t + 1u;
    }

    // Boundary term G(C) Delta_j(C) of a pair stopped by the cap.
    __device__ __forceinline__ void truncation(Lane &s) const
    {
        const uint32_t C = s.t;
        if (C < D->k + 1u) return;
        const uint64_t G = gsum(C, D->k, D->ell, D->W);
        for (uint32_t w = 0; w < D->words_bits; ++w) {
            const uint32_t word = bits(w);
            uint32_t mis = (word ^ (word >> 1)) & 0x55555555u;
            while (mis) {
                const uint32_t b = __builtin_ctz(mis);
                mis &= mis - 1u;
                const uint32_t j = w * 16u + (b >> 1);
                const uint64_t v = ((word >> b) & 1u) ? G : (uint64_t)0 - G;
                event(s, j, s.sgn > 0 ? v : (uint64_t)0 - v);
                if (a.mismatch) mismatch_event(s.sgn, j, (uint64_t)C + 1u);
            }
        }
    }

    // Add a slot's numerator to its N* bucket: S1 += V and the square V^2 =
    // h 2^64 + l as three 64-bit limbs, S2 += (l mod 2^32, l >> 32, h).  All
    // no-return atomics; the host rebuilds the 128-bit sums (the limb sums
    // stay exact while there are fewer than 2^32 slots and the high words
    // sum below 2^64).
    __device__ __forceinline__ void emit(uint32_t nstar, uint32_t j, int64_t v) const
    {
        if (nstar > D->nbuckets) {
            atomicOr(&a.ctrl[1], (uint32_t)ERR_BUCKETS);
            return;
        }
        const size_t idx = (size_t)(nstar - 1u) * (size_t)D->n + j;
        atomicAdd(reinterpret_cast<unsigned long long *>(D->S1 + idx), (unsigned long long)v);
        const uint64_t u = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        const uint64_t lo = u * u;
        const uint64_t hi = __umul64hi(u, u);
        unsigned long long *q = reinterpret_cast<unsigned long long *>(D->S2 + 3 * idx);
        atomicAdd(q, (unsigned long long)(lo & 0xFFFFFFFFull));
        if (lo >> 32) atomicAdd(q + 1, (unsigned long long)(lo >> 32));
        if (hi) atomicAdd(q + 2, (unsigned long long)hi);
    }

    // Take (and clear) the spilled numerators of up to 8 clones at once, so
    // that their round trips overlap, then emit the nonzero ones.
    __device__ __forceinline__ void take8(uint32_t nstar, const uint32_t j[8], uint32_t cnt) const
    {
        int64_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[q] = (uint32_t)q < cnt ? (int64_t)__hip_atomic_exchange(reinterpret_cast<uint64_t *>(acc + j[q]),
                                                                      (uint64_t)0, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_WORKGROUP)
                                     : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (v[q] != 0) emit(nstar, j[q], v[q]);
    }

    __device__ __forceinline__ void flush_slot(Lane &s) const
    {
        const uint32_t nstar = s.nret;
#pragma unroll
        for (int e = 0; e < CACHE; ++e) {
            if (s.ctag[e] != NO_TAG && s.cval[e] != 0) emit(nstar, s.ctag[e], (int64_t)s.cval[e]);
            s.ctag[e] = NO_TAG;
            s.cval[e] = 0;
        }
        if (s.lc > 0) {
            uint32_t j[8];
            if (s.lc <= a.list_cap) {
                for (uint32_t e0 = 0; e0 < s.lc; e0 += 8) {
                    const uint32_t cnt = s.lc - e0 < 8u ? s.lc - e0 : 8u;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        j[q] = (uint32_t)q < cnt ? __hip_atomic_load(list + e0 + q, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_WORKGROUP)
                                                 : 0u;
                    take8(nstar, j, cnt);
                }
            } else {
                stat_add(ST_LIST_OVERFLOWS, 1);
                const uint32_t n = (uint32_t)D->n;
                for (uint32_t j0 = 0; j0 < n; j0 += 8) {
                    const uint32_t cnt = n - j0 < 8u ? n - j0 : 8u;
#pragma unroll
                    for (int q = 0; q < 8; ++q) j[q] = j0 + (uint32_t)q;
                    take8(nstar, j, cnt);
                }
            }
        }
        if (D->slot_nstar) D->slot_nstar[s.p - D->p0] = nstar;
        if (D->slot_units) D->slot_units[s.p - D->p0] = s.S;
        stat_max(ST_NSTAR_MAX, nstar);
        s.mode = MODE_NEED_SLOT;
    }

    __device__ __forceinline__ void begin_rollback(Lane &s, uint32_t draws) const
    {
        stat_add(ST_REPS_ABORTED, 1);
        stat_add(ST_ROLLBACK_UNITS, draws);
        stat_add(ST_PROGRESS, 2ull * draws);
        s.target = draws;
        s.sgn = -1;
        s.mode = MODE_NEED_REP;
    }

    // Bookkeeping once the draw count reaches the lane's limit: completion,
    // retention, abort, end of replay.
    __device__ __forceinline__ void after_step(Lane &s) const
    {
        const uint32_t d = s.t;
        const bool capped = (s.tau == 0u) && (d >= D->capmax);
        const bool ended = capped || (s.tau != 0u && d >= D->ell);
        if (s.sgn < 0) {
            if (d == s.target) {
                if (capped) truncation(s);
                flush_slot(s);
            }
            return;
        }
        if (ended) {
            if (capped) truncation(s);
            const uint64_t C = d;
            const bool retained = (s.r == 1u) || (s.S + C <= D->B);
            if (!retained) { begin_rollback(s, d); return; }
            s.S += C;
            s.nret += 1u;
            stat_add(ST_RETAINED_UNITS, C);
            stat_add(ST_PROGRESS, C);
            stat_add(ST_REPS_RETAINED, 1);
            if (capped) {
                stat_add(ST_CAP_HITS, 1);
                stat_add(ST_SINGLE_SITE, 1 + 2 * (C - 1));
            } else {
                const uint64_t mt = s.tau < d ? s.tau : d;
                stat_add(ST_SINGLE_SITE, 1 + 2 * (mt - 1) + (C - mt));
                stat_add(ST_TAU_SUM, s.tau);
                stat_max(ST_TAU_MAX, s.tau);
                uint32_t bin = s.tau / D->hist_width;
                if (bin >= a.hist_bins) bin = a.hist_bins - 1u;
                atomicAdd(hist_lds + bin, 1u);
            }
            if (s.r == 1u && C > D->B) stat_add(ST_ZERO_COMPLETION, 1);
            if (!a.refill || s.S >= D->B || s.S + D->cmin > D->B) flush_slot(s);
            else s.mode = MODE_NEED_REP;
            return;
        }
        if (s.r >= 2u && (uint64_t)d > D->B - s.S) begin_rollback(s, d);
    }
};

// Copy n32 dwords from global memory into LDS, all threads of the block.
__device__ __forceinline__ void copy_to_lds(uint32_t *dst, const void *src, uint32_t n32)
{
    const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
    for (uint32_t i = threadIdx.x; i < n32; i += blockDim.x) dst[i] = s[i];
}

// One workgroup's share of one instance: place the tables (and state) in
// LDS, let every lane take slots until the instance has none left, then add
// the lanes' statistics and the histogram to the instance's totals.
// A slot of instance D for this workgroup: from its XCD's range first (one
// atomic add), then, checking before adding, from the other ranges in turn.
// Returns P when every range is used up.  Counters only grow, so every
// workgroup eventually sees them all used up.
__device__ __forceinline__ uint32_t take_slot(DescPtr D)
{
    const uint32_t home = blockIdx.x % XCDS, q = D->slot_q, P = D->P;
    for (uint32_t i = 0; i < XCDS; ++i) {
        const uint32_t x = (home + i) % XCDS;
        const uint32_t lo = x * q;
        if (lo >= P) continue;
        const uint32_t n = min(q, P - lo);
        uint32_t *c = D->next_slot + x * SLOT_CTR_STRIDE;
        if (i != 0 && __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) continue;
        const uint32_t k = atomicAdd(c, 1u);
        if (k < n) return lo + k;
    }
    return P;
}

// Whether instance d has a slot left in any range.
__device__ __forceinline__ bool slots_left(const InstDesc *d)
{
    for (uint32_t x = 0; x < XCDS; ++x) {
        const uint32_t lo = x * d->slot_q;
        if (lo >= d->P) break;
        const uint32_t n = min(d->slot_q, d->P - lo);
        if (__hip_atomic_load(d->next_slot + x * SLOT_CTR_STRIDE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n)
            return true;
    }
    return false;
}

template <bool SL, bool TL, int F>
__device__ __forceinline__ void run_item(const LaunchArgs &a, DescPtr D, uint32_t *smem, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t L = WG;
    const uint32_t lane = threadIdx.x;
    uint32_t *hist_lds = smem + D->lds_hist;
    uint32_t *tab = smem + D->lds_tab;
    for (uint32_t b = lane; b < a.hist_bins; b += L) hist_lds[b] = 0u;
    if (TL) {
        copy_to_lds(tab + D->tab_off_thr / 4, D->thr, D->thr_len * 2u);
        copy_to_lds(tab + D->tab_off_alias / 4, D->alias, 1u << D->abits);
        copy_to_lds(tab + D->tab_off_rows / 4, D->rows, (uint32_t)D->n * D->row_bytes / 4u);
    }
    const size_t gl = (size_t)blockIdx.x * L + lane;
    uint64_t *ls = a.lane_stats + gl * ST_COUNT;
#pragma unroll
    for (int i = 0; i < ST_COUNT; ++i) ls[i] = 0;
    __syncthreads();

    // State in LDS is laid out for the instance's active lanes (a narrow
    // workgroup keeps large states in LDS); in global memory for all 256.
    const uint32_t stride = SL ? D->lanes : WG;
    uint32_t *st = SL ? smem : a.gstate + (size_t)blockIdx.x * a.gwords * WG;
    Sampler<SL, TL, F> S{a,
                         D,
                         k0,
                         k1,
                         st,
                         st + (size_t)D->words_bits * stride,
                         stride,
                         TL ? reinterpret_cast<const uint64_t *>(tab + D->tab_off_thr / 4) : D->thr,
                         TL ? tab + D->tab_off_alias / 4 : D->alias,
                         TL ? tab + D->tab_off_rows / 4 : D->rows,
                         lane,
                         a.acc + gl * (size_t)a.acc_stride,
                         a.lists + gl * (size_t)a.list_cap,
                         ls,
                         hist_lds};
    Lane s;
    s.mode = lane < D->lanes ? MODE_NEED_SLOT : MODE_DONE;
    s.p = s.r = s.t = s.nret = s.tau = s.target = s.lim = 0;
    s.mu = 0;
    s.sgn = 1;
    s.S = 0;
    s.lc = 0;
    s.f0 = s.f1 = NO_TAG;
#pragma unroll
    for (int e = 0; e < CACHE; ++e) { s.ctag[e] = NO_TAG; s.cval[e] = 0; }
    const uint32_t P = D->P;
    const uint32_t g = D->g;

    // Pipeline registers: the random block of the current pair of draws
    // (t, t+1) and the site and row of draw t, fetched one draw ahead.
    uint32_t w[4] = {0, 0, 0, 0};
    uint32_t curI = 0;
    Row<F> cur;
#pragma unroll
    for (int i = 0; i < Row<F>::WORDS; ++i) cur.w[i] = 0;

    for (;;) {
        if (s.mode != MODE_RUN) {
            if (s.mode == MODE_NEED_SLOT) {
                const uint32_t p = take_slot(D);
                if (p >= P) {
                    s.mode = MODE_DONE;
                } else {
                    s.p = p + D->p0;   // global slot index (the random-number counter)
                    s.r = 0;
                    s.S = 0;
                    s.nret = 0;
                    s.lc = 0;
                    s.f0 = s.f1 = NO_TAG;
                    s.sgn = 1;
                    s.mode = MODE_NEED_REP;
                }
            }
            if (s.mode == MODE_NEED_REP) {
                if (s.sgn > 0) {
                    s.r += 1u;
                    S.stat_add(ST_REPS_STARTED, 1);
                }
                S.reset_state();
                if (a.init_mode) S.init_prior(s);
                s.t = 0;
                s.tau = 0;
                s.mu = 0;
                S.set_limit(s);
                philox10(0u, s.r, s.p, g, k0, k1, w);
                curI = S.site(w[0]);
                cur.load(S.rows, curI);
                s.mode = MODE_RUN;
            }
        }
        if (__all(s.mode == MODE_DONE)) break;
        if (s.mode == MODE_RUN) {
            // draw t (even): its state reads go out first, then the next
            // random block and draw t+1's site and row while they are in flight
            const typename Sampler<SL, TL, F>::Loads l0 = S.issue(curI, cur);
            uint32_t nx[4];
            philox10((s.t >> 1) + 1u, s.r, s.p, g, k0, k1, nx);
            const uint32_t I1 = S.site(w[2]);
            Row<F> r1;
            r1.load(S.rows, I1);
            S.finish(s, curI, cur, l0, w[1]);
            if (s.t >= s.lim) S.after_step(s);
            if (s.mode == MODE_RUN) {
                // draw t+1 (odd), with draw t+2's site and row fetched behind it
                const typename Sampler<SL, TL, F>::Loads l1 = S.issue(I1, r1);
                const uint32_t I2 = S.site(nx[0]);
                Row<F> r2;
                r2.load(S.rows, I2);
                S.finish(s, I1, r1, l1, w[3]);
                if (s.t >= s.lim) S.after_step(s);
                curI = I2;
                cur = r2;
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = nx[i];
            }
        }
    }

    // Statistics: each lane reads back its own slots, wave reduction, then
    // one atomic per wave.
    uint64_t *stats = D->stats;
#pragma unroll
    for (int i = 0; i < ST_COUNT; ++i) {
        uint64_t v = __hip_atomic_load(ls + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const bool is_max = (i == ST_TAU_MAX || i == ST_NSTAR_MAX);
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(v, off);
            v = is_max ? (o > v ? o : v) : v + o;
        }
        if ((lane & 63u) == 0u && v != 0) {
            if (is_max) atomicMax(reinterpret_cast<unsigned long long *>(stats + i), (unsigned long long)v);
            else atomicAdd(reinterpret_cast<unsigned long long *>(stats + i), (unsigned long long)v);
        }
    }
    __syncthreads();
    uint64_t *hist = D->hist;
    for (uint32_t b = lane; b < a.hist_bins; b += L)
        if (hist_lds[b]) atomicAdd(reinterpret_cast<unsigned long long *>(hist + b), (unsigned long long)hist_lds[b]);
    __syncthreads();
}

// The next ticket of this workgroup: tickets come in one queue per XCD
// (instances spread over the queues by work, so that the workgroups of one
// XCD share few instances' tables in their L2); a workgroup takes from the
// queue of its own XCD, then from the others in turn.  Returns nticket when
// every queue is empty.  Queue counters only grow, so every workgroup
// eventually sees them all empty.
__device__ __forceinline__ uint32_t take_ticket(const LaunchArgs &a)
{
    const uint32_t home = blockIdx.x % XCDS;
    for (uint32_t q = 0; q < XCDS; ++q) {
        const uint32_t x = (home + q) % XCDS;
        const uint32_t n = a.qoff[x + 1] - a.qoff[x];
        if (n == 0) continue;
        if (__hip_atomic_load(&a.ctrl[2 + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) continue;
        const uint32_t it = atomicAdd(&a.ctrl[2 + x], 1u);
        if (it < n) return a.qoff[x] + it;
    }
    return a.nticket;
}

// Persistent kernel over a batch: a workgroup takes tickets until the queues
// are empty.  Every workgroup leaves when every ticket queue is used up, and
// every lane leaves an instance when every range of its slots is used up, so
// the grid always drains.
template <int F>
__global__ void __launch_bounds__(256) sampler_kernel(LaunchArgs a)
{
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t sh_item, sh_skip;
    const uint64_t seed = *(const __attribute__((address_space(4))) uint64_t *)a.seed;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    DescPtr descs = (DescPtr)a.inst;
    const __attribute__((address_space(4))) uint32_t *tickets =
        (const __attribute__((address_space(4))) uint32_t *)a.tickets;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t it = take_ticket(a);
            uint32_t skip = 1;
            if (it < a.nticket) {
                skip = !slots_left(a.inst + a.tickets[it]);
            }
            sh_item = it;
            sh_skip = skip;
        }
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(sh_item);
        const uint32_t skip = __builtin_amdgcn_readfirstlane(sh_skip);
        __syncthreads();
        if (item >= a.nticket) break;
        if (skip) continue;
        DescPtr D = descs + tickets[item];
        switch (D->place) {
        case PLACE_STATE_LDS | PLACE_TABLES_LDS: run_item<true, true, F>(a, D, smem, k0, k1); break;
        case PLACE_STATE_LDS: run_item<true, false, F>(a, D, smem, k0, k1); break;
        case PLACE_TABLES_LDS: run_item<false, true, F>(a, D, smem, k0, k1); break;
        default: run_item<false, false, F>(a, D, smem, k0, k1); break;
        }
    }
}

// ------------------------------------------------------------ cooperative
// A group of GL lanes (8, 16, 32 or 64: a wavefront holds 64 / GL groups)
// runs one slot at a time.  Each step the group's lanes draw the next GL
// updates of the pair speculatively against the current state; a ballot
// finds the first lane whose update changes either chain.  Every lane before
// it changed nothing, so their updates were made on the exact state and
// stand; the first changing lane's update stands too and is applied; the
// lanes after it are dropped and redrawn in the next step.  The committed
// draws and decisions are exactly those of the one-lane sampler.  A slot's
// chain state (0.5 KB for 1298 clones and 97 pools) is small enough that
// every group keeps its own in LDS, and a pair that takes very long to meet
// advances many draws per step.  Smaller groups waste fewer speculative
// draws when changes are frequent; larger ones go further when they are rare.

struct GroupSlot {
    uint32_t mode, p, r, t, nret, tau, target, lim, stop, lc, cptr;
    int32_t mu, sgn;
    uint64_t S;
};

template <bool TL, int F>
struct Coop {
    const LaunchArgs &a;
    DescPtr D;
    uint32_t k0, k1;
    uint32_t *st;           // this group's bit words (LDS)
    uint32_t *cst;          // its count words
    static constexpr bool WPP = coop_word_per_pool(F);   // one count word per pool
    static constexpr bool PT = coop_pattern_table(F);    // threshold index from the pattern table
    const uint8_t *pat8;    // the pattern table (LDS offset 0)
    const uint64_t *thr;
    const uint32_t *alias;
    const uint32_t *rows;
    uint32_t gl;            // lane within the group
    uint32_t gsz;           // lanes per group
    uint32_t leader;        // the group's first lane in the wavefront
    uint64_t gmask;         // the group's lanes in a wavefront ballot
    int64_t *acc;           // this group's numerator row
    uint32_t *list;         // its touched list
    uint32_t *hist_lds;
    uint32_t *lds;          // the workgroup's dynamic LDS
    uint32_t gid;           // the group whose slot this is (index in the workgroup)
    // The slot's numerator cache: one (clone, numerator) entry per lane of
    // the group, no clone held twice.  The events of a slot add up here; an
    // entry moves to the numerator row only when a new clone needs its lane
    // (lanes taken in turn), so most slots never touch the row.  Entries
    // are empty (NO_TAG) between slots, which a merged group relies on.
    mutable uint32_t ckey;
    mutable uint64_t cval;

    // Point at the state, numerator row and touched list of group `g` of
    // this workgroup (its statistics follow from gid).
    __device__ __forceinline__ void point(uint32_t *smem, uint32_t g)
    {
        gid = g;
        st = smem + D->lds_state + g * D->wave_words;
        cst = st + D->words_bits;
        const size_t gi = (size_t)blockIdx.x * a.groups_per_wg + g;
        acc = a.acc + gi * (size_t)a.acc_stride;
        list = a.lists + gi * (size_t)a.list_cap;
    }

    // The group's statistics, written by its leader: in LDS when the layout
    // has room for them (lds_stats != 0), else in global memory.  Both
    // pointers keep their address spaces, so neither access becomes a flat
    // one, and both are formed where they are used (no live registers).
    __device__ __forceinline__ __attribute__((address_space(3))) uint64_t *stats_lds() const
    {
        return (__attribute__((address_space(3))) uint64_t *)(reinterpret_cast<uint64_t *>(lds + D->lds_stats) +
                                                              (size_t)gid * ST_COUNT);
    }
    __device__ __forceinline__ __attribute__((address_space(1))) uint64_t *stats_global() const
    {
        const size_t gi = (size_t)blockIdx.x * a.groups_per_wg + gid;
        return (__attribute__((address_space(1))) uint64_t *)(a.lane_stats + gi * ST_COUNT);
    }

    // Counter i of the group's statistics (LDS or global; the choice is the
    // instance's, so the branch is uniform).
    __device__ __forceinline__ uint64_t stat_get(uint32_t i) const
    {
        return D->lds_stats ? __hip_atomic_load(stats_lds() + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                            : __hip_atomic_load(stats_global() + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ __forceinline__ void stat_clear(uint32_t i) const
    {
        if (D->lds_stats) stats_lds()[i] = 0;
        else stats_global()[i] = 0;
    }

    // The group's statistics into the instance's, once, when it runs out of
    // slots (one atomic per counter).
    __device__ __forceinline__ void flush_stats() const
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        for (uint32_t i = gl; i < (uint32_t)ST_COUNT; i += gsz) {
            const uint64_t v = stat_get(i);
            if (v) {
                if (i == ST_TAU_MAX || i == ST_NSTAR_MAX)
                    atomicMax(reinterpret_cast<unsigned long long *>(D->stats + i), (unsigned long long)v);
                else
                    atomicAdd(reinterpret_cast<unsigned long long *>(D->stats + i), (unsigned long long)v);
            }
        }
    }

    __device__ __forceinline__ void stat_add(int i, uint64_t v) const
    {
        if (gl != 0) return;
        if (D->lds_stats) __hip_atomic_fetch_add(stats_lds() + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else __hip_atomic_fetch_add(stats_global() + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ __forceinline__ void stat_max(int i, uint64_t v) const
    {
        if (gl != 0) return;
        if (D->lds_stats) __hip_atomic_fetch_max(stats_lds() + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else __hip_atomic_fetch_max(stats_global() + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    __device__ __forceinline__ uint32_t site(uint32_t sw) const
    {
        const uint32_t cb = 32u - D->abits;
        const uint32_t col = sw >> cb;
        const uint32_t aw = alias[col];
        const uint32_t kmask = (1u << cb) - 1u;
        return (sw & kmask) < (aw & kmask) ? col : (aw >> cb);
    }

    __device__ __forceinline__ uint64_t low_bits(const GroupSlot &s, uint32_t t) const
    {
        uint32_t o[4];
        philox10(t, s.r, s.p, D->g | (1u << 24), k0, k1, o);
        const uint64_t v = ((uint64_t)o[0] << 32) | (uint64_t)o[1];
        return v >> (11u + a.ubits);
    }

    __device__ __forceinline__ uint32_t decide(const GroupSlot &s, uint32_t t, uint32_t hw, uint64_t T,
                                               bool &have_lo, uint64_t &lo) const
    {
        const uint32_t b = a.ubits;
        const uint32_t hb = hw >> (32u - b);
        const uint32_t th = (uint32_t)(T >> (53u - b));
        if (hb != th) return hb < th ? 1u : 0u;
        if (!have_lo) { lo = low_bits(s, t); have_lo = true; }
        return lo <= (T & ((1ull << (53u - b)) - 1ull)) ? 1u : 0u;
    }

    __device__ __forceinline__ void lds_fence() const
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }

    // All-negative state.  The counts of pool m (one past the last pool) are
    // a sentinel of all ones: padding entries of a row read it and never find
    // a free pool, so the speculative draws need no validity test.
    __device__ __forceinline__ void reset_state() const
    {
        const uint32_t m = D->m;
        const uint32_t nw = D->words_bits + (WPP ? m : (m >> 1)) + 1u;
        for (uint32_t w = gl; w < nw; w += gsz) st[w] = 0u;
        if (gl == 0) {
            if (WPP) cst[m] = 0xFFFFFFFFu;
            else cst[m >> 1] = (m & 1u) ? 0xFFFF0000u : 0xFFFFFFFFu;
        }
        lds_fence();
    }

    // Add (dx, dy) to the X and Y counts of pool j (two's complement, so a
    // decrement of a positive count borrows nothing from the other count).
    __device__ __forceinline__ void count_add(uint32_t j, int dx, int dy) const
    {
        if (WPP)
            __hip_atomic_fetch_add(cst + j, (uint32_t)dx + ((uint32_t)dy << 16), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_fetch_add(cst + (j >> 1), ((uint32_t)dx + ((uint32_t)dy << 8)) << ((j & 1u) << 4),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    // Mismatch-time event of clone j (sign of the replication applied).
    __device__ __forceinline__ void mismatch_event(int32_t sgn, uint32_t j, uint64_t v) const
    {
        atomicAdd(reinterpret_cast<unsigned long long *>(D->Dmis + j), (unsigned long long)(sgn > 0 ? v : (uint64_t)0 - v));
    }

    __device__ __forceinline__ void add(uint32_t j, uint64_t v) const
    {
        __hip_atomic_fetch_add(reinterpret_cast<uint64_t *>(acc + j), v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }

    // Initial state drawn from the prior (init_mode 1), the group's lanes
    // over blocks of 4 clones: clone i starts positive in both chains when
    // word i mod 4 of the block (floor(i/4), r, p, g + 2^25) is below
    // floor(q 2^32); its numerator gets the W terms x_i(s) = 1, s = k..l, and
    // it joins the touched list (ballot-compacted).
    __device__ __forceinline__ void init_prior(GroupSlot &s) const
    {
        using R = Row<F>;
        const uint32_t n = (uint32_t)D->n, nb = (n + 3u) >> 2;
        for (uint32_t b0 = 0; b0 < nb; b0 += gsz) {
            const uint32_t b = b0 + gl;
            uint32_t pm = 0;   // which of the block's 4 clones start positive
            if (b < nb) {
                uint32_t w[4];
                philox10(b, s.r, s.p, D->g | (1u << 25), k0, k1, w);
                const uint32_t q = D->qthr;
#pragma unroll
                for (int e = 0; e < 4; ++e) pm |= (uint32_t)(w[e] < q && 4u * b + (uint32_t)e < n) << e;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t i = 4u * b + (uint32_t)e;
                const bool pos = (pm >> e) & 1u;
                const uint64_t m = (__ballot(pos) & gmask) >> leader;
                if (pos) {
                    __hip_atomic_fetch_or(st + (i >> 4), 3u << ((i & 15u) << 1), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
                    R rr;
                    rr.load(rows, i);
#pragma unroll
                    for (int x = 0; x < R::NE; ++x) {
                        const uint32_t v = rr.raw(x);
                        if (!R::valid(v, (uint32_t)D->m)) continue;
                        const uint32_t j = R::pool(v);
                        count_add(j, 1, 1);
                    }
                    const uint64_t W = D->W;
                    add(i, s.sgn > 0 ? W : (uint64_t)0 - W);
                    const uint32_t at = s.lc + (uint32_t)__builtin_popcountll(m & ((1ull << gl) - 1ull));
                    if (at < a.list_cap)
                        __hip_atomic_store(list + at, i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                s.lc += (uint32_t)__builtin_popcountll(m);
            }
        }
        lds_fence();
    }

    // Event v (signed) of clone j, told to every lane of the group: added to
    // the lane that holds j, else to the lane whose turn it is, whose old
    // entry (if it holds anything) goes to the row and the touched list.
    __device__ __forceinline__ void record(uint32_t j, uint64_t v, GroupSlot &s) const
    {
        if ((__ballot(ckey == j) & gmask) != 0) {
            if (ckey == j) cval += v;
            return;
        }
        const bool mine = gl == s.cptr;
        s.cptr = (s.cptr + 1u) & (gsz - 1u);
        const bool out = mine && ckey != NO_TAG && cval != 0;
        if (out) {
            add(ckey, cval);
            if (s.lc < a.list_cap)
                __hip_atomic_store(list + s.lc, ckey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if ((__ballot(out) & gmask) != 0) s.lc += 1u;
        if (mine) {
            ckey = j;
            cval = v;
        }
    }

    __device__ __forceinline__ void emit(uint32_t nstar, uint32_t j, int64_t v) const
    {
        if (nstar > D->nbuckets) {
            atomicOr(&a.ctrl[1], (uint32_t)ERR_BUCKETS);
            return;
        }
        const size_t idx = (size_t)(nstar - 1u) * (size_t)D->n + j;
        atomicAdd(reinterpret_cast<unsigned long long *>(D->S1 + idx), (unsigned long long)v);
        const uint64_t u = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        const uint64_t lo = u * u;
        const uint64_t hi = __umul64hi(u, u);
        unsigned long long *q = reinterpret_cast<unsigned long long *>(D->S2 + 3 * idx);
        atomicAdd(q, (unsigned long long)(lo & 0xFFFFFFFFull));
        if (lo >> 32) atomicAdd(q + 1, (unsigned long long)(lo >> 32));
        if (hi) atomicAdd(q + 2, (unsigned long long)hi);
    }

    // Boundary term G(C) Delta_j(C) of a pair stopped by the cap, the group's
    // lanes over the bit words; the touched list is given up (the flush scans
    // the row).
    __device__ void truncation(GroupSlot &s) const
    {
        const uint32_t C = s.t;
        if (C < D->k + 1u) return;
        const uint64_t G = gsum(C, D->k, D->ell, D->W);
        for (uint32_t w = gl; w < D->words_bits; w += gsz) {
            const uint32_t word = st[w];
            uint32_t mis = (word ^ (word >> 1)) & 0x55555555u;
            while (mis) {
                const uint32_t b = __builtin_ctz(mis);
                mis &= mis - 1u;
                const uint64_t v = ((word >> b) & 1u) ? G : (uint64_t)0 - G;
                add(w * 16u + (b >> 1), s.sgn > 0 ? v : (uint64_t)0 - v);
                if (a.mismatch) mismatch_event(s.sgn, w * 16u + (b >> 1), (uint64_t)C + 1u);
            }
        }
        s.lc = a.list_cap + 1u;
    }

    __device__ void flush_slot(GroupSlot &s) const
    {
        const uint32_t nstar = s.nret;
        const bool held = ckey != NO_TAG && cval != 0;
        if (s.lc == 0u) {
            // nothing went to the row: the cache holds the slot's numerators
            if (held) emit(nstar, ckey, (int64_t)cval);
            ckey = NO_TAG;
            cval = 0;
            finish_slot(s, nstar);
            return;
        }
        // the row holds part of them: the entries join it, then the row is flushed
        if (held) add(ckey, cval);
        const uint64_t hm = (__ballot(held) & gmask) >> leader;
        const uint32_t at = s.lc + (uint32_t)__builtin_popcountll(hm & ((1ull << gl) - 1ull));
        if (held && at < a.list_cap)
            __hip_atomic_store(list + at, ckey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        s.lc += (uint32_t)__builtin_popcountll(hm);
        ckey = NO_TAG;
        cval = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (s.lc <= a.list_cap) {
            for (uint32_t e = gl; e < s.lc; e += gsz) {
                const uint32_t j = __hip_atomic_load(list + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                const int64_t v = (int64_t)__hip_atomic_exchange(reinterpret_cast<uint64_t *>(acc + j), (uint64_t)0,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (v != 0) emit(nstar, j, v);
            }
        } else {
            stat_add(ST_LIST_OVERFLOWS, 1);
            for (uint32_t j = gl; j < (uint32_t)D->n; j += gsz) {
                const int64_t v = (int64_t)__hip_atomic_exchange(reinterpret_cast<uint64_t *>(acc + j), (uint64_t)0,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (v != 0) emit(nstar, j, v);
            }
        }
        finish_slot(s, nstar);
    }

    __device__ __forceinline__ void finish_slot(GroupSlot &s, uint32_t nstar) const
    {
        if (gl == 0) {
            if (D->slot_nstar) D->slot_nstar[s.p - D->p0] = nstar;
            if (D->slot_units) D->slot_units[s.p - D->p0] = s.S;
        }
        stat_max(ST_NSTAR_MAX, nstar);
        s.mode = MODE_NEED_SLOT;
    }

    __device__ __forceinline__ void begin_rollback(GroupSlot &s, uint32_t draws) const
    {
        stat_add(ST_REPS_ABORTED, 1);
        stat_add(ST_ROLLBACK_UNITS, draws);
        stat_add(ST_PROGRESS, 2ull * draws);
        s.target = draws;
        s.sgn = -1;
        s.mode = MODE_NEED_REP;
    }

    // Once the draw count has reached the replication's limit: completion,
    // retention, abort, end of replay (the one-lane sampler's rules).
    __device__ void after_step(GroupSlot &s) const
    {
        const uint32_t d = s.t;
        const bool capped = (s.tau == 0u) && (d >= D->capmax);
        const bool ended = capped || (s.tau != 0u && d >= D->ell);
        if (s.sgn < 0) {
            if (d == s.target) {
                if (capped) truncation(s);
                flush_slot(s);
            }
            return;
        }
        if (ended) {
            if (capped) truncation(s);
            const uint64_t C = d;
            const bool retained = (s.r == 1u) || (s.S + C <= D->B);
            if (!retained) { begin_rollback(s, d); return; }
            s.S += C;
            s.nret += 1u;
            stat_add(ST_RETAINED_UNITS, C);
            stat_add(ST_PROGRESS, C);
            stat_add(ST_REPS_RETAINED, 1);
            if (capped) {
                stat_add(ST_CAP_HITS, 1);
                stat_add(ST_SINGLE_SITE, 1 + 2 * (C - 1));
            } else {
                const uint64_t mt = s.tau < d ? s.tau : d;
                stat_add(ST_SINGLE_SITE, 1 + 2 * (mt - 1) + (C - mt));
                stat_add(ST_TAU_SUM, s.tau);
                stat_max(ST_TAU_MAX, s.tau);
                uint32_t bin = s.tau / D->hist_width;
                if (bin >= a.hist_bins) bin = a.hist_bins - 1u;
                if (gl == 0) atomicAdd(hist_lds + bin, 1u);
            }
            if (s.r == 1u && C > D->B) stat_add(ST_ZERO_COMPLETION, 1);
            if (!a.refill || s.S >= D->B || s.S + D->cmin > D->B) flush_slot(s);
            else s.mode = MODE_NEED_REP;
            return;
        }
        if (s.r >= 2u && (uint64_t)d > D->B - s.S) begin_rollback(s, d);
    }

    __device__ __forceinline__ void start_rep(GroupSlot &s) const
    {
        if (s.sgn > 0) {
            s.r += 1u;
            stat_add(ST_REPS_STARTED, 1);
        }
        reset_state();
        if (a.init_mode) init_prior(s);
        s.t = 0;
        s.tau = 0;
        s.mu = 0;
        // the first draw count past the window end at which the bookkeeping
        // must look: the cap, the end of a replay, the abort point
        uint32_t stop = D->capmax;
        if (s.sgn < 0 && s.target < stop) stop = s.target;
        if (s.r >= 2u) {
            const uint64_t ab = D->B - s.S + 1u;
            if (ab < (uint64_t)stop) stop = (uint32_t)ab;
        }
        s.stop = stop;
        s.lim = D->ell < stop ? D->ell : stop;
        s.mode = MODE_RUN;
    }

    // One step of the group: up to gsz draws from s.t, of which a prefix stands.
    __device__ __forceinline__ void iterate(GroupSlot &s) const
    {
        using R = Row<F>;
        // the next draw count at which something may have to be decided
        const uint32_t stop = (s.t < D->ell && D->ell < s.stop) ? D->ell : s.stop;
        uint32_t span = stop - s.t;
        if (span > gsz) span = gsz;
        if (s.t == 0u) span = 1u;

        const uint32_t t = s.t + gl;
        const bool act = gl < span;
        const bool updY = (s.tau == 0u) && (t > 0u);
        uint32_t blk[4];
        philox10(t >> 1, s.r, s.p, D->g, k0, k1, blk);
        const uint32_t sw = (t & 1u) ? blk[2] : blk[0];
        const uint32_t hw = (t & 1u) ? blk[3] : blk[1];
        const uint32_t I = act ? site(sw) : 0u;
        Row<F> rc;
        rc.load(rows, I);
        const uint32_t bw_idx = I >> 4;
        const uint32_t bw = st[bw_idx];
        // (X, Y) counts of each entry's pool: X in the low half (a 32-bit
        // word per pool) or the low byte (a 16-bit pair per pool)
        // (padding entries name pool m, whose counts are the all-ones sentinel)
        const uint16_t *c16 = reinterpret_cast<const uint16_t *>(cst);
        constexpr uint32_t CB = WPP ? 16u : 8u;          // bits of one count
        constexpr uint32_t CM = (1u << CB) - 1u;
        uint32_t cp[R::NE];
#pragma unroll
        for (int e = 0; e < R::NE; ++e) {
            const uint32_t j = R::pool(rc.raw(e));
            cp[e] = WPP ? cst[j] : (uint32_t)c16[j];
        }
        const uint32_t sh = (I & 15u) << 1;
        const uint32_t xi = (bw >> sh) & 1u;
        const uint32_t yi = (bw >> (sh + 1u)) & 1u;
        // threshold index of the free-pool outcome pattern (first free pool
        // most significant): from the pattern table, or entry by entry
        uint32_t om = 0;   // outcome bits of the clone's entries
        if constexpr (F == FMT_U8_5) om = rc.w[R::WORDS - 1] >> 24;
        else if constexpr (PT) om = ((rc.w[0] & 0x80808080u) * 0x00204081u) >> 28;   // bits 7, 15, 23, 31
        auto index = [&](bool ych, uint32_t zi) {
            if constexpr (PT) {
                uint32_t fm = 0;
#pragma unroll
                for (int e = 0; e < R::NE; ++e)
                    fm |= (uint32_t)(((ych ? cp[e] >> CB : cp[e] & CM)) == zi) << e;
                return (uint32_t)pat8[(fm << 5) | om];
            } else {
                uint32_t pat = 0, len = 0;
#pragma unroll
                for (int e = 0; e < R::NE; ++e) {
                    const uint32_t o = R::outcome(rc.raw(e));
                    const bool fz = (ych ? cp[e] >> CB : cp[e] & CM) == zi;
                    pat = fz ? ((pat << 1) | o) : pat;
                    len += fz ? 1u : 0u;
                }
                return (1u << len) - 1u + pat;
            }
        };
        bool have_lo = false;
        uint64_t lo = 0;
        const uint32_t ix = index(false, xi);
        const uint32_t xn = decide(s, t, hw, thr[ix], have_lo, lo);
        uint32_t yn = yi;
        // most pairs meet within a few draws, after which only X moves: the
        // Y pattern is built only while the pair has not met
        if (updY) {
            const uint32_t iy = index(true, yi);
            yn = (iy == ix) ? xn : decide(s, t, hw, thr[iy], have_lo, lo);
        }
        const bool flip = act && (xn != xi || yn != yi);
        const uint64_t fm = (__ballot(flip) & gmask) >> leader;
        if (fm == 0) {
            // at the pre-lag draw (span 1) a pair that did not move meets at t = 1
            if (s.tau == 0u && s.mu == 0) s.tau = s.t + 1u;
            s.t += span;
            return;
        }
        const uint32_t f = (uint32_t)__builtin_ctzll(fm);
        // the first changing lane applies its update and its estimator
        // events, then tells the group (mu change + 1, event flag, site)
        uint32_t msg = 0;
        uint64_t ev_val = 0;   // the event's signed value (changing lane)
        if (gl == f) {
            const int dx = (int)xn - (int)xi;
            const int dy = (int)yn - (int)yi;
            st[bw_idx] = bw ^ ((uint32_t)(dx != 0) << sh) ^ ((uint32_t)(dy != 0) << (sh + 1u));
#pragma unroll
            for (int e = 0; e < R::NE; ++e) {
                const uint32_t v = rc.raw(e);
                if (!R::valid(v, (uint32_t)D->m)) continue;
                count_add(R::pool(v), dx, dy);
            }
            int dmu = 0;
            if (s.tau == 0u) dmu = (int)(xn != yn) - (int)(xi != yi);
            if (a.mismatch && dmu != 0) mismatch_event(s.sgn, I, (uint64_t)(int64_t)(-dmu) * (uint64_t)(t + 1u));
            uint64_t val = 0;
            const uint32_t te = t + 1u;
            if (dx != 0 && te <= D->ell) {
                const uint32_t from = te > D->k ? te : D->k;
                val += (uint64_t)(int64_t)dx * (uint64_t)(D->ell - from + 1u);
            }
            if (updY && t >= D->k + 1u && dx != dy)
                val -= (uint64_t)(int64_t)(dx - dy) * gsum(t, D->k, D->ell, D->W);
            uint32_t ev = 0;
            if (val != 0) {
                ev_val = s.sgn > 0 ? val : (uint64_t)0 - val;
                ev = 1;
            }
            msg = (uint32_t)(dmu + 1) | (ev << 2) | (I << 3);
        }
        const int src = (int)(leader + f);
        msg = __shfl(msg, src);
        if (msg & 4u) {
            const uint64_t v = ((uint64_t)(uint32_t)__shfl((uint32_t)(ev_val >> 32), src) << 32) |
                               (uint64_t)(uint32_t)__shfl((uint32_t)ev_val, src);
            record(msg >> 3, v, s);
        }
        if (s.tau == 0u) {
            s.mu += (int)(msg & 3u) - 1;
            if (s.mu == 0) s.tau = s.t + f + 1u;
        }
        s.t += f + 1u;
        lds_fence();
    }
};

template <bool TL, int F>
__device__ __forceinline__ void coop_item(const LaunchArgs &a, DescPtr D, uint32_t *smem, uint32_t k0, uint32_t k1)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    const uint32_t lg = D->group_log2;                // log2 of the lanes per group (the instance's)
    const uint32_t gsz = 1u << lg, groups = 64u >> lg;
    const uint32_t g = lane >> lg;
    uint32_t *hist_lds = smem + D->lds_hist;
    uint32_t *tab = smem + D->lds_tab;
    for (uint32_t b = tid; b < a.hist_bins; b += WG) hist_lds[b] = 0u;
    if (TL) {
        copy_to_lds(tab + D->tab_off_thr / 4, D->thr, D->thr_len * 2u);
        copy_to_lds(tab + D->tab_off_alias / 4, D->alias, 1u << D->abits);
        copy_to_lds(tab + D->tab_off_rows / 4, D->rows, (uint32_t)D->n * D->row_bytes / 4u);
    }
    const uint64_t *thr = D->thr;
    if (TL) {
        thr = reinterpret_cast<const uint64_t *>(tab + D->tab_off_thr / 4);
    } else if (D->place & PLACE_THR_LDS) {
        copy_to_lds(tab, D->thr, D->thr_len * 2u);
        thr = reinterpret_cast<const uint64_t *>(tab);
    }
    const uint32_t gl = lane & (gsz - 1u);
    Coop<TL, F> C{a,
                  D,
                  k0,
                  k1,
                  nullptr,
                  nullptr,
                  reinterpret_cast<const uint8_t *>(smem),
                  thr,
                  TL ? tab + D->tab_off_alias / 4 : D->alias,
                  TL ? tab + D->tab_off_rows / 4 : D->rows,
                  gl,
                  gsz,
                  g << lg,
                  gsz == 64u ? ~0ull : (((1ull << gsz) - 1ull) << (g << lg)),
                  nullptr,
                  nullptr,
                  hist_lds,
                  smem,
                  0u,
                  NO_TAG,
                  0ull};
    C.point(smem, wave * groups + g);
    for (uint32_t i = gl; i < (uint32_t)ST_COUNT; i += gsz) C.stat_clear(i);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __syncthreads();
    const uint32_t P = D->P;
    GroupSlot s;
    s.mode = MODE_NEED_SLOT;
    s.p = s.r = s.t = s.nret = s.tau = s.target = s.lim = s.stop = s.lc = s.cptr = 0;
    s.mu = 0;
    s.sgn = 1;
    s.S = 0;
    for (;;) {
        // slot and replication changes (rare): one wave-wide test when every
        // group is running
        if (!__all(s.mode == MODE_RUN)) {
            if (s.mode == MODE_NEED_SLOT) {
                uint32_t p = 0;
                if (C.gl == 0) p = take_slot(D);
                p = __shfl(p, (int)C.leader);
                if (p >= P) {
                    s.mode = MODE_DONE;
                    C.flush_stats();
                } else {
                    s.p = p + D->p0;   // global slot index (the random-number counter)
                    s.r = 0;
                    s.S = 0;
                    s.nret = 0;
                    s.lc = 0;
                    s.cptr = 0;
                    s.sgn = 1;
                    s.mode = MODE_NEED_REP;
                }
            }
            if (s.mode == MODE_NEED_REP) C.start_rep(s);
            // A group with no slot left joins its buddy (the aligned group of
            // the same size next to it): with a running buddy, the merged
            // group carries on the buddy's slot with twice the lanes and
            // looks twice as far ahead; two finished groups merge so that
            // they can join a larger running group later.  Every group size
            // commits the same draws, so results do not change.
            for (;;) {
                const bool done = s.mode == MODE_DONE;
                const uint32_t bl = (C.leader ^ C.gsz) & 63u;
                const uint32_t bsz = __shfl(C.gsz, (int)bl);
                const bool bdone = __shfl((uint32_t)done, (int)bl) != 0u;
                const bool merge = C.gsz < 64u && bsz == C.gsz && (done || bdone);
                if (!__any(merge)) break;
                // the running group's leader; for two finished groups the lower one
                const uint32_t lower = C.leader < bl ? C.leader : bl;
                const int src = (int)(!done ? C.leader : (!bdone ? bl : lower));
                GroupSlot t;
                t.mode = __shfl(s.mode, src);
                t.p = __shfl(s.p, src);
                t.r = __shfl(s.r, src);
                t.t = __shfl(s.t, src);
                t.nret = __shfl(s.nret, src);
                t.tau = __shfl(s.tau, src);
                t.target = __shfl(s.target, src);
                t.lim = __shfl(s.lim, src);
                t.stop = __shfl(s.stop, src);
                t.lc = __shfl(s.lc, src);
                t.cptr = __shfl(s.cptr, src);
                t.mu = __shfl(s.mu, src);
                t.sgn = __shfl(s.sgn, src);
                t.S = ((uint64_t)__shfl((uint32_t)(s.S >> 32), src) << 32) | (uint64_t)__shfl((uint32_t)s.S, src);
                const uint32_t tg = __shfl(C.gid, src);
                if (merge) {
                    s = t;
                    C.leader = lower;
                    C.gsz *= 2u;
                    C.gl = lane - C.leader;
                    C.gmask = C.gsz == 64u ? ~0ull : (((1ull << C.gsz) - 1ull) << C.leader);
                    C.point(smem, tg);
                }
            }
            if (__all(s.mode == MODE_DONE)) break;
        }
        if (s.mode == MODE_RUN) {
            C.iterate(s);
            if (s.t >= s.lim) C.after_step(s);
        }
    }
    __syncthreads();
    uint64_t *hist = D->hist;
    for (uint32_t b = tid; b < a.hist_bins; b += WG)
        if (hist_lds[b]) atomicAdd(reinterpret_cast<unsigned long long *>(hist + b), (unsigned long long)hist_lds[b]);
    __syncthreads();
}

// The cooperative variant of the persistent kernel (chain state always in
// LDS, one slot per group of lanes).
template <int F>
__global__ void __launch_bounds__(256, coop_waves_per_simd(F)) coop_kernel(LaunchArgs a)
{
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t sh_item, sh_skip;
    const uint64_t seed = *(const __attribute__((address_space(4))) uint64_t *)a.seed;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    DescPtr descs = (DescPtr)a.inst;
    const __attribute__((address_space(4))) uint32_t *tickets =
        (const __attribute__((address_space(4))) uint32_t *)a.tickets;
    if constexpr (coop_pattern_table(F)) {
        // threshold index of every (free mask f, outcome bits o) of a clone's
        // entries: the outcomes of the free entries in entry order, first
        // most significant, as the pattern p of length |f| at (1 << |f|) - 1 + p.
        // Free mask high: draws that find every pool free read 8 consecutive
        // dwords whatever their outcome bits, with no bank conflicts.
        uint8_t *pt = reinterpret_cast<uint8_t *>(smem);
        for (uint32_t x = threadIdx.x; x < PATTERN_TABLE_BYTES; x += WG) {
            const uint32_t f = x >> 5, o = x & 31u;
            uint32_t p = 0, len = 0;
            for (uint32_t e = 0; e < 5u; ++e) {
                if ((f >> e) & 1u) {
                    p = (p << 1) | ((o >> e) & 1u);
                    ++len;
                }
            }
            pt[x] = (uint8_t)((1u << len) - 1u + p);
        }
        // visible to every wavefront after the ticket loop's first barrier
    }
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t it = take_ticket(a);
            uint32_t skip = 1;
            if (it < a.nticket) {
                skip = !slots_left(a.inst + a.tickets[it]);
            }
            sh_item = it;
            sh_skip = skip;
        }
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(sh_item);
        const uint32_t skip = __builtin_amdgcn_readfirstlane(sh_skip);
        __syncthreads();
        if (item >= a.nticket) break;
        if (skip) continue;
        DescPtr D = descs + tickets[item];
        if (D->place & PLACE_TABLES_LDS) coop_item<true, F>(a, D, smem, k0, k1);
        else coop_item<false, F>(a, D, smem, k0, k1);
    }
}

}  // namespace

// Launch of the sampler for row format F.  The build compiles this file once
// per format with MCPD_FMT set (the instantiations take most of the compile
// time) and once without it for the dispatcher and the fill kernel.
template <int F>
int launch_sampler_fmt(const LaunchArgs &a, int grid, size_t lds, void *stream, bool coop)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const void *fn = coop ? reinterpret_cast<const void *>(coop_kernel<F>)
                          : reinterpret_cast<const void *>(sampler_kernel<F>);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return (int)e;
    }
    if (coop) hipLaunchKernelGGL((coop_kernel<F>), dim3(grid), dim3(WG), lds, st, a);
    else hipLaunchKernelGGL((sampler_kernel<F>), dim3(grid), dim3(WG), lds, st, a);
    return (int)hipGetLastError();
}

template int launch_sampler_fmt<MCPD_FMT>(const LaunchArgs &, int, size_t, void *, bool);

#else

__global__ void fill_zero_kernel(uint64_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

int launch_sampler(const LaunchArgs &a, int fmt, int grid, size_t lds, void *stream, bool coop)
{
    switch (fmt) {
    case FMT_U8_4: return launch_sampler_fmt<FMT_U8_4>(a, grid, lds, stream, coop);
    case FMT_U8_5: return launch_sampler_fmt<FMT_U8_5>(a, grid, lds, stream, coop);
    case FMT_U8_8: return launch_sampler_fmt<FMT_U8_8>(a, grid, lds, stream, coop);
    case FMT_U8_12: return launch_sampler_fmt<FMT_U8_12>(a, grid, lds, stream, coop);
    case FMT_U16_4: return launch_sampler_fmt<FMT_U16_4>(a, grid, lds, stream, coop);
    case FMT_U16_8: return launch_sampler_fmt<FMT_U16_8>(a, grid, lds, stream, coop);
    case FMT_U16_12: return launch_sampler_fmt<FMT_U16_12>(a, grid, lds, stream, coop);
    default: return (int)hipErrorInvalidValue;
    }
}

__global__ void put_u64_kernel(uint64_t *p, uint64_t v)
{
    if (threadIdx.x == 0) *p = v;
}

int launch_put_u64(uint64_t *p, uint64_t v, void *stream)
{
    hipLaunchKernelGGL(put_u64_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), p, v);
    return (int)hipGetLastError();
}

int launch_fill_zero(uint64_t *p, size_t n64, void *stream)
{
    if (n64 == 0) return (int)hipSuccess;
    const size_t blocks = std::min<size_t>((n64 + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), p, n64);
    return (int)hipGetLastError();
}
#endif

}  // namespace mcpd
