// Persistent slot-refill sampler for unbiased Markov chain pool decoding on
// gfx950.
//
// One lane owns one logical slot at a time (Algorithm 4: "the GPU scheduler
// maps a logical slot p to one persistent thread") and runs its i.i.d.
// coupled replications (Algorithm 3) one after the other.  Slots are handed
// out dynamically from a global counter; the result does not depend on which
// lane runs which slot because every random number is keyed by
// (instance, slot, replication, draw).
//
// Per-lane chain state (both chains X and Y):
//   bit words   : 16 clones per dword, clone i at bits 2(i mod 16) (x) and
//                 2(i mod 16)+1 (y)
//   count words : 2 pools per dword, pool j at byte 2(j mod 2) (c^X_j) and
//                 2(j mod 2)+1 (c^Y_j), c_j = sum_i A_ji x_i
// laid out structure-of-arrays with the lane index fastest, so that the 64
// lanes of a wave touching any word index hit 64 distinct banks.  The state
// lives in LDS when the instance fits, otherwise in global memory with the
// same layout.
//
// Estimator: the numerator V_j = W H_{k:l}(h_j) (Section "Coupled Estimator
// and Fixed-Budget GPU Execution") is accumulated exactly in 64-bit integers
// from flip events only.  With Delta_j(s) = x_j(s) - y_j(s-1) and
// G(t) = sum_{s=k+1}^{t} min(s-k, W), exchanging the sums gives
//   V_j = sum_{flips of x_j at time s} dx (l - max(s,k) + 1)^+
//       - sum_{changes c of Delta_j at time s} c G(s-1)
//       (+ G(C) Delta_j(C) for a pair stopped by the cap),
// using sum_s c = Delta_j(C) (= 0 once the pair has met, Theorem 1 (d)).
// A draw at t changes Delta at time t+1 by dx - dy.  Numerators go to a
// per-lane row of int64 with no-return atomics; a replication that can no
// longer be retained (it would complete beyond B) is stopped and rolled back
// by replaying its draws with negated contributions.  At the end of a slot
// its numerators are added to integer buckets keyed by N*_p, which makes the
// completion-time-corrected aggregate exact and order-independent.
#include <hip/hip_runtime.h>

#include "mcpd_device.h"

namespace mcpd {
namespace {

constexpr uint32_t MODE_NEED_SLOT = 0;
constexpr uint32_t MODE_NEED_REP = 1;
constexpr uint32_t MODE_RUN = 2;
constexpr uint32_t MODE_DONE = 3;
constexpr uint32_t NO_TAG = 0xFFFFFFFFu;

// Philox4x32-10 (Salmon et al., SC'11).  The key is wave-uniform, so its
// schedule stays on the scalar unit.
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
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
    uint32_t mode, p, r, t, nret, tau, target;
    int32_t mu, sgn;
    uint64_t S;
    uint32_t lc, f0, f1;
    uint64_t st[ST_COUNT];
};

template <int R>
struct RowWords { uint32_t w[R / 2]; };

template <int R>
__device__ __forceinline__ RowWords<R> load_row(const uint16_t *rows, uint32_t I)
{
    RowWords<R> rw;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(rows + (size_t)I * R);
    if constexpr (R == 4) {
        const uint2 v = *reinterpret_cast<const uint2 *>(src);
        rw.w[0] = v.x; rw.w[1] = v.y;
    } else if constexpr (R == 8) {
        const uint4 v = *reinterpret_cast<const uint4 *>(src);
        rw.w[0] = v.x; rw.w[1] = v.y; rw.w[2] = v.z; rw.w[3] = v.w;
    } else {
        const uint4 v = *reinterpret_cast<const uint4 *>(src);
        const uint4 u = *reinterpret_cast<const uint4 *>(src + 4);
        rw.w[0] = v.x; rw.w[1] = v.y; rw.w[2] = v.z; rw.w[3] = v.w;
        rw.w[4] = u.x; rw.w[5] = u.y; rw.w[6] = u.z; rw.w[7] = u.w;
    }
    return rw;
}

template <int R>
__device__ __forceinline__ uint32_t row_entry(const RowWords<R> &rw, int e)
{
    return (rw.w[e >> 1] >> ((e & 1) * 16)) & 0xFFFFu;
}

template <bool LDS, int R>
struct Sampler {
    const RunArgs &a;
    uint32_t *st;      // this workgroup's state base (LDS or global)
    uint32_t L;        // lanes per workgroup (state stride)
    uint32_t lane;     // lane within the workgroup
    int64_t *acc;      // this lane's numerator row
    uint32_t *list;    // this lane's touched list
    uint32_t *hist_lds;

    __device__ __forceinline__ uint32_t &bits(uint32_t w) const { return st[w * L + lane]; }
    __device__ __forceinline__ uint32_t &cnt(uint32_t q) const
    {
        return st[(a.words_bits + q) * L + lane];
    }

    __device__ void reset_state() const
    {
        const uint32_t nw = a.words_bits + a.words_cnt;
        for (uint32_t w = 0; w < nw; ++w) st[w * L + lane] = 0u;
    }

    __device__ __forceinline__ void event(Lane &s, uint32_t j, uint64_t v) const
    {
        atomicAdd(reinterpret_cast<unsigned long long *>(acc + j), (unsigned long long)v);
        if (j != s.f0 && j != s.f1) {
            if (s.lc < a.list_cap) list[s.lc] = j;
            s.lc += 1;
            s.f1 = s.f0;
            s.f0 = j;
        }
    }

    // Low 53-b bits of U of draw t (block (t, r, p, g | 2^24)).
    __device__ uint64_t low_bits(const Lane &s, uint32_t t) const
    {
        uint32_t o[4];
        philox10(t, s.r, s.p, a.g | (1u << 24), (uint32_t)a.seed, (uint32_t)(a.seed >> 32), o);
        const uint64_t v = ((uint64_t)o[0] << 32) | (uint64_t)o[1];
        return v >> (11u + a.ubits);
    }

    // 1{U53 <= T}, U53 = (hw >> (32-b)) << (53-b) | low.
    __device__ __forceinline__ uint32_t decide(const Lane &s, uint32_t t, uint32_t hw, uint64_t T,
                                               bool &have_lo, uint64_t &lo) const
    {
        const uint32_t b = a.ubits;
        const uint64_t hb = (uint64_t)(hw >> (32u - b));
        const uint64_t th = T >> (53u - b);
        if (hb != th) return hb < th ? 1u : 0u;
        if (!have_lo) { lo = low_bits(s, t); have_lo = true; }
        return lo <= (T & ((1ull << (53u - b)) - 1ull)) ? 1u : 0u;
    }

    // One draw t of the current replication with site word sw and U word hw.
    __device__ void step(Lane &s, uint32_t sw, uint32_t hw) const
    {
        const DevTables &T = a.T;
        const uint32_t t = s.t;
        uint32_t I = T.guide[sw >> T.gshift];
        while (T.cum_hi[I] < sw) ++I;
        const RowWords<R> rw = load_row<R>(T.rows, I);
        const uint32_t bw_idx = I >> 4;
        const uint32_t bw = bits(bw_idx);
        const uint32_t sh = (I & 15u) << 1;
        const uint32_t xi = (bw >> sh) & 1u;
        const uint32_t yi = (bw >> (sh + 1u)) & 1u;
        const bool updY = (s.tau == 0u) && (t > 0u);

        uint32_t patX = 0, lenX = 0, patY = 0, lenY = 0;
#pragma unroll
        for (int e = 0; e < R; ++e) {
            const uint32_t v = row_entry<R>(rw, e);
            if (v == 0xFFFFu) continue;
            const uint32_t j = v & 0x7FFFu, yj = v >> 15;
            const uint32_t cw = cnt(j >> 1);
            const uint32_t cs = (j & 1u) << 4;
            const uint32_t cx = (cw >> cs) & 0xFFu;
            const uint32_t cy = (cw >> (cs + 8u)) & 0xFFu;
            if (cx == xi) { patX = (patX << 1) | yj; ++lenX; }
            if (cy == yi) { patY = (patY << 1) | yj; ++lenY; }
        }
        bool have_lo = false;
        uint64_t lo = 0;
        const uint32_t xn = decide(s, t, hw, T.thr[(1u << lenX) - 1u + patX], have_lo, lo);
        uint32_t yn = yi;
        if (updY) yn = decide(s, t, hw, T.thr[(1u << lenY) - 1u + patY], have_lo, lo);
        const int dx = (int)xn - (int)xi;
        const int dy = (int)yn - (int)yi;
        if (dx | dy) {
            bits(bw_idx) = bw ^ ((uint32_t)(dx != 0) << sh) ^ ((uint32_t)(dy != 0) << (sh + 1u));
#pragma unroll
            for (int e = 0; e < R; ++e) {
                const uint32_t v = row_entry<R>(rw, e);
                if (v == 0xFFFFu) continue;
                const uint32_t j = v & 0x7FFFu;
                const uint32_t cs = (j & 1u) << 4;
                const uint32_t delta = ((uint32_t)dx << cs) + ((uint32_t)dy << (cs + 8u));
                cnt(j >> 1) += delta;
            }
        }
        if (s.tau == 0u) s.mu += (int)(xn != yn) - (int)(xi != yi);
        // estimator events at time te = t + 1
        uint64_t val = 0;
        const uint32_t te = t + 1u;
        if (dx != 0 && te <= a.ell) {
            const uint32_t from = te > a.k ? te : a.k;
            val += (uint64_t)(int64_t)dx * (uint64_t)(a.ell - from + 1u);
        }
        if (updY && t >= a.k + 1u && dx != dy) {
            val -= (uint64_t)(int64_t)(dx - dy) * gsum(t, a.k, a.ell, a.W);
        }
        if (val != 0) event(s, I, s.sgn > 0 ? val : (uint64_t)0 - val);
        if (s.tau == 0u && s.mu == 0) s.tau = te;
        s.t = te;
    }

    // Boundary term G(C) Delta_j(C) of a pair stopped by the cap.
    __device__ void truncation(Lane &s) const
    {
        const uint32_t C = s.t;
        if (C < a.k + 1u) return;
        const uint64_t G = gsum(C, a.k, a.ell, a.W);
        for (uint32_t w = 0; w < a.words_bits; ++w) {
            const uint32_t word = bits(w);
            uint32_t mis = (word ^ (word >> 1)) & 0x55555555u;
            while (mis) {
                const uint32_t b = __builtin_ctz(mis);
                mis &= mis - 1u;
                const uint32_t j = w * 16u + (b >> 1);
                const uint64_t v = ((word >> b) & 1u) ? G : (uint64_t)0 - G;
                event(s, j, s.sgn > 0 ? v : (uint64_t)0 - v);
            }
        }
    }

    __device__ void emit(uint32_t nstar, uint32_t j, int64_t v) const
    {
        if (nstar > a.nbuckets) {
            atomicOr(&a.ctrl[1], (uint32_t)ERR_BUCKETS);
            return;
        }
        const size_t idx = (size_t)(nstar - 1u) * (size_t)a.T.n + j;
        atomicAdd(reinterpret_cast<unsigned long long *>(a.S1 + idx), (unsigned long long)v);
        const uint64_t u = v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v;
        const uint64_t lo = u * u;
        const uint64_t hi = __umul64hi(u, u);
        const unsigned long long old =
            atomicAdd(reinterpret_cast<unsigned long long *>(a.S2 + 2 * idx), (unsigned long long)lo);
        const uint64_t carry = ((uint64_t)old + lo < (uint64_t)old) ? 1u : 0u;
        if (hi + carry)
            atomicAdd(reinterpret_cast<unsigned long long *>(a.S2 + 2 * idx + 1),
                      (unsigned long long)(hi + carry));
    }

    __device__ void flush_slot(Lane &s) const
    {
        const uint32_t nstar = s.nret;
        if (s.lc <= a.list_cap) {
            for (uint32_t e = 0; e < s.lc; ++e) {
                const uint32_t j = __hip_atomic_load(list + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int64_t v = (int64_t)atomicExch(reinterpret_cast<unsigned long long *>(acc + j), 0ull);
                if (v != 0) emit(nstar, j, v);
            }
        } else {
            for (uint32_t j = 0; j < (uint32_t)a.T.n; ++j) {
                const int64_t v = (int64_t)atomicExch(reinterpret_cast<unsigned long long *>(acc + j), 0ull);
                if (v != 0) emit(nstar, j, v);
            }
        }
        if (a.slot_nstar) a.slot_nstar[s.p] = nstar;
        if (a.slot_units) a.slot_units[s.p] = s.S;
        if (nstar > s.st[ST_NSTAR_MAX]) s.st[ST_NSTAR_MAX] = nstar;
        s.mode = MODE_NEED_SLOT;
    }

    __device__ void begin_rollback(Lane &s, uint32_t draws) const
    {
        s.st[ST_REPS_ABORTED] += 1;
        s.st[ST_ROLLBACK_UNITS] += draws;
        s.target = draws;
        s.sgn = -1;
        s.mode = MODE_NEED_REP;
    }

    // Bookkeeping after a draw: completion, retention, abort, end of replay.
    __device__ void after_step(Lane &s) const
    {
        const uint32_t d = s.t;
        const bool capped = (s.tau == 0u) && ((uint64_t)d >= a.capmax);
        const bool ended = capped || (s.tau != 0u && d >= a.ell);
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
            const bool retained = (s.r == 1u) || (s.S + C <= a.B);
            if (!retained) { begin_rollback(s, d); return; }
            s.S += C;
            s.nret += 1u;
            s.st[ST_RETAINED_UNITS] += C;
            s.st[ST_REPS_RETAINED] += 1;
            if (capped) {
                s.st[ST_CAP_HITS] += 1;
                s.st[ST_SINGLE_SITE] += 1 + 2 * (C - 1);
            } else {
                const uint64_t mt = s.tau < d ? s.tau : d;
                s.st[ST_SINGLE_SITE] += 1 + 2 * (mt - 1) + (C - mt);
                s.st[ST_TAU_SUM] += s.tau;
                if (s.tau > s.st[ST_TAU_MAX]) s.st[ST_TAU_MAX] = s.tau;
                uint32_t bin = s.tau / a.hist_width;
                if (bin >= a.hist_bins) bin = a.hist_bins - 1u;
                atomicAdd(hist_lds + bin, 1u);
            }
            if (s.r == 1u && C > a.B) s.st[ST_ZERO_COMPLETION] += 1;
            if (!a.refill || s.S >= a.B || s.S + a.cmin > a.B) flush_slot(s);
            else s.mode = MODE_NEED_REP;
            return;
        }
        if (s.r >= 2u && (uint64_t)d > a.B - s.S) begin_rollback(s, d);
    }
};

template <bool LDS, int R>
__global__ void __launch_bounds__(256) sampler_kernel(RunArgs a)
{
    extern __shared__ uint32_t smem[];
    const uint32_t L = blockDim.x;
    const uint32_t lane = threadIdx.x;
    const uint32_t words = a.words_bits + a.words_cnt;
    uint32_t *hist_lds = LDS ? smem + (size_t)words * L : smem;
    for (uint32_t b = lane; b < a.hist_bins; b += L) hist_lds[b] = 0u;
    __syncthreads();

    const size_t gl = (size_t)blockIdx.x * L + lane;
    Sampler<LDS, R> S{a,
                      LDS ? smem : a.gstate + (size_t)blockIdx.x * words * L,
                      L,
                      lane,
                      a.acc + gl * (size_t)a.T.n,
                      a.lists + gl * (size_t)a.list_cap,
                      hist_lds};
    Lane s;
    s.mode = MODE_NEED_SLOT;
    s.p = s.r = s.t = s.nret = s.tau = s.target = 0;
    s.mu = 0;
    s.sgn = 1;
    s.S = 0;
    s.lc = 0;
    s.f0 = s.f1 = NO_TAG;
    for (int i = 0; i < ST_COUNT; ++i) s.st[i] = 0;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);

    for (;;) {
        if (s.mode == MODE_NEED_SLOT) {
            const uint32_t p = atomicAdd(&a.ctrl[0], 1u);
            if (p >= a.P) {
                s.mode = MODE_DONE;
            } else {
                s.p = p;
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
                s.st[ST_REPS_STARTED] += 1;
            }
            S.reset_state();
            s.t = 0;
            s.tau = 0;
            s.mu = 0;
            s.mode = MODE_RUN;
        }
        if (__all(s.mode == MODE_DONE)) break;
        if (s.mode == MODE_RUN) {
            uint32_t w[4];
            philox10(s.t >> 1, s.r, s.p, a.g, k0, k1, w);
            S.step(s, w[0], w[1]);
            s.st[ST_PROGRESS] += 1;
            S.after_step(s);
            if (s.mode == MODE_RUN) {
                S.step(s, w[2], w[3]);
                s.st[ST_PROGRESS] += 1;
                S.after_step(s);
            }
        }
    }

    // Statistics: wave reduction, then one atomic per wave.
    for (int i = 0; i < ST_COUNT; ++i) {
        uint64_t v = s.st[i];
        const bool is_max = (i == ST_TAU_MAX || i == ST_NSTAR_MAX);
        for (int off = 32; off > 0; off >>= 1) {
            const uint64_t o = __shfl_xor(v, off);
            v = is_max ? (o > v ? o : v) : v + o;
        }
        if ((lane & 63u) == 0u) {
            if (is_max) atomicMax(reinterpret_cast<unsigned long long *>(a.stats + i), (unsigned long long)v);
            else atomicAdd(reinterpret_cast<unsigned long long *>(a.stats + i), (unsigned long long)v);
        }
    }
    __syncthreads();
    for (uint32_t b = lane; b < a.hist_bins; b += L)
        if (hist_lds[b]) atomicAdd(reinterpret_cast<unsigned long long *>(a.hist + b), (unsigned long long)hist_lds[b]);
}

template <bool LDS>
int launch_R(const RunArgs &a, int grid, int block, int R, size_t lds, hipStream_t st)
{
    switch (R) {
    case 4: hipLaunchKernelGGL((sampler_kernel<LDS, 4>), dim3(grid), dim3(block), lds, st, a); break;
    case 8: hipLaunchKernelGGL((sampler_kernel<LDS, 8>), dim3(grid), dim3(block), lds, st, a); break;
    case 16: hipLaunchKernelGGL((sampler_kernel<LDS, 16>), dim3(grid), dim3(block), lds, st, a); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace

int launch_sampler(const RunArgs &a, int grid, int block, bool lds_state, int row_stride, void *stream)
{
    const size_t words = (size_t)a.words_bits + a.words_cnt;
    const size_t lds = (lds_state ? words * (size_t)block * 4u : 0u) + (size_t)a.hist_bins * 4u;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (lds_state) {
        if (lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(
                reinterpret_cast<const void *>(row_stride == 4 ? sampler_kernel<true, 4>
                                               : row_stride == 8 ? sampler_kernel<true, 8>
                                                                 : sampler_kernel<true, 16>),
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return (int)e;
        }
        return launch_R<true>(a, grid, block, row_stride, lds, st);
    }
    return launch_R<false>(a, grid, block, row_stride, lds, st);
}

}  // namespace mcpd
