// Internal types shared by the host side of the library and its kernels.
// Not part of the public ABI (include/mcpd.h).
#pragma once

#include <stdint.h>

namespace mcpd {

// Per-instance read-only tables in device memory.
struct DevTables {
    const uint32_t *guide;  // [1 << gbits]: smallest i with cum_hi[i] >= b << gshift
    const uint32_t *cum_hi; // [n]: M_0 + ... + M_i - 1 (inclusive upper bound of clone i's site words)
    const uint16_t *rows;   // [n * R]: pool | (y << 15), ascending, padded with 0xFFFF
    const uint64_t *thr;    // [2^(dmax+1) - 1]: floor(p * 2^53) per ordered free-pool outcome pattern
    int32_t n, m, dmax, R;
    uint32_t gshift;        // 32 - gbits
};

// Slot-block of one launch (one instance).
struct RunArgs {
    DevTables T;
    uint64_t B;         // per-slot horizon
    uint64_t capmax;    // draws after which an unmet pair stops
    uint64_t seed;
    uint32_t P;         // slots
    uint32_t k, ell, W; // window
    uint32_t cmin;      // max(ell, 1): cost of the cheapest replication
    uint32_t g;         // instance id in the random-number counter
    uint32_t refill;
    uint32_t ubits;     // u_hi_bits
    uint32_t hist_bins, hist_width;
    uint32_t words_bits, words_cnt; // per-lane state words (bit pairs, count pairs)
    uint32_t list_cap;  // touched-list capacity per lane
    uint32_t nbuckets;  // rows of S1/S2
    // per-lane storage (lanes_total = gridDim.x * blockDim.x)
    int64_t *acc;       // [lanes_total * n] numerator rows (kept zero between slots)
    uint32_t *lists;    // [lanes_total * list_cap]
    uint32_t *gstate;   // [lanes_total * (words_bits + words_cnt)] when state is not in LDS
    // outputs
    int64_t *S1;        // [nbuckets * n]
    uint64_t *S2;       // [nbuckets * n * 2]
    uint64_t *hist;     // [hist_bins]
    uint64_t *stats;    // [STAT_COUNT]
    uint32_t *slot_nstar;  // [P] or null
    uint64_t *slot_units;  // [P] or null
    uint32_t *ctrl;     // [0]: next slot, [1]: error flags
};

enum Stat {
    ST_PROGRESS = 0, ST_RETAINED_UNITS, ST_SINGLE_SITE, ST_REPS_STARTED, ST_REPS_RETAINED,
    ST_REPS_ABORTED, ST_CAP_HITS, ST_ZERO_COMPLETION, ST_TAU_SUM, ST_TAU_MAX, ST_NSTAR_MAX,
    ST_ROLLBACK_UNITS, ST_COUNT
};

enum ErrFlag { ERR_BUCKETS = 1 };

// Launch the sampler (defined in mcpd_sampler.hip).  Returns a hipError_t
// value as int.
int launch_sampler(const RunArgs &a, int grid, int block, bool lds_state, int row_stride,
                   void *stream);

}  // namespace mcpd
