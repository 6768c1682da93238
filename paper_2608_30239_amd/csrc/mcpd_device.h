// Internal types shared by the host side of the library and its kernels.
// Not part of the public ABI (include/mcpd.h).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace mcpd {

// Clone rows: the pools of one clone in ascending order, each entry
// pool | (outcome << top bit), padded with all-ones entries.  A format fixes
// the entry width and the number of entries the kernel reads (a compile-time
// loop length).
enum RowFmt {
    FMT_U8_4 = 0,   // 4-byte rows, 4 one-byte entries (pools < 127)
    FMT_U8_5 = 1,   // 8-byte rows, 5 one-byte entries
    FMT_U8_8 = 2,   // 8-byte rows, 8 one-byte entries
    FMT_U8_12 = 3,  // 16-byte rows, 12 one-byte entries
    FMT_U16_4 = 4,  // 8-byte rows, 4 two-byte entries (pools < 32767)
    FMT_U16_8 = 5,  // 16-byte rows, 8 two-byte entries
    FMT_U16_12 = 6, // 32-byte rows, 12 two-byte entries
    FMT_COUNT = 7
};

__host__ __device__ constexpr int fmt_entries(int f)
{
    return f == FMT_U8_4 ? 4 : f == FMT_U8_5 ? 5 : f == FMT_U8_8 ? 8 : f == FMT_U8_12 ? 12
         : f == FMT_U16_4 ? 4 : f == FMT_U16_8 ? 8 : 12;
}
__host__ __device__ constexpr bool fmt_wide(int f) { return f >= FMT_U16_4; }
// Count words of the cooperative kernel's chain state: with one-byte entries
// (fewer than 127 pools) one 32-bit word per pool, the X count in the low
// half and the Y count in the high half, so that a count update is one LDS
// add at the pool's word; with two-byte entries one 16-bit pair per pool (X
// in the low byte), two pools per word, to keep large pool counts in LDS.
__host__ __device__ constexpr bool coop_word_per_pool(int f) { return !fmt_wide(f); }
// Formats whose cooperative kernel finds the threshold index of a draw in a
// 1 KB table at the start of LDS, indexed by the free mask of the clone's
// pools (5 bits, high) and its outcome bits (5), instead of building the
// pattern entry by entry.  Rows of FMT_U8_5 carry the outcome bits in their last byte.
__host__ __device__ constexpr bool coop_pattern_table(int f) { return f == FMT_U8_4 || f == FMT_U8_5; }
constexpr uint32_t PATTERN_TABLE_BYTES = 1024;
__host__ __device__ constexpr int fmt_row_bytes(int f)
{
    return f == FMT_U8_4 ? 4 : (f == FMT_U8_5 || f == FMT_U8_8 || f == FMT_U16_4) ? 8
         : (f == FMT_U8_12 || f == FMT_U16_8) ? 16 : 32;
}

// Lanes per workgroup; also the stride of the lane-fastest state layout.
constexpr uint32_t WG_LANES = 256;

enum Place : uint32_t { PLACE_STATE_LDS = 1, PLACE_TABLES_LDS = 2, PLACE_COOP = 4, PLACE_THR_LDS = 8 };
// PLACE_THR_LDS: the cooperative kernel keeps the threshold table in LDS
// while the alias table and rows stay in global memory (rows of up to 8
// entries, at most 511 thresholds), so a draw waits on two global reads
// instead of three.

// Wavefronts of a workgroup of the cooperative kernel.
constexpr uint32_t COOP_WAVES_PER_WG = WG_LANES / 64;

// Wavefronts of the cooperative kernel per SIMD: 5 (at most 96 VGPRs) for
// rows of up to 5 entries and for 16-bit rows of 8 entries, which fit them;
// 4 for the other wide rows, whose extra registers would otherwise spill.
// With 4 SIMDs per CU, that many of its workgroups fit on a CU.
__host__ __device__ constexpr uint32_t coop_waves_per_simd(int f)
{
    return (fmt_entries(f) <= 5 || f == FMT_U16_8) ? 5u : 4u;
}

// One instance of a launch, in device memory.  The kernel reads it with
// scalar loads after a workgroup has taken a ticket for the instance.
struct InstDesc {
    // Read-only tables.  Alias table of the site draw: 2^abits columns of
    // capacity K = 2^(32 - abits); word c = T_c | A_c << (32 - abits), where
    // column c keeps clone c when the coin (low 32 - abits bits of the site
    // word) is below T_c and otherwise gives clone A_c.  A column that always
    // keeps its clone is stored as T_c = 0, A_c = c.
    const uint32_t *alias;
    const uint32_t *rows;   // [n * row_bytes / 4] clone rows in the launch's format
    const uint64_t *thr;    // [2^(dmax+1) - 1]: floor(p * 2^53) per ordered free-pool outcome pattern
    int32_t n, m;
    uint32_t abits, row_bytes, thr_len;
    uint32_t words_bits, words_cnt;   // per-lane state words (bit pairs, count pairs)
    uint32_t lanes;         // slots a workgroup runs at once: active lanes (the LDS state
                            // stride) of the lane kernel, or its groups in the cooperative one
    // Run parameters.
    uint64_t B;             // per-slot horizon
    uint32_t capmax;        // draws after which an unmet pair stops
    uint32_t P;             // slots
    uint32_t p0;            // global index of the first slot (random-number counter)
    uint32_t slot_q;        // slots per counter: counter x hands out [x q, min((x+1) q, P))
    uint32_t k, ell, W;     // window
    uint32_t cmin;          // max(ell, 1): cost of the cheapest replication
    uint32_t g;             // instance id in the random-number counter
    uint32_t hist_width;
    uint32_t qthr;          // floor(q 2^32): Pr{Z_0,i = 1} of the prior initial state
    uint32_t nbuckets;      // rows of S1/S2
    // Placement in the launch's dynamic LDS (dword offsets).
    uint32_t place;         // Place bits
    uint32_t lds_hist, lds_tab;
    uint32_t lds_state, wave_words;   // cooperative kernel: first group's state, words per group
    uint32_t lds_stats;     // cooperative kernel: the groups' statistics (ST_COUNT words of 64 bits each)
    uint32_t group_log2;    // cooperative kernel: log2 of the lanes that run one slot of this instance (3..6)
    uint32_t tab_off_thr, tab_off_alias, tab_off_rows, tab_bytes;   // within the table block (bytes)
    // Outputs (zeroed before the launch).
    int64_t *S1;            // [nbuckets * n]
    uint64_t *S2;           // [nbuckets * n * 3]: limbs of the 128-bit sums of squares
    int64_t *Dmis;          // [n]: mismatch time per clone, summed over retained replications
    uint64_t *hist;         // [hist_bins]
    uint64_t *stats;        // [ST_COUNT]
    uint32_t *next_slot;    // [XCDS * SLOT_CTR_STRIDE]: slot counters, one per XCD
    uint32_t *slot_nstar;   // [P] or null
    uint64_t *slot_units;   // [P] or null
};

// Arguments of one launch over a batch of instances.
// XCDs of the device: workgroup i of a launch runs on XCD i mod XCDS, and
// each XCD has its own L2.
constexpr uint32_t XCDS = 8;
// An instance's slots are split into one contiguous range per XCD, each with
// its own counter in a cache line of its own (SLOT_CTR_STRIDE 32-bit words
// apart), so that taking a slot is not an atomic on one hot address.
constexpr uint32_t SLOT_CTR_STRIDE = 32;

struct LaunchArgs {
    const InstDesc *inst;
    const uint32_t *tickets;    // [nticket]: instance index a workgroup joins
    uint32_t nticket;
    uint32_t qoff[XCDS + 1];    // tickets of XCD x's queue: [qoff[x], qoff[x+1])
    uint32_t refill;
    uint32_t ubits;             // u_hi_bits
    uint32_t hist_bins;
    uint32_t list_cap;          // touched-list capacity per lane
    uint32_t acc_stride;        // >= every n
    uint32_t gwords;            // >= every global-state instance's words_bits + words_cnt
    uint32_t groups_per_wg;     // cooperative kernel: workspace rows (numerator rows, lists,
                                // statistics) per workgroup, the most groups of any instance
    uint32_t init_mode;         // 0: all-negative initial state; 1: drawn from the prior
    uint32_t mismatch;          // 1: count the mismatch times (Dmis of each instance)
    const uint64_t *seed;       // device copy of the 64-bit key
    int64_t *acc;               // [lanes * acc_stride] spilled numerators (kept zero between slots)
    uint32_t *lists;            // [lanes * list_cap]
    uint32_t *gstate;           // [lanes * gwords] chain state of global-state instances
    uint64_t *lane_stats;       // [lanes * ST_COUNT]
    uint32_t *ctrl;             // [1]: error flags, [2 + x]: tickets taken from queue x (zeroed before the launch)
};

enum Stat {
    ST_PROGRESS = 0, ST_RETAINED_UNITS, ST_SINGLE_SITE, ST_REPS_STARTED, ST_REPS_RETAINED,
    ST_REPS_ABORTED, ST_CAP_HITS, ST_ZERO_COMPLETION, ST_TAU_SUM, ST_TAU_MAX, ST_NSTAR_MAX,
    ST_ROLLBACK_UNITS, ST_LIST_OVERFLOWS, ST_COUNT
};

enum ErrFlag { ERR_BUCKETS = 1 };

// Launch the sampler over a batch (defined in mcpd_sampler.hip); fmt is the
// row format every instance's rows use.  Returns a hipError_t value as int.
// coop: the cooperative kernel (one slot per group of lanes, state in LDS).
int launch_sampler(const LaunchArgs &a, int fmt, int grid, size_t lds_bytes, void *stream, bool coop);
template <int F>
int launch_sampler_fmt(const LaunchArgs &a, int grid, size_t lds_bytes, void *stream, bool coop);

// Zero n64 64-bit words at p (a kernel, so that it can sit in a captured
// graph).  Returns a hipError_t value as int.
int launch_fill_zero(uint64_t *p, size_t n64, void *stream);
// Store one 64-bit word at p (a kernel).  Returns a hipError_t value as int.
int launch_put_u64(uint64_t *p, uint64_t v, void *stream);
// Marginals and standard errors of one instance from its integer sums,
// written to device memory (defined in mcpd_finish.hip).
int launch_finish(const int64_t *S1, const uint64_t *S2, uint32_t n, uint32_t nb, uint32_t P, uint32_t W,
                  double *marginals, double *stderr_out, void *stream);

}  // namespace mcpd
