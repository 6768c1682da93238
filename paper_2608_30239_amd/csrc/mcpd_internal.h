// Internal state shared by the host-side sources of the library.  Not part
// of the public ABI (include/mcpd.h).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "mcpd_device.h"

namespace mcpd {
namespace host {
struct Launch;

// Record the detail of a failure for mcpd_last_error and return the code.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
// Host-side score weights and validation (mcpd_host.cpp).
int validate_design(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *pool_idx, const uint8_t *y,
                    double fp, double fn, double q, int32_t *dmax_out);
// mcpd_run_unbiased_dev with every device buffer carved from `arena` (cap
// bytes) instead of allocated (mcpd_host.cpp).
int run_single_arena(mcpd_instance *I, uint64_t budget, uint32_t slots, uint32_t k, uint32_t m, uint64_t seed,
                     const mcpd_run_opts *opts, double *dev_marginals, double *dev_stderr, uint64_t *dev_hist,
                     mcpd_run_stats *stats, void *arena, size_t cap);
}  // namespace host
}  // namespace mcpd

#define HIP_TRY(expr)                                                        \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess) return mcpd::host::hip_fail(e_, #expr);        \
    } while (0)

struct mcpd_instance {
    int32_t n = 0, m = 0, dmax = 0, abits = 1;
    uint32_t thr_len = 1;
    double fp = 0, fn = 0, q = 0;
    std::vector<int32_t> row_ptr, pool_idx;
    std::vector<uint8_t> y;
    std::vector<uint64_t> mass;
    hipStream_t stream = nullptr;
    int device = 0;
    int cus = 0;
    uint32_t *d_alias = nullptr;
    uint64_t *d_thr = nullptr;
    uint32_t *d_rows[mcpd::FMT_COUNT] = {};   // clone rows per format, built when first needed
    mcpd::host::Launch *single = nullptr;      // workspace of mcpd_run_unbiased
    // design as CSR on the device, for the feature kernels (built when first needed)
    int32_t *d_row_ptr = nullptr, *d_pool_idx = nullptr, *d_pool_size = nullptr;
    uint8_t *d_y = nullptr;
};
