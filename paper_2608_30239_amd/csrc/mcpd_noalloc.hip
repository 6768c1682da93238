// Allocation-free variant of mcpd_run_unbiased_dev, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// Every device buffer of the run (output block, key, descriptors, tickets,
// numerator rows, touched lists, statistics rows) is carved from one
// file-scope device array, `scratch`, of MCPD_NOALLOC_SCRATCH_BYTES.  Each
// device the library runs this entry point on holds its own copy of the
// array until the process ends.  Its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and kept; host code
// only ever passes that address, never the array's name, whose host-side
// value is a stand-in and not a device address.
//
// The array keeps whatever the last call left in it, so each call clears
// what must start at zero (the output block and the numerator rows, with a
// fill kernel) and uploads its descriptors again.  Calls that overlap on one
// device race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#pragma GCC visibility push(default)
#include "../../include/mcpd.h"
#pragma GCC visibility pop
#include "mcpd_internal.h"

namespace {

static __device__ __align__(256) uint8_t scratch[MCPD_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_lock;
void *g_scratch[MAX_DEVICES] = {};

// The device address of `scratch` on `device`, looked up on first use with
// that device current (each device holds its own copy at its own address).
int scratch_on(int device, void **out)
{
    using mcpd::host::fail;
    using mcpd::host::hip_fail;
    if (device < 0 || device >= MAX_DEVICES) return fail(MCPD_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> hold(g_lock);
    if (!g_scratch[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(MCPD_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return MCPD_OK;
}

}  // namespace

extern "C" int mcpd_run_unbiased_dev_noalloc(mcpd_instance *inst, uint64_t budget, uint32_t slots, uint32_t k,
                                             uint32_t m, uint64_t seed, const mcpd_run_opts *opts,
                                             double *marginals_dev, double *stderr_dev, uint64_t *hist_dev,
                                             mcpd_run_stats *stats)
{
    using mcpd::host::fail;
    if (!inst) return fail(MCPD_EINVAL, "null instance");
    void *base = nullptr;
    int rc = scratch_on(inst->device, &base);
    if (rc) return rc;
    return mcpd::host::run_single_arena(inst, budget, slots, k, m, seed, opts, marginals_dev, stderr_dev, hist_dev,
                                        stats, base, (size_t)MCPD_NOALLOC_SCRATCH_BYTES);
}
