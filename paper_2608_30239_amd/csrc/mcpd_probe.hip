// Peak-rate probes of the two on-chip resources the sampler can be bound by:
// LDS read bandwidth and 32-bit vector (VALU) issue.  The roofline the
// library's benchmark reports divides achieved rates by these measured
// peaks, not by figures assumed from other chips.
//
// Every probe launches eight workgroups of 256 lanes per compute unit (as
// many run at once as fit; the rest follow), runs a fixed loop of
// independent operations, and folds what it loaded or computed into one
// word per lane so that nothing is dead code.  The rate is the whole
// launch's work over its event-timed duration.  Thread 0 of each workgroup
// reads the shader clock counter (s_memtime) and the constant-rate counter
// (s_memrealtime) around its loop; their ratio gives the clock the probe
// actually ran at, which turns the rate into work per CU per clock.
//
// LDS probes read a 32 KB buffer (five workgroups fit a 160 KB CU):
//   * streaming b32/b64/b128: lane l of a wavefront reads element
//     base + l + 64 u, so the 64 lanes of one read touch consecutive words
//     (no bank conflicts);
//   * random b32: each lane reads 16 fixed pseudo-random words, the pattern
//     of the sampler's table and count reads.
// An empty asm statement with a memory clobber ends each iteration, so the
// compiler reloads every word instead of hoisting the reads.
//
// VALU probes run 8 independent chains per lane of one operation: add,
// 32x32 low product, 32x32 high product, three-input xor (v_bitop3), the
// 64-bit product of two 32-bit words, and whole Philox4x32-10 blocks as the
// sampler computes them.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#pragma GCC visibility push(default)
#include "../../include/mcpd.h"
#pragma GCC visibility pop
#include "mcpd_internal.h"

namespace {

constexpr uint32_t PROBE_WG = 256;
constexpr uint32_t PROBE_WG_PER_CU = 8;
constexpr uint32_t LDS_WORDS = 8192;   // 32 KB per workgroup
constexpr int UNROLL = 16;

struct Clocks {
    unsigned long long t0, t1, r0, r1;
};

__device__ __forceinline__ void clock_start(Clocks *c)
{
    if (threadIdx.x == 0) {
        c[blockIdx.x].t0 = __builtin_amdgcn_s_memtime();
        c[blockIdx.x].r0 = __builtin_amdgcn_s_memrealtime();
    }
}

__device__ __forceinline__ void clock_end(Clocks *c)
{
    if (threadIdx.x == 0) {
        c[blockIdx.x].t1 = __builtin_amdgcn_s_memtime();
        c[blockIdx.x].r1 = __builtin_amdgcn_s_memrealtime();
    }
}

__device__ __forceinline__ uint32_t mix(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// LDS reads: W = 1, 2 or 4 words per lane per read; RANDOM picks fixed
// pseudo-random word addresses (W = 1 only).
template <int W, bool RANDOM>
__global__ void __launch_bounds__(PROBE_WG) lds_probe(uint32_t iters, uint32_t salt, uint32_t *sink, Clocks *clk)
{
    __shared__ __attribute__((aligned(16))) uint32_t buf[LDS_WORDS];
    for (uint32_t i = threadIdx.x; i < LDS_WORDS; i += PROBE_WG) buf[i] = i * 2654435761u;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t off[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        if (RANDOM) {
            uint32_t h = (threadIdx.x * 16u + (uint32_t)u + 1u) * 0x9E3779B1u;
            h ^= h >> 15;
            h *= 0x85EBCA77u;
            h ^= h >> 13;
            off[u] = h & (LDS_WORDS - 1u);
        } else {
            // one wavefront's reads stay in its quarter of the buffer; the
            // runtime salt (zero) keeps the compiler from fusing two reads
            // into one wider instruction
            off[u] = ((wave * (LDS_WORDS / 4u) / (uint32_t)W + lane + 64u * (uint32_t)u) % (LDS_WORDS / (uint32_t)W)) ^ salt;
        }
    }
    uint32_t acc = lane;
    clock_start(clk);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if constexpr (W == 1) {
                acc += buf[off[u]];
            } else if constexpr (W == 2) {
                const uint2 v = reinterpret_cast<const uint2 *>(buf)[off[u]];
                acc = mix(acc, v.x, v.y);
            } else {
                const uint4 v = reinterpret_cast<const uint4 *>(buf)[off[u]];
                acc = mix(mix(acc, v.x, v.y), v.z, v.w);
            }
        }
        asm volatile("" ::: "memory");
    }
    __syncthreads();
    clock_end(clk);
    sink[blockIdx.x * PROBE_WG + threadIdx.x] = acc;
}

constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;

enum ValuOp { OP_ADD, OP_MUL_LO, OP_MUL_HI, OP_BITOP3, OP_MUL64 };

// 8 chains per lane, each step one instruction per chain; a chain's next
// value reads its neighbour's, so the compiler cannot fold repeated steps
// (x + y + y ... into one product) while the 8 steps of a round stay
// independent.  The 64-bit product keeps a 64-bit accumulator per chain:
// z = lo(z) * y + z is one v_mad_u64_u32.
template <int OP>
__global__ void __launch_bounds__(PROBE_WG) valu_probe(uint32_t iters, uint32_t seed, uint32_t *sink, Clocks *clk)
{
    uint32_t x[8];
    uint64_t z[8];
    const uint32_t t = blockIdx.x * PROBE_WG + threadIdx.x;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        x[c] = (t + (uint32_t)c) * 0x9E3779B1u ^ seed;
        z[c] = ((uint64_t)x[c] << 32) | (seed + (uint32_t)c);
    }
    const uint32_t y = seed | 1u, w = seed * 3u + M0;
    clock_start(clk);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < UNROLL / 2; ++u) {
            uint32_t nx[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const uint32_t a = x[c], b = x[(c + 1) & 7];
                if constexpr (OP == OP_ADD) nx[c] = a + b;
                else if constexpr (OP == OP_MUL_LO) nx[c] = a * b;
                else if constexpr (OP == OP_MUL_HI) nx[c] = __umulhi(a, b);
                else if constexpr (OP == OP_BITOP3) nx[c] = __builtin_amdgcn_bitop3_b32(a, b, w, 0x96);
                else z[c] = (uint64_t)(uint32_t)z[c] * (uint64_t)y + z[c];
            }
            if constexpr (OP != OP_MUL64) {
#pragma unroll
                for (int c = 0; c < 8; ++c) x[c] = nx[c];
            }
        }
    }
    __syncthreads();
    clock_end(clk);
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc ^= x[c] ^ (uint32_t)z[c] ^ (uint32_t)(z[c] >> 32);
    sink[t] = acc;
}

// Whole Philox4x32-10 blocks, written as the sampler writes them (two
// 32x32->64 products and two three-input xors per round, key schedule on
// the scalar unit); two independent blocks per lane per iteration.
__device__ __forceinline__ void philox_block(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        const uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c[1], k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c[3], k1, 0x96);
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__global__ void __launch_bounds__(PROBE_WG) philox_probe(uint32_t iters, uint32_t seed, uint32_t *sink, Clocks *clk)
{
    const uint32_t t = blockIdx.x * PROBE_WG + threadIdx.x;
    uint32_t acc = 0;
    clock_start(clk);
    for (uint32_t it = 0; it < iters; ++it) {
        uint32_t a[4] = {2u * it, t, seed, 7u};
        uint32_t b[4] = {2u * it + 1u, t, seed, 7u};
        philox_block(a, seed, ~seed);
        philox_block(b, seed, ~seed);
        acc ^= a[0] ^ a[1] ^ a[2] ^ a[3] ^ b[0] ^ b[1] ^ b[2] ^ b[3];
    }
    __syncthreads();
    clock_end(clk);
    sink[t] = acc;
}

// Units of work per lane per iteration of each probe: bytes (LDS), lane
// operations (VALU) or Philox blocks.
double per_lane_iter(int kind)
{
    switch (kind) {
    case MCPD_PROBE_LDS_B32: return 4.0 * UNROLL;
    case MCPD_PROBE_LDS_B64: return 8.0 * UNROLL;
    case MCPD_PROBE_LDS_B128: return 16.0 * UNROLL;
    case MCPD_PROBE_LDS_B32_RANDOM: return 4.0 * UNROLL;
    case MCPD_PROBE_PHILOX10: return 2.0;
    default: return 8.0 * (UNROLL / 2);
    }
}

int launch(int kind, uint32_t grid, uint32_t iters, uint32_t *sink, Clocks *clk, hipStream_t s)
{
    const dim3 g(grid), b(PROBE_WG);
    const uint32_t seed = 0x1234567u, salt = 0u;
    switch (kind) {
    case MCPD_PROBE_LDS_B32: hipLaunchKernelGGL((lds_probe<1, false>), g, b, 0, s, iters, salt, sink, clk); break;
    case MCPD_PROBE_LDS_B64: hipLaunchKernelGGL((lds_probe<2, false>), g, b, 0, s, iters, salt, sink, clk); break;
    case MCPD_PROBE_LDS_B128: hipLaunchKernelGGL((lds_probe<4, false>), g, b, 0, s, iters, salt, sink, clk); break;
    case MCPD_PROBE_LDS_B32_RANDOM: hipLaunchKernelGGL((lds_probe<1, true>), g, b, 0, s, iters, salt, sink, clk); break;
    case MCPD_PROBE_VALU_ADD: hipLaunchKernelGGL((valu_probe<OP_ADD>), g, b, 0, s, iters, seed, sink, clk); break;
    case MCPD_PROBE_VALU_MUL_LO: hipLaunchKernelGGL((valu_probe<OP_MUL_LO>), g, b, 0, s, iters, seed, sink, clk); break;
    case MCPD_PROBE_VALU_MUL_HI: hipLaunchKernelGGL((valu_probe<OP_MUL_HI>), g, b, 0, s, iters, seed, sink, clk); break;
    case MCPD_PROBE_VALU_BITOP3: hipLaunchKernelGGL((valu_probe<OP_BITOP3>), g, b, 0, s, iters, seed, sink, clk); break;
    case MCPD_PROBE_VALU_MUL64: hipLaunchKernelGGL((valu_probe<OP_MUL64>), g, b, 0, s, iters, seed, sink, clk); break;
    case MCPD_PROBE_PHILOX10: hipLaunchKernelGGL(philox_probe, g, b, 0, s, iters, seed, sink, clk); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace

extern "C" int mcpd_probe(int kind, uint32_t iters, mcpd_probe_result *out)
{
    using mcpd::host::fail;
    if (!out || kind < 0 || kind >= MCPD_PROBE_COUNT || iters == 0)
        return fail(MCPD_EINVAL, "probe kind out of range, iters = 0 or out null");
    std::memset(out, 0, sizeof(*out));
    int dev = 0, cus = 0, wall_khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MCPD_EDEVICE, "hipGetDevice failed");
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || cus <= 0 ||
        wall_khz <= 0)
        return fail(MCPD_EDEVICE, "device attributes unavailable");
    const uint32_t grid = (uint32_t)cus * PROBE_WG_PER_CU;
    uint32_t *sink = nullptr;
    Clocks *clk = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    int rc = MCPD_EDEVICE;
    Clocks *h = new (std::nothrow) Clocks[grid];
    if (!h) return fail(MCPD_ENOMEM, "host allocation failed");
    do {
        if (hipMalloc(reinterpret_cast<void **>(&sink), (size_t)grid * PROBE_WG * 4) != hipSuccess) {
            rc = MCPD_ENOMEM;
            break;
        }
        if (hipMalloc(reinterpret_cast<void **>(&clk), (size_t)grid * sizeof(Clocks)) != hipSuccess) {
            rc = MCPD_ENOMEM;
            break;
        }
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) break;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) break;
        // one untimed launch (code load, clocks up), then the timed one
        if (launch(kind, grid, iters < 64 ? iters : 64, sink, clk, s) != hipSuccess) break;
        if (hipEventRecord(e0, s) != hipSuccess) break;
        if (launch(kind, grid, iters, sink, clk, s) != hipSuccess) break;
        if (hipEventRecord(e1, s) != hipSuccess) break;
        if (hipStreamSynchronize(s) != hipSuccess) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) break;
        if (hipMemcpy(h, clk, (size_t)grid * sizeof(Clocks), hipMemcpyDeviceToHost) != hipSuccess) break;
        double cyc = 0, real = 0;
        for (uint32_t i = 0; i < grid; ++i) {
            cyc += (double)(h[i].t1 - h[i].t0);
            real += (double)(h[i].r1 - h[i].r0);
        }
        const double wall_hz = (double)wall_khz * 1e3;
        const double work = per_lane_iter(kind) * (double)iters * PROBE_WG * (double)grid;
        out->ms = ms;
        out->clock_hz = real > 0 ? cyc / (real / wall_hz) : 0.0;
        out->per_second = ms > 0 ? work / ((double)ms * 1e-3) : 0.0;
        out->per_cu_per_clock = out->clock_hz > 0 ? out->per_second / out->clock_hz / (double)cus : 0.0;
        out->cus = (uint32_t)cus;
        rc = MCPD_OK;
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (sink) (void)hipFree(sink);
    if (clk) (void)hipFree(clk);
    delete[] h;
    if (rc == MCPD_ENOMEM) return fail(rc, "device allocation failed");
    if (rc != MCPD_OK) return fail(rc, "probe launch or timing failed");
    return rc;
}
