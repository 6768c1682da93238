// Device-side finish of a run: marginals and standard errors from the
// integer N* sums (the aggregate of Section "Coupled Estimator and
// Fixed-Budget GPU Execution"), for runs whose outputs stay in device memory.

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mcpd_device.h"

namespace mcpd {

// Marginals and standard errors on the device from the integer sums, one
// clone per thread: with A_pj = V_pj / (W N*_p),
//   marginal_j = (1/P) sum_p A_pj = (1/(P W)) sum_r S1[r][j] / (r+1),
//   sum_p A_pj^2 = (1/W^2) sum_r S2[r][j] / (r+1)^2 (S2 from its three limbs),
//   SE_j = sqrt(((sum A^2) - (sum A)^2 / P) / (P - 1) / P), NaN when P = 1.
__global__ void finish_kernel(const int64_t *S1, const uint64_t *S2, uint32_t n, uint32_t nb, uint32_t P,
                              uint32_t W, double *marginals, double *stderr_out)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double sa = 0.0, sq = 0.0;
    for (uint32_t r = 0; r < nb; ++r) {
        const size_t idx = (size_t)r * n + j;
        const double nn = (double)(r + 1u);
        sa += (double)S1[idx] / nn;
        const double v2 = (double)S2[3 * idx + 2] * 18446744073709551616.0 + (double)S2[3 * idx + 1] * 4294967296.0 +
                          (double)S2[3 * idx];
        sq += v2 / (nn * nn);
    }
    const double w = (double)W, p = (double)P;
    if (marginals) marginals[j] = sa / (p * w);
    if (stderr_out) {
        if (P > 1u) {
            const double sumA = sa / w, sumA2 = sq / (w * w);
            double var = (sumA2 - sumA * sumA / p) / (p - 1.0);
            if (var < 0.0) var = 0.0;
            stderr_out[j] = sqrt(var / p);
        } else {
            stderr_out[j] = __builtin_nan("");
        }
    }
}

int launch_finish(const int64_t *S1, const uint64_t *S2, uint32_t n, uint32_t nb, uint32_t P, uint32_t W,
                  double *marginals, double *stderr_out, void *stream)
{
    hipLaunchKernelGGL(finish_kernel, dim3((n + 255u) / 256u), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       S1, S2, n, nb, P, W, marginals, stderr_out);
    return (int)hipGetLastError();
}

}  // namespace mcpd
