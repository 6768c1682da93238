// Internal launchers of the learned-weights kernels (mcpd_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mcpd {
namespace mlp {

constexpr int MLP_F = 8;         // features per clone
constexpr int MLP_H = 64;        // hidden width
constexpr int MLP_PARAMS = MLP_H * MLP_F + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;   // 4801

// size[j] += 1 for every design entry (size zeroed by the caller).
int launch_pool_size(const int32_t *pool_idx, int64_t nnz, int32_t *size, hipStream_t s);
// Features [n][8] and FP64 base logits of one instance.
int launch_features(const int32_t *row_ptr, const int32_t *pool_idx, const uint8_t *y, const int32_t *size,
                    int32_t n, double a_pos, double a_neg, double log100n, float fp10, float fn10, double *base,
                    float *X, hipStream_t s);
// g[r] for rows of X with the BF16 parameters wb.
int launch_forward(const uint16_t *wb, const float *X, int64_t rows, float *g, int cus, hipStream_t s);
// Per-segment loss and dg (see the kernel).
int launch_loss(const float *f, const double *base, const double *signal, const int64_t *seg_ptr, int32_t nseg,
                double beta, double gamma, double eps, double *seg_loss, float *df, hipStream_t s);
// Blocks of the backward pass and the rows each takes.
int backward_blocks(int64_t rows, int cus, int64_t *rows_per_block);
// Parameter gradient of sum_r dg_r g_r (part: [nblocks][MLP_PARAMS] scratch).
int launch_backward(const uint16_t *wb, const float *X, const float *dg, int64_t rows, int nblocks,
                    int64_t rows_per_block, float *part, float *grad, hipStream_t s);
int launch_adamw(float *theta, float *m, float *v, const float *grad, uint16_t *wb, float lr, float beta1,
                 float beta2, float eps, float wd, float bc1, float bc2, hipStream_t s);
// out[0] = scale * sum of v[0..n)
int launch_sum(const double *v, int n, double scale, double *out, hipStream_t s);
// wb = bf16(theta)
int launch_cast(const float *theta, uint16_t *wb, hipStream_t s);

}  // namespace mlp
}  // namespace mcpd
