// Kernels of the learned selection weights: per-clone features and base
// logits (the log-weights of the score softmax), the 8-64-64-1 ReLU network
// (BF16 weights, FP32 arithmetic) whose output is added to the base logits,
// the per-instance softmax-KL loss and its gradient, the backward pass with
// a fixed-order reduction of the parameter gradient, and AdamW on the FP32
// master copy with the BF16 working copy rewritten after each step.
//
// Selection weights only have to be positive and fixed before the chains
// start for the Gibbs kernel to keep pi invariant (Proposition 1) and for
// the coupled estimator to stay unbiased (Theorem 1); the network is one way
// to choose them, with the uniform floor of the score weights.
//
// Parameter layout (flat, 4801): W1 [64][8] (out, in), b1 [64], W2 [64][64],
// b2 [64], W3 [64], b3.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mcpd_mlp.h"

namespace mcpd {
namespace mlp {
namespace {

constexpr int F = MLP_F, H = MLP_H;
constexpr int O_W1 = 0, O_B1 = O_W1 + H * F, O_W2 = O_B1 + H, O_B2 = O_W2 + H * H, O_W3 = O_B2 + H,
              O_B3 = O_W3 + H;
static_assert(O_B3 + 1 == MLP_PARAMS, "parameter layout");
constexpr int ROWS = 256;          // rows per chunk = threads per block
constexpr int LD = ROWS + 1;       // padded stride of the feature-major LDS tiles

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Nearest bfloat16 of a float32, ties to even: drop the low 16 bits and
// round the kept part up when they are above half a unit, or exactly half
// a unit with the kept part odd.
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t low = u & 0xFFFFu;
    uint32_t kept = u >> 16;
    if (low > 0x8000u || (low == 0x8000u && (kept & 1u))) kept += 1u;
    return (uint16_t)kept;
}

__device__ void load_weights(float *w, const uint16_t *wb)
{
    for (int i = threadIdx.x; i < MLP_PARAMS; i += blockDim.x) w[i] = bf16_to_f32(wb[i]);
}

// ---------------------------------------------------------------- features

__global__ void pool_size_kernel(const int32_t *pool_idx, int64_t nnz, int32_t *size)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(size + pool_idx[e], 1);
}

// Raw features of each clone and its score s_i = sum_j d_j a_j (FP64, pools
// in ascending order, starting from 0), the paper's score of
// Section "Score-Weighted Update Gibbs Sampler".
__global__ void features_raw_kernel(const int32_t *row_ptr, const int32_t *pool_idx, const uint8_t *y,
                                    const int32_t *size, int32_t n, double a_pos, double a_neg, float fp10,
                                    float fn10, double *score, float *X)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int np = 0, nn = 0, spos = 0, sneg = 0, minpos = 0x7FFFFFFF;
    double s = 0.0;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int32_t j = pool_idx[e];
        const int d = size[j];
        if (y[j]) {
            np += 1;
            spos += d;
            minpos = d < minpos ? d : minpos;
            s = s + (double)d * a_pos;
        } else {
            nn += 1;
            sneg += d;
            s = s + (double)d * a_neg;
        }
    }
    score[i] = s;
    float *x = X + (size_t)i * F;
    x[0] = (float)((double)np / 8.0);
    x[1] = (float)((double)nn / 8.0);
    x[2] = np ? (float)(((double)spos / (double)np) / 64.0) : 0.f;
    x[3] = nn ? (float)(((double)sneg / (double)nn) / 64.0) : 0.f;
    x[4] = np ? (float)((double)minpos / 64.0) : 0.f;
    x[5] = 0.f;
    x[6] = fp10;
    x[7] = fn10;
}

// One block: min and max of the scores (exact in any order), then the base
// logits c_i = tau_w (s_i - s_max), tau_w = log(100 n) / (s_max - s_min) (0
// if all scores are equal), written over the scores, and x5 = c_i / 16.
__global__ void features_norm_kernel(double *score, int32_t n, double log100n, float *X)
{
    __shared__ double smin[256], smax[256];
    double lo = INFINITY, hi = -INFINITY;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        lo = fmin(lo, score[i]);
        hi = fmax(hi, score[i]);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
        }
        __syncthreads();
    }
    lo = smin[0];
    hi = smax[0];
    const double tau = hi > lo ? log100n / (hi - lo) : 0.0;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double c = tau * (score[i] - hi);
        score[i] = c;
        X[(size_t)i * F + 5] = (float)(c / 16.0);
    }
}

// ----------------------------------------------------------------- forward

// Hidden layer 1 of one row into registers.
__device__ __forceinline__ void layer1(const float *w, const float *x, float h1[H])
{
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float a = w[O_B1 + o];
#pragma unroll
        for (int f = 0; f < F; ++f) a = __fmaf_rn(w[O_W1 + o * F + f], x[f], a);
        h1[o] = a > 0.f ? a : 0.f;
    }
}

// Pre-activation of unit o of hidden layer 2.
__device__ __forceinline__ float layer2(const float *w, const float h1[H], int o)
{
    float a = w[O_B2 + o];
#pragma unroll
    for (int i = 0; i < H; ++i) a = __fmaf_rn(w[O_W2 + o * H + i], h1[i], a);
    return a;
}

__global__ void __launch_bounds__(ROWS) forward_kernel(const uint16_t *wb, const float *X, int64_t rows, float *g)
{
    __shared__ float w[MLP_PARAMS];
    load_weights(w, wb);
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * ROWS + threadIdx.x; r < rows; r += (int64_t)gridDim.x * ROWS) {
        float x[F];
#pragma unroll
        for (int f = 0; f < F; ++f) x[f] = X[r * F + f];
        float h1[H];
        layer1(w, x, h1);
        float out = w[O_B3];
        for (int o = 0; o < H; ++o) {
            const float z = layer2(w, h1, o);
            out = __fmaf_rn(w[O_W3 + o], z > 0.f ? z : 0.f, out);
        }
        g[r] = out;
    }
}

// -------------------------------------------------------------------- loss

// One block per instance segment [seg_ptr[s], seg_ptr[s+1]), with base
// logits c and network outputs f:
//   t_i = exp(beta c_i) (u_i + eps)^gamma / sum, u = clip(signal, 0, 1)
//   p = softmax(c + f), loss_s = sum t (log t - log p), df = (p - t) / S.
// Reductions in FP64 over a fixed tree.
__device__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

__device__ double block_max(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

__device__ __forceinline__ double target_raw(double p, double c, double beta, double gamma, double eps)
{
    const double u = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
    return exp(beta * c) * pow(u + eps, gamma);
}

__global__ void __launch_bounds__(256) loss_kernel(const float *f, const double *base, const double *signal,
                                                   const int64_t *seg_ptr, int32_t nseg, double beta, double gamma,
                                                   double eps, double *seg_loss, float *dg)
{
    __shared__ double sh[256];
    const int s = blockIdx.x;
    const int64_t a = seg_ptr[s], b = seg_ptr[s + 1];
    double mx = -INFINITY, tsum = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
        mx = fmax(mx, base[i] + (double)f[i]);
        tsum += target_raw(signal[i], base[i], beta, gamma, eps);
    }
    mx = block_max(mx, sh);
    tsum = block_sum(tsum, sh);
    double z = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) z += exp(base[i] + (double)f[i] - mx);
    z = block_sum(z, sh);
    const double logz = log(z);
    double l = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) {
        const double t = target_raw(signal[i], base[i], beta, gamma, eps) / tsum;
        const double lp = base[i] + (double)f[i] - mx - logz;
        l += t * (log(t) - lp);
        dg[i] = (float)((exp(lp) - t) / (double)nseg);
    }
    l = block_sum(l, sh);
    if (threadIdx.x == 0) seg_loss[s] = l;
}

// ---------------------------------------------------------------- backward

// Each block takes chunks of 256 rows (one per thread) and accumulates its
// share of the parameter gradient in registers, every entry owned by one
// thread and summed over rows in ascending order.  Per chunk:
//   A  own row: h1 -> H1 tile, h2 -> BUF tile, x -> XS tile, dg -> DG
//   B  dW3[o] = sum_r dg_r h2[o][r]
//   C  own row: dz2[o] = dg W3[o] 1{z2 > 0} -> BUF
//   D  dW2[o][i] = sum_r dz2[o][r] h1[i][r], db2[o] = sum_r dz2[o][r]
//   E  own row: dz1[i] = 1{h1 > 0} sum_o W2[o][i] dz2[o] -> H1
//   F  dW1[o][f] = sum_r dz1[o][r] x[f][r], db1[o] = sum_r dz1[o][r]
// and writes its partial gradient to part[block] at the end.
__global__ void __launch_bounds__(ROWS) backward_kernel(const uint16_t *wb, const float *X, const float *dgv,
                                                        int64_t rows, int64_t rows_per_block, float *part)
{
    extern __shared__ float smem[];
    float *w = smem;                       // [MLP_PARAMS]
    float *H1 = w + MLP_PARAMS;            // [H][LD]
    float *BUF = H1 + H * LD;              // [H][LD]
    float *XS = BUF + H * LD;              // [F][LD]
    float *DG = XS + F * LD;               // [ROWS]
    const int tid = threadIdx.x;
    load_weights(w, wb);

    // ownership: thread tid owns dW2 rows o2 = tid / 4, columns i2.. i2+15
    const int o2 = tid >> 2, i2 = (tid & 3) * 16;
    // thread tid owns dW1[o1][f1], dW1[o1][f1 + 4]
    const int o1 = tid >> 2, f1 = tid & 3;
    float aW2[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) aW2[q] = 0.f;
    float aW1a = 0.f, aW1b = 0.f, aW3 = 0.f, aB2 = 0.f, aB1 = 0.f, aB3 = 0.f;

    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = std::min<int64_t>(rows, r0 + rows_per_block);
    __syncthreads();
    for (int64_t c0 = r0; c0 < r1; c0 += ROWS) {
        const int64_t r = c0 + tid;
        const bool live = r < r1;
        // A
        float x[F];
#pragma unroll
        for (int f = 0; f < F; ++f) x[f] = live ? X[r * F + f] : 0.f;
        const float dg = live ? dgv[r] : 0.f;
        float h1[H];
        layer1(w, x, h1);
        uint64_t mask2 = 0;
        for (int o = 0; o < H; ++o) {
            const float z = layer2(w, h1, o);
            BUF[o * LD + tid] = z > 0.f ? z : 0.f;
            mask2 |= (uint64_t)(z > 0.f) << o;
        }
#pragma unroll
        for (int i = 0; i < H; ++i) H1[i * LD + tid] = h1[i];
#pragma unroll
        for (int f = 0; f < F; ++f) XS[f * LD + tid] = x[f];
        DG[tid] = dg;
        __syncthreads();
        // B
        if (tid < H) {
            float a = aW3;
            for (int q = 0; q < ROWS; ++q) a = __fmaf_rn(DG[q], BUF[tid * LD + q], a);
            aW3 = a;
        } else if (tid == H) {
            float a = aB3;
            for (int q = 0; q < ROWS; ++q) a += DG[q];
            aB3 = a;
        }
        __syncthreads();
        // C
        for (int o = 0; o < H; ++o) BUF[o * LD + tid] = ((mask2 >> o) & 1u) ? dg * w[O_W3 + o] : 0.f;
        __syncthreads();
        // D
        for (int q = 0; q < ROWS; ++q) {
            const float d = BUF[o2 * LD + q];
#pragma unroll
            for (int c = 0; c < 16; ++c) aW2[c] = __fmaf_rn(d, H1[(i2 + c) * LD + q], aW2[c]);
        }
        if (tid < H) {
            float a = aB2;
            for (int q = 0; q < ROWS; ++q) a += BUF[tid * LD + q];
            aB2 = a;
        }
        __syncthreads();
        // E (h1 of the own row is read back from its tile and replaced)
        for (int i = 0; i < H; ++i) {
            float a = 0.f;
            for (int o = 0; o < H; ++o) a = __fmaf_rn(w[O_W2 + o * H + i], BUF[o * LD + tid], a);
            const float hv = H1[i * LD + tid];
            H1[i * LD + tid] = hv > 0.f ? a : 0.f;
        }
        __syncthreads();
        // F
        {
            float a = aW1a, b = aW1b;
            for (int q = 0; q < ROWS; ++q) {
                const float d = H1[o1 * LD + q];
                a = __fmaf_rn(d, XS[f1 * LD + q], a);
                b = __fmaf_rn(d, XS[(f1 + 4) * LD + q], b);
            }
            aW1a = a;
            aW1b = b;
        }
        if (tid < H) {
            float a = aB1;
            for (int q = 0; q < ROWS; ++q) a += H1[tid * LD + q];
            aB1 = a;
        }
        __syncthreads();
    }
    float *p = part + (size_t)blockIdx.x * MLP_PARAMS;
#pragma unroll
    for (int c = 0; c < 16; ++c) p[O_W2 + o2 * H + i2 + c] = aW2[c];
    p[O_W1 + o1 * F + f1] = aW1a;
    p[O_W1 + o1 * F + f1 + 4] = aW1b;
    if (tid < H) {
        p[O_W3 + tid] = aW3;
        p[O_B2 + tid] = aB2;
        p[O_B1 + tid] = aB1;
    }
    if (tid == H) p[O_B3] = aB3;
}

// grad[k] = sum over blocks (ascending) of part[block][k].
__global__ void reduce_kernel(const float *part, int nblocks, float *grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_PARAMS) return;
    float a = 0.f;
    for (int b = 0; b < nblocks; ++b) a += part[(size_t)b * MLP_PARAMS + k];
    grad[k] = a;
}

// ------------------------------------------------------------------- AdamW

// One AdamW step on the FP32 master copy (decoupled weight decay on every
// parameter); bc1 = 1 - beta1^t and bc2 = 1 - beta2^t come from the host.
__global__ void adamw_kernel(float *theta, float *m, float *v, const float *grad, uint16_t *wb, float lr,
                             float beta1, float beta2, float eps, float wd, float bc1, float bc2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= MLP_PARAMS) return;
    const float gk = grad[k];
    const float mk = beta1 * m[k] + (1.f - beta1) * gk;
    const float vk = beta2 * v[k] + (1.f - beta2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / bc1, vh = vk / bc2;
    const float th = theta[k] - lr * (mh / (sqrtf(vh) + eps) + wd * theta[k]);
    theta[k] = th;
    wb[k] = f32_to_bf16(th);
}

__global__ void cast_kernel(const float *theta, uint16_t *wb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < MLP_PARAMS) wb[k] = f32_to_bf16(theta[k]);
}

int grid_for(int64_t n, int block, int cap)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, cap));
}

}  // namespace

int launch_pool_size(const int32_t *pool_idx, int64_t nnz, int32_t *size, hipStream_t s)
{
    hipLaunchKernelGGL(pool_size_kernel, dim3(grid_for(nnz, 256, 4096)), dim3(256), 0, s, pool_idx, nnz, size);
    return (int)hipGetLastError();
}

int launch_features(const int32_t *row_ptr, const int32_t *pool_idx, const uint8_t *y, const int32_t *size,
                    int32_t n, double a_pos, double a_neg, double log100n, float fp10, float fn10, double *base,
                    float *X, hipStream_t s)
{
    hipLaunchKernelGGL(features_raw_kernel, dim3(grid_for(n, 256, 1 << 20)), dim3(256), 0, s, row_ptr, pool_idx,
                       y, size, n, a_pos, a_neg, fp10, fn10, base, X);
    hipLaunchKernelGGL(features_norm_kernel, dim3(1), dim3(256), 0, s, base, n, log100n, X);
    return (int)hipGetLastError();
}

int launch_forward(const uint16_t *wb, const float *X, int64_t rows, float *g, int cus, hipStream_t s)
{
    hipLaunchKernelGGL(forward_kernel, dim3(grid_for(rows, ROWS, 8 * cus)), dim3(ROWS), 0, s, wb, X, rows, g);
    return (int)hipGetLastError();
}

int launch_loss(const float *f, const double *base, const double *signal, const int64_t *seg_ptr, int32_t nseg,
                double beta, double gamma, double eps, double *seg_loss, float *df, hipStream_t s)
{
    hipLaunchKernelGGL(loss_kernel, dim3(nseg), dim3(256), 0, s, f, base, signal, seg_ptr, nseg, beta, gamma, eps,
                       seg_loss, df);
    return (int)hipGetLastError();
}

size_t backward_lds_bytes() { return (size_t)(MLP_PARAMS + 2 * H * LD + F * LD + ROWS) * sizeof(float); }

int backward_blocks(int64_t rows, int cus, int64_t *rows_per_block)
{
    // about one block per CU, each a whole number of 256-row chunks
    const int64_t chunks = (rows + ROWS - 1) / ROWS;
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(chunks, cus));
    const int64_t per = (chunks + nb - 1) / nb;
    *rows_per_block = per * ROWS;
    return (int)((chunks + per - 1) / per);
}

int launch_backward(const uint16_t *wb, const float *X, const float *dg, int64_t rows, int nblocks,
                    int64_t rows_per_block, float *part, float *grad, hipStream_t s)
{
    const size_t lds = backward_lds_bytes();
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(backward_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(backward_kernel, dim3(nblocks), dim3(ROWS), lds, s, wb, X, dg, rows, rows_per_block, part);
    hipLaunchKernelGGL(reduce_kernel, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, s, part, nblocks, grad);
    return (int)hipGetLastError();
}

int launch_adamw(float *theta, float *m, float *v, const float *grad, uint16_t *wb, float lr, float beta1,
                 float beta2, float eps, float wd, float bc1, float bc2, hipStream_t s)
{
    hipLaunchKernelGGL(adamw_kernel, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, s, theta, m, v, grad, wb, lr,
                       beta1, beta2, eps, wd, bc1, bc2);
    return (int)hipGetLastError();
}

int launch_cast(const float *theta, uint16_t *wb, hipStream_t s)
{
    hipLaunchKernelGGL(cast_kernel, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, s, theta, wb);
    return (int)hipGetLastError();
}

}  // namespace mlp
}  // namespace mcpd

namespace mcpd {
namespace mlp {
namespace {

// out[0] = scale * sum of v (one block, fixed tree order).
__global__ void sum_kernel(const double *v, int n, double scale, double *out)
{
    __shared__ double sh[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) a += v[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] * scale;
}

}  // namespace

int launch_sum(const double *v, int n, double scale, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, v, n, scale, out);
    return (int)hipGetLastError();
}

}  // namespace mlp
}  // namespace mcpd
