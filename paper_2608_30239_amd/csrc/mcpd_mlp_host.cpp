// Host side of the learned-weights C ABI (include/mcpd.h): device buffers
// of the network, the training set and the optimiser, and the sequence of
// kernels of each call (mcpd_mlp.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#pragma GCC visibility push(default)
#include "../../include/mcpd.h"
#pragma GCC visibility pop

#include "mcpd_internal.h"
#include "mcpd_mlp.h"

using mcpd::host::fail;
using mcpd::host::hip_fail;
namespace K = mcpd::mlp;

static_assert(K::MLP_PARAMS == MCPD_MLP_PARAMS, "parameter count");
static_assert(K::MLP_F == MCPD_MLP_FEATURES && K::MLP_H == MCPD_MLP_HIDDEN, "network shape");

namespace {

template <typename T>
int dev_alloc(T **p, size_t count)
{
    *p = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipErrorOutOfMemory) return fail(MCPD_ENOMEM, "device allocation failed");
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    return MCPD_OK;
}

template <typename T>
void dev_free(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

// The design of an instance as CSR on the device, and its pool sizes.
int ensure_device_csr(mcpd_instance *I)
{
    if (I->d_pool_size) return MCPD_OK;
    const size_t nnz = I->pool_idx.size();
    int rc;
    if ((rc = dev_alloc(&I->d_row_ptr, (size_t)I->n + 1)) || (rc = dev_alloc(&I->d_pool_idx, nnz)) ||
        (rc = dev_alloc(&I->d_y, (size_t)I->m)) || (rc = dev_alloc(&I->d_pool_size, (size_t)I->m)))
        return rc;
    HIP_TRY(hipMemcpyAsync(I->d_row_ptr, I->row_ptr.data(), ((size_t)I->n + 1) * 4, hipMemcpyHostToDevice, I->stream));
    HIP_TRY(hipMemcpyAsync(I->d_pool_idx, I->pool_idx.data(), nnz * 4, hipMemcpyHostToDevice, I->stream));
    HIP_TRY(hipMemcpyAsync(I->d_y, I->y.data(), (size_t)I->m, hipMemcpyHostToDevice, I->stream));
    HIP_TRY(hipMemsetAsync(I->d_pool_size, 0, (size_t)I->m * 4, I->stream));
    int e = K::launch_pool_size(I->d_pool_idx, (int64_t)nnz, I->d_pool_size, I->stream);
    if (e != hipSuccess) return hip_fail((hipError_t)e, "pool sizes");
    HIP_TRY(hipStreamSynchronize(I->stream));
    return MCPD_OK;
}

// Features of an instance into device rows X (n * 8 floats) and its base
// logits into device base (n doubles), on stream s.
int device_features(mcpd_instance *I, float *X, double *base, hipStream_t s)
{
    int rc = ensure_device_csr(I);
    if (rc) return rc;
    const double a_pos = std::log(1.0 - I->fn) - std::log(I->fp);
    const double a_neg = std::log(I->fn) - std::log(1.0 - I->fp);
    const double log100n = std::log(100.0 * (double)I->n);
    int e = K::launch_features(I->d_row_ptr, I->d_pool_idx, I->d_y, I->d_pool_size, I->n, a_pos, a_neg, log100n,
                               (float)(10.0 * I->fp), (float)(10.0 * I->fn), base, X, s);
    if (e != hipSuccess) return hip_fail((hipError_t)e, "feature kernels");
    HIP_TRY(hipStreamSynchronize(s));
    return MCPD_OK;
}

bool finite_params(const float *p)
{
    for (int k = 0; k < MCPD_MLP_PARAMS; ++k)
        if (!std::isfinite(p[k])) return false;
    return true;
}

}  // namespace

struct mcpd_mlp {
    hipStream_t stream = nullptr;
    int device = 0, cus = 0;
    float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr;
    uint16_t *d_wb = nullptr;
    int64_t step = 0;
    // training set
    float *d_X = nullptr;
    double *d_base = nullptr, *d_signal = nullptr;
    int64_t *d_seg = nullptr;
    int32_t nseg = 0;
    int64_t rows = 0;
    double beta = 1.0, gamma = 0.0, eps = 1e-3;
    float *d_g = nullptr, *d_dg = nullptr, *d_part = nullptr;
    double *d_seg_loss = nullptr, *d_loss = nullptr;
    int nblocks = 0;
    int64_t rows_per_block = 0;

    void drop_data()
    {
        dev_free(d_X); dev_free(d_base); dev_free(d_signal); dev_free(d_seg); dev_free(d_g); dev_free(d_dg);
        dev_free(d_part); dev_free(d_seg_loss); dev_free(d_loss);
        rows = 0;
        nseg = 0;
    }
    ~mcpd_mlp()
    {
        (void)hipStreamSynchronize(stream);
        drop_data();
        dev_free(d_theta); dev_free(d_m); dev_free(d_v); dev_free(d_grad); dev_free(d_wb);
    }
};

namespace {

int upload_params(mcpd_mlp *M, const float *params)
{
    HIP_TRY(hipMemcpyAsync(M->d_theta, params, MCPD_MLP_PARAMS * 4, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemsetAsync(M->d_m, 0, MCPD_MLP_PARAMS * 4, M->stream));
    HIP_TRY(hipMemsetAsync(M->d_v, 0, MCPD_MLP_PARAMS * 4, M->stream));
    int e = K::launch_cast(M->d_theta, M->d_wb, M->stream);
    if (e != hipSuccess) return hip_fail((hipError_t)e, "cast kernel");
    HIP_TRY(hipStreamSynchronize(M->stream));
    M->step = 0;
    return MCPD_OK;
}

// Allocate the training buffers for `rows` rows in `nseg` segments.
int alloc_data(mcpd_mlp *M, int64_t rows, int32_t nseg)
{
    M->drop_data();
    int rc;
    if ((rc = dev_alloc(&M->d_X, (size_t)rows * MCPD_MLP_FEATURES)) || (rc = dev_alloc(&M->d_signal, (size_t)rows)) ||
        (rc = dev_alloc(&M->d_base, (size_t)rows)) ||
        (rc = dev_alloc(&M->d_seg, (size_t)nseg + 1)) || (rc = dev_alloc(&M->d_g, (size_t)rows)) ||
        (rc = dev_alloc(&M->d_dg, (size_t)rows)) || (rc = dev_alloc(&M->d_seg_loss, (size_t)nseg)) ||
        (rc = dev_alloc(&M->d_loss, (size_t)1)))
        return rc;
    M->nblocks = K::backward_blocks(rows, M->cus, &M->rows_per_block);
    if ((rc = dev_alloc(&M->d_part, (size_t)M->nblocks * MCPD_MLP_PARAMS))) return rc;
    M->rows = rows;
    M->nseg = nseg;
    return MCPD_OK;
}

int check_hp(double beta, double gamma, double eps)
{
    if (!(beta >= 0.0 && gamma >= 0.0) || !std::isfinite(beta) || !std::isfinite(gamma))
        return fail(MCPD_EINVAL, "target exponents must be finite and >= 0");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(MCPD_EINVAL, "eps must be > 0");
    return MCPD_OK;
}

// forward, loss and backward over the training set: M->d_grad and the loss
// (scaled mean over segments) in M->d_loss.
int loss_grad_device(mcpd_mlp *M, double *loss_dst)
{
    int e = K::launch_forward(M->d_wb, M->d_X, M->rows, M->d_g, M->cus, M->stream);
    if (e == hipSuccess)
        e = K::launch_loss(M->d_g, M->d_base, M->d_signal, M->d_seg, M->nseg, M->beta, M->gamma, M->eps,
                           M->d_seg_loss, M->d_dg, M->stream);
    if (e == hipSuccess) e = K::launch_sum(M->d_seg_loss, M->nseg, 1.0 / M->nseg, loss_dst, M->stream);
    if (e == hipSuccess)
        e = K::launch_backward(M->d_wb, M->d_X, M->d_dg, M->rows, M->nblocks, M->rows_per_block, M->d_part,
                               M->d_grad, M->stream);
    if (e != hipSuccess) return hip_fail((hipError_t)e, "training kernels");
    return MCPD_OK;
}

}  // namespace

extern "C" {

int mcpd_features(mcpd_instance *I, float *out, double *base_out)
{
    if (!I || !out) return fail(MCPD_EINVAL, "null argument");
    float *X = nullptr;
    double *base = nullptr;
    int rc = dev_alloc(&X, (size_t)I->n * MCPD_MLP_FEATURES);
    if (!rc) rc = dev_alloc(&base, (size_t)I->n);
    if (!rc) rc = device_features(I, X, base, I->stream);
    if (!rc) {
        hipError_t e = hipMemcpy(out, X, (size_t)I->n * MCPD_MLP_FEATURES * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && base_out) e = hipMemcpy(base_out, base, (size_t)I->n * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy");
    }
    dev_free(X);
    dev_free(base);
    return rc;
}

int mcpd_mlp_create(const float *params, void *hip_stream, mcpd_mlp **out)
{
    if (!out) return fail(MCPD_EINVAL, "out is null");
    *out = nullptr;
    if (!params || !finite_params(params)) return fail(MCPD_EINVAL, "parameters must be given and finite");
    std::unique_ptr<mcpd_mlp> M(new (std::nothrow) mcpd_mlp());
    if (!M) return fail(MCPD_ENOMEM, "host allocation failed");
    M->stream = reinterpret_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipGetDevice(&M->device));
    HIP_TRY(hipDeviceGetAttribute(&M->cus, hipDeviceAttributeMultiprocessorCount, M->device));
    int rc;
    if ((rc = dev_alloc(&M->d_theta, MCPD_MLP_PARAMS)) || (rc = dev_alloc(&M->d_m, MCPD_MLP_PARAMS)) ||
        (rc = dev_alloc(&M->d_v, MCPD_MLP_PARAMS)) || (rc = dev_alloc(&M->d_grad, MCPD_MLP_PARAMS)) ||
        (rc = dev_alloc(&M->d_wb, MCPD_MLP_PARAMS)))
        return rc;
    if ((rc = upload_params(M.get(), params))) return rc;
    *out = M.release();
    return MCPD_OK;
}

int mcpd_mlp_get_params(const mcpd_mlp *M, float *master, uint16_t *bf16)
{
    if (!M) return fail(MCPD_EINVAL, "null network");
    if (master) HIP_TRY(hipMemcpyAsync(master, M->d_theta, MCPD_MLP_PARAMS * 4, hipMemcpyDeviceToHost, M->stream));
    if (bf16) HIP_TRY(hipMemcpyAsync(bf16, M->d_wb, MCPD_MLP_PARAMS * 2, hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    return MCPD_OK;
}

int mcpd_mlp_set_params(mcpd_mlp *M, const float *master)
{
    if (!M) return fail(MCPD_EINVAL, "null network");
    if (!master || !finite_params(master)) return fail(MCPD_EINVAL, "parameters must be given and finite");
    return upload_params(M, master);
}

int mcpd_mlp_forward(mcpd_mlp *M, const float *x, int64_t rows, float *g)
{
    if (!M || !x || !g || rows < 0) return fail(MCPD_EINVAL, "bad argument");
    if (rows == 0) return MCPD_OK;
    float *dX = nullptr, *dg = nullptr;
    int rc = dev_alloc(&dX, (size_t)rows * MCPD_MLP_FEATURES);
    if (!rc) rc = dev_alloc(&dg, (size_t)rows);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(dX, x, (size_t)rows * MCPD_MLP_FEATURES * 4, hipMemcpyHostToDevice, M->stream);
        if (e == hipSuccess) e = (hipError_t)K::launch_forward(M->d_wb, dX, rows, dg, M->cus, M->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(g, dg, (size_t)rows * 4, hipMemcpyDeviceToHost, M->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
        if (e != hipSuccess) rc = hip_fail(e, "forward");
    }
    dev_free(dX);
    dev_free(dg);
    return rc;
}

int mcpd_mlp_set_training_rows(mcpd_mlp *M, const float *x, const double *base, const double *signal, int64_t rows,
                               const int64_t *seg_ptr, int32_t nseg, double beta, double gamma, double eps)
{
    if (!M || !x || !base || !signal || !seg_ptr || rows <= 0 || nseg <= 0) return fail(MCPD_EINVAL, "bad argument");
    int rc = check_hp(beta, gamma, eps);
    if (rc) return rc;
    if (seg_ptr[0] != 0 || seg_ptr[nseg] != rows) return fail(MCPD_EINVAL, "segments must cover the rows");
    for (int32_t s = 0; s < nseg; ++s)
        if (seg_ptr[s + 1] <= seg_ptr[s]) return fail(MCPD_EINVAL, "empty or decreasing segment");
    for (int64_t r = 0; r < rows; ++r)
        if (!std::isfinite(signal[r]) || !std::isfinite(base[r]) || base[r] > 0.0)
            return fail(MCPD_EINVAL, "signal must be finite and base finite and <= 0");
    if ((rc = alloc_data(M, rows, nseg))) return rc;
    M->beta = beta;
    M->gamma = gamma;
    M->eps = eps;
    HIP_TRY(hipMemcpyAsync(M->d_X, x, (size_t)rows * MCPD_MLP_FEATURES * 4, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(M->d_signal, signal, (size_t)rows * 8, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(M->d_base, base, (size_t)rows * 8, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(M->d_seg, seg_ptr, ((size_t)nseg + 1) * 8, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    return MCPD_OK;
}

int mcpd_mlp_set_training_data(mcpd_mlp *M, mcpd_instance *const *insts, const double *const *signal,
                               int32_t count, double beta, double gamma, double eps)
{
    if (!M || !insts || !signal || count <= 0) return fail(MCPD_EINVAL, "bad argument");
    int rc = check_hp(beta, gamma, eps);
    if (rc) return rc;
    std::vector<int64_t> seg((size_t)count + 1, 0);
    for (int32_t i = 0; i < count; ++i) {
        if (!insts[i] || !signal[i]) return fail(MCPD_EINVAL, "null instance or signal");
        seg[i + 1] = seg[i] + insts[i]->n;
        for (int32_t j = 0; j < insts[i]->n; ++j)
            if (!std::isfinite(signal[i][j])) return fail(MCPD_EINVAL, "signal must be finite");
    }
    const int64_t rows = seg[count];
    if ((rc = alloc_data(M, rows, count))) return rc;
    M->beta = beta;
    M->gamma = gamma;
    M->eps = eps;
    for (int32_t i = 0; i < count; ++i) {
        if ((rc = device_features(insts[i], M->d_X + seg[i] * MCPD_MLP_FEATURES, M->d_base + seg[i], M->stream)))
            return rc;
        HIP_TRY(hipMemcpyAsync(M->d_signal + seg[i], signal[i], (size_t)insts[i]->n * 8, hipMemcpyHostToDevice,
                               M->stream));
    }
    HIP_TRY(hipMemcpyAsync(M->d_seg, seg.data(), seg.size() * 8, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    return MCPD_OK;
}

int mcpd_mlp_loss_grad(mcpd_mlp *M, double *loss, float *grad)
{
    if (!M) return fail(MCPD_EINVAL, "null network");
    if (!M->rows) return fail(MCPD_EINVAL, "no training set");
    int rc = loss_grad_device(M, M->d_loss);
    if (rc) return rc;
    if (loss) HIP_TRY(hipMemcpyAsync(loss, M->d_loss, 8, hipMemcpyDeviceToHost, M->stream));
    if (grad) HIP_TRY(hipMemcpyAsync(grad, M->d_grad, MCPD_MLP_PARAMS * 4, hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    return MCPD_OK;
}

int mcpd_mlp_train(mcpd_mlp *M, int32_t steps, const mcpd_adamw *hp, double *loss_history)
{
    if (!M || !hp || steps < 0) return fail(MCPD_EINVAL, "bad argument");
    if (!M->rows) return fail(MCPD_EINVAL, "no training set");
    if (!(hp->lr > 0.f) || !(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f) ||
        !(hp->eps > 0.f) || !(hp->weight_decay >= 0.f))
        return fail(MCPD_EINVAL, "bad AdamW hyper-parameters");
    double *hist = nullptr;
    int rc = dev_alloc(&hist, (size_t)std::max(steps, 1));
    if (rc) return rc;
    for (int32_t s = 0; s < steps && !rc; ++s) {
        rc = loss_grad_device(M, hist + s);
        if (rc) break;
        M->step += 1;
        const double bc1 = 1.0 - std::pow((double)hp->beta1, (double)M->step);
        const double bc2 = 1.0 - std::pow((double)hp->beta2, (double)M->step);
        int e = K::launch_adamw(M->d_theta, M->d_m, M->d_v, M->d_grad, M->d_wb, hp->lr, hp->beta1, hp->beta2,
                                hp->eps, hp->weight_decay, (float)bc1, (float)bc2, M->stream);
        if (e != hipSuccess) rc = hip_fail((hipError_t)e, "adamw kernel");
    }
    hipError_t e = hipSuccess;
    if (!rc && loss_history && steps > 0)
        e = hipMemcpyAsync(loss_history, hist, (size_t)steps * 8, hipMemcpyDeviceToHost, M->stream);
    hipError_t se = hipStreamSynchronize(M->stream);
    dev_free(hist);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
    return MCPD_OK;
}

int mcpd_mlp_backward(mcpd_mlp *M, const float *x, int64_t rows, const float *dg, float *grad)
{
    if (!M || !x || !dg || !grad || rows <= 0) return fail(MCPD_EINVAL, "bad argument");
    int64_t per = 0;
    const int nblocks = K::backward_blocks(rows, M->cus, &per);
    float *dX = nullptr, *ddg = nullptr, *dpart = nullptr, *dgrad = nullptr;
    int rc = dev_alloc(&dX, (size_t)rows * MCPD_MLP_FEATURES);
    if (!rc) rc = dev_alloc(&ddg, (size_t)rows);
    if (!rc) rc = dev_alloc(&dpart, (size_t)nblocks * MCPD_MLP_PARAMS);
    if (!rc) rc = dev_alloc(&dgrad, (size_t)MCPD_MLP_PARAMS);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(dX, x, (size_t)rows * MCPD_MLP_FEATURES * 4, hipMemcpyHostToDevice, M->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(ddg, dg, (size_t)rows * 4, hipMemcpyHostToDevice, M->stream);
        if (e == hipSuccess)
            e = (hipError_t)K::launch_backward(M->d_wb, dX, ddg, rows, nblocks, per, dpart, dgrad, M->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(grad, dgrad, MCPD_MLP_PARAMS * 4, hipMemcpyDeviceToHost, M->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
        if (e != hipSuccess) rc = hip_fail(e, "backward");
    }
    dev_free(dX);
    dev_free(ddg);
    dev_free(dpart);
    dev_free(dgrad);
    return rc;
}

int mcpd_mlp_adamw_step(mcpd_mlp *M, const float *grad, const mcpd_adamw *hp)
{
    if (!M || !grad || !hp) return fail(MCPD_EINVAL, "bad argument");
    if (!(hp->lr > 0.f) || !(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f) ||
        !(hp->eps > 0.f) || !(hp->weight_decay >= 0.f))
        return fail(MCPD_EINVAL, "bad AdamW hyper-parameters");
    if (!finite_params(grad)) return fail(MCPD_EINVAL, "gradient must be finite");
    HIP_TRY(hipMemcpyAsync(M->d_grad, grad, MCPD_MLP_PARAMS * 4, hipMemcpyHostToDevice, M->stream));
    M->step += 1;
    const double bc1 = 1.0 - std::pow((double)hp->beta1, (double)M->step);
    const double bc2 = 1.0 - std::pow((double)hp->beta2, (double)M->step);
    int e = K::launch_adamw(M->d_theta, M->d_m, M->d_v, M->d_grad, M->d_wb, hp->lr, hp->beta1, hp->beta2, hp->eps,
                            hp->weight_decay, (float)bc1, (float)bc2, M->stream);
    if (e != hipSuccess) return hip_fail((hipError_t)e, "adamw kernel");
    HIP_TRY(hipStreamSynchronize(M->stream));
    return MCPD_OK;
}

int mcpd_mlp_get_state(const mcpd_mlp *M, float *master, uint16_t *bf16, float *adam_m, float *adam_v, int64_t *step)
{
    if (!M) return fail(MCPD_EINVAL, "null network");
    if (master) HIP_TRY(hipMemcpyAsync(master, M->d_theta, MCPD_MLP_PARAMS * 4, hipMemcpyDeviceToHost, M->stream));
    if (bf16) HIP_TRY(hipMemcpyAsync(bf16, M->d_wb, MCPD_MLP_PARAMS * 2, hipMemcpyDeviceToHost, M->stream));
    if (adam_m) HIP_TRY(hipMemcpyAsync(adam_m, M->d_m, MCPD_MLP_PARAMS * 4, hipMemcpyDeviceToHost, M->stream));
    if (adam_v) HIP_TRY(hipMemcpyAsync(adam_v, M->d_v, MCPD_MLP_PARAMS * 4, hipMemcpyDeviceToHost, M->stream));
    HIP_TRY(hipStreamSynchronize(M->stream));
    if (step) *step = M->step;
    return MCPD_OK;
}

int mcpd_mlp_set_state(mcpd_mlp *M, const float *master, const float *adam_m, const float *adam_v, int64_t step)
{
    if (!M) return fail(MCPD_EINVAL, "null network");
    if (!master || !adam_m || !adam_v || step < 0) return fail(MCPD_EINVAL, "bad argument");
    if (!finite_params(master) || !finite_params(adam_m) || !finite_params(adam_v))
        return fail(MCPD_EINVAL, "state must be finite");
    for (int k = 0; k < MCPD_MLP_PARAMS; ++k)
        if (adam_v[k] < 0.f) return fail(MCPD_EINVAL, "second moments must be >= 0");
    HIP_TRY(hipMemcpyAsync(M->d_theta, master, MCPD_MLP_PARAMS * 4, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(M->d_m, adam_m, MCPD_MLP_PARAMS * 4, hipMemcpyHostToDevice, M->stream));
    HIP_TRY(hipMemcpyAsync(M->d_v, adam_v, MCPD_MLP_PARAMS * 4, hipMemcpyHostToDevice, M->stream));
    int e = K::launch_cast(M->d_theta, M->d_wb, M->stream);
    if (e != hipSuccess) return hip_fail((hipError_t)e, "cast kernel");
    HIP_TRY(hipStreamSynchronize(M->stream));
    M->step = step;
    return MCPD_OK;
}

int mcpd_set_learned_weights(mcpd_instance *I, mcpd_mlp *M, double alpha, double *w_out)
{
    if (!I || !M) return fail(MCPD_EINVAL, "null argument");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(MCPD_EINVAL, "alpha must be in (0, 1]");
    const size_t n = (size_t)I->n;
    float *X = nullptr, *df = nullptr;
    double *dbase = nullptr;
    int rc = dev_alloc(&X, n * MCPD_MLP_FEATURES);
    if (!rc) rc = dev_alloc(&df, n);
    if (!rc) rc = dev_alloc(&dbase, n);
    std::vector<float> f(n);
    std::vector<double> c(n);
    if (!rc) rc = device_features(I, X, dbase, M->stream);
    if (!rc) {
        hipError_t e = (hipError_t)K::launch_forward(M->d_wb, X, (int64_t)n, df, M->cus, M->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(f.data(), df, n * 4, hipMemcpyDeviceToHost, M->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(c.data(), dbase, n * 8, hipMemcpyDeviceToHost, M->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(M->stream);
        if (e != hipSuccess) rc = hip_fail(e, "forward");
    }
    dev_free(X);
    dev_free(df);
    dev_free(dbase);
    if (rc) return rc;
    // w = (1 - alpha) softmax(c + f) + alpha / n, in FP64
    std::vector<double> w(n);
    double gmax = -INFINITY;
    for (size_t i = 0; i < n; ++i) {
        w[i] = c[i] + (double)f[i];
        if (!std::isfinite(w[i])) return fail(MCPD_EINVAL, "network output is not finite");
        gmax = std::max(gmax, w[i]);
    }
    double z = 0.0;
    for (size_t i = 0; i < n; ++i) {
        w[i] = std::exp(w[i] - gmax);
        z += w[i];
    }
    for (size_t i = 0; i < n; ++i) w[i] = (1.0 - alpha) * (w[i] / z) + alpha / (double)n;
    if (w_out) std::memcpy(w_out, w.data(), n * sizeof(double));
    return mcpd_set_weights(I, w.data());
}

void mcpd_mlp_destroy(mcpd_mlp *M)
{
    delete M;
}

}  // extern "C"
