// Small MLP cost model: predicts log(pass time) from pass features; trained and run on the GPU.
//
// Architecture (FP32): x (NIN) -> Linear(H) -> ReLU -> Linear(H) -> ReLU -> Linear(1). Parameters are one flat
// device array: W1[H][NIN], b1[H], W2[H][H], b2[H], W3[H], b3. Loss: mean squared error over the batch.
// Every reduction (weight gradients, loss) runs in a fixed order (one thread per weight looping over the batch,
// one workgroup tree for the loss), so training is deterministic. Optimiser: Adam.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "qs_internal.h"

namespace {

constexpr int kMlpMaxBatch = 4096;

struct Dims {
    int nin, h;
    int oW1() const { return 0; }
    int ob1() const { return h * nin; }
    int oW2() const { return ob1() + h; }
    int ob2() const { return oW2() + h * h; }
    int oW3() const { return ob2() + h; }
    int ob3() const { return oW3() + h; }
    int total() const { return ob3() + 1; }
};

// Z[s][u] = b[u] + sum_i W[u][i] X[s][i]; A = relu(Z) (or Z for the output layer)
__global__ __launch_bounds__(256) void k_fwd(const float *__restrict__ W, const float *__restrict__ b,
                                             const float *__restrict__ X, float *__restrict__ Z, float *__restrict__ A,
                                             int B, int nin, int nout, int relu)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * nout)
        return;
    const int s = t / nout, u = t % nout;
    float z = b[u];
    for (int i = 0; i < nin; ++i)
        z = fmaf(W[u * nin + i], X[s * nin + i], z);
    Z[t] = z;
    A[t] = relu ? fmaxf(z, 0.0f) : z;
}

// dY[s] = 2 (Y[s] - T[s]) / B; loss = sum (Y - T)^2 / B (one workgroup, fixed-order tree)
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ Y, const float *__restrict__ T,
                                             float *__restrict__ dY, float *__restrict__ loss, int B)
{
    __shared__ float red[256];
    float acc = 0.0f;
    for (int s = threadIdx.x; s < B; s += blockDim.x) {
        const float d = Y[s] - T[s];
        dY[s] = 2.0f * d / (float)B;
        acc = fmaf(d, d, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *loss = red[0] / (float)B;
}

// dZ[s][i] = (sum_u W[u][i] dZn[s][u]) * (Z[s][i] > 0)
__global__ __launch_bounds__(256) void k_bwd_delta(const float *__restrict__ W, const float *__restrict__ dZn,
                                                   const float *__restrict__ Z, float *__restrict__ dZ, int B, int nin,
                                                   int nout)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * nin)
        return;
    const int s = t / nin, i = t % nin;
    float g = 0.0f;
    for (int u = 0; u < nout; ++u)
        g = fmaf(W[u * nin + i], dZn[s * nout + u], g);
    dZ[t] = Z[t] > 0.0f ? g : 0.0f;
}

// gW[u][i] = sum_s dZ[s][u] A[s][i];  gb[u] = sum_s dZ[s][u]  (thread per weight, batch order fixed)
__global__ __launch_bounds__(256) void k_bwd_wgrad(const float *__restrict__ dZ, const float *__restrict__ Ain,
                                                   float *__restrict__ gW, float *__restrict__ gb, int B, int nin,
                                                   int nout)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nout * nin) {
        const int u = t / nin, i = t % nin;
        float g = 0.0f;
        for (int s = 0; s < B; ++s)
            g = fmaf(dZ[s * nout + u], Ain[s * nin + i], g);
        gW[t] = g;
    } else if (t < nout * nin + nout) {
        const int u = t - nout * nin;
        float g = 0.0f;
        for (int s = 0; s < B; ++s)
            g += dZ[s * nout + u];
        gb[u] = g;
    }
}

// Adam: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct qs_mlp {
    Dims d{};
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    // activations / gradients for up to kMlpMaxBatch samples
    float *X = nullptr, *T = nullptr, *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *Y = nullptr;
    float *dY = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *loss = nullptr;
    int step = 0;
    hipStream_t stream = nullptr;
};

namespace {

void mlp_release(qs_mlp *M)
{
    if (!M)
        return;
    float *bufs[] = {M->params, M->grads, M->m, M->v, M->X, M->T, M->Z1, M->A1, M->Z2, M->A2, M->Y, M->dY, M->dZ2,
                     M->dZ1, M->loss};
    for (float *b : bufs)
        if (b)
            (void)hipFree(b);
    delete M;
}

hipError_t forward(qs_mlp *M, int B)
{
    const Dims &d = M->d;
    const float *P = M->params;
    hipLaunchKernelGGL(k_fwd, dim3(blocks(B * d.h)), dim3(256), 0, M->stream, P + d.oW1(), P + d.ob1(), M->X, M->Z1,
                       M->A1, B, d.nin, d.h, 1);
    hipLaunchKernelGGL(k_fwd, dim3(blocks(B * d.h)), dim3(256), 0, M->stream, P + d.oW2(), P + d.ob2(), M->A1, M->Z2,
                       M->A2, B, d.h, d.h, 1);
    hipLaunchKernelGGL(k_fwd, dim3(blocks(B)), dim3(256), 0, M->stream, P + d.oW3(), P + d.ob3(), M->A2, M->Y, M->Y, B,
                       d.h, 1, 0);
    return hipGetLastError();
}

hipError_t backward(qs_mlp *M, int B)
{
    const Dims &d = M->d;
    const float *P = M->params;
    float *G = M->grads;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, M->stream, M->Y, M->T, M->dY, M->loss, B);
    hipLaunchKernelGGL(k_bwd_wgrad, dim3(blocks(d.h + 1)), dim3(256), 0, M->stream, M->dY, M->A2, G + d.oW3(),
                       G + d.ob3(), B, d.h, 1);
    hipLaunchKernelGGL(k_bwd_delta, dim3(blocks(B * d.h)), dim3(256), 0, M->stream, P + d.oW3(), M->dY, M->Z2, M->dZ2,
                       B, d.h, 1);
    hipLaunchKernelGGL(k_bwd_wgrad, dim3(blocks(d.h * d.h + d.h)), dim3(256), 0, M->stream, M->dZ2, M->A1,
                       G + d.oW2(), G + d.ob2(), B, d.h, d.h);
    hipLaunchKernelGGL(k_bwd_delta, dim3(blocks(B * d.h)), dim3(256), 0, M->stream, P + d.oW2(), M->dZ2, M->Z1, M->dZ1,
                       B, d.h, d.h);
    hipLaunchKernelGGL(k_bwd_wgrad, dim3(blocks(d.h * d.nin + d.h)), dim3(256), 0, M->stream, M->dZ1, M->X,
                       G + d.oW1(), G + d.ob1(), B, d.nin, d.h);
    return hipGetLastError();
}

int check_batch(int B)
{
    if (B < 1 || B > kMlpMaxBatch)
        return qs_fail(QS_EINVAL, "batch of %d samples outside [1, %d]", B, kMlpMaxBatch);
    return QS_OK;
}

}  // namespace

extern "C" {

QS_API int qs_mlp_create(qs_mlp **out, int nin, int hidden, void *hip_stream)
{
    qs_clear_error();
    if (!out)
        return qs_fail(QS_EINVAL, "qs_mlp_create: out is NULL");
    *out = nullptr;
    if (nin < 1 || nin > 1024 || hidden < 1 || hidden > 1024)
        return qs_fail(QS_EINVAL, "qs_mlp_create: sizes out of range (nin = %d, hidden = %d)", nin, hidden);
    qs_mlp *M = new (std::nothrow) qs_mlp();
    if (!M)
        return qs_fail(QS_ENOMEM, "qs_mlp_create: out of host memory");
    M->d = Dims{nin, hidden};
    M->stream = (hipStream_t)hip_stream;
    const size_t np = M->d.total();
    const size_t B = kMlpMaxBatch;
    struct {
        float **p;
        size_t n;
    } allocs[] = {{&M->params, np}, {&M->grads, np}, {&M->m, np}, {&M->v, np}, {&M->X, B * nin}, {&M->T, B},
                  {&M->Z1, B * hidden}, {&M->A1, B * hidden}, {&M->Z2, B * hidden}, {&M->A2, B * hidden}, {&M->Y, B},
                  {&M->dY, B}, {&M->dZ2, B * hidden}, {&M->dZ1, B * hidden}, {&M->loss, 1}};
    for (auto &a : allocs) {
        hipError_t e = hipMalloc((void **)a.p, a.n * sizeof(float));
        if (e != hipSuccess) {
            *a.p = nullptr;
            int rc = qs_hip_fail(e, "hipMalloc(mlp)");
            mlp_release(M);
            return rc;
        }
    }
    if (hipMemsetAsync(M->m, 0, np * sizeof(float), M->stream) != hipSuccess ||
        hipMemsetAsync(M->v, 0, np * sizeof(float), M->stream) != hipSuccess) {
        int rc = qs_hip_fail(hipGetLastError(), "hipMemsetAsync(mlp)");
        mlp_release(M);
        return rc;
    }
    *out = M;
    return QS_OK;
}

QS_API int qs_mlp_free(qs_mlp *M)
{
    qs_clear_error();
    if (!M)
        return qs_fail(QS_EINVAL, "qs_mlp_free: NULL model");
    (void)hipStreamSynchronize(M->stream);
    mlp_release(M);
    return QS_OK;
}

QS_API int qs_mlp_num_params(const qs_mlp *M, int *n)
{
    qs_clear_error();
    if (!M || !n)
        return qs_fail(QS_EINVAL, "qs_mlp_num_params: NULL argument");
    *n = M->d.total();
    return QS_OK;
}

QS_API int qs_mlp_set_params(qs_mlp *M, const float *host)
{
    qs_clear_error();
    if (!M || !host)
        return qs_fail(QS_EINVAL, "qs_mlp_set_params: NULL argument");
    const size_t np = M->d.total();
    QS_HIP(hipMemcpyAsync(M->params, host, np * sizeof(float), hipMemcpyHostToDevice, M->stream));
    QS_HIP(hipMemsetAsync(M->m, 0, np * sizeof(float), M->stream));
    QS_HIP(hipMemsetAsync(M->v, 0, np * sizeof(float), M->stream));
    QS_HIP(hipStreamSynchronize(M->stream));
    M->step = 0;
    return QS_OK;
}

QS_API int qs_mlp_get_params(qs_mlp *M, float *host)
{
    qs_clear_error();
    if (!M || !host)
        return qs_fail(QS_EINVAL, "qs_mlp_get_params: NULL argument");
    QS_HIP(hipMemcpyAsync(host, M->params, M->d.total() * sizeof(float), hipMemcpyDeviceToHost, M->stream));
    QS_HIP(hipStreamSynchronize(M->stream));
    return QS_OK;
}

}  // extern "C"

int qs_mlp_nin(const qs_mlp *m) { return m ? m->d.nin : 0; }

extern "C" {

QS_API int qs_mlp_predict(qs_mlp *M, const float *X, int B, float *Y)
{
    qs_clear_error();
    if (!M || !X || !Y)
        return qs_fail(QS_EINVAL, "qs_mlp_predict: NULL argument");
    if (int rc = check_batch(B))
        return rc;
    QS_HIP(hipMemcpyAsync(M->X, X, (size_t)B * M->d.nin * sizeof(float), hipMemcpyHostToDevice, M->stream));
    QS_HIP(forward(M, B));
    QS_HIP(hipMemcpyAsync(Y, M->Y, (size_t)B * sizeof(float), hipMemcpyDeviceToHost, M->stream));
    QS_HIP(hipStreamSynchronize(M->stream));
    return QS_OK;
}

QS_API int qs_mlp_grad(qs_mlp *M, const float *X, const float *T, int B, float *grads, float *loss)
{
    qs_clear_error();
    if (!M || !X || !T)
        return qs_fail(QS_EINVAL, "qs_mlp_grad: NULL argument");
    if (int rc = check_batch(B))
        return rc;
    QS_HIP(hipMemcpyAsync(M->X, X, (size_t)B * M->d.nin * sizeof(float), hipMemcpyHostToDevice, M->stream));
    QS_HIP(hipMemcpyAsync(M->T, T, (size_t)B * sizeof(float), hipMemcpyHostToDevice, M->stream));
    QS_HIP(forward(M, B));
    QS_HIP(backward(M, B));
    if (grads)
        QS_HIP(hipMemcpyAsync(grads, M->grads, M->d.total() * sizeof(float), hipMemcpyDeviceToHost, M->stream));
    if (loss)
        QS_HIP(hipMemcpyAsync(loss, M->loss, sizeof(float), hipMemcpyDeviceToHost, M->stream));
    QS_HIP(hipStreamSynchronize(M->stream));
    return QS_OK;
}

QS_API int qs_mlp_train_step(qs_mlp *M, const float *X, const float *T, int B, float lr, float *loss)
{
    qs_clear_error();
    if (!M || !X || !T)
        return qs_fail(QS_EINVAL, "qs_mlp_train_step: NULL argument");
    if (int rc = check_batch(B))
        return rc;
    if (!(lr > 0.0f))
        return qs_fail(QS_EINVAL, "qs_mlp_train_step: learning rate must be positive");
    QS_HIP(hipMemcpyAsync(M->X, X, (size_t)B * M->d.nin * sizeof(float), hipMemcpyHostToDevice, M->stream));
    QS_HIP(hipMemcpyAsync(M->T, T, (size_t)B * sizeof(float), hipMemcpyHostToDevice, M->stream));
    QS_HIP(forward(M, B));
    QS_HIP(backward(M, B));
    M->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)M->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)M->step));
    const int np = M->d.total();
    hipLaunchKernelGGL(k_adam, dim3(blocks(np)), dim3(256), 0, M->stream, M->params, M->grads, M->m, M->v, np, lr, b1,
                       b2, eps, c1, c2);
    QS_HIP(hipGetLastError());
    if (loss) {
        QS_HIP(hipMemcpyAsync(loss, M->loss, sizeof(float), hipMemcpyDeviceToHost, M->stream));
        QS_HIP(hipStreamSynchronize(M->stream));
    }
    return QS_OK;
}

}  // extern "C"
