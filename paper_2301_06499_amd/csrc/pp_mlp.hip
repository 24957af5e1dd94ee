// Training of the learned direction scheduler's cost model: a fully
// connected 8 -> 32 -> 32 -> 2 network with ReLU hidden layers whose outputs
// predict the logarithm of a round's duration under pull and under push.
// The round loop runs inference inside its round-end phase; these kernels fit
// the weights to measured round times by full-batch Adam on the mean squared
// error 1/(2N) sum_n sum_k (y_nk - t_nk)^2.
//
// Every reduction has a fixed order (one block per parameter, a fixed
// thread-to-sample assignment and a fixed tree), so training is bit-for-bit
// reproducible.

#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "pp_internal.h"

namespace pp {
namespace {

constexpr int MB = 256;   // threads per block

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One thread per sample: forward pass; with targets, the per-sample error
// terms and the back-propagated deltas of both hidden layers.  Activations
// and deltas are stored feature-major ([unit][N]) for the gradient kernel.
__global__ void __launch_bounds__(MB) k_mlp_fwd_bwd(const float *__restrict__ P, const float *__restrict__ X,
                                                    const float *__restrict__ T, int64_t n, float inv_n,
                                                    float *__restrict__ Y, float *__restrict__ H1,
                                                    float *__restrict__ H2, float *__restrict__ D1,
                                                    float *__restrict__ D2, float *__restrict__ DO,
                                                    float *__restrict__ L) {
    __shared__ float w[MLP_PARAMS];
    for (int i = threadIdx.x; i < MLP_PARAMS; i += MB) w[i] = P[i];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)MB + threadIdx.x;
    if (s >= n) return;
    float x[MLP_IN], h1[MLP_HID], h2[MLP_HID];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) x[i] = X[s * MLP_IN + i];
#pragma unroll
    for (int j = 0; j < MLP_HID; ++j) {
        float a = w[MLP_B1 + j];
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) a += w[MLP_W1 + j * MLP_IN + i] * x[i];
        h1[j] = a > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < MLP_HID; ++j) {
        float a = w[MLP_B2 + j];
#pragma unroll
        for (int i = 0; i < MLP_HID; ++i) a += w[MLP_W2 + j * MLP_HID + i] * h1[i];
        h2[j] = a > 0.0f ? a : 0.0f;
    }
    float y[MLP_OUT];
#pragma unroll
    for (int k = 0; k < MLP_OUT; ++k) {
        float a = w[MLP_B3 + k];
#pragma unroll
        for (int i = 0; i < MLP_HID; ++i) a += w[MLP_W3 + k * MLP_HID + i] * h2[i];
        y[k] = a;
    }
    if (Y) {
#pragma unroll
        for (int k = 0; k < MLP_OUT; ++k) Y[s * MLP_OUT + k] = y[k];
    }
    if (!T) return;
    float dout[MLP_OUT];
    float l = 0.0f;
#pragma unroll
    for (int k = 0; k < MLP_OUT; ++k) {
        const float e = y[k] - T[s * MLP_OUT + k];
        l += e * e;
        dout[k] = e * inv_n;
        DO[k * n + s] = dout[k];
    }
    L[s] = 0.5f * l;
    float d2[MLP_HID];
#pragma unroll
    for (int j = 0; j < MLP_HID; ++j) {
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < MLP_OUT; ++k) a += w[MLP_W3 + k * MLP_HID + j] * dout[k];
        d2[j] = h2[j] > 0.0f ? a : 0.0f;
        H2[j * n + s] = h2[j];
        D2[j * n + s] = d2[j];
    }
#pragma unroll
    for (int i = 0; i < MLP_HID; ++i) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < MLP_HID; ++j) a += w[MLP_W2 + j * MLP_HID + i] * d2[j];
        H1[i * n + s] = h1[i];
        D1[i * n + s] = h1[i] > 0.0f ? a : 0.0f;
    }
}

// Block p < MLP_PARAMS: the gradient of parameter p, the sum over samples of
// (delta of its output unit) x (its input: a feature, a hidden activation or
// 1 for a bias).  Block MLP_PARAMS: the loss.  Sums in double.
__global__ void __launch_bounds__(MB) k_mlp_param_grad(const float *__restrict__ X, const float *__restrict__ H1,
                                                       const float *__restrict__ H2, const float *__restrict__ D1,
                                                       const float *__restrict__ D2, const float *__restrict__ DO,
                                                       const float *__restrict__ L, int64_t n, float *__restrict__ grad,
                                                       float *__restrict__ loss) {
    const int p = blockIdx.x;
    const float *a = nullptr;   // delta row
    const float *b = nullptr;   // input row (NULL: bias)
    int64_t bstride = 1;
    double scale = 1.0;
    if (p < MLP_B1) {
        a = D1 + (int64_t)(p / MLP_IN) * n;
        b = X + p % MLP_IN;
        bstride = MLP_IN;
    } else if (p < MLP_W2) {
        a = D1 + (int64_t)(p - MLP_B1) * n;
    } else if (p < MLP_B2) {
        const int q = p - MLP_W2;
        a = D2 + (int64_t)(q / MLP_HID) * n;
        b = H1 + (int64_t)(q % MLP_HID) * n;
    } else if (p < MLP_W3) {
        a = D2 + (int64_t)(p - MLP_B2) * n;
    } else if (p < MLP_B3) {
        const int q = p - MLP_W3;
        a = DO + (int64_t)(q / MLP_HID) * n;
        b = H2 + (int64_t)(q % MLP_HID) * n;
    } else if (p < MLP_PARAMS) {
        a = DO + (int64_t)(p - MLP_B3) * n;
    } else {
        a = L;
        scale = 1.0 / (double)n;
    }
    double acc = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += MB) acc += b ? (double)a[s] * (double)b[s * bstride] : (double)a[s];
    __shared__ double red[MB / 64];
    acc = wave_sum_d(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < MB / 64; ++k) t += red[k];
        if (p < MLP_PARAMS) grad[p] = (float)t;
        else *loss = (float)(t * scale);
    }
}

// Adam (Kingma and Ba, Algorithm 1) with bias corrections c1 = 1/(1-b1^t),
// c2 = 1/(1-b2^t).
__global__ void __launch_bounds__(MB) k_mlp_adam(float *__restrict__ P, const float *__restrict__ G,
                                                 float *__restrict__ M, float *__restrict__ V, float lr, float b1,
                                                 float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * MB + threadIdx.x;
    if (i >= MLP_PARAMS) return;
    const float g = G[i];
    const float m = b1 * M[i] + (1.0f - b1) * g;
    const float v = b2 * V[i] + (1.0f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    P[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// Device buffers of one call.
struct MlpBufs {
    float *P = nullptr, *X = nullptr, *T = nullptr, *Y = nullptr, *H1 = nullptr, *H2 = nullptr, *D1 = nullptr,
          *D2 = nullptr, *DO = nullptr, *L = nullptr, *G = nullptr, *M = nullptr, *V = nullptr, *loss = nullptr;
    hipStream_t st = nullptr;
    ~MlpBufs() {
        if (st) (void)hipStreamSynchronize(st);   // every kernel and copy on the buffers has finished
        for (float *p : {P, X, T, Y, H1, H2, D1, D2, DO, L, G, M, V, loss}) dev_release(p);
        if (st) (void)hipStreamDestroy(st);
    }
};

int alloc_f(float **p, int64_t count) {
    *p = (float *)dev_malloc(sizeof(float) * (size_t)(count > 0 ? count : 1));
    if (!*p) return set_error(PP_ENOMEM, "cost-model buffer of %lld floats", (long long)count);
    return PP_OK;
}

// Allocates and uploads; targets and training buffers only when asked.
int setup(MlpBufs &b, const float *params, const float *x, const float *t, int64_t n, int32_t steps) {
    const bool train = steps > 0;
    if (!params || !x) return set_error(PP_EINVAL, "params or x is NULL");
    if (n < 1 || n > ((int64_t)1 << 26)) return set_error(PP_EINVAL, "sample count %lld outside [1, 2^26]", (long long)n);
    if (hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking) != hipSuccess) return set_error(PP_EDEVICE, "stream");
    AllocStream as(b.st);   // the buffers are used on this call's stream
    int rc;
    if ((rc = alloc_f(&b.P, MLP_PARAMS)) || (rc = alloc_f(&b.X, n * MLP_IN)) || (rc = alloc_f(&b.Y, n * MLP_OUT)))
        return rc;
    if (t && ((rc = alloc_f(&b.T, n * MLP_OUT)) || (rc = alloc_f(&b.H1, n * MLP_HID)) ||
              (rc = alloc_f(&b.H2, n * MLP_HID)) || (rc = alloc_f(&b.D1, n * MLP_HID)) ||
              (rc = alloc_f(&b.D2, n * MLP_HID)) || (rc = alloc_f(&b.DO, n * MLP_OUT)) || (rc = alloc_f(&b.L, n)) ||
              (rc = alloc_f(&b.G, MLP_PARAMS)) || (rc = alloc_f(&b.loss, steps > 1 ? steps : 1))))
        return rc;
    if (train && ((rc = alloc_f(&b.M, MLP_PARAMS)) || (rc = alloc_f(&b.V, MLP_PARAMS)))) return rc;
    hipError_t e = hipMemcpyAsync(b.P, params, sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice, b.st);
    if (!e) e = hipMemcpyAsync(b.X, x, sizeof(float) * MLP_IN * (size_t)n, hipMemcpyHostToDevice, b.st);
    if (!e && t) e = hipMemcpyAsync(b.T, t, sizeof(float) * MLP_OUT * (size_t)n, hipMemcpyHostToDevice, b.st);
    if (!e && train) e = hipMemsetAsync(b.M, 0, sizeof(float) * MLP_PARAMS, b.st);
    if (!e && train) e = hipMemsetAsync(b.V, 0, sizeof(float) * MLP_PARAMS, b.st);
    if (e) return set_error(PP_EDEVICE, "cost-model upload: %s", hipGetErrorString(e));
    return PP_OK;
}

hipError_t fwd_bwd(const MlpBufs &b, int64_t n, bool targets, int32_t step = 0) {
    const int grid = (int)((n + MB - 1) / MB);
    k_mlp_fwd_bwd<<<grid, MB, 0, b.st>>>(b.P, b.X, targets ? b.T : nullptr, n, (float)(1.0 / (double)n), b.Y, b.H1,
                                         b.H2, b.D1, b.D2, b.DO, b.L);
    hipError_t e = hipGetLastError();
    if (e || !targets) return e;
    k_mlp_param_grad<<<MLP_PARAMS + 1, MB, 0, b.st>>>(b.X, b.H1, b.H2, b.D1, b.D2, b.DO, b.L, n, b.G, b.loss + step);
    return hipGetLastError();
}

}  // namespace
}  // namespace pp

using namespace pp;

extern "C" int pp_mlp_forward(const float *params, const float *x, int64_t n, float *y) {
    if (!y) return set_error(PP_EINVAL, "y is NULL");
    MlpBufs b;
    int rc = setup(b, params, x, nullptr, n, 0);
    if (rc) return rc;
    hipError_t e = fwd_bwd(b, n, false);
    if (!e) e = hipMemcpyAsync(y, b.Y, sizeof(float) * MLP_OUT * (size_t)n, hipMemcpyDeviceToHost, b.st);
    if (!e) e = hipStreamSynchronize(b.st);
    if (e) return set_error(PP_EDEVICE, "cost-model forward: %s", hipGetErrorString(e));
    return PP_OK;
}

extern "C" int pp_mlp_loss_grad(const float *params, const float *x, const float *t, int64_t n, float *grad,
                                float *loss) {
    if (!t) return set_error(PP_EINVAL, "t is NULL");
    MlpBufs b;
    int rc = setup(b, params, x, t, n, 0);
    if (rc) return rc;
    hipError_t e = fwd_bwd(b, n, true);
    if (!e && grad) e = hipMemcpyAsync(grad, b.G, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost, b.st);
    if (!e && loss) e = hipMemcpyAsync(loss, b.loss, sizeof(float), hipMemcpyDeviceToHost, b.st);
    if (!e) e = hipStreamSynchronize(b.st);
    if (e) return set_error(PP_EDEVICE, "cost-model gradient: %s", hipGetErrorString(e));
    return PP_OK;
}

extern "C" int pp_mlp_train(float *params, const float *x, const float *t, int64_t n, int32_t steps, float lr,
                            float *loss_log) {
    if (!t) return set_error(PP_EINVAL, "t is NULL");
    if (steps < 0) return set_error(PP_EINVAL, "steps < 0");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return set_error(PP_EINVAL, "learning rate must be positive and finite");
    MlpBufs b;
    int rc = setup(b, params, x, t, n, steps);
    if (rc) return rc;
    const double b1 = 0.9, b2 = 0.999;
    const float eps = 1e-8f;
    double p1 = 1.0, p2 = 1.0;
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < steps && !e; ++k) {
        e = fwd_bwd(b, n, true, k);
        p1 *= b1;
        p2 *= b2;
        if (!e) {
            k_mlp_adam<<<(MLP_PARAMS + MB - 1) / MB, MB, 0, b.st>>>(b.P, b.G, b.M, b.V, lr, (float)b1, (float)b2, eps,
                                                                   (float)(1.0 / (1.0 - p1)), (float)(1.0 / (1.0 - p2)));
            e = hipGetLastError();
        }
    }
    if (!e) e = hipMemcpyAsync(params, b.P, sizeof(float) * MLP_PARAMS, hipMemcpyDeviceToHost, b.st);
    if (!e && loss_log && steps > 0)
        e = hipMemcpyAsync(loss_log, b.loss, sizeof(float) * (size_t)steps, hipMemcpyDeviceToHost, b.st);
    if (!e) e = hipStreamSynchronize(b.st);
    if (e) return set_error(PP_EDEVICE, "cost-model training: %s", hipGetErrorString(e));
    return PP_OK;
}
