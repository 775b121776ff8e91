// mlp.hip -- the cost model's network on gfx950: a fully connected FP32
// network with two hidden layers of kMlpHidden ReLU units and one linear
// output, its forward pass, the gradient of the mean squared error, and
// Adam updates.
//
// Parameters, one flat float array: W1[H][D] (row j holds unit j's input
// weights), b1[H], W2[H][H], b2[H], w3[H], b3.  For sample x (D features):
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3.
// Loss over N samples: (1/N) sum (y - t)^2.  Backward, per sample:
//   dy = 2 (y - t) / N, dh2 = dy w3 * [h2 > 0], dh1 = W2^T dh2 * [h1 > 0],
// and every weight's gradient is a sum over samples of a product of an
// upstream gradient and an activation (dW2[j][i] = sum dh2[j] h1[i], ...).
//
// Forward and the per-sample backward run one thread per sample with the
// weights in LDS (every thread reads the same weight: broadcasts).  Each
// gradient entry is then a sum over samples in a fixed order (chunks in
// sample order, their sums in chunk order), so gradients are bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sym {

namespace {

constexpr int H = kMlpHidden;

struct MlpView {
    const float *W1, *b1, *W2, *b2, *w3, *b3;
};

__device__ __forceinline__ MlpView view(const float *p, int D)
{
    MlpView v;
    v.W1 = p;
    v.b1 = v.W1 + H * D;
    v.W2 = v.b1 + H;
    v.b2 = v.W2 + H * H;
    v.w3 = v.b2 + H;
    v.b3 = v.w3 + H;
    return v;
}

// Forward for one sample; h1, h2 receive the hidden activations.
__device__ __forceinline__ float forward_one(const float *P, const float *x, int D, float *h1,
                                             float *h2)
{
    const MlpView v = view(P, D);
    for (int j = 0; j < H; ++j) {
        float s = v.b1[j];
        for (int i = 0; i < D; ++i) s += v.W1[j * D + i] * x[i];
        h1[j] = s > 0.0f ? s : 0.0f;
    }
    for (int j = 0; j < H; ++j) {
        float s = v.b2[j];
        for (int i = 0; i < H; ++i) s += v.W2[j * H + i] * h1[i];
        h2[j] = s > 0.0f ? s : 0.0f;
    }
    float y = v.b3[0];
    for (int j = 0; j < H; ++j) y += v.w3[j] * h2[j];
    return y;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ params,
                                                     const float *__restrict__ X, int n, int D,
                                                     float *__restrict__ y)
{
    extern __shared__ float sp[];
    const int count = H * D + H + H * H + H + H + 1;
    for (int k = threadIdx.x; k < count; k += blockDim.x) sp[k] = params[k];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[kMlpMaxIn], h1[H], h2[H];
    for (int i = 0; i < D; ++i) x[i] = X[(int64_t)s * D + i];
    y[s] = forward_one(sp, x, D, h1, h2);
}

// Per-sample backward: stores h1, h2, dh1, dh2 (N x H each, sample-major)
// and dy (N) in `work` for the gradient sums.
__global__ __launch_bounds__(256) void k_mlp_backward_samples(const float *__restrict__ params,
                                                              const float *__restrict__ X,
                                                              const float *__restrict__ t, int n,
                                                              int D, float *__restrict__ work)
{
    extern __shared__ float sp[];
    const int count = H * D + H + H * H + H + H + 1;
    for (int k = threadIdx.x; k < count; k += blockDim.x) sp[k] = params[k];
    __syncthreads();
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const MlpView v = view(sp, D);
    float x[kMlpMaxIn], h1[H], h2[H], d2[H];
    for (int i = 0; i < D; ++i) x[i] = X[(int64_t)s * D + i];
    const float y = forward_one(sp, x, D, h1, h2);
    const float dy = 2.0f * (y - t[s]) / (float)n;
    for (int j = 0; j < H; ++j) d2[j] = h2[j] > 0.0f ? dy * v.w3[j] : 0.0f;
    float *H1 = work, *H2 = H1 + (int64_t)n * H, *D1 = H2 + (int64_t)n * H, *D2 = D1 + (int64_t)n * H;
    float *DY = D2 + (int64_t)n * H;
    for (int i = 0; i < H; ++i) {
        float s1 = 0.0f;
        for (int j = 0; j < H; ++j) s1 += v.W2[j * H + i] * d2[j];
        D1[(int64_t)s * H + i] = h1[i] > 0.0f ? s1 : 0.0f;
    }
    for (int j = 0; j < H; ++j) {
        H1[(int64_t)s * H + j] = h1[j];
        H2[(int64_t)s * H + j] = h2[j];
        D2[(int64_t)s * H + j] = d2[j];
    }
    DY[s] = dy;
}

// Gradient entries as sums over samples, in two deterministic steps: the
// samples are cut into kMlpGradChunks consecutive chunks, one thread per
// (parameter, chunk) sums its chunk in sample order, and k_mlp_grad_sum
// adds the chunk sums in chunk order.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ X, int n, int D,
                                                  const float *__restrict__ work,
                                                  float *__restrict__ partial)
{
    const int count = H * D + H + H * H + H + H + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int len = (n + kMlpGradChunks - 1) / kMlpGradChunks;
    const int a0 = min(n, (int)blockIdx.y * len), a1 = min(n, a0 + len);
    const float *H1 = work, *H2 = H1 + (int64_t)n * H, *D1 = H2 + (int64_t)n * H, *D2 = D1 + (int64_t)n * H;
    const float *DY = D2 + (int64_t)n * H;
    float s = 0.0f;
    int q = k;
    if (q < H * D) {                                  // W1[j][i] = sum dh1[j] x[i]
        const int j = q / D, i = q % D;
        for (int a = a0; a < a1; ++a) s += D1[(int64_t)a * H + j] * X[(int64_t)a * D + i];
    } else if ((q -= H * D) < H) {                    // b1[j]
        for (int a = a0; a < a1; ++a) s += D1[(int64_t)a * H + q];
    } else if ((q -= H) < H * H) {                    // W2[j][i] = sum dh2[j] h1[i]
        const int j = q / H, i = q % H;
        for (int a = a0; a < a1; ++a) s += D2[(int64_t)a * H + j] * H1[(int64_t)a * H + i];
    } else if ((q -= H * H) < H) {                    // b2[j]
        for (int a = a0; a < a1; ++a) s += D2[(int64_t)a * H + q];
    } else if ((q -= H) < H) {                        // w3[j] = sum dy h2[j]
        for (int a = a0; a < a1; ++a) s += DY[a] * H2[(int64_t)a * H + q];
    } else {                                          // b3
        for (int a = a0; a < a1; ++a) s += DY[a];
    }
    partial[(int64_t)blockIdx.y * count + k] = s;
}

__global__ __launch_bounds__(256) void k_mlp_grad_sum(const float *__restrict__ partial, int count,
                                                      float *__restrict__ grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    float s = 0.0f;
    for (int c = 0; c < kMlpGradChunks; ++c) s += partial[(int64_t)c * count + k];
    grad[k] = s;
}

__global__ void k_mlp_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, int64_t count, float lr, float c1, float c2)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        m[k] = b1 * m[k] + (1.0f - b1) * g[k];
        v[k] = b2 * v[k] + (1.0f - b2) * g[k] * g[k];
        p[k] -= lr * (m[k] / c1) / (sqrtf(v[k] / c2) + eps);
    }
}

}  // namespace

int64_t mlp_param_count(int D) { return (int64_t)H * D + H + (int64_t)H * H + H + H + 1; }

int64_t mlp_work_floats(int n, int D)
{
    return (int64_t)n * (4 * H + 1) + (int64_t)kMlpGradChunks * mlp_param_count(D);
}

hipError_t launch_mlp_forward(const float *params, const float *X, int n, int D, float *y,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = sizeof(float) * (size_t)mlp_param_count(D);
    k_mlp_forward<<<(n + 255) / 256, 256, lds, s>>>(params, X, n, D, y);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const float *params, const float *X, const float *t, int n, int D,
                               float *grad, float *work, hipStream_t s)
{
    const int64_t count = mlp_param_count(D);
    if (n > 0) {
        const size_t lds = sizeof(float) * (size_t)count;
        k_mlp_backward_samples<<<(n + 255) / 256, 256, lds, s>>>(params, X, t, n, D, work);
    }
    float *partial = work + mlp_work_floats(n, D) - (int64_t)kMlpGradChunks * count;
    const unsigned gx = (unsigned)((count + 255) / 256);
    k_mlp_grad<<<dim3(gx, kMlpGradChunks), 256, 0, s>>>(X, n, D, work, partial);
    k_mlp_grad_sum<<<gx, 256, 0, s>>>(partial, (int)count, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count,
                           int step, float lr, hipStream_t s)
{
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    k_mlp_adam<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(params, grad, m, v, count, lr, c1, c2);
    return hipGetLastError();
}

}  // namespace sym
