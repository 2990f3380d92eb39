// Cost-model multilayer perceptron 16-64-64-1 (ReLU), float, on the GPU.
//
// The model maps the morphology features of a neuron to the logarithm of the
// time the epoch kernel spends on it. Inputs go through log(1+x) and the
// stored standardisation; the output is de-standardised with y_mean, y_std.
// Parameter layout (floats): x_mean[16] x_std[16] W1[64][16] b1[64]
// W2[64][64] b2[64] W3[64] b3 y_mean y_std.
//
// Training is full-batch: k_forward keeps the activations, k_delta forms the
// per-sample error signals, k_wgrad reduces every parameter's gradient over
// the batch in sample order (one thread per parameter, so the sum order is
// fixed and the result is deterministic), k_adam applies Adam.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mmh {
namespace {

constexpr int F = kFeat, H1 = kH1, H2 = kH2;
constexpr int OXM = 0, OXS = OXM + F, OW1 = OXS + F, OB1 = OW1 + H1 * F, OW2 = OB1 + H1,
              OB2 = OW2 + H2 * H1, OW3 = OB2 + H2, OB3 = OW3 + H2, OYM = OB3 + 1,
              OYS = OYM + 1, NP = OYS + 1;
static_assert(NP == kMlpParams, "parameter layout");

// One thread per sample. U, A1, A2 (n x 16/64/64) and Y (n) receive the
// standardised input, the two hidden activations and the raw output.
__global__ void __launch_bounds__(256) k_forward(const float *__restrict__ p,
                                                 const float *__restrict__ x, int64_t n,
                                                 float *__restrict__ U, float *__restrict__ A1,
                                                 float *__restrict__ A2, float *__restrict__ Y,
                                                 float *__restrict__ pred) {
    __shared__ float sp[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    float u[F], h1[H1];
    for (int i = 0; i < F; ++i) {
        u[i] = (logf(1.0f + x[s * F + i]) - sp[OXM + i]) / sp[OXS + i];
        if (U) U[s * F + i] = u[i];
    }
    for (int o = 0; o < H1; ++o) {
        float z = sp[OB1 + o];
        for (int i = 0; i < F; ++i) z = __builtin_fmaf(sp[OW1 + o * F + i], u[i], z);
        h1[o] = z > 0.0f ? z : 0.0f;
        if (A1) A1[s * H1 + o] = h1[o];
    }
    float y = sp[OB3];
    for (int o = 0; o < H2; ++o) {
        float z = sp[OB2 + o];
        for (int i = 0; i < H1; ++i) z = __builtin_fmaf(sp[OW2 + o * H1 + i], h1[i], z);
        const float h = z > 0.0f ? z : 0.0f;
        if (A2) A2[s * H2 + o] = h;
        y = __builtin_fmaf(sp[OW3 + o], h, y);
    }
    if (Y) Y[s] = y;
    if (pred) pred[s] = y * sp[OYS] + sp[OYM];
}

// Error signals of the loss mean((y - (t - y_mean)/y_std)^2): D3 = dL/dy,
// D2 = dL/dz2, D1 = dL/dz1 (pre-activation). sq receives the squared error.
__global__ void __launch_bounds__(256) k_delta(const float *__restrict__ p,
                                               const float *__restrict__ t, int64_t n,
                                               const float *__restrict__ A1,
                                               const float *__restrict__ A2,
                                               const float *__restrict__ Y, float *__restrict__ D1,
                                               float *__restrict__ D2, float *__restrict__ D3,
                                               float *__restrict__ sq) {
    __shared__ float sp[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) sp[i] = p[i];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float ts = (t[s] - sp[OYM]) / sp[OYS];
    const float err = Y[s] - ts;
    sq[s] = err * err;
    const float d3 = 2.0f * err / (float)n;
    D3[s] = d3;
    float d2[H2];
    for (int o = 0; o < H2; ++o) {
        d2[o] = A2[s * H2 + o] > 0.0f ? d3 * sp[OW3 + o] : 0.0f;
        D2[s * H2 + o] = d2[o];
    }
    for (int i = 0; i < H1; ++i) {
        float acc = 0.0f;
        for (int o = 0; o < H2; ++o) acc = __builtin_fmaf(sp[OW2 + o * H1 + i], d2[o], acc);
        D1[s * H1 + i] = A1[s * H1 + i] > 0.0f ? acc : 0.0f;
    }
}

// Gradient of parameter `q` (trainable range OW1 .. OB3), summed over samples
// in order.
__global__ void __launch_bounds__(256) k_wgrad(const float *__restrict__ U,
                                               const float *__restrict__ A1,
                                               const float *__restrict__ A2,
                                               const float *__restrict__ D1,
                                               const float *__restrict__ D2,
                                               const float *__restrict__ D3, int64_t n,
                                               float *__restrict__ g) {
    const int q = OW1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (q > OB3) return;
    float acc = 0.0f;
    if (q < OB1) {
        const int o = (q - OW1) / F, i = (q - OW1) % F;
        for (int64_t s = 0; s < n; ++s) acc = __builtin_fmaf(D1[s * H1 + o], U[s * F + i], acc);
    } else if (q < OW2) {
        const int o = q - OB1;
        for (int64_t s = 0; s < n; ++s) acc += D1[s * H1 + o];
    } else if (q < OB2) {
        const int o = (q - OW2) / H1, i = (q - OW2) % H1;
        for (int64_t s = 0; s < n; ++s) acc = __builtin_fmaf(D2[s * H2 + o], A1[s * H1 + i], acc);
    } else if (q < OW3) {
        const int o = q - OB2;
        for (int64_t s = 0; s < n; ++s) acc += D2[s * H2 + o];
    } else if (q < OB3) {
        const int o = q - OW3;
        for (int64_t s = 0; s < n; ++s) acc = __builtin_fmaf(D3[s], A2[s * H2 + o], acc);
    } else {
        for (int64_t s = 0; s < n; ++s) acc += D3[s];
    }
    g[q] = acc;
}

// Sum of n values in index order by one workgroup (deterministic).
__global__ void __launch_bounds__(256) k_sum(const float *__restrict__ v, int64_t n,
                                             float *__restrict__ out) {
    __shared__ float part[256];
    float acc = 0.0f;
    const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const int64_t b = threadIdx.x * chunk;
    for (int64_t s = b; s < b + chunk && s < n; ++s) acc += v[s];
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.0f;
        for (int i = 0; i < (int)blockDim.x; ++i) tot += part[i];
        *out = tot;
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int q = OW1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (q > OB3) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

}  // namespace

struct MlpWork {
    float *p = nullptr, *x = nullptr, *t = nullptr, *U = nullptr, *A1 = nullptr, *A2 = nullptr,
          *Y = nullptr, *D1 = nullptr, *D2 = nullptr, *D3 = nullptr, *sq = nullptr, *g = nullptr,
          *m = nullptr, *v = nullptr, *loss = nullptr, *pred = nullptr;
};

static void mlp_free(MlpWork &w) {
    float **all[] = {&w.p, &w.x, &w.t, &w.U, &w.A1, &w.A2, &w.Y, &w.D1,
                     &w.D2, &w.D3, &w.sq, &w.g, &w.m, &w.v, &w.loss, &w.pred};
    for (float **q : all)
        if (*q) {
            (void)hipFree(*q);
            *q = nullptr;
        }
}

static hipError_t mlp_alloc(MlpWork &w, int64_t n, bool train) {
    struct {
        float **ptr;
        int64_t count;
        bool need;
    } plan[] = {{&w.p, NP, true},        {&w.x, n * F, true},    {&w.t, n, train},
                {&w.U, n * F, train},    {&w.A1, n * H1, train}, {&w.A2, n * H2, train},
                {&w.Y, n, train},        {&w.D1, n * H1, train}, {&w.D2, n * H2, train},
                {&w.D3, n, train},       {&w.sq, n, train},      {&w.g, NP, train},
                {&w.m, NP, train},       {&w.v, NP, train},      {&w.loss, 1, train},
                {&w.pred, n, true}};
    for (auto &e : plan) {
        if (!e.need) continue;
        hipError_t err = hipMalloc((void **)e.ptr, sizeof(float) * (e.count > 0 ? e.count : 1));
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

static int blocks(int64_t n, int nt) { return (int)((n + nt - 1) / nt); }

hipError_t mlp_forward(const float *params, const float *x, int64_t n, float *out) {
    MlpWork w;
    hipError_t e = mlp_alloc(w, n, false);
    if (e == hipSuccess) e = hipMemcpy(w.p, params, NP * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(w.x, x, n * F * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess && n > 0) {
        hipLaunchKernelGGL(k_forward, dim3(blocks(n, 256)), dim3(256), 0, 0, w.p, w.x, n,
                           nullptr, nullptr, nullptr, nullptr, w.pred);
        e = hipGetLastError();
    }
    if (e == hipSuccess && n > 0) e = hipMemcpy(out, w.pred, n * sizeof(float), hipMemcpyDeviceToHost);
    mlp_free(w);
    return e;
}

static hipError_t grad_pass(MlpWork &w, int64_t n) {
    hipLaunchKernelGGL(k_forward, dim3(blocks(n, 256)), dim3(256), 0, 0, w.p, w.x, n, w.U, w.A1,
                       w.A2, w.Y, nullptr);
    hipLaunchKernelGGL(k_delta, dim3(blocks(n, 256)), dim3(256), 0, 0, w.p, w.t, n, w.A1, w.A2,
                       w.Y, w.D1, w.D2, w.D3, w.sq);
    hipLaunchKernelGGL(k_wgrad, dim3(blocks(OB3 - OW1 + 1, 256)), dim3(256), 0, 0, w.U, w.A1,
                       w.A2, w.D1, w.D2, w.D3, n, w.g);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(const float *params, const float *x, const float *t, int64_t n,
                         float *loss, float *grad) {
    MlpWork w;
    hipError_t e = mlp_alloc(w, n, true);
    if (e == hipSuccess) e = hipMemcpy(w.p, params, NP * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.x, x, n * F * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.t, t, n * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(w.g, 0, NP * sizeof(float));
    if (e == hipSuccess) e = grad_pass(w, n);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, 0, w.sq, n, w.loss);
        e = hipGetLastError();
    }
    float tot = 0.0f;
    if (e == hipSuccess) e = hipMemcpy(&tot, w.loss, sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(grad, w.g, NP * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) *loss = tot / (float)n;
    mlp_free(w);
    return e;
}

hipError_t mlp_train(float *params, const float *x, const float *t, int64_t n, int epochs,
                     float lr, float *final_loss) {
    MlpWork w;
    hipError_t e = mlp_alloc(w, n, true);
    if (e == hipSuccess) e = hipMemcpy(w.p, params, NP * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.x, x, n * F * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.t, t, n * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(w.g, 0, NP * sizeof(float));
    if (e == hipSuccess) e = hipMemset(w.m, 0, NP * sizeof(float));
    if (e == hipSuccess) e = hipMemset(w.v, 0, NP * sizeof(float));
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float c1 = 1.0f, c2 = 1.0f;
    for (int it = 0; it < epochs && e == hipSuccess; ++it) {
        e = grad_pass(w, n);
        c1 *= b1;
        c2 *= b2;
        hipLaunchKernelGGL(k_adam, dim3(blocks(OB3 - OW1 + 1, 256)), dim3(256), 0, 0, w.p, w.g,
                           w.m, w.v, lr, b1, b2, eps, 1.0f - c1, 1.0f - c2);
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e == hipSuccess) e = grad_pass(w, n);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, 0, w.sq, n, w.loss);
        e = hipGetLastError();
    }
    float tot = 0.0f;
    if (e == hipSuccess) e = hipMemcpy(&tot, w.loss, sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(params, w.p, NP * sizeof(float), hipMemcpyDeviceToHost);
    if (e == hipSuccess && final_loss) *final_loss = tot / (float)n;
    mlp_free(w);
    return e;
}

}  // namespace mmh
