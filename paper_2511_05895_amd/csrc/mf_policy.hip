// Value network of the learned phase schedule: forward, loss gradient and
// Adam kernels (fp32).  The network is
//     h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  q = W3 h2 + b3
// with x in R^F, h1, h2 in R^H and one output q[a] per phase action a.  It is
// fitted by regressing the output of the action taken in a sample on that
// sample's target: L = (1/N) sum_i (q_i[a_i] - y_i)^2.  Parameters are one
// flat fp32 vector: W1 (H x F, row-major), b1, W2 (H x H), b2, W3 (K x H), b3.
//
// The gradient kernel gives one workgroup a tile of samples staged in LDS.
// One lane per sample runs the forward pass and the backward pass of the
// taken action (activations and deltas written to LDS); then every
// parameter's gradient is a dot product over the tile's samples read from
// LDS, added to the global gradient with one atomic per parameter and
// workgroup.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_internal.h"

namespace mf {

namespace {

constexpr int F = kPolF, H = kPolH, K = kPolK;
constexpr int oW1 = 0, ob1 = oW1 + H * F, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + K * H;
static_assert(ob3 + K == kPolParams, "parameter layout");
constexpr int kTile = 64;  // samples per workgroup
constexpr int kThreads = 256;

}  // namespace

__global__ void __launch_bounds__(kThreads)
    k_mlp_grad(const float *__restrict__ theta, const float *__restrict__ X, const int32_t *__restrict__ act,
               const float *__restrict__ y, int N, float inv_n, float *__restrict__ grad, float *__restrict__ loss) {
    __shared__ float sW[kPolParams];
    __shared__ float sX[kTile][F + 1];
    __shared__ float sH1[kTile][H + 1];
    __shared__ float sH2[kTile][H + 1];
    __shared__ float sD1[kTile][H + 1];  // d loss / d z1
    __shared__ float sD2[kTile][H + 1];  // d loss / d z2
    __shared__ float sDq[kTile];         // d loss / d q[a] of the sample
    __shared__ int sA[kTile];
    __shared__ float sLoss;
    const int t = threadIdx.x;
    const int base = blockIdx.x * kTile;
    for (int i = t; i < kPolParams; i += kThreads) sW[i] = theta[i];
    for (int i = t; i < kTile * F; i += kThreads) {
        const int s = i / F, f = i % F;
        sX[s][f] = base + s < N ? X[(int64_t)(base + s) * F + f] : 0.f;
    }
    if (t == 0) sLoss = 0.f;
    __syncthreads();
    if (t < kTile) {
        const int s = base + t;
        const bool valid = s < N;
        const int a = valid ? act[s] : 0;
        sA[t] = a;
        float h1[H], h2[H];
        uint32_t m1 = 0, m2 = 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float z = sW[ob1 + j];
#pragma unroll
            for (int i = 0; i < F; ++i) z = fmaf(sW[oW1 + j * F + i], sX[t][i], z);
            m1 |= (z > 0.f ? 1u : 0u) << j;
            h1[j] = z > 0.f ? z : 0.f;
            sH1[t][j] = h1[j];
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float z = sW[ob2 + j];
#pragma unroll
            for (int l = 0; l < H; ++l) z = fmaf(sW[oW2 + j * H + l], h1[l], z);
            m2 |= (z > 0.f ? 1u : 0u) << j;
            h2[j] = z > 0.f ? z : 0.f;
            sH2[t][j] = h2[j];
        }
        float q = sW[ob3 + a];
#pragma unroll
        for (int j = 0; j < H; ++j) q = fmaf(sW[oW3 + a * H + j], h2[j], q);
        const float r = valid ? q - y[s] : 0.f;
        const float dq = 2.f * r * inv_n;
        sDq[t] = dq;
        float d2[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            d2[j] = (m2 >> j & 1u) ? dq * sW[oW3 + a * H + j] : 0.f;
            sD2[t][j] = d2[j];
        }
#pragma unroll
        for (int l = 0; l < H; ++l) {
            float d = 0.f;
#pragma unroll
            for (int j = 0; j < H; ++j) d = fmaf(d2[j], sW[oW2 + j * H + l], d);
            sD1[t][l] = (m1 >> l & 1u) ? d : 0.f;
        }
        atomicAdd(&sLoss, r * r * inv_n);
    }
    __syncthreads();
    const int ns = min(kTile, N - base);
    for (int e = t; e < kPolParams; e += kThreads) {
        float acc = 0.f;
        if (e < ob1) {
            const int l = e / F, i = e % F;
            for (int s = 0; s < ns; ++s) acc = fmaf(sD1[s][l], sX[s][i], acc);
        } else if (e < oW2) {
            const int l = e - ob1;
            for (int s = 0; s < ns; ++s) acc += sD1[s][l];
        } else if (e < ob2) {
            const int j = (e - oW2) / H, l = (e - oW2) % H;
            for (int s = 0; s < ns; ++s) acc = fmaf(sD2[s][j], sH1[s][l], acc);
        } else if (e < oW3) {
            const int j = e - ob2;
            for (int s = 0; s < ns; ++s) acc += sD2[s][j];
        } else if (e < ob3) {
            const int k = (e - oW3) / H, j = (e - oW3) % H;
            for (int s = 0; s < ns; ++s)
                if (sA[s] == k) acc = fmaf(sDq[s], sH2[s][j], acc);
        } else {
            const int k = e - ob3;
            for (int s = 0; s < ns; ++s)
                if (sA[s] == k) acc += sDq[s];
        }
        if (acc != 0.f) atomicAdd(&grad[e], acc);
    }
    if (t == 0) atomicAdd(loss, sLoss);
}

// One thread per sample: all K outputs.
__global__ void k_mlp_forward(const float *__restrict__ theta, const float *__restrict__ X, int N,
                              float *__restrict__ Q) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    float x[F], h1[H], h2[H];
#pragma unroll
    for (int i = 0; i < F; ++i) x[i] = X[(int64_t)s * F + i];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float z = theta[ob1 + j];
#pragma unroll
        for (int i = 0; i < F; ++i) z = fmaf(theta[oW1 + j * F + i], x[i], z);
        h1[j] = z > 0.f ? z : 0.f;
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float z = theta[ob2 + j];
#pragma unroll
        for (int l = 0; l < H; ++l) z = fmaf(theta[oW2 + j * H + l], h1[l], z);
        h2[j] = z > 0.f ? z : 0.f;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float q = theta[ob3 + k];
#pragma unroll
        for (int j = 0; j < H; ++j) q = fmaf(theta[oW3 + k * H + j], h2[j], q);
        Q[(int64_t)s * K + k] = q;
    }
}

// Adam with bias correction (Kingma and Ba, 2015); t counts from 1.
__global__ void k_adam(float *__restrict__ theta, const float *__restrict__ grad, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = 0.9f * m[i] + 0.1f * g;
    const float vi = 0.999f * v[i] + 0.001f * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_fill_f32(float *p, int64_t count, float value) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_mlp_grad(const float *theta, const float *X, const int32_t *act, const float *y, int N,
                           float *grad, float *loss, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(8), dim3(256), 0, st, grad, (int64_t)kPolParams, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, st, loss, (int64_t)1, 0.f);
    const int blocks = (N + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(kThreads), 0, st, theta, X, act, y, N, 1.f / (float)N,
                       grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *theta, const float *X, int N, float *Q, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((N + 127) / 128), dim3(128), 0, st, theta, X, N, Q);
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int step, float lr, hipStream_t st) {
    const float c1 = 1.f - powf(0.9f, (float)step);
    const float c2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((kPolParams + 255) / 256), dim3(256), 0, st, theta, grad, m, v, kPolParams,
                       lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t count, float value, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t b = (count + 255) / 256;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)(b < 8192 ? b : 8192)), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

}  // namespace mf
