// C-ABI of the learned phase schedule's value network (mf_policy_* in
// include/mf.h): parameter storage on the device, seeded initialisation,
// forward / gradient / training calls that run the kernels of mf_policy.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mf.h"
#include "mf_internal.h"

namespace {

thread_local std::string g_policy_error;

int pfail(int code, const std::string &msg) {
    g_policy_error = msg;
    return code;
}

#define PHIP(expr)                                                                      \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) return pfail(MF_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
    } while (0)

// splitmix64 (Steele, Lea and Flood, 2014): the counter-based generator of the
// initial weights.
uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

double unit(uint64_t seed, uint64_t i) {  // uniform in (0, 1)
    return ((double)(splitmix64(seed ^ splitmix64(i)) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

}  // namespace

struct mf_policy {
    int device = 0;
    hipStream_t stream = nullptr;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
    float *X = nullptr, *Y = nullptr, *Q = nullptr;
    int32_t *A = nullptr;
    int64_t cap = 0;  // samples the staging buffers hold
    int64_t steps = 0;
};

namespace {

void release(mf_policy_t *p) {
    if (mf::process_exiting()) return;
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    for (void *q : {(void *)p->theta, (void *)p->grad, (void *)p->m, (void *)p->v, (void *)p->loss, (void *)p->X,
                    (void *)p->Y, (void *)p->Q, (void *)p->A})
        if (q) (void)hipFree(q);
    if (p->stream) (void)hipStreamDestroy(p->stream);
}

int stage(mf_policy_t *p, const float *X, const int32_t *a, const float *y, int32_t N) {
    if (N > p->cap) {
        for (void *q : {(void *)p->X, (void *)p->Y, (void *)p->Q, (void *)p->A})
            if (q) (void)hipFree(q);
        p->X = p->Y = p->Q = nullptr;
        p->A = nullptr;
        p->cap = 0;
        PHIP(hipMalloc(&p->X, sizeof(float) * mf::kPolF * (size_t)N));
        PHIP(hipMalloc(&p->Y, sizeof(float) * (size_t)N));
        PHIP(hipMalloc(&p->Q, sizeof(float) * mf::kPolK * (size_t)N));
        PHIP(hipMalloc(&p->A, sizeof(int32_t) * (size_t)N));
        p->cap = N;
    }
    PHIP(hipMemcpyAsync(p->X, X, sizeof(float) * mf::kPolF * (size_t)N, hipMemcpyHostToDevice, p->stream));
    if (a) PHIP(hipMemcpyAsync(p->A, a, sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice, p->stream));
    if (y) PHIP(hipMemcpyAsync(p->Y, y, sizeof(float) * (size_t)N, hipMemcpyHostToDevice, p->stream));
    return MF_OK;
}

int check_samples(const float *X, const int32_t *a, const float *y, int32_t N) {
    if (N < 1) return pfail(MF_EINVAL, "N must be >= 1");
    if (!X || !a || !y) return pfail(MF_EINVAL, "null sample arrays");
    for (int32_t i = 0; i < N; ++i) {
        if (a[i] < 0 || a[i] >= mf::kPolK) return pfail(MF_EINVAL, "action out of range");
        if (!std::isfinite(y[i])) return pfail(MF_EINVAL, "non-finite target");
    }
    for (int64_t i = 0; i < (int64_t)N * mf::kPolF; ++i)
        if (!std::isfinite(X[i])) return pfail(MF_EINVAL, "non-finite feature");
    return MF_OK;
}

}  // namespace

extern "C" {

MF_API const char *mf_policy_last_error(void) { return g_policy_error.c_str(); }

MF_API int32_t mf_policy_num_params(void) { return mf::kPolParams; }

MF_API int mf_policy_create(int32_t device, uint64_t seed, mf_policy_t **out) {
    if (!out) return pfail(MF_EINVAL, "out is NULL");
    *out = nullptr;
    if (device < 0) return pfail(MF_EINVAL, "device must be >= 0");
    PHIP(hipSetDevice(device));
    mf_policy_t *p = new (std::nothrow) mf_policy_t();
    if (!p) return pfail(MF_ENOMEM, "host allocation failed");
    p->device = device;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipMalloc(&p->theta, sizeof(float) * mf::kPolParams)) != hipSuccess ||
        (e = hipMalloc(&p->grad, sizeof(float) * mf::kPolParams)) != hipSuccess ||
        (e = hipMalloc(&p->m, sizeof(float) * mf::kPolParams)) != hipSuccess ||
        (e = hipMalloc(&p->v, sizeof(float) * mf::kPolParams)) != hipSuccess ||
        (e = hipMalloc(&p->loss, sizeof(float))) != hipSuccess) {
        release(p);
        delete p;
        return pfail(MF_ENOMEM, std::string("policy buffers: ") + hipGetErrorString(e));
    }
    // He initialisation: weights N(0, 2 / fan_in) by Box-Muller over the
    // counter-based uniforms, biases 0
    std::vector<float> w(mf::kPolParams, 0.f);
    const int F = mf::kPolF, H = mf::kPolH, K = mf::kPolK;
    const int layer_off[3] = {0, H * F + H, H * F + H + H * H + H};
    const int layer_n[3] = {H * F, H * H, K * H};
    const int fan_in[3] = {F, H, H};
    uint64_t ctr = 0;
    for (int l = 0; l < 3; ++l) {
        const double sd = std::sqrt(2.0 / fan_in[l]);
        for (int i = 0; i < layer_n[l]; ++i, ctr += 2) {
            const double u1 = unit(seed, ctr), u2 = unit(seed, ctr + 1);
            w[layer_off[l] + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    }
    if ((e = hipMemcpy(p->theta, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = mf::launch_fill_f32(p->m, mf::kPolParams, 0.f, p->stream)) != hipSuccess ||
        (e = mf::launch_fill_f32(p->v, mf::kPolParams, 0.f, p->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(p->stream)) != hipSuccess) {
        release(p);
        delete p;
        return pfail(MF_EDEVICE, std::string("policy init: ") + hipGetErrorString(e));
    }
    *out = p;
    return MF_OK;
}

MF_API void mf_policy_destroy(mf_policy_t *p) {
    if (!p) return;
    release(p);
    delete p;
}

MF_API int mf_policy_get_params(mf_policy_t *p, float *out) {
    if (!p || !out) return pfail(MF_EINVAL, "null argument");
    PHIP(hipSetDevice(p->device));
    PHIP(hipMemcpyAsync(out, p->theta, sizeof(float) * mf::kPolParams, hipMemcpyDeviceToHost, p->stream));
    PHIP(hipStreamSynchronize(p->stream));
    return MF_OK;
}

MF_API int mf_policy_set_params(mf_policy_t *p, const float *in) {
    if (!p || !in) return pfail(MF_EINVAL, "null argument");
    for (int i = 0; i < mf::kPolParams; ++i)
        if (!std::isfinite(in[i])) return pfail(MF_EINVAL, "non-finite parameter");
    PHIP(hipSetDevice(p->device));
    PHIP(hipMemcpyAsync(p->theta, in, sizeof(float) * mf::kPolParams, hipMemcpyHostToDevice, p->stream));
    PHIP(mf::launch_fill_f32(p->m, mf::kPolParams, 0.f, p->stream));
    PHIP(mf::launch_fill_f32(p->v, mf::kPolParams, 0.f, p->stream));
    PHIP(hipStreamSynchronize(p->stream));
    p->steps = 0;
    return MF_OK;
}

MF_API int mf_policy_forward(mf_policy_t *p, const float *X, int32_t N, float *Q) {
    if (!p || !X || !Q) return pfail(MF_EINVAL, "null argument");
    if (N < 1) return pfail(MF_EINVAL, "N must be >= 1");
    PHIP(hipSetDevice(p->device));
    int rc = stage(p, X, nullptr, nullptr, N);
    if (rc) return rc;
    PHIP(mf::launch_mlp_forward(p->theta, p->X, N, p->Q, p->stream));
    PHIP(hipMemcpyAsync(Q, p->Q, sizeof(float) * mf::kPolK * (size_t)N, hipMemcpyDeviceToHost, p->stream));
    PHIP(hipStreamSynchronize(p->stream));
    return MF_OK;
}

MF_API int mf_policy_gradient(mf_policy_t *p, const float *X, const int32_t *actions, const float *targets,
                              int32_t N, float *grad, float *loss) {
    if (!p || !grad || !loss) return pfail(MF_EINVAL, "null argument");
    int rc = check_samples(X, actions, targets, N);
    if (rc) return rc;
    PHIP(hipSetDevice(p->device));
    rc = stage(p, X, actions, targets, N);
    if (rc) return rc;
    PHIP(mf::launch_mlp_grad(p->theta, p->X, p->A, p->Y, N, p->grad, p->loss, p->stream));
    PHIP(hipMemcpyAsync(grad, p->grad, sizeof(float) * mf::kPolParams, hipMemcpyDeviceToHost, p->stream));
    PHIP(hipMemcpyAsync(loss, p->loss, sizeof(float), hipMemcpyDeviceToHost, p->stream));
    PHIP(hipStreamSynchronize(p->stream));
    return MF_OK;
}

MF_API int mf_policy_train(mf_policy_t *p, const float *X, const int32_t *actions, const float *targets, int32_t N,
                           int32_t steps, float lr, float *final_loss) {
    if (!p) return pfail(MF_EINVAL, "null policy");
    if (steps < 1) return pfail(MF_EINVAL, "steps must be >= 1");
    if (!(lr > 0.f) || !std::isfinite(lr)) return pfail(MF_EINVAL, "lr must be positive");
    int rc = check_samples(X, actions, targets, N);
    if (rc) return rc;
    PHIP(hipSetDevice(p->device));
    rc = stage(p, X, actions, targets, N);
    if (rc) return rc;
    for (int32_t s = 0; s < steps; ++s) {
        PHIP(mf::launch_mlp_grad(p->theta, p->X, p->A, p->Y, N, p->grad, p->loss, p->stream));
        PHIP(mf::launch_adam(p->theta, p->grad, p->m, p->v, (int)(++p->steps), lr, p->stream));
    }
    // loss of the trained parameters
    PHIP(mf::launch_mlp_grad(p->theta, p->X, p->A, p->Y, N, p->grad, p->loss, p->stream));
    if (final_loss)
        PHIP(hipMemcpyAsync(final_loss, p->loss, sizeof(float), hipMemcpyDeviceToHost, p->stream));
    PHIP(hipStreamSynchronize(p->stream));
    return MF_OK;
}

}  // extern "C"

namespace mf {
const float *policy_device_params(const mf_policy_t *p) { return p ? p->theta : nullptr; }
int policy_device(const mf_policy_t *p) { return p ? p->device : -1; }
}  // namespace mf
