// Training-loop steps of the paper's protocol (Sec. 4.4) that run on the
// device beside the render, loss and backward:
//  * the Adam update of every parameter tensor in one launch (the paper trains
//    the Gaussians at learning rate 1e-2 and the MLP at 8e-3, hyperparameter
//    table; Adam's moment decays and epsilon are not given: the defaults of
//    Kingma and Ba, 0.9, 0.999, 1e-8, are the caller's to pass);
//  * anneal smoothing (Sec. 4.4, anneal-smoothing equations): the moving
//    position is perturbed by gamma * n * (2 / cbrt(N_s)) * (1 - i / tau) with
//    n a standard 3D normal draw, in the unit cube the positions are
//    normalised to, i.e. scaled by the room's extent in metres. The factor is
//    clamped at 0 once i passes tau (the printed linear decay would change
//    sign there).
#include <math.h>

#include "runtime.h"

namespace swf {

namespace {

constexpr int kMaxAdam = 32;

struct AdamArgs {
    float* p[kMaxAdam];
    const float* g[kMaxAdam];
    float* m[kMaxAdam];
    float* v[kMaxAdam];
    int64_t n[kMaxAdam];
    float lr[kMaxAdam];
    int count;
    float b1, b2, eps, c1, c2;  // c1 = 1 / (1 - b1^t), c2 = 1 / sqrt(1 - b2^t)
};

// Block (x, tensor y): grid-stride over tensor y's elements.
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    const int k = blockIdx.y;
    const int64_t n = a.n[k];
    float* __restrict__ p = a.p[k];
    const float* __restrict__ g = a.g[k];
    float* __restrict__ m = a.m[k];
    float* __restrict__ v = a.v[k];
    const float lr = a.lr[k];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = fmaf(a.b1, m[i], (1.0f - a.b1) * gi);
        const float vi = fmaf(a.b2, v[i], (1.0f - a.b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        // p -= lr * m_hat / (sqrt(v_hat) + eps), m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t)
        p[i] -= lr * (mi * a.c1) / (sqrtf(vi) * a.c2 + a.eps);
    }
}

__global__ void anneal_kernel(const float* __restrict__ tx, const float* __restrict__ noise, int B, float3 scale,
                              float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B) return;
    out[3 * i] = fmaf(scale.x, noise[3 * i], tx[3 * i]);
    out[3 * i + 1] = fmaf(scale.y, noise[3 * i + 1], tx[3 * i + 1]);
    out[3 * i + 2] = fmaf(scale.z, noise[3 * i + 2], tx[3 * i + 2]);
}

}  // namespace

}  // namespace swf

using namespace swf;

extern "C" swf_status swf_adam_step(swf_ctx* h, float* const* params, const float* const* grads, float* const* m,
                                    float* const* v, const int64_t* sizes, const float* lrs, int32_t count,
                                    float beta1, float beta2, float eps, int32_t step, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    if (count < 0 || count > kMaxAdam) return c->fail(SWF_E_INVALID, "count must be in [0, 32]");
    if (step < 1) return c->fail(SWF_E_INVALID, "step must be >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
        return c->fail(SWF_E_INVALID, "betas must be in [0, 1) and eps > 0");
    if (count && (!params || !grads || !m || !v || !sizes || !lrs)) return c->fail(SWF_E_INVALID, "null array");
    AdamArgs a{};
    int64_t nmax = 0;
    for (int k = 0; k < count; ++k) {
        if (sizes[k] < 0 || (sizes[k] > 0 && (!params[k] || !grads[k] || !m[k] || !v[k])))
            return c->fail(SWF_E_INVALID, "bad tensor entry");
        a.p[k] = params[k];
        a.g[k] = grads[k];
        a.m[k] = m[k];
        a.v[k] = v[k];
        a.n[k] = sizes[k];
        a.lr[k] = lrs[k];
        nmax = std::max(nmax, sizes[k]);
    }
    if (count == 0 || nmax == 0) return SWF_OK;
    a.count = count;
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
    a.c2 = (float)(1.0 / sqrt(1.0 - pow((double)beta2, (double)step)));
    const int bx = (int)std::min<int64_t>(1024, (nmax + 255) / 256);
    adam_kernel<<<dim3((unsigned)bx, (unsigned)count), 256, 0, (hipStream_t)stream>>>(a);
    return c->hip(hipGetLastError(), "adam");
}

extern "C" swf_status swf_anneal_tx(swf_ctx* h, const float* tx, const float* noise, int32_t batch, int32_t iter,
                                    float gamma, int32_t tau, int32_t n_positions, const float* room_lo,
                                    const float* room_hi, float* tx_out, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    if (batch < 1 || !tx || !noise || !tx_out || !room_lo || !room_hi || tau < 1 || n_positions < 1 || iter < 0 ||
        !isfinite(gamma))
        return c->fail(SWF_E_INVALID, "bad anneal arguments");
    const double decay = std::max(0.0, 1.0 - (double)iter / (double)tau);
    const double f = (double)gamma * 2.0 / std::cbrt((double)n_positions) * decay;
    const float3 scale = make_float3((float)(f * (room_hi[0] - room_lo[0])), (float)(f * (room_hi[1] - room_lo[1])),
                                     (float)(f * (room_hi[2] - room_lo[2])));
    anneal_kernel<<<(batch + 255) / 256, 256, 0, (hipStream_t)stream>>>(tx, noise, batch, scale, tx_out);
    return c->hip(hipGetLastError(), "anneal");
}
