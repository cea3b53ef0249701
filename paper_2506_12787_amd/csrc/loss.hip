// L1 loss of the training objective (Sec. 4.4, the l1 term): mean |pred - target|
// and its gradient sign(pred - target) / n. Deterministic two-level reduction.
#include "runtime.h"

namespace swf {

namespace {

constexpr int kLossBlocks = 1024;

__global__ __launch_bounds__(256) void l1_partial_kernel(const float* __restrict__ pred,
                                                         const float* __restrict__ target, int64_t n, float inv_n,
                                                         float* __restrict__ grad, double* __restrict__ partial) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = pred[i] - target[i];
        s += fabs((double)d);
        if (grad) grad[i] = d > 0.f ? inv_n : (d < 0.f ? -inv_n : 0.f);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void l1_final_kernel(const double* __restrict__ partial, int m, double inv_n,
                                                       float* __restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(red[0] * inv_n);
}

}  // namespace

}  // namespace swf

using namespace swf;

extern "C" swf_status swf_l1_loss(swf_ctx* h, const float* pred, const float* target, int64_t n, float* loss,
                                  float* grad, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    if (n < 1 || !pred || !target || !loss) return c->fail(SWF_E_INVALID, "bad loss arguments");
    hipStream_t st = (hipStream_t)stream;
    swf_status s = c->ws.grad.reserve(c, kLossBlocks * sizeof(double), st);
    if (s) return s;
    const int blocks = (int)std::min<int64_t>(kLossBlocks, (n + 255) / 256);
    l1_partial_kernel<<<blocks, 256, 0, st>>>(pred, target, n, (float)(1.0 / (double)n), grad, (double*)c->ws.grad.ptr);
    l1_final_kernel<<<1, 256, 0, st>>>((const double*)c->ws.grad.ptr, blocks, 1.0 / (double)n, loss);
    return c->hip(hipGetLastError(), "l1 loss");
}
