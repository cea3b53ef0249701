// RSSI head (paper Sec. 7.2, RSSI case study): the rendered spectrum map is
// pooled by a global average over elevation and azimuth into one scalar per
// query, the received signal strength; its backward spreads the scalar's
// gradient evenly over the pixels and runs the render backward.
//
// The pooling is a deterministic two-level sum: one workgroup per query adds
// its H * W pixels in FP64 (fixed order: strided per thread, then a tree), so
// a query's value does not depend on the batch it was rendered in. It is an
// HBM-bound pass over the spectrum (4 B per pixel), negligible beside the
// render at the paper's 16 x 16 head and small at 90 x 360.
#include "runtime.h"

namespace swf {

namespace {

__global__ __launch_bounds__(256) void pool_mean_kernel(const float* __restrict__ spec, int64_t hw,
                                                        float* __restrict__ rssi) {
    __shared__ double red[256];
    const float* s = spec + (size_t)blockIdx.x * hw;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < hw; i += 256) acc += (double)s[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) rssi[blockIdx.x] = (float)(red[0] / (double)hw);
}

__global__ __launch_bounds__(256) void pool_grad_kernel(const float* __restrict__ grad_rssi, int64_t hw, int64_t n,
                                                        float inv_hw, float* __restrict__ grad_out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        grad_out[i] = grad_rssi[i / hw] * inv_hw;
}

}  // namespace

}  // namespace swf

using namespace swf;

extern "C" swf_status swf_render_rssi(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch, int32_t flags,
                                      float* rssi, float* out, void* aux, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    Scene* sc = c->scene(scene_id);
    if (!sc) return c->fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (!rssi) return c->fail(SWF_E_INVALID, "rssi is NULL");
    if (batch < 1) return c->fail(SWF_E_INVALID, "batch must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    const int64_t hw = (int64_t)sc->d.H * sc->d.W;
    if (!out) {
        swf_status s = c->ws.pool.reserve(c, (size_t)batch * hw * sizeof(float), st);
        if (s) return s;
        out = (float*)c->ws.pool.ptr;
    }
    swf_status s = c->render(c->ws, scene_id, tx, batch, flags, out, aux, st, 0, true);
    if (s) return s;
    pool_mean_kernel<<<batch, 256, 0, st>>>(out, hw, rssi);
    return c->hip(hipGetLastError(), "rssi pooling");
}

extern "C" swf_status swf_render_rssi_backward(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch,
                                               int32_t flags, const float* grad_rssi, const void* aux,
                                               const swf_grads* grads, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    Scene* sc = c->scene(scene_id);
    if (!sc) return c->fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (!grad_rssi) return c->fail(SWF_E_INVALID, "grad_rssi is NULL");
    if (batch < 1) return c->fail(SWF_E_INVALID, "batch must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    const int64_t hw = (int64_t)sc->d.H * sc->d.W;
    const int64_t n = (int64_t)batch * hw;
    swf_status s = c->ws.pool.reserve(c, (size_t)n * sizeof(float), st);
    if (s) return s;
    float* g = (float*)c->ws.pool.ptr;
    const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
    pool_grad_kernel<<<blocks, 256, 0, st>>>(grad_rssi, hw, n, (float)(1.0 / (double)hw), g);
    if ((s = c->hip(hipGetLastError(), "rssi gradient"))) return s;
    return c->backward(c->ws, scene_id, tx, batch, flags, g, aux, grads, st);
}
