// Backward pass orchestration (blend -> preprocess -> MLP) and its C ABI entry.
#include "runtime.h"

namespace swf {

swf_status Ctx::backward(Workspace& w, int sid, const float* tx, int B, int flags, const float* grad_out, const void* aux,
                         const swf_grads* gr, hipStream_t st) {
    if (!grad_out || !aux || !gr) return fail(SWF_E_INVALID, "grad_out, aux and grads are required");
    Scene* sc = scene(sid);
    if (!sc) return fail(SWF_E_NOT_FOUND, "unknown scene id");
    const DevScene& d = sc->d;
    const bool deform = !(flags & SWF_NO_DEFORM);
    // 1. the forward lists again (deterministic: identical to the forward's)
    swf_status s = forward_lists(w, sid, tx, B, flags & ~SWF_KEEP_AUX, st);
    if (s) return s;
    const int64_t P = (int64_t)B * d.n;
    const size_t npix = (size_t)B * d.H * d.W;
    const float* auxT = (const float*)aux;
    const uint32_t* auxL = (const uint32_t*)((const char*)aux + sizeof(float) * npix);
    // 2. blend backward -> per-pair gradients of (mean, M, opacity, amp)
    if ((s = w.dpair.reserve(this, (size_t)P * 8 * sizeof(float) + 16, st))) return s;
    if ((s = w.dbase.reserve(this, (size_t)P * kOut * sizeof(float) + 16, st))) return s;
    if ((s = hip(hipMemsetAsync(w.dpair.ptr, 0, (size_t)P * 8 * sizeof(float), st), "memset dpair"))) return s;
    launch_blend_backward((const uint2*)w.ranges.ptr, w.last.vals, w.rec, B, w.last.grid, grad_out, auxT, auxL,
                          (float*)w.dpair.ptr, st);
    // 3. preprocess backward -> residual-coordinate gradients
    const bool want_mlp = deform && d.has_mlp;
    float* dy = nullptr;
    if (want_mlp) {
        if ((s = w.dy.reserve(this, (size_t)P * kOut * sizeof(float) + 16, st))) return s;
        dy = (float*)w.dy.ptr;
    }
    launch_preprocess_backward((const float*)w.dpair.ptr, w.rec, P, (flags & SWF_PAPER_DEFORM) != 0,
                               (float*)w.dbase.ptr, dy, st);
    // 4. MLP backward (FP32, activations recomputed)
    float* dmu = nullptr;
    if (want_mlp) {
        const int nh = d.n_hidden;
        const size_t actb = (size_t)P * 256 * sizeof(float);
        if ((s = w.act.reserve(this, actb * nh + 16, st))) return s;
        if ((s = w.dz.reserve(this, actb * 2 + 16, st))) return s;
        if ((s = w.part.reserve(this, (size_t)wgrad_chunks(P) * 256 * 256 * sizeof(float) + 16, st))) return s;
        if ((s = w.fmean.reserve(this, (size_t)d.n * kMeanFeat * sizeof(float) + 16, st))) return s;
        if ((s = w.ftx.reserve(this, (size_t)B * kTxFeat * sizeof(float) + 16, st))) return s;
        if ((s = w.dmu.reserve(this, (size_t)d.n * 2 * sizeof(float) + 16, st))) return s;
        if ((s = w.qs.reserve(this, (size_t)B * d.hidden * sizeof(float), st))) return s;
        float* act[8] = {};
        for (int l = 0; l < nh; ++l) act[l] = (float*)((char*)w.act.ptr + actb * l);
        launch_tx_features(d, tx, B, (float*)w.qs.ptr, st, (float*)w.ftx.ptr);
        const Grid g = w.last.grid;
        Records none;
        launch_mlp_fp32(d, (const float*)w.qs.ptr, B, g, false, none, nullptr, st, act);
        launch_mean_features_f32(d, (float*)w.fmean.ptr, st);
        float* dz[2] = {(float*)w.dz.ptr, (float*)((char*)w.dz.ptr + actb)};
        float* part = (float*)w.part.ptr;
        // output layer
        launch_wgrad(dy, kOut, act[nh - 1], 256, nullptr, nullptr, d.n, P, part, gr->weight[nh], gr->bias[nh], st);
        launch_dgrad(dy, kOut, d.w[nh], act[nh - 1], P, dz[0], st);
        int cur = 0;
        for (int l = nh - 1; l >= 1; --l) {
            launch_wgrad(dz[cur], 256, act[l - 1], 256, nullptr, nullptr, d.n, P, part, gr->weight[l], gr->bias[l], st);
            launch_dgrad(dz[cur], 256, d.w[l], act[l - 1], P, dz[cur ^ 1], st);
            cur ^= 1;
        }
        launch_wgrad(dz[cur], 256, nullptr, d.in_dim, (const float*)w.fmean.ptr, (const float*)w.ftx.ptr, d.n, P,
                     part, gr->weight[0], gr->bias[0], st);
        launch_pe_backward(dz[cur], d, B, (float*)w.dmu.ptr, st);
        dmu = (float*)w.dmu.ptr;
    }
    // 5. base parameters: sum over the batch, original ids
    float* outs[kOut] = {gr->mean_x, gr->mean_y, gr->log_scale_x, gr->log_scale_y, gr->rotation, gr->opacity_logit,
                         gr->amplitude};
    if ((s = w.ptrs.reserve(this, sizeof(outs), st))) return s;
    if ((s = hip(hipMemcpyAsync(w.ptrs.ptr, outs, sizeof(outs), hipMemcpyHostToDevice, st), "ptrs H2D"))) return s;
    launch_base_reduce((const float*)w.dbase.ptr, dmu, d.perm, B, d.n, (float* const*)w.ptrs.ptr, st);
    if ((s = hip(hipStreamSynchronize(st), "backward sync"))) return s;  // `outs` lives on this stack
    return hip(hipGetLastError(), "backward launch");
}

}  // namespace swf

using namespace swf;

extern "C" swf_status swf_render_backward(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch, int32_t flags,
                                          const float* grad_out, const void* aux, const swf_grads* grads,
                                          void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    return c->backward(c->ws, scene_id, tx, batch, flags, grad_out, aux, grads, (hipStream_t)stream);
}
