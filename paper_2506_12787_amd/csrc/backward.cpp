// Backward pass orchestration (blend -> preprocess -> MLP) and its C ABI entry.
#include <algorithm>

#include "runtime.h"

namespace swf {

// MLP backward, every GEMM in this library's own kernels. The hidden
// activations are the ones the forward's MLP kernel stored (the values the
// forward used: FP32, or BF16 after a BF16 forward). From dy (gradients of the
// 7 residuals per pair):
//   dW_l = dz_l^T act_{l-1}, db_l = colsum(dz_l), dz_{l-1} = (dz_l W_l) * [act_{l-1} > 0],
// and for layer 1 the weight gradient splits into the mean part
// (sum over queries of dz_0 per Gaussian = S)^T gamma(mu_hat) and the TX part
// (sum over Gaussians of dz_0 per query)^T gamma(s_hat); the mean features'
// gradient is S W1m, taken through the sin / cos features to d mu.
// bf16: the backward of a BF16 forward. dz is stored in BF16 (FP32 sums, then
// one rounding) and the 256 x 256 products run on BF16 matrix cores with FP32
// accumulation; FP32: the products run on the FP32 matrix cores (gemm.hip).
// Weight and bias gradients are accumulated in FP32 either way.
swf_status Ctx::mlp_backward(Workspace& w, const DevScene& d, const float* tx, int B, const float* dy,
                             const swf_grads* gr, bool bf16, hipStream_t st) {
    swf_status s = SWF_OK;
    const int64_t N = d.n, P = (int64_t)B * N;
    const int nh = d.n_hidden, Hd = 256, I = d.in_dim;
    const size_t esz = bf16 ? 2 : 4;                 // activation / dz element size
    const size_t actb = (size_t)P * Hd * esz;
    const size_t f32b = (size_t)P * Hd * sizeof(float);
    if (!w.act.ptr || w.act.cap < actb * nh) return fail(SWF_E_STATE, "the forward's activations are missing");
    // dz ping-pong; BF16 with a single hidden layer: also the FP32 layer-1 gradient (formed inside its sums)
    const bool need_zf = bf16 && nh == 1;
    if ((s = w.dz.reserve(this, need_zf ? actb * 2 + f32b + 16 : actb * 2 + 16, st))) return s;
    // scratch: S (N x 256), R (B x 256), dg (N x 26), split-K partials, column-sum partials, BF16 weights
    const size_t n_split = std::max({gemm_part_floats(Hd, Hd, P), gemm_part_floats(kOut, Hd, P),
                                     gemm_part_floats(Hd, kMeanFeat, N), gemm_part_floats(Hd, kTxFeat, B),
                                     (size_t)layer1_sums_blocks((int)N) * B * Hd,
                                     (size_t)layer1_grad_blocks((int)N) * B * Hd,
                                     (size_t)wgrad_mfma_blocks(P) * (Hd * Hd + Hd),
                                     (size_t)wgrad_out_blocks(P) * kOut * Hd, (size_t)dz_f32_blocks(P) * Hd});
    const size_t n_cs = std::max<size_t>({(size_t)colsum_blocks(P) * Hd, (size_t)colsum_blocks(B) * N * Hd,
                                          (size_t)colsum_blocks(N) * Hd * B,
                                          (size_t)colsum_blocks(wgrad_mfma_blocks(P)) * (Hd * Hd + Hd),
                                          (size_t)colsum_blocks(wgrad_out_blocks(P)) * kOut * Hd});
    const size_t n_wb = bf16 ? ((size_t)(nh - 1) * Hd * Hd + (size_t)kOut * Hd + (size_t)P * kOut + 64) / 2 + 64 : 0;
    const size_t n_wt = bf16 ? 0 : (size_t)(nh - 1) * Hd * Hd;  // FP32: W^T of the 256 x 256 layers, fragment-major
    const size_t small =
        ((size_t)N * Hd + (size_t)B * Hd + (size_t)N * kMeanFeat + 4 + n_split + n_cs + n_wb + n_wt + 64) *
        sizeof(float);
    if ((s = w.part.reserve(this, small, st))) return s;
    if ((s = w.fmean.reserve(this, (size_t)N * kMeanFeat * sizeof(float) + 16, st))) return s;
    if ((s = w.ftx.reserve(this, (size_t)B * kTxFeat * sizeof(float) + 16, st))) return s;
    if ((s = w.dmu.reserve(this, (size_t)N * 2 * sizeof(float) + 16, st))) return s;
    if ((s = w.qs.reserve(this, (size_t)B * Hd * sizeof(float), st))) return s;
    void* act[8] = {};
    for (int l = 0; l < nh; ++l) act[l] = (char*)w.act.ptr + actb * l;
    void* dz[2] = {w.dz.ptr, (char*)w.dz.ptr + actb};
    float* zf = need_zf ? (float*)((char*)w.dz.ptr + actb * 2) : nullptr;  // FP32 layer-1 gradient (nh == 1)
    float* S = (float*)w.part.ptr;               // N x 256
    float* R = S + (size_t)N * Hd;               // B x 256
    float* dg = R + (size_t)B * Hd;              // N x 26
    float* part = dg + ((size_t)N * kMeanFeat + 3) / 4 * 4;  // split-K partials (16-byte aligned)
    float* tmp = part + n_split;                 // column-sum partials
    uint16_t* wb = (uint16_t*)(tmp + n_cs);      // BF16 weights: hidden layers 1.., output, then dy
    float* wt = (float*)(((uintptr_t)(tmp + n_cs + n_wb) + 15) & ~(uintptr_t)15);  // FP32 W^T, 16-byte aligned
    float* fmean = (float*)w.fmean.ptr, *ftx = (float*)w.ftx.ptr, *qs = (float*)w.qs.ptr;
    launch_tx_features(d, tx, B, qs, st, ftx);
    launch_mean_features_f32(d, fmean, st);
    uint16_t* wl[8] = {};
    uint16_t* dyb = nullptr;
    if (bf16) {
        for (int l = 1; l < nh; ++l) {
            wl[l] = wb + (size_t)(l - 1) * Hd * Hd;
            launch_to_bf16(d.w[l], (int64_t)Hd * Hd, wl[l], st);
        }
        wl[nh] = wb + (size_t)(nh - 1) * Hd * Hd;
        launch_to_bf16(d.w[nh], (int64_t)kOut * Hd, wl[nh], st);
        if (nh == 1) {  // the single-hidden-layer path multiplies BF16 dy by the BF16 output weights
            dyb = wl[nh] + (size_t)kOut * Hd;
            launch_to_bf16(dy, P * kOut, dyb, st);
        }
    } else {
        for (int l = 1; l < nh; ++l) launch_pack_wt(d.w[l], wt + (size_t)(l - 1) * Hd * Hd, st);
    }
    // ---- output layer (7 outputs)
    if (bf16) {
        // one pass over the last activations: the weight gradient and, with more than one hidden layer, the
        // masked BF16 gradient of the last hidden pre-activations (K = 7)
        launch_out_bwd_bf16(dy, wl[nh], act[nh - 1], P, nh > 1 ? dz[0] : nullptr, part, tmp, gr->weight[nh], st);
    } else if (gr->weight[nh]) {
        launch_gemm_f32(true, false, kOut, Hd, P, dy, kOut, act[nh - 1], Hd, gr->weight[nh], Hd, part, st);
    }
    if (gr->bias[nh]) launch_colsum(dy, P, kOut, 1, 0, tmp, gr->bias[nh], 0, st);
    if (bf16) {
        if (nh == 1)  // the layer-1 gradient before its ReLU mask (applied inside its sums below)
            launch_gemm_f32(false, false, P, Hd, kOut, dyb, kOut, wl[nh], Hd, zf, Hd, part, st, nullptr, 0, true);
    } else {
        launch_gemm_f32(false, false, P, Hd, kOut, dy, kOut, d.w[nh], Hd, (float*)dz[0], Hd, part, st,
                        (const float*)act[nh - 1], Hd);
    }
    int cur = 0;
    const void* dz1 = nullptr;  // BF16: the second layer's pre-activation gradient
    for (int l = nh - 1; l >= 1; --l) {
        if (gr->weight[l]) {
            if (bf16)  // contraction over pairs; the bias gradient (column sums of dz) rides along
                launch_wgrad_mfma(dz[cur], act[l - 1], P, part, tmp, gr->weight[l], gr->bias[l], st);
            else
                launch_gemm_f32(true, false, Hd, Hd, P, dz[cur], Hd, act[l - 1], Hd, gr->weight[l], Hd, part, st);
        }
        if (bf16 && gr->bias[l] && !gr->weight[l]) launch_colsum_bf16(dz[cur], P, Hd, 1, 0, tmp, gr->bias[l], 0, st);
        if (bf16) {
            // dz W on MFMA in one pass, BF16 and masked by the previous ReLU; the layer-1 gradient is formed
            // inside its sums below
            if (l > 1)
                launch_dz_gemm(dz[cur], wl[l], act[l - 1], P, dz[cur ^ 1], false, st);
            else
                dz1 = dz[cur];
        } else {
            // the input gradient on the FP32 matrix cores with the layer's W^T as register-fed weights, masked;
            // the bias gradient's per-block column sums of dz ride along (into the split-K space, free again)
            float* bp = gr->bias[l] ? part : nullptr;
            launch_dz_f32((const float*)dz[cur], wt + (size_t)(l - 1) * Hd * Hd, (const float*)act[l - 1], P,
                          (float*)dz[cur ^ 1], bp, st);
            if (bp) launch_colsum(bp, dz_f32_blocks(P), Hd, 1, 0, tmp, gr->bias[l], 0, st);
        }
        cur ^= 1;
    }
    // ---- layer 1: the gradient of its pre-activations dz0, FP32; S = its sum over the batch per Gaussian
    // (N x 256), R = its sum over the Gaussians per query (B x 256), b0 = its sum over all pairs
    if (bf16) {
        if (dz1) {
            // dz0 = (dz1 W1) masked, never stored: one pass gives S and per-block partial sums of R
            launch_layer1_grad(dz1, wl[1], act[0], (int)B, (int)N, S, part, st);
            if (gr->weight[0]) launch_colsum(part, layer1_grad_blocks((int)N), B * Hd, 1, 0, tmp, R, 0, st);
        } else {
            // one hidden layer: zf is dz0 before the ReLU mask
            launch_layer1_sums(zf, act[0], (int)B, (int)N, S, part, st);
            if (gr->weight[0]) launch_colsum(part, layer1_sums_blocks((int)N), B * Hd, 1, 0, tmp, R, 0, st);
        }
    } else {
        // dz0 carries layer 1's ReLU mask already (applied where it was formed): one pass gives S and per-block
        // partial sums of R
        launch_layer1_sums((const float*)dz[cur], nullptr, (int)B, (int)N, S, part, st);
        if (gr->weight[0]) launch_colsum(part, layer1_sums_blocks((int)N), B * Hd, 1, 0, tmp, R, 0, st);
    }
    if (gr->bias[0]) launch_colsum(S, N, Hd, 1, 0, tmp, gr->bias[0], 0, st);  // b0: the sum of S over Gaussians
    if (gr->weight[0]) {
        // dW1 [256 x 89] = [S^T gamma(mu_hat) | R^T gamma(s_hat)]
        launch_gemm_f32(true, false, Hd, kMeanFeat, N, S, Hd, fmean, kMeanFeat, gr->weight[0], I, part, st);
        launch_gemm_f32(true, false, Hd, kTxFeat, B, R, Hd, ftx, kTxFeat, gr->weight[0] + kMeanFeat, I, part, st);
    }
    // d gamma(mu_hat) = S W1m (N x 26), then through the features to d mu
    launch_gemm_f32(false, false, N, kMeanFeat, Hd, S, Hd, d.w[0], I, dg, kMeanFeat, part, st);
    launch_pe_chain(dg, d, (float*)w.dmu.ptr, st);
    return hip(hipGetLastError(), "mlp backward");
}

swf_status Ctx::backward(Workspace& w, int sid, const float* tx, int B, int flags, const float* grad_out, const void* aux,
                         const swf_grads* gr, hipStream_t st) {
    if (!grad_out || !aux || !gr) return fail(SWF_E_INVALID, "grad_out, aux and grads are required");
    Scene* sc = scene(sid);
    if (!sc) return fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (sc->d.kind == 1) return fail(SWF_E_INVALID, "paper-model scenes have no backward in this library");
    AuxTag t;
    {
        // the forward state used below must be that of the render that filled aux
        auto it = aux_tags.find(aux);
        if (it == aux_tags.end())
            return fail(SWF_E_STATE, "aux was not filled by a swf_render with SWF_KEEP_AUX on this context");
        t = it->second;
        if (t.scene != sid || t.B != B || t.flags != (flags & ~(SWF_KEEP_AUX | SWF_DETERMINISTIC)))
            return fail(SWF_E_INVALID, "scene, batch or flags differ from the render that filled aux");
        if (t.gen != sc->gen)
            return fail(SWF_E_STATE, "the scene's parameters were updated after the render that filled aux");
    }
    const DevScene& d = sc->d;
    const bool deform = !(flags & SWF_NO_DEFORM);
    const bool want_mlp = deform && d.has_mlp;
    // The MLP backward takes the hidden activations the forward's MLP kernel stored (the values the forward
    // used, FP32 or BF16).
    const bool bf16 = (flags & SWF_MLP_BF16) != 0;
    const bool acts_ready = want_mlp && B >= 1 && (uint64_t)B * (uint64_t)d.n < (1ull << 32);
    if (want_mlp && !acts_ready) return fail(SWF_E_INVALID, "the MLP backward takes fewer than 2^32 pairs");
    swf_status s = SWF_OK;
    // 1. the forward's records and lists: still in the workspace if no pass wrote records since that render
    // (and it was given the same positions), else built again (deterministic: identical to the forward's)
    const bool kept = t.seq == w.seq && t.tx == tx && (!acts_ready || t.acts);
    if (!kept) {
        if (acts_ready) {
            const size_t actb = (size_t)B * d.n * 256 * (bf16 ? sizeof(uint16_t) : sizeof(float));
            if ((s = w.act.reserve(this, actb * d.n_hidden + 16, st))) return s;
            w.act_out = w.act.ptr;
        }
        s = forward_lists(w, sid, tx, B, flags & ~(SWF_KEEP_AUX | SWF_DETERMINISTIC), st);
        w.act_out = nullptr;
        if (s) return s;
    }
    last_bwd_reused = kept;
    const int64_t P = (int64_t)B * d.n;
    const size_t npix = (size_t)B * d.H * d.W;
    const float* auxT = (const float*)aux;
    const uint32_t* auxL = (const uint32_t*)((const char*)aux + sizeof(float) * npix);
    // 2. blend backward -> per-pair gradients of (mean, M, opacity, amp)
    if ((s = w.dpair.reserve(this, (size_t)P * 8 * sizeof(float) + 16, st))) return s;
    if ((s = w.dbase.reserve(this, (size_t)P * kOut * sizeof(float) + 16, st))) return s;
    if ((s = hip(hipMemsetAsync(w.dpair.ptr, 0, (size_t)P * 8 * sizeof(float), st), "memset dpair"))) return s;
    stage_begin(SWF_STAGE_BWD_BLEND, st);
    float* det_part = nullptr;
    const uint32_t* det_off = nullptr;
    if (flags & SWF_DETERMINISTIC) {
        // per (list entry, wave) sums, zero where a wave contributes nothing, stored per pair: a pair's entries
        // from its first slot on (the exclusive scan of the key counts), in the row-major order of its tiles
        const size_t db = (size_t)w.last.n_keys * 32 * sizeof(float);
        if ((s = w.det.reserve(this, db + 16, st))) return s;
        if (db && (s = hip(hipMemsetAsync(w.det.ptr, 0, db, st), "memset entry sums"))) return s;
        det_part = (float*)w.det.ptr;
        const size_t ob = ((size_t)P * sizeof(uint32_t) + 7) / 8 * 8;
        if ((s = w.off.reserve(this, ob + 16, st))) return s;
        if ((s = w.scan.reserve(this, scan_scratch_bytes(P) + 64, st))) return s;
        launch_exclusive_scan(w.rec.count, (uint32_t*)w.off.ptr, (uint64_t*)((char*)w.off.ptr + ob), P, w.scan.ptr,
                              st);
        det_off = (const uint32_t*)w.off.ptr;
    }
    launch_blend_backward((const uint2*)w.ranges.ptr, w.last.vals, w.rec, B, w.last.grid, grad_out, auxT, auxL,
                          (float*)w.dpair.ptr, st, det_part, d.n, det_off);
    stage_end(st);
    // 3. preprocess backward -> residual-coordinate gradients
    float* dy = nullptr;
    if (want_mlp) {
        if ((s = w.dy.reserve(this, (size_t)P * kOut * sizeof(float) + 16, st))) return s;
        dy = (float*)w.dy.ptr;
    }
    stage_begin(SWF_STAGE_BWD_PREPROCESS, st);
    launch_preprocess_backward((const float*)w.dpair.ptr, w.rec, P, (flags & SWF_PAPER_DEFORM) != 0,
                               (float*)w.dbase.ptr, dy, st);
    stage_end(st);
    // 4. MLP backward (the forward's activations; BF16 operands after a BF16 forward)
    float* dmu = nullptr;
    if (want_mlp) {
        stage_begin(SWF_STAGE_BWD_MLP, st);
        s = mlp_backward(w, d, tx, B, dy, gr, bf16, st);
        last_mlp_bwd.valid = s == SWF_OK;
        last_mlp_bwd.scene = sid;
        last_mlp_bwd.B = B;
        last_mlp_bwd.n = d.n;
        last_mlp_bwd.layers = d.n_hidden;
        last_mlp_bwd.bf16 = bf16;
        stage_end(st);
        if (s) return s;
        dmu = (float*)w.dmu.ptr;
    }
    // 5. base parameters: sum over the batch, original ids
    const BaseGrads outs = {{gr->mean_x, gr->mean_y, gr->log_scale_x, gr->log_scale_y, gr->rotation,
                             gr->opacity_logit, gr->amplitude}};
    launch_base_reduce((const float*)w.dbase.ptr, dmu, d.perm, B, d.n, outs, st);
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
