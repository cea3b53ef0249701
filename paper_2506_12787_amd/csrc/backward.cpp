// Backward pass orchestration (blend -> preprocess -> MLP) and its C ABI entry.
#include <rocblas/rocblas.h>

#include <algorithm>

#include "runtime.h"

namespace swf {

namespace {

rocblas_handle blas_of(Ctx* c) { return reinterpret_cast<rocblas_handle>(c->blas); }

// C = op(A) op(B) (+ beta C) for row-major matrices: op(A) is M x K, op(B) is
// K x N, C is M x N with leading dimension ldc. rocBLAS is column-major, where
// a row-major matrix reads as its transpose, so C^T = op(B)^T op(A)^T.
rocblas_status gemm_rm(rocblas_handle h, bool ta, bool tb, int64_t M, int64_t N, int64_t K, const float* A,
                       int64_t lda, const float* Bm, int64_t ldb, float* C, int64_t ldc, float beta = 0.0f) {
    const float one = 1.0f;
    return rocblas_sgemm(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                         ta ? rocblas_operation_transpose : rocblas_operation_none, (rocblas_int)N, (rocblas_int)M,
                         (rocblas_int)K, &one, Bm, (rocblas_int)ldb, A, (rocblas_int)lda, &beta, C,
                         (rocblas_int)ldc);
}

constexpr int kMaxSplit = 64;  // K-slices of a weight-gradient GEMM

int split_of(int64_t P) { return (int)std::max<int64_t>(1, std::min<int64_t>(kMaxSplit, P / 16384)); }

// dW (M x N, row-major) = dz^T act over K = P rows (dz: P x M, act: P x N), as
// split-K: per-slice partial products in rocBLAS, then their sum. part holds
// split_of(P) * M * N floats, tmp colsum_blocks(split) * M * N.
rocblas_status wgrad_rm(rocblas_handle h, int64_t M, int64_t N, int64_t P, const float* dz, const float* act,
                        float* dW, float* part, float* tmp, hipStream_t st) {
    const int sp = split_of(P);
    const int64_t kc = P / sp, last = P - kc * (sp - 1);
    const float one = 1.0f, zero = 0.0f;
    rocblas_status r = rocblas_status_success;
    if (sp > 1)
        r = rocblas_sgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)N,
                                          (rocblas_int)M, (rocblas_int)kc, &one, act, (rocblas_int)N,
                                          (rocblas_stride)(kc * N), dz, (rocblas_int)M, (rocblas_stride)(kc * M), &zero,
                                          part, (rocblas_int)N, (rocblas_stride)(M * N), sp - 1);
    if (r != rocblas_status_success) return r;
    r = gemm_rm(h, true, false, M, N, last, dz + (sp - 1) * kc * M, M, act + (sp - 1) * kc * N, N,
                part + (int64_t)(sp - 1) * M * N, N);
    if (r != rocblas_status_success) return r;
    launch_colsum(part, sp, M * N, 1, 0, tmp, dW, 0, st);
    return rocblas_status_success;
}

// The same with BF16 operands and FP32 accumulation (rocblas_gemm_ex); C is
// FP32 (c_bf16 = false) or BF16.
rocblas_status gemm_rm_bf16(rocblas_handle h, bool ta, bool tb, int64_t M, int64_t N, int64_t K, const void* A,
                            int64_t lda, const void* Bm, int64_t ldb, void* C, int64_t ldc, bool c_bf16 = false) {
    const float one = 1.0f, zero = 0.0f;
    const rocblas_datatype ct = c_bf16 ? rocblas_datatype_bf16_r : rocblas_datatype_f32_r;
    return rocblas_gemm_ex(h, tb ? rocblas_operation_transpose : rocblas_operation_none,
                           ta ? rocblas_operation_transpose : rocblas_operation_none, (rocblas_int)N, (rocblas_int)M,
                           (rocblas_int)K, &one, Bm, rocblas_datatype_bf16_r, (rocblas_int)ldb, A,
                           rocblas_datatype_bf16_r, (rocblas_int)lda, &zero, C, ct, (rocblas_int)ldc, C, ct,
                           (rocblas_int)ldc, rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0, 0);
}

// wgrad_rm with BF16 dz and act (FP32 partials and result).
rocblas_status wgrad_rm_bf16(rocblas_handle h, int64_t M, int64_t N, int64_t P, const uint16_t* dz,
                             const uint16_t* act, float* dW, float* part, float* tmp, hipStream_t st) {
    const int sp = split_of(P);
    const int64_t kc = P / sp, last = P - kc * (sp - 1);
    const float one = 1.0f, zero = 0.0f;
    rocblas_status r = rocblas_status_success;
    if (sp > 1)
        r = rocblas_gemm_strided_batched_ex(
            h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)N, (rocblas_int)M, (rocblas_int)kc,
            &one, act, rocblas_datatype_bf16_r, (rocblas_int)N, (rocblas_stride)(kc * N), dz, rocblas_datatype_bf16_r,
            (rocblas_int)M, (rocblas_stride)(kc * M), &zero, part, rocblas_datatype_f32_r, (rocblas_int)N,
            (rocblas_stride)(M * N), part, rocblas_datatype_f32_r, (rocblas_int)N, (rocblas_stride)(M * N), sp - 1,
            rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0, 0);
    if (r != rocblas_status_success) return r;
    r = gemm_rm_bf16(h, true, false, M, N, last, dz + (sp - 1) * kc * M, M, act + (sp - 1) * kc * N, N,
                     part + (int64_t)(sp - 1) * M * N, N);
    if (r != rocblas_status_success) return r;
    launch_colsum(part, sp, M * N, 1, 0, tmp, dW, 0, st);
    return rocblas_status_success;
}

}  // namespace

void blas_release(Ctx* c) {
    if (c->blas) rocblas_destroy_handle(blas_of(c));
    c->blas = nullptr;
}

// MLP backward with the layer GEMMs in rocBLAS (plain GEMMs; the ReLU and bias
// steps are small kernels). Activations are recomputed: layer 1 from its
// per-Gaussian mean part W1m gamma(mu_hat) plus the per-query TX part (the
// forward's `qs`), later layers as act_l = ReLU(act_{l-1} W_l^T + b_l). Then
// from dy (gradients of the 7 residuals per pair):
//   dW_l = dz_l^T act_{l-1}, db_l = colsum(dz_l), dz_{l-1} = (dz_l W_l) * [act_{l-1} > 0],
// and for layer 1 the weight gradient splits into the mean part
// (sum over queries of dz_0 per Gaussian = S)^T gamma(mu_hat) and the TX part
// (sum over Gaussians of dz_0 per query)^T gamma(s_hat); the mean features'
// gradient is S W1m, taken through the sin / cos features to d mu.
// bf16: the backward of a BF16 forward. Activations and dz are stored in BF16
// (rounded like the forward kernel: FP32 sums, bias, ReLU, then one rounding)
// and every large GEMM runs on BF16 operands with FP32 accumulation; weight
// and bias gradients are accumulated in FP32.
swf_status Ctx::mlp_backward(Workspace& w, const DevScene& d, const float* tx, int B, const float* dy,
                             const swf_grads* gr, bool bf16, bool acts_ready, hipStream_t st) {
    swf_status s = SWF_OK;
    if (!blas) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return fail(SWF_E_DEVICE, "rocblas_create_handle");
        blas = h;
    }
    rocblas_handle h = blas_of(this);
    rocblas_set_stream(h, st);
    const int64_t N = d.n, P = (int64_t)B * N;
    const int nh = d.n_hidden, Hd = 256, I = d.in_dim;
    const size_t esz = bf16 ? 2 : 4;                 // activation / dz element size
    const size_t actb = (size_t)P * Hd * esz;
    const size_t f32b = (size_t)P * Hd * sizeof(float);
    if ((s = w.act.reserve(this, actb * nh + 16, st))) return s;
    // FP32: dz ping-pong. BF16: dz ping-pong in BF16, plus one FP32 GEMM result where one is stored: the
    // layer-1 gradient with a single hidden layer (else it is formed inside its sums), or the recompute's
    // pre-activations when the forward pass did not keep the activations
    const bool need_zf = bf16 && (nh == 1 || !acts_ready);
    if ((s = w.dz.reserve(this, need_zf ? actb * 2 + f32b + 16 : actb * 2 + 16, st))) return s;
    // scratch: Pm / S (N x 256), R (B x 256), dg (N x 26), split-K partials, column-sum partials, BF16 weights
    const size_t n_split = std::max({(size_t)split_of(P) * Hd * Hd, (size_t)layer1_sums_blocks((int)N) * B * Hd,
                                     (size_t)layer1_grad_blocks((int)N) * B * Hd, (size_t)wgrad_mfma_blocks(P) * (Hd * Hd + Hd),
                                     (size_t)wgrad_out_blocks(P) * kOut * Hd});
    const size_t n_cs = std::max<size_t>({(size_t)colsum_blocks(P) * Hd, (size_t)colsum_blocks(B) * N * Hd,
                                          (size_t)colsum_blocks(N) * Hd * B, (size_t)colsum_blocks(kMaxSplit) * Hd * Hd});
    const size_t n_wb = bf16 ? ((size_t)(nh - 1) * Hd * Hd + (size_t)kOut * Hd + (size_t)P * kOut + 64) / 2 + 64 : 0;
    const size_t small =
        ((size_t)N * Hd + (size_t)B * Hd + (size_t)N * kMeanFeat + 4 + n_split + n_cs + n_wb + 64) * sizeof(float);
    if ((s = w.part.reserve(this, small, st))) return s;
    if ((s = w.fmean.reserve(this, (size_t)N * kMeanFeat * sizeof(float) + 16, st))) return s;
    if ((s = w.ftx.reserve(this, (size_t)B * kTxFeat * sizeof(float) + 16, st))) return s;
    if ((s = w.dmu.reserve(this, (size_t)N * 2 * sizeof(float) + 16, st))) return s;
    if ((s = w.qs.reserve(this, (size_t)B * Hd * sizeof(float), st))) return s;
    void* act[8] = {};
    for (int l = 0; l < nh; ++l) act[l] = (char*)w.act.ptr + actb * l;
    void* dz[2] = {w.dz.ptr, (char*)w.dz.ptr + actb};
    float* zf = need_zf ? (float*)((char*)w.dz.ptr + actb * 2) : nullptr;  // FP32 layer-1 gradient (nh == 1)
    float* Pm = (float*)w.part.ptr;             // N x 256: W1m gamma(mu_hat), later S
    float* R = Pm + (size_t)N * Hd;              // B x 256
    float* dg = R + (size_t)B * Hd;              // N x 26
    float* part = dg + ((size_t)N * kMeanFeat + 3) / 4 * 4;  // split-K partials (16-byte aligned)
    float* tmp = part + n_split;                 // column-sum partials
    uint16_t* wb = (uint16_t*)(tmp + n_cs);      // BF16 weights: hidden layers 1.., output, then dy
    float* fmean = (float*)w.fmean.ptr, *ftx = (float*)w.ftx.ptr, *qs = (float*)w.qs.ptr;
    launch_tx_features(d, tx, B, qs, st, ftx);
    launch_mean_features_f32(d, fmean, st);
    auto ok = [&](rocblas_status r, const char* what) -> swf_status {
        return r == rocblas_status_success ? SWF_OK : fail(SWF_E_DEVICE, what);
    };
    uint16_t* wl[8] = {};
    uint16_t* dyb = nullptr;
    if (bf16) {
        for (int l = 1; l < nh; ++l) {
            wl[l] = wb + (size_t)(l - 1) * Hd * Hd;
            launch_to_bf16(d.w[l], (int64_t)Hd * Hd, wl[l], st);
        }
        wl[nh] = wb + (size_t)(nh - 1) * Hd * Hd;
        launch_to_bf16(d.w[nh], (int64_t)kOut * Hd, wl[nh], st);
        if (nh == 1) {  // the library GEMM of the single-hidden-layer path takes BF16 operands
            dyb = wl[nh] + (size_t)kOut * Hd;
            launch_to_bf16(dy, P * kOut, dyb, st);
        }
    }
    // ---- the hidden activations: stored by the forward pass (BF16), else recomputed
    if (!(bf16 && acts_ready)) {
        if ((s = ok(gemm_rm(h, false, true, N, Hd, kMeanFeat, fmean, kMeanFeat, d.w[0], I, Pm, Hd), "sgemm W1m")))
            return s;
        if (bf16)
            launch_layer1_act_bf16(Pm, qs, (int)N, P, act[0], st);
        else
            launch_layer1_act(Pm, qs, (int)N, P, (float*)act[0], st);
        for (int l = 1; l < nh; ++l) {
            if (bf16) {
                if ((s = ok(gemm_rm_bf16(h, false, true, P, Hd, Hd, act[l - 1], Hd, wl[l], Hd, zf, Hd), "gemm fwd")))
                    return s;
                launch_bias_relu_bf16(zf, d.b[l], P, act[l], st);
            } else {
                if ((s = ok(gemm_rm(h, false, true, P, Hd, Hd, (float*)act[l - 1], Hd, d.w[l], Hd, (float*)act[l], Hd),
                            "sgemm fwd")))
                    return s;
                launch_bias_relu((float*)act[l], d.b[l], P, st);
            }
        }
    }
    // ---- output layer (7 outputs)
    if (bf16) {
        // one pass over the last activations: the weight gradient and, with more than one hidden layer, the
        // masked BF16 gradient of the last hidden pre-activations (K = 7)
        launch_out_bwd_bf16(dy, wl[nh], act[nh - 1], P, nh > 1 ? dz[0] : nullptr, part, tmp, gr->weight[nh], st);
    } else if (gr->weight[nh] &&
               (s = ok(wgrad_rm(h, kOut, Hd, P, dy, (const float*)act[nh - 1], gr->weight[nh], part, tmp, st),
                       "dWo"))) {
        return s;
    }
    if (gr->bias[nh]) launch_colsum(dy, P, kOut, 1, 0, tmp, gr->bias[nh], 0, st);
    if (bf16) {
        // BF16 result (masking after rounding equals rounding after masking); the layer-1 gradient stays FP32
        if (nh == 1) {  // the layer-1 gradient, masked inside its sums below
            if ((s = ok(gemm_rm_bf16(h, false, false, P, Hd, kOut, dyb, kOut, wl[nh], Hd, zf, Hd), "gemm dz")))
                return s;
        }
    } else {
        if ((s = ok(gemm_rm(h, false, false, P, Hd, kOut, dy, kOut, d.w[nh], Hd, (float*)dz[0], Hd), "sgemm dz")))
            return s;
        launch_relu_mask((float*)dz[0], (const float*)act[nh - 1], P, st);
    }
    int cur = 0;
    const void* dz1 = nullptr;  // BF16: the second layer's pre-activation gradient
    for (int l = nh - 1; l >= 1; --l) {
        if (gr->weight[l]) {
            if (bf16) {
                // contraction over pairs; the bias gradient (column sums of dz) rides along
                launch_wgrad_mfma(dz[cur], act[l - 1], P, part, tmp, gr->weight[l], gr->bias[l], st);
            } else if ((s = ok(wgrad_rm(h, Hd, Hd, P, (const float*)dz[cur], (const float*)act[l - 1], gr->weight[l],
                                        part, tmp, st),
                               "dW"))) {
                return s;
            }
        }
        if (gr->bias[l] && !(bf16 && gr->weight[l])) {
            if (bf16)
                launch_colsum_bf16(dz[cur], P, Hd, 1, 0, tmp, gr->bias[l], 0, st);
            else
                launch_colsum((const float*)dz[cur], P, Hd, 1, 0, tmp, gr->bias[l], 0, st);
        }
        if (bf16) {
            // dz W on MFMA in one pass: BF16 and masked by the previous ReLU, or FP32 for the layer-1
            // gradient (masked inside its sums below)
            if (l > 1)
                launch_dz_gemm(dz[cur], wl[l], act[l - 1], P, dz[cur ^ 1], false, st);
            else
                dz1 = dz[cur];  // the layer-1 gradient is formed inside its sums below
        } else {
            if ((s = ok(gemm_rm(h, false, false, P, Hd, Hd, (const float*)dz[cur], Hd, d.w[l], Hd,
                                (float*)dz[cur ^ 1], Hd),
                        "sgemm dz")))
                return s;
            launch_relu_mask((float*)dz[cur ^ 1], (const float*)act[l - 1], P, st);
        }
        cur ^= 1;
    }
    // ---- layer 1: the gradient of its pre-activations dz0, FP32; S = its sum over the batch per Gaussian
    // (N x 256), R = its sum over the Gaussians per query (B x 256), b0 = its sum over all pairs
    float* S = Pm;
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
        if (gr->bias[0]) launch_colsum(S, N, Hd, 1, 0, tmp, gr->bias[0], 0, st);
    } else {
        const float* dz0 = (const float*)dz[cur];
        if (gr->bias[0]) launch_colsum(dz0, P, Hd, 1, 0, tmp, gr->bias[0], 0, st);
        launch_colsum(dz0, B, N * Hd, 1, 0, tmp, S, 0, st);
        if (gr->weight[0]) launch_colsum(dz0, N, Hd, B, N * Hd, tmp, R, Hd, st);
    }
    if (gr->weight[0]) {
        // dW1 [256 x 89] = [S^T gamma(mu_hat) | R^T gamma(s_hat)]
        if ((s = ok(gemm_rm(h, true, false, Hd, kMeanFeat, N, S, Hd, fmean, kMeanFeat, gr->weight[0], I), "dW1m")))
            return s;
        if ((s = ok(gemm_rm(h, true, false, Hd, kTxFeat, B, R, Hd, ftx, kTxFeat, gr->weight[0] + kMeanFeat, I),
                    "dW1s")))
            return s;
    }
    // d gamma(mu_hat) = S W1m (N x 26), then through the features to d mu
    if ((s = ok(gemm_rm(h, false, false, N, kMeanFeat, Hd, S, Hd, d.w[0], I, dg, kMeanFeat), "dgm"))) return s;
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
    // After a BF16 forward the MLP backward takes the hidden activations the forward's MLP kernel stored (the
    // same values the forward used).
    const bool bf16 = (flags & SWF_MLP_BF16) != 0;
    const bool acts_ready = want_mlp && bf16 && B >= 1 && (uint64_t)B * (uint64_t)d.n < (1ull << 32);
    swf_status s = SWF_OK;
    // 1. the forward's records and lists: still in the workspace if no pass wrote records since that render
    // (and it was given the same positions), else built again (deterministic: identical to the forward's)
    const bool kept = t.seq == w.seq && t.tx == tx && (!acts_ready || t.acts);
    if (!kept) {
        if (acts_ready) {
            const size_t actb = (size_t)B * d.n * 256 * sizeof(uint16_t);
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
    if (flags & SWF_DETERMINISTIC) {
        // per (list entry, wave) sums, zero where a wave contributes nothing
        const size_t db = (size_t)w.last.n_keys * 32 * sizeof(float);
        if ((s = w.det.reserve(this, db + 16, st))) return s;
        if (db && (s = hip(hipMemsetAsync(w.det.ptr, 0, db, st), "memset entry sums"))) return s;
        det_part = (float*)w.det.ptr;
    }
    launch_blend_backward((const uint2*)w.ranges.ptr, w.last.vals, w.rec, B, w.last.grid, grad_out, auxT, auxL,
                          (float*)w.dpair.ptr, st, det_part, d.n);
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
    // 4. MLP backward (activations recomputed, GEMMs in rocBLAS; BF16 operands after a BF16 forward)
    float* dmu = nullptr;
    if (want_mlp) {
        stage_begin(SWF_STAGE_BWD_MLP, st);
        s = mlp_backward(w, d, tx, B, dy, gr, bf16, acts_ready, st);
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
