/*
 * swiftwrf.h -- C ABI of libswiftwrf.so: the SwiftWRF spectrum render path on
 * one AMD Instinct MI355X (gfx950).
 *
 * The library renders the spatial spectrum seen by a fixed receiver from N
 * anisotropic 2D Gaussians after a deformation MLP has shifted them for a
 * transmitter position: the mapping F: R^3 -> spectrum, s -> F(s), of the
 * problem statement (paper Sec. 3.3, "Problem Definition"). Per query:
 *
 *   gamma(mu_hat), gamma(s_hat)      positional encoding, Sec. 4.2 eq. (posenc)
 *   dG = F_theta(gamma(mu), gamma(s)) deformation MLP, Sec. 4.2
 *   G^s = G^0 + dG                    GOP reference frame + residuals, Sec. 4.2
 *   K = delta exp(-d^T Sigma^-1 d / 2) kernel weight, Sec. 4.1
 *   front-to-back alpha compositing   blending rule reviewed in Sec. 3.2, over
 *                                     16x16 tiles (Sec. 4.1 tile partitioning)
 *
 * Conventions used by every entry point:
 *  - Spectrum layout: B x H x W float32, row-major; row = elevation, column =
 *    azimuth (the matrix of Sec. 3.1). Pixel (row y, column x) samples the
 *    continuous point (x, y) in pixel units. Gaussian means are in pixel units.
 *  - Per-Gaussian parameters (SoA, float32, length n): mean_x, mean_y (pixels),
 *    log_scale_x, log_scale_y (natural log of the standard deviations along the
 *    principal axes, pixels), rotation (radians; principal axis 1 points along
 *    (cos r, sin r)), opacity_logit (opacity = sigmoid(logit)), amplitude (the
 *    real signal response), depth (blending order; ties go to the lower id).
 *  - Blending per pixel, in ascending (depth, id) order: q = d^T Sigma^-1 d;
 *    skip if q > 9; alpha = min(0.99, opacity exp(-q/2)); skip if
 *    alpha < 1/255; T' = T (1 - alpha); stop (without adding) if T' < 1e-4;
 *    else C += amp alpha T and T = T'. No background term.
 *  - Deformation MLP input: [gamma(mu_hat) (2(2*6+1) = 26) | gamma(s_hat)
 *    (3(2*10+1) = 63)], mu_hat = (mean_x / W, mean_y / H) of the canonical mean,
 *    s_hat = (tx - room_lo) / (room_hi - room_lo). gamma(v) = [v, sin(2^k pi v)
 *    for k < L, cos(2^k pi v) for k < L], each block over all components in
 *    order. Hidden layers Linear + ReLU, output Linear with 7 residuals in the
 *    order (d_mean_x, d_mean_y, d_log_scale_x, d_log_scale_y, d_rotation,
 *    d_opacity_logit, d_amplitude). Deformed opacity = sigmoid(logit + d).
 *  - Device pointers are HIP device addresses (e.g. torch CUDA tensors on
 *    ROCm). "stream" is a hipStream_t passed as void*; NULL = default stream.
 *  - Ownership: the caller owns every buffer it passes. The context owns the
 *    scenes it uploaded (deep copies) and all scratch memory.
 *  - Errors: every entry point returns a swf_status. On an argument error
 *    (SWF_E_INVALID) nothing is enqueued. No C++ exception crosses the ABI.
 *  - Threading: a context may be used by one host thread at a time, except the
 *    serving entry points (swf_serve_*), which are thread-safe.
 */
#ifndef SWIFTWRF_H
#define SWIFTWRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t swf_status;
enum {
    SWF_OK = 0,
    SWF_E_INVALID = -1,   /* bad argument; nothing enqueued                     */
    SWF_E_OOM = -2,       /* device or host allocation failed                   */
    SWF_E_DEVICE = -3,    /* a HIP runtime call failed                          */
    SWF_E_NOT_FOUND = -4, /* unknown scene id or ticket                         */
    SWF_E_OVERFLOW = -5,  /* a capacity was exceeded (key buffer, scratch)     */
    SWF_E_STATE = -6,     /* call not valid in the current state               */
    SWF_E_PENDING = -7,   /* serving: result not ready yet                      */
};

/* Render flags (bitwise or). */
enum {
    SWF_MLP_FP32 = 0,        /* deformation MLP in FP32 (FP32 MFMA and sums)     */
    SWF_MLP_BF16 = 1 << 0,   /* deformation MLP on BF16 MFMA, FP32 accumulate    */
    SWF_NO_DEFORM = 1 << 1,  /* static render of the canonical Gaussians         */
    SWF_KEEP_AUX = 1 << 2,   /* write the per-pixel blend state `aux` (training) */
    SWF_FULL_SORT = 1 << 3,  /* sort full 64-bit (tile << 32 | depth) keys
                                instead of eliding the depth digits (same
                                result; used to check the elision)               */
    SWF_TILE8 = 1 << 4,      /* 8x8 tiles instead of 16x16 (same result)         */
    SWF_PAPER_DEFORM = 1 << 5,/* zero the covariance residuals (outputs 2..4), as
                                the paper does not deform the covariance         */
    SWF_WRAP_AZIMUTH = 1 << 6, /* periodic azimuth: columns 0 and W-1 are
                                neighbours (0 and 360 degrees are one direction,
                                Sec. 3.1 spectrum grid); a Gaussian acts at each
                                pixel through the image of its mean (shifted by a
                                whole number of grid widths) nearest to it. Lists
                                are built by binning when a query's tiles form one
                                segment (at most 256), else by key sorting         */
    SWF_DETERMINISTIC = 1 << 7 /* swf_render_backward: gradients summed in a fixed
                                order (bitwise the same from run to run) instead of
                                by atomic adds; takes 128 bytes per list entry of
                                device memory and one more pass                   */
};

typedef struct swf_ctx swf_ctx;

typedef struct {
    int32_t device;             /* HIP device ordinal                             */
    int32_t mlp_pairs_per_wave; /* BF16 MLP tuning: pairs per wave, 48 (default
                                   or 0) or 32 (two waves per SIMD), or 64 (one)  */
    uint32_t max_list_entries;  /* most tile-list entries one launch sequence of
                                   swf_render builds (0: 2^32 - 1, the most the
                                   32-bit list positions address); a batch with
                                   more is rendered in chunks of queries           */
    int32_t reserved[5];
} swf_config;

typedef struct {
    int32_t n;               /* number of Gaussians, >= 0                          */
    const float *mean_x, *mean_y, *log_scale_x, *log_scale_y;
    const float *rotation, *opacity_logit, *amplitude, *depth;
} swf_gaussians;

#define SWF_MAX_LAYERS 8
typedef struct {
    int32_t mean_bands;      /* L of gamma(mu_hat); 6                             */
    int32_t tx_bands;        /* L of gamma(s_hat); 10                             */
    int32_t hidden;          /* hidden width; must be 256                         */
    int32_t n_hidden;        /* number of hidden layers; 1..SWF_MAX_LAYERS-1      */
    const float *weight[SWF_MAX_LAYERS]; /* W_l row-major [out][in], l = 0..n_hidden */
    const float *bias[SWF_MAX_LAYERS];   /* b_l [out]                                */
    float room_lo[3], room_hi[3];        /* TX normalisation box (metres)            */
} swf_mlp;

/* Per-pixel blend state kept for the backward pass (SWF_KEEP_AUX): for each of
 * the B*H*W pixels, T_final (float32) then, in a second plane, the number of
 * tile-list entries consumed up to and including the last added Gaussian
 * (uint32). Size: 8 * B * H * W bytes. */

/* Gradient buffers (device, float32, caller-owned, overwritten). Any may be
 * NULL to skip it. Base-parameter gradients are summed over the batch. */
typedef struct {
    float *mean_x, *mean_y, *log_scale_x, *log_scale_y, *rotation, *opacity_logit, *amplitude;
    float *weight[SWF_MAX_LAYERS];
    float *bias[SWF_MAX_LAYERS];
} swf_grads;

/* ---- context ------------------------------------------------------------ */

/* Create a context on cfg->device (cfg may be NULL: device 0). */
swf_status swf_create(swf_ctx **out, const swf_config *cfg);
/* Destroy a context and everything it owns. Waits for its work to finish. */
swf_status swf_destroy(swf_ctx *ctx);
/* Static string for a status code. */
const char *swf_status_string(swf_status s);
/* Last error message of this context (static storage owned by the context). */
const char *swf_last_error(swf_ctx *ctx);

/* ---- scenes (paper Sec. 4.2: canonical reference frame G^0 plus F_theta) ---
 * Upload n Gaussians (and optionally the deformation MLP) for an H x W grid.
 * The context copies everything (host or device source, src_is_device). The
 * Gaussians are reordered by (depth, id) on upload; ids seen through the debug
 * entry points are the caller's original indices. mlp may be NULL for a static
 * scene. H and W must lie in [1, 4096]. Synchronous. */
swf_status swf_scene_upload(swf_ctx *ctx, const swf_gaussians *g, const swf_mlp *mlp, int32_t height,
                            int32_t width, int32_t src_is_device, int32_t *scene_id);
swf_status swf_scene_release(swf_ctx *ctx, int32_t scene_id);
/* Replace the parameters of an uploaded scene in place (training). g (may be
 * NULL) must have the uploaded n; its depth array is ignored: the scene keeps
 * the (depth, id) order it was uploaded with (depth gets no gradient; upload a
 * new scene to change depths). mlp (may be NULL) must have the uploaded shape.
 * Sources are host or device (src_is_device). Host sources: the call waits
 * for `stream`. Device sources: the copies and the rebuilt BF16 weight stream
 * are enqueued on `stream` and the call returns without waiting. */
swf_status swf_scene_update(swf_ctx *ctx, int32_t scene_id, const swf_gaussians *g, const swf_mlp *mlp,
                            int32_t src_is_device, void *stream);
/* Device bytes held by a scene (its Gaussians, presort data and weights). */
swf_status swf_scene_bytes(swf_ctx *ctx, int32_t scene_id, uint64_t *bytes);

/* ---- render (Sec. 4.3: PE -> MLP -> deform -> tile rasterization) ----------
 * tx: device float32 [batch][3] transmitter positions (ignored with
 * SWF_NO_DEFORM, may be NULL then). out: device float32 [batch][H][W].
 * aux: device buffer of 8*batch*H*W bytes when SWF_KEEP_AUX, else NULL.
 * Enqueued on `stream`; the call returns after enqueueing, except that it waits
 * once for the total key count (an 8-byte device-to-host read after the key
 * scan). The first render of a context sizes the key buffers from that count
 * before enqueueing the rest; later ones enqueue the rest at the buffers'
 * capacity and wait for the count meanwhile, rendering again at the exact size
 * (the same call, still on `stream`) if it did not fit. A batch whose lists
 * would hold more entries than the context's max_list_entries (or whose
 * batch * n reaches 2^32) is rendered in chunks of queries, halving until each
 * fits (not with SWF_KEEP_AUX: SWF_E_OVERFLOW then); the outputs are those of
 * one launch. */
swf_status swf_render(swf_ctx *ctx, int32_t scene_id, const float *tx, int32_t batch, int32_t flags, float *out,
                      void *aux, void *stream);

/* Render on another resolution of the same field of view: the grid of the
 * call, height x width (each in [1, 4096]), covers the elevation x azimuth
 * range of the scene's own grid (the matrix of Sec. 3.1, e.g. 180 x 720 at
 * 0.5 degree per pixel for a scene uploaded at 90 x 360), so scene pixel
 * coordinates scale by (width / W, height / H): means, 3-sigma extents and
 * covariances (Sigma' = S Sigma S) follow, the deformation MLP is unchanged
 * (its mean features are normalised by the scene's own grid). out is
 * batch x height x width. Works for both scene kinds (a paper-model scene
 * renders its magnitude). SWF_KEEP_AUX needs the scene's own grid (the
 * backward renders there): SWF_E_INVALID otherwise. Everything else as
 * swf_render. */
swf_status swf_render_at(swf_ctx *ctx, int32_t scene_id, const float *tx, int32_t batch, int32_t height, int32_t width,
                         int32_t flags, float *out, void *aux, void *stream);

/* One launch sequence for queries over several resident scenes, each with its
 * own Gaussian count, grid and deformation MLP (the problem statement's
 * render(gaussians, tx) -> spectrum, Sec. 3.3, for a batch whose queries name
 * different scenes; the serving loop's mixed batches). scene_ids: host int32
 * [batch]; tx: device float32 [batch][3] (NULL with SWF_NO_DEFORM); out: device
 * float32, the batch's spectra concatenated in query order (query b's H_b x W_b
 * values start at out_offsets[b]); out_offsets (host, may be NULL) receives the
 * batch + 1 offsets (the last is the total). Every query renders exactly the
 * values swf_render gives it alone. flags: SWF_MLP_BF16 or SWF_MLP_FP32 (every
 * scene with a 4 x 256 MLP) or SWF_NO_DEFORM, optionally SWF_PAPER_DEFORM;
 * compositing-model scenes only; lists are built by binning per query (by key
 * sorting over every global tile of the batch when the largest query grid is
 * beyond the binning's tile limit). SWF_E_INVALID for other flags or scenes, SWF_E_NOT_FOUND for an
 * unknown scene. Waits once for the batch's key count, like swf_render; the
 * device status then describes the batch as one query holding every pair. */
swf_status swf_render_mixed(swf_ctx *ctx, const int32_t *scene_ids, const float *tx, int32_t batch, int32_t flags,
                            float *out, uint64_t *out_offsets, void *stream);

/* ---- backward (hand-written; transmittance replayed back to front) --------
 * The gradient that training by back-propagation needs (Sec. 4.4, the loss
 * minimised over the Gaussians and the MLP; the derivative of the Sec. 3.2
 * blending rule with the Sec. 4.1 kernel, through the Sec. 4.2 deformation).
 * Gradient of sum(grad_out * out) with respect to the scene's base parameters
 * and MLP weights, for the same (scene, tx, batch, flags) as the swf_render
 * call that produced `aux` (flags must include SWF_KEEP_AUX there). Every
 * discrete decision is held at its forward outcome; where the 0.99 alpha clamp
 * is active the derivative through opacity and q is zero. Depth gets no
 * gradient. The render that filled aux keeps its records, tile lists and
 * (after a BF16 forward) the MLP's hidden activations in the context's
 * workspace; the backward takes them when no other pass has written records
 * on the context since and tx is the same pointer (tx must hold the same
 * positions in any case), and otherwise repeats the forward pass, which then
 * waits once for its key count. SWF_DEV_BWD_REUSED in swf_last_device_status
 * tells which. With SWF_DETERMINISTIC in flags (here; the render's flags
 * need not carry it) every per-pixel contribution to a Gaussian's gradient is
 * first summed per (list entry, wave) and the sums are added per pair in the
 * order of its tiles, so the result does not depend on scheduling. Enqueued
 * on `stream`; returns after enqueueing. aux must be the
 * buffer such a render on this context filled (the context remembers the last
 * 1024): SWF_E_STATE if it is unknown or the scene's parameters were updated
 * (swf_scene_update) since, SWF_E_INVALID if scene, batch or flags (other
 * than SWF_KEEP_AUX) differ from that render's. */
swf_status swf_render_backward(swf_ctx *ctx, int32_t scene_id, const float *tx, int32_t batch, int32_t flags,
                               const float *grad_out, const void *aux, const swf_grads *grads, void *stream);

/* Hybrid loss of the training objective (paper Sec. 4.4, hybrid-loss
 * equation): loss = lambda1 * mean |pred - target| + (1 - lambda1) *
 * (1 - SSIM(pred, target)), with lambda1 = 0.7 in the paper's hyperparameter
 * table. pred, target: device float32 [batch][height][width] spectra. SSIM
 * (parameters not given by the paper; the common reading): an 11 x 11
 * Gaussian window of standard deviation 1.5 normalised to sum 1, local means,
 * variances and covariance by window sums with zero padding outside the grid,
 * C1 = 0.01^2, C2 = 0.03^2 (data range 1), the map averaged over every pixel
 * of every spectrum. Window sums and the map are formed in FP64.
 * loss: device float32 [3] <- (total, mean l1, mean SSIM). grad (device, may be
 * NULL) <- d loss / d pred, float32 like pred. SWF_E_INVALID (nothing enqueued)
 * for batch outside [1, 65535], height or width outside [1, 4096], lambda1
 * outside [0, 1] or a NULL pred / target / loss. Deterministic (fixed-order
 * reductions). Enqueued on `stream`; scratch 12 bytes per pixel. */
swf_status swf_hybrid_loss(swf_ctx *ctx, const float *pred, const float *target, int32_t batch, int32_t height,
                           int32_t width, float lambda1, float *loss, float *grad, void *stream);

/* Adam update of up to 32 parameter tensors in one launch (the optimiser of
 * the paper's training protocol, Sec. 4.4, at the hyperparameter table's
 * learning rates: Gaussians 1e-2, MLP 8e-3). For tensor k (count of them;
 * params[k], grads[k], m[k], v[k] device float32 arrays of sizes[k] elements;
 * the five arrays of pointers, sizes and lrs are host arrays):
 * m = beta1 m + (1 - beta1) g, v = beta2 v + (1 - beta2) g^2,
 * p -= lrs[k] (m / (1 - beta1^step)) / (sqrt(v) / sqrt(1 - beta2^step) + eps),
 * in place. step >= 1 is the update's number (bias correction). Moments start
 * at zero (the caller clears them). SWF_E_INVALID for count outside [0, 32],
 * step < 1, betas outside [0, 1), eps <= 0 or a NULL entry. Enqueued on
 * `stream`. */
swf_status swf_adam_step(swf_ctx *ctx, float *const *params, const float *const *grads, float *const *m,
                         float *const *v, const int64_t *sizes, const float *lrs, int32_t count, float beta1,
                         float beta2, float eps, int32_t step, void *stream);

/* Anneal smoothing of the moving positions (paper Sec. 4.4, anneal-smoothing
 * equations): tx_out = tx + gamma * noise * (2 / cbrt(n_positions)) *
 * max(0, 1 - iter / tau) * (room_hi - room_lo), i.e. the paper's perturbation
 * of the position in the unit cube the positions are normalised to, expressed
 * in metres; the decay is clamped at zero from tau on. tx, noise, tx_out:
 * device float32 [batch][3]; noise holds standard normal draws (the caller's
 * random numbers). room_lo, room_hi: host float[3]. The paper uses gamma = 1
 * and tau = 10,000. SWF_E_INVALID for batch < 1, tau < 1, n_positions < 1,
 * iter < 0, a non-finite gamma or a NULL pointer. Enqueued on `stream`. */
swf_status swf_anneal_tx(swf_ctx *ctx, const float *tx, const float *noise, int32_t batch, int32_t iter, float gamma,
                         int32_t tau, int32_t n_positions, const float *room_lo, const float *room_hi, float *tx_out,
                         void *stream);

/* L1 loss (paper Sec. 4.4, the l1 term): loss = mean |pred - target| over n
 * values, written to *loss (device float32); grad (device, may be NULL)
 * receives sign(pred - target) / n with sign(0) = 0. */
swf_status swf_l1_loss(swf_ctx *ctx, const float *pred, const float *target, int64_t n, float *loss, float *grad,
                       void *stream);

/* ---- the paper's own spectrum model -------------------------------------------
 * The model as the paper writes it (Sec. 4.1, 4.2, 6.1): a Gaussian n has a raw
 * centre (c_x, c_y) mapped by the hyperbolic normalisation to pixel units,
 * x = (W / 2)(tanh(c_x) + 1), y = (H / 2)(tanh(c_y) + 1) (azimuth onto the
 * grid's columns, elevation onto its rows); a covariance Sigma = L L^T from its
 * Cholesky factor L = [[l1, 0], [l2, l3]] (pixels); an attenuation gate
 * delta = sigmoid(atten_logit); and a complex response psi = (psi_re, psi_im).
 * The spectrum is the order-free GMM sum A(p) = | sum_n psi_n delta_n
 * exp(-q_n(p) / 2) | over the Gaussians with q_n(p) = d^T Sigma^-1 d <= 9 (the
 * 3-sigma support the tiles are built from): no depth, no opacity clamp, no
 * termination. With an MLP the Gaussians are deformed per position s: the MLP
 * maps [gamma(mu_hat) (10 bands, 42) | gamma(s_hat) (6 bands, 39)] through eight
 * ReLU layers of 156 units, the input concatenated after the hidden state
 * entering layers 3, 5 and 7 (skip connections every two layers), to the
 * residuals (d_mu_x, d_mu_y, d_psi_re, d_psi_im, d_delta): centre + d_mu (pixels),
 * psi + d_psi, delta = sigmoid(atten_logit) + d_delta; the covariance is not
 * deformed. FP32 throughout (the paper's precision), forward only. */
typedef struct {
    int32_t n;
    const float *center_x, *center_y;           /* raw centres (before the tanh map)      */
    const float *chol_l1, *chol_l2, *chol_l3;   /* Cholesky factor of Sigma, pixels        */
    const float *atten_logit;                   /* delta = sigmoid(atten_logit)            */
    const float *psi_re, *psi_im;               /* complex response                        */
} swf_paper_gaussians;
typedef struct {
    /* row-major (out, in): 156 x 81, 156 x 156, 156 x 237, 156 x 156, 156 x 237,
       156 x 156, 156 x 237, 156 x 156, then the output layer 5 x 156; inputs of
       layers 3, 5, 7 are [h (156) | x (81)] */
    const float *weight[9];
    const float *bias[9];
    float room_lo[3], room_hi[3]; /* s_hat = (s - room_lo) / (room_hi - room_lo) */
} swf_paper_mlp;
/* Uploads a paper-model scene (copies; n Gaussians in id order; mlp may be NULL
 * for static renders only). A Gaussian with l1 l3 = 0 or a non-finite parameter
 * takes no part (culled). Errors as swf_scene_upload. */
swf_status swf_scene_upload_paper(swf_ctx *ctx, const swf_paper_gaussians *g, const swf_paper_mlp *mlp,
                                  int32_t height, int32_t width, int32_t src_is_device, int32_t *scene_id);
/* Renders a paper-model scene: out [batch][H][W] = |sum| (device, caller-owned);
 * channels (device, may be NULL) [batch][2][H][W] = the real and imaginary sums.
 * flags: SWF_MLP_FP32 (deformable, tx required) or SWF_NO_DEFORM, optionally
 * SWF_FULL_SORT and SWF_WRAP_AZIMUTH; SWF_MLP_BF16, SWF_TILE8 and SWF_KEEP_AUX
 * are SWF_E_INVALID (as is the render backward and swf_scene_update on such a
 * scene). swf_render on a paper-model scene renders the magnitude only. Lists,
 * status word, stream semantics and errors otherwise as swf_render. */
swf_status swf_render_paper(swf_ctx *ctx, int32_t scene_id, const float *tx, int32_t batch, int32_t flags, float *out,
                            float *channels, void *stream);

/* ---- RSSI head --------------------------------------------------------------
 * The RSSI case study (paper Sec. 7.2): the rendered spectrum map is reduced by
 * global average pooling to one received-signal-strength value per query,
 * rssi[b] = (1 / (H W)) sum over the H x W pixels of spectrum b (the paper uses
 * a 16 x 16 spectrum of 50 Gaussians for this head). Renders like swf_render
 * (same scene, tx, batch, flags and aux semantics) into `out` when it is not
 * NULL (B x H x W, caller-owned) or into context scratch otherwise, then pools
 * with an FP64 sum per query in a fixed order (deterministic, independent of
 * the batch). rssi: device float32 [batch], caller-owned. Errors as
 * swf_render, plus SWF_E_INVALID for a NULL rssi. Enqueued on `stream`. */
swf_status swf_render_rssi(swf_ctx *ctx, int32_t scene_id, const float *tx, int32_t batch, int32_t flags,
                           float *rssi, float *out, void *aux, void *stream);
/* Backward of swf_render_rssi: the gradient of sum(grad_rssi * rssi), i.e.
 * swf_render_backward with grad_out[b][y][x] = grad_rssi[b] / (H W) (formed on
 * the device in context scratch). grad_rssi: device float32 [batch]. aux, flags
 * and the other arguments as in swf_render_backward, for the swf_render_rssi
 * call (with SWF_KEEP_AUX) that filled aux. */
swf_status swf_render_rssi_backward(swf_ctx *ctx, int32_t scene_id, const float *tx, int32_t batch, int32_t flags,
                                    const float *grad_rssi, const void *aux, const swf_grads *grads, void *stream);

/* ---- beam-scan spectrum from multipath lists -------------------------------
 * The spatial spectrum a receiver's sqrt(K) x sqrt(K) planar array measures by
 * beam scanning (paper Sec. 3.1: element positions, the path-length and phase
 * differences, the received-signal equation h_mn = sum_l rho_l
 * exp(j dalpha_mn(theta_l, phi_l)), and the beam-scan equation A(theta, phi) =
 * |(1/K) sum_mn exp(-j dalpha_mn(theta, phi)) exp(j angle h_mn)|). A physically
 * shaped target for the renderer.
 *  paths   device float32 [batch][max_paths][3]: (rho, azimuth theta in
 *          radians, elevation phi in radians) per path; slots past a query's
 *          count are not read. May be NULL when max_paths is 0.
 *  counts  device int32 [batch]: paths per query; a count outside
 *          [0, max_paths] is clamped into it. A query with no paths (or an
 *          element whose channel is exactly zero, whose angle is undefined)
 *          contributes zero.
 *  side    sqrt(K), 1..8; element (m, n) at radius D sqrt((m-1)^2 + (n-1)^2)
 *          and angle atan2(m-1, n-1); spacing_over_lambda = D / lambda > 0.
 *  out     device float32 [batch][height][width], caller-owned; row y =
 *          elevation phi = (pi/2) y / height, column x = azimuth
 *          theta = 2 pi x / width (1 degree per pixel at 90 x 360).
 * The per-element channel is formed in FP64, the per-pixel sum in FP32.
 * SWF_E_INVALID (nothing enqueued) for batch outside [1, 65535], side outside
 * [1, 8], max_paths < 0, a non-positive or non-finite spacing, height or
 * width outside [1, 4096], or a NULL counts / out (or paths with
 * max_paths > 0). Enqueued on `stream`; the context's scratch holds
 * batch * K * 8 bytes. Non-finite path values give non-finite outputs for
 * that query. */
swf_status swf_beamscan(swf_ctx *ctx, const float *paths, const int32_t *counts, int32_t batch, int32_t max_paths,
                        int32_t side, float spacing_over_lambda, int32_t height, int32_t width, float *out,
                        void *stream);

/* ---- device status of the last render --------------------------------------
 * What the device saw during the last swf_render (or the forward pass of the
 * last swf_render_backward) on this context, for the problem statement's
 * render(gaussians, tx) -> spectrum (Sec. 3.3): Gaussians that take no part
 * because a deformed parameter is not finite (or the covariance degenerates,
 * or the depth is NaN) and Gaussians whose 3-sigma box misses the grid are
 * culled, not errors; a key count over a fixed capacity is an overflow that
 * the call recovers from by rendering again at the exact size. Counts are
 * over (query, Gaussian) pairs. Waits for the stream of that render.
 * SWF_E_STATE before the first render. */
enum {
    SWF_DEV_KEY_OVERFLOW = 1u << 0,     /* the last list build overflowed its capacity  */
    SWF_DEV_RERENDERED = 1u << 1,       /* ... so the call rendered again, exactly sized */
    SWF_DEV_CULLED_NONFINITE = 1u << 2, /* culled_nonfinite > 0                          */
    SWF_DEV_CULLED_OFFGRID = 1u << 3,   /* culled_offgrid > 0                            */
    SWF_DEV_BWD_REUSED = 1u << 4,       /* the last swf_render_backward took the records
                                           and lists its forward render kept            */
    SWF_DEV_CHUNKED = 1u << 5,          /* the last swf_render split its batch into chunks
                                           of queries (more list entries than
                                           max_list_entries, or 2^32 pairs); the other
                                           fields describe its last chunk               */
};
typedef struct {
    uint32_t flags;             /* SWF_DEV_* bits                                     */
    uint32_t rerenders;         /* exact-size re-renders of the call (0 or 1)         */
    uint64_t pairs;             /* (query, Gaussian) pairs of the render: batch * n   */
    uint64_t culled_nonfinite;  /* pairs with a non-finite or degenerate Gaussian     */
    uint64_t culled_offgrid;    /* pairs whose 3-sigma box misses the grid            */
    uint64_t list_entries;      /* tile-list entries (keys) of the render             */
    uint64_t reserved[3];
} swf_device_status;
swf_status swf_last_device_status(swf_ctx *ctx, swf_device_status *out);

/* ---- stage timing ----------------------------------------------------------
 * When enabled, swf_render records a HIP event pair around each stage on the
 * render stream. swf_stage_times waits for them and returns, per stage, the
 * summed milliseconds and the number of launches since the last reset:
 * stage 0 tx features, 1 MLP+deform+preprocess, 2 scan, 3 emit keys,
 * 4 radix sort, 5 tile ranges, 6 blend. Without SWF_FULL_SORT the lists are
 * built by binning instead: stage 2 is then the per-block tile histograms and
 * their scan, stage 3 is empty and stage 4 the stable placement of the pair
 * indices (same lists as the sort). swf_render_backward adds stage 7 blend
 * backward, 8 preprocess backward and 9 MLP backward (layer GEMMs, masks,
 * column sums, the positional-encoding chain), besides the forward stages of
 * the forward pass it repeats.
 * n_stages is in/out (capacity/used). */
enum { SWF_STAGE_TX = 0, SWF_STAGE_MLP, SWF_STAGE_SCAN, SWF_STAGE_EMIT, SWF_STAGE_SORT, SWF_STAGE_RANGES,
       SWF_STAGE_BLEND, SWF_STAGE_BWD_BLEND, SWF_STAGE_BWD_PREPROCESS, SWF_STAGE_BWD_MLP, SWF_N_STAGES };
swf_status swf_stage_timing(swf_ctx *ctx, int32_t enable);
swf_status swf_stage_times(swf_ctx *ctx, double *ms, int64_t *launches, int32_t *n_stages);

/* ---- debug / step-level entry points --------------------------------------
 * swf_debug_deform: the 7 MLP residuals of every (query, Gaussian) pair, device
 * float32 [batch][n][7], Gaussians in the caller's original order.
 * swf_debug_keys: after a swf_render of the same scene, batch and flags on the
 * same context, copies to HOST buffers: counts [batch*n] and offsets
 * [batch*n] (uint32, pairs in (query, depth-sorted Gaussian) order), the sorted
 * keys [n_keys] as uint64 (global tile << 32 | depth bits), the sorted values
 * [n_keys] as (query << 32 | original Gaussian id), and the tile ranges
 * [batch*tiles][2] (uint32 start, end). Pass NULL for any output to skip it;
 * *n_keys returns the key count. Sizes must hold what is copied. */
swf_status swf_debug_deform(swf_ctx *ctx, int32_t scene_id, const float *tx, int32_t batch, int32_t flags,
                            float *delta, void *stream);
swf_status swf_debug_keys(swf_ctx *ctx, uint32_t *counts, uint32_t *offsets, uint64_t *keys, uint64_t *values,
                          uint32_t *ranges, uint64_t *n_keys, uint64_t capacity);
/* swf_debug_rects: after a render on this context, copies to the HOST buffer
 * rects [batch*n][4] (int32, pairs in (query, original Gaussian id) order) the
 * tile rectangle of every pair as the device computed it (Sec. 4.1 tile
 * partitioning): tx0, ty0, tx1, ty1 (inclusive tile indices), or four -1 for a
 * culled pair. capacity = number of pairs rects holds. Synchronous. */
swf_status swf_debug_rects(swf_ctx *ctx, int32_t *rects, uint64_t capacity);
/* swf_debug_relu_pattern: after a swf_render_backward on this context that ran
 * the MLP backward, copies to the HOST buffer pattern [batch][n][layers][256]
 * (uint8, pairs in (query, original Gaussian id) order) the ReLU decisions of
 * every hidden unit that backward used (1: the unit passed, its activation is
 * positive): the forward kernel's after a BF16 forward, the recomputed ones
 * after an FP32 forward (Sec. 4.2 network; the gradient holds them).
 * capacity = bytes pattern holds. Synchronous. SWF_E_STATE without such a
 * backward. */
swf_status swf_debug_relu_pattern(swf_ctx *ctx, uint8_t *pattern, uint64_t capacity);
/* swf_debug_blend_work: the work of the last swf_render's blend stage (Sec. 3.2
 * front-to-back rule), for roofline accounting: re-walks the same tile lists
 * without writing a spectrum and returns, in host memory, the number of (pixel,
 * list entry) evaluations the rule needs (entries inside the pixel's 3-sigma
 * cutoff, up to and including the one that ends the pixel), the number of
 * records staged into LDS, and the number of list entries. Synchronous; any
 * output may be NULL. */
swf_status swf_debug_blend_work(swf_ctx *ctx, uint64_t *evaluations, uint64_t *staged, uint64_t *n_entries);
/* swf_debug_blend_executed: the lane-evaluations the blend kernel of the last
 * swf_render executes on 16 x 16 tiles (every lane of a wave evaluates each
 * entry its wave visits: the entries that reach its 8 x 8 quadrant, in groups
 * of 8, until all its pixels have ended), counted by the same walk without
 * writing a spectrum; set against the evaluations swf_debug_blend_work reports
 * as needed, the share of the blend's vector work that is the branch-free
 * walk's no-ops. 0 for 8 x 8 tiles. Synchronous. */
swf_status swf_debug_blend_executed(swf_ctx *ctx, uint64_t *lane_evaluations);
/* swf_measure_peaks: on-device peaks for roofline accounting (not part of the
 * method): the rates this GPU sustains in plain loops of BF16 MFMA
 * (v_mfma_f32_16x16x32_bf16 chains held in registers, TFLOP/s), FP32 FMA
 * (T lane-ops/s, one per FMA) and conflict-free 16-byte LDS reads (TB/s), with
 * one 8-wave workgroup per compute unit. Synchronous on the context's device
 * (a few milliseconds); any output may be NULL. */
swf_status swf_measure_peaks(swf_ctx *ctx, double *mfma_bf16_tflops, double *fma_tops, double *lds_tbps);

/* Stable LSD radix sort of n (key, value) pairs in place, device memory, on
 * the key bits [begin_bit, end_bit). key_bytes is 4 (uint32 keys) or 8 (uint64
 * keys). 8-bit digits, wave-ballot ranking. Enqueued on stream. */
swf_status swf_radix_sort(swf_ctx *ctx, void *keys, uint32_t *values, int64_t n, int32_t key_bytes,
                          int32_t begin_bit, int32_t end_bit, void *stream);
/* Exclusive prefix sum of n uint32 counts (device) into offsets (device,
 * uint32); the 64-bit total goes to *total (device uint64). */
swf_status swf_exclusive_scan(swf_ctx *ctx, const uint32_t *counts, uint32_t *offsets, uint64_t *total, int64_t n,
                              void *stream);

/* Allocation-free variant of swf_exclusive_scan, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, same result. It calls no
 * allocating routine; its scratch is a static 32 KiB device array per GPU
 * (4096 + 8 block sums; the scan grid is capped at 4096 blocks, so every n
 * fits, and a larger requirement would fail with SWF_E_OVERFLOW). All calls on
 * one GPU share that array, so calls that overlap on one GPU race: order them
 * (one stream, or events). Nothing in it needs to start at zero. */
swf_status swf_exclusive_scan_noalloc(swf_ctx *ctx, const uint32_t *counts, uint32_t *offsets, uint64_t *total,
                                      int64_t n, void *stream);

/* ---- serving loop (continuous batching over resident scenes) --------------
 * The paper defines no serving interface; these calls serve the problem
 * statement's mapping s -> F(s) (Sec. 3.3) to many concurrent requesters: each
 * request is one render of one transmitter position of a resident scene.
 * A scheduler thread owns n_slots execution slots (own stream + workspace);
 * launches of different slots overlap on the device. Whenever a slot is free,
 * the oldest waiting request's scene is served: up to max_batch of its waiting
 * requests (FIFO) are rendered together, padded to a power-of-two bucket, by
 * replaying the slot's captured hipGraph of the whole render (fixed key
 * capacity = key_factor x calibrated keys per query x bucket, no host sync).
 * A key overflow is detected from the status word and the batch is re-rendered
 * with exact sizing (`fallback` in the stats). hbm_budget (bytes, 0 = none)
 * bounds the sum of all slot workspaces: a batch that does not fit is shrunk,
 * idle workspaces are released, or the requests wait; a single query that can
 * never fit fails with SWF_E_OOM. Scenes must stay uploaded while served.
 * mixed = 1 batches across scenes: the waiting requests in arrival order, of
 * up to 64 distinct scenes sharing the oldest request's deformation mode (all
 * with a 4 x 256 MLP, in the precision of flags, or all static), go into one mixed batch
 * (swf_render_mixed's launches); its graph is keyed by capacities (queries,
 * pairs, tiles, keys, rounded up to four steps per octave), not by scene, so
 * any mix of scenes whose totals fit replays it. Scenes a mixed batch cannot
 * hold (the paper model, other MLP shapes, SWF_TILE8) are served per scene. */
typedef struct {
    int32_t max_batch;    /* largest batch per launch (default 64, <= 1024)    */
    int32_t n_slots;      /* execution slots in flight (default 3, <= 16)      */
    int32_t flags;        /* render flags: SWF_MLP_BF16 (default), ...          */
    float key_factor;     /* key capacity headroom (default 1.5)               */
    uint64_t hbm_budget;  /* workspace bytes over all slots, 0 = unlimited     */
    int32_t use_graphs;   /* 1: replay captured graphs; 0: direct launches     */
    int32_t mixed;        /* 1: batch requests of different scenes together
                             (the default when cfg is NULL)                  */
    int32_t reserved[4];
} swf_serve_config;

typedef struct {
    double queue_us;      /* scheduled arrival -> launch                        */
    double service_us;    /* launch -> result in the caller's buffer            */
    double total_us;      /* scheduled arrival -> result in the caller's buffer */
    int32_t batch;        /* requests in its launch                             */
    int32_t bucket;       /* padded batch size of the launch                    */
    int32_t fallback;     /* 1 if re-rendered after a key overflow              */
    int32_t slot;         /* execution slot                                     */
} swf_req_stats;

/* Start the scheduler (cfg may be NULL for the defaults). */
swf_status swf_serve_start(swf_ctx *ctx, const swf_serve_config *cfg);
/* Queue one query: tx = 3 host floats, out_host = caller-owned host buffer of
 * H*W floats that receives the spectrum (kept valid until the request is
 * polled/waited). arrival_s = scheduled arrival on swf_serve_clock() (0: now).
 * Thread-safe. SWF_E_NOT_FOUND for an unknown scene, SWF_E_INVALID for a
 * non-finite tx. */
swf_status swf_serve_submit(swf_ctx *ctx, int32_t scene_id, const float *tx, float *out_host, double arrival_s,
                            uint64_t *ticket);
/* SWF_OK (result delivered, stats filled, ticket retired), SWF_E_PENDING, or
 * the request's error. Thread-safe. */
swf_status swf_serve_poll(swf_ctx *ctx, uint64_t ticket, swf_req_stats *stats);
/* As swf_serve_poll, blocking until the request is finished. */
swf_status swf_serve_wait(swf_ctx *ctx, uint64_t ticket, swf_req_stats *stats);
/* Finish in-flight launches and stop the scheduler. */
swf_status swf_serve_stop(swf_ctx *ctx);
/* counters[0..n): launches, completed requests, fallbacks, graph builds,
 * budget shrinks, workspace bytes over all slots, mixed launches, and the
 * distinct scenes summed over the mixed launches. */
swf_status swf_serve_counters(swf_ctx *ctx, uint64_t *counters, int32_t n);
/* The steady clock (seconds) that arrival times refer to. */
double swf_serve_clock(void);

#ifdef __cplusplus
}
#endif
#endif /* SWIFTWRF_H */
