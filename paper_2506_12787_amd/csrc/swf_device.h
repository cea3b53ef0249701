// Device-side helpers shared by the HIP translation units of libswiftwrf:
// blending constants, the per-pair record layout and the preprocess step
// (deform -> whitening factor -> 3-sigma extent -> tile rectangle).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swf {

// Blending rule constants (Sec. 3.2 blending with the 3-sigma cutoff).
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;
constexpr float kQMax = 9.0f;
constexpr float kExtentEps = 1e-3f;           // binning margin on the 3-sigma half extent (px)
constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2

constexpr int kMeanBands = 6;
constexpr int kTxBands = 10;
constexpr int kMeanFeat = 2 * (2 * kMeanBands + 1);  // 26
constexpr int kTxFeat = 3 * (2 * kTxBands + 1);      // 63
constexpr int kOut = 7;

// Reason a pair was culled, kept in rect_y of a record whose count is 0 (0: a
// padding pair of a Gaussian with a NaN depth, never preprocessed).
constexpr uint32_t kCullNonFinite = 1;  // a non-finite deformed parameter or a degenerate covariance
constexpr uint32_t kCullOffGrid = 2;    // the 3-sigma box misses the pixel grid

// Per (query, Gaussian) pair record, three arrays of vectors:
//   geo  float4 (mx_hi, my_hi, mx_lo, my_lo): deformed mean as an unevaluated
//        sum hi + lo (exact value of mu0 + d_mu), so that tile-relative offsets
//        keep full precision at any grid width
//   wm   float4 (m11, m12, m21, m22): whitening factor M = S^-1 R^T with
//        Sigma^-1 = M^T M, so q = |M d|^2 (no 2x2 inversion, no cancellation)
//   oa   float2 (opacity, amplitude)
// plus rect (uint2: tx0 | tx1 << 16, ty0 | ty1 << 16) and count (uint32 tiles).
struct PairOut {
    float4 geo;
    float4 wm;
    float2 oa;
    uint32_t rect_x, rect_y;
    uint32_t count;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ bool finitef(float v) { return __builtin_isfinite(v); }

// A render at another resolution of the same field of view: scene pixel
// coordinates scale by (sx, sy) per axis, so the mean (hi + lo, the product's
// rounding error kept in lo), the 3-sigma half extents and Sigma' = S Sigma S
// follow; the whitening factor becomes M S^-1 (its columns divided by sx, sy).
__device__ __forceinline__ void rescale_to_grid(float sx, float sy, float& xh, float& xl, float& yh, float& yl,
                                                float& hx, float& hy, float4& m) {
    const float px = xh * sx, py = yh * sy;
    const float ex = fmaf(xh, sx, -px), ey = fmaf(yh, sy, -py);
    float s, e;
    two_sum(px, fmaf(xl, sx, ex), s, e);
    xh = s;
    xl = e;
    two_sum(py, fmaf(yl, sy, ey), s, e);
    yh = s;
    yl = e;
    hx *= sx;
    hy *= sy;
    const float ix = 1.0f / sx, iy = 1.0f / sy;
    m = make_float4(m.x * ix, m.y * iy, m.z * ix, m.w * iy);
}

// Deformed Gaussian -> record. mean = (mx0 + dmx, my0 + dmy); all other
// parameters already deformed. tile is 8 or 16 (power of two, so the division
// of an edge coordinate by the tile size is exact). wrap: azimuth is periodic
// with period W (0 and 360 degrees are one direction): the box's columns are
// taken modulo W. The box is shifted by whole periods so that its left edge
// lies in [0, W); if its right edge then reaches W it continues at column 0,
// which the record encodes as tx1 < tx0 (columns tx0 .. TW-1, then 0 .. tx1); a
// box at least W wide, or whose two pieces meet, covers every column.
__device__ __forceinline__ PairOut preprocess_pair(float mx0, float my0, float dmx, float dmy, float lsx, float lsy,
                                                   float rot, float logit, float amp, int W, int H, int TW, int TH,
                                                   float inv_tile, int wrap = 0, float gsx = 1.0f,
                                                   float gsy = 1.0f) {
    PairOut r;
    float mxh, mxl, myh, myl;
    two_sum(mx0, dmx, mxh, mxl);
    two_sum(my0, dmy, myh, myl);
    float s, c;
    sincosf(rot, &s, &c);
    const float isx = expf(-lsx), isy = expf(-lsy);
    const float vx = expf(2.0f * lsx), vy = expf(2.0f * lsy);
    const float sxx = c * c * vx + s * s * vy;
    const float syy = s * s * vx + c * c * vy;
    float hx, hy;
    float4 wmv = make_float4(c * isx, s * isx, -s * isy, c * isy);
    if (gsx != 1.0f || gsy != 1.0f) {
        hx = 3.0f * sqrtf(sxx);
        hy = 3.0f * sqrtf(syy);
        rescale_to_grid(gsx, gsy, mxh, mxl, myh, myl, hx, hy, wmv);
        hx += kExtentEps;
        hy += kExtentEps;
    } else {
        hx = 3.0f * sqrtf(sxx) + kExtentEps;
        hy = 3.0f * sqrtf(syy) + kExtentEps;
    }
    const float op = 1.0f / (1.0f + expf(-logit));
    r.geo = make_float4(mxh, myh, mxl, myl);
    r.wm = wmv;
    r.oa = make_float2(op, amp);
    const float x0 = mxh - hx, x1 = mxh + hx, y0 = myh - hy, y1 = myh + hy;
    const bool fin = finitef(x0) && finitef(x1) && finitef(y0) && finitef(y1) && finitef(r.wm.x) &&
                     finitef(r.wm.y) && finitef(r.wm.z) && finitef(r.wm.w) && finitef(op) && finitef(amp) &&
                     finitef(mxl) && finitef(myl);
    const bool on = !(y1 < 0.0f) && !(y0 > (float)(H - 1)) && (wrap || (!(x1 < 0.0f) && !(x0 > (float)(W - 1))));
    if (!(fin && on)) {
        // culled: no tiles; rect_y keeps the reason for the status counters
        r.rect_x = 0;
        r.rect_y = fin ? kCullOffGrid : kCullNonFinite;
        r.count = 0;
        return r;
    }
    int tx0, tx1;
    if (!wrap) {
        tx0 = max(0, min(TW - 1, (int)floorf(x0 * inv_tile)));
        tx1 = max(0, min(TW - 1, (int)floorf(x1 * inv_tile)));
    } else {
        const float Wf = (float)W;
        const float k = floorf(x0 / Wf);
        const float a = x0 - k * Wf, b = x1 - k * Wf;
        tx0 = min(TW - 1, (int)floorf(a * inv_tile));
        tx1 = b < Wf ? min(TW - 1, (int)floorf(b * inv_tile)) : (int)floorf((b - Wf) * inv_tile);
        if (x1 - x0 >= Wf || (b >= Wf && tx1 >= tx0 - 1)) {
            tx0 = 0;
            tx1 = TW - 1;
        }
    }
    const int ty0 = max(0, min(TH - 1, (int)floorf(y0 * inv_tile)));
    const int ty1 = max(0, min(TH - 1, (int)floorf(y1 * inv_tile)));
    r.rect_x = (uint32_t)tx0 | ((uint32_t)tx1 << 16);
    r.rect_y = (uint32_t)ty0 | ((uint32_t)ty1 << 16);
    const int cols = tx1 >= tx0 ? tx1 - tx0 + 1 : TW - tx0 + tx1 + 1;
    r.count = (uint32_t)(cols * (ty1 - ty0 + 1));
    return r;
}

// One blend evaluation of a list entry at a pixel (tile-block-relative
// coordinates): q = |M d|^2 with d = pixel - mean. Forward and backward share
// this code so that their cutoff / skip decisions are bitwise identical.
__device__ __forceinline__ float blend_q(float fx, float fy, float2 p, float4 m, float& dx, float& dy, float& u,
                                         float& w) {
    dx = fx - p.x;
    dy = fy - p.y;
    u = fmaf(m.x, dx, m.y * dy);
    w = fmaf(m.z, dx, m.w * dy);
    return fmaf(u, u, w * w);
}
// The same with periodic azimuth (period Wf, 1/Wf = rw): dx is taken to the
// nearest image of the staged mean, which the staging already chose for the
// tile, so the correction is zero except for pixels more than half a period
// from that image (only a Gaussian wider than about half the grid reaches them).
__device__ __forceinline__ float blend_q_wrap(float fx, float fy, float2 p, float4 m, float Wf, float rw, float& dx,
                                              float& dy, float& u, float& w) {
    dx = fx - p.x;
    dx = fmaf(-Wf, rintf(dx * rw), dx);
    dy = fy - p.y;
    u = fmaf(m.x, dx, m.y * dy);
    w = fmaf(m.z, dx, m.w * dy);
    return fmaf(u, u, w * w);
}

// Block-relative staged mean of a record: (hi - block origin) + lo in full
// precision. With periodic azimuth (Wf > 0) the hi part first moves by whole
// periods to the image nearest the tile centre cx (exact: a multiple of an
// integer subtracted from a value of at most a few periods).
__device__ __forceinline__ float2 staged_mean(float4 g, float x0, float y0, float Wf, float cx) {
    float hx = g.x - x0;
    if (Wf > 0.0f) hx = fmaf(-Wf, rintf((hx - cx) / Wf), hx);
    return make_float2(hx + g.z, (g.y - y0) + g.w);
}

// opacity * exp(-q/2) before the 0.99 clamp
__device__ __forceinline__ float blend_raw_alpha(float q, float op) {
    return op * __builtin_amdgcn_exp2f(q * kNegHalfLog2e);
}

// Order-preserving map of an FP32 depth to uint32 (-0 like +0).
__host__ __device__ __forceinline__ uint32_t depth_key_bits(float d) {
    if (d == 0.0f) d = 0.0f;
    uint32_t u;
    __builtin_memcpy(&u, &d, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// sin(pi x) and cos(pi x) of x = hi + lo (an unevaluated sum, |lo| tiny) after
// scaling by 2^k: the scaled hi is reduced exactly modulo 2 before adding the
// scaled lo, so the phase keeps the accuracy of the two-term input.
__device__ __forceinline__ void sincospi_scaled(float hi, float lo, int k, float& sv, float& cv) {
    const float sh = ldexpf(hi, k);                        // exact
    const float red = sh - 2.0f * rintf(0.5f * sh);        // exact: sh mod 2 in [-1, 1]
    const float t = red + ldexpf(lo, k);
    sv = sinpif(t);
    cv = cospif(t);
}

// (a / b) as hi + lo with lo the rounded residual: a = hi * b + r exactly.
__device__ __forceinline__ void div_two(float a, float b, float& hi, float& lo) {
    hi = a / b;
    const float r = fmaf(-hi, b, a);
    lo = r / b;
}

// gamma(mu_hat) of a canonical mean, mu_hat = (mx / W, my / H), in the
// order [mu_hat, sin(2^k pi mu_hat) for k < 6, cos(2^k pi mu_hat) for k < 6].
__device__ __forceinline__ void mean_features(float mx, float my, int W, int H, float* out) {
    float hx, lx, hy, ly;
    div_two(mx, (float)W, hx, lx);
    div_two(my, (float)H, hy, ly);
    out[0] = hx + lx;
    out[1] = hy + ly;
#pragma unroll
    for (int k = 0; k < kMeanBands; ++k) {
        float sx, cx, sy, cy;
        sincospi_scaled(hx, lx, k, sx, cx);
        sincospi_scaled(hy, ly, k, sy, cy);
        out[2 + 2 * k] = sx;
        out[3 + 2 * k] = sy;
        out[2 + 2 * kMeanBands + 2 * k] = cx;
        out[3 + 2 * kMeanBands + 2 * k] = cy;
    }
}

}  // namespace swf
