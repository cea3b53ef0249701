// Per-wave culling of list entries in the blend kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

namespace swf {

// Minimum over the box [x0, x1] x [y0, y1] (offsets from the mean) of the
// quadratic form a x^2 + 2 b x y + c y^2 (positive definite): 0 if the box
// holds the origin, else the least of the four edge minima (on an edge x = X
// the form is smallest at y = -b X / c, clamped to the edge).
__device__ __forceinline__ float box_min_q(float a, float b, float c, float x0, float x1, float y0, float y1) {
    if (x0 <= 0.0f && x1 >= 0.0f && y0 <= 0.0f && y1 >= 0.0f) return 0.0f;
    const float ra = -b / a, rc = -b / c;
    auto qf = [&](float x, float y) { return fmaf(a * x, x, fmaf(2.0f * b * x, y, c * y * y)); };
    const float ya = fminf(fmaxf(rc * x0, y0), y1), yb = fminf(fmaxf(rc * x1, y0), y1);
    const float xa = fminf(fmaxf(ra * y0, x0), x1), xb = fminf(fmaxf(ra * y1, x0), x1);
    return fminf(fminf(qf(x0, ya), qf(x1, yb)), fminf(qf(xa, y0), qf(xb, y1)));
}

// Bit k set unless the entry (block-relative mean `pos`, whitening factor m,
// q = |m d|^2) exceeds the cutoff, with a margin, on the whole 8 x 8 quadrant
// k of a 16 x 16 tile (k = 2 * row half + column half; c0, r0: its first
// column and row). NaN never culls.
__device__ __forceinline__ uint32_t wave_quads_mask(float4 m, float2 pos, float c0, float r0, float qmax) {
    const float a = fmaf(m.x, m.x, m.z * m.z), b = fmaf(m.x, m.y, m.z * m.w), c = fmaf(m.y, m.y, m.w * m.w);
    const float x0 = c0 - pos.x, y0 = r0 - pos.y;
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float xa = x0 + 8.0f * (k & 1), ya = y0 + 8.0f * (k >> 1);
        const float qm = box_min_q(a, b, c, xa, xa + 7.0f, ya, ya + 7.0f);
        bits |= !(qm > qmax * 1.001f + 1e-3f) ? 1u << k : 0u;
    }
    return bits;
}

}  // namespace swf
