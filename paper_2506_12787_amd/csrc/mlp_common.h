// Arguments and the fused epilogue shared by the FP32 and BF16 deformation-MLP
// kernels: residuals -> deformed Gaussian (Sec. 4.2, G^s = G^0 + dG) -> record.
#pragma once
#include "kernels.h"
#include "swf_device.h"

namespace swf {

__device__ __forceinline__ void write_record(const Records& r, size_t row, const PairOut& o) {
    r.geo[row] = o.geo;
    r.wm[row] = o.wm;
    r.oa[row] = o.oa;
    r.rect[row] = make_uint2(o.rect_x, o.rect_y);
    r.count[row] = o.count;
}

struct MlpArgs {
    int N, B, H, W, TW, TH, n_live, n_mid;
    float inv_tile;
    int paper_mask;
    int wrap;            // periodic azimuth: tile rectangles wrap around the grid width
    int sW, sH;          // the scene's own grid (the mean features' normalisation)
    float sx, sy;        // render pixels per scene pixel
    const float *mx, *my, *lsx, *lsy, *rot, *logit, *amp;
    const float* qs;
    const float4* wf1;   // fragment-major FP32 weights: layer 1's mean part, hidden layers, output layer
    const float4* wfh[7];
    const float* bh[7];
    const float4* wfo;
    const float* bo;     // output bias (7)
    const float* bo16;   // the same padded to 16
    Records rec;         // rec.geo == nullptr: no records (activation recompute only)
    float* delta_out;
    float* act_out[8];   // FP32 kernel: store hidden activations H_l [P][256] when set (the BF16 kernel takes its own)
};


// Epilogue shared by both MLP kernels: residuals -> deformed Gaussian -> record.
__device__ __forceinline__ void deform_epilogue(const MlpArgs& a, size_t row, int p, const float* d) {
    float dv[kOut];
#pragma unroll
    for (int k = 0; k < kOut; ++k) dv[k] = d[k];
    if (a.paper_mask) dv[2] = dv[3] = dv[4] = 0.0f;
    if (a.delta_out) {
#pragma unroll
        for (int k = 0; k < kOut; ++k) a.delta_out[row * kOut + k] = dv[k];
    }
    PairOut o;
    if (p < a.n_live) {
        o = preprocess_pair(a.mx[p], a.my[p], dv[0], dv[1], a.lsx[p] + dv[2], a.lsy[p] + dv[3], a.rot[p] + dv[4],
                            a.logit[p] + dv[5], a.amp[p] + dv[6], a.W, a.H, a.TW, a.TH, a.inv_tile, a.wrap, a.sx,
                            a.sy);
    } else {
        o.geo = make_float4(0, 0, 0, 0);
        o.wm = make_float4(0, 0, 0, 0);
        o.oa = make_float2(0, 0);
        o.rect_x = o.rect_y = 0;
        o.count = 0;
    }
    if (a.rec.geo) write_record(a.rec, row, o);
}

// Records of a mixed batch's pair: residuals -> deformed Gaussian -> record, with the pair's own scene.
__device__ __forceinline__ void mix_epilogue(const MixScene& s, const MlpArgs& a, size_t row, int p, const float* d) {
    float dv[kOut];
#pragma unroll
    for (int k = 0; k < kOut; ++k) dv[k] = d[k];
    if (a.paper_mask) dv[2] = dv[3] = dv[4] = 0.0f;
    PairOut o;
    if (p < s.n_live) {
        o = preprocess_pair(s.mx[p], s.my[p], dv[0], dv[1], s.lsx[p] + dv[2], s.lsy[p] + dv[3], s.rot[p] + dv[4],
                            s.logit[p] + dv[5], s.amp[p] + dv[6], s.W, s.H, s.TW, s.TH, a.inv_tile, a.wrap);
    } else {
        o.geo = make_float4(0, 0, 0, 0);
        o.wm = make_float4(0, 0, 0, 0);
        o.oa = make_float2(0, 0);
        o.rect_x = o.rect_y = 0;
        o.count = 0;
    }
    write_record(a.rec, row, o);
}

inline MlpArgs make_args(const DevScene& s, const float* qs, int B, const Grid& g, bool paper_mask, const Records& r,
                  float* delta_out) {
    MlpArgs a{};
    a.N = s.n;
    a.B = B;
    a.H = g.H;
    a.W = g.W;
    a.TW = g.TW;
    a.TH = g.TH;
    a.n_live = s.n_live;
    a.inv_tile = 1.0f / (float)g.tile;
    a.paper_mask = paper_mask ? 1 : 0;
    a.wrap = g.wrap;
    a.sW = s.W;
    a.sH = s.H;
    a.sx = g.sx;
    a.sy = g.sy;
    a.mx = s.mx; a.my = s.my; a.lsx = s.lsx; a.lsy = s.lsy; a.rot = s.rot; a.logit = s.logit; a.amp = s.amp;
    a.qs = qs;
    a.n_mid = s.has_mlp ? s.n_hidden - 1 : 0;
    if (s.has_mlp && s.f32_frag) {
        a.wf1 = reinterpret_cast<const float4*>(s.f32_frag);
        for (int l = 0; l < a.n_mid && l < 7; ++l)
            a.wfh[l] = reinterpret_cast<const float4*>(s.f32_frag + frag_hidden_at(l + 1));
        a.wfo = reinterpret_cast<const float4*>(s.f32_frag + frag_out_at(s.n_hidden));
        a.bo16 = s.f32_frag + frag_out_at(s.n_hidden) + kFragOut;
    }
    for (int l = 0; l < a.n_mid && l < 7; ++l) a.bh[l] = s.b[l + 1];
    a.bo = s.has_mlp ? s.b[s.n_hidden] : nullptr;
    a.rec = r;
    a.delta_out = delta_out;
    return a;
}


}  // namespace swf
