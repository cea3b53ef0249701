// The paper's own spectrum model (Sec. 4.1, 4.2, 6.1): Gaussians with
// tanh-normalised centres, a Cholesky-parameterised covariance, an attenuation
// gate and a complex response psi in R^2, summed without order (the GMM
// rasterization equation), deformed by the paper's MLP (eight layers of 156
// with skip connections every two layers, residuals of the centre, psi and the
// gate only). The records and lists are those of the compositing path, so
// binning, sorting and tile ranges are shared; what differs is the preprocess,
// the MLP and the per-tile sum.
//
// Record of a pair: geo = centre as hi + lo (the tanh map is evaluated once per
// Gaussian in FP64, so the centre keeps full precision at any grid width),
// wm = the whitening factor M = L^-1 = [[1/l1, 0], [-l2/(l1 l3), 1/l3]]
// (Sigma^-1 = M^T M, q = |M d|^2, no inversion of Sigma), oa = the complex
// weight delta * psi, rect / count = tiles of the 3-sigma box
// (half extents 3 |l1| and 3 sqrt(l2^2 + l3^2)).
#include "cull.h"
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

__device__ __forceinline__ void write_rec(const Records& r, size_t row, const PairOut& o) {
    r.geo[row] = o.geo;
    r.wm[row] = o.wm;
    r.oa[row] = o.oa;
    r.rect[row] = make_uint2(o.rect_x, o.rect_y);
    r.count[row] = o.count;
}

// Deformed paper Gaussian -> record. cen = canonical centre (x_hi, y_hi, x_lo,
// y_lo); d = residuals (d_mu_x, d_mu_y, d_psi_re, d_psi_im, d_delta) or null.
__device__ __forceinline__ PairOut paper_pair(float4 cen, float l1, float l2, float l3, float a, float pr, float pi,
                                              const float* d, int W, int H, int TW, int TH, float inv_tile, int wrap,
                                              float gsx, float gsy) {
    PairOut r;
    float xh = cen.x, xl = cen.z, yh = cen.y, yl = cen.w;
    float dl = 1.0f / (1.0f + expf(-a));
    if (d) {
        float s, e;
        two_sum(xh, d[0], s, e);
        xh = s;
        xl += e;
        two_sum(yh, d[1], s, e);
        yh = s;
        yl += e;
        pr += d[2];
        pi += d[3];
        dl += d[4];
    }
    // renormalise the centre (|lo| small against hi)
    {
        float s, e;
        two_sum(xh, xl, s, e);
        xh = s;
        xl = e;
        two_sum(yh, yl, s, e);
        yh = s;
        yl = e;
    }
    const float i1 = 1.0f / l1, i3 = 1.0f / l3;
    float4 wmv = make_float4(i1, 0.0f, -l2 * i1 * i3, i3);
    float hx = 3.0f * fabsf(l1), hy = 3.0f * sqrtf(fmaf(l2, l2, l3 * l3));
    if (gsx != 1.0f || gsy != 1.0f) rescale_to_grid(gsx, gsy, xh, xl, yh, yl, hx, hy, wmv);
    hx += kExtentEps;
    hy += kExtentEps;
    r.geo = make_float4(xh, yh, xl, yl);
    r.wm = wmv;
    r.oa = make_float2(dl * pr, dl * pi);
    const float x0 = xh - hx, x1 = xh + hx, y0 = yh - hy, y1 = yh + hy;
    const bool fin = l1 != 0.0f && l3 != 0.0f && finitef(x0) && finitef(x1) && finitef(y0) && finitef(y1) &&
                     finitef(r.wm.x) && finitef(r.wm.z) && finitef(r.wm.w) && finitef(r.oa.x) && finitef(r.oa.y) &&
                     finitef(xl) && finitef(yl);
    const bool on = !(y1 < 0.0f) && !(y0 > (float)(H - 1)) && (wrap || (!(x1 < 0.0f) && !(x0 > (float)(W - 1))));
    if (!(fin && on)) {
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
        const float aa = x0 - k * Wf, bb = x1 - k * Wf;
        tx0 = min(TW - 1, (int)floorf(aa * inv_tile));
        tx1 = bb < Wf ? min(TW - 1, (int)floorf(bb * inv_tile)) : (int)floorf((bb - Wf) * inv_tile);
        if (x1 - x0 >= Wf || (bb >= Wf && tx1 >= tx0 - 1)) {
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

// Canonical centres in FP64 (x = (W/2)(tanh(c_x) + 1), y likewise with H) as
// hi + lo pairs, and the centre's positional encoding gamma(mu_hat) with 10
// bands (42 features, padded to 48 with zeros), mu_hat = (x / W, y / H).
__global__ __launch_bounds__(256) void paper_centers_kernel(const float* __restrict__ cx, const float* __restrict__ cy,
                                                            int n, int W, int H, float4* __restrict__ cen,
                                                            float* __restrict__ feat) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double x = 0.5 * (double)W * (tanh((double)cx[i]) + 1.0);
    const double y = 0.5 * (double)H * (tanh((double)cy[i]) + 1.0);
    const float xh = (float)x, yh = (float)y;
    cen[i] = make_float4(xh, yh, (float)(x - (double)xh), (float)(y - (double)yh));
    const double ux = x / (double)W, uy = y / (double)H;
    const float uxh = (float)ux, uyh = (float)uy;
    const float uxl = (float)(ux - (double)uxh), uyl = (float)(uy - (double)uyh);
    float* f = feat + (size_t)i * kPaperFeatStride;
    f[0] = uxh + uxl;
    f[1] = uyh + uyl;
#pragma unroll
    for (int k = 0; k < kPaperCenterBands; ++k) {
        float sx, cxv, sy, cyv;
        sincospi_scaled(uxh, uxl, k, sx, cxv);
        sincospi_scaled(uyh, uyl, k, sy, cyv);
        f[2 + 2 * k] = sx;
        f[3 + 2 * k] = sy;
        f[2 + 2 * kPaperCenterBands + 2 * k] = cxv;
        f[3 + 2 * kPaperCenterBands + 2 * k] = cyv;
    }
    for (int k = kPaperCenterFeat; k < kPaperFeatStride; ++k) f[k] = 0.0f;
}

// gamma(s_hat) with 6 bands per query: 39 features, padded to 48.
__global__ __launch_bounds__(64) void paper_tx_kernel(const float* __restrict__ tx, float lox, float loy, float loz,
                                                      float rx, float ry, float rz, float* __restrict__ out) {
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    float* o = out + (size_t)b * kPaperFeatStride;
    if (t < 3 * (kPaperTxBands + 1)) {
        const int dd = t % 3;
        const int k = t / 3;
        const float v = tx[b * 3 + dd];
        const float lo = dd == 0 ? lox : (dd == 1 ? loy : loz);
        const float rg = dd == 0 ? rx : (dd == 1 ? ry : rz);
        float s, e, hi, lo2;
        two_sum(v, -lo, s, e);
        div_two(s, rg, hi, lo2);
        lo2 += e / rg;
        if (k == 0) {
            o[dd] = hi + lo2;
        } else {
            float sv, cv;
            sincospi_scaled(hi, lo2, k - 1, sv, cv);
            o[3 + 3 * (k - 1) + dd] = sv;
            o[3 + 3 * kPaperTxBands + 3 * (k - 1) + dd] = cv;
        }
    } else if (t >= kPaperTxFeat && t < kPaperFeatStride) {
        o[t] = 0.0f;
    }
}

__global__ __launch_bounds__(256) void paper_static_kernel(PaperArgs a) {
    const size_t row = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t total = (size_t)a.N * a.B;
    if (row >= total) return;
    const int p = (int)(row % a.N);
    const PairOut o = paper_pair(a.cen[p], a.l1[p], a.l2[p], a.l3[p], a.att[p], a.pre[p], a.pim[p], nullptr, a.W,
                                 a.H, a.TW, a.TH, a.inv_tile, a.wrap, a.sx, a.sy);
    write_rec(a.rec, row, o);
}

// ---- paper MLP, FP32 on the matrix cores --------------------------------------
// v_mfma_f32_16x16x4_f32 (FP32 products, FP32 accumulation): per layer D = W H
// with 16 output units x 16 pairs per instruction, K = 4 inputs. A wave holds
// 2 x 16 pairs; every hidden state and the 81 input features stay in
// registers as B operands: lane l holds, for chunk c of a layer's input,
// feature k(c, l / 16) of pair l % 16. The result of output tile t (4 registers
// per lane: units 16 t + 4 (l / 16) + i, i = 0..3) is, after the ReLU, exactly
// the next layer's chunks 4 t + i once that layer's weights list their input
// columns in that order (fragment-major packing on upload, zero rows and
// columns for every pad: the 156 units are padded to 160, the 81 inputs to
// 96). A layer reads its input as [h chunks (40) | x chunks (24)] (layer 1: x
// only; the skip layers 3, 5, 7: both; the others: h only); a fragment of 4
// chunks is one 16-byte load per lane from the L2-resident weights, issued one
// fragment ahead.
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMNB = 2;        // column blocks of 16 pairs per wave
constexpr int kMWaves = 4;     // waves per block
constexpr int kHC = 40, kXC = 24;  // chunks of 4 inputs: hidden state, input features

template <bool kH, bool kX, int kTiles, bool kRelu>
__device__ __forceinline__ void paper_mfma_layer(const float4* __restrict__ wf, const float* __restrict__ bias,
                                                 int lane, const float (&hin)[kMNB][kHC],
                                                 const float (&x)[kMNB][kXC], float (&hout)[kMNB][kHC]) {
    constexpr int G = (kH ? kHC / 4 : 0) + (kX ? kXC / 4 : 0);  // 16-byte fragments per output tile
    constexpr int F = kTiles * G;
    // the next fragment is loaded while the current one's instructions run; the scheduling barrier after them
    // keeps that load where it is written (the compiler would sink it next to its use)
    float4 wn = wf[lane];
#pragma unroll
    for (int t = 0; t < kTiles; ++t) {
        const float4 b4 = *reinterpret_cast<const float4*>(bias + 16 * t + 4 * (lane >> 4));
        f32x4 acc[kMNB];
#pragma unroll
        for (int cb = 0; cb < kMNB; ++cb) acc[cb] = f32x4{b4.x, b4.y, b4.z, b4.w};
#pragma unroll
        for (int gq = 0; gq < G; ++gq) {
            const int f = t * G + gq;
            const float4 w = wn;
            if (f + 1 < F) wn = wf[((size_t)f + 1) * 64 + lane];
            const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = gq * 4 + j;
#pragma unroll
                for (int cb = 0; cb < kMNB; ++cb) {
                    const float bv = (kH && c < kHC) ? hin[cb][c] : x[cb][c - (kH ? kHC : 0)];
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[j], bv, acc[cb], 0, 0, 0);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int cb = 0; cb < kMNB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) hout[cb][4 * t + i] = kRelu ? fmaxf(acc[cb][i], 0.0f) : acc[cb][i];
    }
}

__global__ __launch_bounds__(64 * kMWaves, 2) void paper_mlp_kernel(PaperArgs a) {
    __shared__ float outv[kMWaves][16 * kMNB][kPaperOutPad];
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const size_t total = (size_t)a.N * a.B;
    const size_t p0 = ((size_t)blockIdx.x * kMWaves + wave) * (16 * kMNB);
    if (p0 < total) {  // wave-uniform
        // input features as B operands: x index 4 c + l / 16 (centre features 0..41, position features 42..80)
        float x[kMNB][kXC];
        const int g = lane >> 4;
#pragma unroll
        for (int cb = 0; cb < kMNB; ++cb) {
            const size_t row = p0 + 16 * cb + (lane & 15);
            const bool in = row < total;
            const int p = in ? (int)(row % a.N) : 0, b = in ? (int)(row / a.N) : 0;
#pragma unroll
            for (int c = 0; c < kXC; ++c) {
                const int j = 4 * c + g;
                float v = 0.0f;
                if (in && j < kPaperCenterFeat + kPaperTxFeat)
                    v = j < kPaperCenterFeat ? a.feat[(size_t)p * kPaperFeatStride + j]
                                             : a.txf[(size_t)b * kPaperFeatStride + (j - kPaperCenterFeat)];
                x[cb][c] = v;
            }
        }
        float hA[kMNB][kHC], hB[kMNB][kHC];
        const auto W = [&](int l) { return reinterpret_cast<const float4*>(a.wt[l]); };
        paper_mfma_layer<false, true, 10, true>(W(0), a.bt[0], lane, hB, x, hA);  // layer 1 (hB unused)
        for (int r = 0; r < 3; ++r) {
            paper_mfma_layer<true, false, 10, true>(W(1 + 2 * r), a.bt[1 + 2 * r], lane, hA, x, hB);
            paper_mfma_layer<true, true, 10, true>(W(2 + 2 * r), a.bt[2 + 2 * r], lane, hB, x, hA);  // skip
        }
        paper_mfma_layer<true, false, 10, true>(W(7), a.bt[7], lane, hA, x, hB);
        // output layer: one tile of 16 rows (5 used); lane l holds outputs 4 (l / 16) + i of pair l % 16
        paper_mfma_layer<true, false, 1, false>(reinterpret_cast<const float4*>(a.wo), a.bo, lane, hB, x, hA);
        if (g < 2) {
#pragma unroll
            for (int cb = 0; cb < kMNB; ++cb)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * g + i < kPaperOutPad) outv[wave][16 * cb + (lane & 15)][4 * g + i] = hA[cb][i];
        }
    }
    __syncthreads();
    if (p0 < total && lane < 16 * kMNB) {
        const size_t row = p0 + lane;
        if (row < total) {
            const int p = (int)(row % a.N);
            float d[kPaperOut];
#pragma unroll
            for (int k = 0; k < kPaperOut; ++k) d[k] = outv[wave][lane][k];
            if (a.delta_out)
#pragma unroll
                for (int k = 0; k < kPaperOut; ++k) a.delta_out[row * kPaperOut + k] = d[k];
            const PairOut o = paper_pair(a.cen[p], a.l1[p], a.l2[p], a.l3[p], a.att[p], a.pre[p], a.pim[p], d, a.W,
                                         a.H, a.TW, a.TH, a.inv_tile, a.wrap, a.sx, a.sy);
            if (a.rec.geo) write_rec(a.rec, row, o);
        }
    }
}

// ---- GMM sum per tile ----------------------------------------------------------
// One workgroup per (query, 16 x 16 tile), one pixel per thread, each wave an
// 8 x 8 quadrant. The tile's list is staged 256 records at a time; a wave
// visits only the entries whose 3-sigma ellipse reaches its quadrant (the
// others add nothing to any of its pixels) and adds psi delta exp(-q/2) for
// q <= 9, in list order. No ordering, termination or clamp: the whole list is
// walked. Output |sum| and, when asked, the two channels.
template <bool kWrap>
__global__ __launch_bounds__(256) void gmm_blend_kernel(const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ vals,
                                                        const float4* __restrict__ geo, const float4* __restrict__ wm,
                                                        const float2* __restrict__ oa, int H, int W, int TW,
                                                        int tiles, float* __restrict__ out,
                                                        float* __restrict__ chan) {
    constexpr int kN = 256;
    constexpr int kWaves = 4;
    __shared__ float4 s_rec[2 * kN];
    __shared__ uint8_t s_mask[kN];
    __shared__ uint16_t s_idx[kWaves][kN];
    const int gtile = blockIdx.x;
    const int b = gtile / tiles;
    const int t = gtile - b * tiles;
    const int tx = t % TW, ty = t / TW;
    const int wq = (int)(threadIdx.x >> 6), lq = (int)(threadIdx.x & 63);
    const int lx = (wq & 1) * 8 + (lq & 7), ly = (wq >> 1) * 8 + (lq >> 3);
    const int px = tx * 16 + lx, py = ty * 16 + ly;
    const bool inside = px < W && py < H;
    const int bx0 = (tx * 16) & ~63, by0 = (ty * 16) & ~63;
    const float x0 = (float)bx0, y0 = (float)by0;
    const float fx = (float)(px - bx0), fy = (float)(py - by0);
    const float Wf = kWrap ? (float)W : 0.0f, rw = kWrap ? 1.0f / (float)W : 0.0f;
    const float cx = (float)(tx * 16 - bx0) + 7.5f;
    const uint2 rg = ranges[gtile];
    float re = 0.0f, im = 0.0f;
    for (uint32_t start = rg.x; start < rg.y; start += kN) {
        __syncthreads();
        const uint32_t i = start + threadIdx.x;
        const int cnt = (int)min((uint32_t)kN, rg.y - start);
        if (i < rg.y) {
            const uint32_t v = vals[i];
            const float4 g = geo[v];
            const float2 pos = kWrap ? staged_mean(g, x0, y0, Wf, cx) : make_float2((g.x - x0) + g.z, (g.y - y0) + g.w);
            const float4 m = wm[v];
            const float2 o = oa[v];
            s_rec[2 * threadIdx.x] = make_float4(pos.x, pos.y, o.x, o.y);
            s_rec[2 * threadIdx.x + 1] = m;
            s_mask[threadIdx.x] = (kWrap && fabsf(pos.x - cx) > 0.5f * Wf - 16.0f)
                                      ? (uint8_t)0xf
                                      : (uint8_t)wave_quads_mask(m, pos, (float)(tx * 16 - bx0),
                                                                 (float)(ty * 16 - by0), kQMax);
        }
        __syncthreads();
        uint16_t* idx = s_idx[wq];
        int nlist = 0;
#pragma unroll
        for (int c = 0; c < kWaves; ++c) {
            const int jl = c * 64 + lq;
            const bool f = jl < cnt && ((s_mask[jl] >> wq) & 1u);
            const uint64_t bal = __ballot(f);
            if (f) idx[nlist + __popcll(bal & ((1ull << lq) - 1ull))] = (uint16_t)jl;
            nlist += __popcll(bal);
        }
        __builtin_amdgcn_wave_barrier();
        for (int n = 0; n < nlist; ++n) {
            const int j = idx[n];
            const float4 r0 = s_rec[2 * j];
            const float4 m = s_rec[2 * j + 1];
            float dx, dy, u, w;
            const float q = kWrap ? blend_q_wrap(fx, fy, make_float2(r0.x, r0.y), m, Wf, rw, dx, dy, u, w)
                                  : blend_q(fx, fy, make_float2(r0.x, r0.y), m, dx, dy, u, w);
            const float e = q <= kQMax ? __builtin_amdgcn_exp2f(q * kNegHalfLog2e) : 0.0f;
            re = fmaf(r0.z, e, re);
            im = fmaf(r0.w, e, im);
        }
    }
    if (inside) {
        const size_t pix = (size_t)b * H * W + (size_t)py * W + px;
        out[pix] = sqrtf(fmaf(re, re, im * im));
        if (chan) {
            const size_t plane = (size_t)H * W;
            chan[(size_t)b * 2 * plane + (size_t)py * W + px] = re;
            chan[(size_t)b * 2 * plane + plane + (size_t)py * W + px] = im;
        }
    }
}

}  // namespace

void launch_paper_centers(const DevScene& d, hipStream_t st) {
    if (d.n > 0)
        paper_centers_kernel<<<(d.n + 255) / 256, 256, 0, st>>>(d.pcx, d.pcy, d.n, d.W, d.H, d.pcen, d.pfeat);
}

void launch_paper_tx(const DevScene& d, const float* tx, int B, float* txf, hipStream_t st) {
    paper_tx_kernel<<<B, 64, 0, st>>>(tx, d.room_lo[0], d.room_lo[1], d.room_lo[2], d.room_hi[0] - d.room_lo[0],
                                      d.room_hi[1] - d.room_lo[1], d.room_hi[2] - d.room_lo[2], txf);
}

static PaperArgs paper_args(const DevScene& d, int B, const Grid& g, const Records& r) {
    PaperArgs a{};
    a.N = d.n;
    a.B = B;
    a.H = g.H;
    a.W = g.W;
    a.TW = g.TW;
    a.TH = g.TH;
    a.wrap = g.wrap;
    a.sx = g.sx;
    a.sy = g.sy;
    a.inv_tile = 1.0f / (float)g.tile;
    a.cen = d.pcen;
    a.l1 = d.pl1;
    a.l2 = d.pl2;
    a.l3 = d.pl3;
    a.att = d.patt;
    a.pre = d.ppre;
    a.pim = d.ppim;
    a.feat = d.pfeat;
    for (int l = 0; l < kPaperLayers; ++l) {
        a.wt[l] = d.pwt[l];
        a.bt[l] = d.pbt[l];
    }
    a.wo = d.pwt[kPaperLayers];
    a.bo = d.pbt[kPaperLayers];
    a.rec = r;
    return a;
}

void launch_paper_static(const DevScene& d, int B, const Grid& g, const Records& r, hipStream_t st) {
    const size_t total = (size_t)d.n * B;
    if (!total) return;
    PaperArgs a = paper_args(d, B, g, r);
    paper_static_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(a);
}

void launch_paper_mlp(const DevScene& d, const float* txf, int B, const Grid& g, const Records& r, float* delta_out,
                      hipStream_t st) {
    const size_t total = (size_t)d.n * B;
    if (!total) return;
    PaperArgs a = paper_args(d, B, g, r);
    a.txf = txf;
    a.delta_out = delta_out;
    const size_t per_block = (size_t)kMWaves * 16 * kMNB;
    paper_mlp_kernel<<<(unsigned)((total + per_block - 1) / per_block), 64 * kMWaves, 0, st>>>(a);
}

void launch_gmm_blend(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g, float* out,
                      float* chan, hipStream_t st) {
    const unsigned blocks = (unsigned)(B * g.tiles);
    if (!blocks) return;
    if (g.wrap)
        gmm_blend_kernel<true><<<blocks, 256, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles, out,
                                                       chan);
    else
        gmm_blend_kernel<false><<<blocks, 256, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles,
                                                        out, chan);
}

}  // namespace swf
