// Per-tile front-to-back blending (Sec. 3.2 blending rule applied to the 2D
// Gaussian kernel of Sec. 4.1, one workgroup per (query, tile)).
//
// Each workgroup owns one TILE x TILE pixel tile, one pixel per thread. It walks
// the tile's depth-ordered list in batches of TILE*TILE records: every thread
// stages one record into LDS (mean re-expressed relative to the enclosing
// 64-pixel block, in full precision from the hi + lo pair), then every thread composites its
// pixel over the batch. A block-wide vote ends the walk once every pixel has
// reached the transmittance floor.
#include "cull.h"
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

__device__ __forceinline__ unsigned lane_id() { return threadIdx.x & 63u; }

// kCount: instead of writing the spectrum, add to work[0] the number of (pixel,
// list entry) evaluations the rule needs (entries whose quadratic form is
// within the 3-sigma cutoff at the pixel, up to and including the one that ends
// it) and to work[1] the number of records staged in LDS.
//
// kWrap: periodic azimuth (period W): each staged mean is the image nearest the
// tile, every evaluation takes the displacement to the nearest image, and an
// entry whose image lies nearly half a period from the tile is not culled.
// kMix: the workgroup's global tile belongs to a query of a mixed batch (its
// query, grid and output offset come from the batch's tables; workgroups past
// the batch's tiles exit).
//
// kVisit: the rendering walk itself (culling, termination, groups of 8), but
// instead of writing the spectrum it adds to work[2] the lane-evaluations it
// executes (every lane of a wave evaluates each entry the wave visits), for the
// ratio of executed to needed evaluations.
template <int TILE, bool kCount = false, bool kAux = true, bool kWrap = false, bool kMix = false, bool kVisit = false>
__global__ __launch_bounds__(TILE* TILE) void blend_forward_kernel(const uint2* __restrict__ ranges,
                                                                    const uint32_t* __restrict__ vals,
                                                                    const float4* __restrict__ geo,
                                                                    const float4* __restrict__ wm,
                                                                    const float2* __restrict__ oa, int H, int W,
                                                                    int TW, int tiles, float* __restrict__ out,
                                                                    float* __restrict__ aux_T,
                                                                    uint32_t* __restrict__ aux_last,
                                                                    unsigned long long* __restrict__ work = nullptr,
                                                                    MixBatch mix = MixBatch{}) {
    constexpr int kN = TILE * TILE;
    constexpr int kUnroll = 8;  // entries per unrolled group (kN is a multiple)
    static_assert(kN % 64 == 0, "whole waves per tile");
    // Staged record j, 32 bytes: s_rec[2j] = (block-relative mean x, y, opacity,
    // amplitude), s_rec[2j + 1] = the whitening rows M. Entry kN is a
    // never-contributing dummy (opacity 0) used as padding.
    __shared__ float4 s_rec[2 * (kN + 1)];
    // 16x16 tiles: bit w of s_strip[j] is set unless entry j's quadratic form
    // exceeds the cutoff (with a margin) everywhere on the 8 x 8 quadrant of
    // wave w; each wave walks only those entries (the others
    // fail the cutoff at every one of its pixels), from its own compacted list
    // s_idx[w] (byte offsets of the records in s_rec) padded with the dummy.
    constexpr bool kCull = TILE == 16 && !kCount;
    constexpr int kWaves = kN / 64;
    __shared__ uint8_t s_strip[kCull ? kN : 1];
    __shared__ __attribute__((aligned(16))) uint32_t s_idx[kCull ? kWaves : 1][kN + kUnroll];
    if (threadIdx.x == 0) {
        s_rec[2 * kN] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        s_rec[2 * kN + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }

    const int gtile = blockIdx.x;
    int b, t;
    if constexpr (kMix) {
        // uniform over the workgroup: a query of the batch and its scene's grid
        if (gtile >= mix.queries[mix.B].tile_base) return;
        const int q = mix_find(mix.queries, mix.B, gtile, [](const MixQuery& x) { return x.tile_base; });
        const MixScene& sc = mix.scenes[mix.queries[q].scene];
        H = sc.H;
        W = sc.W;
        TW = sc.TW;
        t = gtile - mix.queries[q].tile_base;
        out += mix.queries[q].out_base;
        b = 0;
    } else {
        b = gtile / tiles;
        t = gtile - b * tiles;
    }
    const int tx = t % TW, ty = t / TW;
    // culled 16x16 tiles: wave w covers the 8x8 quadrant (w & 1, w >> 1) and
    // lane l its pixel (l & 7, l >> 3); otherwise pixels are row-major
    const int wq = (int)(threadIdx.x >> 6), lq = (int)(threadIdx.x & 63);
    const int lx = kCull ? (wq & 1) * 8 + (lq & 7) : (int)threadIdx.x % TILE;
    const int ly = kCull ? (wq >> 1) * 8 + (lq >> 3) : (int)threadIdx.x / TILE;
    const int px = tx * TILE + lx, py = ty * TILE + ly;
    const bool inside = px < W && py < H;
    // Offsets are taken relative to the enclosing 64-pixel block, the same for
    // every tile size <= 64, so the arithmetic does not depend on the tiling.
    const int bx0 = (tx * TILE) & ~63, by0 = (ty * TILE) & ~63;
    const float x0 = (float)bx0, y0 = (float)by0;
    const float fx = (float)(px - bx0), fy = (float)(py - by0);
    const float Wf = kWrap ? (float)W : 0.0f, rw = kWrap ? 1.0f / (float)W : 0.0f;
    const float cx = (float)(tx * TILE - bx0) + 0.5f * (float)(TILE - 1);  // tile centre, block-relative

    const uint2 rg = ranges[gtile];
    float T = 1.0f, C = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    uint32_t evals = 0, staged = 0, visits = 0;

    for (uint32_t start = rg.x; start < rg.y; start += kN) {
        if (__syncthreads_count(done) == kN) break;
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
            if (kCull)  // block-relative first column and row of the tile
                s_strip[threadIdx.x] =
                    (kWrap && fabsf(pos.x - cx) > 0.5f * Wf - (float)TILE)
                        ? (uint8_t)0xf
                        : (uint8_t)wave_quads_mask(m, pos, (float)(tx * TILE - bx0), (float)(ty * TILE - by0), kQMax);
        } else if ((int)threadIdx.x < ((cnt + kUnroll - 1) & ~(kUnroll - 1))) {
            // padding up to the unrolled length: opacity 0 never contributes
            s_rec[2 * threadIdx.x] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_rec[2 * threadIdx.x + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        __syncthreads();
        if (kCount) staged += (uint32_t)cnt;
        const uint32_t base = start - rg.x + 1u;  // 1-based list position of entry 0 of the batch
        // Branch-free walk: every lane evaluates each entry its wave visits and
        // commits it only if it passes the cutoff, the alpha skip and the
        // termination test. The committed arithmetic is exactly the rule's; what
        // is avoided is per-entry divergent control flow (scalar exec-mask work
        // that would otherwise outweigh the vector work). With 16x16 tiles a
        // wave visits only the entries whose band meets its rows (the set bits of
        // a ballot, in list order). A wave leaves the batch once all its pixels
        // are done.
        if (kCull) {
            const int wv = threadIdx.x >> 6;
            uint32_t* idx = s_idx[wv];
            int nlist = 0;
#pragma unroll
            for (int c = 0; c < kWaves; ++c) {
                const int jl = c * 64 + (int)lane_id();
                const bool f = jl < cnt && ((s_strip[jl] >> wv) & 1u);
                const uint64_t bal = __ballot(f);
                if (f) idx[nlist + __popcll(bal & ((1ull << lane_id()) - 1ull))] = (uint32_t)jl * 32u;
                nlist += __popcll(bal);
            }
            if ((int)lane_id() < kUnroll) idx[nlist + lane_id()] = (uint32_t)kN * 32u;  // padding
            __builtin_amdgcn_wave_barrier();
            for (int j0 = 0; j0 < nlist; j0 += kUnroll) {
                if (__all(done)) break;
                if (kVisit) visits += kUnroll;
                const uint4 ja = *reinterpret_cast<const uint4*>(idx + j0);  // 8 record offsets
                const uint4 jb = *reinterpret_cast<const uint4*>(idx + j0 + 4);
                const uint32_t jw[8] = {ja.x, ja.y, ja.z, ja.w, jb.x, jb.y, jb.z, jb.w};
#pragma unroll
                for (int jj = 0; jj < kUnroll; ++jj) {
                    const char* rp = reinterpret_cast<const char*>(s_rec) + jw[jj];
                    const float4 r0 = *reinterpret_cast<const float4*>(rp);
                    const float4 m = *reinterpret_cast<const float4*>(rp + 16);
                    const int j = (int)(jw[jj] >> 5);
                    float dx, dy, u, w;
                    const float q = kWrap ? blend_q_wrap(fx, fy, make_float2(r0.x, r0.y), m, Wf, rw, dx, dy, u, w)
                                          : blend_q(fx, fy, make_float2(r0.x, r0.y), m, dx, dy, u, w);
                    const float2 o = make_float2(r0.z, r0.w);
                    const float a = fminf(kAlphaMax, blend_raw_alpha(q, o.x));
                    const float ae = (!done && q <= kQMax && a >= kAlphaMin) ? a : 0.0f;
                    const float Tn = T * (1.0f - ae);
                    const bool stop = Tn < kTMin;
                    C = stop ? C : fmaf(o.y * ae, T, C);
                    if (kAux) last = (!stop && ae > 0.0f) ? base + (uint32_t)j : last;
                    // without aux the final T is not kept: a stopped lane may
                    // take Tn (< the floor), it adds nothing afterwards either way
                    T = (kAux && stop) ? T : Tn;
                    done = done || stop;
                }
            }
        } else {
            for (int j0 = 0; j0 < cnt; j0 += kUnroll) {
                if (__all(done)) break;
#pragma unroll
                for (int jj = 0; jj < kUnroll; ++jj) {
                    const int j = j0 + jj;
                    const float4 r0 = s_rec[2 * j];
                    float dx, dy, u, w;
                    const float q = kWrap ? blend_q_wrap(fx, fy, make_float2(r0.x, r0.y), s_rec[2 * j + 1], Wf, rw,
                                                         dx, dy, u, w)
                                          : blend_q(fx, fy, make_float2(r0.x, r0.y), s_rec[2 * j + 1], dx, dy, u, w);
                    if (kCount) evals += (!done && j < cnt && q <= kQMax) ? 1u : 0u;
                    const float2 o = make_float2(r0.z, r0.w);
                    const float a = fminf(kAlphaMax, blend_raw_alpha(q, o.x));
                    // a skipped entry (cutoff, alpha floor, or a finished pixel) acts
                    // with alpha 0: T * (1 - 0) and C + 0 * T are exact no-ops
                    const float ae = (!done && q <= kQMax && a >= kAlphaMin) ? a : 0.0f;
                    const float Tn = T * (1.0f - ae);
                    const bool stop = Tn < kTMin;  // only reachable through ae > 0
                    C = stop ? C : fmaf(o.y * ae, T, C);
                    if (kAux) last = (!stop && ae > 0.0f) ? base + (uint32_t)j : last;
                    T = stop ? T : Tn;
                    done = done || stop;
                }
            }
        }
    }
    if (kVisit) {
        __shared__ unsigned long long s_vi;
        if (threadIdx.x == 0) s_vi = 0;
        __syncthreads();
        atomicAdd(&s_vi, (unsigned long long)visits);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&work[2], s_vi);
        return;
    }
    if (kCount) {
        __shared__ unsigned long long s_ev;
        if (threadIdx.x == 0) s_ev = 0;
        __syncthreads();
        atomicAdd(&s_ev, (unsigned long long)evals);
        __syncthreads();
        if (threadIdx.x == 0) {
            atomicAdd(&work[0], s_ev);
            atomicAdd(&work[1], (unsigned long long)staged);
        }
        return;
    }
    if (inside) {
        const size_t pix = (size_t)b * H * W + (size_t)py * W + px;
        out[pix] = C;
        if (kAux) {
            aux_T[pix] = T;
            aux_last[pix] = last;
        }
    }
}

template <int TILE, bool kCount, bool kAux, bool kVisit = false>
void blend_launch(const uint2* ranges, const uint32_t* vals, const Records& r, unsigned blocks, const Grid& g,
                  float* out, float* aux_T, uint32_t* aux_last, unsigned long long* work, hipStream_t st) {
    if (g.wrap)
        blend_forward_kernel<TILE, kCount, kAux, true, false, kVisit><<<blocks, TILE * TILE, 0, st>>>(
            ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles, out, aux_T, aux_last, work);
    else
        blend_forward_kernel<TILE, kCount, kAux, false, false, kVisit><<<blocks, TILE * TILE, 0, st>>>(
            ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles, out, aux_T, aux_last, work);
}

}  // namespace

void launch_mix_blend(const MixBatch& m, int tile_cap, const uint2* ranges, const uint32_t* vals, const Records& r,
                      float* out, hipStream_t st) {
    if (tile_cap <= 0) return;
    blend_forward_kernel<16, false, false, false, true><<<(unsigned)tile_cap, 256, 0, st>>>(
        ranges, vals, r.geo, r.wm, r.oa, 0, 0, 0, 0, out, nullptr, nullptr, nullptr, m);
}

void launch_blend_work(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                       unsigned long long* work, hipStream_t st) {
    const unsigned blocks = (unsigned)(B * g.tiles);
    if (!blocks) return;
    if (g.tile == 8) {
        blend_launch<8, true, true>(ranges, vals, r, blocks, g, nullptr, nullptr, nullptr, work, st);
    } else {
        blend_launch<16, true, true>(ranges, vals, r, blocks, g, nullptr, nullptr, nullptr, work, st);
        // the walk the spectrum render executes (without the blend state, as a plain render)
        blend_launch<16, false, false, true>(ranges, vals, r, blocks, g, nullptr, nullptr, nullptr, work, st);
    }
}

void launch_blend_forward(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                          float* out, float* aux_T, uint32_t* aux_last, hipStream_t st) {
    const unsigned blocks = (unsigned)(B * g.tiles);
    if (!blocks) return;
    const bool aux = aux_T != nullptr;
    if (g.tile == 8) {
        if (aux)
            blend_launch<8, false, true>(ranges, vals, r, blocks, g, out, aux_T, aux_last, nullptr, st);
        else
            blend_launch<8, false, false>(ranges, vals, r, blocks, g, out, nullptr, nullptr, nullptr, st);
    } else {
        if (aux)
            blend_launch<16, false, true>(ranges, vals, r, blocks, g, out, aux_T, aux_last, nullptr, st);
        else
            blend_launch<16, false, false>(ranges, vals, r, blocks, g, out, nullptr, nullptr, nullptr, st);
    }
}

}  // namespace swf
