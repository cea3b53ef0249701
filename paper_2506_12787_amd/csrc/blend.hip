// Per-tile front-to-back blending (Sec. 3.2 blending rule applied to the 2D
// Gaussian kernel of Sec. 4.1, one workgroup per (query, tile)).
//
// Each workgroup owns one TILE x TILE pixel tile, one pixel per thread. It walks
// the tile's depth-ordered list in batches of TILE*TILE records: every thread
// stages one record into LDS (mean re-expressed relative to the enclosing
// 64-pixel block, in full precision from the hi + lo pair), then every thread composites its
// pixel over the batch. A block-wide vote ends the walk once every pixel has
// reached the transmittance floor.
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

// kCount: instead of writing the spectrum, add to work[0] the number of (pixel,
// list entry) evaluations (every entry a pixel examines up to and including the
// one that ends it) and to work[1] the number of records staged in LDS.
template <int TILE, bool kCount = false>
__global__ __launch_bounds__(TILE* TILE) void blend_forward_kernel(const uint2* __restrict__ ranges,
                                                                    const uint32_t* __restrict__ vals,
                                                                    const float4* __restrict__ geo,
                                                                    const float4* __restrict__ wm,
                                                                    const float2* __restrict__ oa, int H, int W,
                                                                    int TW, int tiles, float* __restrict__ out,
                                                                    float* __restrict__ aux_T,
                                                                    uint32_t* __restrict__ aux_last,
                                                                    unsigned long long* __restrict__ work = nullptr) {
    constexpr int kN = TILE * TILE;
    constexpr int kUnroll = 8;  // entries per unrolled group (kN is a multiple)
    __shared__ float2 s_pos[kN];
    __shared__ float4 s_wm[kN];
    __shared__ float2 s_oa[kN];

    const int gtile = blockIdx.x;
    const int b = gtile / tiles;
    const int t = gtile - b * tiles;
    const int tx = t % TW, ty = t / TW;
    const int lx = threadIdx.x % TILE, ly = threadIdx.x / TILE;
    const int px = tx * TILE + lx, py = ty * TILE + ly;
    const bool inside = px < W && py < H;
    // Offsets are taken relative to the enclosing 64-pixel block, the same for
    // every tile size <= 64, so the arithmetic does not depend on the tiling.
    const int bx0 = (tx * TILE) & ~63, by0 = (ty * TILE) & ~63;
    const float x0 = (float)bx0, y0 = (float)by0;
    const float fx = (float)(px - bx0), fy = (float)(py - by0);

    const uint2 rg = ranges[gtile];
    float T = 1.0f, C = 0.0f;
    uint32_t last = 0;
    bool done = !inside;
    uint32_t evals = 0, staged = 0;

    for (uint32_t start = rg.x; start < rg.y; start += kN) {
        if (__syncthreads_count(done) == kN) break;
        const uint32_t i = start + threadIdx.x;
        const int cnt = (int)min((uint32_t)kN, rg.y - start);
        if (i < rg.y) {
            const uint32_t v = vals[i];
            const float4 g = geo[v];
            s_pos[threadIdx.x] = make_float2((g.x - x0) + g.z, (g.y - y0) + g.w);
            s_wm[threadIdx.x] = wm[v];
            s_oa[threadIdx.x] = oa[v];
        } else if ((int)threadIdx.x < ((cnt + kUnroll - 1) & ~(kUnroll - 1))) {
            // padding up to the unrolled length: opacity 0 never contributes
            s_pos[threadIdx.x] = make_float2(0.0f, 0.0f);
            s_wm[threadIdx.x] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            s_oa[threadIdx.x] = make_float2(0.0f, 0.0f);
        }
        __syncthreads();
        if (kCount) staged += (uint32_t)cnt;
        const uint32_t base = start - rg.x + 1u;  // 1-based list position of entry 0 of the batch
        // Branch-free walk: every lane evaluates every entry and commits it only
        // if it passes the cutoff, the alpha skip and the termination test. The
        // committed arithmetic is exactly the rule's; what is skipped is the
        // per-entry divergent control flow (scalar exec-mask work that would
        // otherwise outweigh the vector work). A wave leaves the batch once all
        // its pixels are done.
        for (int j0 = 0; j0 < cnt; j0 += kUnroll) {
            if (__all(done)) break;
#pragma unroll
            for (int jj = 0; jj < kUnroll; ++jj) {
                const int j = j0 + jj;
                float dx, dy, u, w;
                const float q = blend_q(fx, fy, s_pos[j], s_wm[j], dx, dy, u, w);
                const float2 o = s_oa[j];
                const float a = fminf(kAlphaMax, blend_raw_alpha(q, o.x));
                const bool use = !done && q <= kQMax && a >= kAlphaMin;
                const float Tn = T * (1.0f - a);
                const bool stop = use && Tn < kTMin;
                const bool take = use && !stop;
                if (kCount) evals += (!done && j < cnt) ? 1u : 0u;
                C = take ? fmaf(o.y * a, T, C) : C;
                T = take ? Tn : T;
                last = take ? base + (uint32_t)j : last;
                done = done || stop;
            }
        }
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
        if (aux_T) {
            aux_T[pix] = T;
            aux_last[pix] = last;
        }
    }
}

}  // namespace

void launch_blend_work(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                       unsigned long long* work, hipStream_t st) {
    const unsigned blocks = (unsigned)(B * g.tiles);
    if (!blocks) return;
    if (g.tile == 8)
        blend_forward_kernel<8, true><<<blocks, 64, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW,
                                                             g.tiles, nullptr, nullptr, nullptr, work);
    else
        blend_forward_kernel<16, true><<<blocks, 256, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW,
                                                               g.tiles, nullptr, nullptr, nullptr, work);
}

void launch_blend_forward(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                          float* out, float* aux_T, uint32_t* aux_last, hipStream_t st) {
    const unsigned blocks = (unsigned)(B * g.tiles);
    if (!blocks) return;
    if (g.tile == 8)
        blend_forward_kernel<8><<<blocks, 64, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles, out,
                                                       aux_T, aux_last);
    else
        blend_forward_kernel<16><<<blocks, 256, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles,
                                                         out, aux_T, aux_last);
}

}  // namespace swf
