// Backward pass of the render path: blend -> preprocess -> deformation MLP.
//
// Blend backward (Sec. 3.2 blending rule, differentiated): per (query, tile)
// workgroup, each pixel replays its transmittance back to front from the
// stored final T and last-contributor index, T_before = T_after / (1 - alpha)
// (alpha <= 0.99 so the divisor is >= 0.01), and accumulates
//   dC/damp_i   = alpha_i T_i
//   dC/dalpha_i = amp_i T_i - S_i / (1 - alpha_i),  S_i = sum_{j>i} amp_j alpha_j T_j
// through alpha = min(0.99, o exp(-q/2)) (zero derivative when clamped),
// q = |M d|^2, into per-pair gradients of (mean, M, opacity, amplitude).
// Per entry the 64 lanes of a wave are reduced before one atomic per value.
// With 16x16 tiles a wave skips the entries that miss the cutoff on all of its
// pixels.
//
// Preprocess backward maps d(M, opacity) to the 7 residual coordinates
// (d_mean, d_log_scale, d_rotation, d_logit, d_amp); the MLP backward is a
// chain of row-parallel products (dZ_{l-1} = (dZ_l W_l) . [H_{l-1} > 0]) and
// split-K weight-gradient reductions (dW_l = dZ_l^T H_{l-1}) in FP32.
#include "cull.h"
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

__device__ __forceinline__ unsigned lane_id() { return threadIdx.x & 63u; }

// Wave sums of 8 values at once: three halving exchanges leave each lane one
// value summed over 8 lanes, three more finish the sum over the wave (10
// shuffles instead of 48). Lane l < 8 returns the total of value index
// 4 (l & 1) + 2 ((l >> 1) & 1) + ((l >> 2) & 1).
__device__ __forceinline__ float wave_sum8(float (&a)[8]) {
    const unsigned l = lane_id();
    {
        const bool hi = l & 1u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float send = hi ? a[k] : a[k + 4], keep = hi ? a[k + 4] : a[k];
            a[k] = keep + __shfl_xor(send, 1, 64);
        }
    }
    {
        const bool hi = l & 2u;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float send = hi ? a[k] : a[k + 2], keep = hi ? a[k + 2] : a[k];
            a[k] = keep + __shfl_xor(send, 2, 64);
        }
    }
    {
        const bool hi = l & 4u;
        const float send = hi ? a[0] : a[1], keep = hi ? a[1] : a[0];
        a[0] = keep + __shfl_xor(send, 4, 64);
    }
    float v = a[0];
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// With 16x16 tiles each wave (an 8x8 quadrant) walks only the entries that can
// reach the cutoff on its rectangle (the forward kernel's culling): the others
// leave every one of its pixels unchanged.
// kWrap: periodic azimuth, as in the forward kernel (same staged image, same
// displacement, same culling exemption), so that every decision replays exactly.
// kDet: instead of adding into dpair, each wave writes its 8 sums of an entry
// to part[slot * 32 + wave * 8 + k] (zeroed beforehand), slot = the pair's
// first slot (det_off: the exclusive scan of the key counts) + the tile's
// row-major index in the pair's rectangle; det_reduce_kernel then sums each
// pair's slots in that order.
template <int TILE, bool kWrap = false, bool kDet = false>
__global__ __launch_bounds__(TILE* TILE) void blend_backward_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals, const float4* __restrict__ geo,
    const float4* __restrict__ wm, const float2* __restrict__ oa, int H, int W, int TW, int tiles,
    const float* __restrict__ grad_out, const float* __restrict__ aux_T, const uint32_t* __restrict__ aux_last,
    float* __restrict__ dpair, const uint2* __restrict__ rect = nullptr, const uint32_t* __restrict__ det_off = nullptr) {
    constexpr int kN = TILE * TILE;
    constexpr bool kCull = TILE == 16;
    constexpr int kWaves = kN / 64;
    __shared__ float2 s_pos[kN];
    __shared__ float4 s_wm[kN];
    __shared__ float2 s_oa[kN];
    __shared__ uint32_t s_v[kN];
    __shared__ uint32_t s_slot[kDet ? kN : 1];
    __shared__ uint8_t s_strip[kCull ? kN : 1];
    __shared__ uint16_t s_idx[kCull ? kWaves : 1][kN];
    __shared__ uint32_t s_max;

    const int gtile = blockIdx.x;
    const int b = gtile / tiles;
    const int t = gtile - b * tiles;
    const int tx = t % TW, ty = t / TW;
    // culled 16x16 tiles: wave w covers the 8x8 quadrant (w & 1, w >> 1)
    const int wq = (int)(threadIdx.x >> 6), lq = (int)(threadIdx.x & 63);
    const int lx = kCull ? (wq & 1) * 8 + (lq & 7) : (int)threadIdx.x % TILE;
    const int ly = kCull ? (wq >> 1) * 8 + (lq >> 3) : (int)threadIdx.x / TILE;
    const int px = tx * TILE + lx, py = ty * TILE + ly;
    const bool inside = px < W && py < H;
    const int bx0 = (tx * TILE) & ~63, by0 = (ty * TILE) & ~63;
    const float x0 = (float)bx0, y0 = (float)by0;
    const float fx = (float)(px - bx0), fy = (float)(py - by0);
    const float Wf = kWrap ? (float)W : 0.0f, rw = kWrap ? 1.0f / (float)W : 0.0f;
    const float cx = (float)(tx * TILE - bx0) + 0.5f * (float)(TILE - 1);
    const uint2 rg = ranges[gtile];

    float T = 1.0f, G = 0.0f;
    uint32_t last = 0;
    if (inside) {
        const size_t pix = (size_t)b * H * W + (size_t)py * W + px;
        G = grad_out[pix];
        if (G != 0.0f) {
            T = aux_T[pix];
            last = aux_last[pix];
        }
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (last) atomicMax(&s_max, last);
    __syncthreads();
    // never past the tile's list, even for an aux that does not belong to these lists
    const int lmax = (int)min(s_max, rg.y - rg.x);
    float S = 0.0f;

    auto entry = [&](int beg, int jj) {
        const int j = beg + jj;
        float gv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        bool contrib = false;
        if (j < (int)last) {
            const float4 m = s_wm[jj];
            float dx, dy, u, w;
            const float q = kWrap ? blend_q_wrap(fx, fy, s_pos[jj], m, Wf, rw, dx, dy, u, w)
                                  : blend_q(fx, fy, s_pos[jj], m, dx, dy, u, w);
            if (q <= kQMax) {
                const float2 o = s_oa[jj];
                const float raw = blend_raw_alpha(q, o.x);
                const float a = fminf(kAlphaMax, raw);
                if (a >= kAlphaMin) {
                    contrib = true;
                    const float om = 1.0f - a;
                    const float Tb = T / om;
                    const float dC_da = o.y * Tb - S / om;
                    S = fmaf(o.y * a, Tb, S);
                    T = Tb;
                    gv[7] = G * a * Tb;
                    if (!(raw > kAlphaMax)) {
                        const float ga = G * dC_da;
                        gv[6] = ga * (raw / o.x);           // d alpha / d opacity = exp(-q/2)
                        const float dq = ga * (-0.5f * a);  // d alpha / d q = -alpha / 2
                        const float du = 2.0f * dq * u, dw = 2.0f * dq * w;
                        gv[2] = du * dx;
                        gv[3] = du * dy;
                        gv[4] = dw * dx;
                        gv[5] = dw * dy;
                        gv[0] = -(du * m.x + dw * m.z);
                        gv[1] = -(du * m.y + dw * m.w);
                    }
                }
            }
        }
        if (__ballot(contrib) == 0ull) return;
        const float v = wave_sum8(gv);
        const unsigned l = lane_id();
        if (l < 8u && v != 0.0f) {
            const int k = 4 * (int)(l & 1u) + 2 * (int)((l >> 1) & 1u) + (int)((l >> 2) & 1u);
            if constexpr (kDet)
                dpair[(size_t)s_slot[jj] * 32 + (size_t)wq * 8 + k] = v;
            else
                atomicAdd(dpair + (size_t)s_v[jj] * 8 + k, v);
        }
    };

    for (int end = lmax; end > 0; end -= kN) {
        const int beg = end > kN ? end - kN : 0;
        __syncthreads();
        {
            const int j = beg + (int)threadIdx.x;
            if (j < end) {
                const uint32_t v = vals[rg.x + j];
                const float4 g = geo[v];
                const float2 pos =
                    kWrap ? staged_mean(g, x0, y0, Wf, cx) : make_float2((g.x - x0) + g.z, (g.y - y0) + g.w);
                const float4 m = wm[v];
                s_pos[threadIdx.x] = pos;
                s_wm[threadIdx.x] = m;
                s_oa[threadIdx.x] = oa[v];
                s_v[threadIdx.x] = v;
                if constexpr (kDet) {  // this tile's slot of the pair: row-major in its (possibly wrapped) rectangle
                    const uint2 rr = rect[v];
                    const int rx0 = (int)(rr.x & 0xffff), rx1 = (int)(rr.x >> 16), ry0 = (int)(rr.y & 0xffff);
                    const int rw = rx1 >= rx0 ? rx1 - rx0 + 1 : TW - rx0 + rx1 + 1;
                    const int cx = tx >= rx0 ? tx - rx0 : tx - rx0 + TW;
                    s_slot[threadIdx.x] = det_off[v] + (uint32_t)((ty - ry0) * rw + cx);
                }
                if (kCull)
                    s_strip[threadIdx.x] =
                        (kWrap && fabsf(pos.x - cx) > 0.5f * Wf - (float)TILE)
                            ? (uint8_t)0xf
                            : (uint8_t)wave_quads_mask(m, pos, (float)(tx * TILE - bx0), (float)(ty * TILE - by0),
                                                       kQMax);
            }
        }
        __syncthreads();
        const int cnt = end - beg;
        if (kCull) {
            const int wv = threadIdx.x >> 6;
            uint16_t* idx = s_idx[wv];
            int nlist = 0;
#pragma unroll
            for (int c = 0; c < kWaves; ++c) {
                const int jl = c * 64 + (int)lane_id();
                const bool f = jl < cnt && ((s_strip[jl] >> wv) & 1u);
                const uint64_t bal = __ballot(f);
                if (f) idx[nlist + __popcll(bal & ((1ull << lane_id()) - 1ull))] = (uint16_t)jl;
                nlist += __popcll(bal);
            }
            __builtin_amdgcn_wave_barrier();
            for (int n = nlist - 1; n >= 0; --n) entry(beg, (int)idx[n]);
        } else {
            for (int jj = cnt - 1; jj >= 0; --jj) entry(beg, jj);
        }
    }
}

// Deterministic gradient sums: pair i (query b = i / N) adds, for every tile
// of its rectangle in row-major order (a wrapped rectangle's columns from tx0
// on), the four waves' sums of its entry in that tile's list, found by binary
// search (a list holds its pairs in increasing order).
__global__ void det_reduce_kernel(const uint32_t* __restrict__ count, const uint32_t* __restrict__ det_off,
                                  const float* __restrict__ part, int64_t P, float* __restrict__ dpair) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const uint32_t c = count[i];
    const float4* e = reinterpret_cast<const float4*>(part + (size_t)(c ? det_off[i] : 0u) * 32);
    for (uint32_t k = 0; k < c; ++k)  // the pair's tiles in row-major order, then the 4 waves of each
#pragma unroll
        for (int wv = 0; wv < 4; ++wv) {
            const float4 a = e[(size_t)k * 8 + 2 * wv], b = e[(size_t)k * 8 + 2 * wv + 1];
            acc[0] += a.x;
            acc[1] += a.y;
            acc[2] += a.z;
            acc[3] += a.w;
            acc[4] += b.x;
            acc[5] += b.y;
            acc[6] += b.z;
            acc[7] += b.w;
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) dpair[i * 8 + k] = acc[k];
}

// d(mean, M, opacity, amp) -> d(residual coordinates); the unmasked result
// feeds the base parameters, the masked one (paper mode zeroes 2..4) the MLP.
__global__ void preprocess_backward_kernel(const float* __restrict__ dpair, const float4* __restrict__ wm,
                                           const float2* __restrict__ oa, const uint32_t* __restrict__ count,
                                           int64_t P, int paper_mask, float* __restrict__ dbase,
                                           float* __restrict__ dy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    float r[kOut] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (count[i]) {
        const float* g = dpair + i * 8;
        const float4 m = wm[i];
        const float op = oa[i].x;
        r[0] = g[0];
        r[1] = g[1];
        r[2] = -(g[2] * m.x + g[3] * m.y);
        r[3] = -(g[4] * m.z + g[5] * m.w);
        r[4] = -g[2] * m.y + g[3] * m.x - g[4] * m.w + g[5] * m.z;
        r[5] = g[6] * op * (1.0f - op);
        r[6] = g[7];
    }
#pragma unroll
    for (int k = 0; k < kOut; ++k) dbase[i * kOut + k] = r[k];
    if (dy) {
#pragma unroll
        for (int k = 0; k < kOut; ++k) dy[i * kOut + k] = (paper_mask && k >= 2 && k <= 4) ? 0.f : r[k];
    }
}

// Base-parameter gradients: sum over the batch, scatter to original ids.
__global__ void base_reduce_kernel(const float* __restrict__ dbase, const float* __restrict__ dmu_pe,
                                   const uint32_t* __restrict__ perm, int B, int N, BaseGrads out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    float s[kOut] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < B; ++b) {
        const float* r = dbase + ((size_t)b * N + p) * kOut;
#pragma unroll
        for (int k = 0; k < kOut; ++k) s[k] += r[k];
    }
    if (dmu_pe) {
        s[0] += dmu_pe[(size_t)p * 2];
        s[1] += dmu_pe[(size_t)p * 2 + 1];
    }
    const uint32_t id = perm[p];
#pragma unroll
    for (int k = 0; k < kOut; ++k)
        if (out.p[k]) out.p[k][id] = s[k];
}

// Column sums of row-major [rows x cols] matrices (one per z, batch stride
// bs), in two stages: part[z][y][c] over row block y, then out[z][c].
__global__ __launch_bounds__(256) void colsum_stage1_kernel(const float* __restrict__ A, int64_t rows, int64_t cols,
                                                            int64_t rpb, int64_t bs, float* __restrict__ part) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    const float* Az = A + (int64_t)blockIdx.z * bs;
    const int64_t r0 = (int64_t)blockIdx.y * rpb, r1 = min(rows, r0 + rpb);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int64_t r = r0;
    for (; r + 4 <= r1; r += 4) {
        s0 += Az[r * cols + c];
        s1 += Az[(r + 1) * cols + c];
        s2 += Az[(r + 2) * cols + c];
        s3 += Az[(r + 3) * cols + c];
    }
    for (; r < r1; ++r) s0 += Az[r * cols + c];
    part[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * cols + c] = (s0 + s1) + (s2 + s3);
}

// Column sums, vectorised (cols % 4 == 0): 4 consecutive columns per thread,
// 64 threads over 256 columns, 4 row groups per block summed through LDS in a
// fixed order (deterministic). One row block writes the result directly.
__device__ __forceinline__ float4 load4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ float4 load4(const __bf16* p) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                       __uint_as_float(u.y & 0xffff0000u));
}

template <typename T>
__global__ __launch_bounds__(256) void colsum4_stage1_kernel(const T* __restrict__ A, int64_t rows, int64_t cols,
                                                             int64_t rpb, int64_t bs, float* __restrict__ part,
                                                             float* __restrict__ out, int64_t out_bs) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 256 + tx * 4;
    const T* Az = A + (int64_t)blockIdx.z * bs;
    const int64_t r0 = (int64_t)blockIdx.y * rpb, r1 = min(rows, r0 + rpb);
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c < cols) {
#pragma unroll 4
        for (int64_t r = r0 + ty; r < r1; r += 4) {
            const float4 v = load4(Az + r * cols + c);
            s.x += v.x;
            s.y += v.y;
            s.z += v.z;
            s.w += v.w;
        }
    }
    __shared__ float4 red[4][64];
    red[ty][tx] = s;
    __syncthreads();
    if (ty != 0 || c >= cols) return;
    float4 t = red[0][tx];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        const float4 u = red[k][tx];
        t.x += u.x;
        t.y += u.y;
        t.z += u.z;
        t.w += u.w;
    }
    if (gridDim.y == 1) {
        float* o = out + (int64_t)blockIdx.z * out_bs + c;
        o[0] = t.x;
        o[1] = t.y;
        o[2] = t.z;
        o[3] = t.w;
    } else {
        *reinterpret_cast<float4*>(part + ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * cols + c) = t;
    }
}

// Second stage: 8 columns per block, 32 groups of row blocks each, summed
// through LDS in a fixed order.
__global__ __launch_bounds__(256) void colsum8_stage2_kernel(const float* __restrict__ part, int nblk, int64_t cols,
                                                             float* __restrict__ out, int64_t out_bs) {
    const int cc = threadIdx.x & 7, g = threadIdx.x >> 3;
    const int64_t c = (int64_t)blockIdx.x * 8 + cc;
    const float* pz = part + (int64_t)blockIdx.y * nblk * cols;
    float s = 0.f;
    if (c < cols)
        for (int b = g; b < nblk; b += 32) s += pz[(int64_t)b * cols + c];
    __shared__ float red[32][8];
    red[g][cc] = s;
    __syncthreads();
    if (g != 0 || c >= cols) return;
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < 32; ++k) t += red[k][cc];
    out[(int64_t)blockIdx.y * out_bs + c] = t;
}

__global__ void fill_kernel(float* __restrict__ p, float v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// d mu0 per Gaussian from dg = d gamma(mu_hat) (26 per Gaussian, already
// summed over the batch): the chain rule through the sin / cos features.
__global__ void pe_chain_kernel(const float* __restrict__ dgm, const float* __restrict__ mx,
                                const float* __restrict__ my, int N, int Wd, int Hd, float* __restrict__ dmu) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const float* dg = dgm + (size_t)p * kMeanFeat;
    float hx, lx, hy, ly;
    div_two(mx[p], (float)Wd, hx, lx);
    div_two(my[p], (float)Hd, hy, ly);
    float gx = dg[0], gy = dg[1];
#pragma unroll
    for (int k = 0; k < kMeanBands; ++k) {
        float sx, cx, sy, cy;
        sincospi_scaled(hx, lx, k, sx, cx);
        sincospi_scaled(hy, ly, k, sy, cy);
        const float f = 3.14159265358979323846f * (float)(1 << k);
        gx += f * (dg[2 + 2 * k] * cx - dg[2 + 2 * kMeanBands + 2 * k] * sx);
        gy += f * (dg[3 + 2 * k] * cy - dg[3 + 2 * kMeanBands + 2 * k] * sy);
    }
    dmu[(size_t)p * 2] = gx / (float)Wd;
    dmu[(size_t)p * 2 + 1] = gy / (float)Hd;
}

// ---- BF16 variants (the MLP backward of a BF16 forward) ----------------------
__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }  // round to nearest even

// Input gradient of a 256 x 256 layer on BF16 MFMA (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation): out[p][i] = sum_o dz[p][o] W[o][i] for every pair p, W
// row-major [o][i] (the layer's [out][in] weights). kF32: FP32 result (the
// layer-1 gradient, masked later inside its sums). Otherwise the result is
// rounded to BF16 and zeroed where act[p][i] (the BF16 activation) is not > 0,
// the previous layer's ReLU: one pass instead of a library GEMM and a masking
// pass. The whole W sits in LDS in MFMA A-fragment order (fragment (t, c), lane
// 16 g + r, element j = W[32 c + 8 g + j][16 t + r]). Each wave takes groups of
// kDzPairs pairs: their dz rows are the B operands, in registers (16 bytes per
// lane per 32-wide k chunk), the ReLU masks a per-wave bitmap in LDS; the next
// group's rows and activations are loaded while the current one is computed,
// and 16 x 16 output tiles are written as they finish.
constexpr int kDzWaves = 8;
constexpr int kDzNcb = 2;
constexpr int kDzPairs = 16 * kDzNcb;

typedef __bf16 dz_bf16x8 __attribute__((ext_vector_type(8)));
typedef float dz_f32x4 __attribute__((ext_vector_type(4)));
typedef float dz_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 dz_bf16x2 __attribute__((ext_vector_type(2)));

template <bool kF32>
__global__ __launch_bounds__(64 * kDzWaves) void dz_gemm_kernel(const __bf16* __restrict__ dz,
                                                                const __bf16* __restrict__ W,
                                                                const __bf16* __restrict__ act, int64_t P,
                                                                void* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) uint4 s_a[16 * 8 * 64];  // 128 fragments of 1 KiB
    __shared__ uint8_t s_m[kF32 ? 1 : kDzWaves][kDzPairs][32];        // ReLU mask bits, pair-major
    const uint16_t* Wb = reinterpret_cast<const uint16_t*>(W);
    for (int e = threadIdx.x; e < 16 * 8 * 64; e += 64 * kDzWaves) {
        const int f = e >> 6, l = e & 63, t = f >> 3, c = f & 7, g = l >> 4, r = l & 15;
        const uint16_t* col = Wb + (size_t)(32 * c + 8 * g) * 256 + 16 * t + r;
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (uint32_t)col[(2 * q) * 256] | ((uint32_t)col[(2 * q + 1) * 256] << 16);
        s_a[e] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    __syncthreads();
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63), g = lane >> 4, n = lane & 15;
    const int64_t groups = (P + kDzPairs - 1) / kDzPairs;
    const int64_t stride = (int64_t)gridDim.x * kDzWaves;
    // rows (B layout: pair cb*16 + n, k = 32 c + 8 g + j) of group q; zero past P
    auto load_rows = [&](const __bf16* src, int64_t q, dz_bf16x8 (&dst)[8][kDzNcb]) {
#pragma unroll
        for (int cb = 0; cb < kDzNcb; ++cb) {
            const int64_t p = q * kDzPairs + cb * 16 + n;
#pragma unroll
            for (int c = 0; c < 8; ++c)
                dst[c][cb] = (q < groups && p < P) ? *reinterpret_cast<const dz_bf16x8*>(src + p * 256 + 32 * c + 8 * g)
                                                   : dz_bf16x8{};
        }
    };
    // mask byte of 8 activations (bit j set where element j is > 0)
    auto mask_byte = [](dz_bf16x8 v) {
        const uint4 u = __builtin_bit_cast(uint4, v);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            m |= (((w[k] & 0x8000u) == 0 && (w[k] & 0x7fffu) != 0) ? 1u : 0u) << (2 * k);
            m |= (((w[k] & 0x80000000u) == 0 && (w[k] & 0x7fff0000u) != 0) ? 1u : 0u) << (2 * k + 1);
        }
        return (uint8_t)m;
    };
    auto store_masks = [&](dz_bf16x8 (&a)[8][kDzNcb]) {
#pragma unroll
        for (int cb = 0; cb < kDzNcb; ++cb)
#pragma unroll
            for (int c = 0; c < 8; ++c) s_m[kF32 ? 0 : wave][cb * 16 + n][4 * c + g] = mask_byte(a[c][cb]);
        __builtin_amdgcn_wave_barrier();
    };
    int64_t grp = (int64_t)blockIdx.x * kDzWaves + wave;
    dz_bf16x8 b[8][kDzNcb], bn[8][kDzNcb], an[8][kDzNcb];
    load_rows(dz, grp, b);
    if (!kF32) {
        load_rows(act, grp, an);
        store_masks(an);
    }
    for (; grp < groups; grp += stride) {
        const int64_t p0 = grp * kDzPairs;
        load_rows(dz, grp + stride, bn);  // the next group, while this one is computed
        if (!kF32) load_rows(act, grp + stride, an);
#pragma unroll 1
        for (int t = 0; t < 16; ++t) {
            dz_f32x4 acc[kDzNcb];
#pragma unroll
            for (int cb = 0; cb < kDzNcb; ++cb) acc[cb] = dz_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const dz_bf16x8 a = __builtin_bit_cast(dz_bf16x8, s_a[(t * 8 + c) * 64 + lane]);
#pragma unroll
                for (int cb = 0; cb < kDzNcb; ++cb)
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[c][cb], acc[cb], 0, 0, 0);
            }
#pragma unroll
            for (int cb = 0; cb < kDzNcb; ++cb) {
                const int64_t p = p0 + cb * 16 + n;
                if (p >= P) continue;
                if (kF32) {
                    *reinterpret_cast<float4*>(reinterpret_cast<float*>(out) + p * 256 + 16 * t + 4 * g) =
                        make_float4(acc[cb][0], acc[cb][1], acc[cb][2], acc[cb][3]);
                } else {
                    // features 16 t + 4 g + 0..3: bits 4 (g & 1) + 0..3 of mask byte 2 t + g / 2
                    const uint32_t nib = ((uint32_t)s_m[wave][cb * 16 + n][2 * t + (g >> 1)] >> (4 * (g & 1))) & 15u;
                    const dz_f32x2 lo2 = {acc[cb][0], acc[cb][1]}, hi2 = {acc[cb][2], acc[cb][3]};
                    uint32_t v0 = __builtin_bit_cast(uint32_t, __builtin_convertvector(lo2, dz_bf16x2));
                    uint32_t v1 = __builtin_bit_cast(uint32_t, __builtin_convertvector(hi2, dz_bf16x2));
                    v0 &= ((nib & 1u) ? 0x0000ffffu : 0u) | ((nib & 2u) ? 0xffff0000u : 0u);
                    v1 &= ((nib & 4u) ? 0x0000ffffu : 0u) | ((nib & 8u) ? 0xffff0000u : 0u);
                    *reinterpret_cast<uint2*>(reinterpret_cast<__bf16*>(out) + p * 256 + 16 * t + 4 * g) =
                        make_uint2(v0, v1);
                }
            }
        }
        if (!kF32) {
            __builtin_amdgcn_wave_barrier();  // this group's mask reads come before the next group's writes
            store_masks(an);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int cb = 0; cb < kDzNcb; ++cb) b[c][cb] = bn[c][cb];
    }
}

// Layer-1 gradient of a BF16 backward without storing it. For the block's
// Gaussians n0 .. n0 + kL1Rows - 1 and every query b in order: z[b][n] =
// dz1[b][n] W (FP32 accumulation on MFMA; dz1 [B][N][256] BF16, the gradient of
// the second layer's pre-activations; W its 256 x 256 BF16 weights, row-major
// [out][in]), masked by act[b][n] > 0 (the layer-1 ReLU), gives S[n][:] = the sum
// over b (complete, in order) and Rpart[block][b][:] = the sum over the block's
// Gaussians. Pairs are the MFMA rows here (A = a wave's 16 dz1 rows, B = W
// fragments from LDS, laid out as in dz_gemm_kernel), so a lane holds 4 pairs
// of one feature per output tile: S accumulates in registers and the R partial
// is a sum over those 4 and over the wave's 4 lane groups.
constexpr int kL1Waves = 8;
constexpr int kL1Rows = 16 * kL1Waves;

__global__ __launch_bounds__(64 * kL1Waves) void layer1_grad_kernel(const __bf16* __restrict__ dz1,
                                                                    const __bf16* __restrict__ W,
                                                                    const __bf16* __restrict__ act, int B, int N,
                                                                    float* __restrict__ S,
                                                                    float* __restrict__ Rpart) {
    __shared__ __attribute__((aligned(16))) uint4 s_a[16 * 8 * 64];
    __shared__ uint8_t s_m[kL1Waves][16][32];  // ReLU mask bits of the wave's 16 pairs, current query
    __shared__ float s_r[kL1Waves][256];        // per-wave R partial, current query
    const uint16_t* Wb = reinterpret_cast<const uint16_t*>(W);
    for (int e = threadIdx.x; e < 16 * 8 * 64; e += 64 * kL1Waves) {
        const int f = e >> 6, l = e & 63, t = f >> 3, c = f & 7, g = l >> 4, r = l & 15;
        const uint16_t* col = Wb + (size_t)(32 * c + 8 * g) * 256 + 16 * t + r;
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (uint32_t)col[(2 * q) * 256] | ((uint32_t)col[(2 * q + 1) * 256] << 16);
        s_a[e] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63), g = lane >> 4, r = lane & 15;
    const int nw = blockIdx.x * kL1Rows + wave * 16;  // the wave's first Gaussian
    const int na = nw + r;                            // this lane's A row
    // dz1 or act row of this lane's A row for query b (B layout of dz_gemm: k = 32 c + 8 g + j); zero past N
    auto load_rows = [&](const __bf16* src, int b, dz_bf16x8 (&dst)[8]) {
        const int64_t p = (int64_t)b * N + na;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            dst[c] = (b < B && na < N) ? *reinterpret_cast<const dz_bf16x8*>(src + p * 256 + 32 * c + 8 * g)
                                       : dz_bf16x8{};
    };
    auto store_masks = [&](const dz_bf16x8 (&a)[8]) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint4 u = __builtin_bit_cast(uint4, a[c]);
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
            uint32_t m = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                m |= (((w[k] & 0x8000u) == 0 && (w[k] & 0x7fffu) != 0) ? 1u : 0u) << (2 * k);
                m |= (((w[k] & 0x80000000u) == 0 && (w[k] & 0x7fff0000u) != 0) ? 1u : 0u) << (2 * k + 1);
            }
            s_m[wave][r][4 * c + g] = (uint8_t)m;
        }
        __builtin_amdgcn_wave_barrier();
    };
    dz_bf16x8 a_cur[8], a_nxt[8], m_nxt[8];
    load_rows(dz1, 0, a_cur);
    load_rows(act, 0, m_nxt);
    store_masks(m_nxt);
    __syncthreads();  // s_a complete
    dz_f32x4 sacc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) sacc[t] = dz_f32x4{0.f, 0.f, 0.f, 0.f};
    for (int b = 0; b < B; ++b) {
        load_rows(dz1, b + 1, a_nxt);  // the next query's rows while this one is computed
        load_rows(act, b + 1, m_nxt);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            dz_f32x4 acc = dz_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 8; ++c)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    a_cur[c], __builtin_bit_cast(dz_bf16x8, s_a[(t * 8 + c) * 64 + lane]), acc, 0, 0, 0);
            // lane (g, r) holds pairs 4 g + jj of feature 16 t + r: mask bit r % 8 of byte 2 t + r / 8
            float v = 0.f;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t bit = ((uint32_t)s_m[wave][4 * g + jj][2 * t + (r >> 3)] >> (r & 7)) & 1u;
                const float x = bit ? acc[jj] : 0.f;
                sacc[t][jj] += x;
                v += x;
            }
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (g == 0) s_r[wave][16 * t + r] = v;
        }
        __syncthreads();
        for (int k = threadIdx.x; k < 256; k += 64 * kL1Waves) {
            float v = 0.f;
#pragma unroll
            for (int w = 0; w < kL1Waves; ++w) v += s_r[w][k];
            Rpart[((size_t)blockIdx.x * B + b) * 256 + k] = v;
        }
        store_masks(m_nxt);  // this wave's reads of the query-b masks are complete
#pragma unroll
        for (int c = 0; c < 8; ++c) a_cur[c] = a_nxt[c];
        __syncthreads();  // s_r is rewritten for the next query
    }
#pragma unroll
    for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int n = nw + 4 * g + jj;
            if (n < N) S[(size_t)n * 256 + 16 * t + r] = sacc[t][jj];
        }
}

// Weight gradient of a 256 x 256 layer on BF16 MFMA over one slice of pairs:
// part[blk][o][i] = sum over the slice's pairs p of dz[p][o] act[p][i] (dz, act
// [P][256] BF16; FP32 accumulation); the caller adds the slices. The
// contraction runs over pairs, so both operands are staged through LDS
// transposed, feature-major, 32 pairs at a time (rows padded to 80 bytes: the
// 16-byte fragment reads of 16 consecutive features and the 2-byte staging
// writes of consecutive pairs fall in distinct banks). Wave w accumulates the
// 4 x 8 output tiles o in [64 (w % 4), +64), i in [128 (w / 4), +128) in
// registers; the next 32 pairs are loaded while the current ones are multiplied.
// With kBias the layer's bias gradient (the column sums of dz) comes along: waves
// 0..3 multiply their dz fragments by a fragment of ones as well and write
// part[nblk * 65536 + blk * 256 + o].
constexpr int kWgWaves = 8;
constexpr int kWgRow = 40;  // bf16 per staged feature row: 32 pairs + padding

template <bool kBias>
__global__ __launch_bounds__(64 * kWgWaves) void wgrad_mfma_kernel(const __bf16* __restrict__ dz,
                                                                   const __bf16* __restrict__ act, int64_t P,
                                                                   int64_t rpb, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t t_dz[256 * kWgRow];
    __shared__ __attribute__((aligned(16))) uint16_t t_act[256 * kWgRow];
    const int tid = (int)threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, n = lane & 15;
    const int o0 = 64 * (wave & 3), i0 = 128 * (wave >> 2);
    const int64_t beg = (int64_t)blockIdx.x * rpb, end = min(P, beg + rpb);
    // staging: thread -> pair q = tid % 32 of the chunk, 8-feature pieces c = tid / 32 and c + 16
    const int q = tid & 31, c0 = tid >> 5;
    uint4 rd[2], ra[2];
    auto load = [&](int64_t p0) {
        const int64_t p = p0 + q;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = c0 + 16 * h;
            rd[h] = p < end ? *reinterpret_cast<const uint4*>(dz + p * 256 + 8 * c) : make_uint4(0u, 0u, 0u, 0u);
            ra[h] = p < end ? *reinterpret_cast<const uint4*>(act + p * 256 + 8 * c) : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = c0 + 16 * h;
            const uint32_t wd[4] = {rd[h].x, rd[h].y, rd[h].z, rd[h].w};
            const uint32_t wa[4] = {ra[h].x, ra[h].y, ra[h].z, ra[h].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                t_dz[(8 * c + 2 * k) * kWgRow + q] = (uint16_t)(wd[k] & 0xffffu);
                t_dz[(8 * c + 2 * k + 1) * kWgRow + q] = (uint16_t)(wd[k] >> 16);
                t_act[(8 * c + 2 * k) * kWgRow + q] = (uint16_t)(wa[k] & 0xffffu);
                t_act[(8 * c + 2 * k + 1) * kWgRow + q] = (uint16_t)(wa[k] >> 16);
            }
        }
    };
    dz_f32x4 acc[4][8], accb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        accb[a] = dz_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = dz_f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const bool bias_wave = kBias && (wave >> 2) == 0;  // waves 0..3 cover the 16 o-tiles once
    const uint4 one4 = make_uint4(0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u);  // bf16 1.0 x 8
    const dz_bf16x8 ones = __builtin_bit_cast(dz_bf16x8, one4);
    if (beg < end) load(beg);
    for (int64_t p0 = beg; p0 < end; p0 += 32) {
        __syncthreads();  // the previous chunk's fragment reads are complete
        stage();
        __syncthreads();
        if (p0 + 32 < end) load(p0 + 32);
        dz_bf16x8 fa[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)  // A(o, k = pair): 8 consecutive pairs of feature o
            fa[a] = *reinterpret_cast<const dz_bf16x8*>(&t_dz[(o0 + 16 * a + n) * kWgRow + 8 * g]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const dz_bf16x8 fb = *reinterpret_cast<const dz_bf16x8*>(&t_act[(i0 + 16 * b + n) * kWgRow + 8 * g]);
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb, acc[a][b], 0, 0, 0);
        }
        if (bias_wave)
#pragma unroll
            for (int a = 0; a < 4; ++a) accb[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], ones, accb[a], 0, 0, 0);
    }
    if (bias_wave && n == 0) {  // every column of the ones product is the row sum
        float* ob = part + (size_t)gridDim.x * 65536 + (size_t)blockIdx.x * 256;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) ob[o0 + 16 * a + 4 * g + jj] = accb[a][jj];
    }
    // D(row 4 g + jj, col n) of tile (a, b) is dW[o0 + 16 a + 4 g + jj][i0 + 16 b + n]
    float* out = part + (size_t)blockIdx.x * 65536;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) out[(size_t)(o0 + 16 * a + 4 * g + jj) * 256 + i0 + 16 * b + n] = acc[a][b][jj];
}

// Output layer of a BF16 backward in one pass over the last hidden activations
// act [P][256] (BF16), per block of pairs (one slice of rpb pairs): with dy
// [P][7] FP32 (the upstream gradient as computed, not rounded) and Wo [7][256]
// BF16,
//   dz[p][f] = BF16(sum_o dy[p][o] Wo[o][f]), zero where act[p][f] is not > 0
//     (the gradient of the last hidden pre-activations; skipped if dz is NULL),
//   part[blk][o][f] = sum over the slice of dy[p][o] act[p][f] (the weight
//     gradient's partial; skipped if part is NULL; the caller adds the slices).
// Thread: 8 features (16-byte loads and stores) of every 8th pair of the slice.
__global__ __launch_bounds__(256) void out_bwd_bf16_kernel(const float* __restrict__ dy,
                                                           const __bf16* __restrict__ wo,
                                                           const __bf16* __restrict__ act, int64_t P, int64_t rpb,
                                                           __bf16* __restrict__ dz, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) float s_w[kOut][256];
    __shared__ float s_red[4][kOut][256];  // one row per wave after the in-wave pair of rows is added
    for (int i = threadIdx.x; i < kOut * 256; i += 256) s_w[i / 256][i % 256] = (float)wo[i];
    __syncthreads();
    const int f0 = (int)(threadIdx.x & 31) * 8, row = (int)(threadIdx.x >> 5);
    const int64_t beg = (int64_t)blockIdx.x * rpb, end = min(P, beg + rpb);
    float acc[kOut][8];
#pragma unroll
    for (int o = 0; o < kOut; ++o)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[o][j] = 0.f;
    for (int64_t p = beg + row; p < end; p += 8) {
        float y[kOut];
#pragma unroll
        for (int o = 0; o < kOut; ++o) y[o] = dy[p * kOut + o];
        const uint4 a = *reinterpret_cast<const uint4*>(act + p * 256 + f0);
        const uint32_t aw[4] = {a.x, a.y, a.z, a.w};
        float av[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            av[2 * k] = __uint_as_float(aw[k] << 16);
            av[2 * k + 1] = __uint_as_float(aw[k] & 0xffff0000u);
        }
        if (part) {
#pragma unroll
            for (int o = 0; o < kOut; ++o)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[o][j] = fmaf(y[o], av[j], acc[o][j]);
        }
        if (dz) {
            float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int o = 0; o < kOut; ++o) {
                const float4 w0 = *reinterpret_cast<const float4*>(&s_w[o][f0]);
                const float4 w1 = *reinterpret_cast<const float4*>(&s_w[o][f0 + 4]);
                z[0] = fmaf(y[o], w0.x, z[0]);
                z[1] = fmaf(y[o], w0.y, z[1]);
                z[2] = fmaf(y[o], w0.z, z[2]);
                z[3] = fmaf(y[o], w0.w, z[3]);
                z[4] = fmaf(y[o], w1.x, z[4]);
                z[5] = fmaf(y[o], w1.y, z[5]);
                z[6] = fmaf(y[o], w1.z, z[6]);
                z[7] = fmaf(y[o], w1.w, z[7]);
            }
            uint32_t ow[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t lo = __builtin_bit_cast(uint16_t, to_bf16(z[2 * k]));
                const uint32_t hi = __builtin_bit_cast(uint16_t, to_bf16(z[2 * k + 1]));
                const uint32_t x = aw[k];
                const uint32_t ml = ((x & 0x8000u) == 0 && (x & 0x7fffu) != 0) ? 0x0000ffffu : 0u;
                const uint32_t mh = ((x & 0x80000000u) == 0 && (x & 0x7fff0000u) != 0) ? 0xffff0000u : 0u;
                ow[k] = (lo | (hi << 16)) & (ml | mh);
            }
            *reinterpret_cast<uint4*>(dz + p * 256 + f0) = make_uint4(ow[0], ow[1], ow[2], ow[3]);
        }
    }
    if (!part) return;  // block-uniform
    // rows 2 w and 2 w + 1 are the two halves of wave w: add them across lanes l and l + 32
    const int wv = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int o = 0; o < kOut; ++o)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float v = acc[o][j] + __shfl_xor(acc[o][j], 32);
            if ((threadIdx.x & 32) == 0) s_red[wv][o][f0 + j] = v;
        }
    __syncthreads();
    for (int e = threadIdx.x; e < kOut * 256; e += 256) {
        const int o = e / 256, f = e % 256;
        part[(size_t)blockIdx.x * kOut * 256 + e] = s_red[0][o][f] + s_red[1][o][f] + s_red[2][o][f] + s_red[3][o][f];
    }
}

// Layer-1 gradient sums in one pass over the FP32 gradient z [B][N][256]:
// with dz = z * [act > 0] (kMask: the BF16 activations act [B][N][256] mask
// an unmasked z; else z is dz already), S[n][k] = sum_b dz[b][n][k]
// (complete: the block owns Gaussians n0 .. n0 + 31, summed over b in order)
// and Rpart[block][b][k] = sum over the block's Gaussians of dz[b][n][k]
// (4 row groups through LDS).
constexpr int kSumRows = 32;

template <bool kMask>
__global__ __launch_bounds__(256) void layer1_sums_kernel(const float* __restrict__ z, const __bf16* __restrict__ act,
                                                          int B, int N, float* __restrict__ S,
                                                          float* __restrict__ Rpart) {
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = tx * 4;
    const int n0 = blockIdx.x * kSumRows;
    float4 sacc[kSumRows / 4];
#pragma unroll
    for (int i = 0; i < kSumRows / 4; ++i) sacc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __shared__ float4 red[4][64];
    for (int b = 0; b < B; ++b) {
        float4 racc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int i = 0; i < kSumRows / 4; ++i) {
            const int n = n0 + ty + 4 * i;
            if (n < N) {
                const size_t off = ((size_t)b * N + n) * 256 + c;
                const float4 v = load4(z + off);
                float4 m = v;
                if constexpr (kMask) {
                    const float4 a = load4(act + off);
                    m = make_float4(a.x > 0.f ? v.x : 0.f, a.y > 0.f ? v.y : 0.f, a.z > 0.f ? v.z : 0.f,
                                    a.w > 0.f ? v.w : 0.f);
                }
                sacc[i].x += m.x;
                sacc[i].y += m.y;
                sacc[i].z += m.z;
                sacc[i].w += m.w;
                racc.x += m.x;
                racc.y += m.y;
                racc.z += m.z;
                racc.w += m.w;
            }
        }
        red[ty][tx] = racc;
        __syncthreads();
        if (ty == 0) {
            float4 t = red[0][tx];
#pragma unroll
            for (int k = 1; k < 4; ++k) {
                t.x += red[k][tx].x;
                t.y += red[k][tx].y;
                t.z += red[k][tx].z;
                t.w += red[k][tx].w;
            }
            *reinterpret_cast<float4*>(Rpart + ((size_t)blockIdx.x * B + b) * 256 + c) = t;
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < kSumRows / 4; ++i) {
        const int n = n0 + ty + 4 * i;
        if (n < N) *reinterpret_cast<float4*>(S + (size_t)n * 256 + c) = sacc[i];
    }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t n, __bf16* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = to_bf16(x[i]);
}

// Column sums of row-major BF16 matrices, first stage (FP32 partial sums).
__global__ __launch_bounds__(256) void colsum_stage1_bf16_kernel(const __bf16* __restrict__ A, int64_t rows,
                                                                 int64_t cols, int64_t rpb, int64_t bs,
                                                                 float* __restrict__ part) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    const __bf16* Az = A + (int64_t)blockIdx.z * bs;
    const int64_t r0 = (int64_t)blockIdx.y * rpb, r1 = min(rows, r0 + rpb);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int64_t r = r0;
    for (; r + 4 <= r1; r += 4) {
        s0 += (float)Az[r * cols + c];
        s1 += (float)Az[(r + 1) * cols + c];
        s2 += (float)Az[(r + 2) * cols + c];
        s3 += (float)Az[(r + 3) * cols + c];
    }
    for (; r < r1; ++r) s0 += (float)Az[r * cols + c];
    part[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * cols + c] = (s0 + s1) + (s2 + s3);
}

__global__ void mean_features_f32_kernel(const float* __restrict__ mx, const float* __restrict__ my, int n, int W,
                                         int H, float* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float f[kMeanFeat];
    mean_features(mx[p], my[p], W, H, f);
#pragma unroll
    for (int k = 0; k < kMeanFeat; ++k) out[(size_t)p * kMeanFeat + k] = f[k];
}


}  // namespace

void launch_blend_backward(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                           const float* grad_out, const float* aux_T, const uint32_t* aux_last, float* dpair,
                           hipStream_t st, float* det_part, int N, const uint32_t* det_off) {
    const unsigned blocks = (unsigned)(B * g.tiles);
    if (!blocks) return;
    float* dst = det_part ? det_part : dpair;
#define SWF_BLEND_BWD(TILE, WRAP, DET)                                                                         \
    blend_backward_kernel<TILE, WRAP, DET><<<blocks, TILE * TILE, 0, st>>>(                                    \
        ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles, grad_out, aux_T, aux_last, dst, r.rect, det_off)
#define SWF_BLEND_BWD_T(TILE, DET)   \
    do {                             \
        if (g.wrap)                  \
            SWF_BLEND_BWD(TILE, true, DET);  \
        else                         \
            SWF_BLEND_BWD(TILE, false, DET); \
    } while (0)
    if (det_part) {
        if (g.tile == 8)
            SWF_BLEND_BWD_T(8, true);
        else
            SWF_BLEND_BWD_T(16, true);
        const int64_t P = (int64_t)B * N;
        if (P > 0)
            det_reduce_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(r.count, det_off, det_part, P, dpair);
    } else {
        if (g.tile == 8)
            SWF_BLEND_BWD_T(8, false);
        else
            SWF_BLEND_BWD_T(16, false);
    }
#undef SWF_BLEND_BWD_T
#undef SWF_BLEND_BWD
}

void launch_preprocess_backward(const float* dpair, const Records& r, int64_t P, bool paper_mask, float* dbase,
                                float* dy, hipStream_t st) {
    if (P > 0)
        preprocess_backward_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(dpair, r.wm, r.oa, r.count, P,
                                                                                paper_mask ? 1 : 0, dbase, dy);
}

void launch_base_reduce(const float* dbase, const float* dmu_pe, const uint32_t* perm, int B, int N,
                        const BaseGrads& out, hipStream_t st) {
    if (N > 0) base_reduce_kernel<<<(N + 255) / 256, 256, 0, st>>>(dbase, dmu_pe, perm, B, N, out);
}

int colsum_blocks(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(2048, (rows + 255) / 256)); }

namespace {
template <typename T>
void colsum4(const T* A, int64_t rows, int64_t cols, int nz, int64_t bs, float* part, float* out, int64_t out_bs,
             hipStream_t st) {
    const int nblk = colsum_blocks(rows);
    const int64_t rpb = (rows + nblk - 1) / nblk;
    colsum4_stage1_kernel<T><<<dim3((unsigned)((cols + 255) / 256), nblk, nz), 256, 0, st>>>(A, rows, cols, rpb, bs,
                                                                                          part, out, out_bs);
    if (nblk > 1)
        colsum8_stage2_kernel<<<dim3((unsigned)((cols + 7) / 8), nz), 256, 0, st>>>(part, nblk, cols, out, out_bs);
}
}  // namespace

void launch_colsum(const float* A, int64_t rows, int64_t cols, int nz, int64_t bs, float* part, float* out,
                   int64_t out_bs, hipStream_t st) {
    if (cols <= 0 || nz <= 0) return;
    if (cols % 4 == 0 && bs % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0) {
        colsum4(A, rows, cols, nz, bs, part, out, out_bs, st);
        return;
    }
    const int nblk = colsum_blocks(rows);
    const int64_t rpb = (rows + nblk - 1) / nblk;
    const unsigned gx = (unsigned)((cols + 255) / 256);
    colsum_stage1_kernel<<<dim3(gx, nblk, nz), 256, 0, st>>>(A, rows, cols, rpb, bs, part);
    colsum8_stage2_kernel<<<dim3((unsigned)((cols + 7) / 8), nz), 256, 0, st>>>(part, nblk, cols, out, out_bs);
}

void launch_fill(float* p, float v, int64_t n, hipStream_t st) {
    if (n > 0) fill_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, v, n);
}

void launch_pe_chain(const float* dg, const DevScene& s, float* dmu, hipStream_t st) {
    if (s.n > 0) pe_chain_kernel<<<(s.n + 255) / 256, 256, 0, st>>>(dg, s.mx, s.my, s.n, s.W, s.H, dmu);
}

void launch_dz_gemm(const void* dz, const void* W, const void* act, int64_t P, void* out, bool f32_out,
                    hipStream_t st) {
    if (P <= 0) return;
    const int64_t groups = (P + kDzPairs - 1) / kDzPairs;
    const int blocks = (int)std::min<int64_t>(n_compute_units(), (groups + kDzWaves - 1) / kDzWaves);
    if (f32_out)
        dz_gemm_kernel<true><<<blocks, 64 * kDzWaves, 0, st>>>((const __bf16*)dz, (const __bf16*)W, nullptr, P, out);
    else
        dz_gemm_kernel<false><<<blocks, 64 * kDzWaves, 0, st>>>((const __bf16*)dz, (const __bf16*)W,
                                                                (const __bf16*)act, P, out);
}

int wgrad_out_blocks(int64_t P) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (P + 255) / 256)); }

void launch_out_bwd_bf16(const float* dy, const void* wo, const void* act, int64_t P, void* dz, float* part,
                         float* tmp, float* dWo, hipStream_t st) {
    if (!dz && !dWo) return;
    const int nblk = wgrad_out_blocks(P);  // P = 0: one block writes zeros
    const int64_t rpb = ((P + nblk - 1) / nblk + 7) / 8 * 8;
    out_bwd_bf16_kernel<<<nblk, 256, 0, st>>>(dy, (const __bf16*)wo, (const __bf16*)act, P, rpb,
                                              (__bf16*)dz, dWo ? part : nullptr);
    if (dWo) launch_colsum(part, nblk, (int64_t)kOut * 256, 1, 0, tmp, dWo, 0, st);
}

int wgrad_mfma_blocks(int64_t P) { return (int)std::max<int64_t>(1, std::min<int64_t>(256, (P + 1023) / 1024)); }

void launch_wgrad_mfma(const void* dz, const void* act, int64_t P, float* part, float* tmp, float* dW, float* db,
                       hipStream_t st) {
    const int nblk = wgrad_mfma_blocks(P);  // P = 0: one block writes zeros
    const int64_t rpb = ((P + nblk - 1) / nblk + 31) / 32 * 32;
    if (db)
        wgrad_mfma_kernel<true><<<nblk, 64 * kWgWaves, 0, st>>>((const __bf16*)dz, (const __bf16*)act, P, rpb, part);
    else
        wgrad_mfma_kernel<false><<<nblk, 64 * kWgWaves, 0, st>>>((const __bf16*)dz, (const __bf16*)act, P, rpb, part);
    launch_colsum(part, nblk, 65536, 1, 0, tmp, dW, 0, st);
    if (db) launch_colsum(part + (size_t)nblk * 65536, nblk, 256, 1, 0, tmp, db, 0, st);
}

int layer1_grad_blocks(int N) { return (N + kL1Rows - 1) / kL1Rows; }

void launch_layer1_grad(const void* dz1, const void* W, const void* act, int B, int N, float* S, float* Rpart,
                        hipStream_t st) {
    if (N > 0 && B > 0)
        layer1_grad_kernel<<<layer1_grad_blocks(N), 64 * kL1Waves, 0, st>>>(
            (const __bf16*)dz1, (const __bf16*)W, (const __bf16*)act, B, N, S, Rpart);
}

int layer1_sums_blocks(int N) { return (N + kSumRows - 1) / kSumRows; }

void launch_layer1_sums(const float* z, const void* act, int B, int N, float* S, float* Rpart, hipStream_t st) {
    if (N <= 0 || B <= 0) return;
    if (act)
        layer1_sums_kernel<true><<<layer1_sums_blocks(N), 256, 0, st>>>(z, (const __bf16*)act, B, N, S, Rpart);
    else
        layer1_sums_kernel<false><<<layer1_sums_blocks(N), 256, 0, st>>>(z, nullptr, B, N, S, Rpart);
}

void launch_to_bf16(const float* x, int64_t n, void* y, hipStream_t st) {
    if (n > 0) to_bf16_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(x, n, (__bf16*)y);
}

void launch_colsum_bf16(const void* A, int64_t rows, int64_t cols, int nz, int64_t bs, float* part, float* out,
                        int64_t out_bs, hipStream_t st) {
    if (cols <= 0 || nz <= 0) return;
    if (cols % 4 == 0 && bs % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 7) == 0) {
        colsum4((const __bf16*)A, rows, cols, nz, bs, part, out, out_bs, st);
        return;
    }
    const int nblk = colsum_blocks(rows);
    const int64_t rpb = (rows + nblk - 1) / nblk;
    const unsigned gx = (unsigned)((cols + 255) / 256);
    colsum_stage1_bf16_kernel<<<dim3(gx, nblk, nz), 256, 0, st>>>((const __bf16*)A, rows, cols, rpb, bs, part);
    colsum8_stage2_kernel<<<dim3((unsigned)((cols + 7) / 8), nz), 256, 0, st>>>(part, nblk, cols, out, out_bs);
}

void launch_mean_features_f32(const DevScene& s, float* out, hipStream_t st) {
    if (s.n > 0) mean_features_f32_kernel<<<(s.n + 255) / 256, 256, 0, st>>>(s.mx, s.my, s.n, s.W, s.H, out);
}

}  // namespace swf
