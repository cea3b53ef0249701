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
//
// Preprocess backward maps d(M, opacity) to the 7 residual coordinates
// (d_mean, d_log_scale, d_rotation, d_logit, d_amp); the MLP backward is a
// chain of row-parallel products (dZ_{l-1} = (dZ_l W_l) . [H_{l-1} > 0]) and
// split-K weight-gradient reductions (dW_l = dZ_l^T H_{l-1}) in FP32.
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int TILE>
__global__ __launch_bounds__(TILE* TILE) void blend_backward_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals, const float4* __restrict__ geo,
    const float4* __restrict__ wm, const float2* __restrict__ oa, int H, int W, int TW, int tiles,
    const float* __restrict__ grad_out, const float* __restrict__ aux_T, const uint32_t* __restrict__ aux_last,
    float* __restrict__ dpair) {
    constexpr int kN = TILE * TILE;
    __shared__ float2 s_pos[kN];
    __shared__ float4 s_wm[kN];
    __shared__ float2 s_oa[kN];
    __shared__ uint32_t s_v[kN];
    __shared__ uint32_t s_max;

    const int gtile = blockIdx.x;
    const int b = gtile / tiles;
    const int t = gtile - b * tiles;
    const int tx = t % TW, ty = t / TW;
    const int lx = threadIdx.x % TILE, ly = threadIdx.x / TILE;
    const int px = tx * TILE + lx, py = ty * TILE + ly;
    const bool inside = px < W && py < H;
    const int bx0 = (tx * TILE) & ~63, by0 = (ty * TILE) & ~63;
    const float x0 = (float)bx0, y0 = (float)by0;
    const float fx = (float)(px - bx0), fy = (float)(py - by0);
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
    const int lmax = (int)s_max;
    float S = 0.0f;

    for (int end = lmax; end > 0; end -= kN) {
        const int beg = end > kN ? end - kN : 0;
        __syncthreads();
        {
            const int j = beg + (int)threadIdx.x;
            if (j < end) {
                const uint32_t v = vals[rg.x + j];
                const float4 g = geo[v];
                s_pos[threadIdx.x] = make_float2((g.x - x0) + g.z, (g.y - y0) + g.w);
                s_wm[threadIdx.x] = wm[v];
                s_oa[threadIdx.x] = oa[v];
                s_v[threadIdx.x] = v;
            }
        }
        __syncthreads();
        for (int jj = end - beg - 1; jj >= 0; --jj) {
            const int j = beg + jj;
            float gv[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            bool contrib = false;
            if (j < (int)last) {
                const float4 m = s_wm[jj];
                float dx, dy, u, w;
                const float q = blend_q(fx, fy, s_pos[jj], m, dx, dy, u, w);
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
                            gv[6] = ga * (raw / o.x);       // d alpha / d opacity = exp(-q/2)
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
            if (__ballot(contrib) == 0ull) continue;
#pragma unroll
            for (int k = 0; k < 8; ++k) gv[k] = wave_sum(gv[k]);
            if ((threadIdx.x & 63) == 0) {
                float* dst = dpair + (size_t)s_v[jj] * 8;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (gv[k] != 0.0f) atomicAdd(dst + k, gv[k]);
            }
        }
    }
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
                                   const uint32_t* __restrict__ perm, int B, int N, float* const* __restrict__ out) {
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
        if (out[k]) out[k][id] = s[k];
}

// out[r][j] = sum_{k<K} in[r][k] * Wrm[k][j] (* [H[r][j] > 0] when H), r < P,
// j < 256. Wrm is a layer weight read as [K][256] (row-major [out][in] of the
// layer whose output dimension is K). 32 rows per block, thread owns 4 x 8.
__global__ __launch_bounds__(256) void dgrad_kernel(const float* __restrict__ in, int K, const float* __restrict__ Wrm,
                                                    const float* __restrict__ Hm, int64_t P,
                                                    float* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) float xs[32][36];
    __shared__ __attribute__((aligned(16))) float ws[32][256];
    const int tid = threadIdx.x, tr = tid >> 5, tc = tid & 31;
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    float acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[i][c] = 0.f;
    for (int k0 = 0; k0 < K; k0 += 32) {
        __syncthreads();
        for (int e = tid; e < 32 * 32; e += 256) {
            const int rr = e >> 5, kk = e & 31;
            const int64_t r = r0 + rr;
            xs[rr][kk] = (r < P && k0 + kk < K) ? in[r * K + k0 + kk] : 0.f;
        }
        for (int e = tid; e < 32 * 256; e += 256) {
            const int kk = e >> 8, j = e & 255;
            ws[kk][j] = (k0 + kk < K) ? Wrm[(size_t)(k0 + kk) * 256 + j] : 0.f;
        }
        __syncthreads();
        const int kn = min(32, K - k0);
        for (int kk = 0; kk < kn; ++kk) {
            const float4 w0 = *reinterpret_cast<const float4*>(&ws[kk][tc * 8]);
            const float4 w1 = *reinterpret_cast<const float4*>(&ws[kk][tc * 8 + 4]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float x = xs[tr * 4 + i][kk];
                acc[i][0] = fmaf(x, w0.x, acc[i][0]); acc[i][1] = fmaf(x, w0.y, acc[i][1]);
                acc[i][2] = fmaf(x, w0.z, acc[i][2]); acc[i][3] = fmaf(x, w0.w, acc[i][3]);
                acc[i][4] = fmaf(x, w1.x, acc[i][4]); acc[i][5] = fmaf(x, w1.y, acc[i][5]);
                acc[i][6] = fmaf(x, w1.z, acc[i][6]); acc[i][7] = fmaf(x, w1.w, acc[i][7]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + tr * 4 + i;
        if (r >= P) continue;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int j = tc * 8 + c;
            float v = acc[i][c];
            if (Hm && !(Hm[r * 256 + j] > 0.f)) v = 0.f;
            out[r * 256 + j] = v;
        }
    }
}

// Partial weight gradients dW[o][i] = sum_{r in chunk} dz[r][o] X[r][i] for a
// 64 x 64 output tile (thread owns 4 x 4). X rows come from one matrix
// (ld = I) or, for layer 1, from the per-Gaussian mean features (26) and the
// per-query transceiver features (63). part is [chunks][O][I].
__global__ __launch_bounds__(256) void wgrad_partial_kernel(const float* __restrict__ dz, int O,
                                                            const float* __restrict__ X, int I,
                                                            const float* __restrict__ fmean,
                                                            const float* __restrict__ ftx, int N, int64_t P,
                                                            int64_t rows_per_chunk, float* __restrict__ part) {
    __shared__ float zs[32][65];
    __shared__ float xs[32][65];
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const int o0 = blockIdx.x * 64, i0 = blockIdx.y * 64;
    const int64_t rb = (int64_t)blockIdx.z * rows_per_chunk;
    const int64_t re = min(rb + rows_per_chunk, P);
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = 0.f;
    for (int64_t r0 = rb; r0 < re; r0 += 32) {
        __syncthreads();
        for (int e = tid; e < 32 * 64; e += 256) {
            const int rr = e >> 6, cc = e & 63;
            const int64_t r = r0 + rr;
            const bool okr = r < re;
            zs[rr][cc] = (okr && o0 + cc < O) ? dz[r * O + o0 + cc] : 0.f;
            float xv = 0.f;
            const int ii = i0 + cc;
            if (okr && ii < I) {
                if (X) {
                    xv = X[r * I + ii];
                } else {
                    xv = ii < kMeanFeat ? fmean[(r % N) * kMeanFeat + ii] : ftx[(r / N) * kTxFeat + ii - kMeanFeat];
                }
            }
            xs[rr][cc] = xv;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < 32; ++rr) {
            float zv[4], xv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) zv[a] = zs[rr][ty * 4 + a];
#pragma unroll
            for (int c = 0; c < 4; ++c) xv[c] = xs[rr][tx * 4 + c];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[a][c] = fmaf(zv[a], xv[c], acc[a][c]);
        }
    }
    float* dst = part + (size_t)blockIdx.z * O * I;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int o = o0 + ty * 4 + a;
        if (o >= O) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + tx * 4 + c;
            if (i < I) dst[(size_t)o * I + i] = acc[a][c];
        }
    }
}

__global__ void chunk_sum_kernel(const float* __restrict__ part, int chunks, int64_t m, float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(size_t)c * m + e];
    out[e] = s;
}

// Column sums of dz (P x O) per row chunk: part[chunk][o].
__global__ __launch_bounds__(256) void colsum_partial_kernel(const float* __restrict__ dz, int O, int64_t P,
                                                             int64_t rows_per_chunk, float* __restrict__ part) {
    const int o = blockIdx.x * 256 + threadIdx.x;
    if (o >= O) return;
    const int64_t rb = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t re = min(rb + rows_per_chunk, P);
    float s = 0.f;
    for (int64_t r = rb; r < re; ++r) s += dz[r * O + o];
    part[(size_t)blockIdx.y * O + o] = s;
}

// d gamma(mu_hat) (26 per row) -> d mu0 per Gaussian, summed over the batch.
__global__ void pe_backward_kernel(const float* __restrict__ dz0, const float* __restrict__ W0, int in_dim,
                                   const float* __restrict__ mx, const float* __restrict__ my, int B, int N, int Wd,
                                   int Hd, float* __restrict__ dmu) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    float dg[kMeanFeat];
#pragma unroll
    for (int i = 0; i < kMeanFeat; ++i) dg[i] = 0.f;
    for (int b = 0; b < B; ++b) {
        const float* z = dz0 + ((size_t)b * N + p) * 256;
        for (int o = 0; o < 256; ++o) {
            const float zo = z[o];
            if (zo == 0.f) continue;
            const float* w = W0 + (size_t)o * in_dim;
#pragma unroll
            for (int i = 0; i < kMeanFeat; ++i) dg[i] = fmaf(zo, w[i], dg[i]);
        }
    }
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
                           hipStream_t st) {
    const unsigned blocks = (unsigned)(B * g.tiles);
    if (!blocks) return;
    if (g.tile == 8)
        blend_backward_kernel<8><<<blocks, 64, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles,
                                                        grad_out, aux_T, aux_last, dpair);
    else
        blend_backward_kernel<16><<<blocks, 256, 0, st>>>(ranges, vals, r.geo, r.wm, r.oa, g.H, g.W, g.TW, g.tiles,
                                                          grad_out, aux_T, aux_last, dpair);
}

void launch_preprocess_backward(const float* dpair, const Records& r, int64_t P, bool paper_mask, float* dbase,
                                float* dy, hipStream_t st) {
    if (P > 0)
        preprocess_backward_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(dpair, r.wm, r.oa, r.count, P,
                                                                                paper_mask ? 1 : 0, dbase, dy);
}

void launch_base_reduce(const float* dbase, const float* dmu_pe, const uint32_t* perm, int B, int N,
                        float* const* out_dev, hipStream_t st) {
    if (N > 0) base_reduce_kernel<<<(N + 255) / 256, 256, 0, st>>>(dbase, dmu_pe, perm, B, N, out_dev);
}

void launch_dgrad(const float* in, int K, const float* Wrm, const float* Hmask, int64_t P, float* out,
                  hipStream_t st) {
    if (P > 0) dgrad_kernel<<<(unsigned)((P + 31) / 32), 256, 0, st>>>(in, K, Wrm, Hmask, P, out);
}

int64_t wgrad_chunks(int64_t P) { return std::max<int64_t>(1, std::min<int64_t>(256, (P + 4095) / 4096)); }

void launch_wgrad(const float* dz, int O, const float* X, int I, const float* fmean, const float* ftx, int N, int64_t P,
                  float* part, float* dW, float* db, hipStream_t st) {
    const int64_t chunks = wgrad_chunks(P);
    const int64_t rpc = (P + chunks - 1) / chunks;
    if (dW) {
        dim3 grid((O + 63) / 64, (I + 63) / 64, (unsigned)chunks);
        wgrad_partial_kernel<<<grid, 256, 0, st>>>(dz, O, X, I, fmean, ftx, N, P, rpc, part);
        const int64_t m = (int64_t)O * I;
        chunk_sum_kernel<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(part, (int)chunks, m, dW);
    }
    if (db) {
        dim3 grid((O + 255) / 256, (unsigned)chunks);
        colsum_partial_kernel<<<grid, 256, 0, st>>>(dz, O, P, rpc, part);
        chunk_sum_kernel<<<(unsigned)((O + 255) / 256), 256, 0, st>>>(part, (int)chunks, O, db);
    }
}

void launch_pe_backward(const float* dz0, const DevScene& s, int B, float* dmu, hipStream_t st) {
    if (s.n > 0)
        pe_backward_kernel<<<(s.n + 127) / 128, 128, 0, st>>>(dz0, s.w[0], s.in_dim, s.mx, s.my, B, s.n, s.W, s.H,
                                                              dmu);
}

void launch_mean_features_f32(const DevScene& s, float* out, hipStream_t st) {
    if (s.n > 0) mean_features_f32_kernel<<<(s.n + 255) / 256, 256, 0, st>>>(s.mx, s.my, s.n, s.W, s.H, out);
}

}  // namespace swf
