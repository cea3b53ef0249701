// Positional encoding, FP32 deformation MLP with the fused deform + preprocess
// epilogue, and the static (no-MLP) preprocess.
//
// Deformation MLP (Sec. 4.2): residuals = F_theta(gamma(mu_hat), gamma(s_hat)).
// Layer 1 is split: its transceiver part W1s gamma(s_hat) + b1 is the same for
// every Gaussian of a query and is computed once per query (tx_features); its
// mean part W1m gamma(mu_hat) (K = 26) runs per pair. Every later layer is a
// dense 256 x 256 contraction per pair, on the FP32 matrix cores.
#include "kernels.h"
#include "swf_device.h"
#include "mlp_common.h"

namespace swf {

namespace {

// gamma(s_hat) for one query and the per-query layer-1 partial sum
// qs[b][j] = b1[j] + sum_k W1[j][26 + k] gamma_k(s_hat_b).
__global__ __launch_bounds__(256) void tx_features_kernel(const float* __restrict__ tx, const float* __restrict__ w1,
                                                          const float* __restrict__ b1, int hidden, int in_dim,
                                                          float lox, float loy, float loz, float rx, float ry,
                                                          float rz, float* __restrict__ qs,
                                                          float* __restrict__ feat_out) {
    __shared__ float feat[kTxFeat];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    if (t < 3 * (kTxBands + 1)) {
        const int d = t % 3;
        const int k = t / 3;  // 0: identity, 1..L: band k-1
        const float v = tx[b * 3 + d];
        const float lo = d == 0 ? lox : (d == 1 ? loy : loz);
        const float rg = d == 0 ? rx : (d == 1 ? ry : rz);
        float s, e, hi, lo2;
        two_sum(v, -lo, s, e);
        div_two(s, rg, hi, lo2);
        lo2 += e / rg;
        if (k == 0) {
            feat[d] = hi + lo2;
        } else {
            float sv, cv;
            sincospi_scaled(hi, lo2, k - 1, sv, cv);
            feat[3 + 3 * (k - 1) + d] = sv;
            feat[3 + 3 * kTxBands + 3 * (k - 1) + d] = cv;
        }
    }
    __syncthreads();
    if (feat_out && t < kTxFeat) feat_out[(size_t)b * kTxFeat + t] = feat[t];
    for (int j = t; j < hidden; j += blockDim.x) {
        const float* row = w1 + (size_t)j * in_dim + kMeanFeat;
        float acc = b1[j];
        for (int k = 0; k < kTxFeat; ++k) acc = fmaf(row[k], feat[k], acc);
        qs[(size_t)b * hidden + j] = acc;
    }
}

// ---- FP32 MLP on the matrix cores ---------------------------------------------
// v_mfma_f32_16x16x4_f32 (FP32 products and sums): per layer D = W H with 16
// output units x 16 pairs per instruction and K = 4 inputs. A wave holds 16
// pairs; the hidden state stays in registers as B operands: for input chunk c
// lane l holds input k(c, l / 16) of pair l % 16. The result of output tile t
// (4 registers per lane: units 16 t + 4 (l / 16) + i, i = 0..3) is, after the
// ReLU, exactly the next layer's chunks 4 t + i, since the fragment-major
// weights list their input columns in that order. Layer 1 takes the 26 mean
// features (chunk c of lane group g = feature 4 c + g, zero past 26) with the
// per-query TX part qs[b] + b1 as its bias; the output layer is one tile of 16
// rows, 7 used. Weight fragments (16 bytes per lane, 4 instructions each) are
// read from the L2-resident packed copy kPrefetch fragments ahead of their use;
// a scheduling barrier after each fragment's instructions keeps every load
// where it is written (left free, the compiler sinks the loads next to their
// use, which leaves one or two in flight and exposes the L2 latency).
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kFWaves = 4;     // waves per block, 16 pairs each
constexpr int kPrefetch = 2;   // weight fragments in flight ahead of the one in use

// store (optional): the lane's 16-byte slice of each output tile; mask (optional, with store): stored values
// are zeroed where mask <= 0 (read at the tile's start, its latency under the tile's instructions).
template <int kTiles, int kIn, bool kRelu>
__device__ __forceinline__ void f32_mfma_layer(const float4* __restrict__ wf, const float* brow, int lane,
                                               const float (&hin)[kIn], float (&hout)[64], float* store,
                                               const float* mask = nullptr) {
    constexpr int G = kIn / 4;  // fragments per output tile
    constexpr int F = kTiles * G;
    const int g = lane >> 4;
    float4 wq[kPrefetch];
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) wq[i] = i < F ? wf[i * 64 + lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int t = 0; t < kTiles; ++t) {
        const float4 b4 = *reinterpret_cast<const float4*>(brow + 16 * t + 4 * g);
        f32x4 acc = f32x4{b4.x, b4.y, b4.z, b4.w};
        const float4 mk = mask ? *reinterpret_cast<const float4*>(mask + 16 * t + 4 * g)
                               : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int f = t * G + q;
            const float4 w = wq[0];
#pragma unroll
            for (int i = 0; i + 1 < kPrefetch; ++i) wq[i] = wq[i + 1];
            if (f + kPrefetch < F) wq[kPrefetch - 1] = wf[(f + kPrefetch) * 64 + lane];
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, hin[4 * q + 0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.y, hin[4 * q + 1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.z, hin[4 * q + 2], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w, hin[4 * q + 3], acc, 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) hout[4 * t + i] = kRelu ? fmaxf(acc[i], 0.0f) : acc[i];
        if (store)
            *reinterpret_cast<float4*>(store + 16 * t + 4 * g) =
                make_float4(mk.x > 0.0f ? hout[4 * t] : 0.0f, mk.y > 0.0f ? hout[4 * t + 1] : 0.0f,
                            mk.z > 0.0f ? hout[4 * t + 2] : 0.0f, mk.w > 0.0f ? hout[4 * t + 3] : 0.0f);
    }
}

// kMix: the queries of a mixed batch, each with its own scene (parameters, grid
// and weights). A wave's 16 pairs lie in one 384-pair MLP tile of one query
// (the tiling of the batch's tables: a query's pairs padded to whole tiles), so
// every pair of a wave takes the same weights; waves past the batch's tiles or
// past their query's pairs do nothing.
constexpr int kMixGroups = 24;  // 16-pair groups per 384-pair MLP tile of a mixed batch

template <bool kMix>
__global__ __launch_bounds__(64 * kFWaves, 3) void mlp_fp32_kernel(MlpArgs a, MixBatch mix) {
    __shared__ float outv[kFWaves][16][8];
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int g = lane >> 4;
    // the wave's 16 pairs: this lane's record row and its index p in the scene; rows past the query are computed
    // on index 0 and not written
    bool active;  // wave-uniform
    size_t row = 0;
    int p = 0, npairs = 0;
    const MixScene* sc = nullptr;
    const float* qrow = nullptr;  // the layer-1 bias of the lane's query (its TX term)
    if constexpr (kMix) {
        const int gw = (int)blockIdx.x * kFWaves + wave;
        const int tile = gw / kMixGroups;
        active = tile < mix.queries[mix.B].mlp_tile_base;
        if (active) {
            const int q = mix_find(mix.queries, mix.B, tile, [](const MixQuery& x) { return x.mlp_tile_base; });
            sc = &mix.scenes[mix.queries[q].scene];
            const int pb = (tile - mix.queries[q].mlp_tile_base) * (16 * kMixGroups) + (gw % kMixGroups) * 16;
            npairs = sc->N;
            active = pb < npairs;
            p = pb + (lane & 15);
            row = (size_t)mix.queries[q].pair_base + p;
            qrow = a.qs + (size_t)q * 256;
        }
    } else {
        const size_t total = (size_t)a.N * a.B;
        const size_t p0 = ((size_t)blockIdx.x * kFWaves + wave) * 16;
        active = p0 < total;
        row = p0 + (lane & 15);
        npairs = row < total ? a.N : 0;  // a row past the batch: no pair
        p = row < total ? (int)(row % a.N) : 0;
        qrow = a.qs + (size_t)(row < total ? row / a.N : 0) * 256;
    }
    const bool in = kMix ? p < npairs : npairs > 0;
    if (!in) p = 0;
    if (active) {
        float x[8];
        {
            float f[kMeanFeat];
            if constexpr (kMix)
                mean_features(sc->mx[p], sc->my[p], sc->W, sc->H, f);
            else
                mean_features(a.mx[p], a.my[p], a.sW, a.sH, f);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float v0 = 4 * c < kMeanFeat ? f[4 * c] : 0.0f;
                const float v1 = 4 * c + 1 < kMeanFeat ? f[4 * c + 1] : 0.0f;
                const float v2 = 4 * c + 2 < kMeanFeat ? f[4 * c + 2] : 0.0f;
                const float v3 = 4 * c + 3 < kMeanFeat ? f[4 * c + 3] : 0.0f;
                x[c] = g == 0 ? v0 : (g == 1 ? v1 : (g == 2 ? v2 : v3));
            }
        }
        // the network's weights: the batch's scene (kMix, four hidden layers) or the launch's
        const float* frag = kMix ? sc->f32_frag : nullptr;
        const int n_mid = kMix ? 3 : a.n_mid;
        const auto WH = [&](int l) -> const float4* {
            return kMix ? reinterpret_cast<const float4*>(frag + frag_hidden_at(l + 1)) : a.wfh[l];
        };
        const auto BH = [&](int l) -> const float* { return kMix ? sc->bias_h[l] : a.bh[l]; };
        const float4* wf1 = kMix ? reinterpret_cast<const float4*>(frag) : a.wf1;
        const float4* wfo = kMix ? reinterpret_cast<const float4*>(frag + frag_out_at(4)) : a.wfo;
        const float* bo16 = kMix ? frag + frag_out_at(4) + kFragOut : a.bo16;
        const auto st_of = [&](int l) -> float* {
            return (!kMix && in && a.act_out[l]) ? a.act_out[l] + row * 256 : nullptr;
        };
        float hA[64], hB[64];
        f32_mfma_layer<16, 8, true>(wf1, qrow, lane, x, hA, st_of(0));
        int l = 0;
        for (; l + 2 <= n_mid; l += 2) {
            f32_mfma_layer<16, 64, true>(WH(l), BH(l), lane, hA, hB, st_of(l + 1));
            f32_mfma_layer<16, 64, true>(WH(l + 1), BH(l + 1), lane, hB, hA, st_of(l + 2));
        }
        if (l < n_mid) {
            f32_mfma_layer<16, 64, true>(WH(l), BH(l), lane, hA, hB, st_of(l + 1));
#pragma unroll
            for (int k = 0; k < 64; ++k) hA[k] = hB[k];
        }
        // output layer: lane l holds outputs 4 (l / 16) + i of pair l % 16
        f32_mfma_layer<1, 64, false>(wfo, bo16, lane, hA, hB, nullptr);
        if (g < 2) {
#pragma unroll
            for (int i = 0; i < 4; ++i) outv[wave][lane & 15][4 * g + i] = hB[i];
        }
    }
    __syncthreads();
    if (active && lane < 16 && in) {  // lanes 0..15 hold the wave's 16 pairs (lane l: pair l)
        if constexpr (kMix)
            mix_epilogue(*sc, a, row, p, outv[wave][lane]);
        else
            deform_epilogue(a, row, p, outv[wave][lane]);
    }
}

// Input gradient of a 256 x 256 layer of the FP32 backward on the same matrix
// cores: out[p][i] = [act[p][i] > 0] sum_o W[o][i] dz[p][o], the layer function
// above with W^T as its weights (fragment-major, packed by pack_wt_kernel) and
// no bias. A wave takes 16 pairs; lane l = 16 g + r loads input chunk 4 q + j
// (input 16 q + 4 g + j) of pair r as one 16-byte load per q, and stores the
// masked output tile t (units 16 t + 4 g + i) with one 16-byte store. With
// bpart, the layer's bias gradient rides along: bpart[block][o] = the sum of
// dz[p][o] over the block's 64 pairs (fixed order; rows past P count zero).
__device__ float kZeroBias[256];  // zero-initialised: the layer's bias

__global__ __launch_bounds__(64 * kFWaves, 3) void dz_f32_kernel(const float* __restrict__ dz,
                                                                 const float4* __restrict__ wt,
                                                                 const float* __restrict__ act, int64_t P,
                                                                 float* __restrict__ out, float* __restrict__ bpart) {
    __shared__ float4 s_b[kFWaves][64];
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int g = lane >> 4;
    const int64_t p0 = ((int64_t)blockIdx.x * kFWaves + wave) * 16;
    const int64_t row = p0 + (lane & 15);
    const bool in = row < P;
    float hin[64], hout[64];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const float4 v = in ? *reinterpret_cast<const float4*>(dz + row * 256 + 16 * q + 4 * g)
                            : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        hin[4 * q] = v.x;
        hin[4 * q + 1] = v.y;
        hin[4 * q + 2] = v.z;
        hin[4 * q + 3] = v.w;
    }
    if (p0 < P)  // wave-uniform
        f32_mfma_layer<16, 64, false>(wt, kZeroBias, lane, hin, hout, in ? out + row * 256 : nullptr,
                                      in ? act + row * 256 : nullptr);
    if (!bpart) return;  // kernel-uniform: no wave reaches the barrier below
    // Column sums of dz over the wave's 16 rows, halving: at step s a lane keeps
    // the upper half of its values if bit s of r is set (else the lower half)
    // and adds its partner's (lane ^ 2^s) matching half. After four steps lane
    // (r, g) holds columns 16 q + 4 g + j, j = 0..3, with q the 4-bit reversal of r.
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const int half = 32 >> step;
        const bool up = (lane >> step) & 1;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const float send = up ? hin[i] : hin[half + i];
            const float keep = up ? hin[half + i] : hin[i];
            hin[i] = keep + __shfl_xor(send, 1 << step);
        }
    }
    const int r = lane & 15;
    const int q = ((r & 1) << 3) | ((r & 2) << 1) | ((r & 4) >> 1) | ((r & 8) >> 3);
    s_b[wave][4 * q + g] = make_float4(hin[0], hin[1], hin[2], hin[3]);
    __syncthreads();
    static_assert(64 * kFWaves == 256, "one thread per column");
    const int c = (int)threadIdx.x;
    const float* sb = reinterpret_cast<const float*>(s_b);
    float sum = sb[c];
#pragma unroll
    for (int w = 1; w < kFWaves; ++w) sum += sb[w * 256 + c];
    bpart[(size_t)blockIdx.x * 256 + c] = sum;
}

// W^T of a 256 x 256 layer (W row-major [out][in]) in the fragment order of
// f32_mfma_layer: fragment q of output tile t, lane l = 16 g + r, element j
// holds W^T[16 t + r][16 q + 4 g + j] = W[16 q + 4 g + j][16 t + r].
__global__ void pack_wt_kernel(const float* __restrict__ w, float* __restrict__ wt) {
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= 65536) return;
    const int t = e / 4096, q = (e / 256) % 16, l = (e / 4) % 64, j = e % 4;
    wt[e] = w[(size_t)(16 * q + 4 * (l >> 4) + j) * 256 + 16 * t + (l & 15)];
}

__global__ void preprocess_static_kernel(MlpArgs a) {
    const size_t row = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)a.N * a.B;
    if (row >= total) return;
    const int p = (int)(row % a.N);
    PairOut o;
    if (p < a.n_live) {
        o = preprocess_pair(a.mx[p], a.my[p], 0.f, 0.f, a.lsx[p], a.lsy[p], a.rot[p], a.logit[p], a.amp[p], a.W, a.H,
                            a.TW, a.TH, a.inv_tile, a.wrap, a.sx, a.sy);
    } else {
        o.geo = make_float4(0, 0, 0, 0);
        o.wm = make_float4(0, 0, 0, 0);
        o.oa = make_float2(0, 0);
        o.rect_x = o.rect_y = 0;
        o.count = 0;
    }
    write_record(a.rec, row, o);
}

__global__ void permute_delta_kernel(const float* __restrict__ src, const uint32_t* __restrict__ perm, int B, int n,
                                     float* __restrict__ dst) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)B * n) return;
    const size_t b = i / n, p = i % n;
    const size_t o = b * n + perm[p];
#pragma unroll
    for (int k = 0; k < kOut; ++k) dst[o * kOut + k] = src[i * kOut + k];
}

struct Ptr7 {
    const float* s[7];
    float* d[7];
};

__global__ void gather_params_kernel(Ptr7 p, const uint32_t* __restrict__ perm, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t src = perm[i];
#pragma unroll
    for (int k = 0; k < 7; ++k) p.d[k][i] = p.s[k][src];
}

}  // namespace

void launch_gather_params(float* const* src, const uint32_t* perm, int n, float* const* dst, hipStream_t st) {
    Ptr7 p;
    for (int k = 0; k < 7; ++k) {
        p.s[k] = src[k];
        p.d[k] = dst[k];
    }
    if (n > 0) gather_params_kernel<<<(n + 255) / 256, 256, 0, st>>>(p, perm, n);
}

void launch_tx_features(const DevScene& s, const float* tx, int B, float* qs, hipStream_t st, float* feat_out) {
    const float rx = s.room_hi[0] - s.room_lo[0], ry = s.room_hi[1] - s.room_lo[1], rz = s.room_hi[2] - s.room_lo[2];
    tx_features_kernel<<<B, 256, 0, st>>>(tx, s.w[0], s.b[0], s.hidden, s.in_dim, s.room_lo[0], s.room_lo[1],
                                          s.room_lo[2], rx, ry, rz, qs, feat_out);
}

void launch_mlp_fp32(const DevScene& s, const float* qs, int B, const Grid& g, bool paper_mask, const Records& r,
                     float* delta_out, hipStream_t st, float* const* act_out) {
    MlpArgs a = make_args(s, qs, B, g, paper_mask, r, delta_out);
    if (act_out)
        for (int l = 0; l < s.n_hidden && l < 8; ++l) a.act_out[l] = act_out[l];
    const size_t total = (size_t)s.n * B;
    const size_t per_block = (size_t)kFWaves * 16;
    const unsigned blocks = (unsigned)((total + per_block - 1) / per_block);
    if (blocks) mlp_fp32_kernel<false><<<blocks, 64 * kFWaves, 0, st>>>(a, MixBatch{});
}

void launch_mix_mlp_fp32(const MixBatch& m, const float* qs, const Records& r, int64_t pair_cap, int B_cap,
                         hipStream_t st, bool paper_mask, bool wrap) {
    // every 384-pair tile the batch can hold (its pairs, each query padded to whole tiles)
    const int64_t tiles = (pair_cap + 383) / 384 + B_cap;
    const int64_t blocks = (tiles * kMixGroups + kFWaves - 1) / kFWaves;
    MlpArgs a{};
    a.qs = qs;
    a.rec = r;
    a.inv_tile = 1.0f / 16.0f;
    a.paper_mask = paper_mask ? 1 : 0;
    a.wrap = wrap ? 1 : 0;
    if (blocks > 0) mlp_fp32_kernel<true><<<(unsigned)blocks, 64 * kFWaves, 0, st>>>(a, m);
}

void launch_preprocess_static(const DevScene& s, int B, const Grid& g, const Records& r, hipStream_t st) {
    const MlpArgs a = make_args(s, nullptr, B, g, false, r, nullptr);
    const size_t total = (size_t)s.n * B;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (blocks) preprocess_static_kernel<<<blocks, 256, 0, st>>>(a);
}

void launch_permute_delta(const float* delta_sorted, const uint32_t* perm, int B, int n, float* delta_out,
                          hipStream_t st) {
    const size_t total = (size_t)B * n;
    if (total) permute_delta_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(delta_sorted, perm, B, n, delta_out);
}

void launch_pack_wt(const float* w, float* wt, hipStream_t st) { pack_wt_kernel<<<256, 256, 0, st>>>(w, wt); }

int64_t dz_f32_blocks(int64_t P) { return (P + kFWaves * 16 - 1) / (kFWaves * 16); }

void launch_dz_f32(const float* dz, const float* wt, const float* act, int64_t P, float* out, float* bpart,
                   hipStream_t st) {
    if (P > 0)
        dz_f32_kernel<<<(unsigned)dz_f32_blocks(P), 64 * kFWaves, 0, st>>>(dz, reinterpret_cast<const float4*>(wt),
                                                                            act, P, out, bpart);
}

}  // namespace swf
