// Deformation MLP on BF16 MFMA with FP32 accumulation, fused with the deform +
// preprocess epilogue (Sec. 4.2: residuals = F_theta(gamma(mu), gamma(s)),
// G^s = G^0 + residuals).
//
// Formulation: every layer computes D = W * H^T with the weights as the MFMA A
// operand (16 output features x 32 k) and the activations as the B operand
// (32 k x 16 pairs), v_mfma_f32_16x16x32_bf16. The D layout of one 16x16 tile
// puts pair n = lane % 16 in a lane and output features 4*(lane/16) + j
// (j < 4) in its four registers; two vertically adjacent tiles therefore hold
// exactly 8 features per lane, which is the B operand of one 32-wide k-chunk of
// the next layer once the next layer's weights are packed with the same k order
// f(g, j) = j < 4 ? 4g + j : 16 + 4g + (j - 4). Activations never leave the
// registers between layers.
//
// Each wave owns 64 pairs (4 column blocks of 16); a workgroup of 4 waves owns
// 256. Weight fragments (1 KiB each: 64 lanes x 8 bf16, in lane order) are
// streamed from a packed global buffer through a 3-slot LDS ring of 16 KiB
// chunks with one barrier per chunk; the workgroups are persistent so the
// weight stream never drains between tiles.
#include "kernels.h"
#include "mlp_common.h"
#include "swf_device.h"

namespace swf {

bool bf16_available() { return true; }

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kChunkBytes = 16384;          // 16 fragments of 1 KiB
constexpr int kChunkU4 = kChunkBytes / 16;  // uint4 per chunk (1024)
constexpr int kSlots = 3;
constexpr int kPairsPerWave = 64;
constexpr int kPairsPerBlock = 256;

struct Bf16Args {
    MlpArgs m;
    const uint4* stream;      // packed weight chunks
    int n_chunks;             // chunks per tile: 2 + 8 * (n_hidden - 1)
    const bf16x8* mfeat;      // [N][32] bf16 mean features (4 x bf16x8 per Gaussian)
    const float* bias_h[7];   // biases of hidden layers 1..n_hidden-1
    const float* bias_o;      // output bias
    int n_tiles;
};

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 pack_relu(f32x4 lo, f32x4 hi, float4 blo, float4 bhi) {
    bf16x8 r;
    r[0] = (__bf16)fmaxf(lo[0] + blo.x, 0.f);
    r[1] = (__bf16)fmaxf(lo[1] + blo.y, 0.f);
    r[2] = (__bf16)fmaxf(lo[2] + blo.z, 0.f);
    r[3] = (__bf16)fmaxf(lo[3] + blo.w, 0.f);
    r[4] = (__bf16)fmaxf(hi[0] + bhi.x, 0.f);
    r[5] = (__bf16)fmaxf(hi[1] + bhi.y, 0.f);
    r[6] = (__bf16)fmaxf(hi[2] + bhi.z, 0.f);
    r[7] = (__bf16)fmaxf(hi[3] + bhi.w, 0.f);
    return r;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void mlp_bf16_kernel(Bf16Args a) {
    __shared__ __attribute__((aligned(16))) uint4 ring[kSlots * kChunkU4];
    __shared__ float outs[4][kPairsPerWave][8];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int g = lane >> 4;       // lane group (k / feature sub-block)
    const int n16 = lane & 15;     // pair column inside a 16-wide block
    const size_t total = (size_t)a.m.N * a.m.B;
    const int S = a.n_chunks;
    const int n_mid = a.m.n_mid;

    // tiles of this persistent workgroup
    const int my_tiles = a.n_tiles > (int)blockIdx.x ? (a.n_tiles - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
    const int64_t q_end = (int64_t)my_tiles * S;  // chunk steps of this workgroup
    if (my_tiles == 0) return;

    // ring prologue: chunks 0, 1 into slots 0, 1; chunk 2 into registers
    uint4 pf[4];
    auto fetch = [&](int64_t q) {
        const int c = (int)(q % S);
#pragma unroll
        for (int i = 0; i < 4; ++i) pf[i] = a.stream[(size_t)c * kChunkU4 + tid + i * 256];
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ring[slot * kChunkU4 + tid + i * 256] = pf[i];
    };
    fetch(0);
    store(0);
    if (q_end > 1) {
        fetch(1);
        store(1);
    }
    if (q_end > 2) fetch(2);
    __syncthreads();
    int64_t q = 0;  // chunk step being computed
    // per step: store the prefetched chunk q+2, fetch chunk q+3, compute q, barrier
    auto advance = [&]() {
        if (q + 2 < q_end) store((int)((q + 2) % kSlots));
        if (q + 3 < q_end) fetch(q + 3);
    };
    auto frag = [&](int t) -> bf16x8 {
        const uint4 v = ring[(int)(q % kSlots) * kChunkU4 + t * 64 + lane];
        return __builtin_bit_cast(bf16x8, v);
    };

    f32x4 acc[16][4];
    bf16x8 act[8][4];

    for (int it = 0; it < my_tiles; ++it) {
        const size_t tile = (size_t)blockIdx.x + (size_t)it * gridDim.x;
        const size_t base = tile * kPairsPerBlock + (size_t)wave * kPairsPerWave;
        // ---- layer 1 (mean part, K = 32): B = bf16 gamma(mu_hat) ----
        bf16x8 bm[4];
        int qb[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const size_t row = base + cb * 16 + n16;
            if (row < total) {
                const int p = (int)(row % a.m.N);
                bm[cb] = a.mfeat[(size_t)p * 4 + g];
                qb[cb] = (int)(row / a.m.N);
            } else {
                bm[cb] = bf16x8{};
                qb[cb] = 0;
            }
        }
        advance();
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const bf16x8 w = frag(t);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[t][cb] = mfma(w, bm[cb], f32x4{0.f, 0.f, 0.f, 0.f});
        }
        __syncthreads();
        ++q;
        // layer-1 bias is the per-query transceiver part qs[b]
#pragma unroll
        for (int c = 0; c < 8; ++c) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const float* qrow = a.m.qs + (size_t)qb[cb] * 256 + 32 * c + 4 * g;
                const float4 blo = *reinterpret_cast<const float4*>(qrow);
                const float4 bhi = *reinterpret_cast<const float4*>(qrow + 16);
                act[c][cb] = pack_relu(acc[2 * c][cb], acc[2 * c + 1][cb], blo, bhi);
            }
        }
        // ---- hidden layers ----
        for (int l = 0; l < n_mid; ++l) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                advance();
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const bf16x8 w = frag(t);
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb)
                        acc[t][cb] = mfma(w, act[c][cb], c == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : acc[t][cb]);
                }
                __syncthreads();
                ++q;
            }
            const float* bias = a.bias_h[l];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float4 blo = *reinterpret_cast<const float4*>(bias + 32 * c + 4 * g);
                const float4 bhi = *reinterpret_cast<const float4*>(bias + 32 * c + 16 + 4 * g);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) act[c][cb] = pack_relu(acc[2 * c][cb], acc[2 * c + 1][cb], blo, bhi);
            }
        }
        // ---- output layer: one 16-row tile (7 used), 8 k-chunks in one ring chunk ----
        advance();
        f32x4 o[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) o[cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const bf16x8 w = frag(c);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) o[cb] = mfma(w, act[c][cb], o[cb]);
        }
        // lane (g, n16) holds outputs 4g..4g+3 of pair cb*16+n16: transpose via LDS
        if (g < 2) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int oi = 4 * g + j;
                    outs[wave][cb * 16 + n16][oi] = oi < kOut ? o[cb][j] + a.bias_o[oi] : 0.f;
                }
        }
        __syncthreads();
        ++q;
        {
            const size_t row = base + lane;
            if (row < total) deform_epilogue(a.m, row, (int)(row % a.m.N), outs[wave][lane]);
        }
        // `outs` is rewritten only after the next tile's first barrier
    }
}

__global__ void mean_features_bf16_kernel(const float* __restrict__ mx, const float* __restrict__ my, int n, int W,
                                          int H, __bf16* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float f[kMeanFeat];
    mean_features(mx[p], my[p], W, H, f);
#pragma unroll
    for (int k = 0; k < 32; ++k) out[(size_t)p * 32 + k] = (__bf16)(k < kMeanFeat ? f[k] : 0.f);
}

int n_persistent_blocks() {
    static int n = 0;
    if (!n) {
        int dev = 0, cus = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        n = cus > 0 ? cus : 256;
    }
    return n;
}

}  // namespace

void compute_mean_features_bf16(DevScene& s, hipStream_t st) {
    if (s.n > 0)
        mean_features_bf16_kernel<<<(s.n + 255) / 256, 256, 0, st>>>(s.mx, s.my, s.n, s.W, s.H,
                                                                      reinterpret_cast<__bf16*>(s.bf_mfeat));
}

void launch_mlp_bf16(const DevScene& s, const float* qs, int B, const Grid& g, bool paper_mask, const Records& r,
                     float* delta_out, hipStream_t st) {
    Bf16Args a{};
    a.m = make_args(s, qs, B, g, paper_mask, r, delta_out);
    a.stream = reinterpret_cast<const uint4*>(s.bf_stream);
    a.n_chunks = 2 + 8 * (s.n_hidden - 1);
    a.mfeat = reinterpret_cast<const bf16x8*>(s.bf_mfeat);
    for (int l = 0; l + 1 < s.n_hidden && l < 7; ++l) a.bias_h[l] = s.b[l + 1];
    a.bias_o = s.b[s.n_hidden];
    const size_t total = (size_t)s.n * B;
    a.n_tiles = (int)((total + kPairsPerBlock - 1) / kPairsPerBlock);
    if (!a.n_tiles) return;
    const int blocks = std::min(a.n_tiles, n_persistent_blocks());
    mlp_bf16_kernel<<<blocks, 256, 0, st>>>(a);
}

}  // namespace swf
