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
typedef short short2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t cvt_pk_bf16(float a, float b) {
    const bf16x2 v = {(__bf16)a, (__bf16)b};  // v_cvt_pk_bf16_f32, round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}

constexpr int kChunkBytes = 32768;          // one ring step: 32 fragments of 1 KiB
constexpr int kChunkU4 = kChunkBytes / 16;  // uint4 per step (2048)
constexpr int kPF = kChunkU4 / 256;         // uint4 per thread per step (8)
constexpr int kSlots = 3;

struct Bf16Args {
    MlpArgs m;
    const uint4* stream;      // packed weight chunks
    int n_chunks;             // ring steps per tile: 2 + 4 * (n_hidden - 1)
    const bf16x8* mfeat;      // [N][32] bf16 mean features (4 x bf16x8 per Gaussian)
    const float* bias_h[7];   // biases of hidden layers 1..n_hidden-1
    const float* bias_o;      // output bias
    int n_tiles;              // B * tiles_per_query
    int tiles_per_query;      // ceil(N / pairs per block): tiles never straddle two queries
};

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Two accumulator tiles (features 4g..4g+3 and 16+4g..16+4g+3 of a 32-chunk)
// -> ReLU'd bf16 B operand. The bias is already in the accumulators. ReLU is
// applied after rounding as a signed 16-bit max with 0 (a negative bf16 is a
// negative int16), which equals rounding the ReLU'd float.
__device__ __forceinline__ bf16x8 pack_relu(f32x4 lo, f32x4 hi) {
    uint32_t w[4];
    w[0] = cvt_pk_bf16(lo[0], lo[1]);
    w[1] = cvt_pk_bf16(lo[2], lo[3]);
    w[2] = cvt_pk_bf16(hi[0], hi[1]);
    w[3] = cvt_pk_bf16(hi[2], hi[3]);
    const short2v z = {0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i)
        w[i] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(short2v, w[i]), z));
    uint4 u = make_uint4(w[0], w[1], w[2], w[3]);
    return __builtin_bit_cast(bf16x8, u);
}

// NCB column blocks of 16 pairs per wave (64 or 32 pairs); 4 waves per block.
template <int NCB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NCB == 2 ? 2 : 1, NCB == 2 ? 2 : 1))) void
mlp_bf16_kernel(Bf16Args a) {
    constexpr int kPairsPerWave = 16 * NCB;
    constexpr int kPairsPerBlock = 4 * kPairsPerWave;
    __shared__ __attribute__((aligned(16))) uint4 ring[kSlots * kChunkU4];
    __shared__ float outs[4][kPairsPerWave][8];
    // Layer-1 TX term of the current and the next tile's query, hidden and
    // output biases: C operands read from LDS, so no MFMA chain waits on a
    // global load.
    __shared__ __attribute__((aligned(16))) float qs_s[2][256];
    __shared__ __attribute__((aligned(16))) float bias_s[7][256];
    __shared__ __attribute__((aligned(16))) float bias_o_s[16];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int g = lane >> 4;       // lane group (k / feature sub-block)
    const int n16 = lane & 15;     // pair column inside a 16-wide block
    const int S = a.n_chunks;
    const int n_mid = a.m.n_mid;

    // tiles of this persistent workgroup
    const int my_tiles = a.n_tiles > (int)blockIdx.x ? (a.n_tiles - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
    if (my_tiles == 0) return;
    const int q_end = my_tiles * S;  // chunk steps of this workgroup
    for (int l = 0; l < n_mid; ++l) bias_s[l][tid] = a.bias_h[l][tid];
    if (tid < 16) bias_o_s[tid] = tid < kOut ? a.bias_o[tid] : 0.0f;
    qs_s[0][tid] = a.m.qs[(size_t)((int)blockIdx.x / a.tiles_per_query) * 256 + tid];

    // Ring of kSlots chunk slots. Step q computes from slot q % 3; during step q
    // the chunk q + 2 (prefetched into registers during step q - 1) is stored
    // into slot (q + 2) % 3 and chunk q + 3 is fetched; one barrier ends a step.
    // prefetched ring step: eight named registers per thread (an array here is
    // turned into LDS or scratch by the compiler)
    static_assert(kPF == 8, "the prefetch list below names eight registers");
    uint4 pf0, pf1, pf2, pf3, pf4, pf5, pf6, pf7;
    int fetch_chunk = 0;  // stream step index of the next fetch
#define SWF_PF_EACH(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7)
#define SWF_PF_LOAD(i_) pf##i_ = a.stream[(size_t)fetch_chunk * kChunkU4 + tid + (i_) * 256];
#define SWF_RING_FETCH()                                          \
    do {                                                          \
        SWF_PF_EACH(SWF_PF_LOAD)                                  \
        fetch_chunk = fetch_chunk + 1 == S ? 0 : fetch_chunk + 1; \
    } while (0)
#define SWF_PF_PUT(i_) ring[slot_base_ + tid + (i_) * 256] = pf##i_;
#define SWF_RING_STORE(slot_)                    \
    do {                                         \
        const int slot_base_ = (slot_) * kChunkU4; \
        SWF_PF_EACH(SWF_PF_PUT)                  \
    } while (0)
    SWF_RING_FETCH();
    SWF_RING_STORE(0);
    if (q_end > 1) {
        SWF_RING_FETCH();
        SWF_RING_STORE(1);
    }
    if (q_end > 2) SWF_RING_FETCH();
    __syncthreads();
    int q = 0;         // step being computed
    int slot = 0;      // q % 3
    // during step q: store the prefetched step q + 2, fetch step q + 3
#define SWF_RING_ADVANCE()                                      \
    do {                                                        \
        const int s2_ = slot == 0 ? 2 : slot - 1;               \
        if (q + 2 < q_end) SWF_RING_STORE(s2_);                 \
        if (q + 3 < q_end) SWF_RING_FETCH();                    \
    } while (0)
#define SWF_FRAG_AT(s_, t_) __builtin_bit_cast(bf16x8, ring[(s_) * kChunkU4 + (t_) * 64 + lane])
    // Fragment pipeline: the two fragments after the one in use are already in
    // registers, so an LDS read has two MFMA groups to land. Past the end of a
    // step the pipeline reads the first fragments of the next slot: that slot
    // was completed before the previous barrier and is not overwritten until two
    // barriers later, so reading it early is safe (at the last step it holds
    // stale data that is never used).
    bf16x8 w_a = SWF_FRAG_AT(0, 0), w_b = SWF_FRAG_AT(0, 1);
#define SWF_TAKE(dst_, f_, nf_)                                                                          \
    do {                                                                                                 \
        dst_ = w_a;                                                                                      \
        w_a = w_b;                                                                                       \
        const int nxt_ = slot == 2 ? 0 : slot + 1;                                                       \
        w_b = (f_) + 2 < (nf_) ? SWF_FRAG_AT(slot, (f_) + 2) : SWF_FRAG_AT(nxt_, (f_) + 2 - (nf_));      \
    } while (0)
#define SWF_NEXT_STEP()                      \
    do {                                     \
        __syncthreads();                     \
        ++q;                                 \
        slot = slot == 2 ? 0 : slot + 1;     \
    } while (0)

    f32x4 acc[16][NCB];
    bf16x8 act[8][NCB];

    for (int it = 0; it < my_tiles; ++it) {
        const int tile = (int)blockIdx.x + it * (int)gridDim.x;
        const int qry = tile / a.tiles_per_query;                  // block-uniform query
        const int p0 = (tile - qry * a.tiles_per_query) * kPairsPerBlock + wave * kPairsPerWave;
        const size_t row0 = (size_t)qry * a.m.N;                   // first pair of the query
        // ---- layer 1 (mean part, K = 32): B = bf16 gamma(mu_hat); C = qs[query] ----
        bf16x8 bm[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int p = p0 + cb * 16 + n16;
            bm[cb] = p < a.m.N ? a.mfeat[(size_t)p * 4 + g] : bf16x8{};
        }
        SWF_RING_ADVANCE();
        {
            const float* qrow = &qs_s[it & 1][4 * g];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const float4 b4 = *reinterpret_cast<const float4*>(qrow + 16 * t);
                const f32x4 c0 = {b4.x, b4.y, b4.z, b4.w};
                bf16x8 w;
                SWF_TAKE(w, t, 16);
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[t][cb] = mfma(w, bm[cb], c0);
            }
        }
        SWF_NEXT_STEP();
        // TX term of the next tile's query, stored to LDS before this tile's
        // last barrier (the other buffer is read by this tile's layer 1 only)
        const int next_tile = tile + (int)gridDim.x;
        const float qs_next =
            it + 1 < my_tiles ? a.m.qs[(size_t)(next_tile / a.tiles_per_query) * 256 + tid] : 0.0f;
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) act[c][cb] = pack_relu(acc[2 * c][cb], acc[2 * c + 1][cb]);
        // ---- hidden layers: C starts at the bias ----
        for (int l = 0; l < n_mid; ++l) {
            const float* bias = &bias_s[l][4 * g];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if ((c & 1) == 0) SWF_RING_ADVANCE();
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    bf16x8 w;
                    SWF_TAKE(w, (c & 1) * 16 + t, 32);
                    f32x4 c0;
                    if (c == 0) {
                        const float4 b4 = *reinterpret_cast<const float4*>(bias + 16 * t);
                        c0 = f32x4{b4.x, b4.y, b4.z, b4.w};
                    }
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) acc[t][cb] = mfma(w, act[c][cb], c == 0 ? c0 : acc[t][cb]);
                }
                if (c & 1) SWF_NEXT_STEP();
            }
#pragma unroll
            for (int c = 0; c < 8; ++c)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) act[c][cb] = pack_relu(acc[2 * c][cb], acc[2 * c + 1][cb]);
        }
        // ---- output layer: one 16-row tile (7 used), 8 k-chunks in one ring chunk ----
        SWF_RING_ADVANCE();
        f32x4 o[NCB];
        {
            const float4 b4 = *reinterpret_cast<const float4*>(&bias_o_s[4 * (g & 3)]);
            const f32x4 ob = {b4.x, b4.y, b4.z, b4.w};  // rows >= 7 are zero and never stored
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) o[cb] = ob;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            bf16x8 w;
            SWF_TAKE(w, c, 8);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) o[cb] = mfma(w, act[c][cb], o[cb]);
        }
        // lane (g, n16) holds outputs 4g..4g+3 of pair cb*16+n16: transpose via LDS
        if (g < 2) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int j = 0; j < 4; ++j) outs[wave][cb * 16 + n16][4 * g + j] = o[cb][j];
        }
        qs_s[(it + 1) & 1][tid] = qs_next;
        SWF_NEXT_STEP();
        if (lane < kPairsPerWave) {
            const int p = p0 + lane;
            if (p < a.m.N) deform_epilogue(a.m, row0 + p, p, outs[wave][lane]);
        }
        // `outs` is rewritten only after the next tile's first barrier
    }
#undef SWF_PF_EACH
#undef SWF_PF_LOAD
#undef SWF_PF_PUT
#undef SWF_RING_FETCH
#undef SWF_RING_STORE
#undef SWF_RING_ADVANCE
#undef SWF_FRAG_AT
#undef SWF_TAKE
#undef SWF_NEXT_STEP
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

int n_compute_units() {
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

// Workgroups of one variant that fit on a CU at once (registers and LDS decide;
// the grid is persistent, so launching more would only queue them).
int occupancy_query(int ncb) {
    int n = 0;
    const hipError_t e = ncb == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mlp_bf16_kernel<2>, 256, 0)
                                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mlp_bf16_kernel<4>, 256, 0);
    return (e == hipSuccess && n > 0) ? n : 1;
}

int resident_blocks(int ncb) {
    static const int c2 = occupancy_query(2);  // thread-safe one-time initialisation
    static const int c4 = occupancy_query(4);
    return ncb == 2 ? c2 : c4;
}

void launch_mlp_bf16(const DevScene& s, const float* qs, int B, const Grid& g, bool paper_mask, const Records& r,
                     float* delta_out, hipStream_t st, int pairs_per_wave) {
    Bf16Args a{};
    a.m = make_args(s, qs, B, g, paper_mask, r, delta_out);
    a.stream = reinterpret_cast<const uint4*>(s.bf_stream);
    a.n_chunks = 2 + 4 * (s.n_hidden - 1);
    a.mfeat = reinterpret_cast<const bf16x8*>(s.bf_mfeat);
    for (int l = 0; l + 1 < s.n_hidden && l < 7; ++l) a.bias_h[l] = s.b[l + 1];
    a.bias_o = s.b[s.n_hidden];
    const int ncb = pairs_per_wave == 32 ? 2 : 4;
    const int per_block = 64 * ncb;
    a.tiles_per_query = (s.n + per_block - 1) / per_block;
    a.n_tiles = a.tiles_per_query * B;
    if (!a.n_tiles) return;
    const int blocks = std::min(a.n_tiles, n_compute_units() * resident_blocks(ncb));
    if (ncb == 2)
        mlp_bf16_kernel<2><<<blocks, 256, 0, st>>>(a);
    else
        mlp_bf16_kernel<4><<<blocks, 256, 0, st>>>(a);
}

}  // namespace swf
