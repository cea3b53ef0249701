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
// A workgroup owns 384 pairs by default: 8 waves (two per SIMD, all 256
// VGPRs each) of 48 pairs, 3 column blocks of 16, so each weight fragment read
// from LDS feeds 3 MFMAs and each weight step copied into LDS serves 384 pairs.
// Both LDS traffic terms bound this kernel: 8 waves reading every fragment and
// the copies writing them. Variants: 8 waves of 32 pairs or 4 waves of 64
// (256-pair workgroups). Weight fragments (1 KiB each: 64 lanes x 8 bf16, in
// lane order) are streamed from a packed global buffer through a 3-slot LDS ring
// of 32-fragment steps with one barrier per step; the workgroups are persistent
// so the weight stream never drains between tiles.
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
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

typedef float f32x2 __attribute__((ext_vector_type(2)));

// One v_cvt_pk_bf16_f32 (round to nearest even). Written as a vector
// conversion: two scalar conversions would each take an instruction and a
// v_perm_b32 would then merge them.
__device__ __forceinline__ uint32_t cvt_pk_bf16(float a, float b) {
    const f32x2 f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}

constexpr int kUnitU4 = 1024;  // uint4 per 16 KiB unit of the weight stream
constexpr int kSlots = 3;
#ifndef SWF_PF_DEPTH
#define SWF_PF_DEPTH 2
#endif
constexpr int kDepth = SWF_PF_DEPTH;  // weight fragments read ahead of the MFMA using them (<= 8)

struct Bf16Args {
    MlpArgs m;
    const uint4* stream;      // packed weight chunks
    int n_steps;              // ring steps per tile: 2 + (128 / STEP) * (n_hidden - 1)
    const bf16x8* mfeat;      // [N][32] bf16 mean features (4 x bf16x8 per Gaussian)
    const float* bias_h[7];   // biases of hidden layers 1..n_hidden-1
    const float* bias_o;      // output bias
    int n_tiles;              // B * tiles_per_query
    int tiles_per_query;      // ceil(N / pairs per block): tiles never straddle two queries
    uint16_t* act_out;        // kAct: hidden activations (bf16 bits) [n_hidden][B * N][256]
    int64_t act_stride;       // elements per activation layer: B * N * 256
    MixBatch mix;             // kMix: the batch's scene and query tables (per tile: query, scene, stream, biases)
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

// One lane-contiguous 1 KiB piece per wave, global -> LDS without registers:
// lane l's 16 bytes land at lds_addr + 16 l. Written as inline assembly so the
// compiler does not treat every later LDS read as dependent on the copy (it
// would wait for the copy right after issuing it); completion is awaited
// explicitly with vmem_wait_all() before the barrier that publishes the slot.
__device__ __forceinline__ void dma_b128(const uint4* src, uint32_t lds_addr) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                 :
                 : "s"(__builtin_amdgcn_readfirstlane(lds_addr)), "v"(src)
                 : "memory", "m0");
}

// s_waitcnt vmcnt(0): every vector memory operation of this wave has completed.
__device__ __forceinline__ void vmem_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// NCB column blocks of 16 pairs per wave; WAVES waves per block; ring steps of
// STEP fragments; WPE waves per SIMD. kAct: also store every hidden activation
// (after the ReLU, in BF16, exactly the next layer's operand) row-major per
// pair, for the backward pass.
//
// Weight ring: kSlots LDS slots of one step each. The step q + 2 is
// copied global -> LDS directly (global_load_lds, no registers) at the start of
// step q into the slot read during step q - 1; each wave waits for its copies
// before the barrier ending step q, so the slot is complete from step q + 1 on.
// Fragment reads run kDepth fragments ahead, into the next slot past the end of a
// step.
//
// Hidden layers run output-tile-major: tile t (16 features) accumulates its
// 8 k-chunks, so accumulator pairs (2c', 2c'+1) are final early and their ReLU
// + bf16 conversion into the next layer's act[c'] is issued among the MFMAs of
// the following tile (one column block per two fragments) instead of after
// the layer; the last pair is converted during the next layer's first tile.
//
// kMix: the tiles belong to the queries of a mixed batch (per tile its query,
// scene, pair count, weight stream and biases from the batch's tables); the
// ring fetches each step from the stream of the tile it belongs to, and the
// next tile's biases are copied into the other half of a double buffer.
template <int NCB, int WAVES, int STEP, int WPE, bool kAct, bool kMix = false>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(WPE, WPE))) void
mlp_bf16_kernel(Bf16Args a) {
    typedef __attribute__((address_space(3))) void* lds_ptr;
    constexpr int kPairsPerWave = 16 * NCB;
    constexpr int kPairsPerBlock = WAVES * kPairsPerWave;
    static_assert(kPairsPerBlock % 64 == 0, "whole 64-pair groups per block");
    static_assert(STEP == 16 || STEP == 32, "ring steps of 16 or 32 fragments");
    constexpr int kStepU4 = STEP * 64;  // uint4 per ring slot
    __shared__ __attribute__((aligned(16))) uint4 ring[kSlots * kStepU4];
    __shared__ float outs[WAVES][kPairsPerWave][8];
    // Layer-1 TX term of the current and the next tile's query, hidden and
    // output biases: C operands read from LDS.
    __shared__ __attribute__((aligned(16))) float qs_s[2][256];
    constexpr int kBiasBufs = kMix ? 2 : 1;
    __shared__ __attribute__((aligned(16))) float bias_s[kBiasBufs][7][256];
    __shared__ __attribute__((aligned(16))) float bias_o_s[kBiasBufs][16];
    // Layer-1 B operand of the wave's pairs (bf16 gamma(mu_hat), lane order),
    // copied global -> LDS one tile ahead.
    __shared__ __attribute__((aligned(16))) uint4 bm_s[WAVES][NCB][64];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar registers
    const int lane = tid & 63;
    const int g = lane >> 4;       // lane group (k / feature sub-block)
    const int n16 = lane & 15;     // pair column inside a 16-wide block
    const int S = a.n_steps;
    const int n_mid = a.m.n_mid;

    // tiles of this persistent workgroup
    const int n_tiles = kMix ? a.mix.queries[a.mix.B].mlp_tile_base : a.n_tiles;
    const int my_tiles = n_tiles > (int)blockIdx.x ? (n_tiles - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
    if (my_tiles == 0) return;
    const int q_end = my_tiles * S;  // ring steps of this workgroup
    // query of a tile (block-uniform)
    auto tile_query = [&](int t) {
        if constexpr (kMix)
            return mix_find(a.mix.queries, a.mix.B, t, [](const MixQuery& x) { return x.mlp_tile_base; });
        else
            return t / a.tiles_per_query;
    };
    if (tid < 256) {
        const int q0 = tile_query((int)blockIdx.x);
        if constexpr (kMix) {
            const MixScene& s0 = a.mix.scenes[a.mix.queries[q0].scene];
            for (int l = 0; l < n_mid; ++l) bias_s[0][l][tid] = s0.bias_h[l][tid];
            if (tid < 16) bias_o_s[0][tid] = tid < kOut ? s0.bias_o[tid] : 0.0f;
        } else {
            for (int l = 0; l < n_mid; ++l) bias_s[0][l][tid] = a.bias_h[l][tid];
            if (tid < 16) bias_o_s[0][tid] = tid < kOut ? a.bias_o[tid] : 0.0f;
        }
        qs_s[0][tid] = a.m.qs[(size_t)q0 * 256 + tid];
    }
    // weight stream of the tile the ring is fetching for (kMix: it changes with the tile's scene)
    int fetch_it = 0;
    const uint4* fstream = a.stream;
    if constexpr (kMix) fstream = reinterpret_cast<const uint4*>(
        a.mix.scenes[a.mix.queries[tile_query((int)blockIdx.x)].scene].stream);

    int fetch = 0;  // stream step of the next copy
    const uint32_t ring_lds = (uint32_t)(uintptr_t)(lds_ptr)ring;  // LDS byte address of the ring
    // Step `fetch` of the stream: layer 1 (16 fragments) is step 0, the output
    // layer (8 fragments) step S - 1; only the fragments a step holds are copied.
    // Fragment i * WAVES + wave of the step is piece i of the wave.
#define SWF_DMA(slot_)                                                                                     \
    do {                                                                                                   \
        const int unit_ = STEP == 32 ? (fetch == 0 ? 0 : 2 * fetch - 1) : fetch;                           \
        const int nf_ = fetch == 0 ? 16 : (fetch == S - 1 ? 8 : STEP);                                    \
        const uint4* src_ = fstream + (size_t)unit_ * kUnitU4 + tid;                                       \
        const uint32_t dst_ = ring_lds + (uint32_t)((slot_) * STEP * 1024 + wave * 1024);                  \
        _Pragma("unroll") for (int i_ = 0; i_ < STEP / WAVES; ++i_)                                        \
            if (i_ * WAVES + wave < nf_) dma_b128(src_ + i_ * 64 * WAVES, dst_ + i_ * 1024 * WAVES);       \
        fetch = fetch + 1 == S ? 0 : fetch + 1;                                                            \
        if (kMix && fetch == 0) {                                                                          \
            ++fetch_it;                                                                                    \
            const int ft_ = (int)blockIdx.x + fetch_it * (int)gridDim.x;                                   \
            if (ft_ < n_tiles)                                                                             \
                fstream = reinterpret_cast<const uint4*>(                                                  \
                    a.mix.scenes[a.mix.queries[tile_query(ft_)].scene].stream);                            \
        }                                                                                                  \
    } while (0)
    // gamma(mu_hat) of the pairs of tile t_ into bm_s (rows past N read row
    // N - 1; layer 1 zeroes them); awaited by the wait before the next barrier.
    const uint32_t bm_lds = (uint32_t)(uintptr_t)(lds_ptr)&bm_s[wave][0][0];
#define SWF_FETCH_BM(tile_)                                                                              \
    do {                                                                                                 \
        const int t_ = (tile_);                                                                          \
        const int qy_ = tile_query(t_);                                                                  \
        int tb_ = qy_ * a.tiles_per_query, nq_ = a.m.N;                                                  \
        const bf16x8* mf_ = a.mfeat;                                                                     \
        if (kMix) {                                                                                      \
            const MixScene& sc_ = a.mix.scenes[a.mix.queries[qy_].scene];                                \
            tb_ = a.mix.queries[qy_].mlp_tile_base;                                                      \
            nq_ = sc_.N;                                                                                 \
            mf_ = reinterpret_cast<const bf16x8*>(sc_.mfeat);                                            \
        }                                                                                                \
        const int pp_ = (t_ - tb_) * kPairsPerBlock + wave * kPairsPerWave;                              \
        _Pragma("unroll") for (int cb = 0; cb < NCB; ++cb) {                                             \
            const int p_ = min(pp_ + cb * 16 + n16, nq_ - 1);                                            \
            dma_b128(reinterpret_cast<const uint4*>(mf_) + (size_t)p_ * 4 + g, bm_lds + cb * 1024);      \
        }                                                                                                \
    } while (0)
    SWF_FETCH_BM((int)blockIdx.x);
    SWF_DMA(0);
    if (q_end > 1) SWF_DMA(1);
    vmem_wait_all();
    __syncthreads();
    int q = 0;     // step being computed
    int slot = 0;  // q % 3
#define SWF_ADVANCE()                                         \
    do {                                                      \
        if (q + 2 < q_end) SWF_DMA(slot == 0 ? 2 : slot - 1); \
    } while (0)
#define SWF_FRAG_AT(s_, t_) __builtin_bit_cast(bf16x8, ring[(s_) * kStepU4 + (t_) * 64 + lane])
    // fragments f + 1 .. f + kDepth of the stream, read ahead
    bf16x8 wq[kDepth];
#pragma unroll
    for (int i = 0; i < kDepth; ++i) wq[i] = SWF_FRAG_AT(0, i);
#define SWF_TAKE(dst_, f_, nf_)                                                                          \
    do {                                                                                                 \
        dst_ = wq[0];                                                                                    \
        _Pragma("unroll") for (int i_ = 0; i_ + 1 < kDepth; ++i_) wq[i_] = wq[i_ + 1];                  \
        const int nxt_ = slot == 2 ? 0 : slot + 1;                                                       \
        wq[kDepth - 1] = (f_) + kDepth < (nf_) ? SWF_FRAG_AT(slot, (f_) + kDepth)                        \
                                                : SWF_FRAG_AT(nxt_, (f_) + kDepth - (nf_));              \
    } while (0)
#define SWF_NEXT_STEP()                  \
    do {                                 \
        vmem_wait_all();                 \
        __syncthreads();                 \
        ++q;                             \
        slot = slot == 2 ? 0 : slot + 1; \
    } while (0)
    // the empty asm pins the conversion where it is written (it would
    // otherwise be sunk next to its first use, after the MFMAs it should overlap).
    // lay_: index of the activation (0 = layer 1's output). With kAct the lane's
    // 8 values (features 32 cp + 4 g + 0..3 and 32 cp + 16 + 4 g + 0..3 of its
    // pair) are also stored.
#define SWF_PACK(dst_, cp_, cb_, lay_)                                                \
    do {                                                                              \
        u32x4 u_ = __builtin_bit_cast(u32x4, pack_relu(acc[2 * (cp_)][cb_], acc[2 * (cp_) + 1][cb_])); \
        asm volatile("" : "+v"(u_));                                                  \
        dst_[cp_][cb_] = __builtin_bit_cast(bf16x8, u_);                              \
        if (kAct) {                                                                   \
            const int pa_ = p0 + (cb_) * 16 + n16;                                    \
            if (pa_ < a.m.N) {                                                        \
                uint2* d_ = reinterpret_cast<uint2*>(a.act_out + (size_t)(lay_) * a.act_stride + \
                                                     (row0 + pa_) * 256 + 32 * (cp_) + 4 * g);  \
                d_[0] = make_uint2(u_.x, u_.y);                                       \
                d_[4] = make_uint2(u_.z, u_.w);                                       \
            }                                                                         \
        }                                                                             \
    } while (0)

    f32x4 acc[16][NCB];
    bf16x8 act[2][8][NCB];

    // One hidden layer, act[IN_] -> act[OUT_]: 16 output tiles x 8 k-chunks, t-major,
    // four ring steps. On entry the accumulator pair (14, 15) of the previous
    // layer is still unconverted; it becomes act[IN_][7] during tile 0.
#define SWF_HIDDEN(IN_, OUT_, L_)                                                                        \
    do {                                                                                                 \
        const float* bias_ = &bias_s[kMix ? (it & 1) : 0][(L_)][4 * g];                                  \
        _Pragma("unroll") for (int t = 0; t < 16; ++t) {                                                 \
            _Pragma("unroll") for (int c = 0; c < 8; ++c) {                                              \
                const int f = (t * 8 + c) % STEP;                                                        \
                if (f == 0) SWF_ADVANCE();                                                               \
                bf16x8 w;                                                                                \
                SWF_TAKE(w, f, STEP);                                                                    \
                if (c == 0) {                                                                            \
                    const float4 b4 = *reinterpret_cast<const float4*>(bias_ + 16 * t);                 \
                    const f32x4 c0 = {b4.x, b4.y, b4.z, b4.w};                                           \
                    _Pragma("unroll") for (int cb = 0; cb < NCB; ++cb) acc[t][cb] =                      \
                        mfma(w, act[IN_][c][cb], c0);                                                    \
                } else {                                                                                 \
                    _Pragma("unroll") for (int cb = 0; cb < NCB; ++cb) acc[t][cb] =                      \
                        mfma(w, act[IN_][c][cb], acc[t][cb]);                                            \
                }                                                                                        \
                if (t == 0 && c < NCB) SWF_PACK(act[IN_], 7, c, (L_));                                   \
                if (t >= 2 && (t & 1) == 0 && (c & 1) == 0 && c / 2 < NCB)                               \
                    SWF_PACK(act[OUT_], (t - 2) / 2, c / 2, (L_) + 1);                                   \
                __builtin_amdgcn_sched_barrier(0);                                                       \
                if (f == STEP - 1) SWF_NEXT_STEP();                                                      \
            }                                                                                            \
        }                                                                                                \
    } while (0)

    // Output layer from act[IN_] (one 16-row tile, 7 used, 8 k-chunks in one
    // ring step), transposed through LDS to one pair per lane.
#define SWF_OUTPUT(IN_)                                                                                  \
    do {                                                                                                 \
        SWF_ADVANCE();                                                                                   \
        f32x4 o[NCB];                                                                                    \
        const float4 b4 = *reinterpret_cast<const float4*>(&bias_o_s[kMix ? (it & 1) : 0][4 * g]);       \
        _Pragma("unroll") for (int cb = 0; cb < NCB; ++cb) o[cb] = f32x4{b4.x, b4.y, b4.z, b4.w};        \
        _Pragma("unroll") for (int c = 0; c < 8; ++c) {                                                  \
            bf16x8 w;                                                                                    \
            SWF_TAKE(w, c, 8);                                                                           \
            if (c < NCB) SWF_PACK(act[IN_], 7, c, n_mid);                                                \
            _Pragma("unroll") for (int cb = 0; cb < NCB; ++cb) o[cb] = mfma(w, act[IN_][c][cb], o[cb]);  \
            __builtin_amdgcn_sched_barrier(0);                                                           \
        }                                                                                                \
        if (g < 2) {                                                                                     \
            _Pragma("unroll") for (int cb = 0; cb < NCB; ++cb)                                           \
                _Pragma("unroll") for (int j = 0; j < 4; ++j) outs[wave][cb * 16 + n16][4 * g + j] =     \
                    o[cb][j];                                                                            \
        }                                                                                                \
    } while (0)

    for (int it = 0; it < my_tiles; ++it) {
        const int tile = (int)blockIdx.x + it * (int)gridDim.x;
        const int qry = tile_query(tile);                          // block-uniform query
        int Nq = a.m.N, tb = qry * a.tiles_per_query;              // its pairs and first tile
        size_t row0 = (size_t)qry * a.m.N;                         // first pair of the query
        if constexpr (kMix) {
            Nq = a.mix.scenes[a.mix.queries[qry].scene].N;
            tb = a.mix.queries[qry].mlp_tile_base;
            row0 = (size_t)a.mix.queries[qry].pair_base;
        }
        const int p0 = (tile - tb) * kPairsPerBlock + wave * kPairsPerWave;
        // ---- layer 1 (mean part, K = 32): B = bf16 gamma(mu_hat); C = TX term of the query ----
        bf16x8 bm[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int p = p0 + cb * 16 + n16;
            bm[cb] = p < Nq ? __builtin_bit_cast(bf16x8, bm_s[wave][cb][lane]) : bf16x8{};
        }
        SWF_ADVANCE();
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
                // pairs 0..6 as 7 * NCB (pair, column block) units, NCB / 2 per
                // fragment from t = 2 on; pair c' is final once t > 2c' + 1
                if (t >= 2)
#pragma unroll
                    for (int u = (t - 2) * NCB / 2; u < (t - 1) * NCB / 2; ++u)
                        SWF_PACK(act[0], u / NCB, u % NCB, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        SWF_NEXT_STEP();
        // the next tile's layer-1 operand (this wave's reads of bm_s are complete:
        // the MFMAs of layer 1 consumed them)
        if (it + 1 < my_tiles) SWF_FETCH_BM(tile + (int)gridDim.x);
        // TX term of the next tile's query, stored to LDS before this tile's
        // last barrier (the other buffer is read by this tile's layer 1 only)
        const int next_tile = tile + (int)gridDim.x;
        const float qs_next =
            it + 1 < my_tiles && tid < 256 ? a.m.qs[(size_t)tile_query(next_tile) * 256 + tid] : 0.0f;
        // ---- hidden layers, two per iteration so the act buffers alternate statically ----
        int l = 0;
        for (; l + 1 < n_mid; l += 2) {
            SWF_HIDDEN(0, 1, l);
            SWF_HIDDEN(1, 0, l + 1);
        }
        if (l < n_mid) {
            SWF_HIDDEN(0, 1, l);
            SWF_OUTPUT(1);
        } else {
            SWF_OUTPUT(0);
        }
        if (tid < 256) qs_s[(it + 1) & 1][tid] = qs_next;
        if constexpr (kMix) {
            // the next tile's biases into the other half of the double buffer (its previous reader, the tile
            // before this one, is done): hidden layers by wave, one 1 KiB piece each, global -> LDS, awaited
            // before the barrier below
            if (it + 1 < my_tiles) {
                const MixScene& sn = a.mix.scenes[a.mix.queries[tile_query(next_tile)].scene];
                const int nb = (it + 1) & 1;
                if (wave < n_mid)
                    dma_b128(reinterpret_cast<const uint4*>(sn.bias_h[wave]) + lane,
                             (uint32_t)(uintptr_t)(lds_ptr)&bias_s[nb][wave][0]);
                if (tid < 16) bias_o_s[nb][tid] = tid < kOut ? sn.bias_o[tid] : 0.0f;
            }
        }
        SWF_NEXT_STEP();
        if (lane < kPairsPerWave) {
            const int p = p0 + lane;
            if (p < Nq) {
                if constexpr (kMix)
                    mix_epilogue(a.mix.scenes[a.mix.queries[qry].scene], a.m, row0 + p, p, outs[wave][lane]);
                else
                    deform_epilogue(a.m, row0 + p, p, outs[wave][lane]);
            }
        }
        // `outs` is rewritten only after the next tile's first barrier
    }
#undef SWF_DMA
#undef SWF_ADVANCE
#undef SWF_FRAG_AT
#undef SWF_TAKE
#undef SWF_NEXT_STEP
#undef SWF_PACK
#undef SWF_HIDDEN
#undef SWF_OUTPUT
#undef SWF_FETCH_BM
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

}  // namespace

int n_compute_units() {
    static const int n = [] {  // thread-safe one-time initialisation
        int dev = 0, cus = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        return cus > 0 ? cus : 256;
    }();
    return n;
}

void compute_mean_features_bf16(DevScene& s, hipStream_t st) {
    if (s.n > 0)
        mean_features_bf16_kernel<<<(s.n + 255) / 256, 256, 0, st>>>(s.mx, s.my, s.n, s.W, s.H,
                                                                      reinterpret_cast<__bf16*>(s.bf_mfeat));
}

// One kernel variant: NCB column blocks of 16 pairs per wave, WAVES waves per
// workgroup, ring steps of STEP fragments, WPE waves per SIMD. The grid is
// persistent: as many workgroups as fit on the CUs at once (registers and LDS
// decide; launching more would only queue them).
template <int NCB, int WAVES, int STEP, int WPE, bool kAct = false>
void launch_variant(Bf16Args a, int n, int B, int n_hidden, hipStream_t st) {
    constexpr int kPerBlock = 16 * NCB * WAVES;
    static const int resident = [] {  // thread-safe one-time initialisation
        int r = 0;
        const hipError_t e =
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, mlp_bf16_kernel<NCB, WAVES, STEP, WPE, kAct>, 64 * WAVES, 0);
        return (e == hipSuccess && r > 0) ? r : 1;
    }();
    a.n_steps = 2 + (128 / STEP) * (n_hidden - 1);
    a.tiles_per_query = (n + kPerBlock - 1) / kPerBlock;
    a.n_tiles = a.tiles_per_query * B;
    if (!a.n_tiles) return;
    const int blocks = std::min(a.n_tiles, n_compute_units() * resident);
    mlp_bf16_kernel<NCB, WAVES, STEP, WPE, kAct><<<blocks, 64 * WAVES, 0, st>>>(a);
}

void launch_mix_mlp_bf16(const MixBatch& m, const float* qs, const Records& r, hipStream_t st, bool paper_mask,
                         bool wrap) {
    // the default variant (384-pair tiles, 8 waves of 48 pairs) over the batch's tiles; every scene of a mixed
    // batch has four hidden layers of 256
    constexpr int NCB = 3, WAVES = 8, STEP = 32, WPE = 2;
    static const int resident = [] {
        int rr = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &rr, mlp_bf16_kernel<NCB, WAVES, STEP, WPE, false, true>, 64 * WAVES, 0);
        return (e == hipSuccess && rr > 0) ? rr : 1;
    }();
    Bf16Args a{};
    a.m.rec = r;
    a.m.qs = qs;
    a.m.n_mid = 3;
    a.m.inv_tile = 1.0f / 16.0f;
    a.m.paper_mask = paper_mask ? 1 : 0;
    a.m.wrap = wrap ? 1 : 0;
    a.n_steps = 2 + (128 / STEP) * 3;
    a.mix = m;
    mlp_bf16_kernel<NCB, WAVES, STEP, WPE, false, true><<<n_compute_units() * resident, 64 * WAVES, 0, st>>>(a);
}

void launch_mlp_bf16(const DevScene& s, const float* qs, int B, const Grid& g, bool paper_mask, const Records& r,
                     float* delta_out, hipStream_t st, int pairs_per_wave, void* act_out) {
    Bf16Args a{};
    a.m = make_args(s, qs, B, g, paper_mask, r, delta_out);
    a.stream = reinterpret_cast<const uint4*>(s.bf_stream);
    a.mfeat = reinterpret_cast<const bf16x8*>(s.bf_mfeat);
    for (int l = 0; l + 1 < s.n_hidden && l < 7; ++l) a.bias_h[l] = s.b[l + 1];
    a.bias_o = s.b[s.n_hidden];
    if (act_out) {  // the default variant (every variant computes the same values)
        a.act_out = reinterpret_cast<uint16_t*>(act_out);
        a.act_stride = (int64_t)B * s.n * 256;
        launch_variant<3, 8, 32, 2, true>(a, s.n, B, s.n_hidden, st);
    } else if (pairs_per_wave == 64)
        launch_variant<4, 4, 32, 1>(a, s.n, B, s.n_hidden, st);  // 256 pairs, one wave per SIMD
    else if (pairs_per_wave == 32)
        launch_variant<2, 8, 32, 2>(a, s.n, B, s.n_hidden, st);  // 256 pairs, two waves per SIMD
    else
        launch_variant<3, 8, 32, 2>(a, s.n, B, s.n_hidden, st);  // default: 384 pairs, two waves per SIMD
}

}  // namespace swf
