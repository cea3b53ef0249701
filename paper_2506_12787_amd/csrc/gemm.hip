// FP32 GEMM on the matrix cores for the MLP backward (the differentiated
// layers of the deformation network, Sec. 4.2): C = op(A) op(B) over row-major
// matrices, op(A) M x K and op(B) K x N, FP32 products and FP32 sums
// (v_mfma_f32_16x16x4_f32). The operands are FP32, or BF16 bits widened on
// load (a product of two BF16 values is exact in FP32, so this equals a BF16
// product with FP32 accumulation). Optional epilogue: C *= [mask > 0] (the
// ReLU derivative of the layer below).
//
// Block tile 64 x 64, K in steps of 16 staged through LDS (double-buffered,
// one barrier per step); four waves of 32 x 32 = 2 x 2 instructions of
// 16 x 16. Every operand layout is loaded along its contiguous dimension.
// Products with a small C and a long K (weight gradients: K = pairs) are cut
// into K-slices whose partial products are summed afterwards in slice order,
// so every result is the same from run to run.
#include <algorithm>

#include "kernels.h"

namespace swf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kGT = 64;        // block tile (M and N)
constexpr int kGK = 16;        // K per LDS stage
constexpr int kGLd = kGT + 16; // LDS row stride: the 4 k-rows of one read land on disjoint banks

struct GemmArgs {
    const void* A;
    const void* B;
    float* C;           // result (one slice) or the slices' partial products
    const float* mask;  // C *= [mask > 0] (one slice only), or null
    int64_t M, N, K, lda, ldb, ldc, ldm;
    int64_t kc;         // K per slice (blockIdx.z)
    int a_kc, b_kc;     // operand contiguous along K (else along M / N)
};

template <bool kBf>
__device__ __forceinline__ float elem(const void* p, int64_t i) {
    if constexpr (kBf) {
        const uint32_t bits = (uint32_t)reinterpret_cast<const uint16_t*>(p)[i] << 16;
        return __uint_as_float(bits);
    } else {
        return reinterpret_cast<const float*>(p)[i];
    }
}

// The 4 elements this thread stages of a 64 (outer: M or N) x 16 (K) operand
// tile starting at (o0, k0); zero outside olim / klim. kcontig: element
// (o, k) at p[o * ld + k], else at p[k * ld + o].
template <bool kBf>
__device__ __forceinline__ void tile_load(const void* p, int64_t ld, bool kcontig, int64_t o0, int64_t olim,
                                          int64_t k0, int64_t klim, float (&v)[4]) {
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int o = kcontig ? t >> 2 : (t & 15) * 4 + j;
        const int k = kcontig ? (t & 3) * 4 + j : t >> 4;
        const int64_t go = o0 + o, gk = k0 + k;
        v[j] = (go < olim && gk < klim) ? elem<kBf>(p, kcontig ? go * ld + gk : gk * ld + go) : 0.0f;
    }
}

__device__ __forceinline__ void tile_store(float (*s)[kGLd], bool kcontig, const float (&v)[4]) {
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int o = kcontig ? t >> 2 : (t & 15) * 4 + j;
        const int k = kcontig ? (t & 3) * 4 + j : t >> 4;
        s[k][o] = v[j];
    }
}

template <bool kBf>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs g) {
    __shared__ float As[2][kGK][kGLd];
    __shared__ float Bs[2][kGK][kGLd];
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.x * kGT, n0 = (int64_t)blockIdx.y * kGT;
    const int64_t kb = (int64_t)blockIdx.z * g.kc;
    const int64_t ke = g.K < kb + g.kc ? g.K : kb + g.kc;
    const int steps = ke > kb ? (int)((ke - kb + kGK - 1) / kGK) : 0;
    const bool akc = g.a_kc != 0, bkc = g.b_kc != 0;

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    float va[4], vb[4];
    if (steps > 0) {
        tile_load<kBf>(g.A, g.lda, akc, m0, g.M, kb, ke, va);
        tile_load<kBf>(g.B, g.ldb, bkc, n0, g.N, kb, ke, vb);
        tile_store(As[0], akc, va);
        tile_store(Bs[0], bkc, vb);
    }
    __syncthreads();
    for (int s = 0; s < steps; ++s) {
        const int cur = s & 1;
        const bool more = s + 1 < steps;
        if (more) {
            const int64_t k1 = kb + (int64_t)(s + 1) * kGK;
            tile_load<kBf>(g.A, g.lda, akc, m0, g.M, k1, ke, va);
            tile_load<kBf>(g.B, g.ldb, bkc, n0, g.N, k1, ke, vb);
        }
#pragma unroll
        for (int q = 0; q < kGK / 4; ++q) {
            const int kr = 4 * q + (lane >> 4);
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[cur][kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[cur][kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
            tile_store(As[cur ^ 1], akc, va);
            tile_store(Bs[cur ^ 1], bkc, vb);
        }
        __syncthreads();
    }
    // lane l holds rows 4 (l / 16) + r, column l % 16 of each 16 x 16 result
    const bool split = gridDim.z > 1;
    float* C = split ? g.C + (size_t)blockIdx.z * (size_t)(g.M * g.N) : g.C;
    const int64_t ldc = split ? g.N : g.ldc;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t n = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                if (m < g.M && n < g.N) {
                    float v = acc[i][j][r];
                    if (!split && g.mask && !(g.mask[m * g.ldm + n] > 0.0f)) v = 0.0f;
                    C[m * ldc + n] = v;
                }
            }
        }
}

// C[m][n] (ld ldc) = sum over the slices, in slice order, of part[z][m][n]; then the mask
__global__ __launch_bounds__(256) void gemm_reduce_kernel(const float* __restrict__ part, int sp, int64_t M,
                                                          int64_t N, float* __restrict__ C, int64_t ldc,
                                                          const float* __restrict__ mask, int64_t ldm) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M * N) return;
    float s = 0.0f;
    for (int z = 0; z < sp; ++z) s += part[(size_t)z * (size_t)(M * N) + i];
    const int64_t m = i / N, n = i - m * N;
    if (mask && !(mask[m * ldm + n] > 0.0f)) s = 0.0f;
    C[m * ldc + n] = s;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

int gemm_split(int64_t M, int64_t N, int64_t K) {
    const int64_t tiles = cdiv(M, kGT) * cdiv(N, kGT);
    // enough blocks to cover the chip a few times, each slice at least 2048 deep
    const int64_t want = cdiv(2048, tiles), deep = K / 2048;
    return (int)std::max<int64_t>(1, std::min<int64_t>(64, std::min(want, deep)));
}

size_t gemm_part_floats(int64_t M, int64_t N, int64_t K) {
    const int sp = gemm_split(M, N, K);
    return sp > 1 ? (size_t)sp * (size_t)(M * N) : 0;
}

void launch_gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                     int64_t ldb, float* C, int64_t ldc, float* part, hipStream_t st, const float* mask, int64_t ldm,
                     bool bf16) {
    if (M <= 0 || N <= 0) return;
    const int sp = gemm_split(M, N, K);
    const int64_t kc = sp > 1 ? cdiv(cdiv(K, sp), kGK) * kGK : std::max<int64_t>(K, 1);
    const int slices = sp > 1 ? (int)cdiv(K, kc) : 1;  // at most sp
    GemmArgs g;
    g.A = A;
    g.B = B;
    g.C = slices > 1 ? part : C;
    g.mask = mask;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = lda;
    g.ldb = ldb;
    g.ldc = ldc;
    g.ldm = ldm;
    g.kc = kc;
    // op(A) = A (M x K) is contiguous along K; op(A) = A^T (A stored K x M) along M. op(B) = B (K x N) is
    // contiguous along N, B^T (B stored N x K) along K.
    g.a_kc = ta ? 0 : 1;
    g.b_kc = tb ? 1 : 0;
    const dim3 grid((unsigned)cdiv(M, kGT), (unsigned)cdiv(N, kGT), (unsigned)slices);
    if (bf16)
        gemm_f32_kernel<true><<<grid, 256, 0, st>>>(g);
    else
        gemm_f32_kernel<false><<<grid, 256, 0, st>>>(g);
    if (slices > 1)
        gemm_reduce_kernel<<<(unsigned)cdiv(M * N, 256), 256, 0, st>>>(part, slices, M, N, C, ldc, mask, ldm);
}

}  // namespace swf
