// FP32 GEMM on the matrix cores for the MLP backward (the differentiated
// layers of the deformation network, Sec. 4.2): C = op(A) op(B) over row-major
// matrices, op(A) M x K and op(B) K x N, FP32 products and FP32 sums
// (v_mfma_f32_16x16x4_f32). The operands are FP32, or BF16 bits widened on
// load (a product of two BF16 values is exact in FP32, so this equals a BF16
// product with FP32 accumulation). Optional epilogue: C *= [mask > 0] (the
// ReLU derivative of the layer below).
//
// Block tile 128 x 128 for large products, 64 x 64 for small ones, 128 x 32
// when C has at most 32 columns (so no wave computes padding only); four waves
// per block; K in steps of 32 staged through LDS (double-buffered, one barrier
// per step). Every operand layout is loaded along its contiguous dimension, four
// elements per thread and run (one 16-byte load where the run is aligned and
// inside the matrix). Products with a small C and a long K (weight gradients:
// K = pairs or Gaussians) are cut into K-slices whose partial products are
// summed afterwards in a fixed order, so every result is the same from run to
// run.
#include <algorithm>

#include "kernels.h"

namespace swf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kGK = 32;  // K per LDS stage

struct GemmArgs {
    const void* A;
    const void* B;
    float* C;           // result (one slice) or the slices' partial products
    const float* mask;  // C *= [mask > 0] (one slice only), or null
    int64_t M, N, K, lda, ldb, ldc, ldm;
    int64_t kc;         // K per slice (blockIdx.z)
    int a_kc, b_kc;     // operand contiguous along K (else along M / N)
    int a_vec, b_vec;   // FP32 operand whose runs of 4 are 16-byte aligned (ld % 4 == 0, aligned base)
    int c_vec;          // the result (and mask) rows take 16-byte stores (loads) at multiples of 4
    int tc;             // store the transpose: C[n * ldc + m] (no mask)
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

// The elements this thread stages of an O (outer: M or N) x 32 (K) operand
// tile starting at (o0, k0): O / 32 runs of 4 along the contiguous dimension,
// run u = 256 r + t of the tile's 8 O runs; zero outside olim / klim.
// kcontig: element (o, k) at p[o * ld + k], run u covers o = u / 8,
// k = 4 (u % 8) + 0..3; else element (o, k) at p[k * ld + o], run u covers
// k = u / (O / 4), o = 4 (u % (O / 4)) + 0..3. A run inside the matrix is one
// 16-byte load when the operand allows it.
template <bool kBf, int O>
__device__ __forceinline__ void tile_load(const void* p, int64_t ld, bool kcontig, bool vec, int64_t o0,
                                          int64_t olim, int64_t k0, int64_t klim, float (&v)[O / 8]) {
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int r = 0; r < O / 32; ++r) {
        const int u = 256 * r + t;
        const int o = kcontig ? u >> 3 : 4 * (u % (O / 4));
        const int k = kcontig ? 4 * (u & 7) : u / (O / 4);
        const int64_t go = o0 + o, gk = k0 + k;
        const bool whole = kcontig ? (go < olim && gk + 3 < klim) : (gk < klim && go + 3 < olim);
        const int64_t at = kcontig ? go * ld + gk : gk * ld + go;
        if (!kBf && vec && whole) {
            const float4 f = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(p) + at);
            v[4 * r] = f.x;
            v[4 * r + 1] = f.y;
            v[4 * r + 2] = f.z;
            v[4 * r + 3] = f.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in = kcontig ? (go < olim && gk + j < klim) : (gk < klim && go + j < olim);
                v[4 * r + j] = in ? elem<kBf>(p, at + j) : 0.0f;
            }
        }
    }
}

template <int O>
__device__ __forceinline__ void tile_store(float (*s)[O + 16], bool kcontig, const float (&v)[O / 8]) {
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int r = 0; r < O / 32; ++r) {
        const int u = 256 * r + t;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = kcontig ? u >> 3 : 4 * (u % (O / 4)) + j;
            const int k = kcontig ? 4 * (u & 7) + j : u / (O / 4);
            s[k][o] = v[4 * r + j];
        }
    }
}

// Block tile TM x TN: 128 x 128 (2 x 2 waves of 64 x 64), 64 x 64 (2 x 2
// waves of 32 x 32) or 128 x 32 for a narrow C (4 x 1 waves of 32 x 32); a
// wave's tile is I x J instructions of 16 x 16. LDS rows are padded by 16
// floats, so the 4 k-rows one read touches land on disjoint banks.
template <bool kBf, int TM, int TN>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs g) {
    constexpr int kWM = TN == 32 ? 4 : 2, kWN = 4 / kWM;  // waves along M and N
    constexpr int I = TM / kWM / 16, J = TN / kWN / 16;   // 16 x 16 instructions per wave along M and N
    // the K stages, and after the last one the block's C tile (rows padded by 4 floats)
    constexpr int kAs = 2 * kGK * (TM + 16), kBs = 2 * kGK * (TN + 16), kCs = TM * (TN + 4);
    __shared__ __attribute__((aligned(16))) float smem[kAs + kBs > kCs ? kAs + kBs : kCs];
    auto As = reinterpret_cast<float (*)[kGK][TM + 16]>(smem);
    auto Bs = reinterpret_cast<float (*)[kGK][TN + 16]>(smem + kAs);
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int wm = wave % kWM, wn = wave / kWM;
    const int64_t m0 = (int64_t)blockIdx.x * TM, n0 = (int64_t)blockIdx.y * TN;
    const int64_t kb = (int64_t)blockIdx.z * g.kc;
    const int64_t ke = g.K < kb + g.kc ? g.K : kb + g.kc;
    const int steps = ke > kb ? (int)((ke - kb + kGK - 1) / kGK) : 0;
    const bool akc = g.a_kc != 0, bkc = g.b_kc != 0;
    const bool avec = g.a_vec != 0, bvec = g.b_vec != 0;

    f32x4 acc[I][J];
#pragma unroll
    for (int i = 0; i < I; ++i)
#pragma unroll
        for (int j = 0; j < J; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    float va[TM / 8], vb[TN / 8];
    if (steps > 0) {
        tile_load<kBf, TM>(g.A, g.lda, akc, avec, m0, g.M, kb, ke, va);
        tile_load<kBf, TN>(g.B, g.ldb, bkc, bvec, n0, g.N, kb, ke, vb);
        tile_store<TM>(As[0], akc, va);
        tile_store<TN>(Bs[0], bkc, vb);
    }
    __syncthreads();
    for (int s = 0; s < steps; ++s) {
        const int cur = s & 1;
        const bool more = s + 1 < steps;
        if (more) {
            const int64_t k1 = kb + (int64_t)(s + 1) * kGK;
            tile_load<kBf, TM>(g.A, g.lda, akc, avec, m0, g.M, k1, ke, va);
            tile_load<kBf, TN>(g.B, g.ldb, bkc, bvec, n0, g.N, k1, ke, vb);
        }
#pragma unroll
        for (int q = 0; q < kGK / 4; ++q) {
            const int kr = 4 * q + (lane >> 4);
            float a[I], b[J];
#pragma unroll
            for (int i = 0; i < I; ++i) a[i] = As[cur][kr][wm * 16 * I + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < J; ++j) b[j] = Bs[cur][kr][wn * 16 * J + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < I; ++i)
#pragma unroll
                for (int j = 0; j < J; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) {
            tile_store<TM>(As[cur ^ 1], akc, va);
            tile_store<TN>(Bs[cur ^ 1], bkc, vb);
        }
        __syncthreads();
    }
    // lane l holds rows 4 (l / 16) + r, column l % 16 of each 16 x 16 result: staged in LDS (every read of the
    // K stages ended at the last barrier), then written out row by row, 4 consecutive elements per thread, the
    // mask read the same way
    auto Cs = reinterpret_cast<float (*)[TN + 4]>(smem);
#pragma unroll
    for (int i = 0; i < I; ++i)
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Cs[wm * 16 * I + i * 16 + 4 * (lane >> 4) + r][wn * 16 * J + j * 16 + (lane & 15)] = acc[i][j][r];
    __syncthreads();
    const bool split = gridDim.z > 1;
    float* __restrict__ C = split ? g.C + (size_t)blockIdx.z * (size_t)(g.M * g.N) : g.C;
    const float* __restrict__ mk = split ? nullptr : g.mask;
    const int64_t ldc = split ? g.N : g.ldc;
    const bool vec = g.c_vec != 0;
    if (g.tc && !split) {
        // C^T: element (m, n) at C[n * ldc + m]; runs of 4 along m
        for (int e = (int)threadIdx.x; e < TM * TN / 4; e += 256) {
            const int col = e / (TM / 4), r4 = (e % (TM / 4)) * 4;
            const int64_t n = n0 + col, m = m0 + r4;
            if (n >= g.N || m >= g.M) continue;
            const float v[4] = {Cs[r4][col], Cs[r4 + 1][col], Cs[r4 + 2][col], Cs[r4 + 3][col]};
            if (vec && m + 3 < g.M) {
                *reinterpret_cast<float4*>(C + n * ldc + m) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (m + q < g.M) C[n * ldc + m + q] = v[q];
            }
        }
        return;
    }
    for (int e = (int)threadIdx.x; e < TM * TN / 4; e += 256) {
        const int row = e / (TN / 4), c4 = (e % (TN / 4)) * 4;
        const int64_t m = m0 + row, n = n0 + c4;
        if (m >= g.M || n >= g.N) continue;
        float4 v = *reinterpret_cast<const float4*>(&Cs[row][c4]);
        if (vec && n + 3 < g.N) {
            if (mk) {
                const float4 f = *reinterpret_cast<const float4*>(mk + m * g.ldm + n);
                v.x = f.x > 0.0f ? v.x : 0.0f;
                v.y = f.y > 0.0f ? v.y : 0.0f;
                v.z = f.z > 0.0f ? v.z : 0.0f;
                v.w = f.w > 0.0f ? v.w : 0.0f;
            }
            *reinterpret_cast<float4*>(C + m * ldc + n) = v;
        } else {
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (n + q < g.N) C[m * ldc + n + q] = (mk && !(mk[m * g.ldm + n + q] > 0.0f)) ? 0.0f : vv[q];
        }
    }
}

// C[m][n] (ld ldc; tc: C[n][m]) = sum over the slices of part[z][m][n], then
// the mask. A block takes 64 consecutive outputs; thread group w (of 4) sums
// the slices z = w, w + 4, ... in order, and the four partial sums are added
// in the order w = 0..3, so the result does not depend on the launch.
__global__ __launch_bounds__(256) void gemm_reduce_kernel(const float* __restrict__ part, int sp, int64_t M,
                                                          int64_t N, float* __restrict__ C, int64_t ldc,
                                                          const float* __restrict__ mask, int64_t ldm, int tc) {
    __shared__ float red[4][64];
    const int64_t i = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const int w = (int)(threadIdx.x >> 6);
    const size_t plane = (size_t)(M * N);
    float s = 0.0f;
    if (i < M * N)
        for (int z = w; z < sp; z += 4) s += part[(size_t)z * plane + i];
    red[w][threadIdx.x & 63] = s;
    __syncthreads();
    if (w == 0 && i < M * N) {
        const int c = (int)threadIdx.x;
        float v = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
        const int64_t m = i / N, n = i - m * N;
        if (mask && !(mask[m * ldm + n] > 0.0f)) v = 0.0f;
        C[tc ? n * ldc + m : m * ldc + n] = v;
    }
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool narrow(int64_t N) { return N <= 32; }               // the 128 x 32 tile
bool wide(int64_t M, int64_t N) { return M >= 128 && N >= 128; }  // the 128 x 128 tile

}  // namespace

int gemm_split(int64_t M, int64_t N, int64_t K) {
    const int64_t tiles = narrow(N)    ? cdiv(M, 128) * cdiv(N, 32)
                          : wide(M, N) ? cdiv(M, 128) * cdiv(N, 128)
                                       : cdiv(M, 64) * cdiv(N, 64);
    // enough blocks to cover the chip a few times, each slice at least 256 deep
    const int64_t want = cdiv(2048, tiles), deep = K / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(256, std::min(want, deep)));
}

size_t gemm_part_floats(int64_t M, int64_t N, int64_t K) {
    // either orientation (a product with few rows may run as its transpose)
    const int sp = std::max(gemm_split(M, N, K), gemm_split(N, M, K));
    return sp > 1 ? (size_t)sp * (size_t)(M * N) : 0;
}

void launch_gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                     int64_t ldb, float* C, int64_t ldc, float* part, hipStream_t st, const float* mask, int64_t ldm,
                     bool bf16) {
    if (M <= 0 || N <= 0) return;
    // a product with few rows and many columns (without a mask) runs as its transpose, C^T = op(B)^T op(A)^T,
    // on the narrow tile, and stores the transpose back
    const bool tc = M <= 32 && N > 32 && !mask;
    if (tc) {
        std::swap(M, N);
        std::swap(A, B);
        std::swap(lda, ldb);
        const bool t = ta;
        ta = !tb;
        tb = !t;
    }
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
    g.a_vec = !bf16 && lda % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
    g.b_vec = !bf16 && ldb % 4 == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
    g.tc = tc ? 1 : 0;
    // 16-byte rows of the result: the destination of this launch (the slices' partials, or C) and the mask
    const bool c_al = slices > 1 ? (N % 4 == 0 && (reinterpret_cast<uintptr_t>(part) & 15) == 0)
                                 : (ldc % 4 == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0);
    const bool m_al = !mask || (ldm % 4 == 0 && (reinterpret_cast<uintptr_t>(mask) & 15) == 0);
    g.c_vec = c_al && m_al ? 1 : 0;
    if (narrow(N)) {
        const dim3 grid((unsigned)cdiv(M, 128), (unsigned)cdiv(N, 32), (unsigned)slices);
        if (bf16)
            gemm_f32_kernel<true, 128, 32><<<grid, 256, 0, st>>>(g);
        else
            gemm_f32_kernel<false, 128, 32><<<grid, 256, 0, st>>>(g);
    } else if (wide(M, N)) {
        const dim3 grid((unsigned)cdiv(M, 128), (unsigned)cdiv(N, 128), (unsigned)slices);
        if (bf16)
            gemm_f32_kernel<true, 128, 128><<<grid, 256, 0, st>>>(g);
        else
            gemm_f32_kernel<false, 128, 128><<<grid, 256, 0, st>>>(g);
    } else {
        const dim3 grid((unsigned)cdiv(M, 64), (unsigned)cdiv(N, 64), (unsigned)slices);
        if (bf16)
            gemm_f32_kernel<true, 64, 64><<<grid, 256, 0, st>>>(g);
        else
            gemm_f32_kernel<false, 64, 64><<<grid, 256, 0, st>>>(g);
    }
    if (slices > 1)
        gemm_reduce_kernel<<<(unsigned)cdiv(M * N, 64), 256, 0, st>>>(part, slices, M, N, C, ldc, mask, ldm,
                                                                      tc ? 1 : 0);
}

}  // namespace swf
