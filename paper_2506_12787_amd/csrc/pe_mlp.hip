// Positional encoding, FP32 deformation MLP with the fused deform + preprocess
// epilogue, and the static (no-MLP) preprocess.
//
// Deformation MLP (Sec. 4.2): residuals = F_theta(gamma(mu_hat), gamma(s_hat)).
// Layer 1 is split: its transceiver part W1s gamma(s_hat) + b1 is the same for
// every Gaussian of a query and is computed once per query (tx_features); its
// mean part W1m gamma(mu_hat) (K = 26) runs per row. Every later layer is a
// dense 256 x 256 contraction over the rows of the block.
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

constexpr int kR = 32;          // rows per block
constexpr int kHid = 256;       // hidden width
constexpr int kKS = 32;         // k rows per weight slab
constexpr int kActStride = 260; // padded row stride of the activation tile

// FP32 MLP over kR rows per block; 256 threads; thread (tr, tc) owns rows
// tr*4..tr*4+3 and columns tc*8..tc*8+7 of each hidden layer.
__global__ __launch_bounds__(256, 2) void mlp_fp32_kernel(MlpArgs a) {
    __shared__ __attribute__((aligned(16))) float act[kR * kActStride];
    __shared__ __attribute__((aligned(16))) float ws[kKS * kHid];
    __shared__ float xin[kR][kMeanFeat + 2];
    __shared__ float outv[kR][8];

    const int tid = threadIdx.x;
    const int tr = tid >> 5, tc = tid & 31;
    const size_t total = (size_t)a.N * a.B;
    const size_t row0 = (size_t)blockIdx.x * kR;

    // mean features of the block's rows, and the layer-1 mean weights into ws
    if (tid < kR) {
        const size_t row = row0 + tid;
        float f[kMeanFeat];
        if (row < total) {
            const int p = (int)(row % a.N);
            mean_features(a.mx[p], a.my[p], a.sW, a.sH, f);
        } else {
#pragma unroll
            for (int k = 0; k < kMeanFeat; ++k) f[k] = 0.f;
        }
#pragma unroll
        for (int k = 0; k < kMeanFeat; ++k) xin[tid][k] = f[k];
    }
    for (int i = tid; i < kMeanFeat * kHid; i += 256) ws[i] = a.w1m_t[i];
    __syncthreads();

    float acc[4][8];
    // layer 1: relu(qs[b] + W1m x_mean)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const size_t row = row0 + tr * 4 + i;
        const int b = row < total ? (int)(row / a.N) : 0;
        const float4* q4 = reinterpret_cast<const float4*>(a.qs + (size_t)b * kHid + tc * 8);
        const float4 q0 = q4[0], q1 = q4[1];
        acc[i][0] = q0.x; acc[i][1] = q0.y; acc[i][2] = q0.z; acc[i][3] = q0.w;
        acc[i][4] = q1.x; acc[i][5] = q1.y; acc[i][6] = q1.z; acc[i][7] = q1.w;
    }
    for (int k = 0; k < kMeanFeat; ++k) {
        const float4 w0 = *reinterpret_cast<const float4*>(&ws[k * kHid + tc * 8]);
        const float4 w1 = *reinterpret_cast<const float4*>(&ws[k * kHid + tc * 8 + 4]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float x = xin[tr * 4 + i][k];
            acc[i][0] = fmaf(x, w0.x, acc[i][0]); acc[i][1] = fmaf(x, w0.y, acc[i][1]);
            acc[i][2] = fmaf(x, w0.z, acc[i][2]); acc[i][3] = fmaf(x, w0.w, acc[i][3]);
            acc[i][4] = fmaf(x, w1.x, acc[i][4]); acc[i][5] = fmaf(x, w1.y, acc[i][5]);
            acc[i][6] = fmaf(x, w1.z, acc[i][6]); acc[i][7] = fmaf(x, w1.w, acc[i][7]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float4* dst = reinterpret_cast<float4*>(&act[(tr * 4 + i) * kActStride + tc * 8]);
        dst[0] = make_float4(fmaxf(acc[i][0], 0.f), fmaxf(acc[i][1], 0.f), fmaxf(acc[i][2], 0.f), fmaxf(acc[i][3], 0.f));
        dst[1] = make_float4(fmaxf(acc[i][4], 0.f), fmaxf(acc[i][5], 0.f), fmaxf(acc[i][6], 0.f), fmaxf(acc[i][7], 0.f));
        const size_t row = row0 + tr * 4 + i;
        if (a.act_out[0] && row < total) {
            float4* g = reinterpret_cast<float4*>(a.act_out[0] + row * kHid + tc * 8);
            g[0] = dst[0];
            g[1] = dst[1];
        }
    }

    // hidden -> hidden layers; weights streamed through ws in kKS-row slabs
    constexpr int kSlabs = kHid / kKS;
    constexpr int kPf = kKS * kHid / 4 / 256;  // float4 per thread per slab (8)
    float4 pf[kPf];
    for (int l = 0; l < a.n_mid; ++l) {
        const float4* wsrc = reinterpret_cast<const float4*>(a.wh_t[l]);
#pragma unroll
        for (int j = 0; j < kPf; ++j) pf[j] = wsrc[tid + j * 256];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4* b4 = reinterpret_cast<const float4*>(a.bh[l] + tc * 8);
            const float4 b0 = b4[0], b1 = b4[1];
            acc[i][0] = b0.x; acc[i][1] = b0.y; acc[i][2] = b0.z; acc[i][3] = b0.w;
            acc[i][4] = b1.x; acc[i][5] = b1.y; acc[i][6] = b1.z; acc[i][7] = b1.w;
        }
        for (int sl = 0; sl < kSlabs; ++sl) {
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kPf; ++j) reinterpret_cast<float4*>(ws)[tid + j * 256] = pf[j];
            __syncthreads();
            if (sl + 1 < kSlabs) {
                const float4* nsrc = wsrc + (size_t)(sl + 1) * (kKS * kHid / 4);
#pragma unroll
                for (int j = 0; j < kPf; ++j) pf[j] = nsrc[tid + j * 256];
            }
            const int kb = sl * kKS;
#pragma unroll 2
            for (int kk = 0; kk < kKS; kk += 4) {
                float4 av[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    av[i] = *reinterpret_cast<const float4*>(&act[(tr * 4 + i) * kActStride + kb + kk]);
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) {
                    const float4 w0 = *reinterpret_cast<const float4*>(&ws[(kk + k4) * kHid + tc * 8]);
                    const float4 w1 = *reinterpret_cast<const float4*>(&ws[(kk + k4) * kHid + tc * 8 + 4]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float x = k4 == 0 ? av[i].x : (k4 == 1 ? av[i].y : (k4 == 2 ? av[i].z : av[i].w));
                        acc[i][0] = fmaf(x, w0.x, acc[i][0]); acc[i][1] = fmaf(x, w0.y, acc[i][1]);
                        acc[i][2] = fmaf(x, w0.z, acc[i][2]); acc[i][3] = fmaf(x, w0.w, acc[i][3]);
                        acc[i][4] = fmaf(x, w1.x, acc[i][4]); acc[i][5] = fmaf(x, w1.y, acc[i][5]);
                        acc[i][6] = fmaf(x, w1.z, acc[i][6]); acc[i][7] = fmaf(x, w1.w, acc[i][7]);
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float4* dst = reinterpret_cast<float4*>(&act[(tr * 4 + i) * kActStride + tc * 8]);
            dst[0] = make_float4(fmaxf(acc[i][0], 0.f), fmaxf(acc[i][1], 0.f), fmaxf(acc[i][2], 0.f), fmaxf(acc[i][3], 0.f));
            dst[1] = make_float4(fmaxf(acc[i][4], 0.f), fmaxf(acc[i][5], 0.f), fmaxf(acc[i][6], 0.f), fmaxf(acc[i][7], 0.f));
            const size_t row = row0 + tr * 4 + i;
            if (a.act_out[l + 1] && row < total) {
                float4* g = reinterpret_cast<float4*>(a.act_out[l + 1] + row * kHid + tc * 8);
                g[0] = dst[0];
                g[1] = dst[1];
            }
        }
    }
    // output layer: 7 dot products of length 256 per row
    __syncthreads();
    for (int i = tid; i < kHid * kOut; i += 256) ws[i] = a.wo_t[i];
    __syncthreads();
    if (tid < kR * kOut) {
        const int r = tid / kOut, o = tid % kOut;
        float s = a.bo[o];
        for (int k = 0; k < kHid; ++k) s = fmaf(act[r * kActStride + k], ws[k * kOut + o], s);
        outv[r][o] = s;
    }
    __syncthreads();
    if (tid < kR) {
        const size_t row = row0 + tid;
        if (row < total) deform_epilogue(a, row, (int)(row % a.N), outv[tid]);
    }
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
    const unsigned blocks = (unsigned)((total + kR - 1) / kR);
    if (blocks) mlp_fp32_kernel<<<blocks, 256, 0, st>>>(a);
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

}  // namespace swf
