// Device-side repacking of an updated deformation MLP whose new weights are
// already on the device (training): the in-major FP32 copies read by the FP32
// kernel and the BF16 weight stream of the MFMA kernel are rebuilt from the
// FP32 master copies where they live, on the caller's stream, with no host
// round trip. The layouts are those the upload builds on the host.
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

// float -> bfloat16 bits, round to nearest even (quiet NaN kept a NaN)
__device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// k index of element j of lane group g in k-chunk c of a hidden or output
// layer fragment: the order of the previous layer's output tiles in registers
__device__ __forceinline__ int frag_k(int c, int g, int j) { return 32 * c + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4)); }

struct PackArgs {
    const float* w[8];  // FP32 master weights, row-major [out][in]
    int n_hidden, in_dim, n_units;
    uint16_t* stream;   // n_units x 8192 BF16
    float* w1m_t;       // [26][256]
    float* wh_t[8];     // [256][256] per hidden->hidden layer
    float* wo_t;        // [256][7]
};

// One thread per element of the BF16 stream: unit 0 = layer 1 (mean part,
// 16 fragments, k = 8 g + j, K = 26 zero padded to 32); then 8 units per
// hidden->hidden layer (128 fragments, output-tile-major f = 8 t + c); the last
// unit = the output layer (8 fragments, rows 7..15 zero) and zero padding.
// Element (fragment f, lane l, j) sits at f * 512 + 8 l + j; row = 16 t + l % 16.
__global__ void pack_stream_kernel(PackArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)a.n_units * 8192) return;
    const int unit = (int)(e / 8192), r = (int)(e % 8192);
    const int f = r / 512, l = (r / 8) % 64, j = r % 8, g = l >> 4;
    float v = 0.0f;
    if (unit == 0) {
        const int row = 16 * f + (l & 15), k = 8 * g + j;
        if (k < kMeanFeat) v = a.w[0][(size_t)row * a.in_dim + k];
    } else if (unit < a.n_units - 1) {
        const int L = 1 + (unit - 1) / 8;
        const int ff = ((unit - 1) % 8) * 16 + f;  // fragment within the layer
        const int t = ff / 8, c = ff % 8;
        const int row = 16 * t + (l & 15);
        v = a.w[L][(size_t)row * 256 + frag_k(c, g, j)];
    } else if (f < 8) {
        const int o = l & 15;
        if (o < kOut) v = a.w[a.n_hidden][(size_t)o * 256 + frag_k(f, g, j)];
    }
    a.stream[e] = bf16_bits_rne(v);
}

// In-major FP32 copies: w1m_t[k][j] = W0[j][k] (k < 26), wh_t[L-1][k][j] =
// W_L[j][k], wo_t[k][o] = W_out[o][k]. blockIdx.y selects the matrix.
__global__ void pack_transpose_kernel(PackArgs a) {
    const int m = blockIdx.y;  // 0: layer-1 mean part, 1..n_hidden-1: hidden, n_hidden: output
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (m == 0) {
        if (e >= kMeanFeat * 256) return;
        const int k = e / 256, jj = e % 256;
        a.w1m_t[e] = a.w[0][(size_t)jj * a.in_dim + k];
    } else if (m < a.n_hidden) {
        if (e >= 256 * 256) return;
        const int k = e / 256, jj = e % 256;
        a.wh_t[m - 1][e] = a.w[m][(size_t)jj * 256 + k];
    } else {
        if (e >= 256 * kOut) return;
        const int k = e / kOut, o = e % kOut;
        a.wo_t[e] = a.w[a.n_hidden][(size_t)o * 256 + k];
    }
}

}  // namespace

void launch_pack_mlp(const DevScene& d, hipStream_t st) {
    PackArgs a{};
    for (int l = 0; l <= d.n_hidden && l < 8; ++l) a.w[l] = d.w[l];
    a.n_hidden = d.n_hidden;
    a.in_dim = d.in_dim;
    a.n_units = 2 + 8 * (d.n_hidden - 1);
    a.stream = d.bf_stream;
    a.w1m_t = d.w1m_t;
    for (int l = 0; l + 1 < d.n_hidden && l < 8; ++l) a.wh_t[l] = d.wh_t[l];
    a.wo_t = d.wo_t;
    const int64_t ns = (int64_t)a.n_units * 8192;
    pack_stream_kernel<<<(unsigned)((ns + 255) / 256), 256, 0, st>>>(a);
    pack_transpose_kernel<<<dim3(256, d.n_hidden + 1), 256, 0, st>>>(a);
}

}  // namespace swf
