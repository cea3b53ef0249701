// Device-side packing of the deformation MLP from its FP32 master weights on
// the device: the fragment-major FP32 copy read by the FP32 MFMA kernel (built
// here at upload and after every update) and, after a training update, the
// BF16 weight stream of the BF16 MFMA kernel (whose upload builds it on the
// host in the same layout). Runs on the caller's stream with no host round trip.
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
    const float* bout;  // output bias (7)
    float* frag;        // frag_floats(n_hidden) FP32, fragment-major
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

// One thread per float of the FP32 fragment copy. Fragment q of output tile t
// holds, in lane l = 16 g + r, element j: the weight of output unit 16 t + r
// for input chunk c = 4 q + j at input k(c, g). Layer 1 (mean features,
// chunk c of lane group g = feature 4 c + g): k = 4 c + g, zero past 26.
// Hidden and output layers: k = 16 q + 4 g + j, the unit the previous layer's
// output tile q leaves in element j of lane group g.
__global__ void pack_frag_kernel(PackArgs a) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t out_at = (int64_t)frag_out_at(a.n_hidden);
    if (e >= out_at + (int64_t)kFragOut + 16) return;
    float v = 0.0f;
    if (e < (int64_t)kFragL1) {
        const int t = (int)(e / 512), q = (int)(e / 256) % 2, l = (int)(e / 4) % 64, j = (int)(e % 4);
        const int k = 4 * (4 * q + j) + (l >> 4), row = 16 * t + (l & 15);
        if (k < kMeanFeat) v = a.w[0][(size_t)row * a.in_dim + k];
    } else if (e < out_at) {
        const int64_t r = e - (int64_t)kFragL1;
        const int L = 1 + (int)(r / (int64_t)kFragHidden);
        const int rr = (int)(r % (int64_t)kFragHidden);
        const int t = rr / 4096, q = (rr / 256) % 16, l = (rr / 4) % 64, j = rr % 4;
        v = a.w[L][(size_t)(16 * t + (l & 15)) * 256 + 16 * q + 4 * (l >> 4) + j];
    } else if (e < out_at + (int64_t)kFragOut) {
        const int rr = (int)(e - out_at);
        const int q = rr / 256, l = (rr / 4) % 64, j = rr % 4, o = l & 15;
        if (o < kOut) v = a.w[a.n_hidden][(size_t)o * 256 + 16 * q + 4 * (l >> 4) + j];
    } else {
        const int o = (int)(e - out_at - (int64_t)kFragOut);
        if (o < kOut) v = a.bout[o];
    }
    a.frag[e] = v;
}

}  // namespace

static PackArgs pack_args(const DevScene& d) {
    PackArgs a{};
    for (int l = 0; l <= d.n_hidden && l < 8; ++l) a.w[l] = d.w[l];
    a.n_hidden = d.n_hidden;
    a.in_dim = d.in_dim;
    a.n_units = 2 + 8 * (d.n_hidden - 1);
    a.stream = d.bf_stream;
    a.bout = d.b[d.n_hidden];
    a.frag = d.f32_frag;
    return a;
}

void launch_pack_f32_frag(const DevScene& d, hipStream_t st) {
    const PackArgs a = pack_args(d);
    const int64_t nf = (int64_t)frag_floats(d.n_hidden);
    pack_frag_kernel<<<(unsigned)((nf + 255) / 256), 256, 0, st>>>(a);
}

void launch_pack_mlp(const DevScene& d, hipStream_t st) {
    const PackArgs a = pack_args(d);
    const int64_t ns = (int64_t)a.n_units * 8192;
    pack_stream_kernel<<<(unsigned)((ns + 255) / 256), 256, 0, st>>>(a);
    launch_pack_f32_frag(d, st);
}

}  // namespace swf
