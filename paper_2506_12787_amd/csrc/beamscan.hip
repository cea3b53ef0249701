// Beam-scan spatial spectrum from multipath lists (paper Sec. 3.1): the
// receiver's sqrt(K) x sqrt(K) planar array, the per-element narrowband channel
// h_mn summed over the paths (received-signal equation, with the phase shift of
// the phase-shift equation), and the beam-scan spectrum A(theta, phi) =
// |(1/K) sum_mn w_mn(theta, phi) exp(j angle h_mn)| with the steering weights
// w_mn = exp(-j dalpha_mn(theta, phi)).
//
// Two kernels per batch of queries:
//  1. channel_kernel: one wave per query; lane k < K forms h_k in FP64 over the
//     query's paths and stores the unit phasor c_k = h_k / |h_k| (0 where
//     h_k = 0, whose angle is undefined) as FP32. This is K * L complex
//     exponentials per query; FP64 keeps the phase of a nearly cancelling h_k
//     accurate, at no visible cost.
//  2. spectrum_kernel: one thread per pixel and kQ queries. Element (m, n)
//     sits at r cos(theta - beta) = D ((n-1) cos theta + (m-1) sin theta), so
//     the steering phase separates: exp(-j dalpha_mn) = zu^(n-1) zv^(m-1) with
//     zu = exp(j pi U), zv = exp(j pi V), U = 2 (D/lambda) cos phi cos theta,
//     V = 2 (D/lambda) cos phi sin theta. The K-term sum is a bivariate
//     polynomial in (zu, zv), evaluated by Horner's rule: the steering of a
//     pixel (four sincospi) is formed once and serves the kQ queries of the
//     thread, whose phasors are broadcast from LDS; per (pixel, query) that
//     leaves K complex multiply-adds (4K FMA), the modulus and a 4-byte store.
//     Vector-ALU bound (the output store is ~8x cheaper at HBM rate).
#include <math.h>

#include "runtime.h"

namespace swf {

namespace {

constexpr int kMaxSide = 8;  // K <= 64: one lane per element in the channel kernel

__global__ __launch_bounds__(64) void channel_kernel(const float* __restrict__ paths,
                                                     const int32_t* __restrict__ counts, int max_paths, int side,
                                                     double d_over_lambda, float2* __restrict__ phasor) {
    const int q = blockIdx.x;
    const int k = threadIdx.x;
    const int K = side * side;
    const int L = min(max(counts[q], 0), max_paths);  // a count outside [0, max_paths] is clamped
    if (k >= K) return;
    const int m = k / side, n = k - m * side;  // element (m + 1, n + 1), m-major
    const float* p = paths + (size_t)q * max_paths * 3;
    double re = 0.0, im = 0.0;
    for (int l = 0; l < L; ++l) {
        const double rho = (double)p[3 * l], th = (double)p[3 * l + 1], ph = (double)p[3 * l + 2];
        // dalpha / pi = 2 (D / lambda) * (-r cos(theta - beta) cos phi) / D
        const double t = -2.0 * d_over_lambda * cos(ph) * ((double)n * cos(th) + (double)m * sin(th));
        double s, c;
        sincospi(t, &s, &c);
        re += rho * c;
        im += rho * s;
    }
    const double mag = hypot(re, im);
    float2 out = make_float2(0.f, 0.f);
    if (mag > 0.0) out = make_float2((float)(re / mag), (float)(im / mag));
    phasor[(size_t)q * K + k] = out;
}

template <int SIDE>
__device__ __forceinline__ float eval_poly(const float2* __restrict__ c, float ur, float ui, float vr, float vi) {
    // sum over m of zv^m * (sum over n of c[m][n] zu^n), both by Horner's rule
    float ar = 0.f, ai = 0.f;
#pragma unroll
    for (int m = SIDE - 1; m >= 0; --m) {
        float br = 0.f, bi = 0.f;
#pragma unroll
        for (int n = SIDE - 1; n >= 0; --n) {
            const float2 cv = c[m * SIDE + n];
            const float tr = br * ur - bi * ui + cv.x;
            const float ti = br * ui + bi * ur + cv.y;
            br = tr;
            bi = ti;
        }
        const float tr = ar * vr - ai * vi + br;
        const float ti = ar * vi + ai * vr + bi;
        ar = tr;
        ai = ti;
    }
    return sqrtf(ar * ar + ai * ai);
}

constexpr int kQ = 8;  // queries per thread

template <int SIDE>
__global__ __launch_bounds__(256) void spectrum_kernel(const float2* __restrict__ phasor, int B, int H, int W,
                                                       float two_d, float* __restrict__ out) {
    constexpr int K = SIDE * SIDE;
    __shared__ float2 c[kQ][K];
    const int q0 = blockIdx.y * kQ;
    const int nq = min(kQ, B - q0);
    for (int i = threadIdx.x; i < nq * K; i += 256) c[i / K][i % K] = phasor[(size_t)q0 * K + i];
    __syncthreads();
    const int64_t HW = (int64_t)H * W;
    const int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= HW) return;
    const int y = (int)(pix / W), x = (int)(pix - (int64_t)y * W);
    // theta = 2 pi x / W (azimuth), phi = (pi / 2) y / H (elevation)
    float st, ct, sp, cp;
    sincospif(2.0f * (float)x / (float)W, &st, &ct);
    sincospif(0.5f * (float)y / (float)H, &sp, &cp);
    const float a = two_d * cp;
    float ui, ur, vi, vr;
    sincospif(a * ct, &ui, &ur);
    sincospif(a * st, &vi, &vr);
    float* o = out + (size_t)q0 * HW + pix;
    for (int k = 0; k < nq; ++k) o[(size_t)k * HW] = eval_poly<SIDE>(c[k], ur, ui, vr, vi) * (1.0f / (float)K);
}

template <int SIDE>
void launch_spectrum(const float2* phasor, int B, int H, int W, float two_d, float* out, hipStream_t st) {
    const int64_t HW = (int64_t)H * W;
    dim3 grid((unsigned)((HW + 255) / 256), (unsigned)((B + kQ - 1) / kQ));
    spectrum_kernel<SIDE><<<grid, 256, 0, st>>>(phasor, B, H, W, two_d, out);
}

}  // namespace

}  // namespace swf

using namespace swf;

extern "C" swf_status swf_beamscan(swf_ctx* h, const float* paths, const int32_t* counts, int32_t batch,
                                   int32_t max_paths, int32_t side, float spacing_over_lambda, int32_t height,
                                   int32_t width, float* out, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    if (batch < 1 || batch > 65535) return c->fail(SWF_E_INVALID, "batch must be in [1, 65535]");
    if (max_paths < 0) return c->fail(SWF_E_INVALID, "max_paths must be >= 0");
    if (side < 1 || side > kMaxSide) return c->fail(SWF_E_INVALID, "side must be in [1, 8]");
    if (!(spacing_over_lambda > 0.f) || !isfinite(spacing_over_lambda))
        return c->fail(SWF_E_INVALID, "spacing_over_lambda must be finite and > 0");
    if (height < 1 || height > 4096 || width < 1 || width > 4096)
        return c->fail(SWF_E_INVALID, "height and width must be in [1, 4096]");
    if (!counts || !out || (max_paths > 0 && !paths)) return c->fail(SWF_E_INVALID, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int K = side * side;
    swf_status s = c->ws.beam.reserve(c, (size_t)batch * K * sizeof(float2), st);
    if (s) return s;
    float2* ph = (float2*)c->ws.beam.ptr;
    channel_kernel<<<batch, 64, 0, st>>>(paths, counts, max_paths, side, (double)spacing_over_lambda, ph);
    const float two_d = 2.0f * spacing_over_lambda;
    switch (side) {
        case 1: launch_spectrum<1>(ph, batch, height, width, two_d, out, st); break;
        case 2: launch_spectrum<2>(ph, batch, height, width, two_d, out, st); break;
        case 3: launch_spectrum<3>(ph, batch, height, width, two_d, out, st); break;
        case 4: launch_spectrum<4>(ph, batch, height, width, two_d, out, st); break;
        case 5: launch_spectrum<5>(ph, batch, height, width, two_d, out, st); break;
        case 6: launch_spectrum<6>(ph, batch, height, width, two_d, out, st); break;
        case 7: launch_spectrum<7>(ph, batch, height, width, two_d, out, st); break;
        default: launch_spectrum<8>(ph, batch, height, width, two_d, out, st); break;
    }
    return c->hip(hipGetLastError(), "beam-scan launch");
}
