// On-device peak probes for roofline accounting: what this GPU sustains in
// plain loops of one kind of instruction (BF16 MFMA, FP32 FMA, LDS reads). The
// render path never calls them.
#include "kernels.h"

namespace swf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 512;  // 8 waves per workgroup, two per SIMD

// Register-only chains of v_mfma_f32_16x16x32_bf16: 4 independent
// accumulators per wave, each a chain over 8 k-steps per iteration.
__global__ __launch_bounds__(kProbeThreads) void probe_mfma_kernel(const uint4* __restrict__ src, int iters,
                                                                   f32x4* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    bf16x8 a[8], b[4];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = __builtin_bit_cast(bf16x8, src[(k * 64 + lane) & 1023]);
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = __builtin_bit_cast(bf16x8, src[(512 + c * 64 + lane) & 1023]);
    f32x4 acc[4] = {};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[k], b[c], acc[c], 0, 0, 0);
    }
    f32x4 s = acc[0] + acc[1] + acc[2] + acc[3];
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// Independent FP32 FMA chains: 16 per lane.
__global__ __launch_bounds__(kProbeThreads) void probe_fma_kernel(int iters, float seed, float* __restrict__ out) {
    float v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = seed + (float)(threadIdx.x + i);
    const float m = 0.999f, c = 1e-3f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = fmaf(v[i], m, c);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += v[i];
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// ds_read_b128 of consecutive 16-byte words (conflict-free) from a 64 KiB LDS
// array, 4 independent reads per step.
__global__ __launch_bounds__(kProbeThreads) void probe_lds_kernel(const uint4* __restrict__ src, int iters,
                                                                  uint4* __restrict__ out) {
    constexpr int kWords = 4096;  // 64 KiB
    __shared__ uint4 buf[kWords];
    for (int i = threadIdx.x; i < kWords; i += kProbeThreads) buf[i] = src[i & 1023];
    __syncthreads();
    uint4 s = make_uint4(0u, 0u, 0u, 0u);
    int base = (int)threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint4 x = buf[(base + r * kProbeThreads) & (kWords - 1)];
            s.x ^= x.x;
            s.y += x.y;
            s.z ^= x.z;
            s.w += x.w;
        }
        base = (base + 64) & (kWords - 1);  // next step, independent of the data read (stays in the array)
    }
    out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

size_t probe_scratch_bytes(int blocks) { return (size_t)blocks * kProbeThreads * 16 + 1024 * 16; }

// Times each probe on `st` with HIP events (one warm-up launch each). scratch:
// probe_scratch_bytes(blocks) bytes of device memory.
hipError_t run_probes(int blocks, void* scratch, hipStream_t st, double* mfma_tflops, double* fma_tops,
                      double* lds_tbps) {
    uint4* src = reinterpret_cast<uint4*>(scratch);  // 1024 words of input
    void* out = reinterpret_cast<char*>(scratch) + 1024 * 16;
    hipError_t e = hipMemsetAsync(src, 0x3c, 1024 * 16, st);
    if (e != hipSuccess) return e;
    hipEvent_t a, b;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        hipEventDestroy(a);
        return e;
    }
    auto timed = [&](auto&& launch) -> double {
        launch();
        hipEventRecord(a, st);
        launch();
        hipEventRecord(b, st);
        hipEventSynchronize(b);
        float ms = 0.f;
        hipEventElapsedTime(&ms, a, b);
        return (double)ms * 1e-3;
    };
    const int mi = 4000, fi = 20000, li = 8000;
    const double tm = timed([&] {
        probe_mfma_kernel<<<blocks, kProbeThreads, 0, st>>>(src, mi, reinterpret_cast<f32x4*>(out));
    });
    const double tf = timed([&] {
        probe_fma_kernel<<<blocks, kProbeThreads, 0, st>>>(fi, 0.5f, reinterpret_cast<float*>(out));
    });
    const double tl = timed([&] {
        probe_lds_kernel<<<blocks, kProbeThreads, 0, st>>>(src, li, reinterpret_cast<uint4*>(out));
    });
    e = hipGetLastError();
    hipEventDestroy(a);
    hipEventDestroy(b);
    const double waves = (double)blocks * (kProbeThreads / 64);
    if (mfma_tflops) *mfma_tflops = waves * mi * 32 * 16384.0 / tm / 1e12;
    if (fma_tops) *fma_tops = waves * 64 * (double)fi * 16 / tf / 1e12;          // lane-ops (one per FMA)
    if (lds_tbps) *lds_tbps = waves * 64 * (double)li * 4 * 16 / tl / 1e12;      // bytes read
    return e;
}

}  // namespace swf
