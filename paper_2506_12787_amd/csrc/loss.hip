// L1 loss of the training objective (Sec. 4.4, the l1 term): mean |pred - target|
// and its gradient sign(pred - target) / n. Deterministic two-level reduction.
#include "runtime.h"

namespace swf {

namespace {

constexpr int kLossBlocks = 1024;

__global__ __launch_bounds__(256) void l1_partial_kernel(const float* __restrict__ pred,
                                                         const float* __restrict__ target, int64_t n, float inv_n,
                                                         float* __restrict__ grad, double* __restrict__ partial) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = pred[i] - target[i];
        s += fabs((double)d);
        if (grad) grad[i] = d > 0.f ? inv_n : (d < 0.f ? -inv_n : 0.f);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void l1_final_kernel(const double* __restrict__ partial, int m, double inv_n,
                                                       float* __restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(red[0] * inv_n);
}

}  // namespace

}  // namespace swf

using namespace swf;

extern "C" swf_status swf_l1_loss(swf_ctx* h, const float* pred, const float* target, int64_t n, float* loss,
                                  float* grad, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    if (n < 1 || !pred || !target || !loss) return c->fail(SWF_E_INVALID, "bad loss arguments");
    hipStream_t st = (hipStream_t)stream;
    swf_status s = c->ws.grad.reserve(c, kLossBlocks * sizeof(double), st);
    if (s) return s;
    const int blocks = (int)std::min<int64_t>(kLossBlocks, (n + 255) / 256);
    l1_partial_kernel<<<blocks, 256, 0, st>>>(pred, target, n, (float)(1.0 / (double)n), grad, (double*)c->ws.grad.ptr);
    l1_final_kernel<<<1, 256, 0, st>>>((const double*)c->ws.grad.ptr, blocks, 1.0 / (double)n, loss);
    return c->hip(hipGetLastError(), "l1 loss");
}

// ---------------------------------------------------------------------------
// Hybrid loss (Sec. 4.4, hybrid-loss equation): lambda1 * mean |pred - target|
// + (1 - lambda1) * (1 - SSIM), SSIM with an 11 x 11 Gaussian window
// (sigma 1.5, normalised), zero padding, C1 = 0.01^2, C2 = 0.03^2, averaged over
// every pixel of every spectrum. One workgroup per 16 x 16 output tile of one
// spectrum: the tile plus a 5-pixel halo of both images is staged in LDS, the
// five window sums (x, y, x^2, y^2, x y) are taken separably (rows, then
// columns) in FP64, so that the variances E[x^2] - mu^2 keep their digits; the
// same pass stores, scaled by the loss weight, the three derivatives of the
// SSIM map with respect to the window sums that involve the prediction. The
// gradient pass sends them back through the same (symmetric) window.
namespace swf {
namespace {

constexpr int kST = 16, kSH = 5, kSI = kST + 2 * kSH;  // tile, halo, staged width
constexpr double kC1 = 1e-4, kC2 = 9e-4;

struct SsimWin {
    double g[2 * kSH + 1];
};

__global__ __launch_bounds__(256) void ssim_fwd_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                       int H, int W, int TW, SsimWin win, double gscale,
                                                       float* __restrict__ maps, size_t plane,
                                                       double* __restrict__ part) {
    __shared__ double sx[kSI][kSI], sy[kSI][kSI];
    __shared__ double hs[5][kSI][kST];
    __shared__ double red[2][256];
    const int b = blockIdx.y, t = blockIdx.x;
    const int ox = (t % TW) * kST, oy = (t / TW) * kST;
    const float* xb = x + (size_t)b * H * W;
    const float* yb = y + (size_t)b * H * W;
    for (int i = threadIdx.x; i < kSI * kSI; i += 256) {
        const int r = i / kSI, c = i - r * kSI;
        const int gy = oy - kSH + r, gx = ox - kSH + c;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        sx[r][c] = in ? (double)xb[(size_t)gy * W + gx] : 0.0;
        sy[r][c] = in ? (double)yb[(size_t)gy * W + gx] : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSI * kST; i += 256) {
        const int r = i / kST, c = i - r * kST;
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
#pragma unroll
        for (int k = 0; k < 2 * kSH + 1; ++k) {
            const double gx = win.g[k], vx = sx[r][c + k], vy = sy[r][c + k];
            a0 = fma(gx, vx, a0);
            a1 = fma(gx, vy, a1);
            a2 = fma(gx, vx * vx, a2);
            a3 = fma(gx, vy * vy, a3);
            a4 = fma(gx, vx * vy, a4);
        }
        hs[0][r][c] = a0;
        hs[1][r][c] = a1;
        hs[2][r][c] = a2;
        hs[3][r][c] = a3;
        hs[4][r][c] = a4;
    }
    __syncthreads();
    const int ly = threadIdx.x / kST, lx = threadIdx.x - ly * kST;
    double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 2 * kSH + 1; ++k) {
        const double g = win.g[k];
#pragma unroll
        for (int j = 0; j < 5; ++j) m[j] = fma(g, hs[j][ly + k][lx], m[j]);
    }
    const int py = oy + ly, px = ox + lx;
    double s_here = 0.0, l1_here = 0.0;
    if (py < H && px < W) {
        const double mx = m[0], my = m[1];
        const double vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
        const double N1 = 2.0 * mx * my + kC1, N2 = 2.0 * cxy + kC2;
        const double D1 = mx * mx + my * my + kC1, D2 = vx + vy + kC2;
        const double S = N1 * N2 / (D1 * D2);
        const double dm = (2.0 * my * (N2 - N1)) / (D1 * D2) - 2.0 * mx * S / D1 + 2.0 * mx * S / D2;
        const double dexx = -S / D2, dexy = 2.0 * N1 / (D1 * D2);
        const size_t o = (size_t)b * H * W + (size_t)py * W + px;
        maps[o] = (float)(gscale * dm);
        maps[plane + o] = (float)(gscale * dexx);
        maps[2 * plane + o] = (float)(gscale * dexy);
        s_here = S;
        l1_here = fabs(sx[ly + kSH][lx + kSH] - sy[ly + kSH][lx + kSH]);
    }
    red[0][threadIdx.x] = s_here;
    red[1][threadIdx.x] = l1_here;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const size_t blk = (size_t)b * gridDim.x + t;
        part[2 * blk] = red[0][0];
        part[2 * blk + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(256) void ssim_final_kernel(const double* __restrict__ part, int nblk, double inv_n,
                                                         double lambda1, float* __restrict__ loss) {
    __shared__ double red[2][256];
    double s = 0.0, l = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) {
        s += part[2 * i];
        l += part[2 * i + 1];
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ssim = red[0][0] * inv_n, l1 = red[1][0] * inv_n;
        loss[0] = (float)(lambda1 * l1 + (1.0 - lambda1) * (1.0 - ssim));
        loss[1] = (float)l1;
        loss[2] = (float)ssim;
    }
}

__global__ __launch_bounds__(256) void ssim_bwd_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                       const float* __restrict__ maps, size_t plane, int H, int W,
                                                       int TW, SsimWin win, float l1w, float* __restrict__ grad) {
    __shared__ double sm[3][kSI][kSI];
    __shared__ double hs[3][kSI][kST];
    const int b = blockIdx.y, t = blockIdx.x;
    const int ox = (t % TW) * kST, oy = (t / TW) * kST;
    const size_t base = (size_t)b * H * W;
    for (int i = threadIdx.x; i < kSI * kSI; i += 256) {
        const int r = i / kSI, c = i - r * kSI;
        const int gy = oy - kSH + r, gx = ox - kSH + c;
        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
        const size_t o = base + (size_t)gy * W + gx;
#pragma unroll
        for (int j = 0; j < 3; ++j) sm[j][r][c] = in ? (double)maps[j * plane + o] : 0.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSI * kST; i += 256) {
        const int r = i / kST, c = i - r * kST;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < 2 * kSH + 1; ++k) a = fma(win.g[k], sm[j][r][c + k], a);
            hs[j][r][c] = a;
        }
    }
    __syncthreads();
    const int ly = threadIdx.x / kST, lx = threadIdx.x - ly * kST;
    const int py = oy + ly, px = ox + lx;
    if (py >= H || px >= W) return;
    double f[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 2 * kSH + 1; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) f[j] = fma(win.g[k], hs[j][ly + k][lx], f[j]);
    const size_t o = base + (size_t)py * W + px;
    const float xv = x[o], yv = y[o];
    const float d = xv - yv;
    const double g = f[0] + 2.0 * (double)xv * f[1] + (double)yv * f[2];
    grad[o] = (float)(g + (d > 0.f ? (double)l1w : (d < 0.f ? -(double)l1w : 0.0)));
}

}  // namespace
}  // namespace swf

extern "C" swf_status swf_hybrid_loss(swf_ctx* h, const float* pred, const float* target, int32_t batch,
                                      int32_t height, int32_t width, float lambda1, float* loss, float* grad,
                                      void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    if (batch < 1 || batch > 65535 || height < 1 || width < 1 || height > 4096 || width > 4096 || !pred ||
        !target || !loss || !(lambda1 >= 0.f && lambda1 <= 1.f))
        return c->fail(SWF_E_INVALID, "bad hybrid loss arguments");
    hipStream_t st = (hipStream_t)stream;
    const int TW = (width + kST - 1) / kST, TH = (height + kST - 1) / kST;
    const size_t plane = (size_t)batch * height * width;
    const size_t nblk = (size_t)batch * TW * TH;
    swf_status s = c->ws.ssim.reserve(c, plane * 3 * sizeof(float) + nblk * 2 * sizeof(double) + 64, st);
    if (s) return s;
    float* maps = (float*)c->ws.ssim.ptr;
    double* part = (double*)((char*)c->ws.ssim.ptr + ((plane * 3 * sizeof(float) + 15) & ~(size_t)15));
    SsimWin win;
    double sum = 0.0;
    for (int k = 0; k < 2 * kSH + 1; ++k) {
        const double r = (double)(k - kSH);
        win.g[k] = exp(-r * r / (2.0 * 1.5 * 1.5));
        sum += win.g[k];
    }
    for (int k = 0; k < 2 * kSH + 1; ++k) win.g[k] /= sum;
    const double n = (double)plane;
    dim3 grid((unsigned)(TW * TH), (unsigned)batch);
    ssim_fwd_kernel<<<grid, 256, 0, st>>>(pred, target, height, width, TW, win, -(1.0 - (double)lambda1) / n, maps,
                                          plane, part);
    ssim_final_kernel<<<1, 256, 0, st>>>(part, (int)nblk, 1.0 / n, (double)lambda1, loss);
    if (grad)
        ssim_bwd_kernel<<<grid, 256, 0, st>>>(pred, target, maps, plane, height, width, TW, win,
                                              (float)((double)lambda1 / n), grad);
    return c->hip(hipGetLastError(), "hybrid loss");
}
