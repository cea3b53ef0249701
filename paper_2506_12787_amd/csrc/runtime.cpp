// Host runtime of libswiftwrf: context, scene registry, workspace, the render
// pipeline and the C ABI declared in include/swiftwrf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/swiftwrf.h"
#include "kernels.h"
#include "runtime.h"

using namespace swf;

namespace swf {

const char* status_name(swf_status s) {
    switch (s) {
        case SWF_OK: return "ok";
        case SWF_E_INVALID: return "invalid argument";
        case SWF_E_OOM: return "out of memory";
        case SWF_E_DEVICE: return "HIP runtime error";
        case SWF_E_NOT_FOUND: return "not found";
        case SWF_E_OVERFLOW: return "capacity exceeded";
        case SWF_E_STATE: return "invalid state";
        case SWF_E_PENDING: return "pending";
        default: return "unknown status";
    }
}

swf_status Ctx::fail(swf_status s, const std::string& msg) {
    err = msg;
    return s;
}

swf_status Ctx::hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return SWF_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? SWF_E_OOM : SWF_E_DEVICE;
}

swf_status Buf::reserve(Ctx* c, size_t n, hipStream_t st) {
    if (n <= cap) return SWF_OK;
    if (ptr) {
        if (st) hipStreamSynchronize(st);
        hipDeviceSynchronize();
        hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
    size_t want = n + n / 4 + 256;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        return c->hip(e, "hipMalloc(workspace)");
    }
    cap = want;
    ++gen;
    return SWF_OK;
}

swf_status Workspace::init(Ctx* c) {
    if (hipMalloc(&total_dev, 64) != hipSuccess) return c->fail(SWF_E_OOM, "hipMalloc(status)");
    if (hipHostMalloc(&total_host, 64, 0) != hipSuccess) return c->fail(SWF_E_OOM, "hipHostMalloc(status)");
    status_dev = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(total_dev) + 16);
    cull_dev = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(total_dev) + 32);
    if (hipEventCreateWithFlags(&total_ev, hipEventDisableTiming) != hipSuccess)
        return c->fail(SWF_E_DEVICE, "hipEventCreate");
    return c->hip(hipMemset(total_dev, 0, 64), "hipMemset(status)");
}

void Workspace::release() {
    for (Buf* b : bufs()) b->release();
    if (mix_host) hipHostFree(mix_host);
    mix_host = nullptr;
    mix_host_cap = 0;
    if (total_dev) hipFree(total_dev);
    if (total_host) hipHostFree(total_host);
    if (total_ev) hipEventDestroy(total_ev);
    total_dev = nullptr;
    total_host = nullptr;
    total_ev = nullptr;
}

void Buf::release() {
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    cap = 0;
}

static int bits_for(uint64_t m) {
    int b = 0;
    while (b < 64 && (1ull << b) < m) ++b;
    return b;
}

Grid make_grid(int H, int W, int tile, bool wrap, float sx, float sy) {
    Grid g;
    g.wrap = wrap ? 1 : 0;
    g.sx = sx;
    g.sy = sy;
    g.H = H;
    g.W = W;
    g.tile = tile;
    g.TW = (W + tile - 1) / tile;
    g.TH = (H + tile - 1) / tile;
    g.tiles = g.TW * g.TH;
    return g;
}

void Ctx::stage_begin(int stage, hipStream_t st) {
    if (!timing || serve_timing_disabled()) return;
    TimedStage t;
    t.stage = stage;
    if (!event_pool.empty()) {
        t.a = event_pool.back();
        event_pool.pop_back();
    } else {
        hipEventCreate(&t.a);
    }
    if (!event_pool.empty()) {
        t.b = event_pool.back();
        event_pool.pop_back();
    } else {
        hipEventCreate(&t.b);
    }
    hipEventRecord(t.a, st);
    pending.push_back(t);
}

void Ctx::stage_end(hipStream_t st) {
    if (!timing || serve_timing_disabled() || pending.empty()) return;
    hipEventRecord(pending.back().b, st);
    if (pending.size() > 8192) resolve_timing();
}

void Ctx::resolve_timing() {
    for (auto& t : pending) {
        hipEventSynchronize(t.b);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            stage_ms[t.stage] += ms;
            stage_n[t.stage] += 1;
        }
        event_pool.push_back(t.a);
        event_pool.push_back(t.b);
    }
    pending.clear();
}

void Ctx::tag_aux(const void* aux, const AuxTag& t) {
    constexpr size_t kMaxTags = 1024;
    if (!aux_tags.count(aux)) {
        aux_order.push_back(aux);
        if (aux_order.size() > kMaxTags) {
            aux_tags.erase(aux_order.front());
            aux_order.erase(aux_order.begin());
        }
    }
    aux_tags[aux] = t;
}

Scene* Ctx::scene(int id) {
    auto it = scenes.find(id);
    return it == scenes.end() ? nullptr : it->second;
}

static void free_scene(Scene* s) {
    DevScene& d = s->d;
    for (void* p : s->allocs) hipFree(p);
    s->allocs.clear();
    (void)d;
    delete s;
}

// Allocate and copy a host array to the device, tracked by the scene.
template <typename T>
static swf_status upload(Ctx* c, Scene* s, T** dst, const T* src, size_t n) {
    *dst = nullptr;
    const size_t bytes = std::max<size_t>(n * sizeof(T), 16);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return c->hip(e, "hipMalloc(scene)");
    s->allocs.push_back(p);
    s->d.bytes += bytes;
    if (n) {
        e = hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return c->hip(e, "hipMemcpy(scene)");
    }
    *dst = reinterpret_cast<T*>(p);
    return SWF_OK;
}

static swf_status fetch(Ctx* c, std::vector<float>& dst, const float* src, size_t n, bool dev) {
    dst.resize(n);
    if (!n) return SWF_OK;
    if (!src) return c->fail(SWF_E_INVALID, "null parameter array");
    if (dev) return c->hip(hipMemcpy(dst.data(), src, n * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy(D2H)");
    std::memcpy(dst.data(), src, n * sizeof(float));
    return SWF_OK;
}

static uint16_t f32_to_bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

swf_status Ctx::upload_scene(const swf_gaussians* g, const swf_mlp* mlp, int H, int W, bool dev, int* id) {
    if (!g || !id || g->n < 0) return fail(SWF_E_INVALID, "null gaussians/id or n < 0");
    if (H < 1 || H > 4096 || W < 1 || W > 4096) return fail(SWF_E_INVALID, "H and W must lie in [1, 4096]");
    if ((int64_t)g->n * 1 > (int64_t)INT32_MAX) return fail(SWF_E_INVALID, "n too large");
    const size_t n = (size_t)g->n;
    std::vector<float> col[8];
    const float* src[8] = {g->mean_x, g->mean_y, g->log_scale_x, g->log_scale_y,
                           g->rotation, g->opacity_logit, g->amplitude, g->depth};
    for (int k = 0; k < 8; ++k) {
        swf_status st = fetch(this, col[k], src[k], n, dev);
        if (st) return st;
    }
    if (mlp) {
        if (mlp->mean_bands != kMeanBands || mlp->tx_bands != kTxBands)
            return fail(SWF_E_INVALID, "positional encoding bands must be 6 (mean) and 10 (tx)");
        if (mlp->hidden != 256) return fail(SWF_E_INVALID, "hidden width must be 256");
        if (mlp->n_hidden < 1 || mlp->n_hidden > SWF_MAX_LAYERS - 1)
            return fail(SWF_E_INVALID, "n_hidden must lie in [1, 7]");
        for (int l = 0; l <= mlp->n_hidden; ++l)
            if (!mlp->weight[l] || !mlp->bias[l]) return fail(SWF_E_INVALID, "null MLP weight or bias");
        for (int k = 0; k < 3; ++k)
            if (!(mlp->room_hi[k] > mlp->room_lo[k])) return fail(SWF_E_INVALID, "room_hi must exceed room_lo");
    }
    // (depth, id) order; NaN depths last (never rendered)
    std::vector<uint32_t> perm(n);
    for (size_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    const std::vector<float>& dep = col[7];
    std::stable_sort(perm.begin(), perm.end(), [&](uint32_t a, uint32_t b) {
        const bool na = std::isnan(dep[a]), nb = std::isnan(dep[b]);
        if (na != nb) return !na;
        if (na) return false;
        return dep[a] < dep[b];
    });
    size_t n_live = 0;
    for (size_t i = 0; i < n; ++i) n_live += !std::isnan(dep[i]);
    std::vector<float> sorted[7];
    for (int k = 0; k < 7; ++k) {
        sorted[k].resize(n);
        for (size_t p = 0; p < n; ++p) sorted[k][p] = col[k][perm[p]];
    }
    std::vector<uint32_t> dbits(n), inv(n);
    for (size_t p = 0; p < n; ++p) {
        dbits[p] = depth_key_bits(dep[perm[p]]);
        inv[perm[p]] = (uint32_t)p;
    }

    Scene* s = new (std::nothrow) Scene();
    if (!s) return fail(SWF_E_OOM, "host allocation");
    DevScene& d = s->d;
    d.n = (int)n;
    d.n_live = (int)n_live;
    d.H = H;
    d.W = W;
    swf_status st = SWF_OK;
    float** dst[7] = {&d.mx, &d.my, &d.lsx, &d.lsy, &d.rot, &d.logit, &d.amp};
    for (int k = 0; k < 7 && !st; ++k) st = upload(this, s, dst[k], sorted[k].data(), n);
    if (!st) st = upload(this, s, &d.dbits, dbits.data(), n);
    if (!st) st = upload(this, s, &d.perm, perm.data(), n);
    if (!st) st = upload(this, s, &d.inv_perm, inv.data(), n);
    s->host_dbits = dbits;
    s->host_perm = perm;
    if (!st && mlp) st = pack_mlp(s, mlp, dev, true);
    if (st) {
        free_scene(s);
        return st;
    }
    const int sid = next_scene++;
    scenes[sid] = s;
    *id = sid;
    return SWF_OK;
}

// The paper's model: raw parameters in id order (the sum has no order), the
// FP64 centre map and its encoding on the device, and the paper MLP packed for
// paper_mlp_kernel in MFMA fragment order (layout below), every pad row and
// column zero.
swf_status Ctx::upload_paper_scene(const swf_paper_gaussians* g, const swf_paper_mlp* mlp, int H, int W, bool dev,
                                   int* id) {
    if (!g || !id || g->n < 0) return fail(SWF_E_INVALID, "null gaussians/id or n < 0");
    if (H < 1 || H > 4096 || W < 1 || W > 4096) return fail(SWF_E_INVALID, "H and W must lie in [1, 4096]");
    const size_t n = (size_t)g->n;
    std::vector<float> col[8];
    const float* src[8] = {g->center_x, g->center_y, g->chol_l1, g->chol_l2, g->chol_l3, g->atten_logit,
                           g->psi_re, g->psi_im};
    for (int k = 0; k < 8; ++k) {
        swf_status st = fetch(this, col[k], src[k], n, dev);
        if (st) return st;
    }
    static const int kIn[9] = {81, 156, 237, 156, 237, 156, 237, 156, 156};
    static const int kOutDim[9] = {156, 156, 156, 156, 156, 156, 156, 156, 5};
    std::vector<std::vector<float>> Wm(9), Bm(9);
    if (mlp) {
        for (int l = 0; l < 9; ++l) {
            if (!mlp->weight[l] || !mlp->bias[l]) return fail(SWF_E_INVALID, "null paper MLP weight or bias");
            swf_status st = fetch(this, Wm[l], mlp->weight[l], (size_t)kOutDim[l] * kIn[l], dev);
            if (!st) st = fetch(this, Bm[l], mlp->bias[l], (size_t)kOutDim[l], dev);
            if (st) return st;
        }
        for (int k = 0; k < 3; ++k)
            if (!(mlp->room_hi[k] > mlp->room_lo[k])) return fail(SWF_E_INVALID, "room_hi must exceed room_lo");
    }
    Scene* s = new (std::nothrow) Scene();
    if (!s) return fail(SWF_E_OOM, "host allocation");
    DevScene& d = s->d;
    d.kind = 1;
    d.n = (int)n;
    d.n_live = (int)n;
    d.H = H;
    d.W = W;
    std::vector<uint32_t> perm(n), zero(n, 0u);
    for (size_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    swf_status st = SWF_OK;
    float** dst[8] = {&d.pcx, &d.pcy, &d.pl1, &d.pl2, &d.pl3, &d.patt, &d.ppre, &d.ppim};
    for (int k = 0; k < 8 && !st; ++k) st = upload(this, s, dst[k], col[k].data(), n);
    if (!st) st = upload(this, s, &d.dbits, zero.data(), n);
    if (!st) st = upload(this, s, &d.perm, perm.data(), n);
    if (!st) st = upload(this, s, &d.inv_perm, perm.data(), n);
    if (!st) {
        std::vector<float4> c4(n);
        st = upload(this, s, &d.pcen, c4.data(), n);
    }
    if (!st) {
        std::vector<float> f(n * kPaperFeatStride);
        st = upload(this, s, &d.pfeat, f.data(), f.size());
    }
    s->host_dbits = zero;
    s->host_perm = perm;
    if (!st && mlp) {
        d.has_mlp = true;
        for (int k = 0; k < 3; ++k) {
            d.room_lo[k] = mlp->room_lo[k];
            d.room_hi[k] = mlp->room_hi[k];
        }
        for (int l = 0; l < 9 && !st; ++l) {
            st = upload(this, s, &d.pw[l], Wm[l].data(), Wm[l].size());
            if (!st) st = upload(this, s, &d.pb[l], Bm[l].data(), Bm[l].size());
        }
        // MFMA operands, fragment-major (paper.hip): per layer, output tile t (16 units), fragment q of 4 input
        // chunks, lane l, chunk j: W[unit 16 t + l % 16][input of chunk 4 q + j for lane group l / 16]. A layer's
        // chunks are [h (40) | x (24)] as it takes them; h chunk c holds the previous layer's unit
        // 16 (c / 4) + 4 g + c % 4 (g = l / 16), x chunk c the input feature 4 c + g. Pads are zero.
        for (int l = 0; l <= kPaperLayers && !st; ++l) {
            const bool out_layer = l == kPaperLayers;
            const bool hasH = l != 0, hasX = l == 0 || l == 2 || l == 4 || l == 6;
            const int G = (hasH ? 10 : 0) + (hasX ? 6 : 0), tiles = out_layer ? 1 : 10;
            const int units = out_layer ? kPaperOut : kPaperWidth;
            std::vector<float> t((size_t)tiles * G * 64 * 4, 0.0f), b((size_t)tiles * 16, 0.0f);
            for (int tt = 0; tt < tiles; ++tt)
                for (int q = 0; q < G; ++q)
                    for (int ln = 0; ln < 64; ++ln)
                        for (int j = 0; j < 4; ++j) {
                            const int unit = 16 * tt + ln % 16, g = ln / 16, c = 4 * q + j;
                            if (unit >= units) continue;
                            int col = -1;  // the paper layer's input column
                            if (hasH && c < 40) {
                                const int f = 16 * (c / 4) + 4 * g + c % 4;
                                if (f < kPaperWidth) col = f;
                            } else {
                                const int xf = 4 * (c - (hasH ? 40 : 0)) + g;
                                if (xf < kIn[0]) col = l == 0 ? xf : kPaperWidth + xf;
                            }
                            if (col >= 0) t[(((size_t)tt * G + q) * 64 + ln) * 4 + j] = Wm[l][(size_t)unit * kIn[l] + col];
                        }
            for (int u = 0; u < units; ++u) b[u] = Bm[l][u];
            st = upload(this, s, &d.pwt[l], t.data(), t.size());
            if (!st) st = upload(this, s, &d.pbt[l], b.data(), b.size());
        }
    }
    if (!st) {
        launch_paper_centers(d, nullptr);
        st = hip(hipDeviceSynchronize(), "paper centres");
    }
    if (st) {
        free_scene(s);
        return st;
    }
    const int sid = next_scene++;
    scenes[sid] = s;
    *id = sid;
    return SWF_OK;
}

swf_status Ctx::pack_mlp(Scene* s, const swf_mlp* mlp, bool dev, bool alloc) {
    DevScene& d = s->d;
    const size_t n = (size_t)d.n;
    swf_status st = SWF_OK;
    // allocate (first upload) or overwrite in place (update; shapes must match)
    auto put = [&](auto** dst, const auto* src, size_t cnt) -> swf_status {
        if (alloc) return upload(this, s, dst, src, cnt);
        if (!cnt) return SWF_OK;
        return hip(hipMemcpy(*dst, src, cnt * sizeof(*src), hipMemcpyHostToDevice), "hipMemcpy(mlp)");
    };
    {
        d.has_mlp = true;
        d.hidden = mlp->hidden;
        d.n_hidden = mlp->n_hidden;
        d.in_dim = kMeanFeat + kTxFeat;
        for (int k = 0; k < 3; ++k) {
            d.room_lo[k] = mlp->room_lo[k];
            d.room_hi[k] = mlp->room_hi[k];
        }
        const int Hd = d.hidden;
        std::vector<int> rows(d.n_hidden + 1), cols(d.n_hidden + 1);
        for (int l = 0; l <= d.n_hidden; ++l) {
            rows[l] = l == d.n_hidden ? kOut : Hd;
            cols[l] = l == 0 ? d.in_dim : Hd;
        }
        std::vector<std::vector<float>> Wh(d.n_hidden + 1), Bh(d.n_hidden + 1);
        for (int l = 0; l <= d.n_hidden && !st; ++l) {
            st = fetch(this, Wh[l], mlp->weight[l], (size_t)rows[l] * cols[l], dev);
            if (!st) st = fetch(this, Bh[l], mlp->bias[l], (size_t)rows[l], dev);
            if (!st) st = put(&d.w[l], Wh[l].data(), Wh[l].size());
            if (!st) st = put(&d.b[l], Bh[l].data(), Bh[l].size());
        }
        if (!st && alloc) {
            std::vector<float> z(frag_floats(d.n_hidden), 0.0f);
            st = put(&d.f32_frag, z.data(), z.size());
        }
        if (!st) {  // the FP32 MFMA kernel's fragment-major copy, packed on the device from the masters
            launch_pack_f32_frag(d, nullptr);
            st = hip(hipDeviceSynchronize(), "pack FP32 fragments");
        }
        // BF16 weight stream for the MFMA kernel: per tile of pairs the kernel
        // consumes the stream in order; fragment (t, c) of a layer holds, for
        // lane l = 16 g + r and element j, W[16 t + r][k(c, g, j)]. Layer 1 (mean
        // part, K = 26 padded to 32): 16 fragments, k = 8 g + j. Hidden layers:
        // 128 fragments in output-tile-major order (8 t + c), k = 32 c + f(g, j)
        // with f(g, j) = j < 4 ? 4 g + j : 16 + 4 g + j - 4, matching the register
        // layout of the previous layer's output tiles. The output layer (7 rows
        // padded to 16): its 8 k-chunk fragments.
        if (!st) {
            // 16 KiB units: [layer 1] [hidden layers, 8 units each] [output | pad]
            const int n_units = 2 + 8 * (d.n_hidden - 1);
            std::vector<uint16_t> t((size_t)n_units * 8192, 0);
            auto fk = [](int c, int g, int j) { return 32 * c + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4)); };
            for (int tt = 0; tt < 16; ++tt)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        const int row = 16 * tt + (l & 15), k = 8 * (l >> 4) + j;
                        const float w = k < kMeanFeat ? Wh[0][(size_t)row * d.in_dim + k] : 0.f;
                        t[(size_t)tt * 512 + l * 8 + j] = f32_to_bf16_rne(w);
                    }
            for (int L = 1; L < d.n_hidden; ++L)
                for (int tt = 0; tt < 16; ++tt)
                    for (int c = 0; c < 8; ++c) {
                        const int f = 8 * tt + c;  // output-tile-major fragment order
                        const size_t at = (size_t)(1 + 8 * (L - 1)) * 8192 + (size_t)f * 512;
                        for (int l = 0; l < 64; ++l)
                            for (int j = 0; j < 8; ++j) {
                                const int row = 16 * tt + (l & 15), k = fk(c, l >> 4, j);
                                t[at + l * 8 + j] = f32_to_bf16_rne(Wh[L][(size_t)row * Hd + k]);
                            }
                    }
            {
                const size_t ch = (size_t)(n_units - 1) * 8192;
                for (int c = 0; c < 8; ++c)
                    for (int l = 0; l < 64; ++l)
                        for (int j = 0; j < 8; ++j) {
                            const int o = l & 15, k = fk(c, l >> 4, j);
                            const float w = o < kOut ? Wh[d.n_hidden][(size_t)o * Hd + k] : 0.f;
                            t[ch + (size_t)c * 512 + l * 8 + j] = f32_to_bf16_rne(w);
                        }
            }
            st = put(&d.bf_stream, t.data(), t.size());
        }
        if (!st && alloc) {  // BF16 mean features: set up once (they depend on the means only)
            std::vector<uint16_t> z((size_t)n * 32, 0);
            st = put(&d.bf_mfeat, z.data(), z.size());
            if (!st) {
                compute_mean_features_bf16(d, nullptr);
                st = hip(hipDeviceSynchronize(), "mean features");
            }
        }
    }
    return st;
}

swf_status Ctx::update_scene(int id, const swf_gaussians* g, const swf_mlp* mlp, bool dev, hipStream_t st) {
    Scene* s = scene(id);
    if (!s) return fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (s->d.kind == 1) return fail(SWF_E_INVALID, "paper-model scenes are uploaded, not updated");
    DevScene& d = s->d;
    swf_status r = SWF_OK;
    if (g || mlp) ++s->gen;
    if (g) {
        if (g->n != d.n) return fail(SWF_E_INVALID, "n differs from the uploaded scene");
        const float* src[7] = {g->mean_x, g->mean_y, g->log_scale_x, g->log_scale_y, g->rotation, g->opacity_logit,
                               g->amplitude};
        float* dst[7] = {d.mx, d.my, d.lsx, d.lsy, d.rot, d.logit, d.amp};
        const size_t bytes = (size_t)d.n * sizeof(float);
        if ((r = ws.stage.reserve(this, 7 * bytes + 16, st))) return r;
        for (int k = 0; k < 7; ++k) {
            if (!src[k]) return fail(SWF_E_INVALID, "null parameter array");
            float* tmp = (float*)((char*)ws.stage.ptr + k * bytes);
            if ((r = hip(hipMemcpyAsync(tmp, src[k], bytes, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st),
                         "update copy")))
                return r;
        }
        float* tmps[7];
        for (int k = 0; k < 7; ++k) tmps[k] = (float*)((char*)ws.stage.ptr + k * bytes);
        launch_gather_params(tmps, d.perm, d.n, dst, st);
        if (d.has_mlp) compute_mean_features_bf16(d, st);
        // host sources: the copies read pageable memory; device sources stay stream-ordered
        if (!dev && (r = hip(hipStreamSynchronize(st), "update sync"))) return r;
    }
    if (mlp) {
        if (!d.has_mlp) return fail(SWF_E_STATE, "scene was uploaded without an MLP");
        if (mlp->n_hidden != d.n_hidden || mlp->hidden != d.hidden) return fail(SWF_E_INVALID, "MLP shape differs");
        for (int l = 0; l <= mlp->n_hidden; ++l)
            if (!mlp->weight[l] || !mlp->bias[l]) return fail(SWF_E_INVALID, "null MLP weight or bias");
        for (int k = 0; k < 3; ++k)
            if (!(mlp->room_hi[k] > mlp->room_lo[k])) return fail(SWF_E_INVALID, "room_hi must exceed room_lo");
        if (dev) {
            // device sources: copy the masters and rebuild the derived layouts on `st`
            for (int l = 0; l <= d.n_hidden; ++l) {
                const size_t rows = l == d.n_hidden ? kOut : d.hidden, cols = l == 0 ? d.in_dim : d.hidden;
                if ((r = hip(hipMemcpyAsync(d.w[l], mlp->weight[l], rows * cols * sizeof(float),
                                            hipMemcpyDeviceToDevice, st), "update copy")))
                    return r;
                if ((r = hip(hipMemcpyAsync(d.b[l], mlp->bias[l], rows * sizeof(float), hipMemcpyDeviceToDevice, st),
                             "update copy")))
                    return r;
            }
            for (int k = 0; k < 3; ++k) {
                d.room_lo[k] = mlp->room_lo[k];
                d.room_hi[k] = mlp->room_hi[k];
            }
            launch_pack_mlp(d, st);
            if ((r = hip(hipGetLastError(), "mlp repack"))) return r;
        } else {
            if ((r = hip(hipStreamSynchronize(st), "update sync"))) return r;
            if ((r = pack_mlp(s, mlp, dev, false))) return r;
        }
    }
    ws.last.valid = false;
    return SWF_OK;
}

swf_status Ctx::release_scene(int id) {
    auto it = scenes.find(id);
    if (it == scenes.end()) return fail(SWF_E_NOT_FOUND, "unknown scene id");
    hipDeviceSynchronize();
    free_scene(it->second);
    scenes.erase(it);
    return SWF_OK;
}

// Enqueue preprocess (+ MLP) for B queries into the workspace records.
swf_status Ctx::enqueue_preprocess(Workspace& w, Scene* sc, const float* tx, int B, int flags, const Grid& g, float* delta_sorted,
                                   hipStream_t st) {
    ++w.seq;  // the records (and the lists built from them) are about to change
    const DevScene& d = sc->d;
    const bool deform = !(flags & SWF_NO_DEFORM);
    if (d.kind == 1 && (flags & (SWF_MLP_BF16 | SWF_TILE8 | SWF_KEEP_AUX)))
        return fail(SWF_E_INVALID, "paper-model scenes render with the FP32 MLP, 16x16 tiles and no aux");
    if (deform && (flags & SWF_MLP_BF16) && !bf16_available())
        return fail(SWF_E_STATE, "BF16 MLP kernel is not available in this build");
    const size_t pairs = (size_t)B * d.n;
    swf_status s = SWF_OK;
    if ((s = w.geo.reserve(this, pairs * sizeof(float4), st))) return s;
    if ((s = w.wm.reserve(this, pairs * sizeof(float4), st))) return s;
    if ((s = w.oa.reserve(this, pairs * sizeof(float2), st))) return s;
    if ((s = w.rect.reserve(this, pairs * sizeof(uint2), st))) return s;
    if ((s = w.count.reserve(this, pairs * sizeof(uint32_t), st))) return s;
    w.rec.geo = (float4*)w.geo.ptr;
    w.rec.wm = (float4*)w.wm.ptr;
    w.rec.oa = (float2*)w.oa.ptr;
    w.rec.rect = (uint2*)w.rect.ptr;
    w.rec.count = (uint32_t*)w.count.ptr;
    if (d.kind == 1) {
        if (deform) {
            if (!d.has_mlp) return fail(SWF_E_INVALID, "scene has no deformation MLP (use SWF_NO_DEFORM)");
            if (!tx) return fail(SWF_E_INVALID, "tx is NULL");
            if ((s = w.qs.reserve(this, (size_t)B * kPaperFeatStride * sizeof(float), st))) return s;
        }
        stage_begin(SWF_STAGE_MLP, st);
        if (deform) {
            launch_paper_tx(d, tx, B, (float*)w.qs.ptr, st);
            launch_paper_mlp(d, (const float*)w.qs.ptr, B, g, w.rec, delta_sorted, st);
        } else {
            launch_paper_static(d, B, g, w.rec, st);
        }
        stage_end(st);
        return hip(hipGetLastError(), "paper preprocess launch");
    }
    if (deform) {
        if (!d.has_mlp) return fail(SWF_E_INVALID, "scene has no deformation MLP (use SWF_NO_DEFORM)");
        if (!tx) return fail(SWF_E_INVALID, "tx is NULL");
        if ((s = w.qs.reserve(this, (size_t)B * d.hidden * sizeof(float), st))) return s;
        stage_begin(SWF_STAGE_TX, st);
        launch_tx_features(d, tx, B, (float*)w.qs.ptr, st);
        stage_end(st);
        stage_begin(SWF_STAGE_MLP, st);
        if (flags & SWF_MLP_BF16)
            launch_mlp_bf16(d, (const float*)w.qs.ptr, B, g, (flags & SWF_PAPER_DEFORM) != 0, w.rec, delta_sorted, st,
                            mlp_pairs_per_wave, w.act_out);
        else {
            float* ap[8] = {};  // per-layer activation stores, [n_hidden][B * N][256]
            for (int l = 0; w.act_out && l < d.n_hidden && l < 8; ++l)
                ap[l] = (float*)w.act_out + (size_t)l * B * d.n * 256;
            launch_mlp_fp32(d, (const float*)w.qs.ptr, B, g, (flags & SWF_PAPER_DEFORM) != 0, w.rec, delta_sorted, st,
                            w.act_out ? ap : nullptr);
        }
        stage_end(st);
    } else {
        stage_begin(SWF_STAGE_MLP, st);
        launch_preprocess_static(d, B, g, w.rec, st);
        stage_end(st);
    }
    return hip(hipGetLastError(), "preprocess launch");
}

// Forward up to the per-tile lists: preprocess (+ MLP), scan, keys, sort,
// tile ranges. Records the result in `last`.
swf_status Ctx::forward_lists(Workspace& w, int sid, const float* tx, int B, int flags, hipStream_t st,
                              uint64_t key_cap, uint64_t spec_cap, bool* spec_used, int rH, int rW) {
    if (spec_used) *spec_used = false;
    Scene* sc = scene(sid);
    if (!sc) return fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (B < 1) return fail(SWF_E_INVALID, "batch must be >= 1");
    const DevScene& d = sc->d;
    if ((uint64_t)B * (uint64_t)d.n >= (1ull << 32))
        return fail(SWF_E_OVERFLOW, "batch * n must be < 2^32 (32-bit pair indices)");
    // the scene's own grid, or another resolution of the same field of view
    const int gH = rH > 0 ? rH : d.H, gW = rW > 0 ? rW : d.W;
    if (gH > 4096 || gW > 4096) return fail(SWF_E_INVALID, "height and width must lie in [1, 4096]");
    const Grid g = make_grid(gH, gW, (flags & SWF_TILE8) ? 8 : 16, (flags & SWF_WRAP_AZIMUTH) != 0,
                             gW == d.W ? 1.0f : (float)((double)gW / d.W), gH == d.H ? 1.0f : (float)((double)gH / d.H));
    if ((uint64_t)B * g.tiles >= (1ull << 31)) return fail(SWF_E_INVALID, "batch * tiles too large");
    w.last.valid = false;
    w.last.stream = st;
    // the status word and the culled-pair counters start at zero for every render
    launch_clear_u32(w.status_dev, 8, st);
    swf_status s = enqueue_preprocess(w, sc, tx, B, flags, g, nullptr, st);
    if (s) return s;
    const bool full = (flags & SWF_FULL_SORT) != 0;
    const int64_t n_gt = (int64_t)B * g.tiles;
    if ((s = w.ranges.reserve(this, (size_t)n_gt * sizeof(uint2), st))) return s;
    // binning unless the full 64-bit sort is asked for (or the segment grid would exceed the launch limit, or a
    // periodic azimuth spans more than one segment: the multi-segment placement enumerates unwrapped rectangles)
    if (!full && bin_fits(B, d.n, g)) {
        const bool spec = key_cap == 0 && spec_cap > 0 && spec_used;
        s = lists_binned(w, d, B, g, st, spec ? spec_cap : key_cap, spec);
        if (spec) *spec_used = true;
    } else
        s = lists_sorted(w, d, B, g, full, st, key_cap);
    if (s) return s;
    w.last.valid = true;
    w.last.scene = sid;
    w.last.B = B;
    w.last.N = d.n;
    w.last.flags = flags;
    w.last.grid = g;
    w.last.rerenders = 0;
    w.last.chunked = false;
    w.last.nan_depth_pairs = (uint64_t)B * (uint64_t)(d.n - d.n_live);
    return hip(hipGetLastError(), "forward launch");
}

// Key count after an exclusive scan whose 64-bit total is in w.total_dev:
// read back (key_cap == 0), or kept on the device as the effective count
// (total if it fits key_cap, else 0 with the overflow bit set).
swf_status Ctx::key_count(Workspace& w, hipStream_t st, uint64_t key_cap, uint64_t& nk, const uint64_t*& n_dev,
                          bool readback) {
    nk = key_cap;
    n_dev = nullptr;
    if (key_cap == 0) {
        swf_status s;
        if ((s = hip(hipMemcpyAsync(w.total_host, w.total_dev, sizeof(uint64_t), hipMemcpyDeviceToHost, st),
                     "total D2H")))
            return s;
        if ((s = hip(hipStreamSynchronize(st), "stream sync"))) return s;
        nk = *w.total_host;
    } else {
        uint64_t* n_eff = w.total_dev + 1;  // the word after the scan total
        launch_effective_count(w.total_dev, key_cap, n_eff, w.status_dev, st);  // also sets the status word
        n_dev = n_eff;
        if (readback) {
            swf_status s;
            if ((s = hip(hipMemcpyAsync(w.total_host, w.total_dev, sizeof(uint64_t), hipMemcpyDeviceToHost, st),
                         "total D2H")))
                return s;
            if ((s = hip(hipEventRecord(w.total_ev, st), "total event"))) return s;
        }
    }
    if (nk > max_list_entries)
        return fail(SWF_E_OVERFLOW, "more list entries than one launch sequence takes (max_list_entries, at most "
                                    "2^32 - 1)");
    return SWF_OK;
}

// Lists by binning (per tile segment of a query): tile histograms per block of
// pairs, their scan, stable placement, ranges. Same lists as the full sort.
swf_status Ctx::lists_binned(Workspace& w, const DevScene& d, int B, const Grid& g, hipStream_t st,
                             uint64_t key_cap, bool readback) {
    swf_status s;
    const int64_t nh = (int64_t)bin_hist_entries(B, d.n, g);
    if ((s = w.bins.reserve(this, (size_t)nh * sizeof(uint32_t) + 16, st))) return s;
    if ((s = w.scan.reserve(this, scan_scratch_bytes((int64_t)bin_scan_entries(B, d.n, g)) + 64, st))) return s;
    uint32_t* bins = (uint32_t*)w.bins.ptr;
    stage_begin(SWF_STAGE_SCAN, st);
    launch_bin_hist(w.rec, B, d.n, g, bins, w.cull_dev, st);
    launch_bin_offsets(B, d.n, g, bins, w.scan.ptr, w.total_dev, st);
    stage_end(st);
    uint64_t nk;
    const uint64_t* n_dev;
    if ((s = key_count(w, st, key_cap, nk, n_dev, readback))) return s;
    if ((s = w.vals.reserve(this, nk * 4 + 16, st))) return s;
    stage_begin(SWF_STAGE_SORT, st);
    launch_bin_scatter(w.rec, B, d.n, g, bins, n_dev, (uint32_t*)w.vals.ptr, st);
    stage_end(st);
    stage_begin(SWF_STAGE_RANGES, st);
    launch_bin_ranges(bins, B, d.n, g, w.total_dev, n_dev, (uint2*)w.ranges.ptr, st);
    stage_end(st);
    w.last.n_keys = nk;
    w.last.full = false;
    w.last.binned = true;
    w.last.keys = nullptr;
    w.last.vals = (uint32_t*)w.vals.ptr;
    return SWF_OK;
}

// Lists by key emission and LSD radix sort: on the global tile id (stable; the
// pairs are already in depth order), or with SWF_FULL_SORT on the full 64-bit
// (tile, depth) key.
swf_status Ctx::lists_sorted(Workspace& w, const DevScene& d, int B, const Grid& g, bool full, hipStream_t st,
                             uint64_t key_cap) {
    swf_status s;
    const int64_t pairs = (int64_t)B * d.n;
    if ((s = w.off.reserve(this, (size_t)pairs * sizeof(uint32_t) + 16, st))) return s;
    if ((s = w.scan.reserve(this, scan_scratch_bytes(pairs) + 64, st))) return s;
    stage_begin(SWF_STAGE_SCAN, st);
    launch_exclusive_scan(w.rec.count, (uint32_t*)w.off.ptr, w.total_dev, pairs, w.scan.ptr, st);
    stage_end(st);
    uint64_t nk;
    const uint64_t* n_dev;
    if ((s = key_count(w, st, key_cap, nk, n_dev))) return s;
    const size_t kb = full ? 8 : 4;
    if ((s = w.keys.reserve(this, nk * kb + 16, st))) return s;
    if ((s = w.keys2.reserve(this, nk * kb + 16, st))) return s;
    if ((s = w.vals.reserve(this, nk * 4 + 16, st))) return s;
    if ((s = w.vals2.reserve(this, nk * 4 + 16, st))) return s;
    if ((s = w.hist.reserve(this, radix_scratch_bytes((int64_t)nk) + 64, st))) return s;
    const int64_t n_gt = (int64_t)B * g.tiles;
    stage_begin(SWF_STAGE_EMIT, st);
    launch_emit_keys(w.rec, (const uint32_t*)w.off.ptr, d.dbits, B, d.n, g, nk, full, w.keys.ptr,
                     (uint32_t*)w.vals.ptr, w.status_dev, w.cull_dev, st);
    stage_end(st);
    const int tbits = bits_for((uint64_t)n_gt);
    stage_begin(SWF_STAGE_SORT, st);
    const int flip = launch_radix_sort(w.keys.ptr, (uint32_t*)w.vals.ptr, w.keys2.ptr, (uint32_t*)w.vals2.ptr,
                                       (int64_t)nk, (int)kb, 0, full ? 32 + tbits : tbits, w.hist.ptr, st, n_dev);
    stage_end(st);
    void* skeys = flip ? w.keys2.ptr : w.keys.ptr;
    uint32_t* svals = (uint32_t*)(flip ? w.vals2.ptr : w.vals.ptr);
    stage_begin(SWF_STAGE_RANGES, st);
    launch_tile_ranges(skeys, (int)kb, (int64_t)nk, n_gt, (uint2*)w.ranges.ptr, st, n_dev);
    stage_end(st);
    w.last.n_keys = nk;
    w.last.full = full;
    w.last.binned = false;
    w.last.keys = skeys;
    w.last.vals = svals;
    return SWF_OK;
}

swf_status Ctx::render(Workspace& w, int sid, const float* tx, int B, int flags, float* out, void* aux,
                       hipStream_t st, uint64_t key_cap, bool speculate, float* chan, int rH, int rW) {
    if (!out) return fail(SWF_E_INVALID, "out is NULL");
    if ((flags & SWF_KEEP_AUX) && !aux) return fail(SWF_E_INVALID, "SWF_KEEP_AUX needs aux");
    if ((flags & SWF_KEEP_AUX) && (rH > 0 || rW > 0)) {
        Scene* sc0 = scene(sid);
        if (sc0 && ((rH > 0 && rH != sc0->d.H) || (rW > 0 && rW != sc0->d.W)))
            return fail(SWF_E_INVALID, "SWF_KEEP_AUX (the backward) needs the scene's own grid");
    }
    hipSetDevice(device);
    const uint64_t spec_cap = speculate && key_cap == 0 && w.vals.cap >= 16 + 4 * 4096 ? (w.vals.cap - 16) / 4 : 0;
    bool spec = false;
    // a render whose state the backward will need keeps its records and lists in the workspace, and the hidden
    // activations, stored by the MLP kernel (what the backward's GEMMs take)
    const bool keep = (flags & SWF_KEEP_AUX) && &w == &ws;
    bool keep_acts = false;
    swf_status s;
    if (keep) {
        Scene* sc0 = scene(sid);
        if (sc0 && sc0->d.kind == 0 && sc0->d.has_mlp && !(flags & SWF_NO_DEFORM) &&
            (uint64_t)B * (uint64_t)sc0->d.n < (1ull << 32)) {
            const size_t esz = (flags & SWF_MLP_BF16) ? sizeof(uint16_t) : sizeof(float);
            const size_t actb = (size_t)B * sc0->d.n * 256 * esz;
            if ((s = w.act.reserve(this, actb * sc0->d.n_hidden + 16, st))) return s;
            w.act_out = w.act.ptr;
            keep_acts = true;
        }
    }
    s = forward_lists(w, sid, tx, B, flags, st, key_cap, spec_cap, &spec, rH, rW);
    w.act_out = nullptr;
    if (s == SWF_E_OVERFLOW && B > 1 && key_cap == 0 && !(flags & SWF_KEEP_AUX)) {
        // more list entries (or pairs) than one launch sequence addresses: the first half of the queries, then
        // the rest (each split again if needed); the outputs are per query, so they land where one launch puts them
        Scene* sc1 = scene(sid);
        const int oH = rH > 0 ? rH : sc1->d.H, oW = rW > 0 ? rW : sc1->d.W;
        const int b1 = B / 2;
        const size_t plane = (size_t)oH * oW;
        s = render(w, sid, tx, b1, flags, out, nullptr, st, 0, false, chan, rH, rW);
        if (!s)
            s = render(w, sid, tx ? tx + (size_t)3 * b1 : nullptr, B - b1, flags, out + (size_t)b1 * plane, nullptr,
                       st, 0, false, chan ? chan + (size_t)b1 * 2 * plane : nullptr, rH, rW);
        if (!s) w.last.chunked = true;
        return s;
    }
    if (s) return s;
    const DevScene& d = scene(sid)->d;
    float* auxT = nullptr;
    uint32_t* auxL = nullptr;
    if (keep) {
        AuxTag t;
        t.scene = sid;
        t.B = B;
        t.flags = flags & ~(SWF_KEEP_AUX | SWF_DETERMINISTIC);
        t.gen = scene(sid)->gen;
        t.seq = w.seq;
        t.tx = tx;
        t.acts = keep_acts;
        tag_aux(aux, t);
    }
    if (flags & SWF_KEEP_AUX) {
        auxT = (float*)aux;
        auxL = (uint32_t*)((char*)aux + sizeof(float) * (size_t)B * d.H * d.W);
    }
    stage_begin(SWF_STAGE_BLEND, st);
    if (d.kind == 1)
        launch_gmm_blend((const uint2*)w.ranges.ptr, w.last.vals, w.rec, B, w.last.grid, out, chan, st);
    else
        launch_blend_forward((const uint2*)w.ranges.ptr, w.last.vals, w.rec, B, w.last.grid, out, auxT, auxL, st);
    stage_end(st);
    if ((s = hip(hipGetLastError(), "render launch"))) return s;
    if (spec) {
        // the GPU runs the lists and the blend while the count comes back
        if ((s = hip(hipEventSynchronize(w.total_ev), "total event"))) return s;
        const uint64_t total = *w.total_host;
        if (total > spec_cap) {
            // did not fit: nothing was placed and the spectrum is zero; again at the exact size
            s = render(w, sid, tx, B, flags, out, aux, st, 0, false, chan, rH, rW);
            w.last.rerenders = 1;
            return s;
        }
        w.last.n_keys = total;
    }
    return SWF_OK;
}

// Queries over several resident scenes in one launch sequence: per-query TX
// term, BF16 MLP (or static preprocess) over the batch's tiles of pairs, one
// scan over all records, key emission with per-query tile bases, one radix sort
// over every global tile, ranges, and the blend with per-query grids and output
// offsets. plan_mixed validates the batch and writes its tables into the
// workspace's pinned staging (a fixed layout: kMixScenes scene slots, then
// B_cap + 1 queries, the ones past B empty); enqueue_mixed copies them to the
// device and launches the stages, either exactly sized (one wait for the key
// count) or at fixed capacities with no host wait (graph-capturable: a replay
// copies whatever tables the staging holds by then).
swf_status Ctx::plan_mixed(Workspace& w, const int32_t* scene_ids, int B, int flags, int B_cap, MixPlan& p) {
    p = MixPlan{};  // a caller may hand in the previous batch's plan
    if (B < 1 || B > 65535 || B_cap < B || !scene_ids) return fail(SWF_E_INVALID, "bad batch or scene ids");
    const bool deform = !(flags & SWF_NO_DEFORM);
    if (flags & ~(SWF_MLP_BF16 | SWF_NO_DEFORM | SWF_PAPER_DEFORM))
        return fail(SWF_E_INVALID, "mixed batches take SWF_MLP_BF16 (else the FP32 MLP) or SWF_NO_DEFORM, and "
                                   "SWF_PAPER_DEFORM");
    std::vector<MixScene> sc;
    std::map<int, int> index;
    std::vector<MixQuery> q(B_cap + 1);
    int64_t pairs = 0, tiles = 0, outs = 0, mtiles = 0;
    p.out_off.assign(B + 1, 0);
    for (int b = 0; b < B; ++b) {
        Scene* s = scene(scene_ids[b]);
        if (!s) return fail(SWF_E_NOT_FOUND, "unknown scene id in a mixed batch");
        const DevScene& d = s->d;
        if (d.kind != 0) return fail(SWF_E_INVALID, "mixed batches hold compositing-model scenes");
        if (deform && (!d.has_mlp || d.n_hidden != 4 || d.hidden != 256))
            return fail(SWF_E_INVALID, "mixed deformable batches need scenes with a 4 x 256 MLP");
        auto it = index.find(scene_ids[b]);
        if (it == index.end()) {
            if ((int)sc.size() == kMixScenes) return fail(SWF_E_INVALID, "more than 64 scenes in a mixed batch");
            MixScene m{};
            m.mx = d.mx; m.my = d.my; m.lsx = d.lsx; m.lsy = d.lsy; m.rot = d.rot; m.logit = d.logit; m.amp = d.amp;
            m.w1 = d.w[0];
            m.b1 = d.b[0];
            m.stream = d.bf_stream;
            m.f32_frag = d.f32_frag;
            m.mfeat = d.bf_mfeat;
            for (int l = 0; l + 1 < d.n_hidden && l < 7; ++l) m.bias_h[l] = d.b[l + 1];
            m.bias_o = d.has_mlp ? d.b[d.n_hidden] : nullptr;
            for (int k = 0; k < 3; ++k) {
                m.room_lo[k] = d.room_lo[k];
                m.room_hi[k] = d.room_hi[k];
            }
            const Grid g = make_grid(d.H, d.W, 16);
            m.N = d.n;
            m.n_live = d.n_live;
            m.H = d.H;
            m.W = d.W;
            m.TW = g.TW;
            m.TH = g.TH;
            m.tiles = g.tiles;
            it = index.emplace(scene_ids[b], (int)sc.size()).first;
            sc.push_back(m);
        }
        const MixScene& m = sc[it->second];
        q[b] = MixQuery{it->second, (int)pairs, (int)tiles, (int)outs, (int)mtiles};
        p.out_off[b] = (uint64_t)outs;
        p.max_n = std::max(p.max_n, m.N);
        p.max_tiles = std::max(p.max_tiles, m.tiles);
        pairs += m.N;
        tiles += m.tiles;
        outs += (int64_t)m.H * m.W;
        mtiles += (m.N + 383) / 384;
        p.nan_pairs += (uint64_t)(d.n - d.n_live);
    }
    if (pairs >= (1ll << 31) || tiles >= (1ll << 31) || outs >= (1ll << 31))
        return fail(SWF_E_INVALID, "mixed batch too large");
    for (int b = B; b <= B_cap; ++b) q[b] = MixQuery{0, (int)pairs, (int)tiles, (int)outs, (int)mtiles};
    p.out_off[B] = (uint64_t)outs;
    p.B = B;
    p.B_cap = B_cap;
    p.pairs = pairs;
    p.tiles = tiles;
    p.outs = outs;
    p.first_scene = scene_ids[0];
    const size_t qoff = ((size_t)kMixScenes * sizeof(MixScene) + 255) & ~(size_t)255;
    p.query_off = qoff;
    p.table_bytes = qoff + (size_t)(B_cap + 1) * sizeof(MixQuery);
    if (w.mix_host_cap < p.table_bytes) {
        if (w.mix_host) {
            hipDeviceSynchronize();  // a previous copy may still read the old staging
            hipHostFree(w.mix_host);
        }
        w.mix_host = nullptr;
        w.mix_host_cap = 0;
        if (hipHostMalloc(&w.mix_host, p.table_bytes, 0) != hipSuccess) return fail(SWF_E_OOM, "hipHostMalloc(mix)");
        w.mix_host_cap = p.table_bytes;
    }
    std::memset(w.mix_host, 0, qoff);
    std::memcpy(w.mix_host, sc.data(), sc.size() * sizeof(MixScene));
    std::memcpy((char*)w.mix_host + qoff, q.data(), q.size() * sizeof(MixQuery));
    return SWF_OK;
}

swf_status Ctx::enqueue_mixed(Workspace& w, const MixPlan& p, const float* tx, int flags, float* out, hipStream_t st,
                              const MixCaps* caps, bool copy_tables) {
    if (!out) return fail(SWF_E_INVALID, "out is NULL");
    const bool deform = !(flags & SWF_NO_DEFORM);
    if (deform && !tx) return fail(SWF_E_INVALID, "tx is NULL");
    MixCaps k;
    if (caps) {
        k = *caps;
        if (k.B_cap != p.B_cap || k.pair_cap < p.pairs || k.tile_cap < p.tiles || k.bin_n < p.max_n ||
            k.bin_tiles < p.max_tiles || k.key_cap == 0)
            return fail(SWF_E_INVALID, "mixed batch exceeds its capacities");
    } else {
        k.B_cap = p.B_cap;
        k.pair_cap = p.pairs;
        k.tile_cap = p.tiles;
        k.bin_n = p.max_n;
        k.bin_tiles = p.max_tiles;
    }
    const int64_t pair_cap = k.pair_cap, tile_cap = k.tile_cap;
    // lists by binning (per query, the geometry of the largest), else by key emission and radix sort
    const bool binned = mix_bin_fits(k.B_cap, k.bin_tiles);
    swf_status s;
    if ((s = w.mix.reserve(this, p.table_bytes, st))) return s;
    if (copy_tables &&
        (s = hip(hipMemcpyAsync(w.mix.ptr, w.mix_host, p.table_bytes, hipMemcpyHostToDevice, st), "mix tables")))
        return s;
    ++w.seq;  // the records and lists are about to change
    MixBatch mb;
    mb.scenes = (const MixScene*)w.mix.ptr;
    mb.queries = (const MixQuery*)((char*)w.mix.ptr + p.query_off);
    mb.B = p.B_cap;
    // records
    if ((s = w.geo.reserve(this, pair_cap * sizeof(float4) + 16, st))) return s;
    if ((s = w.wm.reserve(this, pair_cap * sizeof(float4) + 16, st))) return s;
    if ((s = w.oa.reserve(this, pair_cap * sizeof(float2) + 16, st))) return s;
    if ((s = w.rect.reserve(this, pair_cap * sizeof(uint2) + 16, st))) return s;
    if ((s = w.count.reserve(this, pair_cap * sizeof(uint32_t) + 16, st))) return s;
    w.rec.geo = (float4*)w.geo.ptr;
    w.rec.wm = (float4*)w.wm.ptr;
    w.rec.oa = (float2*)w.oa.ptr;
    w.rec.rect = (uint2*)w.rect.ptr;
    w.rec.count = (uint32_t*)w.count.ptr;
    w.last.valid = false;
    w.last.stream = st;
    launch_clear_u32(w.status_dev, 8, st);
    stage_begin(SWF_STAGE_MLP, st);
    if (deform) {
        if ((s = w.qs.reserve(this, (size_t)p.B_cap * 256 * sizeof(float), st))) return s;
        launch_mix_tx_features(mb, tx, (float*)w.qs.ptr, st);
        if (flags & SWF_MLP_BF16)
            launch_mix_mlp_bf16(mb, (const float*)w.qs.ptr, w.rec, st, (flags & SWF_PAPER_DEFORM) != 0, false);
        else
            launch_mix_mlp_fp32(mb, (const float*)w.qs.ptr, w.rec, pair_cap, k.B_cap, st,
                                (flags & SWF_PAPER_DEFORM) != 0, false);
        // rows past the batch's pairs: no tiles (the scan of the sort path reads them)
        if (!binned) launch_mix_clear_tail(mb, pair_cap, w.rec, st);
    } else {
        launch_mix_static(mb, pair_cap, make_grid(16, 16, 16), w.rec, st);
    }
    stage_end(st);
    uint64_t nk;
    const uint64_t* n_dev;
    void* skeys = nullptr;
    uint32_t* svals = nullptr;
    if ((s = w.ranges.reserve(this, (size_t)tile_cap * sizeof(uint2) + 16, st))) return s;
    if (binned) {
        // tile histograms per block of pairs of each query, their scan, stable placement, ranges
        const int64_t nh = (int64_t)mix_bin_hist_entries(k.B_cap, k.bin_n, k.bin_tiles);
        const int64_t ns = (int64_t)mix_bin_scan_entries(k.B_cap, k.bin_n, k.bin_tiles);
        if ((s = w.bins.reserve(this, (size_t)nh * sizeof(uint32_t) + 16, st))) return s;
        if ((s = w.scan.reserve(this, scan_scratch_bytes(ns) + 64, st))) return s;
        uint32_t* bins = (uint32_t*)w.bins.ptr;
        stage_begin(SWF_STAGE_SCAN, st);
        launch_mix_bin_hist(mb, k.bin_n, k.bin_tiles, w.rec, bins, w.cull_dev, st);
        launch_mix_bin_offsets(mb, k.bin_n, k.bin_tiles, bins, w.scan.ptr, w.total_dev, st);
        stage_end(st);
        if ((s = key_count(w, st, k.key_cap, nk, n_dev))) return s;
        if ((s = w.vals.reserve(this, nk * 4 + 16, st))) return s;
        stage_begin(SWF_STAGE_SORT, st);
        launch_mix_bin_scatter(mb, k.bin_n, k.bin_tiles, w.rec, bins, n_dev, (uint32_t*)w.vals.ptr, st);
        stage_end(st);
        stage_begin(SWF_STAGE_RANGES, st);
        launch_mix_bin_ranges(mb, k.bin_n, k.bin_tiles, bins, w.total_dev, n_dev, tile_cap, (uint2*)w.ranges.ptr,
                              st);
        stage_end(st);
        svals = (uint32_t*)w.vals.ptr;
    } else {
        // scan of every record's tile count, key emission, radix sort over the batch's global tiles, ranges
        if ((s = w.off.reserve(this, (size_t)pair_cap * sizeof(uint32_t) + 16, st))) return s;
        if ((s = w.scan.reserve(this, scan_scratch_bytes(pair_cap) + 64, st))) return s;
        stage_begin(SWF_STAGE_SCAN, st);
        launch_exclusive_scan(w.rec.count, (uint32_t*)w.off.ptr, w.total_dev, pair_cap, w.scan.ptr, st);
        stage_end(st);
        if ((s = key_count(w, st, k.key_cap, nk, n_dev))) return s;
        if ((s = w.keys.reserve(this, nk * 4 + 16, st))) return s;
        if ((s = w.keys2.reserve(this, nk * 4 + 16, st))) return s;
        if ((s = w.vals.reserve(this, nk * 4 + 16, st))) return s;
        if ((s = w.vals2.reserve(this, nk * 4 + 16, st))) return s;
        if ((s = w.hist.reserve(this, radix_scratch_bytes((int64_t)nk) + 64, st))) return s;
        stage_begin(SWF_STAGE_EMIT, st);
        launch_mix_emit_keys(mb, w.rec, (const uint32_t*)w.off.ptr, pair_cap, nk, (uint32_t*)w.keys.ptr,
                             (uint32_t*)w.vals.ptr, w.status_dev, w.cull_dev, st);
        stage_end(st);
        stage_begin(SWF_STAGE_SORT, st);
        const int flip = launch_radix_sort(w.keys.ptr, (uint32_t*)w.vals.ptr, w.keys2.ptr, (uint32_t*)w.vals2.ptr,
                                           (int64_t)nk, 4, 0, bits_for((uint64_t)tile_cap), w.hist.ptr, st, n_dev);
        stage_end(st);
        skeys = flip ? w.keys2.ptr : w.keys.ptr;
        svals = (uint32_t*)(flip ? w.vals2.ptr : w.vals.ptr);
        stage_begin(SWF_STAGE_RANGES, st);
        launch_tile_ranges(skeys, 4, (int64_t)nk, tile_cap, (uint2*)w.ranges.ptr, st, n_dev);
        stage_end(st);
    }
    stage_begin(SWF_STAGE_BLEND, st);
    launch_mix_blend(mb, (int)tile_cap, (const uint2*)w.ranges.ptr, svals, w.rec, out, st);
    stage_end(st);
    // the last render, as the status query sees it: one "query" holding every pair of the batch
    w.last.valid = true;
    w.last.scene = p.first_scene;
    w.last.B = 1;
    w.last.N = (int)p.pairs;
    w.last.flags = flags;
    w.last.grid = make_grid(16, 16, 16);
    w.last.grid.tiles = (int)p.tiles;
    w.last.n_keys = nk;
    w.last.full = false;
    w.last.binned = binned;
    w.last.keys = skeys;
    w.last.vals = svals;
    w.last.rerenders = 0;
    w.last.nan_depth_pairs = p.nan_pairs;
    return hip(hipGetLastError(), "mixed render");
}

swf_status Ctx::render_mixed(Workspace& w, const int32_t* scene_ids, const float* tx, int B, int flags, float* out,
                             uint64_t* out_offsets, hipStream_t st) {
    if (!out) return fail(SWF_E_INVALID, "out is NULL");
    // the staging is about to be rewritten: the previous mixed batch's table copy must be done
    if (w.mix_host && w.last.stream) {
        swf_status s = hip(hipStreamSynchronize(w.last.stream), "stream sync");
        if (s) return s;
    }
    MixPlan p;
    swf_status s = plan_mixed(w, scene_ids, B, flags, B, p);
    if (s) return s;
    if (out_offsets)
        for (int b = 0; b <= B; ++b) out_offsets[b] = p.out_off[b];
    return enqueue_mixed(w, p, tx, flags, out, st);
}

}  // namespace swf

// ============================================================================
// C ABI
// ============================================================================
#define CTX_GUARD(c)                                               \
    if (!(c)) return SWF_E_INVALID;                                \
    std::lock_guard<std::recursive_mutex> _lock((c)->mu);          \
    hipSetDevice((c)->device)

extern "C" {

const char* swf_status_string(swf_status s) { return swf::status_name(s); }

swf_status swf_create(swf_ctx** out, const swf_config* cfg) {
    if (!out) return SWF_E_INVALID;
    *out = nullptr;
    int dev = cfg ? cfg->device : 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SWF_E_DEVICE;
    if (dev < 0 || dev >= ndev) return SWF_E_INVALID;
    if (hipSetDevice(dev) != hipSuccess) return SWF_E_DEVICE;
    Ctx* c = new (std::nothrow) Ctx();
    if (!c) return SWF_E_OOM;
    c->device = dev;
    c->mlp_pairs_per_wave = cfg ? cfg->mlp_pairs_per_wave : 0;
    if (cfg && cfg->max_list_entries) c->max_list_entries = cfg->max_list_entries;
    if (c->ws.init(c) != SWF_OK) {
        c->ws.release();
        delete c;
        return SWF_E_OOM;
    }
    if (noalloc_setup(c) != SWF_OK) {
        c->ws.release();
        delete c;
        return SWF_E_DEVICE;
    }
    *out = reinterpret_cast<swf_ctx*>(c);
    return SWF_OK;
}

swf_status swf_destroy(swf_ctx* h) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    hipSetDevice(c->device);
    serve_shutdown(c);
    hipDeviceSynchronize();
    for (auto& kv : c->scenes) {
        for (void* p : kv.second->allocs) hipFree(p);
        delete kv.second;
    }
    c->scenes.clear();
    c->ws.release();
    c->resolve_timing();
    for (auto e : c->event_pool) hipEventDestroy(e);
    delete c;
    return SWF_OK;
}

const char* swf_last_error(swf_ctx* h) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    return c ? c->err.c_str() : "null context";
}

swf_status swf_scene_upload(swf_ctx* h, const swf_gaussians* g, const swf_mlp* mlp, int32_t height, int32_t width,
                            int32_t src_is_device, int32_t* scene_id) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    return c->upload_scene(g, mlp, height, width, src_is_device != 0, scene_id);
}

swf_status swf_scene_update(swf_ctx* h, int32_t scene_id, const swf_gaussians* g, const swf_mlp* mlp,
                            int32_t src_is_device, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    return c->update_scene(scene_id, g, mlp, src_is_device != 0, (hipStream_t)stream);
}

swf_status swf_scene_release(swf_ctx* h, int32_t scene_id) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    return c->release_scene(scene_id);
}

swf_status swf_scene_bytes(swf_ctx* h, int32_t scene_id, uint64_t* bytes) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    Scene* s = c->scene(scene_id);
    if (!s) return c->fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (!bytes) return c->fail(SWF_E_INVALID, "bytes is NULL");
    *bytes = s->d.bytes;
    return SWF_OK;
}

swf_status swf_render(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch, int32_t flags, float* out,
                      void* aux, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    return c->render(c->ws, scene_id, tx, batch, flags, out, aux, (hipStream_t)stream, 0, true);
}

swf_status swf_scene_upload_paper(swf_ctx* h, const swf_paper_gaussians* g, const swf_paper_mlp* mlp,
                                  int32_t height, int32_t width, int32_t src_is_device, int32_t* scene_id) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    return c->upload_paper_scene(g, mlp, height, width, src_is_device != 0, scene_id);
}

swf_status swf_render_paper(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch, int32_t flags, float* out,
                            float* channels, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    Scene* sc = c->scene(scene_id);
    if (!sc) return c->fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (sc->d.kind != 1) return c->fail(SWF_E_INVALID, "not a paper-model scene");
    return c->render(c->ws, scene_id, tx, batch, flags, out, nullptr, (hipStream_t)stream, 0, true, channels);
}

swf_status swf_render_at(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch, int32_t height, int32_t width,
                         int32_t flags, float* out, void* aux, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (height < 1 || width < 1) return c->fail(SWF_E_INVALID, "height and width must lie in [1, 4096]");
    return c->render(c->ws, scene_id, tx, batch, flags, out, aux, (hipStream_t)stream, 0, true, nullptr, height,
                     width);
}

swf_status swf_render_mixed(swf_ctx* h, const int32_t* scene_ids, const float* tx, int32_t batch, int32_t flags,
                            float* out, uint64_t* out_offsets, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    return c->render_mixed(c->ws, scene_ids, tx, batch, flags, out, out_offsets, (hipStream_t)stream);
}

swf_status swf_stage_timing(swf_ctx* h, int32_t enable) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    c->resolve_timing();
    c->timing = enable != 0;
    return SWF_OK;
}

swf_status swf_stage_times(swf_ctx* h, double* ms, int64_t* launches, int32_t* n_stages) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (!n_stages) return c->fail(SWF_E_INVALID, "n_stages is NULL");
    c->resolve_timing();
    const int n = std::min<int>(*n_stages, SWF_N_STAGES);
    for (int i = 0; i < n; ++i) {
        if (ms) ms[i] = c->stage_ms[i];
        if (launches) launches[i] = c->stage_n[i];
        c->stage_ms[i] = 0.0;
        c->stage_n[i] = 0;
    }
    *n_stages = n;
    return SWF_OK;
}

swf_status swf_debug_deform(swf_ctx* h, int32_t scene_id, const float* tx, int32_t batch, int32_t flags, float* delta,
                            void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    Scene* sc = c->scene(scene_id);
    if (!sc) return c->fail(SWF_E_NOT_FOUND, "unknown scene id");
    if (batch < 1 || !delta || !tx) return c->fail(SWF_E_INVALID, "bad batch, delta or tx");
    if (flags & SWF_NO_DEFORM) return c->fail(SWF_E_INVALID, "deform debug needs the MLP");
    hipStream_t st = (hipStream_t)stream;
    const DevScene& d = sc->d;
    if (d.kind == 1) {
        // paper-model scene: 5 residuals per pair, already in id order
        const Grid g = make_grid(d.H, d.W, 16);
        swf_status s = c->enqueue_preprocess(c->ws, sc, tx, batch, flags, g, delta, st);
        c->ws.last.valid = false;
        return s ? s : c->hip(hipGetLastError(), "debug deform");
    }
    const size_t cnt = (size_t)batch * d.n * kOut;
    swf_status s = c->ws.delta.reserve(c, cnt * sizeof(float) + 16, st);
    if (s) return s;
    const Grid g = make_grid(d.H, d.W, (flags & SWF_TILE8) ? 8 : 16);
    s = c->enqueue_preprocess(c->ws, sc, tx, batch, flags, g, (float*)c->ws.delta.ptr, st);
    if (s) return s;
    launch_permute_delta((const float*)c->ws.delta.ptr, d.perm, batch, d.n, delta, st);
    c->ws.last.valid = false;
    return c->hip(hipGetLastError(), "debug deform");
}

swf_status swf_debug_relu_pattern(swf_ctx* h, uint8_t* pattern, uint64_t capacity) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (!pattern) return c->fail(SWF_E_INVALID, "pattern is NULL");
    const auto& L = c->last_mlp_bwd;
    if (!L.valid) return c->fail(SWF_E_STATE, "no MLP backward to inspect");
    Scene* sc = c->scene(L.scene);
    if (!sc) return c->fail(SWF_E_STATE, "scene of the last backward was released");
    const size_t pairs = (size_t)L.B * L.n, per = (size_t)L.layers * 256;
    if (capacity < pairs * per) return c->fail(SWF_E_OVERFLOW, "capacity below batch * n * layers * 256");
    swf_status s;
    if ((s = c->hip(hipDeviceSynchronize(), "device sync"))) return s;
    const size_t esz = L.bf16 ? 2 : 4, layer_bytes = pairs * 256 * esz;
    std::vector<uint8_t> a(layer_bytes);
    for (int l = 0; l < L.layers; ++l) {
        if ((s = c->hip(hipMemcpy(a.data(), (const char*)c->ws.act.ptr + layer_bytes * l, layer_bytes,
                                  hipMemcpyDeviceToHost),
                        "D2H activations")))
            return s;
        for (size_t i = 0; i < pairs; ++i) {
            const size_t q = i / L.n, id = sc->host_perm[i % L.n];
            uint8_t* o = pattern + ((q * L.n + id) * L.layers + l) * 256;
            for (int k = 0; k < 256; ++k) {
                // positive activation: BF16 sign bit clear and not zero; FP32 likewise
                if (L.bf16) {
                    uint16_t v;
                    std::memcpy(&v, a.data() + (i * 256 + k) * 2, 2);
                    o[k] = (v & 0x8000u) == 0 && (v & 0x7fffu) != 0;
                } else {
                    float v;
                    std::memcpy(&v, a.data() + (i * 256 + k) * 4, 4);
                    o[k] = v > 0.0f;
                }
            }
        }
    }
    return SWF_OK;
}

swf_status swf_debug_rects(swf_ctx* h, int32_t* rects, uint64_t capacity) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (!rects) return c->fail(SWF_E_INVALID, "rects is NULL");
    if (!c->ws.last.valid) return c->fail(SWF_E_STATE, "no render to inspect");
    Scene* sc = c->scene(c->ws.last.scene);
    if (!sc) return c->fail(SWF_E_STATE, "scene of the last render was released");
    const auto& L = c->ws.last;
    const size_t pairs = (size_t)L.B * L.N;
    if (capacity < pairs) return c->fail(SWF_E_OVERFLOW, "capacity below batch * n");
    swf_status s;
    if ((s = c->hip(hipStreamSynchronize(L.stream), "stream sync"))) return s;
    std::vector<uint32_t> r(2 * pairs), cnt(pairs);
    if (pairs && (s = c->hip(hipMemcpy(r.data(), c->ws.rec.rect, pairs * 8, hipMemcpyDeviceToHost), "D2H rects")))
        return s;
    if (pairs && (s = c->hip(hipMemcpy(cnt.data(), c->ws.rec.count, pairs * 4, hipMemcpyDeviceToHost), "D2H counts")))
        return s;
    for (size_t i = 0; i < pairs; ++i) {
        const size_t q = i / L.N, id = sc->host_perm[i % L.N];
        int32_t* o = rects + 4 * (q * L.N + id);
        if (!cnt[i]) {
            o[0] = o[1] = o[2] = o[3] = -1;
        } else {
            o[0] = (int32_t)(r[2 * i] & 0xffffu);
            o[1] = (int32_t)(r[2 * i + 1] & 0xffffu);
            o[2] = (int32_t)(r[2 * i] >> 16);
            o[3] = (int32_t)(r[2 * i + 1] >> 16);
        }
    }
    return SWF_OK;
}

swf_status swf_debug_keys(swf_ctx* h, uint32_t* counts, uint32_t* offsets, uint64_t* keys, uint64_t* values,
                          uint32_t* ranges, uint64_t* n_keys, uint64_t capacity) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (!c->ws.last.valid) return c->fail(SWF_E_STATE, "no render to inspect");
    Scene* sc = c->scene(c->ws.last.scene);
    if (!sc) return c->fail(SWF_E_STATE, "scene of the last render was released");
    hipDeviceSynchronize();
    const auto& L = c->ws.last;
    const size_t pairs = (size_t)L.B * L.N;
    if (n_keys) *n_keys = L.n_keys;
    swf_status s = SWF_OK;
    if (counts && (s = c->hip(hipMemcpy(counts, c->ws.rec.count, pairs * 4, hipMemcpyDeviceToHost), "D2H counts")))
        return s;
    if (offsets) {
        if (L.binned) {
            // the binning path never forms per-pair offsets: scan the counts here
            std::vector<uint32_t> cnt(pairs);
            if (pairs && (s = c->hip(hipMemcpy(cnt.data(), c->ws.rec.count, pairs * 4, hipMemcpyDeviceToHost),
                                     "D2H counts")))
                return s;
            uint32_t run = 0;
            for (size_t i = 0; i < pairs; ++i) {
                offsets[i] = run;
                run += cnt[i];
            }
        } else if ((s = c->hip(hipMemcpy(offsets, c->ws.off.ptr, pairs * 4, hipMemcpyDeviceToHost), "D2H offsets"))) {
            return s;
        }
    }
    if ((keys || values) && L.n_keys > capacity) return c->fail(SWF_E_OVERFLOW, "capacity below key count");
    if (keys || values) {
        std::vector<uint32_t> v(L.n_keys);
        if (L.n_keys && (s = c->hip(hipMemcpy(v.data(), L.vals, L.n_keys * 4, hipMemcpyDeviceToHost), "D2H vals")))
            return s;
        std::vector<uint64_t> k64(L.n_keys);
        if (L.binned) {
            // keys of the binned lists: the tile of each list position, from the ranges
            const size_t m = (size_t)L.B * L.grid.tiles;
            std::vector<uint32_t> rg(2 * m);
            if (m && (s = c->hip(hipMemcpy(rg.data(), c->ws.ranges.ptr, m * 8, hipMemcpyDeviceToHost), "D2H ranges")))
                return s;
            for (size_t t = 0; t < m; ++t)
                for (uint32_t i = rg[2 * t]; i < rg[2 * t + 1] && i < L.n_keys; ++i)
                    k64[i] = ((uint64_t)t << 32) | sc->host_dbits[v[i] % L.N];
        } else if (L.full) {
            if (L.n_keys && (s = c->hip(hipMemcpy(k64.data(), L.keys, L.n_keys * 8, hipMemcpyDeviceToHost), "D2H keys")))
                return s;
        } else {
            std::vector<uint32_t> k32(L.n_keys);
            if (L.n_keys && (s = c->hip(hipMemcpy(k32.data(), L.keys, L.n_keys * 4, hipMemcpyDeviceToHost), "D2H keys")))
                return s;
            for (uint64_t i = 0; i < L.n_keys; ++i)
                k64[i] = ((uint64_t)k32[i] << 32) | sc->host_dbits[v[i] % L.N];
        }
        for (uint64_t i = 0; i < L.n_keys; ++i) {
            if (keys) keys[i] = k64[i];
            if (values) values[i] = ((uint64_t)(v[i] / L.N) << 32) | sc->host_perm[v[i] % L.N];
        }
    }
    if (ranges) {
        const size_t m = (size_t)L.B * L.grid.tiles;
        if ((s = c->hip(hipMemcpy(ranges, c->ws.ranges.ptr, m * 8, hipMemcpyDeviceToHost), "D2H ranges"))) return s;
    }
    return SWF_OK;
}

swf_status swf_last_device_status(swf_ctx* h, swf_device_status* out) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!out) return SWF_E_INVALID;
    CTX_GUARD(c);
    Workspace& w = c->ws;
    if (!w.last.valid) return c->fail(SWF_E_STATE, "no render on this context yet");
    swf_status s;
    if ((s = c->hip(hipStreamSynchronize(w.last.stream), "stream sync"))) return s;
    uint32_t word = 0;
    unsigned long long cull[2] = {0, 0};
    if ((s = c->hip(hipMemcpy(&word, w.status_dev, sizeof(word), hipMemcpyDeviceToHost), "status D2H"))) return s;
    if ((s = c->hip(hipMemcpy(cull, w.cull_dev, sizeof(cull), hipMemcpyDeviceToHost), "status D2H"))) return s;
    std::memset(out, 0, sizeof(*out));
    out->flags = (word & 1u ? SWF_DEV_KEY_OVERFLOW : 0u) | (w.last.rerenders ? SWF_DEV_RERENDERED : 0u);
    out->rerenders = w.last.rerenders;
    out->pairs = (uint64_t)w.last.B * (uint64_t)w.last.N;
    out->culled_nonfinite = cull[0] + w.last.nan_depth_pairs;
    out->culled_offgrid = cull[1];
    out->list_entries = w.last.n_keys;
    if (out->culled_nonfinite) out->flags |= SWF_DEV_CULLED_NONFINITE;
    if (out->culled_offgrid) out->flags |= SWF_DEV_CULLED_OFFGRID;
    if (c->last_bwd_reused) out->flags |= SWF_DEV_BWD_REUSED;
    if (w.last.chunked) out->flags |= SWF_DEV_CHUNKED;
    return SWF_OK;
}

swf_status swf_debug_blend_work(swf_ctx* h, uint64_t* evaluations, uint64_t* staged, uint64_t* n_entries) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (!c->ws.last.valid) return c->fail(SWF_E_STATE, "no render to inspect");
    if (!c->scene(c->ws.last.scene)) return c->fail(SWF_E_STATE, "scene of the last render was released");
    const auto& L = c->ws.last;
    if (n_entries) *n_entries = L.n_keys;
    swf_status s = c->hip(hipDeviceSynchronize(), "sync");
    if (s) return s;
    if ((s = c->ws.work.reserve(c, 3 * sizeof(unsigned long long), nullptr))) return s;
    unsigned long long* d = (unsigned long long*)c->ws.work.ptr;
    launch_clear_u32((uint32_t*)d, 6, nullptr);
    launch_blend_work((const uint2*)c->ws.ranges.ptr, L.vals, c->ws.rec, L.B, L.grid, d, nullptr);
    unsigned long long hw[3] = {0, 0, 0};
    if ((s = c->hip(hipMemcpy(hw, d, sizeof(hw), hipMemcpyDeviceToHost), "D2H work"))) return s;
    if (evaluations) *evaluations = hw[0];
    if (staged) *staged = hw[1];
    c->last_blend_executed = hw[2];
    return SWF_OK;
}

swf_status swf_debug_blend_executed(swf_ctx* h, uint64_t* lane_evaluations) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (!lane_evaluations) return c->fail(SWF_E_INVALID, "lane_evaluations is NULL");
    uint64_t ev = 0, st = 0, ne = 0;
    swf_status s = swf_debug_blend_work(h, &ev, &st, &ne);
    if (s) return s;
    *lane_evaluations = c->last_blend_executed;
    return SWF_OK;
}

swf_status swf_measure_peaks(swf_ctx* h, double* mfma_bf16_tflops, double* fma_tops, double* lds_tbps) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    const int blocks = n_compute_units();
    swf_status s = c->hip(hipDeviceSynchronize(), "sync");
    if (s) return s;
    if ((s = c->ws.work.reserve(c, probe_scratch_bytes(blocks), nullptr))) return s;
    if ((s = c->hip(run_probes(blocks, c->ws.work.ptr, nullptr, mfma_bf16_tflops, fma_tops, lds_tbps), "probes")))
        return s;
    return c->hip(hipDeviceSynchronize(), "sync");
}

swf_status swf_radix_sort(swf_ctx* h, void* keys, uint32_t* values, int64_t n, int32_t key_bytes, int32_t begin_bit,
                          int32_t end_bit, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (n < 0 || (n > 0 && (!keys || !values))) return c->fail(SWF_E_INVALID, "bad keys/values/n");
    if (key_bytes != 4 && key_bytes != 8) return c->fail(SWF_E_INVALID, "key_bytes must be 4 or 8");
    if (begin_bit < 0 || end_bit > 8 * key_bytes || begin_bit > end_bit)
        return c->fail(SWF_E_INVALID, "bad bit range");
    if (n >= (1ll << 32)) return c->fail(SWF_E_INVALID, "n must be < 2^32");
    hipStream_t st = (hipStream_t)stream;
    swf_status s = SWF_OK;
    if ((s = c->ws.sortk.reserve(c, (size_t)n * key_bytes + 16, st))) return s;
    if ((s = c->ws.sortv.reserve(c, (size_t)n * 4 + 16, st))) return s;
    if ((s = c->ws.hist.reserve(c, radix_scratch_bytes(n) + 64, st))) return s;
    c->ws.last.valid = false;
    const int flip = launch_radix_sort(keys, values, c->ws.sortk.ptr, (uint32_t*)c->ws.sortv.ptr, n, key_bytes,
                                       begin_bit, end_bit, c->ws.hist.ptr, st);
    if (flip) {
        hipMemcpyAsync(keys, c->ws.sortk.ptr, (size_t)n * key_bytes, hipMemcpyDeviceToDevice, st);
        hipMemcpyAsync(values, c->ws.sortv.ptr, (size_t)n * 4, hipMemcpyDeviceToDevice, st);
    }
    return c->hip(hipGetLastError(), "radix sort");
}

swf_status swf_exclusive_scan(swf_ctx* h, const uint32_t* counts, uint32_t* offsets, uint64_t* total, int64_t n,
                              void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    CTX_GUARD(c);
    if (n < 0 || !total || (n > 0 && (!counts || !offsets))) return c->fail(SWF_E_INVALID, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    swf_status s = c->ws.scan.reserve(c, scan_scratch_bytes(n) + 64, st);
    if (s) return s;
    launch_exclusive_scan(counts, offsets, total, n, c->ws.scan.ptr, st);
    return c->hip(hipGetLastError(), "scan");
}

}  // extern "C"
