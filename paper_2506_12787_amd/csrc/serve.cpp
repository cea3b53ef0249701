// Serving loop: continuous batching of spectrum queries over resident scenes.
//
// Requests (scene, tx) are queued by any thread. A scheduler thread owns
// `n_slots` execution slots; each slot has its own stream and workspace, so
// the launches of different slots overlap on the device. Whenever a slot is
// free, the scheduler admits a batch and replays a captured graph of its whole
// render (fixed capacities, no host sync), then queues the result and status
// download and a completion event. Completed slots are refilled immediately
// (continuous batching).
//
// Per-scene mode: the oldest waiting request's scene, up to `max_batch` of its
// waiting requests (FIFO), padded to a power-of-two bucket; one graph per
// (scene, bucket). Mixed mode: the waiting requests in arrival order, of any
// scenes (at most 64 distinct) that share the oldest one's deformation mode,
// rendered as one mixed batch; its scene and query tables are planned on the
// host and copied ahead of the replay, so one graph serves every batch whose
// totals fit its capacities (queries, pairs, tiles, keys: each rounded up to
// four steps per octave). Scenes a mixed batch cannot hold (another MLP shape,
// the paper model) are served per scene.
//
// A graph is captured right after the eager render of the first batch that
// needs it (that render is the batch's result). Finished slots go to a
// delivery thread, which copies the results into the callers' buffers (after a
// key-capacity overflow, seen in the status word, it first re-renders the
// batch with exact sizing) and frees the slot; the scheduler keeps admitting
// into the other slots meanwhile.
//
// Admission is bounded by a device-memory budget over all slot workspaces (a
// batch that does not fit is shrunk, idle workspaces are released, or the
// requests wait). Latency is measured from the request's scheduled arrival
// time.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "runtime.h"

namespace swf {

double serve_clock() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    int scene = 0;
    float tx[3] = {0, 0, 0};
    float* out = nullptr;  // caller-owned host buffer of H*W floats
    double t_arrival = 0, t_launch = 0, t_done = 0;
    int state = 0;  // 0 waiting, 1 running, 2 done, < 0 error status
    int batch = 0, bucket = 0, fallback = 0, slot = -1;
};

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = 0;
    uint64_t key_cap = 0;
};

// A mixed batch's graph: flags and the capacities it was captured at.
using MixKey = std::tuple<int, int, int64_t, int64_t, uint64_t, int, int>;
MixKey mix_key(int flags, const MixCaps& k) {
    return std::make_tuple(flags, k.B_cap, k.pair_cap, k.tile_cap, k.key_cap, k.bin_n, k.bin_tiles);
}

struct Slot {
    int index = 0;
    hipStream_t stream = nullptr;
    Workspace ws;
    Buf tx_dev, out_dev;
    float* tx_host = nullptr;   // pinned, max_batch * 3
    float* out_host = nullptr;  // pinned, grows
    size_t out_host_cap = 0;
    uint32_t* status_host = nullptr;
    hipEvent_t done = nullptr;
    std::atomic<int> phase{0};  // 0 free, 1 rendering, 2 results being delivered
    bool busy() const { return phase.load() != 0; }
    int scene = -1, bucket = 0;
    std::vector<Request*> reqs;
    std::map<std::pair<int, int>, GraphEntry> graphs;
    // mixed batches
    bool mixed = false;
    int mix_flags = 0;
    MixPlan plan;
    std::vector<int32_t> ids;
    std::map<MixKey, GraphEntry> mgraphs;
    std::map<int, MixCaps> mix_hw;  // per B_cap: the largest capacities launched so far (its graph's)
};

struct ServeState {
    swf_serve_config cfg{};
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Request*> waiting;
    std::unordered_map<uint64_t, Request*> table;
    uint64_t next_ticket = 1;
    std::vector<Slot*> slots;
    std::map<int, uint64_t> keys_per_query;  // calibrated per scene
    Workspace cal;                           // mixed mode: calibration renders, released after each
    std::atomic<uint64_t> launched{0}, completed{0}, fallbacks{0}, graph_builds{0}, shrinks{0};
    std::atomic<uint64_t> mixed_launches{0}, mixed_scenes{0};
    // delivery: finished slots whose results go to the callers' buffers (and, after a key overflow, are
    // re-rendered first) on a thread of their own, so that the scheduler keeps admitting meanwhile
    std::thread deliverer;
    std::mutex dmu;
    std::condition_variable dcv;
    std::deque<Slot*> finished;
    bool dstop = false;
};

namespace {

thread_local bool t_no_timing = false;

uint64_t slot_bytes(Slot* s) {
    uint64_t b = 0;
    for (Buf* x : s->ws.bufs()) b += x->cap;
    return b + s->tx_dev.cap + s->out_dev.cap;
}

void drop_graphs(Slot* s) {
    for (auto& kv : s->graphs)
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    s->graphs.clear();
    for (auto& kv : s->mgraphs)
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    s->mgraphs.clear();
    s->mix_hw.clear();
}

int pow2_at_least(int64_t x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// x rounded up to one of four steps per octave (5/8, 6/8, 7/8, 8/8 of the next power of two), at least `lo`.
int64_t round_cap(int64_t x, int64_t lo) {
    x = std::max(x, lo);
    int64_t p = 1;
    while (p < x) p <<= 1;
    const int64_t step = std::max<int64_t>(p / 8, 1);
    return (x + step - 1) / step * step;
}

// Upper bound of a slot's workspace for a mixed batch at these capacities
// (the terms of estimate_bytes below, at the batch's totals).
uint64_t estimate_mixed_bytes(const MixCaps& k) {
    const uint64_t raw = (uint64_t)k.pair_cap * 56 + k.key_cap * 16 + (uint64_t)k.tile_cap * 8 +
                         (uint64_t)k.outs * 4 + (uint64_t)k.B_cap * (256 * 4 + 1024) + (uint64_t)k.pair_cap / 64 +
                         mix_bin_hist_entries(k.B_cap, k.bin_n, k.bin_tiles) * 4 + (1u << 20);
    return raw + raw / 4 + 64 * 256;
}

// Upper bound of a slot's workspace for (scene, bucket, key capacity): records
// (52 B) + offsets (4 B) per pair, keys and values double-buffered (16 B per
// key), tile ranges, output and TX, per-query MLP state, binning histogram,
// scan/sort scratch;
// times the 1.25 growth factor of the buffers.
uint64_t estimate_bytes(const DevScene& d, int bucket, uint64_t key_cap) {
    const uint64_t pairs = (uint64_t)bucket * d.n;
    const uint64_t tiles = (uint64_t)bucket * ((d.W + 15) / 16) * ((d.H + 15) / 16);
    // binning histogram bounded with the finer (8-pixel) tiling
    const uint64_t bins = bin_hist_entries(bucket, d.n, make_grid(d.H, d.W, 8)) * 4;
    const uint64_t raw = pairs * 56 + key_cap * 16 + tiles * 8 + (uint64_t)bucket * ((uint64_t)d.H * d.W * 4 + 1024) +
                         (uint64_t)bucket * 256 * 4 + bins + (1u << 20);
    return raw + raw / 4 + 64 * 256;
}

}  // namespace

bool serve_timing_disabled() { return t_no_timing; }

// Render `count` requests of one scene on a slot (padded to `bucket`).
static swf_status launch_batch(Ctx* c, ServeState* S, Slot* sl, int scene, std::vector<Request*>& reqs, int bucket) {
    Scene* sc = c->scene(scene);
    if (!sc) return SWF_E_NOT_FOUND;
    const DevScene& d = sc->d;
    const int count = (int)reqs.size();
    int flags = S->cfg.flags & (SWF_MLP_BF16 | SWF_PAPER_DEFORM | SWF_TILE8);
    if (!d.has_mlp) flags |= SWF_NO_DEFORM;
    // inputs: pad with the last request's TX
    for (int i = 0; i < bucket; ++i) {
        const Request* r = reqs[std::min(i, count - 1)];
        std::memcpy(sl->tx_host + 3 * i, r->tx, sizeof(float) * 3);
    }
    const size_t out_floats = (size_t)bucket * d.H * d.W;
    swf_status s = SWF_OK;
    if ((s = sl->tx_dev.reserve(c, (size_t)bucket * 3 * sizeof(float), sl->stream))) return s;
    if ((s = sl->out_dev.reserve(c, out_floats * sizeof(float), sl->stream))) return s;
    if (sl->out_host_cap < out_floats) {
        if (sl->out_host) hipHostFree(sl->out_host);
        sl->out_host = nullptr;
        if (hipHostMalloc(&sl->out_host, out_floats * sizeof(float), 0) != hipSuccess) return SWF_E_OOM;
        sl->out_host_cap = out_floats;
    }
    uint64_t kpq = S->keys_per_query[scene];
    const uint64_t key_cap = (uint64_t)std::ceil((double)kpq * bucket * S->cfg.key_factor) + 4096;
    hipStream_t st = sl->stream;
    if ((s = c->hip(hipMemcpyAsync(sl->tx_dev.ptr, sl->tx_host, (size_t)bucket * 3 * sizeof(float),
                                   hipMemcpyHostToDevice, st),
                    "serve tx H2D")))
        return s;
    if (S->cfg.use_graphs) {
        auto key = std::make_pair(scene, bucket);
        GraphEntry& ge = sl->graphs[key];
        const uint64_t gen = sl->ws.generation() + sl->tx_dev.gen + sl->out_dev.gen;
        bool rendered = false;
        if (!ge.exec || ge.gen != gen || ge.key_cap != key_cap) {
            if (ge.exec) hipGraphExecDestroy(ge.exec);
            ge.exec = nullptr;
            // this batch renders eagerly, which sizes every buffer; the capture right after it records the same
            // launches for the next batches (it executes nothing, so it needs no wait for the eager work)
            if ((s = c->render(sl->ws, scene, (const float*)sl->tx_dev.ptr, bucket, flags, (float*)sl->out_dev.ptr,
                               nullptr, st, key_cap)))
                return s;
            rendered = true;
            hipGraph_t graph = nullptr;
            if ((s = c->hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture"))) return s;
            swf_status rs = c->render(sl->ws, scene, (const float*)sl->tx_dev.ptr, bucket, flags,
                                      (float*)sl->out_dev.ptr, nullptr, st, key_cap);
            hipError_t ce = hipStreamEndCapture(st, &graph);
            if (rs) return rs;
            if ((s = c->hip(ce, "end capture"))) return s;
            hipError_t ie = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if ((s = c->hip(ie, "graph instantiate"))) return s;
            ge.gen = sl->ws.generation() + sl->tx_dev.gen + sl->out_dev.gen;
            ge.key_cap = key_cap;
            ++S->graph_builds;
        }
        if (!rendered && (s = c->hip(hipGraphLaunch(ge.exec, st), "graph launch"))) return s;
    } else {
        if ((s = c->render(sl->ws, scene, (const float*)sl->tx_dev.ptr, bucket, flags, (float*)sl->out_dev.ptr,
                           nullptr, st, key_cap)))
            return s;
    }
    if ((s = c->hip(hipMemcpyAsync(sl->out_host, sl->out_dev.ptr, (size_t)count * d.H * d.W * sizeof(float),
                                   hipMemcpyDeviceToHost, st),
                    "serve out D2H")))
        return s;
    if ((s = c->hip(hipMemcpyAsync(sl->status_host, sl->ws.status_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, st),
                    "serve status D2H")))
        return s;
    if ((s = c->hip(hipEventRecord(sl->done, st), "serve event"))) return s;
    const double now = serve_clock();
    for (Request* r : reqs) {
        r->t_launch = now;
        r->batch = count;
        r->bucket = bucket;
        r->slot = sl->index;
        r->state = 1;
    }
    sl->phase = 1;
    sl->mixed = false;
    sl->scene = scene;
    sl->bucket = bucket;
    sl->reqs = reqs;
    ++S->launched;
    return SWF_OK;
}

// Exact-size re-render of a finished slot's requests after a key overflow.
static swf_status fallback_batch(Ctx* c, Slot* sl) {
    if (sl->mixed) {
        const int count = (int)sl->reqs.size();
        swf_status s = c->render_mixed(sl->ws, sl->ids.data(), (const float*)sl->tx_dev.ptr, count, sl->mix_flags,
                                       (float*)sl->out_dev.ptr, nullptr, sl->stream);
        if (s) return s;
        if ((s = c->hip(hipMemcpyAsync(sl->out_host, sl->out_dev.ptr, (size_t)sl->plan.outs * sizeof(float),
                                       hipMemcpyDeviceToHost, sl->stream),
                        "fallback D2H")))
            return s;
        return c->hip(hipStreamSynchronize(sl->stream), "fallback sync");
    }
    const DevScene& d = c->scene(sl->scene)->d;
    const int count = (int)sl->reqs.size();
    int flags = c->serve->cfg.flags & (SWF_MLP_BF16 | SWF_PAPER_DEFORM | SWF_TILE8);
    if (!d.has_mlp) flags |= SWF_NO_DEFORM;
    swf_status s = c->render(sl->ws, sl->scene, (const float*)sl->tx_dev.ptr, count, flags, (float*)sl->out_dev.ptr,
                             nullptr, sl->stream, 0);
    if (s) return s;
    if ((s = c->hip(hipMemcpyAsync(sl->out_host, sl->out_dev.ptr, (size_t)count * d.H * d.W * sizeof(float),
                                   hipMemcpyDeviceToHost, sl->stream),
                    "fallback D2H")))
        return s;
    return c->hip(hipStreamSynchronize(sl->stream), "fallback sync");
}

static void finish_slot(Ctx* c, ServeState* S, Slot* sl) {
    int fb = 0;
    size_t px = 0;
    {
        std::lock_guard<std::recursive_mutex> lk(c->mu);
        if (*sl->status_host != 0u) {
            // the next graph for these scenes gets a larger key capacity
            if (sl->mixed) {
                for (int id : std::set<int>(sl->ids.begin(), sl->ids.end()))
                    S->keys_per_query[id] = (uint64_t)(S->keys_per_query[id] * 1.5) + 1024;
            } else {
                S->keys_per_query[sl->scene] = (uint64_t)(S->keys_per_query[sl->scene] * 1.5) + 1024;
            }
            fb = fallback_batch(c, sl) == SWF_OK ? 1 : -1;
            ++S->fallbacks;
        }
        if (!sl->mixed) {
            const DevScene& d = c->scene(sl->scene)->d;
            px = (size_t)d.H * d.W;
        }
    }
    // results to the callers' buffers (the requests are in state "running": no
    // other thread touches them), then publish under the lock
    if (fb >= 0)
        for (size_t i = 0; i < sl->reqs.size(); ++i) {
            const size_t off = sl->mixed ? (size_t)sl->plan.out_off[i] : i * px;
            const size_t n = sl->mixed ? (size_t)(sl->plan.out_off[i + 1] - sl->plan.out_off[i]) : px;
            std::memcpy(sl->reqs[i]->out, sl->out_host + off, n * sizeof(float));
        }
    const double now = serve_clock();
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < sl->reqs.size(); ++i) {
        Request* r = sl->reqs[i];
        r->state = fb < 0 ? SWF_E_DEVICE : 2;
        r->fallback = fb > 0;
        r->t_done = now;
        ++S->completed;
    }
    sl->reqs.clear();
    sl->phase = 0;
    S->cv.notify_all();
}

// Mixed mode of a scene: 1 deformable (a 4 x 256 MLP, in the server's precision),
// 0 static (no MLP), -1 served per scene (another MLP shape or model, or flags a
// mixed batch does not take), -2 unknown.
static int mix_mode(Ctx* c, const ServeState* S, int id) {
    Scene* sc = c->scene(id);
    if (!sc) return -2;
    const DevScene& d = sc->d;
    if (d.kind != 0 || (S->cfg.flags & SWF_TILE8)) return -1;
    if (!d.has_mlp) return 0;
    return (d.n_hidden == 4 && d.hidden == 256) ? 1 : -1;
}

// Grow a slot's pinned output staging to n floats.
static swf_status reserve_out_host(Slot* sl, size_t n) {
    if (sl->out_host_cap >= n) return SWF_OK;
    if (sl->out_host) hipHostFree(sl->out_host);
    sl->out_host = nullptr;
    sl->out_host_cap = 0;
    if (hipHostMalloc(&sl->out_host, n * sizeof(float), 0) != hipSuccess) return SWF_E_OOM;
    sl->out_host_cap = n;
    return SWF_OK;
}

// Render a mixed batch on a slot: tables planned into the workspace's staging,
// TX (padded to B_cap with the last request's), tables and the graph of the
// launches at these capacities.
static swf_status launch_mixed(Ctx* c, ServeState* S, Slot* sl, std::vector<Request*>& reqs, int flags,
                               const MixCaps& k) {
    const int count = (int)reqs.size();
    sl->ids.resize(count);
    for (int i = 0; i < count; ++i) sl->ids[i] = reqs[i]->scene;
    swf_status s = c->plan_mixed(sl->ws, sl->ids.data(), count, flags, k.B_cap, sl->plan);
    if (s) return s;
    const MixPlan& p = sl->plan;
    for (int i = 0; i < k.B_cap; ++i) std::memcpy(sl->tx_host + 3 * i, reqs[std::min(i, count - 1)]->tx, 12);
    hipStream_t st = sl->stream;
    if ((s = sl->tx_dev.reserve(c, (size_t)k.B_cap * 3 * sizeof(float), st))) return s;
    if ((s = sl->out_dev.reserve(c, (size_t)k.outs * sizeof(float), st))) return s;
    if ((s = reserve_out_host(sl, (size_t)p.outs))) return s;
    if ((s = c->hip(hipMemcpyAsync(sl->tx_dev.ptr, sl->tx_host, (size_t)k.B_cap * 3 * sizeof(float),
                                   hipMemcpyHostToDevice, st),
                    "serve tx H2D")))
        return s;
    const float* tx = (const float*)sl->tx_dev.ptr;
    float* out = (float*)sl->out_dev.ptr;
    if (S->cfg.use_graphs) {
        GraphEntry& ge = sl->mgraphs[mix_key(flags, k)];
        auto gen = [&] { return sl->ws.generation() + sl->tx_dev.gen + sl->out_dev.gen; };
        bool rendered = false;
        if (!ge.exec || ge.gen != gen()) {
            if (ge.exec) hipGraphExecDestroy(ge.exec);
            ge.exec = nullptr;
            // this batch renders eagerly (tables copied), which sizes every buffer; the capture right after it
            // records the launches alone, for the next batches
            if ((s = c->enqueue_mixed(sl->ws, p, tx, flags, out, st, &k))) return s;
            rendered = true;
            hipGraph_t graph = nullptr;
            if ((s = c->hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture"))) return s;
            swf_status rs = c->enqueue_mixed(sl->ws, p, tx, flags, out, st, &k, false);
            hipError_t ce = hipStreamEndCapture(st, &graph);
            if (rs) return rs;
            if ((s = c->hip(ce, "end capture"))) return s;
            hipError_t ie = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if ((s = c->hip(ie, "graph instantiate"))) return s;
            ge.gen = gen();
            ge.key_cap = k.key_cap;
            ++S->graph_builds;
        }
        if (!rendered) {
            if ((s = c->hip(hipMemcpyAsync(sl->ws.mix.ptr, sl->ws.mix_host, p.table_bytes, hipMemcpyHostToDevice,
                                           st),
                            "mix tables H2D")))
                return s;
            if ((s = c->hip(hipGraphLaunch(ge.exec, st), "graph launch"))) return s;
        }
    } else {
        if ((s = c->enqueue_mixed(sl->ws, p, tx, flags, out, st, &k))) return s;
    }
    if ((s = c->hip(hipMemcpyAsync(sl->out_host, out, (size_t)p.outs * sizeof(float), hipMemcpyDeviceToHost, st),
                    "serve out D2H")))
        return s;
    if ((s = c->hip(hipMemcpyAsync(sl->status_host, sl->ws.status_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, st),
                    "serve status D2H")))
        return s;
    if ((s = c->hip(hipEventRecord(sl->done, st), "serve event"))) return s;
    const double now = serve_clock();
    for (Request* r : reqs) {
        r->t_launch = now;
        r->batch = count;
        r->bucket = k.B_cap;
        r->slot = sl->index;
        r->state = 1;
    }
    sl->phase = 1;
    sl->mixed = true;
    sl->mix_flags = flags;
    sl->scene = reqs[0]->scene;
    sl->bucket = k.B_cap;
    sl->reqs = reqs;
    ++S->launched;
    ++S->mixed_launches;
    S->mixed_scenes += std::set<int>(sl->ids.begin(), sl->ids.end()).size();
    return SWF_OK;
}

// Mixed-mode admission into a free slot. Returns 0 (nothing to admit), 1 (a
// batch launched or failed), 2 (the batch waits for memory) or 3 (the oldest
// request is served per scene).
static int admit_mixed(Ctx* c, ServeState* S, Slot* sl) {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    std::vector<Request*> batch;
    int mode;
    {
        std::lock_guard<std::mutex> lk2(S->mu);
        if (S->stop || S->waiting.empty()) return 0;
        mode = mix_mode(c, S, S->waiting.front()->scene);
        if (mode < 0) return 3;
        std::set<int> scenes;
        for (auto it = S->waiting.begin(); it != S->waiting.end() && (int)batch.size() < S->cfg.max_batch;) {
            const int id = (*it)->scene;
            if (mix_mode(c, S, id) == mode && (scenes.count(id) || (int)scenes.size() < kMixScenes)) {
                scenes.insert(id);
                batch.push_back(*it);
                it = S->waiting.erase(it);
            } else {
                ++it;
            }
        }
    }
    const int flags = mode ? (S->cfg.flags & (SWF_MLP_BF16 | SWF_PAPER_DEFORM)) : SWF_NO_DEFORM;
    swf_status st = SWF_OK;
    // calibrate the key count per query of each new scene once: exact-size lists of one query, in a workspace of
    // their own that is released afterwards (the slot's workspace holds only what its launches use, as the
    // memory budget counts it)
    bool calibrated = false;
    for (Request* r : batch) {
        if (st || S->keys_per_query.count(r->scene)) continue;
        if (!S->cal.total_dev) st = S->cal.init(c);
        if (!st) st = sl->tx_dev.reserve(c, 3 * sizeof(float), sl->stream);
        if (!st)
            st = c->hip(hipMemcpyAsync(sl->tx_dev.ptr, r->tx, 3 * sizeof(float), hipMemcpyHostToDevice, sl->stream),
                        "calibration tx");
        if (!st)
            st = c->forward_lists(S->cal, r->scene, (const float*)sl->tx_dev.ptr, 1, flags, sl->stream, 0);
        if (!st) S->keys_per_query[r->scene] = std::max<uint64_t>(S->cal.last.n_keys, 1);
        calibrated = true;
    }
    if (calibrated) {
        hipStreamSynchronize(sl->stream);
        S->cal.release();
    }
    auto caps = [&](int n) {
        MixCaps k;
        int64_t pairs = 0, tiles = 0;
        double keys = 0;
        for (int i = 0; i < n; ++i) {
            const DevScene& d = c->scene(batch[i]->scene)->d;
            const int t = ((d.W + 15) / 16) * ((d.H + 15) / 16);
            pairs += d.n;
            tiles += t;
            k.outs += (int64_t)d.H * d.W;
            keys += (double)S->keys_per_query[batch[i]->scene];
            k.bin_n = std::max(k.bin_n, d.n);
            k.bin_tiles = std::max(k.bin_tiles, t);
        }
        k.B_cap = pow2_at_least(n);
        k.pair_cap = round_cap(pairs, 1 << 14);
        k.tile_cap = round_cap(tiles, 256);
        k.bin_n = (int)round_cap(k.bin_n, 1024);
        k.key_cap = (uint64_t)round_cap((int64_t)std::ceil(keys * S->cfg.key_factor) + 4096, 1 << 16);
        k.outs = round_cap(k.outs, 1 << 16);  // the output buffer (its address is in the graphs) grows rarely
        // capacities only grow per slot and batch size, so that after the largest batches one graph per size
        // serves them all (the binning path's cost does not grow with them: its grids follow the largest
        // query and the batch's own totals, read on the device)
        auto it = sl->mix_hw.find(k.B_cap);
        if (it != sl->mix_hw.end()) {
            const MixCaps& h = it->second;
            k.pair_cap = std::max(k.pair_cap, h.pair_cap);
            k.tile_cap = std::max(k.tile_cap, h.tile_cap);
            k.key_cap = std::max(k.key_cap, h.key_cap);
            k.bin_n = std::max(k.bin_n, h.bin_n);
            k.bin_tiles = std::max(k.bin_tiles, h.bin_tiles);
            k.outs = std::max(k.outs, h.outs);
        }
        return k;
    };
    int count = (int)batch.size();
    if (!st && S->cfg.hbm_budget) {
        auto fits = [&](int n) {
            uint64_t others = 0;
            for (Slot* o : S->slots)
                if (o != sl) others += slot_bytes(o);
            return others + std::max<uint64_t>(slot_bytes(sl), estimate_mixed_bytes(caps(n))) <= S->cfg.hbm_budget;
        };
        if (!fits(count)) {
            for (Slot* o : S->slots)
                if (!o->busy() && o != sl && slot_bytes(o)) {
                    drop_graphs(o);
                    o->ws.release();
                    o->ws.init(c);
                    o->tx_dev.release();
                    o->out_dev.release();
                }
            while (count > 1 && !fits(count)) count = (count + 1) / 2;
            if (!fits(count) && slot_bytes(sl)) {
                drop_graphs(sl);
                sl->ws.release();
                sl->ws.init(c);
                sl->tx_dev.release();
                sl->out_dev.release();
            }
            if (!fits(count)) {
                bool others_busy = false;
                for (Slot* o : S->slots) others_busy = others_busy || (o != sl && o->busy());
                if (others_busy) {
                    std::lock_guard<std::mutex> lk2(S->mu);
                    for (auto it = batch.rbegin(); it != batch.rend(); ++it) S->waiting.push_front(*it);
                    return 2;
                }
                st = SWF_E_OOM;
            }
            if (!st && count < (int)batch.size()) {
                // the tail goes back to the front of the queue, in its order
                std::lock_guard<std::mutex> lk2(S->mu);
                for (int i = (int)batch.size() - 1; i >= count; --i) S->waiting.push_front(batch[i]);
                batch.resize(count);
                ++S->shrinks;
            }
        }
    }
    if (!st) {
        const MixCaps k = caps(count);
        st = launch_mixed(c, S, sl, batch, flags, k);
        if (!st) sl->mix_hw[k.B_cap] = k;
    }
    if (st) {
        std::lock_guard<std::mutex> lk2(S->mu);
        for (Request* r : batch) {
            r->state = st;
            r->t_done = serve_clock();
        }
        S->cv.notify_all();
    }
    return 1;
}

static void scheduler(Ctx* c) {
    ServeState* S = c->serve;
    t_no_timing = true;
    hipSetDevice(c->device);
    for (;;) {
        bool any_busy = false;
        for (Slot* sl : S->slots) {
            const int ph = sl->phase.load();
            if (ph == 1 && hipEventQuery(sl->done) == hipSuccess) {
                sl->phase = 2;
                {
                    std::lock_guard<std::mutex> lk(S->dmu);
                    S->finished.push_back(sl);
                }
                S->dcv.notify_one();
            }
            any_busy = any_busy || ph != 0;
        }
        // admission into free slots
        for (Slot* sl : S->slots) {
            if (sl->busy()) continue;
            if (S->cfg.mixed) {
                const int r = admit_mixed(c, S, sl);
                if (r == 1) {
                    any_busy = any_busy || sl->busy();
                    continue;
                }
                if (r != 3) break;
            }
            std::vector<Request*> batch;
            int scene = -1;
            {
                std::unique_lock<std::mutex> lk(S->mu);
                if (S->stop) break;
                if (S->waiting.empty()) break;
                scene = S->waiting.front()->scene;
                for (auto it = S->waiting.begin(); it != S->waiting.end() && (int)batch.size() < S->cfg.max_batch;) {
                    if ((*it)->scene == scene) {
                        batch.push_back(*it);
                        it = S->waiting.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            std::lock_guard<std::recursive_mutex> lk(c->mu);
            Scene* sc = c->scene(scene);
            swf_status st = sc ? SWF_OK : SWF_E_NOT_FOUND;
            if (!st && !S->keys_per_query.count(scene)) {
                // calibrate the key count per query once: exact-size lists of one query
                st = sl->tx_dev.reserve(c, 3 * sizeof(float), sl->stream);
                if (!st)
                    st = c->hip(hipMemcpyAsync(sl->tx_dev.ptr, batch[0]->tx, 3 * sizeof(float), hipMemcpyHostToDevice,
                                               sl->stream),
                                "calibration tx");
                if (!st)
                    st = c->forward_lists(sl->ws, scene, (const float*)sl->tx_dev.ptr, 1,
                                          sc->d.has_mlp ? (S->cfg.flags & SWF_MLP_BF16) : SWF_NO_DEFORM, sl->stream,
                                          0);
                if (!st) S->keys_per_query[scene] = std::max<uint64_t>(sl->ws.last.n_keys, 1);
            }
            // bucket: smallest power of two >= count; shrink to the memory budget
            int count = (int)batch.size();
            int bucket = 1;
            while (bucket < count) bucket <<= 1;
            if (!st && S->cfg.hbm_budget) {
                auto fits = [&](int b) {
                    uint64_t others = 0;
                    for (Slot* o : S->slots)
                        if (o != sl) others += slot_bytes(o);
                    const uint64_t kc = (uint64_t)(S->keys_per_query[scene] * b * S->cfg.key_factor) + 4096;
                    const uint64_t need = std::max<uint64_t>(slot_bytes(sl), estimate_bytes(sc->d, b, kc));
                    return others + need <= S->cfg.hbm_budget;
                };
                if (!fits(bucket)) {
                    // release idle workspaces first, then shrink the batch
                    for (Slot* o : S->slots)
                        if (!o->busy() && o != sl && slot_bytes(o)) {
                            drop_graphs(o);
                            o->ws.release();
                            o->ws.init(c);
                            o->tx_dev.release();
                            o->out_dev.release();
                        }
                    while (bucket > 1 && !fits(bucket)) bucket >>= 1;
                    if (!fits(bucket) && slot_bytes(sl)) {
                        drop_graphs(sl);
                        sl->ws.release();
                        sl->ws.init(c);
                        sl->tx_dev.release();
                        sl->out_dev.release();
                    }
                    if (!fits(bucket)) {
                        bool others_busy = false;
                        for (Slot* o : S->slots) others_busy = others_busy || (o != sl && o->busy());
                        if (others_busy) {
                            // does not fit now: requeue at the front, wait for a slot to finish
                            std::lock_guard<std::mutex> lk2(S->mu);
                            for (auto it = batch.rbegin(); it != batch.rend(); ++it) S->waiting.push_front(*it);
                            break;
                        }
                        st = SWF_E_OOM;  // a single query of this scene exceeds the budget
                    }
                    if (!st && bucket < count) {
                        std::lock_guard<std::mutex> lk2(S->mu);
                        for (int i = count - 1; i >= bucket; --i) S->waiting.push_front(batch[i]);
                        batch.resize(bucket);
                        count = bucket;
                        ++S->shrinks;
                    }
                }
            }
            if (!st) st = launch_batch(c, S, sl, scene, batch, bucket);
            if (st) {
                std::lock_guard<std::mutex> lk2(S->mu);
                for (Request* r : batch) {
                    r->state = st;
                    r->t_done = serve_clock();
                }
                S->cv.notify_all();
            } else {
                any_busy = true;
            }
        }
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->stop) {
            bool idle = true;
            for (Slot* sl : S->slots) idle = idle && !sl->busy();
            if (idle) break;
        }
        if (any_busy) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        } else if (S->waiting.empty() && !S->stop) {
            S->cv.wait_for(lk, std::chrono::milliseconds(50));
        }
    }
}

static void deliverer(Ctx* c) {
    ServeState* S = c->serve;
    t_no_timing = true;
    hipSetDevice(c->device);
    for (;;) {
        Slot* sl;
        {
            std::unique_lock<std::mutex> lk(S->dmu);
            S->dcv.wait(lk, [&] { return !S->finished.empty() || S->dstop; });
            if (S->finished.empty()) return;
            sl = S->finished.front();
            S->finished.pop_front();
        }
        finish_slot(c, S, sl);
    }
}

void serve_shutdown(Ctx* c) {
    ServeState* S = c->serve;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    // the scheduler ends once every slot is free, which the deliverer's last results make it
    if (S->thr.joinable()) S->thr.join();
    {
        std::lock_guard<std::mutex> lk(S->dmu);
        S->dstop = true;
    }
    S->dcv.notify_all();
    if (S->deliverer.joinable()) S->deliverer.join();
    for (Slot* sl : S->slots) {
        drop_graphs(sl);
        sl->ws.release();
        sl->tx_dev.release();
        sl->out_dev.release();
        if (sl->tx_host) hipHostFree(sl->tx_host);
        if (sl->out_host) hipHostFree(sl->out_host);
        if (sl->status_host) hipHostFree(sl->status_host);
        if (sl->done) hipEventDestroy(sl->done);
        if (sl->stream) hipStreamDestroy(sl->stream);
        delete sl;
    }
    if (S->cal.total_dev) S->cal.release();
    for (auto& kv : S->table) delete kv.second;
    for (Request* r : S->waiting)
        if (!S->table.count(r->ticket)) delete r;
    delete S;
    c->serve = nullptr;
}

}  // namespace swf

using namespace swf;

extern "C" {

swf_status swf_serve_start(swf_ctx* h, const swf_serve_config* cfg) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    if (c->serve) return c->fail(SWF_E_STATE, "serving already started");
    hipSetDevice(c->device);
    ServeState* S = new ServeState();
    S->cfg.max_batch = 64;
    S->cfg.n_slots = 3;
    S->cfg.mixed = 1;
    S->cfg.flags = SWF_MLP_BF16;
    S->cfg.key_factor = 1.5f;
    S->cfg.hbm_budget = 0;
    S->cfg.use_graphs = 1;
    if (cfg) {
        if (cfg->max_batch > 0) S->cfg.max_batch = cfg->max_batch;
        if (cfg->n_slots > 0) S->cfg.n_slots = cfg->n_slots;
        S->cfg.flags = cfg->flags;
        if (cfg->key_factor > 0) S->cfg.key_factor = cfg->key_factor;
        S->cfg.hbm_budget = cfg->hbm_budget;
        S->cfg.use_graphs = cfg->use_graphs;
        S->cfg.mixed = cfg->mixed;
    }
    if (S->cfg.max_batch > 1024 || S->cfg.n_slots > 16) {
        delete S;
        return c->fail(SWF_E_INVALID, "max_batch must be <= 1024 and n_slots <= 16");
    }
    for (int i = 0; i < S->cfg.n_slots; ++i) {
        Slot* sl = new Slot();
        sl->index = i;
        bool ok = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sl->done, hipEventDisableTiming) == hipSuccess &&
                  hipHostMalloc(&sl->tx_host, sizeof(float) * 3 * pow2_at_least(S->cfg.max_batch), 0) == hipSuccess &&
                  hipHostMalloc(&sl->status_host, 64, 0) == hipSuccess && sl->ws.init(c) == SWF_OK;
        S->slots.push_back(sl);
        if (!ok) {
            c->serve = S;
            serve_shutdown(c);
            return c->fail(SWF_E_DEVICE, "serving slot setup failed");
        }
    }
    c->serve = S;
    S->deliverer = std::thread(deliverer, c);
    S->thr = std::thread(scheduler, c);
    return SWF_OK;
}

swf_status swf_serve_submit(swf_ctx* h, int32_t scene_id, const float* tx, float* out_host, double arrival_s,
                            uint64_t* ticket) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !ticket) return SWF_E_INVALID;
    ServeState* S = c->serve;
    if (!S) return SWF_E_STATE;
    if (!tx || !out_host) return SWF_E_INVALID;
    if (!std::isfinite(tx[0]) || !std::isfinite(tx[1]) || !std::isfinite(tx[2])) return SWF_E_INVALID;
    {
        std::lock_guard<std::recursive_mutex> lock(c->mu);
        if (!c->scene(scene_id)) return SWF_E_NOT_FOUND;
    }
    Request* r = new Request();
    r->scene = scene_id;
    std::memcpy(r->tx, tx, sizeof(float) * 3);
    r->out = out_host;
    r->t_arrival = arrival_s > 0 ? arrival_s : serve_clock();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
        delete r;
        return SWF_E_STATE;
    }
    r->ticket = S->next_ticket++;
    S->table[r->ticket] = r;
    S->waiting.push_back(r);
    *ticket = r->ticket;
    S->cv.notify_all();
    return SWF_OK;
}

static swf_status take_result(ServeState* S, Request* r, swf_req_stats* st) {
    if (st) {
        st->queue_us = 1e6 * (r->t_launch - r->t_arrival);
        st->service_us = 1e6 * (r->t_done - r->t_launch);
        st->total_us = 1e6 * (r->t_done - r->t_arrival);
        st->batch = r->batch;
        st->bucket = r->bucket;
        st->fallback = r->fallback;
        st->slot = r->slot;
    }
    const swf_status s = r->state == 2 ? SWF_OK : (swf_status)r->state;
    S->table.erase(r->ticket);
    delete r;
    return s;
}

swf_status swf_serve_poll(swf_ctx* h, uint64_t ticket, swf_req_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !c->serve) return SWF_E_STATE;
    ServeState* S = c->serve;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->table.find(ticket);
    if (it == S->table.end()) return SWF_E_NOT_FOUND;
    Request* r = it->second;
    if (r->state == 0 || r->state == 1) return SWF_E_PENDING;
    return take_result(S, r, stats);
}

swf_status swf_serve_wait(swf_ctx* h, uint64_t ticket, swf_req_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !c->serve) return SWF_E_STATE;
    ServeState* S = c->serve;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->table.find(ticket);
    if (it == S->table.end()) return SWF_E_NOT_FOUND;
    Request* r = it->second;
    S->cv.wait(lk, [&] { return r->state != 0 && r->state != 1; });
    return take_result(S, r, stats);
}

swf_status swf_serve_stop(swf_ctx* h) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    if (!c->serve) return SWF_E_STATE;
    serve_shutdown(c);
    return SWF_OK;
}

swf_status swf_serve_counters(swf_ctx* h, uint64_t* counters, int32_t n) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !counters) return SWF_E_INVALID;
    if (!c->serve) return SWF_E_STATE;
    ServeState* S = c->serve;
    uint64_t bytes = 0;
    for (Slot* sl : S->slots) bytes += slot_bytes(sl);
    const uint64_t v[8] = {S->launched.load(),     S->completed.load(), S->fallbacks.load(),
                           S->graph_builds.load(), S->shrinks.load(),   bytes,
                           S->mixed_launches.load(), S->mixed_scenes.load()};
    for (int i = 0; i < n && i < 8; ++i) counters[i] = v[i];
    return SWF_OK;
}

double swf_serve_clock(void) { return serve_clock(); }

}  // extern "C"
