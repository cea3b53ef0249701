// Serving loop: continuous batching of spectrum queries over resident scenes.
//
// Requests (scene, tx) are queued by any thread. A scheduler thread owns
// `n_slots` execution slots; each slot has its own stream and workspace, so
// the launches of different slots overlap on the device. Whenever a slot is
// free, the scheduler takes the scene of the oldest waiting request, admits up
// to `max_batch` of that scene's waiting requests (FIFO), pads the batch to a
// power-of-two bucket and replays the slot's captured graph for (scene,
// bucket): TX upload -> the whole render (fixed key capacity, no host sync) ->
// result and status download -> completion event. Completed slots are refilled
// immediately (continuous batching). Admission is bounded by a device-memory
// budget over all slot workspaces (a batch that does not fit is shrunk, idle
// workspaces are released, or the requests wait). A key-capacity overflow is
// detected from the status word and the batch is re-rendered with exact sizing.
// Latency is measured from the request's scheduled arrival time.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
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
    bool busy = false;
    int scene = -1, bucket = 0;
    std::vector<Request*> reqs;
    std::map<std::pair<int, int>, GraphEntry> graphs;
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
    std::atomic<uint64_t> launched{0}, completed{0}, fallbacks{0}, graph_builds{0}, shrinks{0};
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
        if (!ge.exec || ge.gen != gen || ge.key_cap != key_cap) {
            if (ge.exec) hipGraphExecDestroy(ge.exec);
            ge.exec = nullptr;
            // eager run sizes every buffer, then capture the same launches
            if ((s = c->render(sl->ws, scene, (const float*)sl->tx_dev.ptr, bucket, flags, (float*)sl->out_dev.ptr,
                               nullptr, st, key_cap)))
                return s;
            if ((s = c->hip(hipStreamSynchronize(st), "serve sync"))) return s;
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
        if ((s = c->hip(hipGraphLaunch(ge.exec, st), "graph launch"))) return s;
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
    sl->busy = true;
    sl->scene = scene;
    sl->bucket = bucket;
    sl->reqs = reqs;
    ++S->launched;
    return SWF_OK;
}

// Exact-size re-render of a finished slot's requests after a key overflow.
static swf_status fallback_batch(Ctx* c, Slot* sl) {
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
            // the next graph for this scene gets a larger key capacity
            S->keys_per_query[sl->scene] = (uint64_t)(S->keys_per_query[sl->scene] * 1.5) + 1024;
            fb = fallback_batch(c, sl) == SWF_OK ? 1 : -1;
            ++S->fallbacks;
        }
        const DevScene& d = c->scene(sl->scene)->d;
        px = (size_t)d.H * d.W;
    }
    // results to the callers' buffers (the requests are in state "running": no
    // other thread touches them), then publish under the lock
    if (fb >= 0)
        for (size_t i = 0; i < sl->reqs.size(); ++i)
            std::memcpy(sl->reqs[i]->out, sl->out_host + i * px, px * sizeof(float));
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
    sl->busy = false;
    S->cv.notify_all();
}

static void scheduler(Ctx* c) {
    ServeState* S = c->serve;
    t_no_timing = true;
    hipSetDevice(c->device);
    for (;;) {
        bool any_busy = false;
        for (Slot* sl : S->slots) {
            if (!sl->busy) continue;
            if (hipEventQuery(sl->done) == hipSuccess)
                finish_slot(c, S, sl);
            else
                any_busy = true;
        }
        // admission into free slots
        for (Slot* sl : S->slots) {
            if (sl->busy) continue;
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
                        if (!o->busy && o != sl && slot_bytes(o)) {
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
                        for (Slot* o : S->slots) others_busy = others_busy || (o != sl && o->busy);
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
            for (Slot* sl : S->slots) idle = idle && !sl->busy;
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

void serve_shutdown(Ctx* c) {
    ServeState* S = c->serve;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->thr.joinable()) S->thr.join();
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
    S->cfg.n_slots = 2;
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
                  hipHostMalloc(&sl->tx_host, sizeof(float) * 3 * S->cfg.max_batch, 0) == hipSuccess &&
                  hipHostMalloc(&sl->status_host, 64, 0) == hipSuccess && sl->ws.init(c) == SWF_OK;
        S->slots.push_back(sl);
        if (!ok) {
            c->serve = S;
            serve_shutdown(c);
            return c->fail(SWF_E_DEVICE, "serving slot setup failed");
        }
    }
    c->serve = S;
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
    const uint64_t v[6] = {S->launched.load(), S->completed.load(), S->fallbacks.load(), S->graph_builds.load(),
                           S->shrinks.load(), 0};
    uint64_t bytes = 0;
    for (Slot* sl : S->slots) bytes += slot_bytes(sl);
    for (int i = 0; i < n && i < 6; ++i) counters[i] = i == 5 ? bytes : v[i];
    return SWF_OK;
}

double swf_serve_clock(void) { return serve_clock(); }

}  // extern "C"
