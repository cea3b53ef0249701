// Host-side runtime state of libswiftwrf (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/swiftwrf.h"
#include "kernels.h"
#include "swf_device.h"

namespace swf {

struct Ctx;

// Grow-only device buffer. `gen` counts reallocations (captured graphs that
// hold the old address must be rebuilt).
struct Buf {
    void* ptr = nullptr;
    size_t cap = 0;
    uint32_t gen = 0;
    swf_status reserve(Ctx* c, size_t bytes, hipStream_t st);
    void release();
};

struct Scene {
    DevScene d;
    uint64_t gen = 0;  // parameter generation: incremented by every swf_scene_update
    std::vector<void*> allocs;
    std::vector<uint32_t> host_dbits;  // per sorted position
    std::vector<uint32_t> host_perm;   // sorted position -> original id
};

struct TimedStage {
    int stage;
    hipEvent_t a, b;
};

struct LastRender {
    bool valid = false;
    int scene = -1, B = 0, N = 0, flags = 0;
    Grid grid{};
    uint64_t n_keys = 0;
    bool full = false;
    bool binned = false;    // lists built by the binning path (no key array)
    void* keys = nullptr;
    uint32_t* vals = nullptr;
    hipStream_t stream = nullptr;  // stream of the last render (status reads wait for it)
    uint32_t rerenders = 0;        // exact-size re-renders after a speculative key overflow
    uint64_t nan_depth_pairs = 0;  // pairs of Gaussians with a NaN depth (never preprocessed)
    bool chunked = false;          // the call rendered its batch in chunks of queries (this is the last chunk)
};

// Scratch memory of one render stream: every pipeline stage writes here.
struct Workspace {
    Buf qs, geo, wm, oa, rect, count, off, scan, keys, keys2, vals, vals2, hist, ranges, bins, delta, sortk, sortv,
        grad, dpair, dbase, dy, act, dz, part, fmean, ftx, dmu, stage, work, beam, pool, ssim, mix, det;
    Records rec;
    uint64_t* total_dev = nullptr;           // device status block: scan total, effective count, then:
    uint32_t* status_dev = nullptr;          //   status word (bit 0: key overflow at a fixed capacity)
    unsigned long long* cull_dev = nullptr;  //   culled pairs: [0] non-finite/degenerate, [1] off the grid
    uint64_t* total_host = nullptr;  // pinned
    hipEvent_t total_ev = nullptr;   // the scan total has reached total_host (speculative renders)
    void* act_out = nullptr;         // set during a forward pass whose hidden activations are kept: they go here
    uint64_t seq = 0;                // record generation: incremented by every pass that writes the records
    void* mix_host = nullptr;        // pinned staging of a mixed batch's scene and query tables
    size_t mix_host_cap = 0;
    LastRender last;
    std::vector<Buf*> bufs() {
        return {&qs, &geo, &wm, &oa, &rect, &count, &off, &scan, &keys, &keys2, &vals, &vals2, &hist, &ranges, &bins,
                &delta, &sortk, &sortv, &grad, &dpair, &dbase, &dy, &act, &dz, &part, &fmean, &ftx, &dmu,
                &stage, &work, &beam, &pool, &ssim, &mix, &det};
    }
    uint64_t generation() {
        uint64_t g = 0;
        for (Buf* b : bufs()) g += b->gen;
        return g;
    }
    swf_status init(Ctx* c);
    void release();
};

// What a render with SWF_KEEP_AUX wrote into a caller's aux buffer: the
// backward re-runs that forward pass and must see the same scene parameters.
struct AuxTag {
    int scene = -1, B = 0, flags = 0;
    uint64_t gen = 0;
    // the forward's records, lists (and, after a BF16 forward, hidden activations) stay in the workspace until
    // the next pass that writes records: seq is the workspace's record generation right after that forward
    uint64_t seq = 0;
    const float* tx = nullptr;
    bool acts = false;
};

// A mixed batch's plan (runtime.cpp): totals, output offsets and the layout of
// its tables in the workspace's pinned staging.
constexpr int kMixScenes = 64;  // distinct scenes per mixed batch
struct MixPlan {
    int B = 0, B_cap = 0, first_scene = -1;
    int64_t pairs = 0, tiles = 0, outs = 0;
    int max_n = 0, max_tiles = 0;  // the largest query's pairs and tiles
    uint64_t nan_pairs = 0;
    std::vector<uint64_t> out_off;  // B + 1 entries
    size_t query_off = 0, table_bytes = 0;
};
// Capacities a mixed batch is launched at: no host wait for the key count,
// every grid fixed by these values (graph-capturable).
struct MixCaps {
    int B_cap = 0;
    int64_t pair_cap = 0, tile_cap = 0;
    uint64_t key_cap = 0;
    int bin_n = 0, bin_tiles = 0;  // binning geometry: the largest query it covers
    int64_t outs = 0;              // output floats of the batch (not a launch parameter)
};

struct ServeState;
struct Ctx;

struct Ctx {
    int device = 0;
    std::recursive_mutex mu;
    std::string err;
    std::map<int, Scene*> scenes;
    int next_scene = 1;

    Workspace ws;  // scratch of the direct (non-serving) entry points

    // stage timing
    bool timing = false;
    std::vector<TimedStage> pending;
    std::vector<hipEvent_t> event_pool;
    double stage_ms[SWF_N_STAGES] = {};
    int64_t stage_n[SWF_N_STAGES] = {};

    // aux buffers filled by direct renders (device address -> tag), newest last;
    // bounded, the oldest forgotten first
    std::map<const void*, AuxTag> aux_tags;
    bool last_bwd_reused = false;  // the last backward took the forward's kept records and lists
    uint64_t last_blend_executed = 0;  // lane-evaluations of the last blend walk counted (swf_debug_blend_executed)
    // the last backward that ran the MLP backward: its hidden activations stay in ws.act (layer-major rows of
    // 256 per pair, BF16 or FP32)
    struct {
        bool valid = false;
        int scene = -1, B = 0, n = 0, layers = 0;
        bool bf16 = false;
    } last_mlp_bwd;
    std::vector<const void*> aux_order;
    void tag_aux(const void* aux, const AuxTag& t);

    ServeState* serve = nullptr;
    int mlp_pairs_per_wave = 0;  // BF16 MLP register tile: 48 (default, 0), 32 or 64 pairs per wave
    uint64_t max_list_entries = 0xffffffffull;  // list entries per launch sequence; more: chunks of queries

    swf_status fail(swf_status s, const std::string& msg);
    swf_status hip(hipError_t e, const char* what);
    Scene* scene(int id);
    swf_status upload_scene(const swf_gaussians* g, const swf_mlp* mlp, int H, int W, bool dev, int* id);
    swf_status release_scene(int id);
    swf_status pack_mlp(Scene* s, const swf_mlp* mlp, bool dev, bool alloc);
    swf_status update_scene(int id, const swf_gaussians* g, const swf_mlp* mlp, bool dev, hipStream_t st);
    swf_status enqueue_preprocess(Workspace& w, Scene* sc, const float* tx, int B, int flags, const Grid& g,
                                  float* delta_sorted, hipStream_t st);
    // key_cap == 0: size the key buffers from the scan total (one 8-byte
    // device-to-host read and a stream wait). key_cap > 0: fixed capacity, no
    // host synchronisation (graph-capturable); overflow sets the status word.
    // spec_cap > 0 (direct renders only): when the lists are built by binning,
    // build them at that fixed capacity with the scan total copied back
    // asynchronously (w.total_ev); *spec_used tells whether that happened.
    swf_status forward_lists(Workspace& w, int sid, const float* tx, int B, int flags, hipStream_t st,
                             uint64_t key_cap = 0, uint64_t spec_cap = 0, bool* spec_used = nullptr, int rH = 0,
                             int rW = 0);
    swf_status key_count(Workspace& w, hipStream_t st, uint64_t key_cap, uint64_t& nk, const uint64_t*& n_dev,
                         bool readback = false);
    swf_status lists_binned(Workspace& w, const DevScene& d, int B, const Grid& g, hipStream_t st, uint64_t key_cap,
                            bool readback = false);
    swf_status lists_sorted(Workspace& w, const DevScene& d, int B, const Grid& g, bool full, hipStream_t st,
                            uint64_t key_cap);
    // speculate: a direct render whose key buffer is already sized by an
    // earlier one builds its lists at that capacity while the exact count is
    // read back, instead of waiting for the count first; it renders again at
    // the exact size if the count did not fit.
    swf_status render(Workspace& w, int sid, const float* tx, int B, int flags, float* out, void* aux, hipStream_t st,
                      uint64_t key_cap = 0, bool speculate = false, float* chan = nullptr, int rH = 0, int rW = 0);
    swf_status upload_paper_scene(const swf_paper_gaussians* g, const swf_paper_mlp* mlp, int H, int W, bool dev,
                                  int* id);
    // One launch sequence for queries over several scenes (outputs concatenated in query order).
    swf_status render_mixed(Workspace& w, const int32_t* scene_ids, const float* tx, int B, int flags, float* out,
                            uint64_t* out_offsets, hipStream_t st);
    swf_status plan_mixed(Workspace& w, const int32_t* scene_ids, int B, int flags, int B_cap, MixPlan& p);
    // caps == NULL: exactly sized (waits for the key count); else launched at those capacities, no host wait.
    // copy_tables = false leaves the staging -> device copy of the tables to the caller (a graph of the
    // launches alone).
    swf_status enqueue_mixed(Workspace& w, const MixPlan& p, const float* tx, int flags, float* out, hipStream_t st,
                             const MixCaps* caps = nullptr, bool copy_tables = true);
    swf_status backward(Workspace& w, int sid, const float* tx, int B, int flags, const float* grad_out,
                        const void* aux, const swf_grads* grads, hipStream_t st);
    swf_status mlp_backward(Workspace& w, const DevScene& d, const float* tx, int B, const float* dy,
                            const swf_grads* gr, bool bf16, hipStream_t st);
    void* noalloc_scratch = nullptr;  // device address of the static scan scratch (noalloc.hip) on `device`
    void stage_begin(int stage, hipStream_t st);
    void stage_end(hipStream_t st);
    void resolve_timing();
};

Grid make_grid(int H, int W, int tile, bool wrap = false, float sx = 1.0f, float sy = 1.0f);
swf_status noalloc_setup(Ctx* c);  // resolves Ctx::noalloc_scratch (noalloc.hip)
const char* status_name(swf_status s);
void serve_shutdown(Ctx* c);
bool serve_timing_disabled();  // true on the serving scheduler thread

}  // namespace swf
