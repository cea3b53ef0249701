// One launch sequence for a batch of queries over several resident scenes,
// each with its own Gaussian count, grid and deformation MLP (the serving
// loop's mixed batches). Every stage reads the batch's scene and query tables
// from device memory: a query's pairs are records [pair_base, pair_base + N)
// in the scene's (depth, id) order, its tiles are global tiles
// [tile_base, tile_base + tiles), its spectrum lands at out + out_base. The
// per-query arithmetic is exactly that of a single-scene render (same
// kernels' code paths, same record layout), so a query renders the same values
// alone and inside a mixed batch.
//
// Here: the per-query TX term of layer 1, the static preprocess, and the key
// emission of the sort path (per pair, the owning query by binary search over
// the query table). The MLP and the blend take the tables in their own files.
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(256) void mix_tx_kernel(MixBatch m, const float* __restrict__ tx,
                                                     float* __restrict__ qs) {
    __shared__ float feat[kTxFeat];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    const MixScene& s = m.scenes[m.queries[b].scene];
    if (t < 3 * (kTxBands + 1)) {
        const int d = t % 3;
        const int k = t / 3;
        const float v = tx[b * 3 + d];
        const float lo = s.room_lo[d];
        const float rg = s.room_hi[d] - s.room_lo[d];
        float sm, e, hi, lo2;
        two_sum(v, -lo, sm, e);
        div_two(sm, rg, hi, lo2);
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
    constexpr int kIn = kMeanFeat + kTxFeat;
    const float* row = s.w1 + (size_t)t * kIn + kMeanFeat;
    float acc = s.b1[t];
    for (int k = 0; k < kTxFeat; ++k) acc = fmaf(row[k], feat[k], acc);
    qs[(size_t)b * 256 + t] = acc;
}

__device__ __forceinline__ void put_record(const Records& r, size_t row, const PairOut& o) {
    r.geo[row] = o.geo;
    r.wm[row] = o.wm;
    r.oa[row] = o.oa;
    r.rect[row] = make_uint2(o.rect_x, o.rect_y);
    r.count[row] = o.count;
}

// Static records of the batch; rows past the batch's pairs (up to pair_cap)
// get no tiles.
__global__ __launch_bounds__(256) void mix_static_kernel(MixBatch m, int64_t pair_cap, float inv_tile, int wrap,
                                                         Records r) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= pair_cap) return;
    const int total = m.queries[m.B].pair_base;
    if (row >= total) {
        r.count[row] = 0u;
        r.rect[row] = make_uint2(0u, 0u);
        return;
    }
    const int q = mix_find(m.queries, m.B, (int)row, [](const MixQuery& x) { return x.pair_base; });
    const MixScene& s = m.scenes[m.queries[q].scene];
    const int p = (int)row - m.queries[q].pair_base;
    PairOut o;
    if (p < s.n_live) {
        o = preprocess_pair(s.mx[p], s.my[p], 0.f, 0.f, s.lsx[p], s.lsy[p], s.rot[p], s.logit[p], s.amp[p], s.W, s.H,
                            s.TW, s.TH, inv_tile, wrap);
    } else {
        o.geo = make_float4(0, 0, 0, 0);
        o.wm = make_float4(0, 0, 0, 0);
        o.oa = make_float2(0, 0);
        o.rect_x = o.rect_y = 0;
        o.count = 0;
    }
    put_record(r, (size_t)row, o);
}

// Culled pairs of a wave by reason (see the sort path's key emission).
__device__ __forceinline__ void tally(uint32_t why, unsigned long long* cull) {
    const uint64_t nf = __ballot(why == kCullNonFinite), og = __ballot(why == kCullOffGrid);
    if (cull && (threadIdx.x & 63u) == 0) {
        if (nf) atomicAdd(&cull[0], (unsigned long long)__popcll(nf));
        if (og) atomicAdd(&cull[1], (unsigned long long)__popcll(og));
    }
}

// One thread per pair: one u32 key (the global tile) per tile of its
// rectangle, value = the pair's record index. A wrapped rectangle (tx1 < tx0)
// spans columns tx0 .. TW-1, then 0 .. tx1.
__global__ __launch_bounds__(256) void mix_emit_keys_kernel(MixBatch m, const uint2* __restrict__ rect,
                                                            const uint32_t* __restrict__ count,
                                                            const uint32_t* __restrict__ offsets, int64_t pair_cap,
                                                            uint64_t capacity, uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ vals, uint32_t* __restrict__ status,
                                                            unsigned long long* __restrict__ cull) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int total = m.queries[m.B].pair_base;
    const bool in = i < pair_cap && i < total;
    const uint32_t c = in ? count[i] : 0u;
    tally(in && c == 0 ? rect[i].y : 0u, cull);
    if (!in || c == 0) return;
    const uint64_t off = offsets[i];
    if (off + c > capacity) {
        atomicOr(status, 1u);
        return;
    }
    const int q = mix_find(m.queries, m.B, (int)i, [](const MixQuery& x) { return x.pair_base; });
    const MixScene& s = m.scenes[m.queries[q].scene];
    const uint32_t base = (uint32_t)m.queries[q].tile_base;
    const uint2 r = rect[i];
    const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff, ty1 = r.y >> 16;
    const int TW = s.TW;
    const int ncol = tx1 >= tx0 ? tx1 - tx0 + 1 : TW - tx0 + tx1 + 1;
    uint64_t o = off;
    for (int ty = ty0; ty <= ty1; ++ty) {
        for (int k = 0; k < ncol; ++k) {
            const int tx = tx0 + k < TW ? tx0 + k : tx0 + k - TW;
            keys[o] = base + (uint32_t)(ty * TW + tx);
            vals[o] = (uint32_t)i;
            ++o;
        }
    }
}

// Rows past the batch's pairs (up to the capacity) hold no tiles.
__global__ __launch_bounds__(256) void mix_clear_tail_kernel(MixBatch m, int64_t pair_cap, Records r) {
    const int64_t row = (int64_t)m.queries[m.B].pair_base + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= pair_cap) return;
    r.count[row] = 0u;
    r.rect[row] = make_uint2(0u, 0u);
}

}  // namespace

void launch_mix_clear_tail(const MixBatch& m, int64_t pair_cap, const Records& r, hipStream_t st) {
    // every row the tail can hold: launched at the capacity, the rows before the batch's total return at once
    if (pair_cap > 0) mix_clear_tail_kernel<<<(unsigned)((pair_cap + 255) / 256), 256, 0, st>>>(m, pair_cap, r);
}

void launch_mix_tx_features(const MixBatch& m, const float* tx, float* qs, hipStream_t st) {
    if (m.B > 0) mix_tx_kernel<<<m.B, 256, 0, st>>>(m, tx, qs);
}

void launch_mix_static(const MixBatch& m, int64_t pair_cap, const Grid& g, const Records& r, hipStream_t st) {
    if (pair_cap > 0)
        mix_static_kernel<<<(unsigned)((pair_cap + 255) / 256), 256, 0, st>>>(m, pair_cap, 1.0f / (float)g.tile, g.wrap,
                                                                              r);
}

void launch_mix_emit_keys(const MixBatch& m, const Records& r, const uint32_t* offsets, int64_t pair_cap,
                          uint64_t capacity, uint32_t* keys, uint32_t* vals, uint32_t* status,
                          unsigned long long* cull, hipStream_t st) {
    if (pair_cap > 0)
        mix_emit_keys_kernel<<<(unsigned)((pair_cap + kThreads - 1) / kThreads), kThreads, 0, st>>>(
            m, r.rect, r.count, offsets, pair_cap, capacity, keys, vals, status, cull);
}

}  // namespace swf
