// Device prefix scan, key emission, stable LSD radix sort and tile ranges:
// the binning stage that turns per-pair tile rectangles into per-tile,
// front-to-back Gaussian lists (the tile partitioning of Sec. 4.1).
//
// Sort: reduce-then-scan LSD radix sort with 8-bit digits and a fixed grid (no
// inter-workgroup waits, so no forward-progress assumption). Each pass:
// per-block digit histograms -> per-digit exclusive scans over the blocks
// (digit offsets folded into the scatter prologue) -> scatter, where keys are ranked stably inside a 2048-key tile with wave64
// ballots (8 ballots give each lane the mask of lanes sharing its digit).
#include "kernels.h"
#include "swf_device.h"

namespace swf {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // keys per scatter tile
constexpr int kMaxGrid = 1024;

__device__ __forceinline__ unsigned lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Inclusive scan across a wave64.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T t = __shfl_up(v, o, 64);
        if ((int)lane_id() >= o) v += t;
    }
    return v;
}

// Exclusive scan across a block of W waves (256 threads by default); returns the block total in *tot.
template <typename T, int W = kWaves>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds /* W + 1 */, T* tot) {
    const T inc = wave_inclusive_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) lds[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < W; ++i) {
            const T t = lds[i];
            lds[i] = run;
            run += t;
        }
        lds[W] = run;
    }
    __syncthreads();
    const T r = lds[w] + inc - v;
    *tot = lds[W];
    __syncthreads();
    return r;
}

// ---- exclusive scan of uint32 counts (3 kernels; 1 up to kScanSingleMax) ---
__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                               int64_t chunk, uint64_t* __restrict__ sums) {
    __shared__ uint64_t lds[kWaves + 1];
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(beg + chunk, n);
    uint64_t s = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kThreads) s += in[i];
    uint64_t tot;
    block_exclusive_scan<uint64_t>(s, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void scan_top_kernel(uint64_t* __restrict__ sums, int G,
                                                            uint64_t* __restrict__ total) {
    __shared__ uint64_t lds[kWaves + 1];
    uint64_t base = 0;
    for (int c = 0; c < G; c += kThreads) {
        const int i = c + threadIdx.x;
        const uint64_t v = i < G ? sums[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan<uint64_t>(v, lds, &tot);
        if (i < G) sums[i] = base + ex;
        base += tot;
    }
    if (threadIdx.x == 0) *total = base;
}

__global__ __launch_bounds__(kThreads) void scan_down_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                             int64_t chunk, const uint64_t* __restrict__ sums,
                                                             uint32_t* __restrict__ out) {
    __shared__ uint64_t lds[kWaves + 1];
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(beg + chunk, n);
    uint64_t base = sums[blockIdx.x];
    // per-thread runs of kItems consecutive elements for coalescing-friendly reads
    for (int64_t t0 = beg; t0 < end; t0 += (int64_t)kThreads * kItems) {
        uint32_t v[kItems];
        uint64_t s = 0;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = t0 + (int64_t)threadIdx.x * kItems + j;
            v[j] = i < end ? in[i] : 0u;
            s += v[j];
        }
        uint64_t tot;
        uint64_t ex = block_exclusive_scan<uint64_t>(s, lds, &tot) + base;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = t0 + (int64_t)threadIdx.x * kItems + j;
            if (i < end) out[i] = (uint32_t)ex;
            ex += v[j];
        }
        base += tot;
    }
}

// Small inputs (n <= kScanSingleMax) in one launch: one 1024-thread workgroup
// stages the counts in LDS with coalesced loads, scans 16 consecutive counts
// per thread around one block scan, and writes the offsets back through LDS
// with coalesced stores (in and out may be the same array); writes the total.
constexpr int kScanSingleThreads = 1024;
constexpr int kScanSingleItems = 16;
constexpr int64_t kScanSingleMax = (int64_t)kScanSingleThreads * kScanSingleItems;  // 16384

__global__ __launch_bounds__(kScanSingleThreads) void scan_single_kernel(const uint32_t* in, int64_t n, uint32_t* out,
                                                                         uint64_t* __restrict__ total) {
    constexpr int W = kScanSingleThreads / 64;
    __shared__ uint4 s_v[kScanSingleMax / 4];
    __shared__ uint64_t lds[W + 1];
    uint32_t* sv = reinterpret_cast<uint32_t*>(s_v);
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int k = 0; k < kScanSingleItems; ++k) {
        const int i = k * kScanSingleThreads + t;
        sv[i] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanSingleItems];
#pragma unroll
    for (int q = 0; q < kScanSingleItems / 4; ++q) {
        const uint4 u = s_v[t * (kScanSingleItems / 4) + q];
        v[4 * q] = u.x;
        v[4 * q + 1] = u.y;
        v[4 * q + 2] = u.z;
        v[4 * q + 3] = u.w;
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanSingleItems; ++j) s += v[j];
    uint64_t tot;
    uint64_t ex = block_exclusive_scan<uint64_t, W>(s, lds, &tot);  // ends with a barrier: every read above is done
#pragma unroll
    for (int q = 0; q < kScanSingleItems / 4; ++q) {
        uint4 u;
        u.x = (uint32_t)ex;
        ex += v[4 * q];
        u.y = (uint32_t)ex;
        ex += v[4 * q + 1];
        u.z = (uint32_t)ex;
        ex += v[4 * q + 2];
        u.w = (uint32_t)ex;
        ex += v[4 * q + 3];
        s_v[t * (kScanSingleItems / 4) + q] = u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanSingleItems; ++k) {
        const int i = k * kScanSingleThreads + t;
        if (i < n) out[i] = sv[i];
    }
    if (t == 0) *total = tot;
}

// Culled pairs of a wave by reason (the reason a record with no tiles keeps in
// rect.y; 0 for pairs that are not culled): one atomic per reason and wave into
// cull[0] (non-finite or degenerate) and cull[1] (off the grid). Every lane of
// the wave must call it. cull may be null.
__device__ __forceinline__ void tally_culled(uint32_t why, unsigned long long* cull) {
    const uint64_t nf = __ballot(why == kCullNonFinite), og = __ballot(why == kCullOffGrid);
    if (cull && lane_id() == 0) {
        if (nf) atomicAdd(&cull[0], (unsigned long long)__popcll(nf));
        if (og) atomicAdd(&cull[1], (unsigned long long)__popcll(og));
    }
}

// ---- key emission -----------------------------------------------------------
// One thread per pair: one key per tile of the pair's rectangle, row-major.
// key = global tile (query * tiles + ty * TW + tx), or with full keys
// (global tile << 32 | depth bits); value = pair index.
template <bool kFull>
__global__ __launch_bounds__(kThreads) void emit_keys_kernel(const uint2* __restrict__ rect,
                                                             const uint32_t* __restrict__ count,
                                                             const uint32_t* __restrict__ offsets,
                                                             const uint32_t* __restrict__ dbits, int N, int64_t total,
                                                             int TW, int tiles, uint64_t capacity,
                                                             void* __restrict__ keys, uint32_t* __restrict__ vals,
                                                             uint32_t* __restrict__ status,
                                                             unsigned long long* __restrict__ cull) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool in = i < total;
    const uint32_t c = in ? count[i] : 0u;
    tally_culled(in && c == 0 ? rect[i].y : 0u, cull);
    if (!in || c == 0) return;
    const uint64_t off = offsets[i];
    if (off + c > capacity) {
        atomicOr(status, 1u);
        return;
    }
    const uint2 r = rect[i];
    const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff, ty1 = r.y >> 16;
    // a wrapped rectangle (periodic azimuth, tx1 < tx0) spans columns tx0 .. TW-1, then 0 .. tx1
    const int ncol = tx1 >= tx0 ? tx1 - tx0 + 1 : TW - tx0 + tx1 + 1;
    const uint32_t q = (uint32_t)(i / N);
    const uint32_t base = q * (uint32_t)tiles;
    const uint32_t db = kFull ? dbits[i % N] : 0u;
    uint64_t o = off;
    for (int ty = ty0; ty <= ty1; ++ty) {
        for (int k = 0; k < ncol; ++k) {
            const int tx = tx0 + k < TW ? tx0 + k : tx0 + k - TW;
            const uint32_t gt = base + (uint32_t)(ty * TW + tx);
            if (kFull)
                reinterpret_cast<uint64_t*>(keys)[o] = ((uint64_t)gt << 32) | db;
            else
                reinterpret_cast<uint32_t*>(keys)[o] = gt;
            vals[o] = (uint32_t)i;
            ++o;
        }
    }
}

// ---- radix sort ---------------------------------------------------------------
// Key count and per-block chunk: from the host, or (n_dev != nullptr) read on
// the device as min(*n_dev, n) so that a captured graph needs no host sync.
__device__ __forceinline__ void sort_extent(const uint64_t* n_dev, int64_t& n, int64_t& chunk, int G) {
    if (n_dev) {
        const uint64_t d = *n_dev;
        n = (int64_t)(d < (uint64_t)n ? d : (uint64_t)n);
        chunk = (n + G - 1) / G;
        chunk = ((chunk + kTile - 1) / kTile) * kTile;
    }
}

template <typename K>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const K* __restrict__ keys, int64_t n, int shift,
                                                              int64_t chunk, uint32_t* __restrict__ hist, int G,
                                                              const uint64_t* __restrict__ n_dev) {
    __shared__ uint32_t h[kWaves][256];
    sort_extent(n_dev, n, chunk, G);
    for (int i = threadIdx.x; i < kWaves * 256; i += kThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(beg + chunk, n);
    for (int64_t i = beg + threadIdx.x; i < end; i += kThreads) {
        const uint32_t d = (uint32_t)(keys[i] >> shift) & 255u;
        atomicAdd(&h[w][d], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kThreads) {
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) s += h[k][d];
        hist[(size_t)d * G + blockIdx.x] = s;
    }
}

// Per-digit exclusive scan over the G block counts (digit-major histogram):
// block d scans hist[d][0..G) in place and writes the digit total.
__global__ __launch_bounds__(kThreads) void digit_scan_kernel(uint32_t* __restrict__ hist, int G,
                                                              uint32_t* __restrict__ dtot) {
    __shared__ uint32_t lds[kWaves + 1];
    uint32_t* h = hist + (size_t)blockIdx.x * G;
    uint32_t base = 0;
    for (int c = 0; c < G; c += kThreads) {
        const int i = c + threadIdx.x;
        const uint32_t v = i < G ? h[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<uint32_t>(v, lds, &tot);
        if (i < G) h[i] = base + ex;
        base += tot;
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = base;
}

template <typename K>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(const K* __restrict__ kin,
                                                                 const uint32_t* __restrict__ vin,
                                                                 K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                                 int64_t n, int shift, int64_t chunk,
                                                                 const uint32_t* __restrict__ hist, int G,
                                                                 const uint32_t* __restrict__ dtot,
                                                                 const uint64_t* __restrict__ n_dev) {
    sort_extent(n_dev, n, chunk, G);
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t base[256];
    __shared__ uint32_t ttot[256];
    __shared__ uint32_t lds[kWaves + 1];
    const int w = threadIdx.x >> 6;
    {
        // digit offsets: exclusive scan of the digit totals
        static_assert(kThreads == 256, "one thread per digit");
        uint32_t tot;
        const uint32_t doff = block_exclusive_scan<uint32_t>(dtot[threadIdx.x], lds, &tot);
        base[threadIdx.x] = doff + hist[(size_t)threadIdx.x * G + blockIdx.x];
    }
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(beg + chunk, n);
    for (int64_t t0 = beg; t0 < end; t0 += kTile) {
        for (int i = threadIdx.x; i < kWaves * 256; i += kThreads) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        K k[kItems];
        uint32_t v[kItems], dig[kItems], lr[kItems];
        bool ok[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t idx = t0 + (int64_t)(w * kItems + j) * 64 + lane_id();
            ok[j] = idx < end;
            k[j] = ok[j] ? kin[idx] : (K)0;
            v[j] = ok[j] ? vin[idx] : 0u;
            const uint32_t d = (uint32_t)(k[j] >> shift) & 255u;
            dig[j] = d;
            const uint64_t valid = __ballot(ok[j]);
            uint64_t match = valid;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bal = __ballot(bit && ok[j]);
                match &= bit ? bal : ~bal;
            }
            const uint32_t rank = (uint32_t)__popcll(match & lanemask_lt());
            const uint32_t cnt = (uint32_t)__popcll(match);
            uint32_t prev = 0;
            if (ok[j]) prev = wcnt[w][d];
            lr[j] = prev + rank;
            __builtin_amdgcn_wave_barrier();
            if (ok[j] && rank == 0) wcnt[w][d] = prev + cnt;
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        for (int d = threadIdx.x; d < 256; d += kThreads) {
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                const uint32_t c = wcnt[q][d];
                wcnt[q][d] = run;
                run += c;
            }
            ttot[d] = run;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            if (ok[j]) {
                const uint32_t pos = base[dig[j]] + wcnt[w][dig[j]] + lr[j];
                kout[pos] = k[j];
                vout[pos] = v[j];
            }
        }
        __syncthreads();
        for (int d = threadIdx.x; d < 256; d += kThreads) base[d] += ttot[d];
        __syncthreads();
    }
}

// ---- binning: per-query stable counting sort by tile -----------------------
// Pairs are stored in (query, depth) order and a pair covers a tile at most
// once, so the list of a tile is the pairs covering it in pair order. A query's
// tiles are split into S segments of 2^db tiles (db = 8 with at most 256 tiles
// per query, one segment; else 9); every query is binned by a stable counting
// pass per segment, which gives exactly the order of the full (tile, depth)
// sort without materialising keys in memory.
//   bin_hist:    block (j, q) histograms the tiles covered by pairs
//                [j * pb, (j + 1) * pb) of query q, for every segment s, into
//                its own row: hist[((q * S + s) * nbq + j) * 2^db + tile - 2^db s]
//   bin_colscan: per column (q, s, tile) the exclusive prefix over the blocks,
//                in place, and the column total; an exclusive scan of the totals
//                in (query, tile) order gives every tile's first list position
//                (`starts`, stored after the histogram) and the entry count. A
//                block's first position in a tile's list is the tile's start
//                plus the block's column prefix.
//   bin_place:   (one segment) the block places its pairs batch by batch: each
//                key sets its pair's bit in a per-tile mask of the batch, and
//                its rank in the tile's list is the number of the batch's pairs
//                below its own in that mask
//   bin_scatter: (several segments) the block, segment by segment, ranks its
//                keys stably with wave64 ballots over the db digit bits
//   bin_ranges:  tile (q, t) spans [start(q, t), start(q, t + 1))
// A periodic azimuth (wrapped rectangles, tx1 < tx0: columns tx0 .. TW - 1,
// then 0 .. tx1) is binned when a query has one segment.
struct BinGeom {
    int N, TW, tiles, db, S, pb, nbq;  // pairs per query, tile grid, digit bits, segments, pairs/block, blocks/query
};

constexpr int kWideDb = 9;       // digit bits when a query has more than 256 tiles (segments of 512)
constexpr int kMaxTiles = 4096;           // tiles per query the binning path takes

BinGeom bin_geom(int N, const Grid& g) {
    BinGeom b;
    b.N = N;
    b.TW = g.TW;
    b.tiles = g.tiles;
    b.db = g.tiles <= 256 ? 8 : kWideDb;
    b.S = std::max(1, (g.tiles + (1 << b.db) - 1) >> b.db);
    b.pb = b.S == 1 ? 1024 : 8192;  // larger blocks keep the (S x 256 x blocks) histogram small
    b.nbq = std::max(1, (N + b.pb - 1) / b.pb);
    return b;
}

// Every tile of a pair's rectangle (rows top to bottom, columns from tx0, a
// wrapped rectangle continuing at column 0): calls f(tile).
template <typename F>
__device__ __forceinline__ void for_rect_tiles(uint2 r, int TW, F&& f) {
    const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff, ty1 = r.y >> 16;
    const int w = tx1 >= tx0 ? tx1 - tx0 + 1 : TW - tx0 + tx1 + 1;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int k = 0; k < w; ++k) {
            const int col = tx0 + k < TW ? tx0 + k : tx0 + k - TW;
            f((uint32_t)(ty * TW + col));
        }
}

__device__ __forceinline__ uint32_t seg_count(uint2 r, int TW, int t0, int seg) {
    const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff, ty1 = r.y >> 16;
    if (ty1 * TW + tx1 < t0 || ty0 * TW + tx0 >= t0 + seg) return 0;
    uint32_t c = 0;
    for (int ty = ty0; ty <= ty1; ++ty) {
        const int a = max(ty * TW + tx0, t0), b = min(ty * TW + tx1, t0 + seg - 1);
        c += b >= a ? (uint32_t)(b - a + 1) : 0u;
    }
    return c;
}

// A query's pairs and tile grid for the binning kernels: uniform over a
// single-scene batch (G), from the batch's tables for a mixed one, whose
// geometry G (segments, block size, blocks per query) covers its largest
// query: a smaller query leaves its extra blocks and segments empty.
struct BinQuery {
    int N, TW, tiles, S;
    size_t row0;
};

template <bool kMix>
__device__ __forceinline__ BinQuery bin_query(const BinGeom& G, const MixBatch& mix, int q) {
    BinQuery b;
    if constexpr (kMix) {
        const MixQuery& a = mix.queries[q];
        const MixQuery& e = mix.queries[q + 1];
        b.N = e.pair_base - a.pair_base;  // 0 for the padding queries of a capacity-sized batch
        b.tiles = e.tile_base - a.tile_base;
        b.TW = mix.scenes[a.scene].TW;
        b.S = (b.tiles + (1 << G.db) - 1) >> G.db;
        b.row0 = (size_t)a.pair_base;
    } else {
        b.N = G.N;
        b.tiles = G.tiles;
        b.TW = G.TW;
        b.S = G.S;
        b.row0 = (size_t)q * G.N;
    }
    return b;
}

// Tile histogram of one block of pairs of one query, for every tile segment, in
// the block's own row: hist[((q * S + segment) * nbq + block) * 2^db + tile % 2^db].
// With one segment the counts are kept per wave (less atomic contention).
template <bool kMix = false>
__global__ __launch_bounds__(kThreads) void bin_hist_kernel(const uint2* __restrict__ rect,
                                                            const uint32_t* __restrict__ count, BinGeom G,
                                                            uint32_t* __restrict__ hist,
                                                            unsigned long long* __restrict__ cull,
                                                            MixBatch mix = MixBatch{}) {
    __shared__ uint32_t h[kMaxTiles + 1024];  // S segments of 2^db tiles: at most kMaxTiles + 2^db - 1
    __shared__ uint32_t nculled[2];
    const int kSegTiles = 1 << G.db;
    const bool one = G.S == 1;
    const int n = one ? kWaves * kSegTiles : G.S * kSegTiles;
    for (int i = threadIdx.x; i < n; i += kThreads) h[i] = 0;
    if (threadIdx.x < 2) nculled[threadIdx.x] = 0;
    __syncthreads();
    uint32_t* hw = one ? h + (threadIdx.x >> 6) * kSegTiles : h;
    const int j = blockIdx.x, q = blockIdx.y;
    const BinQuery Q = bin_query<kMix>(G, mix, q);
    const int p_beg = j * G.pb, p_end = min(p_beg + G.pb, Q.N);
    const size_t row0 = Q.row0;
    uint32_t nf = 0, og = 0;  // culled pairs seen by this thread, by reason
    for (int p = p_beg + (int)threadIdx.x; p < p_end; p += kThreads) {
        const uint2 r = rect[row0 + p];
        if (count[row0 + p] == 0) {
            nf += r.y == kCullNonFinite;
            og += r.y == kCullOffGrid;
            continue;
        }
        for_rect_tiles(r, Q.TW, [&](uint32_t t) { atomicAdd(&hw[t], 1u); });
    }
    if (nf) atomicAdd(&nculled[0], nf);
    if (og) atomicAdd(&nculled[1], og);
    __syncthreads();
    if (cull && threadIdx.x < 2 && nculled[threadIdx.x]) atomicAdd(&cull[threadIdx.x], (unsigned long long)nculled[threadIdx.x]);
    for (int i = threadIdx.x; i < G.S * kSegTiles; i += kThreads) {
        uint32_t v = h[i];
        if (one)
#pragma unroll
            for (int k = 1; k < kWaves; ++k) v += h[k * kSegTiles + i];
        const int sg = i / kSegTiles, d = i - sg * kSegTiles;
        hist[(((size_t)(q * G.S + sg) * G.nbq + j) << G.db) + d] = v;
    }
}

// Column (query-segment, tile) i of the histogram: the exclusive prefix over
// its nbq blocks, in place, and the column total. Consecutive threads take
// consecutive tiles, so every access is coalesced.
__global__ __launch_bounds__(kThreads) void bin_colscan_kernel(uint32_t* __restrict__ hist, int64_t cols, int nbq,
                                                               int db, uint32_t* __restrict__ totals) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= cols) return;
    const int64_t qs = i >> db, d = i & ((1 << db) - 1);
    uint32_t* col = hist + ((qs * nbq) << db) + d;
    const size_t stride = (size_t)1 << db;
    uint32_t run = 0;
    int j = 0;
    for (; j + 8 <= nbq; j += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = col[(size_t)(j + k) * stride];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            col[(size_t)(j + k) * stride] = run;
            run += v[k];
        }
    }
    for (; j < nbq; ++j) {
        const uint32_t v = col[(size_t)j * stride];
        col[(size_t)j * stride] = run;
        run += v;
    }
    totals[i] = run;
}

// Placement for one segment (at most 256 tiles per query): one block of pairs
// of one query, in batches of 256 pairs (one per thread). A batch's keys, in
// pair order, are processed in chunks of kTile positions; every lane computes
// the key at its position directly (the owning pair by binary search over the
// batch's key offsets, the tile by enumerating the pair's rectangle row by row)
// and sets the pair's bit in the tile's 256-bit mask. The key's rank in the
// tile's list is then the tile's start for this block, plus the batch's earlier
// pairs covering the tile (their keys all lie at earlier positions, so their
// bits are set by then), plus the entries of the block's earlier batches.
template <bool kMix = false>
__global__ __launch_bounds__(kThreads) void bin_place_kernel(const uint2* __restrict__ rect,
                                                             const uint32_t* __restrict__ count, BinGeom G,
                                                             const uint32_t* __restrict__ hs,
                                                             const uint32_t* __restrict__ starts,
                                                             const uint64_t* __restrict__ n_dev,
                                                             uint32_t* __restrict__ vals, MixBatch mix = MixBatch{}) {
    constexpr int kSeg = 256;
    constexpr int kBatch = kThreads;
    constexpr int kWords = kBatch / 64;
    static_assert(kSeg == kThreads, "one tile per thread in the per-tile steps");
    // fixed-capacity run that overflowed: nothing is placed (block-uniform)
    if (n_dev && *n_dev == 0) return;
    // word-major, so the tiles of consecutive keys (consecutive tiles) fall on consecutive banks
    __shared__ unsigned long long mask[kWords][kSeg];  // bit p of word w: pair 64 w + p of the batch covers the tile
    __shared__ uint32_t pre[kWords][kSeg];             // pairs covering the tile in the words before
    __shared__ uint32_t base[kSeg];
    __shared__ uint32_t lds[kWaves + 1];
    __shared__ uint32_t s_o[kBatch], s_w[kBatch];
    __shared__ int s_ty0[kBatch], s_tx0[kBatch];
    __shared__ float s_rw[kBatch];
    const int j = blockIdx.x, q = blockIdx.y;
    const int t = threadIdx.x;
    const BinQuery Q = bin_query<kMix>(G, mix, q);
    const int p_beg = j * G.pb, p_end = min(p_beg + G.pb, Q.N);
    const size_t row0 = Q.row0;
    const int TW = Q.TW;
    base[t] = hs[(((size_t)q * G.nbq + j) << 8) + t] + starts[((size_t)q << 8) + t];
#pragma unroll
    for (int k = 0; k < kWords; ++k) mask[k][t] = 0ull;
    uint32_t c_next = 0u;
    uint2 r_next = make_uint2(0u, 0u);
    if (p_beg + t < p_end) {
        c_next = count[row0 + p_beg + t];
        r_next = rect[row0 + p_beg + t];
    }
    for (int s0 = p_beg; s0 < p_end; s0 += kBatch) {
        const uint32_t c = c_next;
        const uint2 r = r_next;
        const int pn = s0 + kBatch + t;
        c_next = pn < p_end ? count[row0 + pn] : 0u;
        if (pn < p_end) r_next = rect[row0 + pn];
        uint32_t K;
        const uint32_t o = block_exclusive_scan<uint32_t>(c, lds, &K);  // synchronises
        if (K == 0) continue;
        s_o[t] = o;
        if (c) {
            const int tx0 = r.x & 0xffff, tx1 = r.x >> 16;
            const uint32_t w = (uint32_t)(tx1 >= tx0 ? tx1 - tx0 + 1 : TW - tx0 + tx1 + 1);
            s_ty0[t] = (int)(r.y & 0xffff);
            s_tx0[t] = tx0;
            s_w[t] = w;
            s_rw[t] = 1.0f / (float)w;
        }
        for (uint32_t c0 = 0; c0 < K; c0 += kTile) {
            __syncthreads();  // the batch's pair table is complete; the previous chunk's ranks are read
            uint32_t dig[kItems], own[kItems];
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const uint32_t gp = c0 + (uint32_t)(i * kThreads + t);
                own[i] = kBatch;  // no key at this position
                dig[i] = 0u;
                if (gp < K) {
                    // last pair whose first key is at or before gp (s_o is non-decreasing; a pair without keys
                    // shares its offset with the next pair, so the last one is the owner)
                    int lo = 0;
#pragma unroll
                    for (int step = kBatch / 2; step > 0; step >>= 1)
                        if (s_o[lo + step] <= gp) lo += step;
                    const uint32_t m = gp - s_o[lo], w = s_w[lo];
                    // m < 256 keys, w <= 256 columns: the product is at most one below the quotient
                    uint32_t qr = (uint32_t)((float)m * s_rw[lo]);
                    uint32_t cc = m - qr * w;
                    if (cc >= w) {
                        ++qr;
                        cc -= w;
                    }
                    const int col = s_tx0[lo] + (int)cc;
                    const uint32_t d = (uint32_t)((s_ty0[lo] + (int)qr) * TW + (col < TW ? col : col - TW));
                    dig[i] = d;
                    own[i] = (uint32_t)lo;
                    atomicOr(&mask[lo >> 6][d], 1ull << (lo & 63));
                }
            }
            __syncthreads();
            {
                uint32_t run = 0;
#pragma unroll
                for (int k = 0; k < kWords; ++k) {
                    pre[k][t] = run;
                    run += (uint32_t)__popcll(mask[k][t]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                if (own[i] < (uint32_t)kBatch) {
                    const uint32_t d = dig[i], lo = own[i];
                    const uint32_t rank = pre[lo >> 6][d] +
                                          (uint32_t)__popcll(mask[lo >> 6][d] & ((1ull << (lo & 63)) - 1ull));
                    vals[base[d] + rank] = (uint32_t)(row0 + s0 + lo);
                }
            }
        }
        __syncthreads();  // every rank of the batch is read
        uint32_t tot = 0;
#pragma unroll
        for (int k = 0; k < kWords; ++k) {
            tot += (uint32_t)__popcll(mask[k][t]);
            mask[k][t] = 0ull;
        }
        base[t] += tot;  // the next batch's scan synchronises before anything reads base or the masks
    }
}

// Lanes of the wave (among those with `ok`) whose DB-bit digit equals this
// lane's: the AND over the digit's bits of the bit's ballot where this lane's
// bit is 1 and of its complement where it is 0, written as ~(ballot ^ s) with s
// the lane's bit sign-extended to a word. Returns (rank among them in lane
// order, their number).
template <int DB>
__device__ __forceinline__ uint2 digit_match(uint32_t d, bool ok) {
    const uint64_t v = __ballot(ok);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < DB; ++b) {
        const uint32_t sb = (uint32_t)((int32_t)(d << (31 - b)) >> 31);  // 0 or ~0
        const uint64_t bal = __ballot(sb != 0u);
        lo &= ~((uint32_t)bal ^ sb);
        hi &= ~((uint32_t)(bal >> 32) ^ sb);
    }
    const uint64_t m = ((uint64_t)hi << 32) | lo;
    return make_uint2((uint32_t)__popcll(m & lanemask_lt()), (uint32_t)__popcll(m));
}

// Enumeration of the keys a pair has in a tile segment [t0, t0 + seg), in the
// row-major order of for_rect_tiles: the first intersecting row of the rectangle
// (possibly clipped by the segment start) gives keys 0 .. n0 - 1 at tiles
// a0 + m; the later rows are whole (only the last can be clipped by the segment
// end, which the key count already excludes) and hold key n0 + q * w + c at
// tile rb + q * TW + c. Tiles are relative to t0.
struct SegRun {
    int a0, rb;
    uint32_t n0, w;
    float rw;  // 1 / w
};

__device__ __forceinline__ SegRun seg_run(uint2 r, int TW, int t0, int seg) {
    const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff;
    const int ya = ty0 * TW + tx1 >= t0 ? ty0 : (t0 - tx1 + TW - 1) / TW;
    const int a = max(ya * TW + tx0, t0), e = min(ya * TW + tx1, t0 + seg - 1);
    SegRun s;
    s.a0 = a - t0;
    s.n0 = (uint32_t)(e - a + 1);
    s.rb = (ya + 1) * TW + tx0 - t0;
    s.w = (uint32_t)(tx1 - tx0 + 1);
    s.rw = 1.0f / (float)s.w;
    return s;
}

// Tile (relative to t0) of key m < the pair's key count in the segment.
__device__ __forceinline__ uint32_t seg_tile_at(int a0, int rb, uint32_t n0, uint32_t w, float rw, int TW,
                                                uint32_t m) {
    if (m < n0) return (uint32_t)(a0 + (int)m);
    const uint32_t mm = m - n0;
    uint32_t q = (uint32_t)((float)mm * rw);  // m < 2^24: exact operands, at most one below
    uint32_t c = mm - q * w;
    if (c >= w) {
        ++q;
        c -= w;
    }
    return (uint32_t)(rb + (int)q * TW + (int)c);
}

// Stable placement of one block of pairs of one query, segment by segment
// (the block's output positions then lie in 256 tile lists at a time). Pairs
// are taken in batches of 256 * PPT (PPT consecutive pairs per thread; several
// when a query has several segments, so that a batch still holds many keys of
// one segment); the batch's keys in the segment, in pair order, are processed
// in chunks of kTile positions, split into whole 64-key items over the waves in
// order. Every lane computes the key at its position directly (load-balanced:
// the owning pair is found by binary search over the batch's key offsets),
// ranks it among equal tiles with wave64 ballots, and the ranks are offset per
// wave and per tile through LDS counters; base[] holds each tile's next output
// position for this block.
template <int PPT, int DB, bool kMix = false>
__global__ __launch_bounds__(kThreads) void bin_scatter_kernel(const uint2* __restrict__ rect,
                                                               const uint32_t* __restrict__ count, BinGeom G,
                                                               const uint32_t* __restrict__ hs,
                                                               const uint32_t* __restrict__ starts,
                                                               const uint64_t* __restrict__ n_dev,
                                                               uint32_t* __restrict__ vals,
                                                               MixBatch mix = MixBatch{}) {
    constexpr int kSeg = 1 << DB;
    constexpr int kBatch = kThreads * PPT;
    // fixed-capacity run that overflowed: nothing is placed (block-uniform)
    if (n_dev && *n_dev == 0) return;
    __shared__ uint32_t base[kSeg];
    __shared__ uint32_t wcnt[kWaves][kSeg];
    __shared__ uint32_t ttot[kSeg];
    __shared__ uint32_t lds[kWaves + 1];
    // per pair of the batch: first key offset and the enumeration of its keys
    __shared__ uint32_t s_o[kBatch], s_n0[kBatch], s_w[kBatch];
    __shared__ int s_a0[kBatch], s_rb[kBatch];
    __shared__ float s_rw[kBatch];
    const int w = threadIdx.x >> 6;
    const int j = blockIdx.x, q = blockIdx.y;
    const BinQuery Q = bin_query<kMix>(G, mix, q);
    const int p_beg = j * G.pb, p_end = min(p_beg + G.pb, Q.N);
    const size_t row0 = Q.row0;
    // segments past the query's tiles hold no keys (their histogram entries are zero)
    for (int sg = 0; sg < Q.S; ++sg) {
        const int t0 = sg * kSeg;
        __syncthreads();  // the previous segment is placed
        for (int d = threadIdx.x; d < kSeg; d += kThreads)
            base[d] = hs[(((size_t)(q * G.S + sg) * G.nbq + j) << DB) + d] + starts[((size_t)(q * G.S + sg) << DB) + d];
        // the next batch's (count, rect) are loaded while this one is placed
        uint32_t c_next[PPT];
        uint2 r_next[PPT];
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int p = p_beg + (int)threadIdx.x * PPT + i;
            c_next[i] = p < p_end ? count[row0 + p] : 0u;
            r_next[i] = p < p_end ? rect[row0 + p] : make_uint2(0u, 0u);
        }
        for (int s0 = p_beg; s0 < p_end; s0 += kBatch) {
            uint32_t c[PPT];
            uint2 r[PPT];
            uint32_t csum = 0;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                r[i] = r_next[i];
                c[i] = !c_next[i] ? 0u : (Q.S == 1 ? c_next[i] : seg_count(r[i], Q.TW, t0, kSeg));
                csum += c[i];
                const int pn = s0 + kBatch + (int)threadIdx.x * PPT + i;
                c_next[i] = pn < p_end ? count[row0 + pn] : 0u;
                if (pn < p_end) r_next[i] = rect[row0 + pn];
            }
            uint32_t K;
            uint32_t o = block_exclusive_scan<uint32_t>(csum, lds, &K);  // synchronises
            if (K == 0) continue;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int e = (int)threadIdx.x * PPT + i;  // pair within the batch
                s_o[e] = o;
                if (c[i]) {
                    const SegRun sr = seg_run(r[i], Q.TW, t0, kSeg);
                    s_a0[e] = sr.a0;
                    s_rb[e] = sr.rb;
                    s_n0[e] = sr.n0;
                    s_w[e] = sr.w;
                    s_rw[e] = sr.rw;
                }
                o += c[i];
            }
            for (uint32_t c0 = 0; c0 < K; c0 += kTile) {
                for (int i = threadIdx.x; i < kWaves * kSeg; i += kThreads) (&wcnt[0][0])[i] = 0;
                __syncthreads();  // counters cleared; the batch's pair table is complete
                const uint32_t n_here = min(K - c0, (uint32_t)kTile);
                const uint32_t ipw = ((n_here + 63) / 64 + kWaves - 1) / kWaves;  // items per wave
                uint32_t dig[kItems], lr[kItems], pl[kItems];
                bool ok[kItems];
#pragma unroll
                for (int jj = 0; jj < kItems; ++jj) {
                    const uint32_t idx0 = ((uint32_t)w * ipw + (uint32_t)jj) * 64;
                    ok[jj] = false;
                    dig[jj] = lr[jj] = pl[jj] = 0;
                    if ((uint32_t)jj >= ipw || idx0 >= n_here) continue;  // wave-uniform
                    const uint32_t idx = idx0 + lane_id();
                    ok[jj] = idx < n_here;
                    uint32_t d = 0, pr = 0;
                    if (ok[jj]) {
                        const uint32_t gp = c0 + idx;  // key position in the batch
                        // last pair whose first key is at or before gp (s_o is
                        // non-decreasing; a pair without keys shares its offset
                        // with the next pair, so the last one is the owner)
                        int lo = 0;
#pragma unroll
                        for (int step = kBatch / 2; step > 0; step >>= 1)
                            if (s_o[lo + step] <= gp) lo += step;
                        pr = (uint32_t)lo;
                        d = seg_tile_at(s_a0[lo], s_rb[lo], s_n0[lo], s_w[lo], s_rw[lo], Q.TW, gp - s_o[lo]);
                    }
                    dig[jj] = d;
                    pl[jj] = pr;
                    const uint2 rc = digit_match<DB>(d, ok[jj]);
                    const uint32_t rank = rc.x, cnt = rc.y;
                    uint32_t prev = 0;
                    if (ok[jj]) prev = wcnt[w][d];
                    lr[jj] = prev + rank;
                    __builtin_amdgcn_wave_barrier();
                    if (ok[jj] && rank == 0) wcnt[w][d] = prev + cnt;
                    __builtin_amdgcn_wave_barrier();
                }
                __syncthreads();
                for (int d = threadIdx.x; d < kSeg; d += kThreads) {
                    uint32_t run = 0;
#pragma unroll
                    for (int k = 0; k < kWaves; ++k) {
                        const uint32_t cc = wcnt[k][d];
                        wcnt[k][d] = run;
                        run += cc;
                    }
                    ttot[d] = run;
                }
                __syncthreads();
#pragma unroll
                for (int jj = 0; jj < kItems; ++jj)
                    if (ok[jj]) vals[base[dig[jj]] + wcnt[w][dig[jj]] + lr[jj]] = (uint32_t)(row0 + s0 + pl[jj]);
                __syncthreads();
                for (int d = threadIdx.x; d < kSeg; d += kThreads) base[d] += ttot[d];
                __syncthreads();
            }
        }
    }
}

// Ranges of a mixed batch's global tiles: tile t of query q starts at entry
// (q, segment t >> db, t mod 2^db) of the scanned tile totals.
__global__ void mix_bin_ranges_kernel(const uint32_t* __restrict__ starts, MixBatch mix, BinGeom G,
                                      const uint64_t* __restrict__ total, const uint64_t* __restrict__ n_dev,
                                      int64_t tile_cap, uint2* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tile_cap || i >= mix.queries[mix.B].tile_base) return;  // the blend skips tiles past the batch
    if (n_dev && *n_dev == 0) {
        ranges[i] = make_uint2(0u, 0u);
        return;
    }
    const int q = mix_find(mix.queries, mix.B, (int)i, [](const MixQuery& x) { return x.tile_base; });
    const int64_t t = i - mix.queries[q].tile_base;
    const size_t e = ((size_t)q * G.S << G.db) + t;
    const uint32_t a = starts[e];
    const uint32_t b = e + 1 < ((size_t)mix.B * G.S << G.db) ? starts[e + 1] : (uint32_t)*total;
    ranges[i] = a < b ? make_uint2(a, b) : make_uint2(0u, 0u);
}

__global__ void bin_ranges_kernel(const uint32_t* __restrict__ starts, int B, BinGeom G,
                                  const uint64_t* __restrict__ total, const uint64_t* __restrict__ n_dev,
                                  uint2* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * G.tiles) return;
    if (n_dev && *n_dev == 0) {
        ranges[i] = make_uint2(0u, 0u);
        return;
    }
    const int64_t q = i / G.tiles, t = i - q * G.tiles;
    const size_t e = ((size_t)q * G.S << G.db) + t;  // segments of a query are consecutive
    const uint32_t a = starts[e];
    const uint32_t b = e + 1 < ((size_t)B * G.S << G.db) ? starts[e + 1] : (uint32_t)*total;
    ranges[i] = a < b ? make_uint2(a, b) : make_uint2(0u, 0u);
}

// ---- tile ranges -----------------------------------------------------------
__global__ void zero_ranges_kernel(uint2* __restrict__ r, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) r[i] = make_uint2(0u, 0u);
}

template <bool kFull>
__global__ void tile_ranges_kernel(const void* __restrict__ keys, int64_t n, uint2* __restrict__ r,
                                   const uint64_t* __restrict__ n_dev) {
    if (n_dev) {
        const uint64_t d = *n_dev;
        n = (int64_t)(d < (uint64_t)n ? d : (uint64_t)n);
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    auto tile_of = [&](int64_t j) -> uint32_t {
        return kFull ? (uint32_t)(reinterpret_cast<const uint64_t*>(keys)[j] >> 32)
                     : reinterpret_cast<const uint32_t*>(keys)[j];
    };
    const uint32_t t = tile_of(i);
    if (i == 0 || tile_of(i - 1) != t) r[t].x = (uint32_t)i;
    if (i == n - 1 || tile_of(i + 1) != t) r[t].y = (uint32_t)(i + 1);
}

int radix_grid(int64_t n) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, kMaxGrid));
}

template <typename K>
int radix_sort_t(K* keys, uint32_t* vals, K* kalt, uint32_t* valt, int64_t n, int begin_bit, int end_bit,
                 uint32_t* hist, hipStream_t st, const uint64_t* n_dev) {
    if (n <= 1 || end_bit <= begin_bit) return 0;
    const int G = radix_grid(n);
    uint32_t* dtot = hist + (size_t)256 * G;
    int64_t chunk = (n + G - 1) / G;
    chunk = ((chunk + kTile - 1) / kTile) * kTile;
    K* ki = keys;
    uint32_t* vi = vals;
    K* ko = kalt;
    uint32_t* vo = valt;
    int flips = 0;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        radix_hist_kernel<K><<<G, kThreads, 0, st>>>(ki, n, shift, chunk, hist, G, n_dev);
        digit_scan_kernel<<<256, kThreads, 0, st>>>(hist, G, dtot);
        radix_scatter_kernel<K><<<G, kThreads, 0, st>>>(ki, vi, ko, vo, n, shift, chunk, hist, G, dtot, n_dev);
        std::swap(ki, ko);
        std::swap(vi, vo);
        flips ^= 1;
    }
    return flips;
}

}  // namespace

int scan_grid(int64_t n) {
    const int64_t per = (int64_t)kThreads * kItems;
    const int64_t g = (n + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

size_t scan_scratch_bytes(int64_t n) { return sizeof(uint64_t) * (size_t)(scan_grid(n) + 1); }

void launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t* total, int64_t n, void* scratch,
                           hipStream_t st) {
    uint64_t* sums = reinterpret_cast<uint64_t*>(scratch);
    if (n <= 0) {
        launch_clear_u32(reinterpret_cast<uint32_t*>(total), 2, st);  // kernel, not a memset node
        return;
    }
    if (n <= kScanSingleMax) {  // e.g. the per-tile list totals of a batch: one launch instead of three
        scan_single_kernel<<<1, kScanSingleThreads, 0, st>>>(in, n, out, total);
        return;
    }
    const int G = scan_grid(n);
    int64_t chunk = (n + G - 1) / G;
    chunk = ((chunk + kThreads * kItems - 1) / (kThreads * kItems)) * (kThreads * kItems);
    scan_reduce_kernel<<<G, kThreads, 0, st>>>(in, n, chunk, sums);
    scan_top_kernel<<<1, kThreads, 0, st>>>(sums, G, total);
    scan_down_kernel<<<G, kThreads, 0, st>>>(in, n, chunk, sums, out);
}

void launch_emit_keys(const Records& r, const uint32_t* offsets, const uint32_t* dbits, int B, int N, const Grid& g,
                      uint64_t capacity, bool full_keys, void* keys, uint32_t* vals, uint32_t* status,
                      unsigned long long* cull, hipStream_t st) {
    const int64_t total = (int64_t)B * N;
    if (total <= 0) return;
    const unsigned blocks = (unsigned)((total + kThreads - 1) / kThreads);
    if (full_keys)
        emit_keys_kernel<true><<<blocks, kThreads, 0, st>>>(r.rect, r.count, offsets, dbits, N, total, g.TW, g.tiles,
                                                            capacity, keys, vals, status, cull);
    else
        emit_keys_kernel<false><<<blocks, kThreads, 0, st>>>(r.rect, r.count, offsets, dbits, N, total, g.TW,
                                                             g.tiles, capacity, keys, vals, status, cull);
}

size_t radix_scratch_bytes(int64_t n) { return sizeof(uint32_t) * 256 * ((size_t)radix_grid(n) + 1); }

int launch_radix_sort(void* keys, uint32_t* vals, void* kalt, uint32_t* valt, int64_t n, int key_bytes, int begin_bit,
                      int end_bit, void* scratch, hipStream_t st, const uint64_t* n_dev) {
    uint32_t* hist = reinterpret_cast<uint32_t*>(scratch);
    if (key_bytes == 8)
        return radix_sort_t<uint64_t>(reinterpret_cast<uint64_t*>(keys), vals, reinterpret_cast<uint64_t*>(kalt), valt,
                                      n, begin_bit, end_bit, hist, st, n_dev);
    return radix_sort_t<uint32_t>(reinterpret_cast<uint32_t*>(keys), vals, reinterpret_cast<uint32_t*>(kalt), valt, n,
                                  begin_bit, end_bit, hist, st, n_dev);
}

namespace {
__global__ void clear_u32_kernel(uint32_t* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
}  // namespace

namespace {
// Key count the sort may use after a fixed-capacity emission: the scan total
// if it fits, else 0 (the emission skipped pairs, so the key array has holes;
// the batch renders empty and the caller re-runs it with exact sizing).
// An overflow also sets bit 0 of the status word.
__global__ void effective_count_kernel(const uint64_t* __restrict__ total, uint64_t cap, uint64_t* __restrict__ n_eff,
                                       uint32_t* __restrict__ status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint64_t t = *total;
        *n_eff = t <= cap ? t : 0ull;
        if (status) *status = t > cap ? 1u : 0u;  // stored, not or-ed: this sets the word for the launch's lists
    }
}
}  // namespace

void launch_effective_count(const uint64_t* total, uint64_t cap, uint64_t* n_eff, uint32_t* status, hipStream_t st) {
    effective_count_kernel<<<1, 64, 0, st>>>(total, cap, n_eff, status);
}

void launch_clear_u32(uint32_t* p, int n, hipStream_t st) {
    if (n > 0) clear_u32_kernel<<<(n + 255) / 256, 256, 0, st>>>(p, n);
}

void launch_tile_ranges(const void* keys, int key_bytes, int64_t n, int64_t n_gtiles, uint2* ranges, hipStream_t st,
                        const uint64_t* n_dev) {
    if (n_gtiles > 0) zero_ranges_kernel<<<(unsigned)((n_gtiles + 255) / 256), 256, 0, st>>>(ranges, n_gtiles);
    if (n <= 0) return;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (key_bytes == 8)
        tile_ranges_kernel<true><<<blocks, 256, 0, st>>>(keys, n, ranges, n_dev);
    else
        tile_ranges_kernel<false><<<blocks, 256, 0, st>>>(keys, n, ranges, n_dev);
}

bool bin_fits(int B, int N, const Grid& g) {
    // a periodic azimuth is binned with one segment
    return B <= 65535 && g.tiles <= kMaxTiles && (!g.wrap || g.tiles <= 256);
}

// The bins buffer: the histogram (B * S * nbq rows of 2^db), then the scanned
// tile totals (B * S * 2^db).
static size_t hist_entries(int B, const BinGeom& G) { return ((size_t)B * G.S * G.nbq) << G.db; }
static size_t start_entries(int B, const BinGeom& G) { return ((size_t)B * G.S) << G.db; }

size_t bin_hist_entries(int B, int N, const Grid& g) {
    const BinGeom G = bin_geom(N, g);
    return hist_entries(B, G) + start_entries(B, G);
}

size_t bin_scan_entries(int B, int N, const Grid& g) { return start_entries(B, bin_geom(N, g)); }

static void hist_launch(const BinGeom& G, int B, const Records& r, uint32_t* bins, unsigned long long* cull,
                        hipStream_t st, const MixBatch* m) {
    if (m)
        bin_hist_kernel<true><<<dim3(G.nbq, B), kThreads, 0, st>>>(r.rect, r.count, G, bins, cull, *m);
    else
        bin_hist_kernel<false><<<dim3(G.nbq, B), kThreads, 0, st>>>(r.rect, r.count, G, bins, cull);
}

static void offsets_launch(const BinGeom& G, int B, uint32_t* bins, void* scratch, uint64_t* total, hipStream_t st) {
    const int64_t cols = (int64_t)start_entries(B, G);
    uint32_t* starts = bins + hist_entries(B, G);
    bin_colscan_kernel<<<(unsigned)((cols + kThreads - 1) / kThreads), kThreads, 0, st>>>(bins, cols, G.nbq, G.db,
                                                                                          starts);
    launch_exclusive_scan(starts, starts, total, cols, scratch, st);
}

static void place_launch(const BinGeom& G, int B, const Records& r, const uint32_t* bins, const uint64_t* n_dev,
                         uint32_t* vals, hipStream_t st, const MixBatch* m) {
    const uint32_t* starts = bins + hist_entries(B, G);
    const dim3 grid(G.nbq, B);
    if (G.S == 1 && G.db == 8) {
        if (m)
            bin_place_kernel<true><<<grid, kThreads, 0, st>>>(r.rect, r.count, G, bins, starts, n_dev, vals, *m);
        else
            bin_place_kernel<false><<<grid, kThreads, 0, st>>>(r.rect, r.count, G, bins, starts, n_dev, vals);
    } else {
        if (m)
            bin_scatter_kernel<4, kWideDb, true><<<grid, kThreads, 0, st>>>(r.rect, r.count, G, bins, starts, n_dev,
                                                                            vals, *m);
        else
            bin_scatter_kernel<4, kWideDb><<<grid, kThreads, 0, st>>>(r.rect, r.count, G, bins, starts, n_dev, vals);
    }
}

void launch_bin_hist(const Records& r, int B, int N, const Grid& g, uint32_t* bins, unsigned long long* cull,
                     hipStream_t st) {
    if (B <= 0) return;
    const BinGeom G = bin_geom(N, g);
    if (N <= 0) {
        launch_clear_u32(bins, (int)hist_entries(B, G), st);
        return;
    }
    hist_launch(G, B, r, bins, cull, st, nullptr);
}

void launch_bin_offsets(int B, int N, const Grid& g, uint32_t* bins, void* scratch, uint64_t* total,
                        hipStream_t st) {
    if (B <= 0) {
        launch_clear_u32(reinterpret_cast<uint32_t*>(total), 2, st);
        return;
    }
    offsets_launch(bin_geom(N, g), B, bins, scratch, total, st);
}

void launch_bin_scatter(const Records& r, int B, int N, const Grid& g, const uint32_t* bins, const uint64_t* n_dev,
                        uint32_t* vals, hipStream_t st) {
    if (B <= 0 || N <= 0) return;
    place_launch(bin_geom(N, g), B, r, bins, n_dev, vals, st, nullptr);
}

void launch_bin_ranges(const uint32_t* bins, int B, int N, const Grid& g, const uint64_t* total,
                       const uint64_t* n_dev, uint2* ranges, hipStream_t st) {
    const int64_t m = (int64_t)B * g.tiles;
    if (m <= 0) return;
    const BinGeom G = bin_geom(N, g);
    bin_ranges_kernel<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(bins + hist_entries(B, G), B, G, total, n_dev,
                                                                    ranges);
}

// Mixed batches: the geometry of the batch's largest query (max_n pairs, max_tiles tiles) for every query.
static BinGeom mix_geom(int max_n, int max_tiles) {
    Grid g{};
    g.tiles = max_tiles;
    return bin_geom(max_n, g);
}

bool mix_bin_fits(int B, int max_tiles) { return B <= 65535 && max_tiles <= kMaxTiles; }

size_t mix_bin_hist_entries(int B, int max_n, int max_tiles) {
    const BinGeom G = mix_geom(max_n, max_tiles);
    return hist_entries(B, G) + start_entries(B, G);
}

size_t mix_bin_scan_entries(int B, int max_n, int max_tiles) { return start_entries(B, mix_geom(max_n, max_tiles)); }

void launch_mix_bin_hist(const MixBatch& m, int max_n, int max_tiles, const Records& r, uint32_t* bins,
                         unsigned long long* cull, hipStream_t st) {
    if (m.B <= 0) return;
    hist_launch(mix_geom(max_n, max_tiles), m.B, r, bins, cull, st, &m);
}

void launch_mix_bin_offsets(const MixBatch& m, int max_n, int max_tiles, uint32_t* bins, void* scratch,
                            uint64_t* total, hipStream_t st) {
    if (m.B <= 0) return;
    offsets_launch(mix_geom(max_n, max_tiles), m.B, bins, scratch, total, st);
}

void launch_mix_bin_scatter(const MixBatch& m, int max_n, int max_tiles, const Records& r, const uint32_t* bins,
                            const uint64_t* n_dev, uint32_t* vals, hipStream_t st) {
    if (m.B <= 0) return;
    place_launch(mix_geom(max_n, max_tiles), m.B, r, bins, n_dev, vals, st, &m);
}

void launch_mix_bin_ranges(const MixBatch& m, int max_n, int max_tiles, const uint32_t* bins, const uint64_t* total,
                           const uint64_t* n_dev, int64_t tile_cap, uint2* ranges, hipStream_t st) {
    if (tile_cap <= 0 || m.B <= 0) return;
    const BinGeom G = mix_geom(max_n, max_tiles);
    mix_bin_ranges_kernel<<<(unsigned)((tile_cap + 255) / 256), 256, 0, st>>>(bins + hist_entries(m.B, G), m, G,
                                                                               total, n_dev, tile_cap, ranges);
}

}  // namespace swf
