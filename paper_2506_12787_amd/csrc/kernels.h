// Host-side launch interface between the runtime (runtime.cpp) and the HIP
// kernel translation units of libswiftwrf.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swf {

// Device-resident scene. Gaussians are stored in ascending (depth, id) order
// ("sorted position" p); perm[p] is the caller's original index. Positions
// p >= n_live (NaN depth) never render.
struct DevScene {
    int n = 0, n_live = 0, H = 0, W = 0;
    float *mx = nullptr, *my = nullptr, *lsx = nullptr, *lsy = nullptr;
    float *rot = nullptr, *logit = nullptr, *amp = nullptr;
    uint32_t *dbits = nullptr;  // order-preserving depth bits
    uint32_t *perm = nullptr;   // sorted position -> original id
    uint32_t *inv_perm = nullptr;  // original id -> sorted position
    // deformation MLP (hidden width 256)
    bool has_mlp = false;
    int hidden = 0, n_hidden = 0, in_dim = 0;
    float *w[8] = {}, *b[8] = {};   // FP32 master, row-major [out][in]
    float *f32_frag = nullptr;      // FP32 weights in MFMA fragment order (layout below)
    uint16_t *bf_stream = nullptr;  // BF16 weights in MFMA fragment order (16 KiB units)
    uint16_t *bf_mfeat = nullptr;   // [n][32] BF16 gamma(mu_hat), zero padded
    float room_lo[3] = {0, 0, 0}, room_hi[3] = {6, 6, 3};
    uint64_t bytes = 0;
    // kind 1: the paper's own model (GMM sum over Cholesky Gaussians with tanh centres and complex responses,
    // in id order; paper.hip). Raw parameters, the FP64-mapped centres (hi, lo) and their 10-band encoding, and
    // the paper MLP: FP32 masters (out, in) and the kernel's fragment-major layers with padded biases.
    int kind = 0;
    float *pcx = nullptr, *pcy = nullptr, *pl1 = nullptr, *pl2 = nullptr, *pl3 = nullptr;
    float *patt = nullptr, *ppre = nullptr, *ppim = nullptr;
    float4* pcen = nullptr;
    float* pfeat = nullptr;
    float *pw[9] = {}, *pb[9] = {};
    float *pwt[9] = {}, *pbt[9] = {};
};

// FP32 weights of the deformation MLP in the fragment order of the FP32 MFMA
// kernel (pe_mlp.hip), one float4 per lane and fragment (16 output units x 4
// input chunks of 4): layer 1's mean part (16 tiles x 2 fragments, K = 26
// padded to 32), each hidden -> hidden layer (16 tiles x 16 fragments), the
// output layer (1 tile x 16 fragments, rows 7..15 zero), then the output bias
// padded to 16. Built on the device from the FP32 masters (pack.hip).
constexpr size_t kFragL1 = 16 * 2 * 64 * 4;
constexpr size_t kFragHidden = 16 * 16 * 64 * 4;
constexpr size_t kFragOut = 16 * 64 * 4;
__host__ __device__ inline size_t frag_hidden_at(int L) { return kFragL1 + (size_t)(L - 1) * kFragHidden; }  // L = 1 .. n_hidden - 1
__host__ __device__ inline size_t frag_out_at(int n_hidden) { return kFragL1 + (size_t)(n_hidden - 1) * kFragHidden; }
__host__ __device__ inline size_t frag_floats(int n_hidden) { return frag_out_at(n_hidden) + kFragOut + 16; }

// The paper's model (paper.hip): positional encoding bands, layer sizes and
// padded layouts of its MLP.
constexpr int kPaperCenterBands = 10;
constexpr int kPaperTxBands = 6;
constexpr int kPaperCenterFeat = 2 * (2 * kPaperCenterBands + 1);  // 42
constexpr int kPaperTxFeat = 3 * (2 * kPaperTxBands + 1);          // 39
constexpr int kPaperFeatStride = 48;
constexpr int kPaperLayers = 8;
constexpr int kPaperWidth = 156;
constexpr int kPaperOut = 5;
constexpr int kPaperOutPad = 8;

struct Records {
    float4 *geo = nullptr;
    float4 *wm = nullptr;
    float2 *oa = nullptr;
    uint2 *rect = nullptr;
    uint32_t *count = nullptr;
};

struct Grid {
    int H, W, tile, TW, TH, tiles;  // tiles per query
    int wrap;                       // 1: periodic azimuth (period W)
    float sx, sy;                   // render pixels per scene pixel (1 at the scene's own grid)
};

struct PaperArgs {
    int N, B, H, W, TW, TH, wrap;
    float inv_tile, sx, sy;
    const float4* cen;
    const float *l1, *l2, *l3, *att, *pre, *pim;
    const float* feat;  // [N][48] centre features
    const float* txf;   // [B][48] position features
    const float* wt[kPaperLayers];  // fragment-major MFMA operands (paper.hip)
    const float* bt[kPaperLayers];  // biases padded to 160
    const float* wo;                // output layer, one 16-row tile
    const float* bo;                // output biases padded to 16
    Records rec;
    float* delta_out;  // [B * N][5] residuals (debug), or null
};

// A batch of queries over several resident scenes, each with its own Gaussian
// count and grid (mixed.hip): a table of the distinct scenes and one of the
// queries (B + 1 entries; the last holds the totals), both in device memory.
struct MixScene {
    const float *mx, *my, *lsx, *lsy, *rot, *logit, *amp;  // canonical parameters, (depth, id) order
    const float *w1, *b1;                                   // layer 1, row-major [256][89], for the TX term
    const uint16_t* stream;                                 // BF16 weight stream
    const float* f32_frag;                                  // FP32 weights, fragment-major (frag_floats(4))
    const uint16_t* mfeat;                                  // BF16 gamma(mu_hat) [N][32]
    const float* bias_h[7];
    const float* bias_o;
    float room_lo[3], room_hi[3];
    int N, n_live, H, W, TW, TH, tiles;
};
struct MixQuery {
    int scene;          // index into the scene table
    int pair_base;      // first record of the query
    int tile_base;      // first global tile of the query
    int out_base;       // first output value of the query (spectra concatenated in query order)
    int mlp_tile_base;  // first MLP tile (block of pairs) of the query
};
struct MixBatch {
    const MixScene* scenes;
    const MixQuery* queries;
    int B;
};
// Index q of the query whose range [field(q), field(q + 1)) holds v (B + 1 entries, non-decreasing).
template <typename F>
__device__ __forceinline__ int mix_find(const MixQuery* qs, int B, int v, F field) {
    int lo = 0, hi = B;  // field(lo) <= v < field(hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (field(qs[mid]) <= v)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// mixed.hip
void launch_mix_tx_features(const MixBatch& m, const float* tx, float* qs, hipStream_t st);
void launch_mix_static(const MixBatch& m, int64_t pair_cap, const Grid& tile, const Records& r, hipStream_t st);
void launch_mix_clear_tail(const MixBatch& m, int64_t pair_cap, const Records& r, hipStream_t st);
// Lists of a mixed batch by binning (sort.hip), with the geometry of its largest query (max_n pairs, max_tiles
// tiles) for every query; ranges over its global tiles.
bool mix_bin_fits(int B, int max_tiles);
size_t mix_bin_hist_entries(int B, int max_n, int max_tiles);
size_t mix_bin_scan_entries(int B, int max_n, int max_tiles);
void launch_mix_bin_hist(const MixBatch& m, int max_n, int max_tiles, const Records& r, uint32_t* bins,
                         unsigned long long* cull, hipStream_t st);
void launch_mix_bin_offsets(const MixBatch& m, int max_n, int max_tiles, uint32_t* bins, void* scan_scratch,
                            uint64_t* total, hipStream_t st);
void launch_mix_bin_scatter(const MixBatch& m, int max_n, int max_tiles, const Records& r, const uint32_t* bins,
                            const uint64_t* n_dev, uint32_t* vals, hipStream_t st);
void launch_mix_bin_ranges(const MixBatch& m, int max_n, int max_tiles, const uint32_t* bins, const uint64_t* total,
                           const uint64_t* n_dev, int64_t tile_cap, uint2* ranges, hipStream_t st);
void launch_mix_emit_keys(const MixBatch& m, const Records& r, const uint32_t* offsets, int64_t pair_cap,
                          uint64_t capacity, uint32_t* keys, uint32_t* vals, uint32_t* status,
                          unsigned long long* cull, hipStream_t st);
// blend.hip: one workgroup per global tile of the batch, tile_cap of them (the extra ones exit)
void launch_mix_blend(const MixBatch& m, int tile_cap, const uint2* ranges, const uint32_t* vals, const Records& r,
                      float* out, hipStream_t st);
// mlp_bf16.hip: the BF16 MLP over the batch's tiles of pairs (the default 384-pair variant)
void launch_mix_mlp_bf16(const MixBatch& m, const float* qs, const Records& r, hipStream_t st, bool paper_mask,
                         bool wrap);
// The FP32 MLP over a mixed batch (every scene with four hidden layers of 256): every 16-pair group of the batch's
// 384-pair MLP tiles, at most pair_cap pairs over B_cap queries (graph-capturable: the batch's totals are read from
// its tables).
void launch_mix_mlp_fp32(const MixBatch& m, const float* qs, const Records& r, int64_t pair_cap, int B_cap,
                         hipStream_t st, bool paper_mask, bool wrap);

// paper.hip
void launch_paper_centers(const DevScene& d, hipStream_t st);
void launch_paper_tx(const DevScene& d, const float* tx, int B, float* txf, hipStream_t st);
void launch_paper_static(const DevScene& d, int B, const Grid& g, const Records& r, hipStream_t st);
void launch_paper_mlp(const DevScene& d, const float* txf, int B, const Grid& g, const Records& r, float* delta_out,
                      hipStream_t st);
// out [B][H][W] = |sum|; chan (may be null) [B][2][H][W] = (re, im)
void launch_gmm_blend(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g, float* out,
                      float* chan, hipStream_t st);

// pe_mlp.hip
void launch_tx_features(const DevScene& s, const float* tx, int B, float* qs, hipStream_t st,
                        float* feat_out = nullptr);
// FP32 backward of a 256 x 256 layer on the FP32 matrix cores: wt = W^T packed fragment-major (65536 floats, from
// W [256][256] row-major); out [P][256] = (dz [P][256] W) masked by act [P][256] > 0; with bpart (non-null,
// [dz_f32_blocks(P)][256]) also the per-block column sums of dz (the layer's bias gradient before their sum).
void launch_pack_wt(const float* w, float* wt, hipStream_t st);
int64_t dz_f32_blocks(int64_t P);
void launch_dz_f32(const float* dz, const float* wt, const float* act, int64_t P, float* out, float* bpart,
                   hipStream_t st);
void launch_mlp_fp32(const DevScene& s, const float* qs, int B, const Grid& g, bool paper_mask, const Records& r,
                     float* delta_out, hipStream_t st, float* const* act_out = nullptr);
void launch_preprocess_static(const DevScene& s, int B, const Grid& g, const Records& r, hipStream_t st);
void launch_gather_params(float* const* src, const uint32_t* perm, int n, float* const* dst, hipStream_t st);
void launch_permute_delta(const float* delta_sorted, const uint32_t* perm, int B, int n, float* delta_out,
                          hipStream_t st);

// mlp_bf16.hip
bool bf16_available();
void compute_mean_features_bf16(DevScene& s, hipStream_t st);
// pack.hip: rebuild the fragment-major FP32 copy and the BF16 weight stream from
// the FP32 master weights d.w[] on the device (after a device-side MLP update)
void launch_pack_mlp(const DevScene& d, hipStream_t st);
// the fragment-major FP32 copy alone (frag_floats(n_hidden) floats at d.f32_frag)
void launch_pack_f32_frag(const DevScene& d, hipStream_t st);

// act_out (optional): also store the hidden activations, BF16 [n_hidden][B * N][256] (the backward's operands)
void launch_mlp_bf16(const DevScene& s, const float* qs, int B, const Grid& g, bool paper_mask, const Records& r,
                     float* delta_out, hipStream_t st, int pairs_per_wave, void* act_out = nullptr);

// sort.hip
int scan_grid(int64_t n);
size_t scan_scratch_bytes(int64_t n);
void launch_exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t* total, int64_t n, void* scratch,
                           hipStream_t st);
void launch_emit_keys(const Records& r, const uint32_t* offsets, const uint32_t* dbits, int B, int N,
                      const Grid& g, uint64_t capacity, bool full_keys, void* keys, uint32_t* vals,
                      uint32_t* status, unsigned long long* cull, hipStream_t st);
size_t radix_scratch_bytes(int64_t n);
// Sorts (keys, vals) on bits [begin_bit, end_bit); returns 1 if the result
// ended in the alternate buffers (kalt, valt), 0 if in (keys, vals).
// n_dev (optional): key count on the device; then n is the capacity and the
// kernels use min(*n_dev, n) (no host synchronisation, graph-capturable).
int launch_radix_sort(void* keys, uint32_t* vals, void* kalt, uint32_t* valt, int64_t n, int key_bytes,
                      int begin_bit, int end_bit, void* scratch, hipStream_t st, const uint64_t* n_dev = nullptr);
void launch_tile_ranges(const void* keys, int key_bytes, int64_t n, int64_t n_gtiles, uint2* ranges,
                        hipStream_t st, const uint64_t* n_dev = nullptr);
void launch_clear_u32(uint32_t* p, int n, hipStream_t st);
// n_eff = total if total <= cap else 0; *status (if not null) is set to 1 if total > cap, else to 0
void launch_effective_count(const uint64_t* total, uint64_t cap, uint64_t* n_eff, uint32_t* status, hipStream_t st);
// Binning path: per-block histograms of each tile segment of a query, their
// column prefixes and the scanned tile totals (`bins` holds both), then the
// stable placement of pair indices into per-tile lists and the tile ranges.
bool bin_fits(int B, int N, const Grid& g);  // the segment grid fits one launch
size_t bin_hist_entries(int B, int N, const Grid& g);  // uint32 entries of `bins`
size_t bin_scan_entries(int B, int N, const Grid& g);  // entries the tile-total scan runs over
// cull (may be null): two device counters that receive the number of culled
// pairs, non-finite / degenerate and off the grid (also launch_emit_keys)
void launch_bin_hist(const Records& r, int B, int N, const Grid& g, uint32_t* bins, unsigned long long* cull,
                     hipStream_t st);
// column prefixes in place, tile starts, and the number of list entries in *total
void launch_bin_offsets(int B, int N, const Grid& g, uint32_t* bins, void* scan_scratch, uint64_t* total,
                        hipStream_t st);
void launch_bin_scatter(const Records& r, int B, int N, const Grid& g, const uint32_t* bins,
                        const uint64_t* n_dev, uint32_t* vals, hipStream_t st);
void launch_bin_ranges(const uint32_t* bins, int B, int N, const Grid& g, const uint64_t* total,
                       const uint64_t* n_dev, uint2* ranges, hipStream_t st);

// backward.hip
// det_part (may be null): per (list entry, wave) sums, 32 floats per entry of the lists, zeroed by the caller;
// with it the per-pair sums in dpair are taken in a fixed order (N: Gaussians per query)
void launch_blend_backward(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                           const float* grad_out, const float* aux_T, const uint32_t* aux_last, float* dpair,
                           hipStream_t st, float* det_part = nullptr, int N = 0, const uint32_t* det_off = nullptr);
void launch_preprocess_backward(const float* dpair, const Records& r, int64_t P, bool paper_mask, float* dbase,
                                float* dy, hipStream_t st);
struct BaseGrads {  // destinations of the 7 base-parameter gradients (device; NULL skips one)
    float* p[7];
};
void launch_base_reduce(const float* dbase, const float* dmu_pe, const uint32_t* perm, int B, int N,
                        const BaseGrads& out, hipStream_t st);
// gemm.hip: C = op(A) op(B) in FP32 on the matrix cores, row-major (op(A) M x K, op(B) K x N; A / B FP32, or
// BF16 bits when bf16). mask (optional, leading dimension ldm): C *= [mask > 0]. A small C over a long K is
// split into gemm_split(M, N, K) K-slices summed in slice order; part then holds gemm_part_floats(M, N, K)
// floats (unused otherwise).
int gemm_split(int64_t M, int64_t N, int64_t K);
size_t gemm_part_floats(int64_t M, int64_t N, int64_t K);
void launch_gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                     int64_t ldb, float* C, int64_t ldc, float* part, hipStream_t st, const float* mask = nullptr,
                     int64_t ldm = 0, bool bf16 = false);
void launch_fill(float* p, float v, int64_t n, hipStream_t st);
// out[z * out_bs + c] = sum_r A[z * bs + r * cols + c] for z < nz; part holds
// colsum_blocks(rows) * cols * nz floats
int colsum_blocks(int64_t rows);
void launch_colsum(const float* A, int64_t rows, int64_t cols, int nz, int64_t bs, float* part, float* out,
                   int64_t out_bs, hipStream_t st);
// dg: [N][26] gradient of gamma(mu_hat) summed over the batch -> dmu [N][2]
void launch_pe_chain(const float* dg, const DevScene& s, float* dmu, hipStream_t st);
// Input gradient of a 256 x 256 layer on MFMA: out = dz W (dz [P][256] BF16, W [256][256] BF16 row-major
// [out][in]); FP32 output (f32_out) or BF16 output masked by act > 0 (act [P][256] BF16)
void launch_dz_gemm(const void* dz, const void* W, const void* act, int64_t P, void* out, bool f32_out,
                    hipStream_t st);
// Weight gradient of a 256 x 256 layer on MFMA: dW [256][256] = dz^T act (dz, act [P][256] BF16; FP32 sums),
// and, when db is not NULL, the bias gradient db [256] = the column sums of dz.
// part: wgrad_mfma_blocks(P) * (65536 + 256) floats; tmp: column-sum scratch.
int wgrad_mfma_blocks(int64_t P);
void launch_wgrad_mfma(const void* dz, const void* act, int64_t P, float* part, float* tmp, float* dW, float* db,
                       hipStream_t st);
// Layer-1 gradient sums of a BF16 backward straight from dz1 [B][N][256] (the second layer's pre-activation
// gradient, BF16) and W (its 256 x 256 BF16 weights): S [N][256] = sum over b of (dz1 W) masked by act > 0, and
// Rpart [layer1_grad_blocks(N)][B][256] per-block sums over the Gaussians.
int layer1_grad_blocks(int N);
void launch_layer1_grad(const void* dz1, const void* W, const void* act, int B, int N, float* S, float* Rpart,
                        hipStream_t st);
// Output layer of a BF16 backward in one pass over act [P][256]: dz (may be NULL) = (dy Wo) rounded to BF16 and
// masked by act > 0; dWo [7][256] (may be NULL) = dy^T act. part: wgrad_out_blocks(P) * 7 * 256 floats.
void launch_out_bwd_bf16(const float* dy, const void* wo, const void* act, int64_t P, void* dz, float* part,
                         float* tmp, float* dWo, hipStream_t st);
int wgrad_out_blocks(int64_t P);  // blocks (pair slices) of launch_out_bwd_bf16
// S [N][256] = sum_b of z * [act > 0] (act BF16; null: z is masked already) and Rpart [layer1_sums_blocks(N)][B][256]
// partial sums over Gaussians
int layer1_sums_blocks(int N);
void launch_layer1_sums(const float* z, const void* act, int B, int N, float* S, float* Rpart, hipStream_t st);
void launch_to_bf16(const float* x, int64_t n, void* y, hipStream_t st);
void launch_colsum_bf16(const void* A, int64_t rows, int64_t cols, int nz, int64_t bs, float* part, float* out,
                        int64_t out_bs, hipStream_t st);
void launch_mean_features_f32(const DevScene& s, float* out, hipStream_t st);

// blend.hip
void launch_blend_forward(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                          float* out, float* aux_T, uint32_t* aux_last, hipStream_t st);
// work[0] += (pixel, entry) evaluations, work[1] += records staged (counting run, no output)
void launch_blend_work(const uint2* ranges, const uint32_t* vals, const Records& r, int B, const Grid& g,
                       unsigned long long* work, hipStream_t st);

// peak probes (probe.hip)
size_t probe_scratch_bytes(int blocks);
hipError_t run_probes(int blocks, void* scratch, hipStream_t st, double* mfma_tflops, double* fma_tops,
                      double* lds_tbps);
int n_compute_units();

}  // namespace swf
