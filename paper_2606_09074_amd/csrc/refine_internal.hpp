// Internal declarations of the REFINE HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "../../include/refine.h"

namespace refine {

constexpr int kPlanes = 59;
constexpr int kScorePlanes = 14;   // centre, log-scale, quaternion, opacity, SH DC
constexpr int kGeomPlanes = 11;    // planes stored in the scene's dtype; the rest in its sh_dtype

// Supported scene storage formats (dtype of planes 0..10, dtype of 11..58).
enum Storage : int {
    kStoreF32 = 0,       // FP32, FP32
    kStoreBF16F16 = 1,   // BF16, FP16
    kStoreF16 = 2        // FP16, FP16
};

// Calls f with the storage format as a compile-time constant.
template <class F>
inline void with_storage(int st, F&& f)
{
    switch (st) {
    case kStoreF32: f(std::integral_constant<int, kStoreF32>{}); break;
    case kStoreBF16F16: f(std::integral_constant<int, kStoreBF16F16>{}); break;
    default: f(std::integral_constant<int, kStoreF16>{}); break;
    }
}

__host__ __device__ inline size_t storage_bytes(int st) { return st == kStoreF32 ? 4 : 2; }
constexpr int kCamFields = 18;
constexpr int kBlock = 256;        // threads per block of the tile kernels (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kItems = 16;         // elements per thread of the tile kernels
constexpr int kTile = kBlock * kItems;
constexpr int kCamRec = 32;        // floats per prepared camera record
constexpr int kHistBits = 11;
constexpr int kHistBins = 1 << kHistBits;
constexpr int kHistCopies = 8;    // selection histogram copies: spreads the atomics on crowded bins
constexpr int kSuperWidth = 32;    // bins per super-bin of a pass's coarse histogram
constexpr int kCoarseBins = kHistBins / kSuperWidth;   // 64
// one pass: kHistCopies copies of the kHistBins bins, then kHistCopies copies of the coarse bins
constexpr int kPassWords = kHistCopies * (kHistBins + kCoarseBins);
constexpr int kSelectHistWords = 3 * kPassWords;   // one set per radix pass
constexpr int kSelectStates = 4;   // selection state before pass 0, after passes 0, 1 and 2
constexpr int kSelectLastBins = 1 << 10;   // digits of the last radix pass (its per-tile rows)
constexpr int kStatSlots = 8;      // doubles per stats partial
constexpr int kNoAllocStatTiles = REFINE_STATS_NOALLOC_MAX_N / kTile;   // tiles of refine_stats_noalloc
static_assert(REFINE_STATS_NOALLOC_MAX_N % kTile == 0, "whole tiles of scratch");

// Prepared camera record (fp32, 128 bytes), built by camera_prep.  Pixel
// quantities are scaled by sv = 1 / sqrt(fx^2 + fy^2): the gate is invariant
// under that scaling and the projection term of mode COV becomes
// (a + c) / (z^2 + eta) with no per-camera factor.
// The image coordinates are taken about the image centre: with
// ox = sv (cx - W/2), X = sv fx x + ox z gives X / z = sv (u - W/2).
struct CamRec {
    float px[4];       // sv fx R_v row 0 + ox R_v row 2, sv fx t_x + ox t_z
    float py[4];       // sv fy R_v row 1 + oy R_v row 2, sv fy t_y + oy t_z
    float pz[4];       // R_v row 2, t_z               -> z
    float cx0, cx1;    // EWA clamp interval of X / z: ox -+ sv clamp_k W/2
    float cy0, cy1;    // of Y / z: oy -+ sv clamp_k H/2
    float hw, hh;      // sv W/2, sv H/2
    float kvs;         // sv kv3: a pair whose footprint can reach the image has d z < kvs s_max
    float pad[13];
};
static_assert(sizeof(CamRec) == kCamRec * sizeof(float), "camera record size");

// Device-resident state of one selection (lives in the workspace, one slot
// per stage: kSelectStates consecutive records).
struct SelectState {
    int64_t n;
    int64_t n_prune;
    int64_t rank;       // 0-based rank still to be located inside the current prefix bucket
    int64_t k_eq;       // pruned primitives whose key equals the threshold
    int64_t n_keep;
    uint32_t prefix;    // resolved high bits of the threshold key
    uint32_t mask;
    uint32_t threshold;
    uint32_t pad[7];
};

// The state a selection starts from (the threshold search has resolved no
// bits yet and looks for rank n_prune - 1).
__host__ __device__ inline SelectState select_start(int64_t n, int64_t n_prune)
{
    SelectState s = {};
    s.n = n;
    s.n_prune = n_prune;
    s.rank = n_prune - 1;
    s.k_eq = 0;
    s.n_keep = n - n_prune;
    return s;
}

// Conservative view-frustum test data of one view (fp32, 128 bytes): the
// world-space half-spaces every visible primitive's centre must satisfy,
// given a bound on its footprint radius.  Built by camera_prep.
struct CullRec {
    float nz[4];        // R_v row 2, t_z: depth = nz . mu + nz[3]
    float side[4][4];   // per image edge: n (3), d; visible => n . mu + d + 3 s_max kv > 0
    float nn[4];        // |n| of each side
    float kv3;          // 3 (1 + margin) max |z J|_2 over the clamp box (footprint: r z <= kv3 s_max)
    float pad[7];
};
static_assert(sizeof(CullRec) == 32 * sizeof(float), "cull record size");

// Activated primitive in binned order (64 bytes), written by bin_scatter;
// the centre and largest scale come first, so the group-bounds pass reads
// only the first 16 bytes.
struct PrimRec {
    float mu[3];
    float smax;        // largest scale
    float L[9];        // 3 R(q) diag(s), row-major (the 3-sigma factor folded in)
    float pre;         // epilogue factor V K [/ (9 sbar^2) in COV mode]
    int32_t idx;       // input index
    float pad;
};
static_assert(sizeof(PrimRec) == 64, "primitive record size");

// Conservative bounds of a group of kGroup consecutive binned records: the
// box c +- h and the sphere (c, rm) hold every centre (both inflated by the
// culling margin), sg is the group's largest scale.
struct GroupBound {
    float c[3];
    float h[3];
    float rm;
    float sg;
};
static_assert(sizeof(GroupBound) == 32, "group bound size");

constexpr int kGroup = 64;         // records per group: one per lane of a wave
constexpr int kOrderBuckets = 32;  // work classes of the group order (most views first)
constexpr int kOrderCopies = 8;    // copies of the class counts (one per block residue: fewer atomics per address)
// view-loop order state: kOrderBuckets cursors, then kOrderCopies x kOrderBuckets class counts
constexpr int kOrderAuxWords = kOrderBuckets * (1 + kOrderCopies);

__host__ __device__ inline int64_t num_groups(int64_t n, int per) { return (n + per - 1) / per; }

constexpr int kEvalSlots = 64;                     // counters the evaluated pairs are spread over

constexpr int kCellBits = 4;                       // per axis
constexpr int kCells = 1 << (3 * kCellBits);       // 4096 Morton cells (16 KB of LDS counters)
constexpr int kBinCopies = 8;                      // global cell counters per cell (one per block residue)

struct Workspace {
    SelectState* sel;
    uint32_t* hist;          // [3 passes][kHistCopies][kHistBins]
    double* stat_part;       // [ntiles][kStatSlots]
    uint32_t* tile_cnt;      // [ntiles]
    uint32_t* tile_off;      // [ntiles]
    uint32_t* tile_rows;     // [ntiles][kSelectLastBins] when ntiles <= kPrefixTilesMax, else null
    // refine_score only:
    CamRec* cams;            // [n_views]
    CullRec* culls;          // [n_views]
    uint32_t* cell_cnt;      // [kBinCopies][kCells]
    uint32_t* cell_cur;      // [kBinCopies][kCells]
    uint32_t* dest;          // [n] binned position of each primitive
    PrimRec* recs;           // [n] activated primitives in binned order
    GroupBound* gbound;      // [num_groups(n, kGroup)]
    int32_t* gorder;         // [num_groups(n, kGroup)] group order of the view loop
    uint32_t* gcount;        // [num_groups(n, kGroup)] views each view-loop group evaluates
    uint32_t* gaux;          // [kOrderAuxWords] work-class cursors and counts
    uint64_t* gmask;         // [num_groups(n, kGroup)][ceil(n_views / 64)] views each group evaluates
    unsigned long long* evaluated;   // [2][kEvalSlots] pairs evaluated in full / screened out by the last view loop
};

__host__ __device__ inline int64_t num_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

// Views scored: all, or the subsample of n_sub_views (views floor(j V / m)).
inline int views_of(const refine_params& prm, int32_t n_views)
{
    return (prm.n_sub_views > 0 && prm.n_sub_views < n_views) ? prm.n_sub_views : n_views;
}

// One prune of a grouped launch (refine_prune_batch): its inputs, outputs,
// workspace slices and its first tile / 256-primitive block in the batch's
// numbering.  A device copy of the table is read by every grouped kernel.
struct BatchJob {
    const void* planes;
    int64_t stride;
    int32_t n;
    int32_t st;              // Storage
    const float* cams;
    int32_t n_views;
    int32_t nv;              // views actually scored (subsampling)
    refine_stats_t* stats;
    float* scores;
    uint8_t* keep;
    int64_t n_prune;
    int64_t* n_keep_out;
    void* out;
    int64_t out_stride;
    int64_t capacity;
    int32_t* index_map;
    int64_t* n_out;
    double* stat_part;       // [ntiles][kStatSlots]
    struct CamRec* cam_rec;  // [nv]
    struct SelectState* sel;
    uint32_t* hist;          // [kSelectHistWords]
    uint32_t* tile_cnt;      // [ntiles]
    uint32_t* tile_rows;     // [ntiles][kSelectLastBins]
    int32_t tile0;           // first tile in the batch's tile numbering
    int32_t block0;          // first 256-primitive block in the batch's block numbering
    int32_t vec_compact;     // 16-byte-load compaction applies
    int32_t pair_store;      // 2-byte output written two elements per store
    int32_t vec_stats;       // 16-byte-load statistics apply (as in the single-scene call)
};

// Index of the job whose range [first, next first) holds b (first of job 0 is 0).
template <bool BY_TILE>
__device__ inline int batch_job_of(const BatchJob* __restrict__ jobs, int nj, int b)
{
    int lo = 0, hi = nj - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int first = BY_TILE ? jobs[mid].tile0 : jobs[mid].block0;
        if (first <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Bytes of a workspace for (n, n_views); fills *ws when base != nullptr.  With
// score == false only the prefix used by stats/select/compact is counted.
size_t workspace_layout(int64_t n, int32_t n_views, bool score, void* base, Workspace* ws);

// Launchers (validated arguments; return the hipGetLastError of the launch).
// `st` is the scene's Storage.
hipError_t launch_stats(const void* planes, int st, int64_t stride, int64_t n, const refine_params& prm,
                        refine_stats_t* d_stats, const Workspace& ws, hipStream_t stream);
hipError_t launch_score_prepare(const void* planes, int st, int64_t stride, int64_t n, const float* d_cams,
                                int32_t n_views, const refine_params& prm, const refine_stats_t* d_stats,
                                const Workspace& ws, hipStream_t stream);
// Device address of this device's refine_stats_noalloc scratch (the tile
// partials of kNoAllocStatTiles tiles), resolved on the first call per device
// (the current device).
hipError_t stats_scratch(double** out);
hipError_t launch_stats_batch(const BatchJob* d_jobs, int n_jobs, int total_tiles, const refine_params& prm,
                              hipStream_t stream);
hipError_t launch_score_batch(const BatchJob* d_jobs, int n_jobs, int total_blocks, const refine_params& prm,
                              hipStream_t stream);
hipError_t launch_select_batch(const BatchJob* d_jobs, int n_jobs, int total_tiles, hipStream_t stream);
hipError_t launch_compact_batch(const BatchJob* d_jobs, int n_jobs, int total_tiles, hipStream_t stream);
hipError_t launch_score_cameras(const float* d_cams, int32_t n_views, int64_t n, const refine_params& prm,
                                const Workspace& ws, hipStream_t stream);
hipError_t launch_score_views(const void* planes, int st, int64_t stride, int64_t n, int32_t n_views,
                              const refine_params& prm, const refine_stats_t* d_stats, float* d_scores,
                              int64_t* d_evaluated, const Workspace& ws, hipStream_t stream);
hipError_t launch_select(const float* d_scores, int64_t n, int64_t n_prune, uint8_t* d_keep,
                         int64_t* d_n_keep, uint32_t* d_threshold, const Workspace& ws,
                         hipStream_t stream);
hipError_t launch_compact(const void* in, int st, int64_t in_stride, int64_t n, const uint8_t* d_keep,
                          void* out, int64_t out_stride, int64_t capacity, int32_t* d_index_map,
                          int64_t* d_n_out, const Workspace& ws, hipStream_t stream);

// ------------------------------------------------------------ device helpers

// Sum over a wave64 by xor butterflies: every lane ends with the same value,
// and the association order depends only on lane positions (deterministic).
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// A 2-byte element of plane p as FP32, exactly: BF16 (its bits are the high
// half of an FP32) for the geometry planes of kStoreBF16F16, FP16 (every
// half is a float) otherwise.
template <int ST>
__device__ __forceinline__ float widen2(uint16_t b, int p)
{
    if (ST == kStoreBF16F16 && p < kGeomPlanes) return __uint_as_float((uint32_t)b << 16);
    return (float)__builtin_bit_cast(_Float16, b);
}

// Plane p of primitive i as FP32.
template <int ST>
__device__ __forceinline__ float load_plane(const void* __restrict__ planes, int64_t stride, int p, int64_t i)
{
    const int64_t at = (int64_t)p * stride + i;
    if constexpr (ST == kStoreF32) {
        return static_cast<const float*>(planes)[at];
    } else {
        return widen2<ST>(static_cast<const uint16_t*>(planes)[at], p);
    }
}

// Number of set bits of a wave ballot below this lane.
__device__ inline uint32_t lanes_below(uint64_t ballot)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

// Order-preserving unsigned key of a float: a < b  <=>  key(a) < key(b);
// -0 maps to the key of +0 and every NaN to the largest key.
__device__ inline uint32_t float_key(float f)
{
    if (f != f) return 0xFFFFFFFFu;
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

}  // namespace refine

namespace refine {

constexpr int kScanThreads = 1024;

// Exclusive prefix sum of cnt[0..m) into off[0..m) by one block of THREADS
// threads (each thread scans a contiguous chunk); returns the total in every
// thread.  Integer only, so the result is exact.
template <int THREADS>
__device__ inline uint32_t block_exclusive_scan_t(const uint32_t* __restrict__ cnt, uint32_t* __restrict__ off, int m)
{
    __shared__ uint32_t wave_tot[THREADS / 64];
    const int chunk = (m + THREADS - 1) / THREADS;
    const int lo = threadIdx.x * chunk;
    const int hi = min(lo + chunk, m);
    uint32_t local = 0;
    for (int j = lo; j < hi; ++j) local += cnt[j];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < THREADS / 64; ++w) {
        if (w < wave) before += wave_tot[w];
        total += wave_tot[w];
    }
    uint32_t run = before + incl - local;
    for (int j = lo; j < hi; ++j) {
        const uint32_t c = cnt[j];
        off[j] = run;
        run += c;
    }
    return total;
}

__device__ inline uint32_t block_exclusive_scan(const uint32_t* __restrict__ cnt, uint32_t* __restrict__ off, int m)
{
    return block_exclusive_scan_t<kScanThreads>(cnt, off, m);
}

// Tiles at most this many: a block finds its output offset by summing the
// counts of the tiles before it (no separate scan launch).
constexpr int kPrefixTilesMax = 4096;

// Sum of cnt[0], cnt[stride], ... (m terms) by one block of kBlock threads;
// every thread gets it.
__device__ inline uint64_t block_sum_prefix(const uint32_t* __restrict__ cnt, int m, int stride = 1)
{
    __shared__ uint64_t part[kWaves];
    uint64_t s = 0;
    for (int t = threadIdx.x; t < m; t += kBlock) s += cnt[(size_t)t * stride];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    uint64_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tot += part[w];
    return tot;
}

}  // namespace refine
