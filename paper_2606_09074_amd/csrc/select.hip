// Global ranking and ratio selection (paper Sec. 3.3) on gfx950.
//
// Scores become order-preserving 32-bit keys.  The key of the n_prune-th
// smallest primitive (the threshold T) is found by three most-significant-
// digit-first radix passes (11, 11, 10 bits).  Each pass histograms, into
// one LDS histogram per tile, the keys that share the prefix resolved so far,
// adds them into a global histogram with integer atomics (exact and
// order-independent; 8 copies, one per block residue, so the crowded bins of
// the first pass take 8x fewer atomics per address), and a one-block pass
// sums the copies, scans them and picks the bucket holding the target rank.
// (Folding that pass into the last histogram block would need a device-scope
// fence per block, which on this multi-die part writes back the L2: a
// separate launch is cheaper; so is this than having every histogram block
// rescan the previous histograms itself.)  Ties at T are broken by
// index: the pruned primitives are every key < T plus the k_eq lowest-index
// keys == T, located with wave ballots and the exact count of equal keys in
// the tiles before.  Integer arithmetic throughout, so the mask equals a
// stable sort by (score, index).
//
// The last histogram pass also writes each tile's row of last-digit counts
// (4 KB per tile, from the LDS histogram it builds anyway): once T is known,
// the count of keys equal to T in tile t is row t at T's last digit, so no
// separate counting pass over the keys is needed.  (Inputs of more than
// kPrefixTilesMax tiles count per tile and scan in separate launches.)
//
// Launches: init, 3 x (histogram, find), mask -- once per call, or once for
// all the jobs of a batch (select_*_batch, the same bodies; there the init
// rides in the statistics finalisation).
#include "refine_internal.hpp"

namespace refine {

namespace {

constexpr int kPassShift[3] = {21, 10, 0};
constexpr int kPassBits[3] = {11, 11, 10};
static_assert(1 << kPassBits[2] == kSelectLastBins, "last-pass rows hold one counter per digit");

// Clears the histograms of all three passes and sets up the state.
__global__ void select_init(SelectState* __restrict__ st, uint32_t* __restrict__ hist, int64_t n, int64_t n_prune)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < kSelectHistWords; b += gridDim.x * blockDim.x)
        hist[b] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *st = select_start(n, n_prune);
}

// Locate the bucket holding the target rank in this pass's histogram (the
// sum of its copies) and fold it into the prefix (one block).
__device__ __forceinline__ void select_find_body(SelectState* __restrict__ st,
                                                              const uint32_t* __restrict__ hist, int shift, int bits,
                                                              int last_pass)
{
    constexpr int kPer = kHistBins / kScanThreads;   // 2 bins per thread
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    __shared__ int64_t found_run;
    __shared__ int found_bin;
    const int64_t rank = st->rank;
    const int nb = 1 << bits;
    uint32_t h[kPer];
    uint32_t local = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int b = threadIdx.x * kPer + j;
        uint32_t c = 0;
        if (b < nb)
#pragma unroll
            for (int r = 0; r < kHistCopies; ++r) c += hist[r * kHistBins + b];
        h[j] = c;
        local += h[j];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wave_tot[wave] = incl;
    if (threadIdx.x == 0) found_bin = -1;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wave_tot[w];
    int64_t run = (int64_t)before + incl - local;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int b = threadIdx.x * kPer + j;
        if (rank >= run && rank < run + (int64_t)h[j]) {   // exactly one bin of one thread
            found_bin = b;
            found_run = run;
        }
        run += h[j];
    }
    __syncthreads();
    if (threadIdx.x == 0 && found_bin >= 0) {
        SelectState s = *st;
        s.prefix |= (uint32_t)found_bin << shift;
        s.mask |= ((1u << bits) - 1u) << shift;
        s.rank = rank - found_run;
        if (last_pass) {
            s.threshold = s.prefix;
            s.k_eq = s.rank + 1;
        }
        *st = s;
    }
}

__global__ __launch_bounds__(kScanThreads) void select_find(SelectState* __restrict__ st,
                                                              const uint32_t* __restrict__ hist, int shift, int bits,
                                                              int last_pass)
{
    select_find_body(st, hist, shift, bits, last_pass);
}

// One tile per block: all 16 keys of a thread are loaded before any is
// counted, and the crowded bins (many equal exponents, exact zeros) are
// counted per wave -- the lanes that share the lowest counting lane's bin
// add with one LDS atomic.  rows (last pass only, else null): the tile's
// counts are also stored as its row.
__device__ __forceinline__ void select_hist_body(const float* __restrict__ scores, int n,
                                                        const SelectState* __restrict__ st, int shift, int bits,
                                                        uint32_t* __restrict__ hist, uint32_t* __restrict__ rows,
                                                        int blk)
{
    constexpr uint32_t kNoBin = 0xFFFFFFFFu;
    __shared__ uint32_t h[kHistBins];
    const int nb = 1 << bits;
    for (int b = threadIdx.x; b < nb; b += kBlock) h[b] = 0u;
    const uint32_t prefix = st->prefix, mask = st->mask;
    const uint32_t dmask = (uint32_t)nb - 1u;
    const int base = blk * kTile;
    float v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        v[k] = i < n ? scores[i] : 0.0f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        const uint32_t key = float_key(v[k]);
        const uint32_t bin = (i < n && (key & mask) == prefix) ? (key >> shift) & dmask : kNoBin;
        const uint64_t valid = __ballot(bin != kNoBin);
        if (valid == 0ull) continue;
        const int leader = __builtin_ctzll(valid);
        const uint32_t lead_bin = __builtin_amdgcn_readlane(bin, leader);
        const uint64_t same = __ballot(bin == lead_bin);
        if (bin == lead_bin) {
            if (lane == leader) atomicAdd(&h[lead_bin], (uint32_t)__popcll(same));
        } else if (bin != kNoBin) {
            atomicAdd(&h[bin], 1u);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        const uint32_t c = h[b];
        if (c) atomicAdd(&hist[(blk % kHistCopies) * kHistBins + b], c);
        if (rows) rows[(size_t)blk * kSelectLastBins + b] = c;
    }
}

__global__ __launch_bounds__(kBlock) void select_hist(const float* __restrict__ scores, int n,
                                                        const SelectState* __restrict__ st, int shift, int bits,
                                                        uint32_t* __restrict__ hist, uint32_t* __restrict__ rows)
{
    select_hist_body(scores, n, st, shift, bits, hist, rows, blockIdx.x);
}

__device__ __forceinline__ void select_count_body(const float* __restrict__ scores, int n,
                                                         const SelectState* __restrict__ st,
                                                         uint32_t* __restrict__ tile_cnt, int blk)
{
    const uint32_t T = st->threshold;
    const int base = blk * kTile;
    float v[kItems];   // all keys loaded before any is compared
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = scores[min(base + k * kBlock + (int)threadIdx.x, n - 1)];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        c += (base + k * kBlock + (int)threadIdx.x < n && float_key(v[k]) == T) ? 1u : 0u;
    c = wave_sum_u32(c);
    __shared__ uint32_t red[kWaves];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += red[w];
        tile_cnt[blk] = t;
    }
}

__global__ __launch_bounds__(kBlock) void select_count(const float* __restrict__ scores, int n,
                                                         const SelectState* __restrict__ st,
                                                         uint32_t* __restrict__ tile_cnt)
{
    select_count_body(scores, n, st, tile_cnt, blockIdx.x);
}

__global__ __launch_bounds__(kScanThreads) void select_scan(const uint32_t* __restrict__ tile_cnt,
                                                              uint32_t* __restrict__ tile_off, int ntiles)
{
    block_exclusive_scan(tile_cnt, tile_off, ntiles);
}

// Equal keys before this tile: from the last pass's rows when given, else
// from select_scan (off_from_scan, many tiles) or the preceding tiles'
// select_count totals.  Not needed (and not read) when no key equal to T is
// pruned.
__device__ __forceinline__ void select_mask_body(const float* __restrict__ scores, int n,
                                                        const SelectState* __restrict__ st,
                                                        const uint32_t* __restrict__ rows,
                                                        const uint32_t* __restrict__ tile_cnt,
                                                        const uint32_t* __restrict__ tile_off, int off_from_scan,
                                                        uint8_t* __restrict__ keep, int64_t* __restrict__ d_n_keep,
                                                        uint32_t* __restrict__ d_threshold, int blk,
                                                        uint32_t* __restrict__ kept_cnt = nullptr)
{
    __shared__ uint32_t cnt[kItems][kWaves];
    __shared__ uint32_t kept_red[kWaves];
    const uint32_t T = st->threshold;
    const int64_t k_eq = st->k_eq;
    if (blk == 0 && threadIdx.x == 0) {
        if (d_n_keep) *d_n_keep = st->n_keep;
        if (d_threshold) *d_threshold = T;
    }
    int64_t tile_start = 0;
    if (k_eq > 0) {
        if (rows)
            tile_start = (int64_t)block_sum_prefix(rows + (T & (kSelectLastBins - 1)), blk, kSelectLastBins);
        else
            tile_start = off_from_scan ? (int64_t)tile_off[blk] : (int64_t)block_sum_prefix(tile_cnt, blk);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = blk * kTile;
    uint32_t key[kItems];
    uint64_t eqb[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        key[k] = i < n ? float_key(scores[i]) : 0u;
        eqb[k] = __ballot(i < n && key[k] == T);
        if (lane == 0) cnt[k][wave] = (uint32_t)__popcll(eqb[k]);
    }
    __syncthreads();
    int64_t row = tile_start;
    uint32_t kept = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave) before += cnt[k][w];
            tot += cnt[k][w];
        }
        const int64_t eq_rank = row + before + lanes_below(eqb[k]);
        const bool pruned = key[k] < T || (key[k] == T && eq_rank < k_eq);
        if (i < n) keep[i] = pruned ? 0 : 1;
        kept += (i < n && !pruned) ? 1u : 0u;
        row += tot;
    }
    if (kept_cnt) {   // survivors of the tile, for a compaction that follows in the same launch sequence
        kept = wave_sum_u32(kept);
        if (lane == 0) kept_red[wave] = kept;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < kWaves; ++w) t += kept_red[w];
            kept_cnt[blk] = t;
        }
    }
}

__global__ __launch_bounds__(kBlock) void select_mask(const float* __restrict__ scores, int n,
                                                        const SelectState* __restrict__ st,
                                                        const uint32_t* __restrict__ rows,
                                                        const uint32_t* __restrict__ tile_cnt,
                                                        const uint32_t* __restrict__ tile_off, int off_from_scan,
                                                        uint8_t* __restrict__ keep, int64_t* __restrict__ d_n_keep,
                                                        uint32_t* __restrict__ d_threshold)
{
    select_mask_body(scores, n, st, rows, tile_cnt, tile_off, off_from_scan, keep, d_n_keep, d_threshold,
                     blockIdx.x);
}

__global__ void select_outputs(const SelectState* __restrict__ st, int64_t* __restrict__ d_n_keep,
                               uint32_t* __restrict__ d_threshold)
{
    if (d_n_keep) *d_n_keep = st->n_keep;
    if (d_threshold) *d_threshold = st->threshold;
}

// Grouped launches over the jobs of a batch (jobs that prune nothing skip the
// histogram passes, as the single-job launch sequence does).  Each job's
// state and histograms are set up by the batch's statistics finalisation,
// which runs one block per job earlier in the same launch sequence.

__global__ __launch_bounds__(kBlock) void select_hist_batch(const BatchJob* __restrict__ jobs, int nj, int pass)
{
    const BatchJob& b = jobs[batch_job_of<true>(jobs, nj, blockIdx.x)];
    if (b.n_prune == 0) return;
    select_hist_body(b.scores, b.n, b.sel, kPassShift[pass], kPassBits[pass],
                     b.hist + pass * kHistCopies * kHistBins, pass == 2 ? b.tile_rows : nullptr,
                     (int)blockIdx.x - b.tile0);
}

__global__ __launch_bounds__(kScanThreads) void select_find_batch(const BatchJob* __restrict__ jobs, int pass)
{
    const BatchJob& b = jobs[blockIdx.x];
    if (b.n_prune == 0) return;
    select_find_body(b.sel, b.hist + pass * kHistCopies * kHistBins, kPassShift[pass], kPassBits[pass],
                     pass == 2 ? 1 : 0);
}

__global__ __launch_bounds__(kBlock) void select_mask_batch(const BatchJob* __restrict__ jobs, int nj)
{
    const BatchJob& b = jobs[batch_job_of<true>(jobs, nj, blockIdx.x)];
    // also stores each tile's survivor count, which the batch's compaction uses
    select_mask_body(b.scores, b.n, b.sel, b.tile_rows, nullptr, nullptr, 0, b.keep, b.n_keep_out, nullptr,
                     (int)blockIdx.x - b.tile0, b.tile_cnt);
}

}  // namespace

hipError_t launch_select_batch(const BatchJob* d_jobs, int n_jobs, int total_tiles, hipStream_t stream)
{
    for (int p = 0; p < 3; ++p) {
        hipLaunchKernelGGL(select_hist_batch, dim3(total_tiles), dim3(kBlock), 0, stream, d_jobs, n_jobs, p);
        hipLaunchKernelGGL(select_find_batch, dim3(n_jobs), dim3(kScanThreads), 0, stream, d_jobs, p);
    }
    hipLaunchKernelGGL(select_mask_batch, dim3(total_tiles), dim3(kBlock), 0, stream, d_jobs, n_jobs);
    return hipGetLastError();
}


hipError_t launch_select(const float* d_scores, int64_t n, int64_t n_prune, uint8_t* d_keep, int64_t* d_n_keep,
                         uint32_t* d_threshold, const Workspace& ws, hipStream_t stream)
{
    const int ntiles = (int)num_tiles(n);
    hipLaunchKernelGGL(select_init, dim3(kSelectHistWords / kBlock), dim3(kBlock), 0, stream, ws.sel, ws.hist, n,
                       n_prune);
    if (ntiles == 0) {
        hipLaunchKernelGGL(select_outputs, dim3(1), dim3(1), 0, stream, ws.sel, d_n_keep, d_threshold);
        return hipGetLastError();
    }
    // rows exist for up to kPrefixTilesMax tiles; beyond, count and scan
    const uint32_t* rows = ntiles <= kPrefixTilesMax ? ws.tile_rows : nullptr;
    if (n_prune > 0) {
        for (int p = 0; p < 3; ++p) {
            uint32_t* h = ws.hist + p * kHistCopies * kHistBins;
            hipLaunchKernelGGL(select_hist, dim3(ntiles), dim3(kBlock), 0, stream, d_scores, (int)n, ws.sel,
                               kPassShift[p], kPassBits[p], h, p == 2 ? const_cast<uint32_t*>(rows) : nullptr);
            hipLaunchKernelGGL(select_find, dim3(1), dim3(kScanThreads), 0, stream, ws.sel, h, kPassShift[p],
                               kPassBits[p], p == 2 ? 1 : 0);
        }
    }
    const int from_scan = (n_prune > 0 && !rows) ? 1 : 0;
    if (from_scan) {
        hipLaunchKernelGGL(select_count, dim3(ntiles), dim3(kBlock), 0, stream, d_scores, (int)n, ws.sel,
                           ws.tile_cnt);
        hipLaunchKernelGGL(select_scan, dim3(1), dim3(kScanThreads), 0, stream, ws.tile_cnt, ws.tile_off, ntiles);
    }
    hipLaunchKernelGGL(select_mask, dim3(ntiles), dim3(kBlock), 0, stream, d_scores, (int)n, ws.sel, rows,
                       ws.tile_cnt, ws.tile_off, from_scan, d_keep, d_n_keep, d_threshold);
    return hipGetLastError();
}

}  // namespace refine
