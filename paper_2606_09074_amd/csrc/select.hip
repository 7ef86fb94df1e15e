// Global ranking and ratio selection (paper Sec. 3.3) on gfx950.
//
// Scores become order-preserving 32-bit keys.  The key of the n_prune-th
// smallest primitive (the threshold T) is found by three most-significant-
// digit-first radix passes (11, 11, 10 bits).  Each pass histograms, into
// one LDS histogram per tile, the keys that share the prefix resolved so far,
// and adds them into a global histogram with integer atomics (exact and
// order-independent; 8 copies, one per block residue, so the crowded bins of
// the first pass take 8x fewer atomics per address), together with a coarse
// histogram of 32-bin super-bins.
//
// The bucket of a pass that holds the target rank is resolved at the start of
// the next launch by every block itself: one wave sums the copies of the 64
// super-bins, scans them across its lanes and finds the super-bin, then does
// the same for that super-bin's 32 bins (about 3 KB read, exact integer
// arithmetic, so every block gets the same bucket).  Block 0 records the
// resolved state for the launch after it, in the next of four state slots
// (so no block reads a slot the launch writes).  This replaces a one-block
// find launch per pass: the five launches are init, 3 histogram passes and
// the mask, which resolves the last pass.
//
// Ties at T are broken by index: the pruned primitives are every key < T plus
// the k_eq lowest-index keys == T, located with wave ballots and the exact
// count of equal keys in the tiles before.  The last histogram pass writes
// each tile's row of last-digit counts (4 KB per tile, from the LDS histogram
// it builds anyway): once T is known, the count of keys equal to T in tile t
// is row t at T's last digit, so no separate counting pass is needed.
// (Inputs of more than kPrefixTilesMax tiles resolve T in a one-block launch,
// then count per tile and scan in separate launches.)  Integer arithmetic
// throughout, so the mask equals a stable sort by (score, index).
//
// The batch launches (select_*_batch) run the same bodies for all the jobs of
// a batch, whose selection state and histograms are set up by the batch's
// statistics finalisation.
#include "refine_internal.hpp"

namespace refine {

namespace {

constexpr int kPassShift[3] = {21, 10, 0};
constexpr int kPassBits[3] = {11, 11, 10};
static_assert(1 << kPassBits[2] == kSelectLastBins, "last-pass rows hold one counter per digit");
static_assert(kCoarseBins <= 64 && kSuperWidth <= 64, "a super-bin and the coarse bins each fit in one wave");

// Clears the histograms of all three passes and sets up the first state.
__global__ void select_init(SelectState* __restrict__ st, uint32_t* __restrict__ hist, int64_t n, int64_t n_prune)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < kSelectHistWords; b += gridDim.x * blockDim.x)
        hist[b] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) st[0] = select_start(n, n_prune);
}

// Sum over the wave's lanes up to this one (inclusive).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// The lane whose [excl, incl) range holds r among the first m lanes (0 when
// none does, which consistent counts rule out).
__device__ __forceinline__ int wave_find(uint32_t r, uint32_t excl, uint32_t incl, int m)
{
    const int lane = threadIdx.x & 63;
    const uint64_t hit = __ballot(lane < m && r >= excl && r < incl);
    return hit ? __builtin_ctzll(hit) : 0;
}

// One wave: the digit of the pass whose histogram is `ph` (kPassWords words)
// that holds rank `rank` among the keys that pass counted, and the rank
// within that digit's bucket.  Every lane returns the same values.
__device__ __forceinline__ void resolve_digit(const uint32_t* __restrict__ ph, int bits, int64_t rank,
                                              uint32_t& digit, int64_t& rank_in)
{
    const int lane = threadIdx.x & 63;
    const int nsb = (1 << bits) / kSuperWidth;
    const uint32_t* coarse = ph + kHistCopies * kHistBins;
    uint32_t c = 0;
    if (lane < nsb)
#pragma unroll
        for (int r = 0; r < kHistCopies; ++r) c += coarse[r * kCoarseBins + lane];
    uint32_t incl = wave_incl_scan(c);
    const uint32_t rk = (uint32_t)rank;   // < n <= 2^31 - 1
    const int sb = wave_find(rk, incl - c, incl, nsb);
    const uint32_t rk2 = rk - __shfl(incl - c, sb, 64);
    uint32_t d = 0;
    if (lane < kSuperWidth)
#pragma unroll
        for (int r = 0; r < kHistCopies; ++r) d += ph[r * kHistBins + sb * kSuperWidth + lane];
    incl = wave_incl_scan(d);
    const int b = wave_find(rk2, incl - d, incl, kSuperWidth);
    digit = (uint32_t)(sb * kSuperWidth + b);
    rank_in = (int64_t)(rk2 - __shfl(incl - d, b, 64));
}

// The state after pass `pass` from the state before it and that pass's
// histogram (wave 0 of the block computes it; every thread gets it through
// LDS).  The last pass also fixes the threshold key and k_eq.
__device__ __forceinline__ SelectState resolve_pass(const SelectState* __restrict__ before,
                                                    const uint32_t* __restrict__ ph, int pass)
{
    __shared__ SelectState res;
    if (threadIdx.x < 64) {
        SelectState s = *before;
        uint32_t digit;
        int64_t r;
        resolve_digit(ph, kPassBits[pass], s.rank, digit, r);
        s.prefix |= digit << kPassShift[pass];
        s.mask |= ((1u << kPassBits[pass]) - 1u) << kPassShift[pass];
        s.rank = r;
        if (pass == 2) {
            s.threshold = s.prefix;
            s.k_eq = r + 1;
        }
        if (threadIdx.x == 0) res = s;
    }
    __syncthreads();
    return res;
}

// One tile per block: all 16 keys of a thread are loaded before any is
// counted, and the crowded bins (many equal exponents, exact zeros) are
// counted per wave -- the lanes that share the lowest counting lane's bin
// add with one LDS atomic.  Pass p > 0 first resolves pass p - 1 from
// states[p - 1] (block 0 stores the result in states[p]).  rows (last pass
// only, else null): the tile's counts are also stored as its row.
__device__ __forceinline__ void select_hist_body(const float* __restrict__ scores, int n,
                                                 SelectState* __restrict__ states, int pass,
                                                 uint32_t* __restrict__ hist, uint32_t* __restrict__ rows, int blk)
{
    constexpr uint32_t kNoBin = 0xFFFFFFFFu;
    __shared__ uint32_t h[kHistBins];
    const int shift = kPassShift[pass], bits = kPassBits[pass];
    const int nb = 1 << bits;
    const int base = blk * kTile;
    float v[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        v[k] = i < n ? scores[i] : 0.0f;
    }
    for (int b = threadIdx.x; b < nb; b += kBlock) h[b] = 0u;
    uint32_t prefix = 0u, mask = 0u;
    if (pass > 0) {
        const SelectState s = resolve_pass(states + pass - 1, hist + (pass - 1) * kPassWords, pass - 1);
        prefix = s.prefix;
        mask = s.mask;
        if (blk == 0 && threadIdx.x == 0) states[pass] = s;
    } else {
        __syncthreads();
    }
    uint32_t* const ph = hist + pass * kPassWords;
    const uint32_t dmask = (uint32_t)nb - 1u;
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
    const int copy = blk % kHistCopies;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        const uint32_t c = h[b];
        if (c) atomicAdd(&ph[copy * kHistBins + b], c);
        if (rows) rows[(size_t)blk * kSelectLastBins + b] = c;
    }
    // the tile's super-bin sums into the coarse histogram
    if ((int)threadIdx.x < nb / kSuperWidth) {
        uint32_t c = 0;
        for (int j = 0; j < kSuperWidth; ++j) c += h[threadIdx.x * kSuperWidth + j];
        if (c) atomicAdd(&ph[kHistCopies * kHistBins + copy * kCoarseBins + threadIdx.x], c);
    }
}

__global__ __launch_bounds__(kBlock) void select_hist(const float* __restrict__ scores, int n,
                                                        SelectState* __restrict__ states, int pass,
                                                        uint32_t* __restrict__ hist, uint32_t* __restrict__ rows)
{
    select_hist_body(scores, n, states, pass, hist, rows, blockIdx.x);
}

// Resolves the last pass into states[3] (one block; the many-tiles path,
// whose counting launch needs the threshold).
__global__ void select_final(SelectState* __restrict__ states, const uint32_t* __restrict__ hist)
{
    const SelectState s = resolve_pass(states + 2, hist + 2 * kPassWords, 2);
    if (threadIdx.x == 0) states[3] = s;
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

// The final state comes from states[3] (resolve = 0: no key pruned, whose
// states[0] serves as final, or the many-tiles path) or from resolving the
// last pass from states[2] here (resolve = 1; block 0 stores it in
// states[3]).  Equal keys before this tile: from the last pass's rows when
// given, else from select_scan (off_from_scan, many tiles) or the preceding
// tiles' select_count totals.  Not needed (and not read) when no key equal
// to T is pruned.
__device__ __forceinline__ void select_mask_body(const float* __restrict__ scores, int n,
                                                 SelectState* __restrict__ states, int final_slot, int resolve,
                                                 const uint32_t* __restrict__ hist,
                                                 const uint32_t* __restrict__ rows,
                                                 const uint32_t* __restrict__ tile_cnt,
                                                 const uint32_t* __restrict__ tile_off, int off_from_scan,
                                                 uint8_t* __restrict__ keep, int64_t* __restrict__ d_n_keep,
                                                 uint32_t* __restrict__ d_threshold, int blk,
                                                 uint32_t* __restrict__ kept_cnt = nullptr)
{
    __shared__ uint32_t cnt[kItems][kWaves];
    __shared__ uint32_t kept_red[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = blk * kTile;
    uint32_t key[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        key[k] = i < n ? float_key(scores[i]) : 0u;
    }
    SelectState fin;
    if (resolve) {
        fin = resolve_pass(states + 2, hist + 2 * kPassWords, 2);
        if (blk == 0 && threadIdx.x == 0) states[3] = fin;
    } else {
        fin = states[final_slot];
    }
    const uint32_t T = fin.threshold;
    const int64_t k_eq = fin.k_eq;
    if (blk == 0 && threadIdx.x == 0) {
        if (d_n_keep) *d_n_keep = fin.n_keep;
        if (d_threshold) *d_threshold = T;
    }
    int64_t tile_start = 0;
    if (k_eq > 0) {
        if (rows)
            tile_start = (int64_t)block_sum_prefix(rows + (T & (kSelectLastBins - 1)), blk, kSelectLastBins);
        else
            tile_start = off_from_scan ? (int64_t)tile_off[blk] : (int64_t)block_sum_prefix(tile_cnt, blk);
    }
    uint64_t eqb[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
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
                                                        SelectState* __restrict__ states, int final_slot, int resolve,
                                                        const uint32_t* __restrict__ hist,
                                                        const uint32_t* __restrict__ rows,
                                                        const uint32_t* __restrict__ tile_cnt,
                                                        const uint32_t* __restrict__ tile_off, int off_from_scan,
                                                        uint8_t* __restrict__ keep, int64_t* __restrict__ d_n_keep,
                                                        uint32_t* __restrict__ d_threshold)
{
    select_mask_body(scores, n, states, final_slot, resolve, hist, rows, tile_cnt, tile_off, off_from_scan, keep,
                     d_n_keep, d_threshold, blockIdx.x);
}

__global__ void select_outputs(const SelectState* __restrict__ st, int64_t* __restrict__ d_n_keep,
                               uint32_t* __restrict__ d_threshold)
{
    if (d_n_keep) *d_n_keep = st->n_keep;
    if (d_threshold) *d_threshold = st->threshold;
}

// Grouped launches over the jobs of a batch (jobs that prune nothing skip the
// histogram passes, as the single-job launch sequence does).  Each job's
// states and histograms are set up by the batch's statistics finalisation,
// which runs one block per job earlier in the same launch sequence.

__global__ __launch_bounds__(kBlock) void select_hist_batch(const BatchJob* __restrict__ jobs, int nj, int pass)
{
    const BatchJob& b = jobs[batch_job_of<true>(jobs, nj, blockIdx.x)];
    if (b.n_prune == 0) return;
    select_hist_body(b.scores, b.n, b.sel, pass, b.hist, pass == 2 ? b.tile_rows : nullptr,
                     (int)blockIdx.x - b.tile0);
}

__global__ __launch_bounds__(kBlock) void select_mask_batch(const BatchJob* __restrict__ jobs, int nj)
{
    const BatchJob& b = jobs[batch_job_of<true>(jobs, nj, blockIdx.x)];
    // also stores each tile's survivor count, which the batch's compaction uses
    const int resolve = b.n_prune > 0 ? 1 : 0;
    select_mask_body(b.scores, b.n, b.sel, 0, resolve, b.hist, b.tile_rows, nullptr, nullptr, 0, b.keep,
                     b.n_keep_out, nullptr, (int)blockIdx.x - b.tile0, b.tile_cnt);
}

}  // namespace

hipError_t launch_select_batch(const BatchJob* d_jobs, int n_jobs, int total_tiles, hipStream_t stream)
{
    for (int p = 0; p < 3; ++p)
        hipLaunchKernelGGL(select_hist_batch, dim3(total_tiles), dim3(kBlock), 0, stream, d_jobs, n_jobs, p);
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
    if (n_prune > 0)
        for (int p = 0; p < 3; ++p)
            hipLaunchKernelGGL(select_hist, dim3(ntiles), dim3(kBlock), 0, stream, d_scores, (int)n, ws.sel, p,
                               ws.hist, p == 2 ? const_cast<uint32_t*>(rows) : nullptr);
    const int from_scan = (n_prune > 0 && !rows) ? 1 : 0;
    if (from_scan) {
        hipLaunchKernelGGL(select_final, dim3(1), dim3(64), 0, stream, ws.sel, ws.hist);
        hipLaunchKernelGGL(select_count, dim3(ntiles), dim3(kBlock), 0, stream, d_scores, (int)n, ws.sel + 3,
                           ws.tile_cnt);
        hipLaunchKernelGGL(select_scan, dim3(1), dim3(kScanThreads), 0, stream, ws.tile_cnt, ws.tile_off, ntiles);
    }
    // the final state: resolved in the mask launch (rows path), already in
    // states[3] (many tiles), or the start state when nothing is pruned
    const int resolve = (n_prune > 0 && rows) ? 1 : 0;
    const int final_slot = n_prune > 0 ? 3 : 0;
    hipLaunchKernelGGL(select_mask, dim3(ntiles), dim3(kBlock), 0, stream, d_scores, (int)n, ws.sel, final_slot,
                       resolve, ws.hist, rows, ws.tile_cnt, ws.tile_off, from_scan, d_keep, d_n_keep, d_threshold);
    return hipGetLastError();
}

}  // namespace refine
