// Survivor compaction (paper Sec. 3.3: the pruned primitives are removed
// and the rest written out) on gfx950.
//
// compact_count: kept primitives per 4096-primitive tile.  compact_scatter:
// one block per tile takes its output offset from the preceding tiles'
// counts (compact_scan turns them into offsets first when there are very
// many tiles), finds each survivor's output position from wave ballots (the
// order inside the tile is the index order, so the copy is stable) and then
// streams all 59 planes: each row of 256 consecutive primitives is one
// coalesced load per plane, and the survivors of a row land in one
// contiguous output range.  Bit copies of 4-byte (FP32) or 2-byte (BF16 /
// FP16) elements, no arithmetic on the values.  FP32 survivors are written
// with non-temporal stores: left as dirty lines in the last-level cache,
// their write-back would compete with whatever reads HBM next (measured on
// back-to-back prunes: the next statistics pass 45 -> 32 us, the compaction
// itself +2 us).  For 2-byte elements the same stores made the compaction
// 25 us slower than they saved, so those use ordinary stores.  The aligned
// scatter reads the scene with non-temporal loads (both storages: the
// compaction 14 us faster for FP32, 6 us for 2-byte, at ~4 us to the next
// statistics and binning passes).  The kernel bodies take the
// tile index, so the grouped launches of a batch (compact_*_batch) run the
// same code per job.
#include "refine_internal.hpp"

namespace refine {

namespace {

// Output stores: non-temporal for 4-byte elements (and then for the index
// map too), ordinary for 2-byte ones.
template <class E>
__device__ __forceinline__ void store_out(E v, E* p)
{
    if constexpr (sizeof(E) == 4) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <class E>
__device__ __forceinline__ void store_index(int32_t v, int32_t* p)
{
    if constexpr (sizeof(E) == 4) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// The aligned scatter splits the 59 planes over this many blocks per tile
// (grid.y): each recomputes the tile's positions from the mask (4 KB) and
// copies its planes, so a launch has several blocks per CU to balance.
constexpr int kCompactPlaneGroups = 4;

__device__ __forceinline__ void compact_count_body(const uint8_t* __restrict__ keep, int n,
                                                          uint32_t* __restrict__ tile_cnt, int blk)
{
    const int base = blk * kTile;
    uint8_t f[kItems];   // all flags loaded before any is counted
#pragma unroll
    for (int k = 0; k < kItems; ++k) f[k] = keep[min(base + k * kBlock + (int)threadIdx.x, n - 1)];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) c += (base + k * kBlock + (int)threadIdx.x < n && f[k]) ? 1u : 0u;
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

__global__ __launch_bounds__(kBlock) void compact_count(const uint8_t* __restrict__ keep, int n,
                                                          uint32_t* __restrict__ tile_cnt)
{
    compact_count_body(keep, n, tile_cnt, blockIdx.x);
}

__global__ __launch_bounds__(kScanThreads) void compact_scan(const uint32_t* __restrict__ tile_cnt,
                                                               uint32_t* __restrict__ tile_off, int ntiles)
{
    block_exclusive_scan(tile_cnt, tile_off, ntiles);
}

__global__ void compact_empty(int64_t* __restrict__ d_n_out)
{
    if (d_n_out) *d_n_out = 0;
}

// Offset of this block's tile in the output: from compact_scan when there are
// many tiles, else the sum of the preceding tiles' counts; block 0 also
// reports the total number of survivors.
__device__ inline int64_t tile_start(const uint32_t* __restrict__ tile_cnt, const uint32_t* __restrict__ tile_off,
                                     int ntiles, int off_from_scan, int64_t* __restrict__ d_n_out, int tile)
{
    if (tile == 0 && d_n_out) {
        const uint64_t total = block_sum_prefix(tile_cnt, ntiles);
        if (threadIdx.x == 0) *d_n_out = (int64_t)total;
    }
    return off_from_scan ? (int64_t)tile_off[tile] : (int64_t)block_sum_prefix(tile_cnt, tile);
}

template <class E>
__device__ __forceinline__ void compact_scatter_body(const E* __restrict__ in, int64_t in_stride, int n,
                                                            const uint8_t* __restrict__ keep,
                                                            const uint32_t* __restrict__ tile_cnt,
                                                            const uint32_t* __restrict__ tile_off, int ntiles,
                                                            int off_from_scan, int64_t* __restrict__ d_n_out,
                                                            E* __restrict__ out, int64_t out_stride,
                                                            int64_t capacity, int32_t* __restrict__ index_map, int blk)
{
    const int64_t tstart = tile_start(tile_cnt, tile_off, ntiles, off_from_scan, d_n_out, blk);
    __shared__ uint32_t cnt[kItems][kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = blk * kTile;
    uint64_t kb[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        kb[k] = __ballot(i < n && keep[i] != 0);
        if (lane == 0) cnt[k][wave] = (uint32_t)__popcll(kb[k]);
    }
    __syncthreads();
    // output position of this lane's element in each row (or -1 when not written)
    int64_t pos[kItems];
    uint32_t kept_bits = 0;
    int64_t row = tstart;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave) before += cnt[k][w];
            tot += cnt[k][w];
        }
        pos[k] = row + before + lanes_below(kb[k]);
        if (((kb[k] >> lane) & 1ull) && pos[k] < capacity) kept_bits |= 1u << k;
        row += tot;
    }
    if (index_map) {
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if ((kept_bits >> k) & 1u) store_index<E>(base + k * kBlock + (int)threadIdx.x, index_map + pos[k]);
    }
    if (kept_bits == 0u && __ballot(kept_bits != 0u) == 0ull) return;
    for (int p = 0; p < kPlanes; ++p) {
        const E* src = in + (int64_t)p * in_stride + base + (int)threadIdx.x;
        E* dst = out + (int64_t)p * out_stride;
        E v[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if ((kept_bits >> k) & 1u) v[k] = src[k * kBlock];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if ((kept_bits >> k) & 1u) store_out(v[k], dst + pos[k]);
    }
}

template <class E>
__global__ __launch_bounds__(kBlock) void compact_scatter(const E* __restrict__ in, int64_t in_stride, int n,
                                                            const uint8_t* __restrict__ keep,
                                                            const uint32_t* __restrict__ tile_cnt,
                                                            const uint32_t* __restrict__ tile_off, int ntiles,
                                                            int off_from_scan, int64_t* __restrict__ d_n_out,
                                                            E* __restrict__ out, int64_t out_stride,
                                                            int64_t capacity, int32_t* __restrict__ index_map)
{
    compact_scatter_body<E>(in, in_stride, n, keep, tile_cnt, tile_off, ntiles, off_from_scan, d_n_out, out,
                            out_stride, capacity, index_map, blockIdx.x);
}

// compact_scatter for 16-byte aligned planes (stride a multiple of 16 bytes)
// and a 4-byte aligned mask.  A tile is rows of 16 bytes per lane: 4 rows of
// 1024 FP32 primitives, or 2 rows of 2048 2-byte primitives; each lane loads
// its PER consecutive primitives of a row with one 16-byte load per plane.
// The survivors of 16 KB of planes at a time (one FP32 plane or two 2-byte
// planes of the tile) are packed in LDS at their tile-local positions (per-row exclusive scans in index order: the copy
// stays stable), then written out with contiguous, fully active stores of 4
// bytes (two 2-byte elements when `pair_store`: output 4-byte aligned with an
// even stride).
template <class E, int PER>
__device__ inline void unpack16(const uint4& x, E (&v)[PER])
{
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
    if constexpr (PER == 4) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = w[j];
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[2 * j] = (E)(w[j] & 0xFFFFu);
            v[2 * j + 1] = (E)(w[j] >> 16);
        }
    }
}

template <class E>
__device__ __forceinline__ void compact_scatter_lds_body(const E* __restrict__ in, int64_t in_stride, int n,
                                                                const uint8_t* __restrict__ keep,
                                                                const uint32_t* __restrict__ tile_cnt,
                                                                const uint32_t* __restrict__ tile_off, int ntiles,
                                                                int off_from_scan, int64_t* __restrict__ d_n_out,
                                                                E* __restrict__ out, int64_t out_stride,
                                                                int64_t capacity, int32_t* __restrict__ index_map,
                                                                int pair_store, int blk, int p_begin, int p_end)
{
    constexpr int PER = 16 / sizeof(E);               // primitives per lane per row
    constexpr int ROWS = kTile / (PER * kBlock);      // 4 or 2
    constexpr int kStagePlanes = 4 / sizeof(E);       // 16 KB of LDS: many blocks per CU
    const int64_t out0 = tile_start(tile_cnt, tile_off, ntiles, off_from_scan, p_begin == 0 ? d_n_out : nullptr, blk);
    __shared__ uint32_t wtot[ROWS][kWaves];
    __shared__ E stage[kStagePlanes][kTile];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = blk * kTile;
    uint32_t flags[ROWS], incl[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int i0 = base + r * PER * kBlock + PER * (int)threadIdx.x;
        uint32_t f = 0u;
        if (i0 + PER - 1 < n) {
#pragma unroll
            for (int h = 0; h < PER / 4; ++h) {
                const uint32_t w = *reinterpret_cast<const uint32_t*>(keep + i0 + 4 * h);
#pragma unroll
                for (int j = 0; j < 4; ++j) f |= ((w >> (8 * j)) & 0xFFu) ? (1u << (4 * h + j)) : 0u;
            }
        } else {
#pragma unroll
            for (int j = 0; j < PER; ++j) f |= (i0 + j < n && keep[i0 + j]) ? (1u << j) : 0u;
        }
        flags[r] = f;
        uint32_t c = (uint32_t)__popc(f);
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(c, o, 64);
            if (lane >= o) c += y;
        }
        incl[r] = c;
        if (lane == 63) wtot[r][wave] = c;
    }
    __syncthreads();
    // tile-local position of this lane's first survivor in each row
    uint32_t lstart[ROWS];
    uint32_t row = 0;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        uint32_t before = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave) before += wtot[r][w];
            tot += wtot[r][w];
        }
        lstart[r] = row + before + incl[r] - (uint32_t)__popc(flags[r]);
        row += tot;
    }
    const int64_t room = capacity - out0;
    const int kept = (int)min((int64_t)tile_cnt[blk], room > 0 ? room : (int64_t)0);
    if (index_map && p_begin == 0) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int i0 = base + r * PER * kBlock + PER * (int)threadIdx.x;
            uint32_t k = 0;
#pragma unroll
            for (int j = 0; j < PER; ++j)
                if ((flags[r] >> j) & 1u) {
                    if ((int)(lstart[r] + k) < kept) store_index<E>(i0 + j, index_map + out0 + lstart[r] + k);
                    ++k;
                }
        }
    }
    if (kept == 0) return;   // uniform across the block
    // elements before the first 4-byte boundary of the output range (pair stores)
    const int lead = (sizeof(E) == 2 && pair_store) ? (int)(out0 & 1) : 0;
    for (int p0 = p_begin; p0 < p_end; p0 += kStagePlanes) {
#pragma unroll
        for (int q = 0; q < kStagePlanes; ++q) {
            if (p0 + q >= p_end) break;
            const E* src = in + (int64_t)(p0 + q) * in_stride;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                if (!flags[r]) continue;
                const int i0 = base + r * PER * kBlock + PER * (int)threadIdx.x;
                E v[PER];
                if (i0 + PER - 1 < n) {
                    // non-temporal: the scene is streamed once, so its lines
                    // should not displace (and force the write-back of)
                    // what the cache holds
                    typedef unsigned v4u __attribute__((ext_vector_type(4)));
                    const v4u t = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(src + i0));
                    unpack16<E, PER>(make_uint4(t.x, t.y, t.z, t.w), v);
                } else {
#pragma unroll
                    for (int j = 0; j < PER; ++j) v[j] = (i0 + j < n) ? src[i0 + j] : E(0);
                }
                uint32_t k = 0;
#pragma unroll
                for (int j = 0; j < PER; ++j)
                    if ((flags[r] >> j) & 1u) stage[q][lstart[r] + k++] = v[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kStagePlanes; ++q) {
            if (p0 + q >= p_end) break;
            E* dst = out + (int64_t)(p0 + q) * out_stride + out0;
            if (sizeof(E) == 2 && pair_store) {
                if (lead && threadIdx.x == 0) dst[0] = stage[q][0];
                const int npairs = (kept - lead) >> 1;
                uint32_t* dst2 = reinterpret_cast<uint32_t*>(dst + lead);
                for (int j = threadIdx.x; j < npairs; j += kBlock)
                    dst2[j] = (uint32_t)stage[q][lead + 2 * j] | ((uint32_t)stage[q][lead + 2 * j + 1] << 16);
                if (((kept - lead) & 1) && threadIdx.x == 0) dst[kept - 1] = stage[q][kept - 1];
            } else {
                for (int j = threadIdx.x; j < kept; j += kBlock) store_out(stage[q][j], dst + j);
            }
        }
        __syncthreads();
    }
}

template <class E>
__global__ __launch_bounds__(kBlock) void compact_scatter_lds(const E* __restrict__ in, int64_t in_stride, int n,
                                                                const uint8_t* __restrict__ keep,
                                                                const uint32_t* __restrict__ tile_cnt,
                                                                const uint32_t* __restrict__ tile_off, int ntiles,
                                                                int off_from_scan, int64_t* __restrict__ d_n_out,
                                                                E* __restrict__ out, int64_t out_stride,
                                                                int64_t capacity, int32_t* __restrict__ index_map,
                                                                int pair_store, int planes_per_group)
{
    const int p_begin = (int)blockIdx.y * planes_per_group;
    compact_scatter_lds_body<E>(in, in_stride, n, keep, tile_cnt, tile_off, ntiles, off_from_scan, d_n_out, out,
                                out_stride, capacity, index_map, pair_store, blockIdx.x, p_begin,
                                min(p_begin + planes_per_group, kPlanes));
}

template <class E>
void launch_compact_t(const E* in, int64_t in_stride, int n, const uint8_t* d_keep, E* out, int64_t out_stride,
                      int64_t capacity, int32_t* d_index_map, int64_t* d_n_out, const Workspace& ws, int ntiles,
                      int from_scan, hipStream_t stream)
{
    const bool vec = (reinterpret_cast<uintptr_t>(in) % 16 == 0) && ((in_stride * sizeof(E)) % 16 == 0) &&
                     (reinterpret_cast<uintptr_t>(d_keep) % 4 == 0);
    const int pair_store = (reinterpret_cast<uintptr_t>(out) % 4 == 0) && (out_stride % 2 == 0) ? 1 : 0;
    if (vec) {
        constexpr int stage = 4 / sizeof(E);   // kStagePlanes of the kernel
        const int per_group = (kPlanes + kCompactPlaneGroups - 1) / kCompactPlaneGroups;
        const int planes_per_group = (per_group + stage - 1) / stage * stage;
        const int groups = (kPlanes + planes_per_group - 1) / planes_per_group;
        hipLaunchKernelGGL(compact_scatter_lds<E>, dim3(ntiles, groups), dim3(kBlock), 0, stream, in, in_stride, n,
                           d_keep, ws.tile_cnt, ws.tile_off, ntiles, from_scan, d_n_out, out, out_stride, capacity,
                           d_index_map, pair_store, planes_per_group);
    } else
        hipLaunchKernelGGL(compact_scatter<E>, dim3(ntiles), dim3(kBlock), 0, stream, in, in_stride, n, d_keep,
                           ws.tile_cnt, ws.tile_off, ntiles, from_scan, d_n_out, out, out_stride, capacity,
                           d_index_map);
}

// Grouped launches over the jobs of a batch.  The tile offsets come from the
// per-block sums of the job's preceding tiles (jobs of a batch have at most
// kPrefixTilesMax tiles).
template <class E>
__device__ __forceinline__ void compact_job_tile(const BatchJob& b, int tile)
{
    const int ntiles = (int)num_tiles(b.n);
    if (b.vec_compact)
        compact_scatter_lds_body<E>(static_cast<const E*>(b.planes), b.stride, b.n, b.keep, b.tile_cnt, nullptr,
                                    ntiles, 0, b.n_out, static_cast<E*>(b.out), b.out_stride, b.capacity,
                                    b.index_map, b.pair_store, tile, 0, kPlanes);
    else
        compact_scatter_body<E>(static_cast<const E*>(b.planes), b.stride, b.n, b.keep, b.tile_cnt, nullptr,
                                ntiles, 0, b.n_out, static_cast<E*>(b.out), b.out_stride, b.capacity, b.index_map,
                                tile);
}

__global__ __launch_bounds__(kBlock) void compact_scatter_batch(const BatchJob* __restrict__ jobs, int nj)
{
    const BatchJob& b = jobs[batch_job_of<true>(jobs, nj, blockIdx.x)];
    const int tile = (int)blockIdx.x - b.tile0;
    if (storage_bytes(b.st) == 4)
        compact_job_tile<uint32_t>(b, tile);
    else
        compact_job_tile<uint16_t>(b, tile);
}

}  // namespace

// The batch's selection has stored every tile's survivor count (the mask
// pass counts them), so no counting pass is needed here.
hipError_t launch_compact_batch(const BatchJob* d_jobs, int n_jobs, int total_tiles, hipStream_t stream)
{
    hipLaunchKernelGGL(compact_scatter_batch, dim3(total_tiles), dim3(kBlock), 0, stream, d_jobs, n_jobs);
    return hipGetLastError();
}


hipError_t launch_compact(const void* in, int st, int64_t in_stride, int64_t n, const uint8_t* d_keep, void* out,
                          int64_t out_stride, int64_t capacity, int32_t* d_index_map, int64_t* d_n_out,
                          const Workspace& ws, hipStream_t stream)
{
    const int ntiles = (int)num_tiles(n);
    if (ntiles == 0) {
        hipLaunchKernelGGL(compact_empty, dim3(1), dim3(1), 0, stream, d_n_out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(compact_count, dim3(ntiles), dim3(kBlock), 0, stream, d_keep, (int)n, ws.tile_cnt);
    const int from_scan = ntiles > kPrefixTilesMax ? 1 : 0;
    if (from_scan)
        hipLaunchKernelGGL(compact_scan, dim3(1), dim3(kScanThreads), 0, stream, ws.tile_cnt, ws.tile_off, ntiles);
    if (storage_bytes(st) == 4)
        launch_compact_t(static_cast<const uint32_t*>(in), in_stride, (int)n, d_keep, static_cast<uint32_t*>(out),
                         out_stride, capacity, d_index_map, d_n_out, ws, ntiles, from_scan, stream);
    else
        launch_compact_t(static_cast<const uint16_t*>(in), in_stride, (int)n, d_keep, static_cast<uint16_t*>(out),
                         out_stride, capacity, d_index_map, d_n_out, ws, ntiles, from_scan, stream);
    return hipGetLastError();
}

}  // namespace refine
