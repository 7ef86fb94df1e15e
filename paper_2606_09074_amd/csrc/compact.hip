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
// contiguous output range.  Bit copies, no arithmetic on the values.
#include "refine_internal.hpp"

namespace refine {

namespace {

__global__ __launch_bounds__(kBlock) void compact_count(const uint8_t* __restrict__ keep, int n,
                                                          uint32_t* __restrict__ tile_cnt)
{
    const int base = blockIdx.x * kTile;
    uint32_t c = 0;
#pragma unroll 4
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        if (i < n && keep[i]) ++c;
    }
    c = wave_sum_u32(c);
    __shared__ uint32_t red[kWaves];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += red[w];
        tile_cnt[blockIdx.x] = t;
    }
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
                                     int ntiles, int off_from_scan, int64_t* __restrict__ d_n_out)
{
    if (blockIdx.x == 0 && d_n_out) {
        const uint64_t total = block_sum_prefix(tile_cnt, ntiles);
        if (threadIdx.x == 0) *d_n_out = (int64_t)total;
    }
    return off_from_scan ? (int64_t)tile_off[blockIdx.x] : (int64_t)block_sum_prefix(tile_cnt, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void compact_scatter(const float* __restrict__ in, int64_t in_stride, int n,
                                                            const uint8_t* __restrict__ keep,
                                                            const uint32_t* __restrict__ tile_cnt,
                                                            const uint32_t* __restrict__ tile_off, int ntiles,
                                                            int off_from_scan, int64_t* __restrict__ d_n_out,
                                                            float* __restrict__ out, int64_t out_stride,
                                                            int64_t capacity, int32_t* __restrict__ index_map)
{
    const int64_t tstart = tile_start(tile_cnt, tile_off, ntiles, off_from_scan, d_n_out);
    __shared__ uint32_t cnt[kItems][kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = blockIdx.x * kTile;
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
            if ((kept_bits >> k) & 1u) index_map[pos[k]] = base + k * kBlock + (int)threadIdx.x;
    }
    if (kept_bits == 0u && __ballot(kept_bits != 0u) == 0ull) return;
    for (int p = 0; p < kPlanes; ++p) {
        const float* src = in + (int64_t)p * in_stride + base + (int)threadIdx.x;
        float* dst = out + (int64_t)p * out_stride;
        float v[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if ((kept_bits >> k) & 1u) v[k] = src[k * kBlock];
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if ((kept_bits >> k) & 1u) dst[pos[k]] = v[k];
    }
}

// compact_scatter for 16-byte aligned planes (stride a multiple of 4) and a
// 4-byte aligned mask.  A tile is 4 rows of 1024 primitives; each lane loads
// 4 consecutive primitives of a row with one 16-byte load per plane.  The
// survivors of two planes are packed in LDS at their tile-local positions
// (per-row exclusive scans in index order: the copy stays stable), then
// written out with contiguous, fully active 4-byte stores.
constexpr int kVecRows = kTile / (4 * kBlock);   // 4
constexpr int kStagePlanes = 2;

__global__ __launch_bounds__(kBlock) void compact_scatter_lds(const float* __restrict__ in, int64_t in_stride, int n,
                                                                const uint8_t* __restrict__ keep,
                                                                const uint32_t* __restrict__ tile_cnt,
                                                                const uint32_t* __restrict__ tile_off, int ntiles,
                                                                int off_from_scan, int64_t* __restrict__ d_n_out,
                                                                float* __restrict__ out, int64_t out_stride,
                                                                int64_t capacity, int32_t* __restrict__ index_map)
{
    const int64_t out0 = tile_start(tile_cnt, tile_off, ntiles, off_from_scan, d_n_out);
    __shared__ uint32_t wtot[kVecRows][kWaves];
    __shared__ float stage[kStagePlanes][kTile];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int base = blockIdx.x * kTile;
    uint32_t flags[kVecRows], incl[kVecRows];
#pragma unroll
    for (int r = 0; r < kVecRows; ++r) {
        const int i0 = base + r * 4 * kBlock + 4 * (int)threadIdx.x;
        uint32_t f = 0u;
        if (i0 + 3 < n) {
            const uint32_t w = *reinterpret_cast<const uint32_t*>(keep + i0);
#pragma unroll
            for (int j = 0; j < 4; ++j) f |= ((w >> (8 * j)) & 0xFFu) ? (1u << j) : 0u;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) f |= (i0 + j < n && keep[i0 + j]) ? (1u << j) : 0u;
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
    uint32_t lstart[kVecRows];
    uint32_t row = 0;
#pragma unroll
    for (int r = 0; r < kVecRows; ++r) {
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
    const int kept = (int)min((int64_t)tile_cnt[blockIdx.x], room > 0 ? room : (int64_t)0);
    if (index_map) {
#pragma unroll
        for (int r = 0; r < kVecRows; ++r) {
            const int i0 = base + r * 4 * kBlock + 4 * (int)threadIdx.x;
            uint32_t k = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((flags[r] >> j) & 1u) {
                    if ((int)(lstart[r] + k) < kept) index_map[out0 + lstart[r] + k] = i0 + j;
                    ++k;
                }
        }
    }
    if (kept == 0) return;   // uniform across the block
    for (int p0 = 0; p0 < kPlanes; p0 += kStagePlanes) {
#pragma unroll
        for (int q = 0; q < kStagePlanes; ++q) {
            if (p0 + q >= kPlanes) break;
            const float* src = in + (int64_t)(p0 + q) * in_stride;
#pragma unroll
            for (int r = 0; r < kVecRows; ++r) {
                if (!flags[r]) continue;
                const int i0 = base + r * 4 * kBlock + 4 * (int)threadIdx.x;
                float v[4];
                if (i0 + 3 < n) {
                    const float4 x = *reinterpret_cast<const float4*>(src + i0);
                    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) v[j] = (i0 + j < n) ? src[i0 + j] : 0.0f;
                }
                uint32_t k = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((flags[r] >> j) & 1u) stage[q][lstart[r] + k++] = v[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kStagePlanes; ++q) {
            if (p0 + q >= kPlanes) break;
            float* dst = out + (int64_t)(p0 + q) * out_stride + out0;
            for (int j = threadIdx.x; j < kept; j += kBlock) dst[j] = stage[q][j];
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_compact(const float* in, int64_t in_stride, int64_t n, const uint8_t* d_keep, float* out,
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
    const bool vec = (reinterpret_cast<uintptr_t>(in) % 16 == 0) && (in_stride % 4 == 0) &&
                     (reinterpret_cast<uintptr_t>(d_keep) % 4 == 0);
    if (vec)
        hipLaunchKernelGGL(compact_scatter_lds, dim3(ntiles), dim3(kBlock), 0, stream, in, in_stride, (int)n, d_keep,
                           ws.tile_cnt, ws.tile_off, ntiles, from_scan, d_n_out, out, out_stride, capacity,
                           d_index_map);
    else
        hipLaunchKernelGGL(compact_scatter, dim3(ntiles), dim3(kBlock), 0, stream, in, in_stride, (int)n, d_keep,
                           ws.tile_cnt, ws.tile_off, ntiles, from_scan, d_n_out, out, out_stride, capacity,
                           d_index_map);
    return hipGetLastError();
}

}  // namespace refine
