// Survivor compaction (paper Sec. 3.3: the pruned primitives are removed
// and the rest written out) on gfx950.
//
// compact_count: kept primitives per 4096-primitive tile.  compact_scan: one
// block turns the counts into exact tile offsets.  compact_scatter: one block
// per tile finds each survivor's output position from wave ballots (the
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
                                                               uint32_t* __restrict__ tile_off, int ntiles,
                                                               int64_t* __restrict__ d_n_out)
{
    const uint32_t total = block_exclusive_scan(tile_cnt, tile_off, ntiles);
    if (threadIdx.x == 0 && d_n_out) *d_n_out = (int64_t)total;
}

__global__ __launch_bounds__(kBlock) void compact_scatter(const float* __restrict__ in, int64_t in_stride, int n,
                                                            const uint8_t* __restrict__ keep,
                                                            const uint32_t* __restrict__ tile_off,
                                                            float* __restrict__ out, int64_t out_stride,
                                                            int64_t capacity, int32_t* __restrict__ index_map)
{
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
    int64_t row = (int64_t)tile_off[blockIdx.x];
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

}  // namespace

hipError_t launch_compact(const float* in, int64_t in_stride, int64_t n, const uint8_t* d_keep, float* out,
                          int64_t out_stride, int64_t capacity, int32_t* d_index_map, int64_t* d_n_out,
                          const Workspace& ws, hipStream_t stream)
{
    const int ntiles = (int)num_tiles(n);
    if (ntiles > 0)
        hipLaunchKernelGGL(compact_count, dim3(ntiles), dim3(kBlock), 0, stream, d_keep, (int)n, ws.tile_cnt);
    hipLaunchKernelGGL(compact_scan, dim3(1), dim3(kScanThreads), 0, stream, ws.tile_cnt, ws.tile_off, ntiles,
                       d_n_out);
    if (ntiles > 0)
        hipLaunchKernelGGL(compact_scatter, dim3(ntiles), dim3(kBlock), 0, stream, in, in_stride, (int)n, d_keep,
                           ws.tile_off, out, out_stride, capacity, d_index_map);
    return hipGetLastError();
}

}  // namespace refine
