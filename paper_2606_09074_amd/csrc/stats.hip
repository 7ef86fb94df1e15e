// Scene features and content-adaptive weights (paper Eq. features, Eq. 18,
// Eq. 19) on gfx950.
//
// stats_partial: one block per 4096-primitive tile.  Per primitive, in FP32:
//   luma Y of the DC colour, alpha (1 - alpha), max(s) / (min(s) + eta), and
//   a non-finite check of the 14 planes the scoring reads.
// Each thread accumulates its 16 primitives in FP64; the block reduces by
// wave butterflies, then across its 4 waves in a fixed order, and writes one
// partial per tile.  stats_finalize (one block) sums the partials in a fixed
// order and derives the features and lambda in FP64.  No floating-point
// atomics: the result is bit-identical run to run.
//
// The same pass records the axis-aligned box of the finite centres (min/max
// are order independent, so this is deterministic too); refine_score's
// spatial binning quantises centres inside it.
//
// HBM traffic: 14 planes x 4 B = 56 B per primitive read (the 28 B of the
// feature planes plus the non-finite check of the rest; half of that for
// BF16/FP16 storage), 64 B per tile written.
#include <mutex>

#include "refine_internal.hpp"

namespace refine {

// Tile partials of refine_stats_noalloc, for callers that cannot allocate a
// workspace: a fixed array in device memory (every GPU the library runs on
// holds its own copy until the process ends).  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): it uses the device address hipGetSymbolAddress returns, resolved
// once per device.
static __device__ __align__(256) double scratch[(size_t)kNoAllocStatTiles * kStatSlots];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

constexpr float kShC0 = 0.28209479177387814f;   // real SH band-0 basis value 1/(2 sqrt(pi))

__device__ inline bool finite_bits(float f) { return (__float_as_uint(f) & 0x7f800000u) != 0x7f800000u; }

// Per-thread accumulators of the tile: FP64 sums of the features, the
// non-finite count and the box of the finite centres.
struct Acc {
    double sY = 0.0, sY2 = 0.0, sOpa = 0.0, sGem = 0.0;
    uint32_t bad = 0;
    float bmin[3] = {INFINITY, INFINITY, INFINITY}, bmax[3] = {-INFINITY, -INFINITY, -INFINITY};

    __device__ void add(const float (&v)[kScorePlanes], float eta)
    {
        bool ok = true;
#pragma unroll
        for (int p = 0; p < kScorePlanes; ++p) ok = ok && finite_bits(v[p]);
        bad += ok ? 0u : 1u;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (finite_bits(v[c])) {
                bmin[c] = fminf(bmin[c], v[c]);
                bmax[c] = fmaxf(bmax[c], v[c]);
            }
        // luma of the DC colour (BT.601 weights)
        const float r = fmaf(kShC0, v[11], 0.5f);
        const float g = fmaf(kShC0, v[12], 0.5f);
        const float b = fmaf(kShC0, v[13], 0.5f);
        const float Y = 0.299f * r + 0.587f * g + 0.114f * b;
        // alpha (1 - alpha) = e alpha^2 with e = exp(-logit): no cancellation near alpha = 1
        const float e = __expf(-v[10]);
        const float alpha = 1.0f / (1.0f + e);
        const float amb = e * alpha * alpha;
        const float s0 = __expf(v[3]), s1 = __expf(v[4]), s2 = __expf(v[5]);
        const float smax = fmaxf(s0, fmaxf(s1, s2));
        const float smin = fminf(s0, fminf(s1, s2));
        const float gem = smax / (smin + eta);
        sY += (double)Y;
        sY2 += (double)Y * (double)Y;
        sOpa += (double)amb;
        sGem += (double)gem;
    }
};

// Block reduction of the accumulators and the tile's partial record.
__device__ void reduce_and_store(Acc& a, int tile, double* __restrict__ part)
{
    double sY = a.sY, sY2 = a.sY2, sOpa = a.sOpa, sGem = a.sGem;
    uint32_t bad = a.bad;
    float* bmin = a.bmin;
    float* bmax = a.bmax;
    sY = wave_sum(sY);
    sY2 = wave_sum(sY2);
    sOpa = wave_sum(sOpa);
    sGem = wave_sum(sGem);
    bad = wave_sum_u32(bad);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bmin[k] = wave_min(bmin[k]);
        bmax[k] = wave_max(bmax[k]);
    }
    __shared__ double red[kWaves][5];
    __shared__ float box[kWaves][6];
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        red[wave][0] = sY;
        red[wave][1] = sY2;
        red[wave][2] = sOpa;
        red[wave][3] = sGem;
        red[wave][4] = (double)bad;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            box[wave][k] = bmin[k];
            box[wave][3 + k] = bmax[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double acc = 0.0;
        for (int w = 0; w < kWaves; ++w) acc += red[w][threadIdx.x];
        part[(int64_t)tile * kStatSlots + threadIdx.x] = acc;
    } else if (threadIdx.x < 8) {
        // slots 5..7 carry the tile's box as bit patterns: min in the low and max in the high 32 bits
        const int k = threadIdx.x - 5;
        float lo = box[0][k], hi = box[0][3 + k];
        for (int w = 1; w < kWaves; ++w) {
            lo = fminf(lo, box[w][k]);
            hi = fmaxf(hi, box[w][3 + k]);
        }
        const uint64_t bits = (uint64_t)__float_as_uint(lo) | ((uint64_t)__float_as_uint(hi) << 32);
        part[(int64_t)tile * kStatSlots + threadIdx.x] = __longlong_as_double((long long)bits);
    }
}


template <int ST>
__device__ __forceinline__ void stats_partial_body(const void* __restrict__ planes, int64_t stride, int n,
                                                   float eta, double* __restrict__ part, int tile)
{
    const int base = tile * kTile;
    Acc a;
    // kBatch items' planes are loaded before any is used (14 kBatch loads in
    // flight per lane); lanes past the end load primitive n - 1 and skip it
    constexpr int kBatch = 4;
    for (int k0 = 0; k0 < kItems; k0 += kBatch) {
        if (base + k0 * kBlock >= n) break;   // uniform
        float v[kBatch][kScorePlanes];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int i = min(base + (k0 + k) * kBlock + (int)threadIdx.x, n - 1);
#pragma unroll
            for (int p = 0; p < kScorePlanes; ++p) v[k][p] = load_plane<ST>(planes, stride, p, i);
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k)
            if (base + (k0 + k) * kBlock + (int)threadIdx.x < n) a.add(v[k], eta);
    }
    reduce_and_store(a, tile, part);
}

// stats_partial for 16-byte aligned planes (stride a multiple of 16 bytes):
// a tile is rows of 16 bytes per lane (4 rows of 1024 FP32 primitives, or 2
// rows of 2048 2-byte primitives), each plane of a lane's PER consecutive
// primitives one 16-byte load; the same items, accumulated in the same
// order per thread as a lane's share of the tile (a different order from
// stats_partial: the sums agree to FP64 rounding).
template <int ST>
__device__ __forceinline__ void stats_partial_vec_body(const void* __restrict__ planes, int64_t stride, int n,
                                                       float eta, double* __restrict__ part, int tile)
{
    constexpr int PER = ST == kStoreF32 ? 4 : 8;        // primitives per 16-byte load
    constexpr int ROWS = kTile / (PER * kBlock);        // 4 or 2
    const int base = tile * kTile;
    Acc a;
    for (int r = 0; r < ROWS; ++r) {
        const int i0 = base + r * PER * kBlock + PER * (int)threadIdx.x;
        if (base + r * PER * kBlock >= n) break;   // uniform
        if (i0 + PER - 1 < n) {
            uint4 w[kScorePlanes];
#pragma unroll
            for (int p = 0; p < kScorePlanes; ++p) {
                const char* pl = static_cast<const char*>(planes) + ((int64_t)p * stride + i0) * storage_bytes(ST);
                w[p] = *reinterpret_cast<const uint4*>(pl);
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                float v[kScorePlanes];
#pragma unroll
                for (int p = 0; p < kScorePlanes; ++p) {
                    const uint32_t word = j / (PER / 4) == 0 ? w[p].x : j / (PER / 4) == 1 ? w[p].y
                                        : j / (PER / 4) == 2 ? w[p].z : w[p].w;
                    if constexpr (ST == kStoreF32) {
                        v[p] = __uint_as_float(word);
                    } else {
                        v[p] = widen2<ST>((uint16_t)((j & 1) ? (word >> 16) : (word & 0xFFFFu)), p);
                    }
                }
                a.add(v, eta);
            }
        } else {
            for (int j = 0; j < PER; ++j) {
                if (i0 + j >= n) break;
                float v[kScorePlanes];
#pragma unroll
                for (int p = 0; p < kScorePlanes; ++p) v[p] = load_plane<ST>(planes, stride, p, i0 + j);
                a.add(v, eta);
            }
        }
    }
    reduce_and_store(a, tile, part);
}

template <int ST>
__global__ __launch_bounds__(kBlock) void stats_partial_vec(const void* __restrict__ planes, int64_t stride, int n,
                                                              float eta, double* __restrict__ part)
{
    stats_partial_vec_body<ST>(planes, stride, n, eta, part, blockIdx.x);
}

template <int ST>
__global__ __launch_bounds__(kBlock) void stats_partial(const void* __restrict__ planes, int64_t stride,
                                                          int n, float eta, double* __restrict__ part)
{
    stats_partial_body<ST>(planes, stride, n, eta, part, blockIdx.x);
}

__device__ __forceinline__ void stats_finalize_body(const double* __restrict__ part, int ntiles, int64_t n,
                                                    const refine_params& prm, refine_stats_t* __restrict__ out)
{
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    float bmin[3] = {INFINITY, INFINITY, INFINITY}, bmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int t = threadIdx.x; t < ntiles; t += kBlock) {
#pragma unroll
        for (int s = 0; s < 5; ++s) acc[s] += part[(int64_t)t * kStatSlots + s];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint64_t bits = (uint64_t)__double_as_longlong(part[(int64_t)t * kStatSlots + 5 + k]);
            bmin[k] = fminf(bmin[k], __uint_as_float((uint32_t)bits));
            bmax[k] = fmaxf(bmax[k], __uint_as_float((uint32_t)(bits >> 32)));
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bmin[k] = wave_min(bmin[k]);
        bmax[k] = wave_max(bmax[k]);
    }
    __shared__ float box[kWaves][6];
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 3; ++k) {
            box[threadIdx.x / 64][k] = bmin[k];
            box[threadIdx.x / 64][3 + k] = bmax[k];
        }
    __shared__ double red[kWaves][5];
#pragma unroll
    for (int s = 0; s < 5; ++s) acc[s] = wave_sum(acc[s]);
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
        for (int s = 0; s < 5; ++s) red[wave][s] = acc[s];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot[5];
    for (int s = 0; s < 5; ++s) {
        tot[s] = 0.0;
        for (int w = 0; w < kWaves; ++w) tot[s] += red[w][s];
    }
    refine_stats_t r;
    for (int k = 0; k < 3; ++k) {
        float lo = box[0][k], hi = box[0][3 + k];
        for (int w = 1; w < kWaves; ++w) {
            lo = fminf(lo, box[w][k]);
            hi = fmaxf(hi, box[w][3 + k]);
        }
        // no finite centre: an empty box at the origin
        r.bbox_min[k] = lo <= hi ? lo : 0.0f;
        r.bbox_max[k] = lo <= hi ? hi : 0.0f;
    }
    r.n = n;
    r.n_nonfinite = (int64_t)tot[4];
    if (n > 0) {
        const double N = (double)n;
        r.ybar = tot[0] / N;
        const double var = tot[1] / N - r.ybar * r.ybar;
        r.f_col = var > 0.0 ? var : 0.0;
        r.f_opa = tot[2] / N;
        r.f_gem = tot[3] / N;
    } else {
        r.ybar = r.f_col = r.f_opa = r.f_gem = 0.0;
    }
    if (prm.equal_lambda || n == 0) {
        r.lambda[0] = r.lambda[1] = r.lambda[2] = 1.0 / 3.0;
    } else {
        // Eq. 18: calibrated features, Eq. 19: normalised to sum 1
        const double lg = log(r.f_gem + prm.eta) / prm.e_lngem;
        const double lc = r.f_col / prm.e_col;
        const double lo = r.f_opa / prm.e_opa;
        const double sum = lg + lc + lo;
        r.lambda[0] = lg / sum;
        r.lambda[1] = lc / sum;
        r.lambda[2] = lo / sum;
    }
    *out = r;
}

__global__ __launch_bounds__(kBlock) void stats_finalize(const double* __restrict__ part, int ntiles, int64_t n,
                                                           refine_params prm, refine_stats_t* __restrict__ out)
{
    stats_finalize_body(part, ntiles, n, prm, out);
}

// Grouped launches: one tile of one job per block / one job per block.
__global__ __launch_bounds__(kBlock) void stats_partial_batch(const BatchJob* __restrict__ jobs, int nj, float eta)
{
    const BatchJob& b = jobs[batch_job_of<true>(jobs, nj, blockIdx.x)];
    const int tile = (int)blockIdx.x - b.tile0;
    // the same kernel body the single-scene call picks, so the results agree bit for bit
    if (b.st == kStoreF32 && b.vec_stats)
        stats_partial_vec_body<kStoreF32>(b.planes, b.stride, b.n, eta, b.stat_part, tile);
    else if (b.st == kStoreF32)
        stats_partial_body<kStoreF32>(b.planes, b.stride, b.n, eta, b.stat_part, tile);
    else if (b.st == kStoreBF16F16 && b.vec_stats)
        stats_partial_vec_body<kStoreBF16F16>(b.planes, b.stride, b.n, eta, b.stat_part, tile);
    else if (b.st == kStoreBF16F16)
        stats_partial_body<kStoreBF16F16>(b.planes, b.stride, b.n, eta, b.stat_part, tile);
    else if (b.vec_stats)
        stats_partial_vec_body<kStoreF16>(b.planes, b.stride, b.n, eta, b.stat_part, tile);
    else
        stats_partial_body<kStoreF16>(b.planes, b.stride, b.n, eta, b.stat_part, tile);
}

// Also sets up each job's selection (its state and cleared histograms): the
// selection passes come later in the batch's launch sequence, and one launch
// fewer matters for batches of small scenes.
__global__ __launch_bounds__(kBlock) void stats_finalize_batch(const BatchJob* __restrict__ jobs, refine_params prm)
{
    const BatchJob& b = jobs[blockIdx.x];
    stats_finalize_body(b.stat_part, (int)num_tiles(b.n), b.n, prm, b.stats);
    for (int w = threadIdx.x; w < kSelectHistWords; w += kBlock) b.hist[w] = 0u;
    if (threadIdx.x == 0) *b.sel = select_start(b.n, b.n_prune);
}

}  // namespace

hipError_t launch_stats_batch(const BatchJob* d_jobs, int n_jobs, int total_tiles, const refine_params& prm,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(stats_partial_batch, dim3(total_tiles), dim3(kBlock), 0, stream, d_jobs, n_jobs,
                       (float)prm.eta);
    hipLaunchKernelGGL(stats_finalize_batch, dim3(n_jobs), dim3(kBlock), 0, stream, d_jobs, prm);
    return hipGetLastError();
}

hipError_t stats_scratch(double** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_stats(const void* planes, int st, int64_t stride, int64_t n, const refine_params& prm,
                        refine_stats_t* d_stats, const Workspace& ws, hipStream_t stream)
{
    const int ntiles = (int)num_tiles(n);
    if (ntiles > 0) {
        const bool vec = reinterpret_cast<uintptr_t>(planes) % 16 == 0 && (stride * storage_bytes(st)) % 16 == 0;
        with_storage(st, [&](auto st_c) {
            constexpr int ST = decltype(st_c)::value;
            if (vec)
                hipLaunchKernelGGL(stats_partial_vec<ST>, dim3(ntiles), dim3(kBlock), 0, stream, planes, stride,
                                   (int)n, (float)prm.eta, ws.stat_part);
            else
                hipLaunchKernelGGL(stats_partial<ST>, dim3(ntiles), dim3(kBlock), 0, stream, planes, stride, (int)n,
                                   (float)prm.eta, ws.stat_part);
        });
    }
    hipLaunchKernelGGL(stats_finalize, dim3(1), dim3(kBlock), 0, stream, ws.stat_part, ntiles, n, prm, d_stats);
    return hipGetLastError();
}

}  // namespace refine
