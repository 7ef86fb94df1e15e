// Rendering-free importance scores (paper Eq. 7-20) on gfx950.
//
// camera_prep: one thread per (possibly subsampled) view builds two 128-byte
// fp32 records: the constants of the per-pair evaluation (every pixel
// quantity scaled by sv = 1/sqrt(fx^2 + fy^2): the gate is scale invariant
// and the projection term's 1/(fx^2 + fy^2) becomes 1), and the world-space
// frustum half-spaces of the conservative culling test.
//
// Per (primitive, view) pair, FP32 (eval_pair; identical in both paths):
//   X = sv (fx x + (cx - W/2) z), Y likewise, z   camera-space centre with the
//                                     image centre as origin (Eq. 13 numerators)
//   q = 1/(z (z^2 + eta)):  1/z = q (z^2 + eta),  1/(z^2 + eta) = q z
//   ux = X/z, uy = Y/z                projected centre about the image centre
//   x^ = clamp(ux, ox -+ lx), y^ likewise   EWA clamp of x/z (scaled pixels,
//                                     shifted by ox = sv (cx - W/2))
//   r0 = sv fx R_v,0 + ox R_v,2 - x^ R_v,2,  r1 likewise
//       [r0; r1] / z is the scaled EWA Jacobian times the view rotation (Eq. 14)
//   A0 = r0 L, A1 = r1 L with L = R(q) diag(s);  a = |A0|^2, b = A0.A1, c = |A1|^2
//       z^2 Sigma' = [[a, b], [b, c]] as sums of squares (no cancellation for
//       needle-like primitives, unlike T Sigma T^T in FP32); the kernels hold
//       3 L, so their sums are 9 a, 9 b, 9 c
//   gate: z > z_near, and the centre lies within the 3-sigma radius
//       r = 3 sqrt(lambda_max(Sigma')) of the image rectangle; with
//       d = max(|ux| - hw, |uy| - hh) the test d < r reads
//       d z < 0  or  (d z)^2 < 4.5 (a + c + sqrt((a - c)^2 + 4 b^2)),
//       evaluated without the square root (g = (d z)^2 / 9, u = g - a,
//       v = g - c: u + v < 0 or u v < b^2)
//   d z itself is max(|X| - hw z, |Y| - hh z)
//   projection term: COV (a + c)/(z^2 + eta) (1/sbar^2 applied in the
//       epilogue, as 1/(9 sbar^2) with the kernels' 3 L), DEPTH
//       1/(z^2 + eta) (Eq. 17), NONE 1
// Views are accumulated in view order within blocks of 64 (kViewBlock), the
// block sums added in order into one FP32 total per primitive; the
// epilogue forms D = (V K [/ sbar^2]) S / |V| (Eq. 20, then Eq. 7).  The
// binned records hold V K [/ sbar^2], which does not depend on the cameras,
// so a new camera set only needs new camera records (refine_score_cameras).
//
// Direct path (score_direct): one primitive per lane in input order, every
// pair evaluated; score_direct_batch runs it for the jobs of a batch in one
// grouped launch (camera_prep_batch builds their camera records).
//
// Binned path, preparation (camera independent): bin_hist / bin_scan /
// bin_rank / bin_scatter counting-sort the primitives by the Morton code of a
// 16^3 grid over the centres' bounding box (per-tile LDS histograms, so a
// crowded cell costs one global atomic per tile, not per primitive) and write
// each activated primitive as a record in cell order; group_bounds bounds
// each group of 64 consecutive records by a box and a sphere about its
// centres and by its largest scale s_max.  (Finer grids cull more pairs but
// do not fit the per-tile LDS histograms, and one global atomic per primitive
// costs more than they save.)
//
// Binned path, per camera set: cull_groups gives every group the set of
// views it evaluates: a view is dropped only when no point of the group's
// bounds can pass the near plane or one image edge even with the largest
// footprint any of its primitives can have, r <= 3 s_max |J|_2 (the clamp
// bounds the spectral norm |z J|_2 by kv), inflated by a 1% margin, so every dropped pair
// would have added exactly +0 and both paths give bit-identical scores.
// place_groups orders the groups by how many views they keep (most first,
// so no long group runs alone at the end), and score_binned gives each wave
// one group and evaluates its kept views in increasing view order.  For each
// kept view a wave first computes only its records' camera-space centres and
// d z, and stops there when no record can pass under the same footprint
// bound with its own s_max (pair_may_pass): those terms are +0 as well.
#include <type_traits>

#include "refine_internal.hpp"

namespace refine {

namespace {

constexpr float kShC0 = 0.28209479177387814f;
constexpr float kCullMargin = 1.01f;
constexpr int64_t kBinnedMinPrims = 65536;
constexpr int kDefaultPPL = 2;   // binned records per lane unless the caller picks (2: half the culling tests)
constexpr int kDefaultVPI = 1;   // views per iteration of the binned view loop unless the caller picks

// 3 (1 + margin) times a bound on the spectral norm of z J over the clamp
// box |x/z| <= limx, |y/z| <= limy, where z J = [[fx, 0, -fx x^], [0, fy,
// -fy y^]]: a primitive's footprint radius obeys r z <= 3 s_max |z J R_v|_2
// = 3 s_max |z J|_2.  |z J|_2^2 is the larger eigenvalue of
// [[fx^2 (1 + x^2), fx fy x y], [fx fy x y, fy^2 (1 + y^2)]], which grows
// with |x^| and |y^|, so its largest value is at a corner of the box.
__device__ __forceinline__ float footprint_bound(float fx, float fy, float limx, float limy)
{
    const float a = fx * fx * (1.0f + limx * limx), c = fy * fy * (1.0f + limy * limy);
    const float b = fx * fy * limx * limy;
    const float h = 0.5f * (a - c);
    return 3.0f * kCullMargin * sqrtf(0.5f * (a + c) + sqrtf(h * h + b * b));
}

// The records of view slot j (cull may be null: no culling records).
__device__ __forceinline__ void camera_prep_body(const float* __restrict__ cams, int n_views, int nv, float clamp_k,
                                                 CamRec* __restrict__ out, CullRec* __restrict__ cull, int j)
{
    const int v = (nv == n_views) ? j : (int)(((int64_t)j * n_views) / nv);
    const float* c = cams + (int64_t)v * kCamFields;
    const float fx = c[12], fy = c[13], cx = c[14], cy = c[15], W = c[16], H = c[17];
    const float sv = rsqrtf(fx * fx + fy * fy);
    const float sx = sv * fx, sy = sv * fy;
    CamRec r;
    const float ox = sv * (cx - 0.5f * W), oy = sv * (cy - 0.5f * H);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.px[k] = fmaf(ox, c[6 + k], sx * c[k]);
        r.py[k] = fmaf(oy, c[6 + k], sy * c[3 + k]);
        r.pz[k] = c[6 + k];
    }
    r.px[3] = fmaf(ox, c[11], sx * c[9]);
    r.py[3] = fmaf(oy, c[11], sy * c[10]);
    r.pz[3] = c[11];
    r.hw = sv * (0.5f * W);
    r.hh = sv * (0.5f * H);
    const float lx = clamp_k * r.hw, ly = clamp_k * r.hh;
    r.cx0 = ox - lx;
    r.cx1 = ox + lx;
    r.cy0 = oy - ly;
    r.cy1 = oy + ly;
    const float kv3 = footprint_bound(fx, fy, clamp_k * W / (2.0f * fx), clamp_k * H / (2.0f * fy));
    r.kvs = sv * kv3;   // the same bound in the scaled units of this record
#pragma unroll
    for (int k = 0; k < 13; ++k) r.pad[k] = 0.0f;
    out[j] = r;
    if (!cull) return;

    // culling half-spaces: u + r > 0, W - u + r > 0, v + r > 0, H - v + r > 0,
    // multiplied by z > 0 and written as n . mu + d + r z > 0 with r z <= 3 s_max kv
    CullRec q;
    const float* R0 = c;
    const float* R1 = c + 3;
    const float* R2 = c + 6;
    const float tx = c[9], ty = c[10], tz = c[11];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q.nz[k] = R2[k];
        q.side[0][k] = fx * R0[k] + cx * R2[k];
        q.side[1][k] = (W - cx) * R2[k] - fx * R0[k];
        q.side[2][k] = fy * R1[k] + cy * R2[k];
        q.side[3][k] = (H - cy) * R2[k] - fy * R1[k];
    }
    q.nz[3] = tz;
    q.side[0][3] = fx * tx + cx * tz;
    q.side[1][3] = (W - cx) * tz - fx * tx;
    q.side[2][3] = fy * ty + cy * tz;
    q.side[3][3] = (H - cy) * tz - fy * ty;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        q.nn[s] = sqrtf(q.side[s][0] * q.side[s][0] + q.side[s][1] * q.side[s][1] + q.side[s][2] * q.side[s][2]);
    q.kv3 = kv3;
#pragma unroll
    for (int k = 0; k < 7; ++k) q.pad[k] = 0.0f;
    cull[j] = q;
}

// Also clears the binning cell counts (cell_cnt is null when the scene is
// not binned) and the work-class counts the culling adds into (aux is null
// on the direct path).
__global__ __launch_bounds__(kBlock) void camera_prep(const float* __restrict__ cams, int n_views, int nv,
                                                        float clamp_k, CamRec* __restrict__ out,
                                                        CullRec* __restrict__ cull, uint32_t* __restrict__ cell_cnt,
                                                        uint32_t* __restrict__ aux)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (cell_cnt && j < kCells * kBinCopies) cell_cnt[j] = 0u;
    if (aux && j < kOrderBuckets * kOrderCopies) aux[kOrderBuckets + j] = 0u;
    if (j < nv) camera_prep_body(cams, n_views, nv, clamp_k, out, cull, j);
}

// Registers a lane keeps for one primitive across the view loop.
// Each primitive's sum over views is blocked: views in order within a block
// of 64 (one 64-bit mask word of the binned path), block sums added in
// order, so the FP32 rounding error grows with 64 + n_views / 64 instead of
// n_views.
constexpr int kViewBlock = 64;
static_assert(kViewBlock == 64, "a block is one 64-bit mask word");

struct Prim {
    float mx, my, mz;
    float L00, L01, L02, L10, L11, L12, L20, L21, L22;
    float S;
};

// The evaluation constants of a camera record (its first 80 bytes), held in
// vector registers.
struct CamEval {
    float px[4], py[4], pz[4];
    float cx0, cx1, cy0, cy1, hw, hh, kvs;
};
constexpr int kStageVec = 5;   // float4s staged per view
static_assert(offsetof(CamRec, kvs) + sizeof(float) <= kStageVec * sizeof(float4), "staged camera fields");

// Activation (Sec. 3.1 readings) of primitive i; pre is the epilogue factor.
template <int ST>
__device__ inline void activate(const void* __restrict__ planes, int64_t stride, int i, Prim& p, float& pre,
                                float& smax, const refine_stats_t* __restrict__ st, int proj, int vis_alpha)
{
    float a[kScorePlanes];
#pragma unroll
    for (int k = 0; k < kScorePlanes; ++k) a[k] = load_plane<ST>(planes, stride, k, i);
    p.mx = a[0];
    p.my = a[1];
    p.mz = a[2];
    const float s0 = __expf(a[3]), s1 = __expf(a[4]), s2 = __expf(a[5]);
    float qw = a[6], qx = a[7], qy = a[8], qz = a[9];
    const float qn = qw * qw + qx * qx + qy * qy + qz * qz;
    if (qn > 0.0f) {
        const float inv = rsqrtf(qn);
        qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    } else {
        qw = 1.0f; qx = qy = qz = 0.0f;
    }
    // L = 3 R(q) diag(s): the factor 3 of the 3-sigma radius rides in L, so
    // the gate compares (d z)^2 with the projected covariance directly; the
    // COV epilogue factor below divides the resulting 9 back out
    const float t0 = 3.0f * s0, t1 = 3.0f * s1, t2 = 3.0f * s2;
    p.L00 = (1.0f - 2.0f * (qy * qy + qz * qz)) * t0;
    p.L01 = (2.0f * (qx * qy - qw * qz)) * t1;
    p.L02 = (2.0f * (qx * qz + qw * qy)) * t2;
    p.L10 = (2.0f * (qx * qy + qw * qz)) * t0;
    p.L11 = (1.0f - 2.0f * (qx * qx + qz * qz)) * t1;
    p.L12 = (2.0f * (qy * qz - qw * qx)) * t2;
    p.L20 = (2.0f * (qx * qz - qw * qy)) * t0;
    p.L21 = (2.0f * (qy * qz + qw * qx)) * t1;
    p.L22 = (1.0f - 2.0f * (qx * qx + qy * qy)) * t2;
    p.S = 0.0f;
    smax = fmaxf(s0, fmaxf(s1, s2));
    const float ssq = s0 * s0 + s1 * s1 + s2 * s2;   // 3 sbar^2
    const float alpha = 1.0f / (1.0f + __expf(-a[10]));
    const float cr = fmaf(kShC0, a[11], 0.5f), cg = fmaf(kShC0, a[12], 0.5f), cb = fmaf(kShC0, a[13], 0.5f);
    // attribute magnitudes G~ (Eq. 7): two largest scales' product, |DC colour|, alpha
    const float g_gem = fmaxf(s0 * s1, fmaxf(s0 * s2, s1 * s2));
    const float g_col = sqrtf(cr * cr + cg * cg + cb * cb);
    const float K = (float)st->lambda[0] * g_gem + (float)st->lambda[1] * g_col + (float)st->lambda[2] * alpha;
    pre = (vis_alpha ? alpha : 1.0f) * K;
    if (proj == REFINE_PROJ_COV) pre = pre / (3.0f * ssq);   // 1 / (9 sbar^2): L carries 3
}

// The first part of a pair's evaluation: the camera-space centre and d z.
struct PairHead {
    float X, Y, z, dz;
};

template <class Cam>
__device__ __forceinline__ PairHead pair_head(const Cam& c, const Prim& p)
{
    PairHead hd;
    hd.X = fmaf(c.px[0], p.mx, fmaf(c.px[1], p.my, fmaf(c.px[2], p.mz, c.px[3])));
    hd.Y = fmaf(c.py[0], p.mx, fmaf(c.py[1], p.my, fmaf(c.py[2], p.mz, c.py[3])));
    hd.z = fmaf(c.pz[0], p.mx, fmaf(c.pz[1], p.my, fmaf(c.pz[2], p.mz, c.pz[3])));
    // d z with d = max(|ux| - hw, |uy| - hh) (z > 0 wherever it matters)
    hd.dz = fmaxf(fmaf(-c.hw, hd.z, fabsf(hd.X)), fmaf(-c.hh, hd.z, fabsf(hd.Y)));
    return hd;
}

// Whether the pair can pass the gate at all: the footprint radius r obeys
// r z <= 3 s_max |z J R_v|_2 <= kvs s_max / (1 + margin) under the clamp, so a
// pair with d z >= kvs s_max (or behind the near plane) adds exactly +0.
// Written so that a NaN bound or d z counts as "can pass".
__device__ __forceinline__ bool pair_may_pass(const PairHead& hd, float kvs, float smax, float z_near)
{
    return (hd.z > z_near) && !(hd.dz >= kvs * smax);
}

template <int PROJ, class Cam>
__device__ __forceinline__ void pair_tail(const Cam& c, Prim& p, const PairHead& hd, float eta, float z_near)
{
    const float z = hd.z, dz = hd.dz;
    const float zz = fmaf(z, z, eta);
    const float q = __builtin_amdgcn_rcpf(z * zz);
    const float rz = q * zz;
    const float ux = hd.X * rz;
    const float uy = hd.Y * rz;
    const float xh = __builtin_amdgcn_fmed3f(ux, c.cx0, c.cx1);
    const float yh = __builtin_amdgcn_fmed3f(uy, c.cy0, c.cy1);
    const float r00 = fmaf(-xh, c.pz[0], c.px[0]);
    const float r01 = fmaf(-xh, c.pz[1], c.px[1]);
    const float r02 = fmaf(-xh, c.pz[2], c.px[2]);
    const float r10 = fmaf(-yh, c.pz[0], c.py[0]);
    const float r11 = fmaf(-yh, c.pz[1], c.py[1]);
    const float r12 = fmaf(-yh, c.pz[2], c.py[2]);
    const float A00 = fmaf(r00, p.L00, fmaf(r01, p.L10, r02 * p.L20));
    const float A01 = fmaf(r00, p.L01, fmaf(r01, p.L11, r02 * p.L21));
    const float A02 = fmaf(r00, p.L02, fmaf(r01, p.L12, r02 * p.L22));
    const float A10 = fmaf(r10, p.L00, fmaf(r11, p.L10, r12 * p.L20));
    const float A11 = fmaf(r10, p.L01, fmaf(r11, p.L11, r12 * p.L21));
    const float A12 = fmaf(r10, p.L02, fmaf(r11, p.L12, r12 * p.L22));
    const float sa = fmaf(A00, A00, fmaf(A01, A01, A02 * A02));
    const float sc = fmaf(A10, A10, fmaf(A11, A11, A12 * A12));
    const float sb = fmaf(A00, A10, fmaf(A01, A11, A02 * A12));
    const float ss = sa + sc;
    float P;
    if (PROJ == REFINE_PROJ_COV)
        P = ss * (q * z);
    else if (PROJ == REFINE_PROJ_DEPTH)
        P = q * z;
    else
        P = 1.0f;
    // With L scaled by 3, sa, sb, sc are 9 a, 9 b, 9 c, and the footprint
    // test (d z)^2 < 4.5 (a + c + sqrt((a - c)^2 + 4 b^2)) reads
    // g < (sa + sc)/2 + sqrt(((sa - sc)/2)^2 + sb^2) with g = (d z)^2; with
    // u = g - sa, v = g - sc it holds iff u + v < 0 or u v < sb^2 (both
    // sides squared), so no square root is needed
    const float gq = dz * dz;
    const float u = gq - sa, v = gq - sc;
    const float h = fmaf(-sb, sb, u * v);
    // dz < 0 or u + v < 0 or h < 0, as one compare: the others are NaN
    // whenever dz is, and fminf returns the other operand when one is NaN
    const bool g = (z > z_near) && (fminf(dz, fminf(u + v, h)) < 0.0f);
    p.S += g ? P : 0.0f;
}

template <int PROJ, class Cam>
__device__ __forceinline__ void eval_pair(const Cam& c, Prim& p, float eta, float z_near)
{
    pair_tail<PROJ>(c, p, pair_head(c, p), eta, z_near);
}

template <int PROJ, int ST>
__device__ __forceinline__ void score_direct_body(const void* __restrict__ planes, int64_t stride, int n,
                                                  const CamRec* __restrict__ cams, int nv,
                                                  const refine_stats_t* __restrict__ st, float eta, float z_near,
                                                  int vis_alpha, float* __restrict__ out, int i)
{
    if (i >= n) return;
    Prim p;
    float pre, smax;
    activate<ST>(planes, stride, i, p, pre, smax, st, PROJ, vis_alpha);
    // views summed in order within each block of kViewBlock, the block sums
    // added in order (the binned path takes the same blocks: its mask words)
    float total = 0.0f;
    for (int v0 = 0; v0 < nv; v0 += kViewBlock) {
        const int v1 = min(v0 + kViewBlock, nv);
        for (int v = v0; v < v1; ++v) eval_pair<PROJ>(cams[v], p, eta, z_near);
        total += p.S;
        p.S = 0.0f;
    }
    out[i] = pre * total / (float)nv;
}

template <int PROJ, int ST>
__global__ __launch_bounds__(kBlock) void score_direct(const void* __restrict__ planes, int64_t stride, int n,
                                                         const CamRec* __restrict__ cams, int nv,
                                                         const refine_stats_t* __restrict__ st, float eta,
                                                         float z_near, int vis_alpha, float* __restrict__ out)
{
    score_direct_body<PROJ, ST>(planes, stride, n, cams, nv, st, eta, z_near, vis_alpha, out,
                                blockIdx.x * kBlock + threadIdx.x);
}

// The opacity-only ranking (score_kind = OPACITY): D_i = alpha_i, the same
// FP32 sigmoid the activation computes.
template <int ST>
__device__ __forceinline__ void score_opacity_body(const void* __restrict__ planes, int64_t stride, int n,
                                                   float* __restrict__ out, int i)
{
    if (i < n) out[i] = 1.0f / (1.0f + __expf(-load_plane<ST>(planes, stride, 10, i)));
}

template <int ST>
__global__ __launch_bounds__(kBlock) void score_opacity(const void* __restrict__ planes, int64_t stride, int n,
                                                          float* __restrict__ out)
{
    score_opacity_body<ST>(planes, stride, n, out, blockIdx.x * kBlock + threadIdx.x);
}

// Grouped launches: the camera records of one job per block, and the direct
// view loop over 256 primitives of one job per block.
__global__ __launch_bounds__(kBlock) void camera_prep_batch(const BatchJob* __restrict__ jobs, float clamp_k)
{
    const BatchJob& b = jobs[blockIdx.x];
    for (int j = threadIdx.x; j < b.nv; j += kBlock)
        camera_prep_body(b.cams, b.n_views, b.nv, clamp_k, b.cam_rec, nullptr, j);
}

__global__ __launch_bounds__(kBlock) void score_opacity_batch(const BatchJob* __restrict__ jobs, int nj)
{
    const BatchJob& b = jobs[batch_job_of<false>(jobs, nj, blockIdx.x)];
    const int i = ((int)blockIdx.x - b.block0) * kBlock + (int)threadIdx.x;
    if (b.st == kStoreF32)
        score_opacity_body<kStoreF32>(b.planes, b.stride, b.n, b.scores, i);
    else if (b.st == kStoreBF16F16)
        score_opacity_body<kStoreBF16F16>(b.planes, b.stride, b.n, b.scores, i);
    else
        score_opacity_body<kStoreF16>(b.planes, b.stride, b.n, b.scores, i);
}

template <int PROJ>
__global__ __launch_bounds__(kBlock) void score_direct_batch(const BatchJob* __restrict__ jobs, int nj, float eta,
                                                               float z_near, int vis_alpha)
{
    const BatchJob& b = jobs[batch_job_of<false>(jobs, nj, blockIdx.x)];
    const int i = ((int)blockIdx.x - b.block0) * kBlock + (int)threadIdx.x;
    if (b.st == kStoreF32)
        score_direct_body<PROJ, kStoreF32>(b.planes, b.stride, b.n, b.cam_rec, b.nv, b.stats, eta, z_near,
                                           vis_alpha, b.scores, i);
    else if (b.st == kStoreBF16F16)
        score_direct_body<PROJ, kStoreBF16F16>(b.planes, b.stride, b.n, b.cam_rec, b.nv, b.stats, eta, z_near,
                                               vis_alpha, b.scores, i);
    else
        score_direct_body<PROJ, kStoreF16>(b.planes, b.stride, b.n, b.cam_rec, b.nv, b.stats, eta, z_near,
                                           vis_alpha, b.scores, i);
}

// ------------------------------------------------------------- binned path

__device__ inline uint32_t spread_bits(uint32_t x)
{
    // the low kCellBits bits of x moved to every third bit
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < kCellBits; ++b) r |= ((x >> b) & 1u) << (3 * b);
    return r;
}

// Morton cell of a centre in the kCells-cell grid over the centres' box.
__device__ inline uint32_t cell_of(float x, float y, float z, const refine_stats_t* __restrict__ st)
{
    const float k = (float)(1 << kCellBits);
    const float in[3] = {x, y, z};
    uint32_t q[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = st->bbox_min[a], span = st->bbox_max[a] - lo;
        const float t = span > 0.0f ? (in[a] - lo) * (k / span) : 0.0f;
        q[a] = (uint32_t)fminf(fmaxf(t, 0.0f), k - 1.0f);   // NaN -> 0
    }
    return spread_bits(q[0]) | (spread_bits(q[1]) << 1) | (spread_bits(q[2]) << 2);
}

// Binning tiles are the 4096-primitive tiles of the other kernels.  Each
// tile counts its cells in LDS and touches the global cell arrays once per
// occupied cell, in cell order (consecutive lanes hit consecutive counters,
// so the atomics coalesce); global atomics are memory transactions here, so
// their number, not the LDS work, sets the cost.  The global counters come
// in kBinCopies copies (tile t uses copy t mod kBinCopies, copy-major so the
// lanes stay coalesced), which divides the atomics per address by 8; a
// cell's range holds copy 0's primitives, then copy 1's, and so on.
constexpr int kCellsPerThread = kCells / kBlock;   // 16

// Cells of this thread's kItems primitives of the tile: every centre is
// loaded before any is quantised (lanes past the end load primitive n - 1;
// the callers skip them).
template <int ST>
__device__ inline void tile_cells(const void* __restrict__ planes, int64_t stride, int n, int base,
                                  const refine_stats_t* __restrict__ st, uint32_t (&cell)[kItems])
{
    float x[kItems], y[kItems], z[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = min(base + k * kBlock + (int)threadIdx.x, n - 1);
        x[k] = load_plane<ST>(planes, stride, 0, i);
        y[k] = load_plane<ST>(planes, stride, 1, i);
        z[k] = load_plane<ST>(planes, stride, 2, i);
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) cell[k] = cell_of(x[k], y[k], z[k], st);
}

// Cell histogram of the tile's primitives.
template <int ST>
__global__ __launch_bounds__(kBlock) void bin_hist(const void* __restrict__ planes, int64_t stride, int n,
                                                     const refine_stats_t* __restrict__ st,
                                                     uint32_t* __restrict__ cnt)
{
    __shared__ uint32_t h[kCells];
    for (int c = threadIdx.x; c < kCells; c += kBlock) h[c] = 0u;
    __syncthreads();
    const int base = blockIdx.x * kTile;
    uint32_t cell[kItems];
    tile_cells<ST>(planes, stride, n, base, st, cell);
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k * kBlock + (int)threadIdx.x < n) atomicAdd(&h[cell[k]], 1u);
    __syncthreads();
    const int copy = blockIdx.x % kBinCopies;
#pragma unroll
    for (int j = 0; j < kCellsPerThread; ++j) {
        const int c = j * kBlock + (int)threadIdx.x;
        if (h[c]) atomicAdd(&cnt[copy * kCells + c], h[c]);
    }
}

// Cell offsets (one block): each cell's range starts at the exclusive scan of
// the cell totals, and the range of copy k of the cell after copies 0..k-1.
__global__ __launch_bounds__(kScanThreads) void bin_scan(const uint32_t* __restrict__ cnt, uint32_t* __restrict__ cur)
{
    constexpr int kPer = kCells / kScanThreads;   // 4 cells per thread
    static_assert(kPer == 4, "one 16-byte load per copy");
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    uint32_t c8[kPer][kBinCopies];
    uint32_t local = 0;
#pragma unroll
    for (int k = 0; k < kBinCopies; ++k) {
        const uint4 a = reinterpret_cast<const uint4*>(cnt + k * kCells)[threadIdx.x];
        c8[0][k] = a.x; c8[1][k] = a.y; c8[2][k] = a.z; c8[3][k] = a.w;
        local += a.x + a.y + a.z + a.w;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    uint32_t run = incl - local;
    for (int w = 0; w < wave; ++w) run += wave_tot[w];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        uint32_t o[kBinCopies];
#pragma unroll
        for (int k = 0; k < kBinCopies; ++k) {
            o[k] = run;
            run += c8[j][k];
        }
#pragma unroll
        for (int k = 0; k < kBinCopies; ++k) cur[k * kCells + threadIdx.x * kPer + j] = o[k];
    }
}

// Counting-sort ranks: each tile reserves one output range per occupied cell
// with a single global atomic; its primitives take consecutive slots in it.
template <int ST>
__global__ __launch_bounds__(kBlock) void bin_rank(const void* __restrict__ planes, int64_t stride, int n,
                                                     const refine_stats_t* __restrict__ st, uint32_t* __restrict__ cur,
                                                     uint32_t* __restrict__ dest)
{
    __shared__ uint32_t h[kCells];
    for (int c = threadIdx.x; c < kCells; c += kBlock) h[c] = 0u;
    __syncthreads();
    const int base = blockIdx.x * kTile;
    uint32_t cell[kItems], rank[kItems];
    tile_cells<ST>(planes, stride, n, base, st, cell);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        rank[k] = 0u;
        if (base + k * kBlock + (int)threadIdx.x < n) rank[k] = atomicAdd(&h[cell[k]], 1u);
    }
    __syncthreads();
    // all reservations of this thread are issued before any result is used
    uint32_t got[kCellsPerThread];
    const int copy = blockIdx.x % kBinCopies;
#pragma unroll
    for (int j = 0; j < kCellsPerThread; ++j) {
        const int c = j * kBlock + (int)threadIdx.x;
        const uint32_t m = h[c];
        got[j] = m ? atomicAdd(&cur[copy * kCells + c], m) : 0u;
    }
#pragma unroll
    for (int j = 0; j < kCellsPerThread; ++j) h[j * kBlock + (int)threadIdx.x] = got[j];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int i = base + k * kBlock + (int)threadIdx.x;
        if (i < n) dest[i] = h[cell[k]] + rank[k];
    }
}

// Activated primitives written as records at their binned positions.  The
// block's records pass through LDS so that each quad of lanes stores one
// whole 64-byte record (16 records per store instruction instead of 64
// scattered 16-byte pieces).
template <int PROJ, int ST>
__global__ __launch_bounds__(kBlock) void bin_scatter(const void* __restrict__ planes, int64_t stride, int n,
                                                        const refine_stats_t* __restrict__ st, int vis_alpha,
                                                        const uint32_t* __restrict__ dest, PrimRec* __restrict__ recs)
{
    __shared__ float4 srec[kBlock][4];
    __shared__ uint32_t spos[kBlock];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        Prim p;
        float pre, smax;
        activate<ST>(planes, stride, i, p, pre, smax, st, PROJ, vis_alpha);
        spos[threadIdx.x] = dest[i];
        srec[threadIdx.x][0] = make_float4(p.mx, p.my, p.mz, smax);
        srec[threadIdx.x][1] = make_float4(p.L00, p.L01, p.L02, p.L10);
        srec[threadIdx.x][2] = make_float4(p.L11, p.L12, p.L20, p.L21);
        srec[threadIdx.x][3] = make_float4(p.L22, pre, __int_as_float(i), 0.0f);
        static_assert(offsetof(PrimRec, L) == 16 && offsetof(PrimRec, idx) == 56, "record layout");
    } else {
        spos[threadIdx.x] = 0xFFFFFFFFu;
    }
    __syncthreads();
    const int piece = threadIdx.x & 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int rr = k * (kBlock / 4) + (threadIdx.x >> 2);
        const uint32_t pos = spos[rr];
        // always true for filled slots: the ranks are a permutation of [0, n)
        if (pos < (uint32_t)n) reinterpret_cast<float4*>(recs + pos)[piece] = srec[rr][piece];
    }
}

// Bounds of each group of kGroup consecutive binned records (16 lanes per
// group, 4 records per lane; records past the end repeat the last one): the
// box and sphere of the centres, inflated by the culling margin plus a
// relative slack, and the largest scale.  They do not depend on the cameras.
constexpr int kBoundLanes = 16;
constexpr int kBoundPer = kGroup / kBoundLanes;   // 4

__device__ inline float seg_min(float x)
{
#pragma unroll
    for (int o = kBoundLanes / 2; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o, kBoundLanes));
    return x;
}

__device__ inline float seg_max(float x)
{
#pragma unroll
    for (int o = kBoundLanes / 2; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, kBoundLanes));
    return x;
}

__global__ __launch_bounds__(kBlock) void group_bounds(const PrimRec* __restrict__ recs, int n,
                                                         GroupBound* __restrict__ gb, int ngroups)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int g = t / kBoundLanes, sl = t % kBoundLanes;
    const bool ok = g < ngroups;   // whole 16-lane segments
    float4 r[kBoundPer];
#pragma unroll
    for (int k = 0; k < kBoundPer; ++k) {
        const int j = ok ? min(g * kGroup + k * kBoundLanes + sl, n - 1) : 0;
        r[k] = *reinterpret_cast<const float4*>(recs + j);   // centre, s_max
    }
    float lo[3] = {r[0].x, r[0].y, r[0].z}, hi[3] = {r[0].x, r[0].y, r[0].z}, sg = r[0].w;
#pragma unroll
    for (int k = 1; k < kBoundPer; ++k) {
        lo[0] = fminf(lo[0], r[k].x); hi[0] = fmaxf(hi[0], r[k].x);
        lo[1] = fminf(lo[1], r[k].y); hi[1] = fmaxf(hi[1], r[k].y);
        lo[2] = fminf(lo[2], r[k].z); hi[2] = fmaxf(hi[2], r[k].z);
        sg = fmaxf(sg, r[k].w);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = seg_min(lo[a]);
        hi[a] = seg_max(hi[a]);
    }
    sg = seg_max(sg);
    const float cx = 0.5f * (lo[0] + hi[0]);
    const float cy = 0.5f * (lo[1] + hi[1]);
    const float cz = 0.5f * (lo[2] + hi[2]);
    float d2 = 0.0f;
#pragma unroll
    for (int k = 0; k < kBoundPer; ++k) {
        const float dx = r[k].x - cx, dy = r[k].y - cy, dz = r[k].z - cz;
        d2 = fmaxf(d2, dx * dx + dy * dy + dz * dz);
    }
    d2 = seg_max(d2);
    if (ok && sl == 0) {
        const float ca = fabsf(cx) + fabsf(cy) + fabsf(cz);
        const float abs_m = 1e-4f * (ca + 1.0f);
        GroupBound b;
        b.c[0] = cx;
        b.c[1] = cy;
        b.c[2] = cz;
        b.h[0] = 0.5f * (hi[0] - lo[0]) * kCullMargin + abs_m;
        b.h[1] = 0.5f * (hi[1] - lo[1]) * kCullMargin + abs_m;
        b.h[2] = 0.5f * (hi[2] - lo[2]) * kCullMargin + abs_m;
        b.rm = sqrtf(d2) * kCullMargin + abs_m;
        b.sg = sg;
        gb[g] = b;
    }
}

// May any primitive of the wave's group be visible in this view?  The group's
// centres lie in the box c +- h and in the sphere |x - c| <= rm; the largest
// value of n . x over that set is at most n . c + min(|n_0| h_0 + |n_1| h_1 +
// |n_2| h_2, rm |n|).
__device__ inline float support(float n0, float n1, float n2, float nn, float hx, float hy, float hz, float rm)
{
    return fminf(fmaf(fabsf(n0), hx, fmaf(fabsf(n1), hy, fabsf(n2) * hz)), rm * nn);
}

template <class Rec>
__device__ inline bool cull_pass(const Rec& q, float cx, float cy, float cz, float hx, float hy, float hz,
                                 float rm, float sg, float ca, float z_near)
{
    const float depth = fmaf(q.nz[0], cx, fmaf(q.nz[1], cy, fmaf(q.nz[2], cz, q.nz[3])));
    bool ok = depth + support(q.nz[0], q.nz[1], q.nz[2], 1.0f, hx, hy, hz, rm) + 1e-4f * (ca + fabsf(q.nz[3])) >
              z_near;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const float val = fmaf(q.side[s][0], cx, fmaf(q.side[s][1], cy, fmaf(q.side[s][2], cz, q.side[s][3])));
        const float slack = 1e-4f * (q.nn[s] * (ca + 1.0f) + fabsf(q.side[s][3]));
        const float sup = support(q.side[s][0], q.side[s][1], q.side[s][2], q.nn[s], hx, hy, hz, rm);
        // no short circuit: all five tests and the loads of the record they
        // read are independent, so they issue together
        ok = ok & (val + sup + sg * q.kv3 + slack > 0.0f);
    }
    return ok;
}

// The staged evaluation constants of one view (five LDS float4 reads).
__device__ __forceinline__ void load_cam(const float4* __restrict__ r, CamEval& c)
{
    const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3], r4 = r[4];
    c.px[0] = r0.x; c.px[1] = r0.y; c.px[2] = r0.z; c.px[3] = r0.w;
    c.py[0] = r1.x; c.py[1] = r1.y; c.py[2] = r1.z; c.py[3] = r1.w;
    c.pz[0] = r2.x; c.pz[1] = r2.y; c.pz[2] = r2.z; c.pz[3] = r2.w;
    c.cx0 = r3.x; c.cx1 = r3.y; c.cy0 = r3.z; c.cy1 = r3.w;
    c.hw = r4.x; c.hh = r4.y; c.kvs = r4.z;
}

constexpr int kViewChunk = 256;   // views staged in LDS at a time (20 KB)
static_assert(kViewChunk % kViewBlock == 0, "chunks hold whole blocks");

// Bounds of view-loop group G (PPL groups of kGroup records), merged from
// the PPL bound records it covers: the union box, and a sphere about the
// union box's centre holding every member sphere (conservative).
template <int PPL>
__device__ inline GroupBound loop_group_bound(const GroupBound* __restrict__ gb, int ngroups64, int G)
{
    GroupBound b = gb[G * PPL];
    if (PPL == 1) return b;
    float lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = b.c[a] - b.h[a];
        hi[a] = b.c[a] + b.h[a];
    }
    float sg = b.sg;
#pragma unroll
    for (int k = 1; k < PPL; ++k) {
        if (G * PPL + k >= ngroups64) break;
        const GroupBound o = gb[G * PPL + k];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], o.c[a] - o.h[a]);
            hi[a] = fmaxf(hi[a], o.c[a] + o.h[a]);
        }
        sg = fmaxf(sg, o.sg);
    }
    GroupBound m;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m.c[a] = 0.5f * (lo[a] + hi[a]);
        m.h[a] = 0.5f * (hi[a] - lo[a]);
    }
    float rm = 0.0f;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        if (G * PPL + k >= ngroups64) break;
        const GroupBound o = gb[G * PPL + k];
        const float dx = o.c[0] - m.c[0], dy = o.c[1] - m.c[1], dz = o.c[2] - m.c[2];
        rm = fmaxf(rm, sqrtf(dx * dx + dy * dy + dz * dz) * kCullMargin + o.rm);
    }
    m.rm = rm;
    m.sg = sg;
    return m;
}

// Work class of a group that evaluates `cnt` of nv views: 0 for the most.
__device__ inline int work_class(uint32_t cnt, int nv)
{
    const int c = (int)(((uint64_t)cnt * kOrderBuckets) / (uint64_t)(nv + 1));
    return kOrderBuckets - 1 - min(c, kOrderBuckets - 1);
}

// Clears the pair counters when the view loop does not run (n = 0).
__global__ void views_init(unsigned long long* __restrict__ evaluated)
{
    if (threadIdx.x < 2 * kEvalSlots) evaluated[threadIdx.x] = 0ull;
}

// The views each view-loop group evaluates, as 64-bit masks.  Lane l of a
// block holds the bounds of group 64 b + l in registers; its 16 waves split
// the views into runs of 16, and every view's culling record is wave-uniform,
// so it comes in through scalar loads and no LDS traffic or cross-lane step
// is needed per test (the many short runs let the waves hide each other's
// load latency).  Each wave writes the 16-bit pieces of its runs (pieces past
// the last view are written as 0).  A view is dropped only when no point
// of the group's bounds can pass the near plane or one image edge even with
// the largest footprint any of its primitives can have.  Also counts each
// group's views into the block's work classes.
constexpr int kCullWaves = 16;
constexpr int kCullThreads = 64 * kCullWaves;
constexpr int kCullBlockGroups = 64;
constexpr int kCullRun = 16;   // views per run (a run's mask bits are stored as one piece)
using CullPiece = std::conditional_t<kCullRun == 16, uint16_t, uint32_t>;
static_assert(kCullRun == 8 * (int)sizeof(CullPiece), "one mask piece per run");

template <int PPL>
__global__ __launch_bounds__(kCullThreads) void cull_groups(const GroupBound* __restrict__ gb, int ngroups64, int ngroups,
                                                        const CullRec* __restrict__ culls, int nv, float z_near,
                                                        uint64_t* __restrict__ mask, uint32_t* __restrict__ counts,
                                                        uint32_t* __restrict__ aux,
                                                        unsigned long long* __restrict__ evaluated)
{
    __shared__ GroupBound sb[kCullBlockGroups];
    __shared__ uint32_t part[kCullWaves][kCullBlockGroups];
    __shared__ uint32_t hist[kOrderBuckets];
    // the class counts are cleared before this kernel (by camera_prep); the
    // cursors aux[0, kOrderBuckets) are used only by the kernels after it,
    // and the pair counters start from zero for the next view loop
    if (blockIdx.x == 0) {
        if (threadIdx.x < kOrderBuckets) aux[threadIdx.x] = 0u;
        if (evaluated && threadIdx.x < 2 * kEvalSlots) evaluated[threadIdx.x] = 0ull;
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int G = blockIdx.x * kCullBlockGroups + lane;
    const bool live = G < ngroups;
    if (wave == 0) {
        GroupBound z = {};
        sb[lane] = live ? loop_group_bound<PPL>(gb, ngroups64, G) : z;
    }
    if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = 0u;
    __syncthreads();
    const GroupBound g = sb[lane];
    const float ca = fabsf(g.c[0]) + fabsf(g.c[1]) + fabsf(g.c[2]);
    // a non-finite bound (non-finite input) disables culling for the group
    const bool no_cull = !(g.rm < INFINITY) || !(g.sg < INFINITY) || !(ca < INFINITY);
    const int nwords = (nv + 63) / 64;
    // little-endian pieces of the group's mask row (lanes past the last group
    // compute but never store)
    CullPiece* const row = reinterpret_cast<CullPiece*>(mask + (size_t)(live ? G : 0) * nwords);
    uint32_t cnt = 0;
    for (int r = wave; r < (64 / kCullRun) * nwords; r += kCullWaves) {
        const int v0 = r * kCullRun;
        const int vn = max(0, min(kCullRun, nv - v0));
        uint32_t m = 0u;
        for (int j = 0; j < vn; ++j) {
            const bool vis = no_cull | cull_pass(culls[v0 + j], g.c[0], g.c[1], g.c[2], g.h[0], g.h[1], g.h[2],
                                                 g.rm, g.sg, ca, z_near);
            m |= vis ? 1u << j : 0u;
        }
        if (live) row[r] = (CullPiece)m;
        cnt += (uint32_t)__popc(m);
    }
    part[wave][lane] = cnt;
    __syncthreads();
    if (wave == 0 && live) {
        uint32_t total = 0;
#pragma unroll
        for (int w = 0; w < kCullWaves; ++w) total += part[w][lane];
        counts[G] = total;
        atomicAdd(&hist[work_class(total, nv)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kOrderBuckets && hist[threadIdx.x])
        atomicAdd(&aux[kOrderBuckets * (1 + blockIdx.x % kOrderCopies) + threadIdx.x], hist[threadIdx.x]);
}

// Orders the view-loop groups by work class (most views first) so that the
// longest groups start early and none is left running alone at the end.
// Within a class the order is arbitrary: each group's result does not
// depend on when it runs.
__global__ __launch_bounds__(kBlock) void place_groups(const uint32_t* __restrict__ counts, int ngroups, int nv,
                                                         uint32_t* __restrict__ aux, int32_t* __restrict__ order)
{
    __shared__ uint32_t tot[kOrderBuckets], base[kOrderBuckets], cls[kOrderBuckets], off[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) {
        uint32_t t = 0;
        for (int k = 0; k < kOrderCopies; ++k) t += aux[kOrderBuckets * (1 + k) + threadIdx.x];
        tot[threadIdx.x] = t;
        cls[threadIdx.x] = 0u;
    }
    __syncthreads();
    if (threadIdx.x < kOrderBuckets) {
        uint32_t s = 0;
        for (int c = 0; c < (int)threadIdx.x; ++c) s += tot[c];
        base[threadIdx.x] = s;
    }
    __syncthreads();
    const int G = blockIdx.x * kBlock + threadIdx.x;
    int c = 0;
    uint32_t rank = 0;
    if (G < ngroups) {
        c = work_class(counts[G], nv);
        rank = atomicAdd(&cls[c], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kOrderBuckets && cls[threadIdx.x])
        off[threadIdx.x] = atomicAdd(&aux[threadIdx.x], cls[threadIdx.x]);
    __syncthreads();
    const uint32_t pos = base[c] + off[c] + rank;   // < ngroups: the classes partition the groups
    if (G < ngroups && pos < (uint32_t)ngroups) order[pos] = G;
}

// The view loop: wave w takes group order[w] (PPL kGroup-record groups;
// lane l holds records l, l + 64, ... of it) and evaluates every view its
// mask keeps, in increasing view order, for all its records; VPI = 2 takes
// two kept views per iteration (two independent evaluation chains to
// interleave; the sums still add the views in the same order).  A block is 1 to
// kMaxLoopWaves waves, which share one LDS copy of the camera table.
constexpr int kMaxLoopWaves = 8;
constexpr int kDefaultLoopWaves = 4;

template <int PROJ, int PPL, int VPI>
__global__ __launch_bounds__(64 * kMaxLoopWaves) void score_binned(const PrimRec* __restrict__ recs, int n,
                                                         const CamRec* __restrict__ cams,
                                                         const uint64_t* __restrict__ mask,
                                                         const int32_t* __restrict__ order, int ngroups, int nv,
                                                         float eta, float z_near, float* __restrict__ out,
                                                         unsigned long long* __restrict__ evaluated)
{
    const int lane = threadIdx.x & 63;
    // wave-uniform values (readfirstlane tells the compiler so: the mask
    // words then come in through scalar loads and the loop over their bits
    // runs on the scalar unit)
    const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const bool active = w < ngroups;   // waves past the last group still help load the camera table
    const int G = active ? min(max(__builtin_amdgcn_readfirstlane(order[w]), 0), ngroups - 1) : 0;
    const int g0 = G * kGroup * PPL;
    Prim p[PPL];
    float pre[PPL], smax[PPL], total[PPL];
    int idx[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int j = g0 + k * 64 + lane;
        const int jj = min(j, n - 1);   // lanes past the end repeat the last record
        const PrimRec r = recs[jj];
        p[k].mx = r.mu[0]; p[k].my = r.mu[1]; p[k].mz = r.mu[2];
        smax[k] = r.smax;
        p[k].L00 = r.L[0]; p[k].L01 = r.L[1]; p[k].L02 = r.L[2];
        p[k].L10 = r.L[3]; p[k].L11 = r.L[4]; p[k].L12 = r.L[5];
        p[k].L20 = r.L[6]; p[k].L21 = r.L[7]; p[k].L22 = r.L[8];
        p[k].S = 0.0f;
        total[k] = 0.0f;
        pre[k] = r.pre;
        idx[k] = (active && j < n) ? r.idx : -1;
    }
    const int nwords = (nv + 63) / 64;
    const uint64_t* gm = mask + (size_t)G * nwords;
    // the evaluation constants of up to kViewChunk views, loaded into LDS by
    // the whole block, so that every camera operand of the pair arithmetic
    // is a vector register (an instruction may read only one scalar register)
    __shared__ float4 table[kViewChunk * kStageVec];
    uint32_t n_eval = 0, n_screened = 0;   // kept views evaluated in full / screened out
    for (int c0 = 0; c0 < nv; c0 += kViewChunk) {
        const int cn = min(kViewChunk, nv - c0);
        __syncthreads();   // the previous chunk's reads are done
        for (int t = threadIdx.x; t < cn * kStageVec; t += blockDim.x)
            table[t] = reinterpret_cast<const float4*>(cams + c0 + t / kStageVec)[t % kStageVec];
        __syncthreads();
        for (int v0 = c0; v0 < c0 + cn; v0 += kViewBlock) {   // one mask word
            uint64_t m = active ? gm[v0 / 64] : 0ull;
            while (m != 0ull) {
                const int b = __builtin_ctzll(m);
                m &= m - 1ull;
                CamEval c;
                load_cam(table + (v0 - c0 + b) * kStageVec, c);
                // screen: when no record of the group can pass for this view,
                // all its terms are exactly +0 and the rest is skipped
                PairHead hd[PPL];
                bool may = false;
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    hd[k] = pair_head(c, p[k]);
                    may = may || pair_may_pass(hd[k], c.kvs, smax[k], z_near);
                }
                const bool live = __builtin_amdgcn_ballot_w64(may) != 0ull;
                if (VPI == 2 && m != 0ull) {
                    const int b2 = __builtin_ctzll(m);
                    m &= m - 1ull;
                    CamEval c2;
                    load_cam(table + (v0 - c0 + b2) * kStageVec, c2);
                    PairHead hd2[PPL];
                    bool may2 = false;
#pragma unroll
                    for (int k = 0; k < PPL; ++k) {
                        hd2[k] = pair_head(c2, p[k]);
                        may2 = may2 || pair_may_pass(hd2[k], c2.kvs, smax[k], z_near);
                    }
                    const bool live2 = __ballot(may2) != 0ull;
                    n_eval += (live ? 1u : 0u) + (live2 ? 1u : 0u);
                    n_screened += (live ? 0u : 1u) + (live2 ? 0u : 1u);
                    if (live && live2) {
#pragma unroll
                        for (int k = 0; k < PPL; ++k) {   // each record still adds its views in order
                            pair_tail<PROJ>(c, p[k], hd[k], eta, z_near);
                            pair_tail<PROJ>(c2, p[k], hd2[k], eta, z_near);
                        }
                    } else if (live) {
#pragma unroll
                        for (int k = 0; k < PPL; ++k) pair_tail<PROJ>(c, p[k], hd[k], eta, z_near);
                    } else if (live2) {
#pragma unroll
                        for (int k = 0; k < PPL; ++k) pair_tail<PROJ>(c2, p[k], hd2[k], eta, z_near);
                    }
                } else {
                    if (live) {
                        ++n_eval;
#pragma unroll
                        for (int k = 0; k < PPL; ++k) pair_tail<PROJ>(c, p[k], hd[k], eta, z_near);
                    } else {
                        ++n_screened;
                    }
                }
            }
            // the word's sum (its kept views, in order; the others add +0)
            // joins the total, as the direct path's block sums do
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                total[k] += p[k].S;
                p[k].S = 0.0f;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < PPL; ++k)
        if (idx[k] >= 0) out[idx[k]] = pre[k] * total[k] / (float)nv;
    if (evaluated && active && lane == 0) {
        const int valid = max(0, min(kGroup * PPL, n - g0));   // records of this group
        const int slot = G % kEvalSlots;   // spread: one address would serialise the waves
        atomicAdd(evaluated + slot, (unsigned long long)n_eval * (unsigned long long)valid);
        atomicAdd(evaluated + kEvalSlots + slot, (unsigned long long)n_screened * (unsigned long long)valid);
    }
}

// out[0]: pairs evaluated in full, out[1]: pairs screened out after their
// first step (the direct path evaluates every pair).
// The counters restart from zero for the next view loop.
__global__ void counter_store(unsigned long long* c, int64_t* out, int64_t direct_pairs)
{
    unsigned long long t = 0, sc = 0;
    for (int s = 0; s < kEvalSlots; ++s) {
        t += c[s];
        sc += c[kEvalSlots + s];
        c[s] = 0ull;
        c[kEvalSlots + s] = 0ull;
    }
    out[0] = direct_pairs >= 0 ? direct_pairs : (int64_t)t;
    out[1] = direct_pairs >= 0 ? 0 : (int64_t)sc;
}

template <int PROJ, int ST>
void prepare_mode(const void* planes, int64_t stride, int n, const refine_params& prm, const refine_stats_t* d_stats,
                  const Workspace& ws, hipStream_t stream)
{
    const int vis = prm.vis_mode == REFINE_VIS_ALPHA ? 1 : 0;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    const dim3 tiles((unsigned)num_tiles(n));
    hipLaunchKernelGGL(bin_hist<ST>, tiles, dim3(kBlock), 0, stream, planes, stride, n, d_stats, ws.cell_cnt);
    hipLaunchKernelGGL(bin_scan, dim3(1), dim3(kScanThreads), 0, stream, ws.cell_cnt, ws.cell_cur);
    hipLaunchKernelGGL(bin_rank<ST>, tiles, dim3(kBlock), 0, stream, planes, stride, n, d_stats, ws.cell_cur,
                       ws.dest);
    hipLaunchKernelGGL((bin_scatter<PROJ, ST>), grid, dim3(kBlock), 0, stream, planes, stride, n, d_stats, vis, ws.dest,
                       ws.recs);
    const int ng = (int)num_groups(n, kGroup);
    hipLaunchKernelGGL(group_bounds, dim3((unsigned)num_groups(ng, kBlock / kBoundLanes)), dim3(kBlock), 0, stream,
                       ws.recs, n, ws.gbound, ng);
}

int records_per_lane(const refine_params& prm) { return prm.records_per_lane > 0 ? prm.records_per_lane : kDefaultPPL; }

// The camera-set dependent stage of the binned path: each view-loop group's
// kept views (cull_groups) and the groups' order (place_groups).  Clears the
// pair counters of the next view loop.
void cull_and_order(int n, int nv, const refine_params& prm, const Workspace& ws, hipStream_t stream)
{
    const float zn = (float)prm.z_near;
    const int ppl = records_per_lane(prm);
    const int ng64 = (int)num_groups(n, kGroup);
    const int ng = (int)num_groups(n, kGroup * ppl);
    const unsigned gblocks = (unsigned)num_groups(ng, kBlock);
    const unsigned cblocks = (unsigned)num_groups(ng, kCullBlockGroups);
    if (ppl == 2)
        hipLaunchKernelGGL(cull_groups<2>, dim3(cblocks), dim3(kCullThreads), 0, stream, ws.gbound, ng64, ng, ws.culls,
                           nv, zn, ws.gmask, ws.gcount, ws.gaux, ws.evaluated);
    else
        hipLaunchKernelGGL(cull_groups<1>, dim3(cblocks), dim3(kCullThreads), 0, stream, ws.gbound, ng64, ng, ws.culls,
                           nv, zn, ws.gmask, ws.gcount, ws.gaux, ws.evaluated);
    hipLaunchKernelGGL(place_groups, dim3(gblocks), dim3(kBlock), 0, stream, ws.gcount, ng, nv, ws.gaux, ws.gorder);
}

template <int PROJ, int ST>
void views_mode(const void* planes, int64_t stride, int n, const refine_params& prm, const refine_stats_t* d_stats,
                float* d_scores, unsigned long long* evaluated, const Workspace& ws, int nv, bool binned,
                hipStream_t stream)
{
    const int vis = prm.vis_mode == REFINE_VIS_ALPHA ? 1 : 0;
    const float eta = (float)prm.eta, zn = (float)prm.z_near;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    if (binned) {
        const int ppl = records_per_lane(prm);
        const int ng = (int)num_groups(n, kGroup * ppl);
        const int waves = prm.waves_per_block > 0 ? prm.waves_per_block : kDefaultLoopWaves;
        const unsigned loop_blocks = (unsigned)num_groups(ng, waves);
        const int vpi = prm.views_per_iteration > 0 ? prm.views_per_iteration : kDefaultVPI;
        auto loop = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3(loop_blocks), dim3(64 * waves), 0, stream, ws.recs, n, ws.cams, ws.gmask,
                               ws.gorder, ng, nv, eta, zn, d_scores, evaluated);
        };
        if (ppl == 2)
            vpi == 2 ? loop(score_binned<PROJ, 2, 2>) : loop(score_binned<PROJ, 2, 1>);
        else
            vpi == 2 ? loop(score_binned<PROJ, 1, 2>) : loop(score_binned<PROJ, 1, 1>);
    } else {
        hipLaunchKernelGGL((score_direct<PROJ, ST>), grid, dim3(kBlock), 0, stream, planes, stride, n, ws.cams, nv,
                           d_stats, eta, zn, vis, d_scores);
    }
}


bool binned_path(const refine_params& prm, int64_t n)
{
    if (prm.score_kind == REFINE_SCORE_OPACITY) return false;   // no pairs to schedule
    return prm.score_path == REFINE_PATH_BINNED || (prm.score_path == REFINE_PATH_AUTO && n >= kBinnedMinPrims);
}

}  // namespace

// Calls f with the compile-time projection mode and storage format.
template <class F>
void dispatch_mode(int proj, int st, F&& f)
{
    auto by_storage = [&](auto proj_c) { with_storage(st, [&](auto st_c) { f(proj_c, st_c); }); };
    switch (proj) {
    case REFINE_PROJ_COV: by_storage(std::integral_constant<int, REFINE_PROJ_COV>{}); break;
    case REFINE_PROJ_DEPTH: by_storage(std::integral_constant<int, REFINE_PROJ_DEPTH>{}); break;
    default: by_storage(std::integral_constant<int, REFINE_PROJ_NONE>{}); break;
    }
}

hipError_t launch_score_prepare(const void* planes, int st, int64_t stride, int64_t n, const float* d_cams,
                                int32_t n_views, const refine_params& prm, const refine_stats_t* d_stats,
                                const Workspace& ws, hipStream_t stream)
{
    if (prm.score_kind == REFINE_SCORE_OPACITY) return hipSuccess;   // nothing depends on the cameras
    const int nv = views_of(prm, n_views);
    const bool binned = n > 0 && binned_path(prm, n);
    const int threads = binned ? (nv > kCells * kBinCopies ? nv : kCells * kBinCopies) : nv;
    hipLaunchKernelGGL(camera_prep, dim3((threads + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, d_cams, n_views, nv,
                       (float)prm.clamp_k, ws.cams, ws.culls, binned ? ws.cell_cnt : nullptr,
                       binned ? ws.gaux : nullptr);
    if (!binned) return hipGetLastError();
    dispatch_mode(prm.proj_mode, st, [&](auto proj_c, auto st_c) {
        prepare_mode<decltype(proj_c)::value, decltype(st_c)::value>(planes, stride, (int)n, prm, d_stats, ws, stream);
    });
    cull_and_order((int)n, nv, prm, ws, stream);
    return hipGetLastError();
}

hipError_t launch_score_batch(const BatchJob* d_jobs, int n_jobs, int total_blocks, const refine_params& prm,
                              hipStream_t stream)
{
    const int vis = prm.vis_mode == REFINE_VIS_ALPHA ? 1 : 0;
    const float eta = (float)prm.eta, zn = (float)prm.z_near;
    if (prm.score_kind == REFINE_SCORE_OPACITY) {
        hipLaunchKernelGGL(score_opacity_batch, dim3(total_blocks), dim3(kBlock), 0, stream, d_jobs, n_jobs);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(camera_prep_batch, dim3(n_jobs), dim3(kBlock), 0, stream, d_jobs, (float)prm.clamp_k);
    switch (prm.proj_mode) {
    case REFINE_PROJ_COV:
        hipLaunchKernelGGL((score_direct_batch<REFINE_PROJ_COV>), dim3(total_blocks), dim3(kBlock), 0, stream, d_jobs,
                           n_jobs, eta, zn, vis);
        break;
    case REFINE_PROJ_DEPTH:
        hipLaunchKernelGGL((score_direct_batch<REFINE_PROJ_DEPTH>), dim3(total_blocks), dim3(kBlock), 0, stream,
                           d_jobs, n_jobs, eta, zn, vis);
        break;
    default:
        hipLaunchKernelGGL((score_direct_batch<REFINE_PROJ_NONE>), dim3(total_blocks), dim3(kBlock), 0, stream,
                           d_jobs, n_jobs, eta, zn, vis);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_score_cameras(const float* d_cams, int32_t n_views, int64_t n, const refine_params& prm,
                                const Workspace& ws, hipStream_t stream)
{
    if (prm.score_kind == REFINE_SCORE_OPACITY) return hipSuccess;   // nothing depends on the cameras
    const int nv = views_of(prm, n_views);
    const bool binned = n > 0 && binned_path(prm, n);
    const int threads = nv > kOrderBuckets * kOrderCopies ? nv : kOrderBuckets * kOrderCopies;
    hipLaunchKernelGGL(camera_prep, dim3((threads + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, d_cams, n_views, nv,
                       (float)prm.clamp_k, ws.cams, ws.culls, nullptr, binned ? ws.gaux : nullptr);
    if (binned) cull_and_order((int)n, nv, prm, ws, stream);
    return hipGetLastError();
}

hipError_t launch_score_views(const void* planes, int st, int64_t stride, int64_t n, int32_t n_views,
                              const refine_params& prm, const refine_stats_t* d_stats, float* d_scores,
                              int64_t* d_evaluated, const Workspace& ws, hipStream_t stream)
{
    const int nv = views_of(prm, n_views);
    const bool binned = binned_path(prm, n);
    unsigned long long* counter = (d_evaluated && binned) ? ws.evaluated : nullptr;
    if (binned && n == 0 && counter)   // no culling stage has cleared the pair counters
        hipLaunchKernelGGL(views_init, dim3(1), dim3(2 * kEvalSlots), 0, stream, counter);
    if (prm.score_kind == REFINE_SCORE_OPACITY) {
        if (n > 0) {
            const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
            with_storage(st, [&](auto st_c) {
                hipLaunchKernelGGL(score_opacity<decltype(st_c)::value>, grid, dim3(kBlock), 0, stream, planes, stride,
                                   (int)n, d_scores);
            });
        }
        if (d_evaluated)   // no pairs are evaluated
            hipLaunchKernelGGL(counter_store, dim3(1), dim3(1), 0, stream, ws.evaluated, d_evaluated, (int64_t)0);
        return hipGetLastError();
    }
    if (n > 0)
        dispatch_mode(prm.proj_mode, st, [&](auto proj_c, auto st_c) {
            views_mode<decltype(proj_c)::value, decltype(st_c)::value>(planes, stride, (int)n, prm, d_stats, d_scores,
                                                                       counter, ws, nv, binned, stream);
        });
    if (d_evaluated)
        hipLaunchKernelGGL(counter_store, dim3(1), dim3(1), 0, stream, ws.evaluated, d_evaluated,
                           binned ? (int64_t)-1 : n * (int64_t)nv);
    return hipGetLastError();
}

}  // namespace refine
