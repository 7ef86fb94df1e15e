// C ABI of the REFINE library: argument validation (before any HIP call),
// workspace layout and dispatch to the kernel launchers.
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "refine_internal.hpp"

namespace refine {

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// the Python binding mirrors these layouts (tests/test_abi.py checks the same sizes)
static_assert(sizeof(refine_scene) == 32, "refine_scene layout");
static_assert(sizeof(refine_params) == 88, "refine_params layout");
static_assert(sizeof(refine_stats_t) == 96, "refine_stats_t layout");

bool finite(double x) { return std::isfinite(x); }

bool known_dtype(int32_t d) { return d == REFINE_F32 || d == REFINE_BF16 || d == REFINE_F16; }

// Storage format of a scene (call after check_scene succeeded).
int storage_of(const refine_scene* s)
{
    return s->dtype == REFINE_F32 ? kStoreF32 : (s->dtype == REFINE_BF16 ? kStoreBF16F16 : kStoreF16);
}

refine_status check_scene(const refine_scene* s)
{
    if (!s) return REFINE_E_INVALID;
    if (s->n < 0 || s->stride < 0 || s->stride < s->n) return REFINE_E_INVALID;
    if (!known_dtype(s->dtype) || !known_dtype(s->sh_dtype)) return REFINE_E_INVALID;
    const bool f32 = s->dtype == REFINE_F32 && s->sh_dtype == REFINE_F32;
    const bool mixed = s->dtype == REFINE_BF16 && s->sh_dtype == REFINE_F16;
    const bool half = s->dtype == REFINE_F16 && s->sh_dtype == REFINE_F16;
    if (!f32 && !mixed && !half) return REFINE_E_UNSUPPORTED;
    if (s->n > (int64_t)std::numeric_limits<int32_t>::max()) return REFINE_E_UNSUPPORTED;
    if (s->stride > std::numeric_limits<int64_t>::max() / (kPlanes * 4)) return REFINE_E_INVALID;
    if (s->n > 0 && !s->planes) return REFINE_E_INVALID;
    return REFINE_OK;
}

refine_status check_params(const refine_params* p)
{
    if (!p) return REFINE_E_INVALID;
    if (!finite(p->eta) || p->eta <= 0.0) return REFINE_E_INVALID;
    if (!finite(p->z_near) || p->z_near < 0.0) return REFINE_E_INVALID;
    if (!finite(p->clamp_k) || p->clamp_k <= 0.0) return REFINE_E_INVALID;
    if (!finite(p->e_col) || p->e_col == 0.0) return REFINE_E_INVALID;
    if (!finite(p->e_opa) || p->e_opa == 0.0) return REFINE_E_INVALID;
    if (!finite(p->e_lngem) || p->e_lngem == 0.0) return REFINE_E_INVALID;
    if (p->proj_mode < REFINE_PROJ_COV || p->proj_mode > REFINE_PROJ_NONE) return REFINE_E_INVALID;
    if (p->vis_mode < REFINE_VIS_ALPHA || p->vis_mode > REFINE_VIS_NONE) return REFINE_E_INVALID;
    if (p->equal_lambda != 0 && p->equal_lambda != 1) return REFINE_E_INVALID;
    if (p->n_sub_views < 0) return REFINE_E_INVALID;
    if (p->score_path < REFINE_PATH_AUTO || p->score_path > REFINE_PATH_BINNED) return REFINE_E_INVALID;
    if (p->records_per_lane < 0 || p->records_per_lane > 2) return REFINE_E_INVALID;
    if (p->views_per_iteration < 0 || p->views_per_iteration > 2) return REFINE_E_INVALID;
    if (p->score_kind != REFINE_SCORE_IMPORTANCE && p->score_kind != REFINE_SCORE_OPACITY) return REFINE_E_INVALID;
    const int32_t w = p->waves_per_block;
    if (w != 0 && w != 1 && w != 2 && w != 4 && w != 8) return REFINE_E_INVALID;
    return REFINE_OK;
}

constexpr int32_t kMaxViews = 1 << 20;

refine_status check_workspace(int64_t n, int32_t n_views, bool score, const void* ws, size_t ws_bytes,
                              Workspace* out)
{
    const size_t need = workspace_layout(n, n_views, score, nullptr, nullptr);
    if (ws_bytes < need || (need > 0 && !ws)) return REFINE_E_WORKSPACE;
    workspace_layout(n, n_views, score, const_cast<void*>(ws), out);
    return REFINE_OK;
}

}  // namespace

size_t workspace_layout(int64_t n, int32_t n_views, bool score, void* base, Workspace* ws)
{
    const size_t nt = (size_t)(num_tiles(n) > 0 ? num_tiles(n) : 1);
    const size_t nv = (size_t)(n_views > 0 ? n_views : 0);
    size_t off = 0;
    const size_t o_sel = off;   off += align_up(sizeof(SelectState) * kSelectStates);
    const size_t o_hist = off;  off += align_up(sizeof(uint32_t) * kSelectHistWords);
    const size_t o_part = off;  off += align_up(sizeof(double) * kStatSlots * nt);
    const size_t o_cnt = off;   off += align_up(sizeof(uint32_t) * nt);
    const size_t o_toff = off;  off += align_up(sizeof(uint32_t) * nt);
    const bool rows = num_tiles(n) <= kPrefixTilesMax;
    const size_t o_rows = off;  off += rows ? align_up(sizeof(uint32_t) * kSelectLastBins * nt) : 0;
    // sections only refine_score uses come after, so the other calls need a
    // prefix only; the camera tables come last, so that no other section's
    // place depends on the number of views (a workspace prepared for one
    // camera set keeps its binned scene when the tables are rebuilt)
    const size_t o_eval = off;  off += score ? align_up(sizeof(unsigned long long) * 2 * kEvalSlots) : 0;
    const size_t o_ccnt = off;  off += score ? align_up(sizeof(uint32_t) * kCells * kBinCopies) : 0;
    const size_t o_ccur = off;  off += score ? align_up(sizeof(uint32_t) * kCells * kBinCopies) : 0;
    const size_t o_dest = off;  off += score ? align_up(sizeof(uint32_t) * (size_t)n) : 0;
    const size_t ng = (size_t)num_groups(n, kGroup);
    const size_t o_recs = off;  off += score ? align_up(sizeof(PrimRec) * (size_t)n) : 0;
    const size_t o_gbnd = off;  off += score ? align_up(sizeof(GroupBound) * ng) : 0;
    const size_t o_gord = off;  off += score ? align_up(sizeof(int32_t) * ng) : 0;
    const size_t o_gcnt = off;  off += score ? align_up(sizeof(uint32_t) * ng) : 0;
    const size_t o_gaux = off;  off += score ? align_up(sizeof(uint32_t) * kOrderAuxWords) : 0;
    const size_t o_cams = off;  off += score ? align_up(sizeof(CamRec) * nv) : 0;
    const size_t o_cull = off;  off += score ? align_up(sizeof(CullRec) * nv) : 0;
    const size_t o_gmsk = off;  off += score ? align_up(sizeof(uint64_t) * ng * ((nv + 63) / 64)) : 0;
    if (base && ws) {
        char* b = static_cast<char*>(base);
        ws->sel = reinterpret_cast<SelectState*>(b + o_sel);
        ws->hist = reinterpret_cast<uint32_t*>(b + o_hist);
        ws->stat_part = reinterpret_cast<double*>(b + o_part);
        ws->tile_cnt = reinterpret_cast<uint32_t*>(b + o_cnt);
        ws->tile_off = reinterpret_cast<uint32_t*>(b + o_toff);
        ws->tile_rows = rows ? reinterpret_cast<uint32_t*>(b + o_rows) : nullptr;
        ws->cams = score ? reinterpret_cast<CamRec*>(b + o_cams) : nullptr;
        ws->culls = score ? reinterpret_cast<CullRec*>(b + o_cull) : nullptr;
        ws->cell_cnt = score ? reinterpret_cast<uint32_t*>(b + o_ccnt) : nullptr;
        ws->cell_cur = score ? reinterpret_cast<uint32_t*>(b + o_ccur) : nullptr;
        ws->dest = score ? reinterpret_cast<uint32_t*>(b + o_dest) : nullptr;
        ws->recs = score ? reinterpret_cast<PrimRec*>(b + o_recs) : nullptr;
        ws->gbound = score ? reinterpret_cast<GroupBound*>(b + o_gbnd) : nullptr;
        ws->gorder = score ? reinterpret_cast<int32_t*>(b + o_gord) : nullptr;
        ws->gcount = score ? reinterpret_cast<uint32_t*>(b + o_gcnt) : nullptr;
        ws->gaux = score ? reinterpret_cast<uint32_t*>(b + o_gaux) : nullptr;
        ws->gmask = score ? reinterpret_cast<uint64_t*>(b + o_gmsk) : nullptr;
        ws->evaluated = score ? reinterpret_cast<unsigned long long*>(b + o_eval) : nullptr;
    }
    return off;
}

}  // namespace refine

using namespace refine;

namespace {

constexpr int32_t kMaxBatchJobs = 4096;

// Bytes of one job's workspace slice: selection state and histograms, tile
// partials, counts and last-pass rows, camera records.
size_t batch_job_bytes(int64_t n, int32_t nv)
{
    const size_t nt = (size_t)num_tiles(n);
    return align_up(sizeof(SelectState) * kSelectStates) + align_up(sizeof(uint32_t) * kSelectHistWords) +
           align_up(sizeof(double) * kStatSlots * nt) + align_up(sizeof(uint32_t) * nt) +
           align_up(sizeof(uint32_t) * kSelectLastBins * nt) + align_up(sizeof(CamRec) * nv);
}

refine_status check_batch_job(const refine_prune_job& j)
{
    refine_status s = check_scene(&j.scene);
    if (s != REFINE_OK) return s;
    if ((s = check_scene(&j.out)) != REFINE_OK) return s;
    if (j.scene.n < 1 || j.reserved != 0) return REFINE_E_INVALID;
    if (num_tiles(j.scene.n) > kPrefixTilesMax) return REFINE_E_UNSUPPORTED;
    if (j.scene.dtype != j.out.dtype || j.scene.sh_dtype != j.out.sh_dtype) return REFINE_E_INVALID;
    if (!j.d_cams || j.n_views < 1) return REFINE_E_INVALID;
    if (j.n_views > kMaxViews) return REFINE_E_UNSUPPORTED;
    if (refine_prune_count(j.scene.n, j.ratio) < 0) return REFINE_E_INVALID;
    if (!j.d_stats || !j.d_scores || !j.d_keep) return REFINE_E_INVALID;
    const size_t es = storage_bytes(storage_of(&j.scene));
    if (j.out.n > 0) {
        const char* a0 = static_cast<const char*>(j.scene.planes);
        const char* a1 = a0 + (size_t)kPlanes * (size_t)j.scene.stride * es;
        const char* b0 = static_cast<const char*>(j.out.planes);
        const char* b1 = b0 + (size_t)kPlanes * (size_t)j.out.stride * es;
        if (a0 < b1 && b0 < a1) return REFINE_E_INVALID;
    }
    return REFINE_OK;
}

refine_status batch_size(const refine_prune_job* jobs, int32_t n_jobs, const refine_params* params, size_t* bytes)
{
    if (!jobs || !bytes || n_jobs < 1) return REFINE_E_INVALID;
    if (n_jobs > kMaxBatchJobs) return REFINE_E_UNSUPPORTED;
    refine_status s = check_params(params);
    if (s != REFINE_OK) return s;
    size_t total = align_up(sizeof(BatchJob) * (size_t)n_jobs);
    for (int32_t k = 0; k < n_jobs; ++k) {
        if ((s = check_batch_job(jobs[k])) != REFINE_OK) return s;
        total += batch_job_bytes(jobs[k].scene.n, views_of(*params, jobs[k].n_views));
    }
    *bytes = total;
    return REFINE_OK;
}

}  // namespace

extern "C" {

const char* refine_version(void) { return "refine-mi355x 0.1.0 (gfx950, HIP)"; }

const char* refine_status_string(int32_t status)
{
    switch (status) {
    case REFINE_OK: return "REFINE_OK";
    case REFINE_E_INVALID: return "REFINE_E_INVALID: invalid argument";
    case REFINE_E_UNSUPPORTED: return "REFINE_E_UNSUPPORTED: well-formed but outside what the library handles";
    case REFINE_E_WORKSPACE: return "REFINE_E_WORKSPACE: workspace missing or too small";
    case REFINE_E_HIP: return "REFINE_E_HIP: HIP launch failed";
    default: return "unknown refine_status";
    }
}

void refine_params_default(refine_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->eta = 0.05;
    p->z_near = 0.2;
    p->clamp_k = 1.3;
    p->e_col = 8.892106e-3;
    p->e_opa = 0.1767277;
    p->e_lngem = -0.4890595;
    p->proj_mode = REFINE_PROJ_COV;
    p->vis_mode = REFINE_VIS_ALPHA;
    p->equal_lambda = 0;
    p->n_sub_views = 0;
    p->score_kind = REFINE_SCORE_IMPORTANCE;
}

int64_t refine_prune_count(int64_t n, double ratio)
{
    if (n < 0 || !std::isfinite(ratio) || !(ratio > 0.0) || !(ratio < 1.0)) return -1;
    double k = std::floor(ratio * (double)n + 0.5);
    if (k < 0.0) k = 0.0;
    if (k > (double)n) k = (double)n;
    return (int64_t)k;
}

refine_status refine_workspace_size(int64_t n, int32_t n_views, size_t* bytes)
{
    if (!bytes || n < 0 || n_views < 0) return REFINE_E_INVALID;
    if (n > (int64_t)std::numeric_limits<int32_t>::max() || n_views > kMaxViews) return REFINE_E_UNSUPPORTED;
    *bytes = workspace_layout(n, n_views, n_views > 0, nullptr, nullptr);
    return REFINE_OK;
}

refine_status refine_stats(const refine_scene* scene, const refine_params* params, refine_stats_t* d_stats,
                           void* d_ws, size_t ws_bytes, void* stream)
{
    refine_status s = check_scene(scene);
    if (s != REFINE_OK) return s;
    if ((s = check_params(params)) != REFINE_OK) return s;
    if (!d_stats) return REFINE_E_INVALID;
    Workspace ws;
    if ((s = check_workspace(scene->n, 0, false, d_ws, ws_bytes, &ws)) != REFINE_OK) return s;
    const hipError_t e = launch_stats(scene->planes, storage_of(scene), scene->stride, scene->n, *params, d_stats,
                                      ws, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? REFINE_OK : REFINE_E_HIP;
}

refine_status refine_stats_noalloc(const refine_scene* scene, const refine_params* params, refine_stats_t* d_stats,
                                   void* stream)
{
    refine_status s = check_scene(scene);
    if (s != REFINE_OK) return s;
    if ((s = check_params(params)) != REFINE_OK) return s;
    if (!d_stats) return REFINE_E_INVALID;
    if (scene->n > (int64_t)REFINE_STATS_NOALLOC_MAX_N) return REFINE_E_UNSUPPORTED;
    double* part = nullptr;
    if (stats_scratch(&part) != hipSuccess) return REFINE_E_HIP;
    Workspace ws = {};
    ws.stat_part = part;   // the only workspace section the statistics kernels use
    const hipError_t e = launch_stats(scene->planes, storage_of(scene), scene->stride, scene->n, *params, d_stats,
                                      ws, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? REFINE_OK : REFINE_E_HIP;
}

namespace {

refine_status check_score_args(const refine_scene* scene, int32_t n_views, const refine_params* params,
                               const refine_stats_t* d_stats)
{
    refine_status s = check_scene(scene);
    if (s != REFINE_OK) return s;
    if ((s = check_params(params)) != REFINE_OK) return s;
    if (n_views < 1 || !d_stats) return REFINE_E_INVALID;
    if (n_views > kMaxViews) return REFINE_E_UNSUPPORTED;
    return REFINE_OK;
}

}  // namespace

refine_status refine_score_prepare(const refine_scene* scene, const float* d_cams, int32_t n_views,
                                   const refine_params* params, const refine_stats_t* d_stats, void* d_ws,
                                   size_t ws_bytes, void* stream)
{
    refine_status s = check_score_args(scene, n_views, params, d_stats);
    if (s != REFINE_OK) return s;
    if (!d_cams) return REFINE_E_INVALID;
    Workspace ws;
    if ((s = check_workspace(scene->n, n_views, true, d_ws, ws_bytes, &ws)) != REFINE_OK) return s;
    const hipError_t e = launch_score_prepare(scene->planes, storage_of(scene), scene->stride, scene->n, d_cams,
                                              n_views, *params, d_stats, ws, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? REFINE_OK : REFINE_E_HIP;
}

refine_status refine_score_cameras(const refine_scene* scene, const float* d_cams, int32_t n_views,
                                   const refine_params* params, void* d_ws, size_t ws_bytes, void* stream)
{
    refine_status s = check_scene(scene);
    if (s != REFINE_OK) return s;
    if ((s = check_params(params)) != REFINE_OK) return s;
    if (n_views < 1 || !d_cams) return REFINE_E_INVALID;
    if (n_views > kMaxViews) return REFINE_E_UNSUPPORTED;
    Workspace ws;
    if ((s = check_workspace(scene->n, n_views, true, d_ws, ws_bytes, &ws)) != REFINE_OK) return s;
    const hipError_t e = launch_score_cameras(d_cams, n_views, scene->n, *params, ws, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? REFINE_OK : REFINE_E_HIP;
}

refine_status refine_score_views(const refine_scene* scene, int32_t n_views, const refine_params* params,
                                 const refine_stats_t* d_stats, float* d_scores, int64_t* d_evaluated, void* d_ws,
                                 size_t ws_bytes, void* stream)
{
    refine_status s = check_score_args(scene, n_views, params, d_stats);
    if (s != REFINE_OK) return s;
    if (scene->n > 0 && !d_scores) return REFINE_E_INVALID;
    Workspace ws;
    if ((s = check_workspace(scene->n, n_views, true, d_ws, ws_bytes, &ws)) != REFINE_OK) return s;
    const hipError_t e = launch_score_views(scene->planes, storage_of(scene), scene->stride, scene->n, n_views,
                                            *params, d_stats, d_scores, d_evaluated, ws,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? REFINE_OK : REFINE_E_HIP;
}

refine_status refine_score(const refine_scene* scene, const float* d_cams, int32_t n_views,
                           const refine_params* params, const refine_stats_t* d_stats, float* d_scores,
                           void* d_ws, size_t ws_bytes, void* stream)
{
    refine_status s = check_score_args(scene, n_views, params, d_stats);
    if (s != REFINE_OK) return s;
    if (!d_cams || (scene->n > 0 && !d_scores)) return REFINE_E_INVALID;
    s = refine_score_prepare(scene, d_cams, n_views, params, d_stats, d_ws, ws_bytes, stream);
    if (s != REFINE_OK) return s;
    return refine_score_views(scene, n_views, params, d_stats, d_scores, nullptr, d_ws, ws_bytes, stream);
}

refine_status refine_select(const float* d_scores, int64_t n, double ratio, int64_t n_prune_override,
                            uint8_t* d_keep, int64_t* d_n_keep, uint32_t* d_threshold, void* d_ws,
                            size_t ws_bytes, void* stream)
{
    if (n < 0) return REFINE_E_INVALID;
    if (n > (int64_t)std::numeric_limits<int32_t>::max()) return REFINE_E_UNSUPPORTED;
    if (n > 0 && (!d_scores || !d_keep)) return REFINE_E_INVALID;
    int64_t n_prune;
    if (n_prune_override >= 0) {
        if (n_prune_override > n) return REFINE_E_INVALID;
        n_prune = n_prune_override;
    } else {
        n_prune = refine_prune_count(n, ratio);
        if (n_prune < 0) return REFINE_E_INVALID;
    }
    Workspace ws;
    refine_status s = check_workspace(n, 0, false, d_ws, ws_bytes, &ws);
    if (s != REFINE_OK) return s;
    const hipError_t e = launch_select(d_scores, n, n_prune, d_keep, d_n_keep, d_threshold, ws,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? REFINE_OK : REFINE_E_HIP;
}

refine_status refine_compact(const refine_scene* in, const uint8_t* d_keep, const refine_scene* out,
                             int32_t* d_index_map, int64_t* d_n_out, void* d_ws, size_t ws_bytes, void* stream)
{
    refine_status s = check_scene(in);
    if (s != REFINE_OK) return s;
    if ((s = check_scene(out)) != REFINE_OK) return s;
    if (in->dtype != out->dtype || in->sh_dtype != out->sh_dtype) return REFINE_E_INVALID;
    if (in->n > 0 && !d_keep) return REFINE_E_INVALID;
    const size_t es = storage_bytes(storage_of(in));
    if (in->n > 0 && out->n > 0) {
        const char* a0 = static_cast<const char*>(in->planes);
        const char* a1 = a0 + (size_t)kPlanes * (size_t)in->stride * es;
        const char* b0 = static_cast<const char*>(out->planes);
        const char* b1 = b0 + (size_t)kPlanes * (size_t)out->stride * es;
        if (a0 < b1 && b0 < a1) return REFINE_E_INVALID;
    }
    Workspace ws;
    if ((s = check_workspace(in->n, 0, false, d_ws, ws_bytes, &ws)) != REFINE_OK) return s;
    const hipError_t e = launch_compact(in->planes, storage_of(in), in->stride, in->n, d_keep, out->planes,
                                        out->stride, out->n, d_index_map, d_n_out, ws,
                                        static_cast<hipStream_t>(stream));
    return e == hipSuccess ? REFINE_OK : REFINE_E_HIP;
}

refine_status refine_prune_batch_workspace_size(const refine_prune_job* jobs, int32_t n_jobs,
                                                const refine_params* params, size_t* bytes)
{
    return batch_size(jobs, n_jobs, params, bytes);
}

static_assert(sizeof(BatchJob) <= REFINE_BATCH_STAGING_BYTES_PER_JOB, "staging bytes per job");
static_assert(alignof(BatchJob) == 8, "the staging alignment the header states");

refine_status refine_prune_batch(const refine_prune_job* jobs, int32_t n_jobs, const refine_params* params,
                                 void* d_ws, size_t ws_bytes, void* h_staging, size_t staging_bytes, void* stream)
{
    size_t need = 0;
    refine_status s = batch_size(jobs, n_jobs, params, &need);
    if (s != REFINE_OK) return s;
    if (!d_ws || ws_bytes < need) return REFINE_E_WORKSPACE;
    if (h_staging && staging_bytes < (size_t)n_jobs * REFINE_BATCH_STAGING_BYTES_PER_JOB) return REFINE_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(h_staging) % alignof(BatchJob)) return REFINE_E_INVALID;
    char* base = static_cast<char*>(d_ws);
    BatchJob* d_table = reinterpret_cast<BatchJob*>(base);
    size_t off = align_up(sizeof(BatchJob) * (size_t)n_jobs);
    // the table is built in the caller's pinned buffer when there is one (an
    // asynchronous copy), else in pageable memory (HIP takes the copy before
    // hipMemcpyAsync returns)
    std::vector<BatchJob> pageable(h_staging ? 0 : (size_t)n_jobs);
    BatchJob* table = h_staging ? static_cast<BatchJob*>(h_staging) : pageable.data();
    int64_t tiles = 0, blocks = 0;
    for (int32_t k = 0; k < n_jobs; ++k) {
        const refine_prune_job& j = jobs[k];
        BatchJob& b = table[(size_t)k];
        std::memset(&b, 0, sizeof(b));
        const int64_t n = j.scene.n;
        const int nv = views_of(*params, j.n_views);
        const int st = storage_of(&j.scene);
        const size_t es = storage_bytes(st);
        b.planes = j.scene.planes;
        b.stride = j.scene.stride;
        b.n = (int32_t)n;
        b.st = st;
        b.cams = j.d_cams;
        b.n_views = j.n_views;
        b.nv = nv;
        b.stats = j.d_stats;
        b.scores = j.d_scores;
        b.keep = j.d_keep;
        b.n_prune = refine_prune_count(n, j.ratio);
        b.n_keep_out = j.d_n_keep;
        b.out = j.out.planes;
        b.out_stride = j.out.stride;
        b.capacity = j.out.n;
        b.index_map = j.d_index_map;
        b.n_out = j.d_n_out;
        const size_t nt = (size_t)num_tiles(n);
        b.sel = reinterpret_cast<SelectState*>(base + off);
        off += align_up(sizeof(SelectState) * kSelectStates);
        b.hist = reinterpret_cast<uint32_t*>(base + off);
        off += align_up(sizeof(uint32_t) * kSelectHistWords);
        b.stat_part = reinterpret_cast<double*>(base + off);
        off += align_up(sizeof(double) * kStatSlots * nt);
        b.tile_cnt = reinterpret_cast<uint32_t*>(base + off);
        off += align_up(sizeof(uint32_t) * nt);
        b.tile_rows = reinterpret_cast<uint32_t*>(base + off);
        off += align_up(sizeof(uint32_t) * kSelectLastBins * nt);
        b.cam_rec = reinterpret_cast<CamRec*>(base + off);
        off += align_up(sizeof(CamRec) * (size_t)nv);
        b.tile0 = (int32_t)tiles;
        b.block0 = (int32_t)blocks;
        tiles += (int64_t)nt;
        blocks += (n + kBlock - 1) / kBlock;
        b.vec_compact = (reinterpret_cast<uintptr_t>(j.scene.planes) % 16 == 0) &&
                        (((size_t)j.scene.stride * es) % 16 == 0) &&
                        (reinterpret_cast<uintptr_t>(j.d_keep) % 4 == 0);
        b.pair_store = (reinterpret_cast<uintptr_t>(j.out.planes) % 4 == 0) && (j.out.stride % 2 == 0);
        b.vec_stats = (reinterpret_cast<uintptr_t>(j.scene.planes) % 16 == 0) &&
                      (((size_t)j.scene.stride * es) % 16 == 0);
    }
    if (tiles > INT32_MAX || blocks > INT32_MAX) return REFINE_E_UNSUPPORTED;
    hipStream_t strm = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(d_table, table, sizeof(BatchJob) * (size_t)n_jobs, hipMemcpyHostToDevice, strm) != hipSuccess)
        return REFINE_E_HIP;
    if (launch_stats_batch(d_table, n_jobs, (int)tiles, *params, strm) != hipSuccess) return REFINE_E_HIP;
    if (launch_score_batch(d_table, n_jobs, (int)blocks, *params, strm) != hipSuccess) return REFINE_E_HIP;
    if (launch_select_batch(d_table, n_jobs, (int)tiles, strm) != hipSuccess) return REFINE_E_HIP;
    if (launch_compact_batch(d_table, n_jobs, (int)tiles, strm) != hipSuccess) return REFINE_E_HIP;
    return REFINE_OK;
}

}  // extern "C"
