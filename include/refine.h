/*
 * refine.h -- C ABI of the REFINE importance-scoring and pruning library for
 * AMD Instinct MI355X (gfx950).
 *
 * REFINE (arXiv 2606.09074) scores every Gaussian primitive of a trained 3D
 * Gaussian Splatting scene without rendering: a diagonal, analytically
 * approximated Hessian weight per attribute group (Sec. 3.2, Eq. 7-20),
 * averaged over a set of cameras, is coupled with the primitive's attribute
 * magnitudes; the bottom beta*N primitives are then removed (Sec. 3.3).
 *
 * Conventions shared by every call below:
 *  - All pointers named d_* and the planes/camera arrays are DEVICE memory,
 *    allocated and owned by the caller; the library never allocates, frees or
 *    synchronises.  Every call only enqueues work on `stream` (a hipStream_t;
 *    NULL = the default stream) and returns.
 *  - Argument validation happens on the host before any HIP call; a failed
 *    validation returns REFINE_E_INVALID / REFINE_E_UNSUPPORTED /
 *    REFINE_E_WORKSPACE and enqueues nothing.  A failed kernel launch returns
 *    REFINE_E_HIP.  Data-dependent conditions are reported in device memory
 *    (refine_stats_t.n_nonfinite, the *d_n_out of refine_compact).
 *  - One workspace of refine_workspace_size(n, n_views) bytes serves every
 *    call for scenes of up to n primitives and n_views cameras.  Calls that
 *    share a workspace must be ordered (same stream); calls on different
 *    streams need different workspaces.
 *  - No global mutable state: calls are re-entrant across streams.  The one
 *    exception is refine_stats_noalloc, whose fixed per-GPU array is shared
 *    by all its calls on that GPU (see there).
 */
#ifndef REFINE_H
#define REFINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    REFINE_OK = 0,
    REFINE_E_INVALID = -1,      /* a null pointer, negative size, out-of-domain value */
    REFINE_E_UNSUPPORTED = -2,  /* well-formed but outside what the library handles */
    REFINE_E_WORKSPACE = -3,    /* workspace missing or smaller than required */
    REFINE_E_HIP = -4           /* a HIP launch failed */
} refine_status;

/* Storage type of scene planes.  Arithmetic is FP32 whatever the storage:
 * BF16 and FP16 values are widened exactly on load. */
typedef enum { REFINE_F32 = 0, REFINE_BF16 = 1, REFINE_F16 = 2 } refine_dtype;

/* Projection term of the per-view Hessian weight (Eq. 14-17). */
typedef enum {
    REFINE_PROJ_COV = 0,    /* Tr(Sigma') z^2 / (sbar^2 (fx^2+fy^2) (z^2+eta)), Sigma' the EWA
                               projected covariance; equals Eq. 17 on the optical axis */
    REFINE_PROJ_DEPTH = 1,  /* 1 / (z^2 + eta), Eq. 17 verbatim */
    REFINE_PROJ_NONE = 2    /* 1 (ablation "w/o P" of Table 3) */
} refine_proj_mode;

/* Visibility term (Eq. 12 with the zero-occlusion approximation T = 1). */
typedef enum {
    REFINE_VIS_ALPHA = 0,   /* V = alpha */
    REFINE_VIS_NONE = 1     /* V = 1 (ablation "w/o V" of Table 3) */
} refine_vis_mode;

/*
 * A scene of n Gaussians stored attribute-major: 59 planes of `stride`
 * elements each, plane p of primitive i at element p * stride + i.  Planes:
 *   0..2 centre x,y,z | 3..5 log-scale | 6..9 quaternion w,x,y,z (any norm;
 *   zero = identity) | 10 opacity logit | 11..13 SH DC r,g,b | 14..58 higher
 *   SH coefficients.
 * These are the 59 parameters per primitive of Eq. 1 (Sec. 3.1).  Planes
 * 0..10 are stored as `dtype`, planes 11..58 as `sh_dtype`; the supported
 * pairs are (REFINE_F32, REFINE_F32) (4-byte elements),
 * (REFINE_BF16, REFINE_F16) (2-byte elements: BF16 geometry and opacity, FP16
 * colour) and (REFINE_F16, REFINE_F16) (2-byte elements, all FP16: centres
 * kept to 11 significant bits instead of BF16's 8); other pairs return
 * REFINE_E_UNSUPPORTED.
 * n >= 0, stride >= n, n <= 2^31 - 1.  For an output scene (refine_compact)
 * n is the capacity in primitives.
 */
typedef struct {
    int64_t n;
    int64_t stride;
    int32_t dtype;          /* refine_dtype of planes 0..10 */
    int32_t sh_dtype;       /* refine_dtype of planes 11..58 */
    void* planes;           /* device */
} refine_scene;

/*
 * Method constants (defaults from refine_params_default):
 *  eta      stability constant of Eq. 17, also used in the scene features and
 *           Eq. 18 (0.05, as in the paper)
 *  z_near   a view only counts when the centre's depth exceeds this (0.2)
 *  clamp_k  EWA Jacobian clamp in multiples of the half field of view (1.3)
 *  e_col, e_opa, e_lngem
 *           the calibration expectations E[F_col], E[F_opa], E[ln F_gem] of
 *           Eq. 18 (defaults: expectations under a scene with SH DC ~ N(0,0.5),
 *           logit ~ N(0,1.5), log-scale ~ N(-4.5,1): 8.892106e-3, 0.1767277,
 *           -0.4890595)
 *  proj_mode, vis_mode, equal_lambda
 *           term switches (refine_proj_mode, refine_vis_mode; equal_lambda = 1
 *           sets lambda^k = 1/3, the "Equal lambda" row of Table 3)
 *  n_sub_views
 *           0 = every camera; m > 0 = cameras floor(j * V / m), j < m (the
 *           view subsampling of Table B.1 uses m = 64)
 *  score_path
 *           execution choice of refine_score, never a change of results
 *           (every path gives bit-identical scores): REFINE_PATH_AUTO (0),
 *           REFINE_PATH_DIRECT (1: every (primitive, view) pair evaluated in
 *           input order) or REFINE_PATH_BINNED (2: primitives grouped by
 *           spatial cell, (group, view) pairs whose conservative footprint
 *           bound misses the view frustum skipped)
 *  records_per_lane
 *           binned path only, again never a change of results: 0 = the
 *           library's choice, 1 or 2 primitives per lane (a wave's group is
 *           64 or 128 spatially close primitives sharing one view list)
 *  views_per_iteration
 *           binned path only, never a change of results: 0 = the library's
 *           choice, 1 or 2 views evaluated per iteration of the view loop (two
 *           independent evaluations interleaved; each primitive's sum still
 *           adds the views in the order of refine_score)
 *  waves_per_block
 *           binned path only, never a change of results: 0 = the library's
 *           choice (4), or 1, 2, 4 or 8 wave64s (primitive groups of 64 or
 *           128) per block of the view loop; a block's waves share one LDS
 *           copy of the camera constants
 *  score_kind
 *           REFINE_SCORE_IMPORTANCE (0): the importance score of Eq. 7 with
 *           the Hessian weights of Eq. 20 (every switch above applies);
 *           REFINE_SCORE_OPACITY (1): the parameter-space "Opacity" ranking the
 *           introduction (Sec. 1) contrasts REFINE with, D_i = alpha_i =
 *           sigmoid(opacity logit); cameras, statistics and the other switches
 *           are then not used (refine_score still validates its arguments)
 */
typedef struct {
    double eta;
    double z_near;
    double clamp_k;
    double e_col;
    double e_opa;
    double e_lngem;
    int32_t proj_mode;
    int32_t vis_mode;
    int32_t equal_lambda;
    int32_t n_sub_views;
    int32_t score_path;
    int32_t records_per_lane;
    int32_t views_per_iteration;
    int32_t score_kind;
    int32_t waves_per_block;
} refine_params;

typedef enum { REFINE_PATH_AUTO = 0, REFINE_PATH_DIRECT = 1, REFINE_PATH_BINNED = 2 } refine_score_path;
typedef enum { REFINE_SCORE_IMPORTANCE = 0, REFINE_SCORE_OPACITY = 1 } refine_score_kind;

/*
 * Scene statistics written to device memory by refine_stats:
 *  ybar, f_col, f_opa, f_gem   the features of Eq. (features): mean luma,
 *                              luma variance, mean alpha(1-alpha), mean
 *                              max(s)/(min(s)+eta)
 *  lambda[3]                   {gem, col, opa} weights of Eq. 18-19 (sum 1)
 *  n                           primitives reduced
 *  n_nonfinite                 primitives with a non-finite value in one of
 *                              the 14 planes the scoring reads; when > 0 the
 *                              features and scores are not meaningful
 *  bbox_min, bbox_max          axis-aligned bounds of the finite centres
 *                              (refine_score's spatial binning reads them)
 */
typedef struct {
    double ybar;
    double f_col;
    double f_opa;
    double f_gem;
    double lambda[3];
    int64_t n;
    int64_t n_nonfinite;
    float bbox_min[3];
    float bbox_max[3];
} refine_stats_t;

/* Library version string (static storage). */
const char* refine_version(void);

/* Human-readable name of a refine_status (static storage). */
const char* refine_status_string(int32_t status);

/* Fill *p with the defaults listed above.  No-op on NULL. */
void refine_params_default(refine_params* p);

/* Number of primitives removed at prune ratio `ratio` in (0, 1): beta*N to
 * the nearest integer, halves up (Sec. 3.3).  Returns -1 on invalid input. */
int64_t refine_prune_count(int64_t n, double ratio);

/* Workspace bytes needed by every call below for scenes of up to n
 * primitives and n_views cameras; with n_views = 0, the (much smaller) size
 * that refine_stats, refine_select and refine_compact need, which take no
 * cameras.  REFINE_E_INVALID on negative sizes or a NULL `bytes`. */
refine_status refine_workspace_size(int64_t n, int32_t n_views, size_t* bytes);

/*
 * Scene features (Eq. features) and content-adaptive weights (Eq. 18, 19).
 * Per-primitive terms in FP32, reduced in FP64 with a fixed order (results
 * are bit-identical run to run).  Writes *d_stats (device).
 * n = 0 writes zeros and lambda = 1/3.
 */
refine_status refine_stats(const refine_scene* scene, const refine_params* params,
                           refine_stats_t* d_stats, void* d_ws, size_t ws_bytes, void* stream);

/*
 * refine_stats without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The same kernels and results as refine_stats, bit for
 * bit; the tile partials live in a fixed 1 MiB array in device memory that
 * the library holds on every GPU it runs on until the process ends.
 *  - n <= REFINE_STATS_NOALLOC_MAX_N, else REFINE_E_UNSUPPORTED (nothing is
 *    enqueued); other arguments and errors as for refine_stats.
 *  - The work runs on the CURRENT device's array (stream must belong to the
 *    current device).  The first call on a device resolves the array's
 *    address there (no allocation); that call is best made before any graph
 *    capture starts.
 *  - Every call on one GPU shares that GPU's array: calls that overlap on one
 *    GPU (concurrent streams, or threads) race and give wrong statistics;
 *    order them on one stream.  Nothing needs clearing between calls.
 */
#define REFINE_STATS_NOALLOC_MAX_N 67108864
refine_status refine_stats_noalloc(const refine_scene* scene, const refine_params* params, refine_stats_t* d_stats,
                                   void* stream);

/*
 * Importance scores D_i (Eq. 7 with the Hessian weights of Eq. 20):
 *   D_i = sum_k lambda^k G~_i^k * (1/|V|) sum_v g_i^v V_i P_i^v
 * with the visibility V_i and projection P_i^v of the selected modes and the
 * gate g_i^v (depth > z_near and the 3-sigma footprint of the projected
 * covariance overlapping the image).  FP32 arithmetic; each primitive's
 * views are summed in order within blocks of 64 and the block sums added in
 * order, so the rounding error of the mean grows with 64 + n_views / 64 (to
 * first order at most (66 + n_views / 64) * 2^-24 relative, about 1e-3 at
 * the 2^20 views a call accepts).
 * params->score_path picks how the pairs are scheduled (results identical).
 *  d_cams    device float32 [n_views][18]: world-to-camera rotation R
 *            (row-major), translation t (p_cam = R p + t), fx, fy, cx, cy,
 *            W, H (pixels; Eq. 13), camera axes x right, y down, z forward
 *  d_stats   device, the output of refine_stats for the same scene
 *  d_scores  device float32 [n]
 * n_views >= 1.
 */
refine_status refine_score(const refine_scene* scene, const float* d_cams, int32_t n_views,
                           const refine_params* params, const refine_stats_t* d_stats,
                           float* d_scores, void* d_ws, size_t ws_bytes, void* stream);

/*
 * refine_score in two phases (refine_score = prepare, then views):
 *  refine_score_prepare  builds the per-view constant tables and, on the
 *                        binned path, the spatially binned, activated copy of
 *                        the scene in the workspace, then the views each group
 *                        of binned primitives keeps (the conservative frustum
 *                        test) and the order the view loop takes the groups
 *                        in.  It depends only on the scene, the cameras, the
 *                        parameters and d_stats.
 *  refine_score_cameras  rebuilds what depends on the cameras -- the per-view
 *                        tables and, on the binned path, the groups' kept
 *                        views and order -- for a new camera set (any n_views
 *                        the workspace was sized for; the scene's planes are
 *                        not read).  The binned copy of the scene does not
 *                        depend on the cameras, so a scene prepared once can
 *                        be scored for many camera sets: prepare once, then
 *                        cameras + views per camera set, with the same scene,
 *                        params and d_stats.
 *  refine_score_views    evaluates every (primitive, view) pair that can
 *                        contribute and writes d_scores: one kernel launch
 *                        (plus one when d_evaluated is given).  It reads the
 *                        tables the last prepare / cameras call on the same
 *                        workspace built, so the same scene, n_views, params
 *                        (records_per_lane included) and d_stats must be
 *                        passed (scene->planes is read only on the direct
 *                        path).  Several views calls may follow one prepare.
 *  d_evaluated (nullable, device int64[2]) receives [0] the number of pairs
 *  the view loop evaluated in full and [1] the number it screened out after
 *  their first step (the camera-space centre and its distance outside the
 *  image), because no record of their group could pass for that view.
 *  On the direct path these are n * |V| and 0. On the binned path, [0] + [1]
 *  counts the pairs of 64-primitive groups whose bound reaches the view.
 */
refine_status refine_score_prepare(const refine_scene* scene, const float* d_cams, int32_t n_views,
                                   const refine_params* params, const refine_stats_t* d_stats,
                                   void* d_ws, size_t ws_bytes, void* stream);
refine_status refine_score_cameras(const refine_scene* scene, const float* d_cams, int32_t n_views,
                                   const refine_params* params, void* d_ws, size_t ws_bytes, void* stream);
refine_status refine_score_views(const refine_scene* scene, int32_t n_views, const refine_params* params,
                                 const refine_stats_t* d_stats, float* d_scores, int64_t* d_evaluated,
                                 void* d_ws, size_t ws_bytes, void* stream);

/*
 * Global ranking and ratio selection (Sec. 3.3): primitives are ordered by
 * (score, index) and the first n_prune are removed, n_prune =
 * refine_prune_count(n, ratio), or n_prune_override when it is >= 0 (then
 * 0 <= n_prune_override <= n and ratio is ignored).  NaN scores rank above
 * every number; -0 equals +0.
 *  d_keep        device uint8 [n]: 1 = kept, 0 = pruned
 *  d_n_keep      device int64 (nullable): n - n_prune
 *  d_threshold   device uint32 (nullable): order-preserving key of the score
 *                of the last pruned primitive (0 when nothing is pruned)
 */
refine_status refine_select(const float* d_scores, int64_t n, double ratio, int64_t n_prune_override,
                            uint8_t* d_keep, int64_t* d_n_keep, uint32_t* d_threshold,
                            void* d_ws, size_t ws_bytes, void* stream);

/*
 * The removal step of Sec. 3.3: the bottom beta*N primitives are removed
 * permanently, so the pruned scene is the survivors of the keep mask (the
 * paper's timings include saving them, Sec. 4.2 with Table 2).
 * Survivors of a keep mask, in their original order, all 59 planes
 * (bit copies): out->planes[p * out->stride + j] = in->planes[p * in->stride
 * + i_j] with i_j the j-th index whose d_keep is non-zero.  d_index_map
 * (nullable, device int32 [out->n]) receives i_j.  out->n is the capacity:
 * survivors beyond it are not written.  d_n_out (nullable, device int64)
 * receives the number of survivors (which may exceed the capacity).
 * in and out must have the same dtype and sh_dtype and must not overlap.
 * Speed, not results, depends on alignment: with in->planes 16-byte aligned,
 * in->stride times the element size a multiple of 16 bytes and d_keep 4-byte
 * aligned, each plane is read with 16-byte loads; for 2-byte storage an
 * output 4-byte aligned with an even stride is written two elements per
 * store.  Other layouts take a scalar path.
 */
refine_status refine_compact(const refine_scene* in, const uint8_t* d_keep, const refine_scene* out,
                             int32_t* d_index_map, int64_t* d_n_out, void* d_ws, size_t ws_bytes,
                             void* stream);

/*
 * Batched pruning of many (small) scenes in one grouped launch per kernel:
 * for every job, refine_stats, then refine_score evaluating every pair (the
 * direct path: params->score_path and records_per_lane are not used; the
 * scores equal refine_score's bit for bit), refine_select at the job's ratio
 * and refine_compact -- the same results as those calls made job by job,
 * with 9 launches (and one table copy) for the whole batch instead of 11 per
 * job.  For serving loops that gather the small scenes that arrive together.
 *  jobs       host array of n_jobs descriptions, read during the call (the
 *             table is copied into the workspace with a host-to-device copy
 *             on `stream`); 1 <= n_jobs <= 4096
 *  scene      input scene, 1 <= scene.n <= 16,777,216 (4096 tiles)
 *  d_cams     device [n_views][18] as for refine_score; n_views >= 1
 *  ratio      prune ratio in (0, 1), as for refine_select
 *  d_stats, d_scores, d_keep    device outputs as for refine_stats,
 *             refine_score and refine_select; d_n_keep nullable
 *  out        survivors as for refine_compact (out.n = capacity, same dtypes
 *             as scene, no overlap with it); d_index_map, d_n_out nullable
 *  params     shared by all jobs
 * The workspace size comes from refine_prune_batch_workspace_size for the
 * same jobs (it depends on each job's n and n_views).
 */
typedef struct {
    refine_scene scene;
    const float* d_cams;
    int32_t n_views;
    int32_t reserved;            /* must be 0 */
    double ratio;
    refine_stats_t* d_stats;
    float* d_scores;
    uint8_t* d_keep;
    int64_t* d_n_keep;
    refine_scene out;
    int32_t* d_index_map;
    int64_t* d_n_out;
} refine_prune_job;

refine_status refine_prune_batch_workspace_size(const refine_prune_job* jobs, int32_t n_jobs,
                                                const refine_params* params, size_t* bytes);

/*
 * h_staging (nullable): PINNED host memory (hipHostMalloc) of
 * staging_bytes >= n_jobs * REFINE_BATCH_STAGING_BYTES_PER_JOB bytes (else
 * REFINE_E_WORKSPACE), aligned to 8 bytes (else REFINE_E_INVALID), owned by
 * the caller; staging_bytes is ignored when h_staging is NULL.
 * The call writes the device job table there and copies it to the workspace
 * asynchronously on `stream`, so the caller must leave the buffer untouched
 * until the stream has passed this call (an event recorded after it has
 * completed).  With NULL the table goes through pageable memory and the call
 * returns only once the copy has been taken.
 */
#define REFINE_BATCH_STAGING_BYTES_PER_JOB 256
refine_status refine_prune_batch(const refine_prune_job* jobs, int32_t n_jobs, const refine_params* params,
                                 void* d_ws, size_t ws_bytes, void* h_staging, size_t staging_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* REFINE_H */
