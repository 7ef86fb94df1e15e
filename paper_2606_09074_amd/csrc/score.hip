// Rendering-free importance scores (paper Eq. 7-20) on gfx950.
//
// camera_prep: one thread per (possibly subsampled) view builds a 128-byte
// fp32 record of the constants the view loop needs.
//
// score_views: one primitive per lane.  The prologue activates the primitive
// (Eq. 1 readings) and keeps its centre mu and the factored 3D covariance
// L = R(q) diag(s) (Sigma = L L^T) in VGPRs for the whole view loop.  Camera
// records are read through the scalar cache (the index is wave-uniform), so
// the loop body is pure VALU work.  Per (primitive, view), in FP32:
//   p = R_v mu + t_v                               camera-space centre
//   ux = fx x/z, uy = fy y/z                        Eq. 13 about the principal point
//   x^ = clamp(ux, +-k W/2), y^ = clamp(uy, +-k H/2) clamped, in pixels
//   r0 = fx R_v,0 - x^ R_v,2,  r1 = fy R_v,1 - y^ R_v,2
//       so that the EWA Jacobian times the view rotation is [r0; r1] / z (Eq. 14)
//   A0 = r0 L, A1 = r1 L;  a = |A0|^2, b = A0.A1, c = |A1|^2
//       z^2 Sigma' = [[a, b], [b, c]]: sums of squares, free of the
//       cancellation that T Sigma T^T suffers for needle-like primitives
//   gate: z > z_near and the 3-sigma box of Sigma' overlaps the image
//   projection term (mode COV): (a + c) / ((fx^2 + fy^2) (z^2 + eta)), the
//       1/sbar^2 factor being applied once in the epilogue
// The views are accumulated in order into one FP32 sum per primitive; the
// epilogue forms D = V K S / |V| (Eq. 20 then Eq. 7).
#include "refine_internal.hpp"

namespace refine {

namespace {

constexpr float kShC0 = 0.28209479177387814f;

__global__ __launch_bounds__(kBlock) void camera_prep(const float* __restrict__ cams, int n_views, int nv,
                                                        float clamp_k, CamRec* __restrict__ out)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= nv) return;
    const int v = (nv == n_views) ? j : (int)(((int64_t)j * n_views) / nv);
    const float* c = cams + (int64_t)v * kCamFields;
    CamRec r;
#pragma unroll
    for (int k = 0; k < 9; ++k) r.r[k] = c[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) r.t[k] = c[9 + k];
    const float fx = c[12], fy = c[13], cx = c[14], cy = c[15], W = c[16], H = c[17];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r.fr0[k] = fx * c[k];
        r.fr1[k] = fy * c[3 + k];
    }
    r.fx = fx;
    r.fy = fy;
    r.hw = 0.5f * W;
    r.hh = 0.5f * H;
    r.ox = cx - r.hw;
    r.oy = cy - r.hh;
    r.lx = clamp_k * r.hw;
    r.ly = clamp_k * r.hh;
    r.kv = 1.0f / (fx * fx + fy * fy);
#pragma unroll
    for (int k = 0; k < 5; ++k) r.pad[k] = 0.0f;
    out[j] = r;
}

// PROJ: refine_proj_mode
template <int PROJ>
__global__ __launch_bounds__(kBlock) void score_views(const float* __restrict__ planes, int64_t stride, int n,
                                                        const CamRec* __restrict__ cams, int nv,
                                                        const refine_stats_t* __restrict__ st, float eta,
                                                        float z_near, int vis_alpha, float* __restrict__ out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float a[kScorePlanes];
#pragma unroll
    for (int p = 0; p < kScorePlanes; ++p) a[p] = planes[(int64_t)p * stride + i];

    // ---- activation (Sec. 3.1): s = exp(log-scale), unit quaternion, alpha = sigmoid(logit)
    const float mx = a[0], my = a[1], mz = a[2];
    const float s0 = __expf(a[3]), s1 = __expf(a[4]), s2 = __expf(a[5]);
    float qw = a[6], qx = a[7], qy = a[8], qz = a[9];
    const float qn = qw * qw + qx * qx + qy * qy + qz * qz;
    if (qn > 0.0f) {
        const float inv = rsqrtf(qn);
        qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    } else {
        qw = 1.0f; qx = qy = qz = 0.0f;
    }
    // L = R(q) diag(s)
    const float L00 = (1.0f - 2.0f * (qy * qy + qz * qz)) * s0;
    const float L01 = (2.0f * (qx * qy - qw * qz)) * s1;
    const float L02 = (2.0f * (qx * qz + qw * qy)) * s2;
    const float L10 = (2.0f * (qx * qy + qw * qz)) * s0;
    const float L11 = (1.0f - 2.0f * (qx * qx + qz * qz)) * s1;
    const float L12 = (2.0f * (qy * qz - qw * qx)) * s2;
    const float L20 = (2.0f * (qx * qz - qw * qy)) * s0;
    const float L21 = (2.0f * (qy * qz + qw * qx)) * s1;
    const float L22 = (1.0f - 2.0f * (qx * qx + qy * qy)) * s2;

    const float sbar2 = (s0 * s0 + s1 * s1 + s2 * s2) * (1.0f / 3.0f);
    const float alpha = 1.0f / (1.0f + __expf(-a[10]));
    const float cr = fmaf(kShC0, a[11], 0.5f), cg = fmaf(kShC0, a[12], 0.5f), cb = fmaf(kShC0, a[13], 0.5f);
    // attribute magnitudes (Eq. 7): two largest scales' product, |colour|, alpha
    const float g_gem = fmaxf(s0 * s1, fmaxf(s0 * s2, s1 * s2));
    const float g_col = sqrtf(cr * cr + cg * cg + cb * cb);
    const float K = (float)st->lambda[0] * g_gem + (float)st->lambda[1] * g_col + (float)st->lambda[2] * alpha;

    // ---- view loop (Eq. 20)
    float S = 0.0f;
    for (int v = 0; v < nv; ++v) {
        const CamRec& c = cams[v];
        const float x = fmaf(c.r[0], mx, fmaf(c.r[1], my, fmaf(c.r[2], mz, c.t[0])));
        const float y = fmaf(c.r[3], mx, fmaf(c.r[4], my, fmaf(c.r[5], mz, c.t[1])));
        const float z = fmaf(c.r[6], mx, fmaf(c.r[7], my, fmaf(c.r[8], mz, c.t[2])));
        const float rz = __builtin_amdgcn_rcpf(z);
        const float ux = c.fx * x * rz;
        const float uy = c.fy * y * rz;
        const float xh = fminf(fmaxf(ux, -c.lx), c.lx);
        const float yh = fminf(fmaxf(uy, -c.ly), c.ly);
        const float r00 = fmaf(-xh, c.r[6], c.fr0[0]);
        const float r01 = fmaf(-xh, c.r[7], c.fr0[1]);
        const float r02 = fmaf(-xh, c.r[8], c.fr0[2]);
        const float r10 = fmaf(-yh, c.r[6], c.fr1[0]);
        const float r11 = fmaf(-yh, c.r[7], c.fr1[1]);
        const float r12 = fmaf(-yh, c.r[8], c.fr1[2]);
        const float A00 = fmaf(r00, L00, fmaf(r01, L10, r02 * L20));
        const float A01 = fmaf(r00, L01, fmaf(r01, L11, r02 * L21));
        const float A02 = fmaf(r00, L02, fmaf(r01, L12, r02 * L22));
        const float A10 = fmaf(r10, L00, fmaf(r11, L10, r12 * L20));
        const float A11 = fmaf(r10, L01, fmaf(r11, L11, r12 * L21));
        const float A12 = fmaf(r10, L02, fmaf(r11, L12, r12 * L22));
        const float sa = fmaf(A00, A00, fmaf(A01, A01, A02 * A02));
        const float sc = fmaf(A10, A10, fmaf(A11, A11, A12 * A12));
        const float sb = fmaf(A00, A10, fmaf(A01, A11, A02 * A12));
        // 3-sigma footprint: r = 3 sqrt(lambda_max) / z, lambda_max of [[sa, sb], [sb, sc]]
        const float hm = 0.5f * (sa - sc);
        const float lmax = fmaf(0.5f, sa + sc, sqrtf(fmaf(hm, hm, sb * sb)));
        const float rad = 3.0f * sqrtf(lmax) * rz;
        const float d = fmaxf(fabsf(ux + c.ox) - c.hw, fabsf(uy + c.oy) - c.hh);
        const bool g = (z > z_near) && (d < rad);
        float P;
        if (PROJ == REFINE_PROJ_COV)
            P = c.kv * (sa + sc) * __builtin_amdgcn_rcpf(fmaf(z, z, eta));
        else if (PROJ == REFINE_PROJ_DEPTH)
            P = __builtin_amdgcn_rcpf(fmaf(z, z, eta));
        else
            P = 1.0f;
        S += g ? P : 0.0f;
    }
    float pre = (vis_alpha ? alpha : 1.0f) * K / (float)nv;
    if (PROJ == REFINE_PROJ_COV) pre = pre / sbar2;
    out[i] = pre * S;
}

}  // namespace

hipError_t launch_score(const float* planes, int64_t stride, int64_t n, const float* d_cams, int32_t n_views,
                        const refine_params& prm, const refine_stats_t* d_stats, float* d_scores,
                        const Workspace& ws, hipStream_t stream)
{
    const int nv = (prm.n_sub_views > 0 && prm.n_sub_views < n_views) ? prm.n_sub_views : n_views;
    hipLaunchKernelGGL(camera_prep, dim3((nv + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, d_cams, n_views, nv,
                       (float)prm.clamp_k, ws.cams);
    if (n == 0) return hipGetLastError();
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    const int vis = prm.vis_mode == REFINE_VIS_ALPHA ? 1 : 0;
    switch (prm.proj_mode) {
    case REFINE_PROJ_COV:
        hipLaunchKernelGGL(score_views<REFINE_PROJ_COV>, grid, dim3(kBlock), 0, stream, planes, stride, (int)n,
                           ws.cams, nv, d_stats, (float)prm.eta, (float)prm.z_near, vis, d_scores);
        break;
    case REFINE_PROJ_DEPTH:
        hipLaunchKernelGGL(score_views<REFINE_PROJ_DEPTH>, grid, dim3(kBlock), 0, stream, planes, stride, (int)n,
                           ws.cams, nv, d_stats, (float)prm.eta, (float)prm.z_near, vis, d_scores);
        break;
    default:
        hipLaunchKernelGGL(score_views<REFINE_PROJ_NONE>, grid, dim3(kBlock), 0, stream, planes, stride, (int)n,
                           ws.cams, nv, d_stats, (float)prm.eta, (float)prm.z_near, vis, d_scores);
        break;
    }
    return hipGetLastError();
}

}  // namespace refine
