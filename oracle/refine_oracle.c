/*
 * refine_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of REFINE's rendering-free
 * primitive-importance scoring and ratio pruning (Sec. 3.2-3.3 of the paper).
 * Only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header or constant with the GPU
 * library: everything below is written from the paper's equations and the
 * readings of them listed in the design notes.
 *
 * Every floating-point step runs in double precision, in the order the paper
 * states it.  The only parallelism is an OpenMP loop over primitives, whose
 * per-primitive work (the loop over views) is sequential in view order.
 *
 * Input layout: a float32 scene planes[59][stride] (centre xyz, log-scale x3,
 * quaternion w,x,y,z, opacity logit, SH DC rgb, 45 higher SH coefficients)
 * and float32 cameras cams[V][18] (world-to-camera R row-major, t, fx, fy,
 * cx, cy, W, H).
 *
 * Parity status (also recorded in the design notes):
 *   oracle_stats, oracle_lambda     pinned (closed forms on hand-built scenes,
 *                                   brute-force fsum, normalisation)
 *   oracle_pair / oracle_score      pinned (on-axis closed form of Eq. 16/17,
 *                                   finite differences of Eq. 13, Sigma' vs a
 *                                   brute-force splat renderer's moments,
 *                                   invariances, gate special cases)
 *   oracle_select, oracle_compact   pinned (brute-force sort / boolean index)
 *   absolute score values vs the paper: parity unpinned (the paper prints no
 *   per-primitive numbers).
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define NPL 59
#define NCAM 18
#define NOUT 20   /* doubles written by one pair evaluation */

/* SH band-0 constant 1/(2 sqrt(pi)): converts a DC coefficient to colour. */
static const double SH_C0 = 0.28209479177387814;

typedef struct {
    double eta;        /* stability constant of Eq. (17), also used in Eq. (features) and (18) */
    double z_near;     /* visibility gate: depth must exceed this (reading of Eq. 12) */
    double clamp_k;    /* EWA Jacobian clamp, in multiples of the half field of view */
    double e_col;      /* calibration expectation E[F_col] of Eq. (18) */
    double e_opa;      /* calibration expectation E[F_opa] of Eq. (18) */
    double e_lngem;    /* calibration expectation E[ln F_gem] of Eq. (18) */
    int32_t proj_mode; /* 0: projected-covariance energy (default), 1: Eq. (17) depth term, 2: P = 1 */
    int32_t vis_mode;  /* 0: V = alpha (Eq. 12, T = 1), 1: V = 1 */
    int32_t equal_lambda; /* 1: lambda^k = 1/3 ("Equal lambda" of Table 3) */
    int32_t n_sub_views;  /* 0: all views; m > 0: views floor(j V / m), j < m */
    double amb_k;      /* FP32-reach band of the gate decisions, in units of the FP32
                          roundoff 2^-24 times the error magnitudes below */
    int32_t score_kind;   /* 0: importance of Eq. (7) with Eq. (20); 1: opacity alone (Sec. 1) */
} oracle_params;

/* Unit roundoff of IEEE single precision (round to nearest). */
static const double FP32_U = 5.9604644775390625e-08;

/* Number of threads the OpenMP loops use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- helpers */

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Activated primitive (Sec. 3.1, Eq. 1): scales are exp(log-scale), opacity
 * is sigmoid(logit), the rotation comes from the normalised quaternion. */
typedef struct {
    double mu[3];
    double s[3];
    double Rq[3][3];
    double Sigma[3][3];   /* 3D covariance Rq diag(s^2) Rq^T */
    double sbar2;         /* mean squared scale (s0^2 + s1^2 + s2^2) / 3 */
    double smax;          /* largest scale */
    double lsmax;         /* largest |log-scale| (the error of an FP32 exp grows with it) */
    double alpha;
    double rgb[3];        /* DC colour 0.5 + C0 * dc */
    double Y;             /* perceptual luma (BT.601 weights) */
    double gt_gem, gt_col, gt_opa;  /* attribute magnitudes G~^k of Eq. (7) */
} prim_t;

static double plane(const float* planes, int64_t stride, int p, int64_t i)
{
    return (double)planes[(int64_t)p * stride + i];
}

static void quat_to_rot(double w, double x, double y, double z, double R[3][3])
{
    double nrm = sqrt(w * w + x * x + y * y + z * z);
    if (nrm == 0.0) { w = 1.0; x = y = z = 0.0; } else { w /= nrm; x /= nrm; y /= nrm; z /= nrm; }
    R[0][0] = 1.0 - 2.0 * (y * y + z * z); R[0][1] = 2.0 * (x * y - w * z);       R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);       R[1][1] = 1.0 - 2.0 * (x * x + z * z); R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);       R[2][1] = 2.0 * (y * z + w * x);       R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

static void activate(const float* planes, int64_t stride, int64_t i, prim_t* p)
{
    for (int k = 0; k < 3; ++k) p->mu[k] = plane(planes, stride, 0 + k, i);
    p->lsmax = 0.0;
    for (int k = 0; k < 3; ++k) {
        double ls = plane(planes, stride, 3 + k, i);
        p->s[k] = exp(ls);
        if (fabs(ls) > p->lsmax) p->lsmax = fabs(ls);
    }
    p->smax = p->s[0];
    for (int k = 1; k < 3; ++k) if (p->s[k] > p->smax) p->smax = p->s[k];
    quat_to_rot(plane(planes, stride, 6, i), plane(planes, stride, 7, i),
                plane(planes, stride, 8, i), plane(planes, stride, 9, i), p->Rq);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += p->Rq[r][k] * p->s[k] * p->s[k] * p->Rq[c][k];
            p->Sigma[r][c] = acc;
        }
    p->sbar2 = (p->s[0] * p->s[0] + p->s[1] * p->s[1] + p->s[2] * p->s[2]) / 3.0;
    p->alpha = sigmoid(plane(planes, stride, 10, i));
    for (int k = 0; k < 3; ++k) p->rgb[k] = 0.5 + SH_C0 * plane(planes, stride, 11 + k, i);
    p->Y = 0.299 * p->rgb[0] + 0.587 * p->rgb[1] + 0.114 * p->rgb[2];
    /* geometry area: product of the two largest scales */
    double lo = p->s[0];
    for (int k = 1; k < 3; ++k) if (p->s[k] < lo) lo = p->s[k];
    p->gt_gem = p->s[0] * p->s[1] * p->s[2] / lo;
    p->gt_col = sqrt(p->rgb[0] * p->rgb[0] + p->rgb[1] * p->rgb[1] + p->rgb[2] * p->rgb[2]);
    p->gt_opa = p->alpha;
}

/* ------------------------------------------------------------ statistics */

/* Number of primitives with a non-finite value in any of the 14 planes the
 * scoring reads (centre, log-scale, quaternion, opacity, SH DC). */
int64_t oracle_nonfinite(const float* planes, int64_t n, int64_t stride)
{
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int ok = 1;
        for (int p = 0; p < 14; ++p) if (!isfinite(plane(planes, stride, p, i))) ok = 0;
        bad += !ok;
    }
    return bad;
}

/* Scene features of Eq. (features): out = {Ybar, F_col, F_opa, F_gem}.
 * F_col is the (biased, 1/N) variance of luma, computed in two passes. */
void oracle_stats(const float* planes, int64_t n, int64_t stride, double eta, double out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (n <= 0) return;
    double sumY = 0.0, sumOpa = 0.0, sumGem = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        prim_t p;
        activate(planes, stride, i, &p);
        sumY += p.Y;
        sumOpa += p.alpha * (1.0 - p.alpha);
        double smax = p.s[0], smin = p.s[0];
        for (int k = 1; k < 3; ++k) { if (p.s[k] > smax) smax = p.s[k]; if (p.s[k] < smin) smin = p.s[k]; }
        sumGem += smax / (smin + eta);
    }
    double Ybar = sumY / (double)n;
    double sumDev = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        prim_t p;
        activate(planes, stride, i, &p);
        sumDev += (p.Y - Ybar) * (p.Y - Ybar);
    }
    out[0] = Ybar;
    out[1] = sumDev / (double)n;
    out[2] = sumOpa / (double)n;
    out[3] = sumGem / (double)n;
}

/* Content-adaptive weights: Eq. (18) then the normalisation of Eq. (19).
 * F = {Ybar, F_col, F_opa, F_gem}; lam = {gem, col, opa}. */
void oracle_lambda(const double F[4], const oracle_params* prm, double lam[3])
{
    if (prm->equal_lambda) { lam[0] = lam[1] = lam[2] = 1.0 / 3.0; return; }
    double lt_gem = log(F[3] + prm->eta) / prm->e_lngem;
    double lt_col = F[1] / prm->e_col;
    double lt_opa = F[2] / prm->e_opa;
    double sum = lt_gem + lt_col + lt_opa;
    lam[0] = lt_gem / sum;
    lam[1] = lt_col / sum;
    lam[2] = lt_opa / sum;
}

/* ------------------------------------------------------- per-view terms */

/* One (primitive, view) evaluation.  out (NOUT doubles):
 *  0..2  x, y, z   camera-space centre
 *  3..4  u, v      projected centre, Eq. (13)
 *  5..10 J         2x3 EWA Jacobian of the projection (clamped), row-major, Eq. (14)
 *  11..13 a, b, c  projected 2D covariance Sigma' = J W Sigma W^T J^T
 *  14    r         footprint radius 3 sqrt(lambda_max(Sigma'))
 *  15    P         projection term of the selected mode (Eq. 14-17 reading)
 *  16    m         signed footprint margin min(u + r, W - u + r, v + r, H - v + r)
 *  17, 18          FP32-reach bands of the left/right and top/bottom edge margins
 *  19              FP32-reach band of the depth z
 * returns the gate g (1 visible, 0 not) and writes ambiguity into *amb:
 * bit 0 = near-plane decision within FP32 reach, bit 1 = footprint decision
 * within FP32 reach; *could = 1 when an evaluation perturbed within that
 * reach could find the pair visible.  When z <= 0 only x, y, z are written.
 *
 * FP32 reach.  The gate is discontinuous, so an FP32 evaluation of the same
 * formulas (any operation order, fused or not, approximate reciprocals) can
 * take the other decision when a margin is within its rounding error.  With
 * u = 2^-24 and K = amb_k, the bands bound that error to first order:
 *  depth:   z = R_2 . mu + t_z is a 3-term dot product of FP32 values, so its
 *           error is a few u times mag_z = |R_2| . |mu| + |t_z|:
 *           band_z = K u (mag_z + z_near).
 *  centre:  u_px = fx x / z + cx carries the errors of x and z (u mag_x,
 *           u mag_z), of the division and of the offsets:
 *           E_x = (fx mag_x + (|cx| + W + |u_px - cx|) mag_z) / z + |u_px| + W,
 *           and E_y likewise (these also bound forms that premultiply the
 *           rows by intrinsics or shift the origin to the image centre).
 *  radius:  r = sigma_max(3 J W L) with L = R(q) diag(s) (Sigma = L L^T), and
 *           sigma_max moves by at most the spectral norm of the error of its
 *           argument.  J's entries carry the relative error of 1/z (u mag_z / z)
 *           and the centre errors through x/z and y/z (E_x / z, E_y / z); L's
 *           entries the error of an FP32 exp, which grows with |log-scale|;
 *           forming lambda_max from the 2x2 sums costs a few u of r:
 *           E_r = r + 3 s_max ((1 + mag_z / z + max|log-scale|) |J|_F
 *                               + (E_x + E_y) / z).
 *  Each edge margin (u_px + r, W - u_px + r, ...) then has the band
 *  K u (E_x + E_r) or K u (E_y + E_r), and the footprint decision is
 *  ambiguous when the smallest margin could reach either sign within them. */
static int pair_eval(const prim_t* p, const float* cam, const oracle_params* prm,
                     double out[NOUT], int* amb, int* could)
{
    double Rv[3][3], t[3];
    for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) Rv[r][c] = (double)cam[3 * r + c];
    for (int k = 0; k < 3; ++k) t[k] = (double)cam[9 + k];
    double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15], W = cam[16], H = cam[17];

    double pc[3], mag[3];
    for (int r = 0; r < 3; ++r) {
        pc[r] = Rv[r][0] * p->mu[0] + Rv[r][1] * p->mu[1] + Rv[r][2] * p->mu[2] + t[r];
        mag[r] = fabs(Rv[r][0] * p->mu[0]) + fabs(Rv[r][1] * p->mu[1]) + fabs(Rv[r][2] * p->mu[2]) + fabs(t[r]);
    }
    double x = pc[0], y = pc[1], z = pc[2];
    out[0] = x; out[1] = y; out[2] = z;
    for (int k = 3; k < NOUT; ++k) out[k] = 0.0;
    *amb = 0;
    *could = 0;

    double ku = prm->amb_k * FP32_U;
    double tz = ku * (mag[2] + prm->z_near);
    out[19] = tz;
    int near_ok = z > prm->z_near;
    if (fabs(z - prm->z_near) <= tz) *amb |= 1;
    if (z <= 0.0) { *amb = 0; return 0; }

    /* Eq. (13): pinhole projection of the centre */
    double u = fx * x / z + cx;
    double v = fy * y / z + cy;
    /* Eq. (14): local affine (EWA) Jacobian; x/z, y/z clamped to k times the half FOV */
    double limx = prm->clamp_k * W / (2.0 * fx);
    double limy = prm->clamp_k * H / (2.0 * fy);
    double xh = clampd(x / z, -limx, limx);
    double yh = clampd(y / z, -limy, limy);
    double J[2][3] = {{fx / z, 0.0, -fx * xh / z}, {0.0, fy / z, -fy * yh / z}};
    /* Sigma' = J W Sigma W^T J^T with W the camera rotation */
    double T[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            T[r][c] = J[r][0] * Rv[0][c] + J[r][1] * Rv[1][c] + J[r][2] * Rv[2][c];
    double TS[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            TS[r][c] = T[r][0] * p->Sigma[0][c] + T[r][1] * p->Sigma[1][c] + T[r][2] * p->Sigma[2][c];
    double a = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2];
    double b = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
    double c = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2];
    /* 3-sigma footprint of the projected ellipse */
    double half = 0.5 * (a - c);
    double lmax = 0.5 * (a + c) + sqrt(half * half + b * b);
    double r = 3.0 * sqrt(lmax);
    double edge[4] = {u + r, W - u + r, v + r, H - v + r};
    double m = edge[0];
    for (int e = 1; e < 4; ++e) if (edge[e] < m) m = edge[e];
    int foot_ok = m > 0.0;
    /* FP32 reach of each edge margin (see above) */
    double Ex = (fx * mag[0] + (fabs(cx) + W + fabs(u - cx)) * mag[2]) / z + fabs(u) + W;
    double Ey = (fy * mag[1] + (fabs(cy) + H + fabs(v - cy)) * mag[2]) / z + fabs(v) + H;
    double Jf = sqrt(J[0][0] * J[0][0] + J[0][2] * J[0][2] + J[1][1] * J[1][1] + J[1][2] * J[1][2]);
    double Er = r + 3.0 * p->smax * ((1.0 + mag[2] / z + p->lsmax) * Jf + (Ex + Ey) / z);
    double band[4] = {ku * (Ex + Er), ku * (Ex + Er), ku * (Ey + Er), ku * (Ey + Er)};
    double mlo = edge[0] - band[0], mhi = edge[0] + band[0];
    for (int e = 1; e < 4; ++e) {
        if (edge[e] - band[e] < mlo) mlo = edge[e] - band[e];
        if (edge[e] + band[e] < mhi) mhi = edge[e] + band[e];
    }
    if (mlo <= 0.0 && mhi >= 0.0) *amb |= 2;
    out[16] = m;
    out[17] = band[0];
    out[18] = band[2];

    double P;
    if (prm->proj_mode == 0)
        P = (a + c) * z * z / (p->sbar2 * (fx * fx + fy * fy) * (z * z + prm->eta));
    else if (prm->proj_mode == 1)
        P = 1.0 / (z * z + prm->eta);   /* Eq. (17) */
    else
        P = 1.0;

    out[3] = u; out[4] = v;
    out[5] = J[0][0]; out[6] = J[0][1]; out[7] = J[0][2];
    out[8] = J[1][0]; out[9] = J[1][1]; out[10] = J[1][2];
    out[11] = a; out[12] = b; out[13] = c; out[14] = r; out[15] = P;
    *could = (near_ok || (*amb & 1)) && (foot_ok || (*amb & 2));
    return near_ok && foot_ok;
}

/* Exposed for the tests: evaluate one pair from raw (unactivated) values.
 * prim14 = {x,y,z, ls0,ls1,ls2, qw,qx,qy,qz, logit, dc_r,dc_g,dc_b}. */
int oracle_pair(const float* prim14, const float* cam, const oracle_params* prm,
                double out[NOUT], int32_t* amb)
{
    prim_t p;
    activate(prim14, 1, 0, &p);
    int a = 0, could = 0;
    int g = pair_eval(&p, cam, prm, out, &a, &could);
    if (amb) *amb = a;
    return g;
}

/* Attribute magnitudes etc. of one raw primitive, for the tests:
 * out = {s0,s1,s2, sbar2, alpha, Y, gt_gem, gt_col, gt_opa, R (9, row-major)}. */
void oracle_activate(const float* prim14, double out[18])
{
    prim_t p;
    activate(prim14, 1, 0, &p);
    out[0] = p.s[0]; out[1] = p.s[1]; out[2] = p.s[2]; out[3] = p.sbar2; out[4] = p.alpha;
    out[5] = p.Y; out[6] = p.gt_gem; out[7] = p.gt_col; out[8] = p.gt_opa;
    for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) out[9 + 3 * r + c] = p.Rq[r][c];
}

/* ---------------------------------------------------------------- score */

/* Importance scores (Eq. 20 then Eq. 7) of primitives idx[0..m) (all n when
 * idx is NULL, m = n).  lam = {gem, col, opa}.  D[j] is the score of primitive
 * idx[j]; Dlo/Dhi (nullable) bound it when gate-ambiguous pairs are excluded /
 * included; namb (nullable) counts the ambiguous pairs.
 * With score_kind = 1 the score is the parameter-space opacity ranking the
 * introduction (Sec. 1) sets REFINE against: D = alpha, no views. */
void oracle_score(const float* planes, int64_t n, int64_t stride, const float* cams, int32_t n_views,
                  const oracle_params* prm, const double lam[3], const int64_t* idx, int64_t m,
                  double* D, double* Dlo, double* Dhi, int32_t* namb)
{
    if (idx == NULL) m = n;
    int32_t nv = n_views;
    if (prm->n_sub_views > 0 && prm->n_sub_views < n_views) nv = prm->n_sub_views;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < m; ++j) {
        int64_t i = idx ? idx[j] : j;
        prim_t p;
        activate(planes, stride, i, &p);
        if (prm->score_kind == 1) {
            D[j] = p.alpha;
            if (Dlo) Dlo[j] = p.alpha;
            if (Dhi) Dhi[j] = p.alpha;
            if (namb) namb[j] = 0;
            continue;
        }
        double S = 0.0, Slo = 0.0, Shi = 0.0;
        int32_t na = 0;
        for (int32_t jv = 0; jv < nv; ++jv) {
            int64_t v = (nv == n_views) ? jv : ((int64_t)jv * n_views) / nv;
            double o[NOUT];
            int amb = 0, could = 0;
            int g = pair_eval(&p, cams + v * NCAM, prm, o, &amb, &could);
            double P = o[15];
            double Vis = prm->vis_mode == 0 ? p.alpha : 1.0;   /* Eq. (12), T = 1 */
            double term = Vis * P;                              /* Eq. (new1) up to lambda */
            int lo = g && !amb;
            if (g) S += term;
            if (lo) Slo += term;
            if (could) Shi += term;
            if (lo != could) ++na;
        }
        /* Eq. (20): w^k = lambda^k * mean over views; Eq. (7): D = sum_k w^k G~^k */
        double gt[3] = {p.gt_gem, p.gt_col, p.gt_opa};
        double d = 0.0, dlo = 0.0, dhi = 0.0;
        for (int k = 0; k < 3; ++k) {
            d += lam[k] * (S / nv) * gt[k];
            dlo += lam[k] * (Slo / nv) * gt[k];
            dhi += lam[k] * (Shi / nv) * gt[k];
        }
        D[j] = d;
        if (Dlo) Dlo[j] = dlo < dhi ? dlo : dhi;
        if (Dhi) Dhi[j] = dlo < dhi ? dhi : dlo;
        if (namb) namb[j] = na;
    }
}

/* --------------------------------------------------------------- select */

/* Number of primitives removed: beta * N to the nearest integer, halves away
 * from zero, clamped to [0, N] (Sec. 3.3). */
int64_t oracle_n_prune(int64_t n, double ratio)
{
    double k = floor(ratio * (double)n + 0.5);
    if (k < 0) k = 0;
    if (k > (double)n) k = (double)n;
    return (int64_t)k;
}

static const double* g_sort_keys;

static int cmp_rank(const void* pa, const void* pb)
{
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    double da = g_sort_keys[a], db = g_sort_keys[b];
    if (da < db) return -1;
    if (da > db) return 1;
    return a < b ? -1 : (a > b);
}

/* Global ranking of Sec. 3.3: order by (score ascending, index ascending),
 * remove the first n_prune.  keep[i] = 1 for survivors.  order (nullable)
 * receives the ranking. Not re-entrant (qsort comparator state). */
void oracle_select(const double* D, int64_t n, int64_t n_prune, uint8_t* keep, int64_t* order)
{
    int64_t* ord = order ? order : (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) ord[i] = i;
    g_sort_keys = D;
    qsort(ord, (size_t)n, sizeof(int64_t), cmp_rank);
    for (int64_t k = 0; k < n; ++k) keep[ord[k]] = (uint8_t)(k >= n_prune);
    if (!order) free(ord);
}

/* -------------------------------------------------------------- compact */

/* Survivors in their original order: out[p][j] = in[p][idx_j] for every one
 * of the 59 planes, with idx_j the j-th kept index; idxmap (nullable) gets
 * idx_j.  Returns the number kept. */
int64_t oracle_compact(const float* planes, int64_t n, int64_t stride, const uint8_t* keep,
                       float* out, int64_t out_stride, int32_t* idxmap)
{
    int64_t j = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!keep[i]) continue;
        for (int p = 0; p < NPL; ++p) out[(int64_t)p * out_stride + j] = planes[(int64_t)p * stride + i];
        if (idxmap) idxmap[j] = (int32_t)i;
        ++j;
    }
    return j;
}
