/*
 * FP64 CPU oracle for the differentiable Gaussian pointmap rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, per-pixel definition of
 * what the rendering path computes; it is used by the tests, the smoke check and the
 * benchmark's CPU baseline, and by nothing on the product path.  It shares no code,
 * header or constant with the HIP library.
 *
 * What it follows (paper: "Outdoor Monocular SLAM with Global Scale-Consistent 3D
 * Gaussian Pointmaps"):
 *   - Sec. 3.1, Eq. 1: world covariance Sigma = R S S^T R^T from rotation and scale.
 *   - Sec. 3.1: Gaussians projected to the image plane (EWA, perspective Jacobian).
 *   - Sec. 3.1, Eq. 2: colour  C = sum_i c_i a_i prod_{j<i} (1 - a_j).
 *   - Sec. 3.2.1, Eq. 3: depth D = sum_k z_k a_k prod_{l<k} (1 - a_l), Gaussians
 *     sorted by z_k (read as camera-frame depth, the third row of Eq. 4).
 *   - Sec. 3.2.1, Eq. 4-5: pointmap from depth, X = D * K^-1 [i, j, 1]^T.
 *   - The "3D Gaussian pointmap" as the alpha-composited Gaussian centres, in the
 *     world frame or the camera frame.
 *   - Sec. 3.2.2, Eq. 11: gradient with respect to the camera pose through the
 *     projected means and covariances, with the pose linearised in se(3).
 *
 * Conventions where the paper is silent (each one is a setting, shared with the
 * library through the caller): per-pixel alpha = min(alpha_max, a * exp(-e/2)) with
 * a = sigmoid(logit) and e the Mahalanobis distance under the 2D conic; fragments with
 * alpha < alpha_min are skipped; compositing stops before the fragment that would take
 * transmittance below t_min; a low-pass eps2d is added to the 2D covariance; the
 * Jacobian's x/z and y/z are clamped to jac_clamp times the half field of view;
 * Gaussians with z <= near_z are dropped; pixel (i, j) (i = column) is sampled at
 * exactly (i, j), as Eq. 4 writes it; ties in depth are broken by Gaussian index.
 *
 * Everything is double precision.  No tiling: a pixel's candidates are all Gaussians
 * whose candidate box contains it, taken from a per-pixel-row list of Gaussians (an index
 * that only avoids scanning every Gaussian for every pixel; the candidate set is the
 * same).  The candidate box is the bounding box of the ellipse where alpha reaches
 * alpha_min, at an opacity widened by a relative 1e-4 and grown by one pixel: it skips
 * only Gaussians that provably cannot reach alpha_min at the pixel, and it keeps those
 * whose alpha comes within float32 rounding of alpha_min (including Gaussians whose
 * opacity itself lies just below alpha_min), so that the ambiguity flags below see them.
 *
 * Depth order.  Gaussians are composited in ascending order of their depth rounded to
 * float32, ties by index.  The paper sorts by z_k without fixing a precision, and an
 * ordering is a discrete decision taken on floating-point values, so the oracle takes it
 * in the precision of the kernels it checks: its double depth rounded to float32.
 *
 * Ambiguity flags.  A float32 implementation may take a different discrete decision
 * than this oracle where a value sits on a threshold.  Each pixel is flagged when,
 * within a first-order float32 error bound (times a safety factor), a fragment's alpha
 * is at alpha_min or alpha_max or a transmittance step is at t_min, or when a
 * contributing fragment's double depth lies within a few double ulps of a float32
 * rounding midpoint (a depth computed with another rounding of its last bit may round to
 * the other float32 neighbour).  Parity tests compare unflagged pixels only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS32 (1.0 / 16777216.0) /* 2^-24: unit roundoff of float32 */

typedef struct {
    int64_t n;
    const double *means;         /* [3][n] */
    const double *log_scales;    /* [3][n] */
    const double *quats;         /* [4][n] (w, x, y, z), not necessarily unit */
    const double *opacity_logit; /* [n] */
    const double *rgb;           /* [3][n] */
} orc_gaussians;

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double T[12]; /* world -> camera, row-major [R | t] */
} orc_view;

typedef struct {
    double near_z, alpha_min, alpha_max, t_min, eps2d, jac_clamp;
    double bg[3];
    double flag_factor; /* width of the ambiguity bands, in first-order error bounds */
} orc_settings;

/* Projection of one Gaussian into one view. */
typedef struct {
    int32_t visible; /* the support box below is not empty */
    int32_t clamp_x, clamp_y;
    int32_t rect[4]; /* imin, imax, jmin, jmax (inclusive pixel indices) */
    int32_t cand;    /* the candidate box below is not empty */
    int32_t crect[4];/* candidate box (see the header), inclusive pixel indices */
    double m[3];     /* camera-frame centre */
    double u, v, z;
    double a;        /* sigmoid(logit) */
    double s[3];     /* exp(log_scale) */
    double qn[4];    /* unit quaternion */
    double qnorm;
    double Rq[9];    /* rotation of the Gaussian, row-major */
    double Sig[9];   /* world covariance (Eq. 1) */
    double Sigc[9];  /* camera-frame covariance */
    double J[6];     /* 2x3 perspective Jacobian, row-major */
    double cov2[3];  /* 2D covariance xx, xy, yy (with eps2d) */
    double Q[3];     /* conic = inverse 2D covariance: xx, xy, yy */
    double rx, ry;   /* half extents of the support box */
    double bounds[4];/* u - rx, u + rx, v - ry, v + ry (before rounding to pixels) */
} orc_proj;

/* Per-pixel result. */
typedef struct {
    double rgb[3];
    double depth;
    double alpha;
    double pm_world[3];
    double pm_cam[3];
    double pm_eq5[3];
    double T_final;
    int32_t n_frag;    /* contributing fragments */
    int32_t n_cand;    /* candidates looked at (support box contains the pixel) */
    int32_t ambiguous; /* bit 0 alpha_min, 1 t_min, 2 alpha_max, 3 depth at a float32 midpoint */
    int32_t pad;
    double margin;     /* smallest |value - threshold| / (first-order bound) over the
                          pixel's alpha_min, alpha_max and t_min decisions */
} orc_pixel;

/* Gradients, accumulated (+=). */
typedef struct {
    double *means;      /* [3][n] */
    double *log_scales; /* [3][n] */
    double *quats;      /* [4][n] */
    double *opacity_logit; /* [n] */
    double *rgb;        /* [3][n] */
    double *pose;       /* [6]: d/d(rho), d/d(phi) for T <- Exp(xi) T */
} orc_grads;

/* ------------------------------------------------------------------------- */
/* Small linear algebra, written out.                                          */

static void quat_to_rot(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* dR[e][k]: derivative of rotation entry e with respect to quaternion component k. */
static void quat_to_rot_jac(const double q[4], double dR[9][4])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    double t[9][4] = {
        {0.0, 0.0, -4.0 * y, -4.0 * z},
        {-2.0 * z, 2.0 * y, 2.0 * x, -2.0 * w},
        {2.0 * y, 2.0 * z, 2.0 * w, 2.0 * x},
        {2.0 * z, 2.0 * y, 2.0 * x, 2.0 * w},
        {0.0, -4.0 * x, 0.0, -4.0 * z},
        {-2.0 * x, -2.0 * w, 2.0 * z, 2.0 * y},
        {-2.0 * y, 2.0 * z, -2.0 * w, 2.0 * x},
        {2.0 * x, 2.0 * w, 2.0 * z, 2.0 * y},
        {0.0, -4.0 * x, -4.0 * y, 0.0},
    };
    memcpy(dR, t, sizeof(t));
}

static void mat3_mul(const double A[9], const double B[9], double C[9])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += A[3 * r + k] * B[3 * k + c];
            C[3 * r + c] = acc;
        }
}

static void mat3_transpose(const double A[9], double B[9])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[3 * c + r] = A[3 * r + c];
}

static void skew(const double w[3], double K[9])
{
    K[0] = 0.0;   K[1] = -w[2]; K[2] = w[1];
    K[3] = w[2];  K[4] = 0.0;   K[5] = -w[0];
    K[6] = -w[1]; K[7] = w[0];  K[8] = 0.0;
}

/* ------------------------------------------------------------------------- */
/* Projection (Eq. 1 and the EWA step of Sec. 3.1).                           */

void orc_project_one(const orc_gaussians *G, int64_t g, const orc_view *V,
                     const orc_settings *S, orc_proj *P)
{
    const int64_t n = G->n;
    memset(P, 0, sizeof(*P));
    const double mu[3] = {G->means[g], G->means[n + g], G->means[2 * n + g]};
    const double q[4] = {G->quats[g], G->quats[n + g], G->quats[2 * n + g], G->quats[3 * n + g]};

    for (int k = 0; k < 3; ++k) P->s[k] = exp(G->log_scales[k * n + g]);
    P->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    P->a = 1.0 / (1.0 + exp(-G->opacity_logit[g]));
    if (!(P->qnorm > 0.0) || !isfinite(P->qnorm)) return;
    for (int k = 0; k < 4; ++k) P->qn[k] = q[k] / P->qnorm;
    quat_to_rot(P->qn, P->Rq);

    /* Eq. 1: Sigma = R S S^T R^T. */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += P->Rq[3 * r + k] * P->s[k] * P->s[k] * P->Rq[3 * c + k];
            P->Sig[3 * r + c] = acc;
        }

    /* Camera-frame centre m = R mu + t. */
    const double *T = V->T;
    for (int r = 0; r < 3; ++r)
        P->m[r] = T[4 * r + 0] * mu[0] + T[4 * r + 1] * mu[1] + T[4 * r + 2] * mu[2] + T[4 * r + 3];
    P->z = P->m[2];
    if (!(P->z > S->near_z) || !isfinite(P->z) || !isfinite(P->m[0]) || !isfinite(P->m[1])) return;

    P->u = V->fx * P->m[0] / P->z + V->cx;
    P->v = V->fy * P->m[1] / P->z + V->cy;

    /* Perspective Jacobian, with x/z and y/z clamped to jac_clamp times the half FOV. */
    const double limx = S->jac_clamp * (double)V->width / (2.0 * V->fx);
    const double limy = S->jac_clamp * (double)V->height / (2.0 * V->fy);
    double xz = P->m[0] / P->z, yz = P->m[1] / P->z;
    if (xz < -limx) { xz = -limx; P->clamp_x = 1; }
    if (xz > limx) { xz = limx; P->clamp_x = 1; }
    if (yz < -limy) { yz = -limy; P->clamp_y = 1; }
    if (yz > limy) { yz = limy; P->clamp_y = 1; }
    const double xt = xz * P->z, yt = yz * P->z;
    P->J[0] = V->fx / P->z; P->J[1] = 0.0; P->J[2] = -V->fx * xt / (P->z * P->z);
    P->J[3] = 0.0; P->J[4] = V->fy / P->z; P->J[5] = -V->fy * yt / (P->z * P->z);

    /* Sigma_c = W Sigma W^T with W the camera rotation. */
    double W[9], Wt[9], tmp[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) W[3 * r + c] = T[4 * r + c];
    mat3_transpose(W, Wt);
    mat3_mul(W, P->Sig, tmp);
    mat3_mul(tmp, Wt, P->Sigc);

    /* 2D covariance J Sigma_c J^T + eps2d I. */
    double c2[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += P->J[3 * r + k] * P->Sigc[3 * k + l] * P->J[3 * c + l];
            c2[2 * r + c] = acc;
        }
    P->cov2[0] = c2[0] + S->eps2d;
    P->cov2[1] = 0.5 * (c2[1] + c2[2]);
    P->cov2[2] = c2[3] + S->eps2d;
    const double det = P->cov2[0] * P->cov2[2] - P->cov2[1] * P->cov2[1];
    if (!(det > 0.0) || !isfinite(det)) return;
    P->Q[0] = P->cov2[2] / det;
    P->Q[1] = -P->cov2[1] / det;
    P->Q[2] = P->cov2[0] / det;

    /* Candidate box: the bounding box of the same ellipse at a level where the opacity is
     * widened by a relative 1e-4, plus one pixel on each side. */
    const double qc = 2.0 * log(P->a * (1.0 + 1e-4) / S->alpha_min);
    if (qc > 0.0) {
        const double rcx = sqrt(qc * P->cov2[0]), rcy = sqrt(qc * P->cov2[2]);
        double c0 = ceil(P->u - rcx) - 1.0, c1 = floor(P->u + rcx) + 1.0;
        double c2 = ceil(P->v - rcy) - 1.0, c3 = floor(P->v + rcy) + 1.0;
        if (c0 < 0.0) c0 = 0.0;
        if (c2 < 0.0) c2 = 0.0;
        if (c1 > V->width - 1) c1 = V->width - 1;
        if (c3 > V->height - 1) c3 = V->height - 1;
        if (c0 <= c1 && c2 <= c3) {
            P->cand = 1;
            P->crect[0] = (int32_t)c0; P->crect[1] = (int32_t)c1;
            P->crect[2] = (int32_t)c2; P->crect[3] = (int32_t)c3;
        }
    }

    /* Support: the alpha >= alpha_min ellipse {d : d^T Q d <= 2 ln(a / alpha_min)}. */
    if (!(P->a >= S->alpha_min)) return;
    const double qmax = 2.0 * log(P->a / S->alpha_min);
    P->rx = sqrt(qmax * P->cov2[0]);
    P->ry = sqrt(qmax * P->cov2[2]);
    P->bounds[0] = P->u - P->rx;
    P->bounds[1] = P->u + P->rx;
    P->bounds[2] = P->v - P->ry;
    P->bounds[3] = P->v + P->ry;
    double imin = ceil(P->bounds[0]), imax = floor(P->bounds[1]);
    double jmin = ceil(P->bounds[2]), jmax = floor(P->bounds[3]);
    if (imin < 0.0) imin = 0.0;
    if (jmin < 0.0) jmin = 0.0;
    if (imax > V->width - 1) imax = V->width - 1;
    if (jmax > V->height - 1) jmax = V->height - 1;
    if (imin > imax || jmin > jmax) return;
    P->rect[0] = (int32_t)imin; P->rect[1] = (int32_t)imax;
    P->rect[2] = (int32_t)jmin; P->rect[3] = (int32_t)jmax;
    P->visible = 1;
}

int orc_project(const orc_gaussians *G, const orc_view *V, const orc_settings *S, orc_proj *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < G->n; ++g) orc_project_one(G, g, V, S, &out[g]);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Per-pixel compositing (Eq. 2, Eq. 3, pointmaps).                           */

typedef struct {
    int64_t g;
    double z; /* the depth rounded to float32 (the ordering key, see the header) */
} cand_t;

/* Whether z lies within 8 double ulps of a midpoint between two float32 values. */
static int near_f32_midpoint(double z)
{
    const float f = (float)z;
    const double lo = 0.5 * ((double)f + (double)nextafterf(f, -INFINITY));
    const double hi = 0.5 * ((double)f + (double)nextafterf(f, INFINITY));
    const double tol = 8.0 * (nextafter(fabs(z), INFINITY) - fabs(z));
    return fabs(z - lo) <= tol || fabs(z - hi) <= tol;
}

static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->z < b->z) return -1;
    if (a->z > b->z) return 1;
    return (a->g < b->g) ? -1 : (a->g > b->g);
}

/* One fragment of a pixel's list. */
typedef struct {
    int64_t g;
    double alpha;   /* after clamp */
    double T;       /* transmittance before this fragment */
    double dx, dy;
    int32_t clamped;/* alpha hit alpha_max */
    int32_t pad;
} frag_t;

/* Per pixel row j, the Gaussians whose candidate box spans row j (in index order). */
typedef struct {
    int32_t height;
    int64_t *start; /* [height + 1] */
    int64_t *items;
} rows_t;

static void rows_free(rows_t *r)
{
    free(r->start);
    free(r->items);
    r->start = NULL;
    r->items = NULL;
}

static int rows_build(const orc_proj *P, int64_t n, int32_t height, rows_t *r)
{
    r->height = height;
    r->start = (int64_t *)calloc((size_t)height + 1, sizeof(int64_t));
    r->items = NULL;
    if (!r->start) return -1;
    for (int64_t g = 0; g < n; ++g)
        if (P[g].cand)
            for (int32_t j = P[g].crect[2]; j <= P[g].crect[3]; ++j) r->start[j + 1]++;
    for (int32_t j = 0; j < height; ++j) r->start[j + 1] += r->start[j];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(height > 0 ? height : 1));
    r->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(r->start[height] > 0 ? r->start[height] : 1));
    if (!cur || !r->items) {
        free(cur);
        rows_free(r);
        return -1;
    }
    memcpy(cur, r->start, sizeof(int64_t) * (size_t)height);
    for (int64_t g = 0; g < n; ++g)
        if (P[g].cand)
            for (int32_t j = P[g].crect[2]; j <= P[g].crect[3]; ++j) r->items[cur[j]++] = g;
    free(cur);
    return 0;
}

/* Candidates of pixel (i, j): the Gaussians whose candidate box contains it, sorted by
 * (float32 depth, g). */
static int64_t gather(const orc_proj *P, const rows_t *rows, int32_t i, int32_t j, cand_t *buf)
{
    int64_t c = 0;
    if (j < 0 || j >= rows->height) return 0;
    for (int64_t k = rows->start[j]; k < rows->start[j + 1]; ++k) {
        const int64_t g = rows->items[k];
        const orc_proj *p = &P[g];
        if (i < p->crect[0] || i > p->crect[1]) continue;
        buf[c].g = g;
        buf[c].z = (double)(float)p->z;
        ++c;
    }
    qsort(buf, (size_t)c, sizeof(cand_t), cand_cmp);
    return c;
}

/* Composite one pixel front to back.  Writes the contributing fragments to frags (may be
 * NULL) and returns their number. */
static int64_t composite(const orc_gaussians *G, const orc_proj *P, const orc_view *V,
                         const orc_settings *S, int32_t i, int32_t j, const cand_t *cand,
                         int64_t nc, orc_pixel *px, frag_t *frags)
{
    const int64_t n = G->n;
    double T = 1.0, C[3] = {0, 0, 0}, D = 0.0, A = 0.0, Xw[3] = {0, 0, 0}, Xc[3] = {0, 0, 0};
    double errT = 0.0; /* first-order float32 relative error bound on T */
    int64_t nf = 0;
    int amb = 0;
    int64_t looked = 0;
    double margin = INFINITY;
    const double ff = S->flag_factor;
    for (int64_t k = 0; k < nc; ++k) {
        const orc_proj *p = &P[cand[k].g];
        const double dx = (double)i - p->u, dy = (double)j - p->v;
        const double e = p->Q[0] * dx * dx + 2.0 * p->Q[1] * dx * dy + p->Q[2] * dy * dy;
        const double gval = exp(-0.5 * e);
        const double a_pre = p->a * gval;
        /* First-order float32 error bound of alpha (relative): 8 roundings of the
         * quadratic form's terms and 8 of the exponential and the products. */
        const double sabs = fabs(p->Q[0]) * dx * dx + 2.0 * fabs(p->Q[1] * dx * dy) + fabs(p->Q[2]) * dy * dy;
        const double erra = 8.0 * ORC_EPS32 * sabs + 8.0 * ORC_EPS32;
        ++looked;
        const double r_min = fabs(a_pre - S->alpha_min) / (erra * S->alpha_min);
        if (r_min < margin) margin = r_min;
        if (r_min <= ff) amb |= 1;
        if (a_pre < S->alpha_min) continue;
        double alpha = a_pre;
        int clamped = 0;
        const double r_max = fabs(a_pre - S->alpha_max) / (erra * S->alpha_max);
        if (r_max < margin) margin = r_max;
        if (r_max <= ff) amb |= 4;
        if (alpha > S->alpha_max) { alpha = S->alpha_max; clamped = 1; }
        const double Tn = T * (1.0 - alpha);
        /* T picks up alpha's error through 1 - alpha, and one rounding per step. */
        const double errTn = errT + (clamped ? 0.0 : erra * alpha / (1.0 - alpha)) + ORC_EPS32;
        const double r_t = fabs(Tn - S->t_min) / (errTn * S->t_min);
        if (r_t < margin) margin = r_t;
        if (r_t <= ff) amb |= 2;
        if (Tn < S->t_min) break;
        if (near_f32_midpoint(p->z)) amb |= 8;

        const double w = alpha * T;
        const int64_t g = cand[k].g;
        for (int c = 0; c < 3; ++c) C[c] += w * G->rgb[c * n + g];
        D += w * p->z;
        A += w;
        for (int c = 0; c < 3; ++c) Xw[c] += w * G->means[c * n + g];
        for (int c = 0; c < 3; ++c) Xc[c] += w * p->m[c];
        if (frags) {
            frags[nf].g = g;
            frags[nf].alpha = alpha;
            frags[nf].T = T;
            frags[nf].dx = dx;
            frags[nf].dy = dy;
            frags[nf].clamped = clamped;
        }
        ++nf;
        T = Tn;
        errT = errTn;
    }
    if (px) {
        for (int c = 0; c < 3; ++c) px->rgb[c] = C[c] + T * S->bg[c];
        px->depth = D;
        px->alpha = 1.0 - T;
        for (int c = 0; c < 3; ++c) px->pm_world[c] = Xw[c];
        for (int c = 0; c < 3; ++c) px->pm_cam[c] = Xc[c];
        /* Eq. 5: X = (D (i - cx) / fx, D (j - cy) / fy, D). */
        px->pm_eq5[0] = D * ((double)i - V->cx) / V->fx;
        px->pm_eq5[1] = D * ((double)j - V->cy) / V->fy;
        px->pm_eq5[2] = D;
        px->T_final = T;
        px->n_frag = (int32_t)nf;
        px->n_cand = (int32_t)looked;
        px->ambiguous = amb;
        px->margin = margin;
        (void)A;
    }
    return nf;
}

static int64_t count_cand(const orc_proj *P, int64_t n)
{
    int64_t c = 0;
    for (int64_t g = 0; g < n; ++g) c += P[g].cand ? 1 : 0;
    return c;
}

/* Render npix pixels (pix = [npix][2] as (i, j)); proj must come from orc_project. */
int orc_render(const orc_gaussians *G, const orc_view *V, const orc_settings *S,
               const orc_proj *proj, int64_t npix, const int32_t *pix, orc_pixel *out)
{
    const int64_t ncand = count_cand(proj, G->n);
    rows_t rows;
    if (rows_build(proj, G->n, V->height, &rows)) return -1;
    int err = 0;
#pragma omp parallel
    {
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * (size_t)(ncand > 0 ? ncand : 1));
        if (!buf) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            if (!buf) continue;
            const int32_t i = pix[2 * p], j = pix[2 * p + 1];
            const int64_t nc = gather(proj, &rows, i, j, buf);
            composite(G, proj, V, S, i, j, buf, nc, &out[p], NULL);
        }
        free(buf);
    }
    rows_free(&rows);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Frozen-decision trace and replay (for finite differences).                  */

/* Records, per pixel, the contributing fragments (Gaussian index and whether alpha was
 * clamped at alpha_max).  offsets has npix + 1 entries.  Returns the total number of
 * fragments, or -(needed) if cap is too small. */
int64_t orc_trace(const orc_gaussians *G, const orc_view *V, const orc_settings *S,
                  const orc_proj *proj, int64_t npix, const int32_t *pix, int64_t cap,
                  int64_t *offsets, int64_t *frag_g, int8_t *frag_clamped)
{
    const int64_t ncand = count_cand(proj, G->n);
    int64_t *counts = (int64_t *)calloc((size_t)npix + 1, sizeof(int64_t));
    rows_t rows;
    if (!counts || rows_build(proj, G->n, V->height, &rows)) {
        free(counts);
        return 0;
    }
    const size_t nb = (size_t)(ncand > 0 ? ncand : 1);
#pragma omp parallel
    {
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * nb);
        frag_t *fr = (frag_t *)malloc(sizeof(frag_t) * nb);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            const int64_t nc = gather(proj, &rows, pix[2 * p], pix[2 * p + 1], buf);
            counts[p] = composite(G, proj, V, S, pix[2 * p], pix[2 * p + 1], buf, nc, NULL, fr);
        }
        free(buf);
        free(fr);
    }
    int64_t total = 0;
    for (int64_t p = 0; p < npix; ++p) {
        offsets[p] = total;
        total += counts[p];
    }
    offsets[npix] = total;
    free(counts);
    if (total > cap) {
        rows_free(&rows);
        return -total;
    }
#pragma omp parallel
    {
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * nb);
        frag_t *fr = (frag_t *)malloc(sizeof(frag_t) * nb);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            const int64_t nc = gather(proj, &rows, pix[2 * p], pix[2 * p + 1], buf);
            const int64_t nf = composite(G, proj, V, S, pix[2 * p], pix[2 * p + 1], buf, nc, NULL, fr);
            for (int64_t k = 0; k < nf; ++k) {
                frag_g[offsets[p] + k] = fr[k].g;
                frag_clamped[offsets[p] + k] = (int8_t)fr[k].clamped;
            }
        }
        free(buf);
        free(fr);
    }
    rows_free(&rows);
    return total;
}

/* Evaluate L = sum_p g(p) . out(p) on a frozen trace: the same fragments in the same
 * order, the same alpha clamps and the same Jacobian clamp flags (clamp_xy[2 g] and
 * [2 g + 1]) as the base point; only the smooth arithmetic is re-evaluated.
 * pointmap_frame: 0 world, 1 camera, 2 Eq. 5 back-projection.  Upstream gradients
 * are [npix][3], [npix], [npix], [npix][3]. */
double orc_replay_loss(const orc_gaussians *G, const orc_view *V, const orc_settings *S,
                       const int8_t *clamp_xy, int32_t pointmap_frame, int64_t npix,
                       const int32_t *pix, const int64_t *offsets, const int64_t *frag_g,
                       const int8_t *frag_clamped, const double *g_rgb, const double *g_depth,
                       const double *g_alpha, const double *g_pm)
{
    const int64_t n = G->n;
    /* Re-project with the frozen Jacobian clamp decisions. */
    orc_proj *P = (orc_proj *)malloc(sizeof(orc_proj) * (size_t)n);
    if (!P) return NAN;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        orc_project_one(G, g, V, S, &P[g]);
        /* Override the clamp decision with the frozen one and recompute J, cov2, Q. */
        orc_proj *p = &P[g];
        if (!(p->z != 0.0) || !(p->qnorm > 0.0)) continue;
        const double limx = S->jac_clamp * (double)V->width / (2.0 * V->fx);
        const double limy = S->jac_clamp * (double)V->height / (2.0 * V->fy);
        double xz = p->m[0] / p->z, yz = p->m[1] / p->z;
        if (clamp_xy[2 * g]) xz = xz < 0 ? -limx : limx;
        if (clamp_xy[2 * g + 1]) yz = yz < 0 ? -limy : limy;
        if (!clamp_xy[2 * g]) xz = p->m[0] / p->z;
        if (!clamp_xy[2 * g + 1]) yz = p->m[1] / p->z;
        const double xt = xz * p->z, yt = yz * p->z;
        p->J[0] = V->fx / p->z; p->J[2] = -V->fx * xt / (p->z * p->z);
        p->J[4] = V->fy / p->z; p->J[5] = -V->fy * yt / (p->z * p->z);
        double c2[4];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += p->J[3 * r + k] * p->Sigc[3 * k + l] * p->J[3 * c + l];
                c2[2 * r + c] = acc;
            }
        p->cov2[0] = c2[0] + S->eps2d;
        p->cov2[1] = 0.5 * (c2[1] + c2[2]);
        p->cov2[2] = c2[3] + S->eps2d;
        const double det = p->cov2[0] * p->cov2[2] - p->cov2[1] * p->cov2[1];
        p->Q[0] = p->cov2[2] / det;
        p->Q[1] = -p->cov2[1] / det;
        p->Q[2] = p->cov2[0] / det;
    }
    double L = 0.0;
#pragma omp parallel for reduction(+ : L) schedule(dynamic, 16)
    for (int64_t px = 0; px < npix; ++px) {
        const int32_t i = pix[2 * px], j = pix[2 * px + 1];
        double T = 1.0, C[3] = {0, 0, 0}, D = 0.0, Xw[3] = {0, 0, 0}, Xc[3] = {0, 0, 0};
        for (int64_t k = offsets[px]; k < offsets[px + 1]; ++k) {
            const int64_t g = frag_g[k];
            const orc_proj *p = &P[g];
            double alpha;
            if (frag_clamped[k]) {
                alpha = S->alpha_max;
            } else {
                const double dx = (double)i - p->u, dy = (double)j - p->v;
                const double e = p->Q[0] * dx * dx + 2.0 * p->Q[1] * dx * dy + p->Q[2] * dy * dy;
                alpha = p->a * exp(-0.5 * e);
            }
            const double w = alpha * T;
            for (int c = 0; c < 3; ++c) C[c] += w * G->rgb[c * n + g];
            D += w * p->z;
            for (int c = 0; c < 3; ++c) Xw[c] += w * G->means[c * n + g];
            for (int c = 0; c < 3; ++c) Xc[c] += w * p->m[c];
            T *= (1.0 - alpha);
        }
        double l = 0.0;
        for (int c = 0; c < 3; ++c) l += g_rgb[3 * px + c] * (C[c] + T * S->bg[c]);
        l += g_depth[px] * D;
        l += g_alpha[px] * (1.0 - T);
        double X[3];
        for (int c = 0; c < 3; ++c) X[c] = pointmap_frame == 0 ? Xw[c] : Xc[c];
        if (pointmap_frame == 2) {
            X[0] = D * ((double)i - V->cx) / V->fx;
            X[1] = D * ((double)j - V->cy) / V->fy;
            X[2] = D;
        }
        for (int c = 0; c < 3; ++c) l += g_pm[3 * px + c] * X[c];
        L += l;
    }
    free(P);
    return L;
}

/* ------------------------------------------------------------------------- */
/* Analytic backward (hand-derived from the forward above).                   */

/* Per-Gaussian accumulators of the image-plane gradients. */
typedef struct {
    double gu, gv;      /* mean2D */
    double gQ[3];       /* conic xx, xy (the single off-diagonal value), yy */
    double ga;          /* activated opacity */
    double gz;          /* depth as composited in Eq. 3 */
    double gc[3];       /* colour */
    double gpw[3];      /* world-frame composited centre */
    double gpc[3];      /* camera-frame composited centre */
} acc2d_t;

int orc_backward(const orc_gaussians *G, const orc_view *V, const orc_settings *S,
                 const orc_proj *proj, int32_t pointmap_frame, int64_t npix, const int32_t *pix,
                 const double *g_rgb, const double *g_depth, const double *g_alpha,
                 const double *g_pm, orc_grads *out)
{
    const int64_t n = G->n;
    const int64_t ncand = count_cand(proj, n);
    rows_t rows;
    if (rows_build(proj, n, V->height, &rows)) return -1;
    /* The Gaussians some requested pixel has as a candidate get a slot in the per-thread
     * accumulators (a crop of a large view touches few of them). */
    int8_t *touched = (int8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!touched || !slot) {
        free(touched); free(slot); rows_free(&rows);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t px = 0; px < npix; ++px) {
        const int32_t i = pix[2 * px], j = pix[2 * px + 1];
        if (j < 0 || j >= rows.height) continue;
        for (int64_t k = rows.start[j]; k < rows.start[j + 1]; ++k) {
            const int64_t g = rows.items[k];
            if (i < proj[g].crect[0] || i > proj[g].crect[1] || touched[g]) continue;
#pragma omp atomic write
            touched[g] = 1;
        }
    }
    int64_t nslot = 0;
    for (int64_t g = 0; g < n; ++g) slot[g] = touched[g] ? nslot++ : -1;
    free(touched);

    /* Pixels are split statically over the threads; each thread sums its pixels'
     * image-plane gradients into its own accumulators, which are then added in thread
     * order, so the result depends only on the thread count. */
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    acc2d_t *acc = (acc2d_t *)calloc((size_t)nthreads * (size_t)(nslot > 0 ? nslot : 1), sizeof(acc2d_t));
    if (!acc) {
        free(slot); rows_free(&rows);
        return -1;
    }
    int err = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        acc2d_t *mine = acc + (size_t)tid * (size_t)(nslot > 0 ? nslot : 1);
        const size_t nb = (size_t)(ncand > 0 ? ncand : 1);
        cand_t *buf = (cand_t *)malloc(sizeof(cand_t) * nb);
        frag_t *fr = (frag_t *)malloc(sizeof(frag_t) * nb);
        double *sk = (double *)malloc(sizeof(double) * nb);
        if (!buf || !fr || !sk) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(static)
        for (int64_t px = 0; px < npix; ++px) {
            if (!buf || !fr || !sk) continue;
            const int32_t i = pix[2 * px], j = pix[2 * px + 1];
            double gC[3] = {g_rgb[3 * px], g_rgb[3 * px + 1], g_rgb[3 * px + 2]};
            double gD = g_depth[px], gA = g_alpha[px];
            double gX[3] = {g_pm[3 * px], g_pm[3 * px + 1], g_pm[3 * px + 2]};
            if (gC[0] == 0.0 && gC[1] == 0.0 && gC[2] == 0.0 && gD == 0.0 && gA == 0.0 &&
                gX[0] == 0.0 && gX[1] == 0.0 && gX[2] == 0.0)
                continue;
            if (pointmap_frame == 2) {
                /* Eq. 5 pointmap is a function of D only. */
                gD += gX[0] * ((double)i - V->cx) / V->fx + gX[1] * ((double)j - V->cy) / V->fy + gX[2];
                gX[0] = gX[1] = gX[2] = 0.0;
            }
            const int64_t nc = gather(proj, &rows, i, j, buf);
            const int64_t nf = composite(G, proj, V, S, i, j, buf, nc, NULL, fr);
            double Tfin = 1.0;
            for (int64_t k = 0; k < nf; ++k) Tfin *= (1.0 - fr[k].alpha);

            /* s_k = g . e_k with e_k the per-fragment value composited into each channel. */
            for (int64_t k = 0; k < nf; ++k) {
                const int64_t g = fr[k].g;
                const orc_proj *p = &proj[g];
                double sv = 0.0;
                for (int c = 0; c < 3; ++c) sv += gC[c] * G->rgb[c * n + g];
                sv += gD * p->z + gA;
                for (int c = 0; c < 3; ++c)
                    sv += gX[c] * (pointmap_frame == 0 ? G->means[c * n + g] : p->m[c]);
                sk[k] = sv;
            }
            /* Suffix sums, accumulated back to front: after_k = sum_{j > k} w_j s_j. */
            double after = 0.0;
            const double bgterm = Tfin * (gC[0] * S->bg[0] + gC[1] * S->bg[1] + gC[2] * S->bg[2]);
            for (int64_t k = nf - 1; k >= 0; --k) {
                const frag_t *f = &fr[k];
                const int64_t g = f->g;
                const orc_proj *p = &proj[g];
                const double w = f->alpha * f->T;
                acc2d_t *ag = &mine[slot[g]];
                for (int c = 0; c < 3; ++c) ag->gc[c] += w * gC[c];
                ag->gz += w * gD;
                if (pointmap_frame == 0)
                    for (int c = 0; c < 3; ++c) ag->gpw[c] += w * gX[c];
                else
                    for (int c = 0; c < 3; ++c) ag->gpc[c] += w * gX[c];
                const double dLda = f->T * sk[k] - (after + bgterm) / (1.0 - f->alpha);
                if (!f->clamped) {
                    /* alpha = a exp(-e/2), e = Qxx dx^2 + 2 Qxy dx dy + Qyy dy^2. */
                    const double dx = f->dx, dy = f->dy;
                    const double dLde = dLda * (-0.5 * f->alpha);
                    ag->ga += dLda * f->alpha / p->a;
                    ag->gQ[0] += dLde * dx * dx;
                    ag->gQ[1] += dLde * 2.0 * dx * dy;
                    ag->gQ[2] += dLde * dy * dy;
                    /* de/du = -2 (Qxx dx + Qxy dy), de/dv = -2 (Qxy dx + Qyy dy). */
                    ag->gu += dLde * (-2.0) * (p->Q[0] * dx + p->Q[1] * dy);
                    ag->gv += dLde * (-2.0) * (p->Q[1] * dx + p->Q[2] * dy);
                }
                after += w * sk[k];
            }
        }
        free(buf);
        free(fr);
        free(sk);
    }
    rows_free(&rows);
    if (err) {
        free(acc); free(slot);
        return -1;
    }
    /* Thread partials, added in thread order. */
    for (int t = 1; t < nthreads; ++t) {
        const acc2d_t *src = acc + (size_t)t * (size_t)nslot;
        for (int64_t k = 0; k < nslot; ++k) {
            const double *a = (const double *)&src[k];
            double *b = (double *)&acc[k];
            for (size_t q = 0; q < sizeof(acc2d_t) / sizeof(double); ++q) b[q] += a[q];
        }
    }

    /* Image plane -> Gaussian parameters and pose. */
    double pose[6] = {0, 0, 0, 0, 0, 0};
    const double *T = V->T;
    double W[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) W[3 * r + c] = T[4 * r + c];
    for (int64_t g = 0; g < n; ++g) {
        const orc_proj *p = &proj[g];
        if (!p->visible || slot[g] < 0) continue;
        const acc2d_t *ag = &acc[slot[g]];
        for (int c = 0; c < 3; ++c) out->rgb[c * n + g] += ag->gc[c];
        out->opacity_logit[g] += ag->ga * p->a * (1.0 - p->a);

        /* Conic Q = [C, -B, A] / (AC - B^2) for cov2 = [[A, B], [B, C]]. */
        const double A = p->cov2[0], B = p->cov2[1], Cc = p->cov2[2];
        const double d = A * Cc - B * B, d2 = d * d;
        const double gA2 = ag->gQ[0] * (-Cc * Cc / d2) + ag->gQ[1] * (B * Cc / d2) + ag->gQ[2] * (1.0 / d - A * Cc / d2);
        const double gB2 = ag->gQ[0] * (2.0 * B * Cc / d2) + ag->gQ[1] * (-1.0 / d - 2.0 * B * B / d2) + ag->gQ[2] * (2.0 * A * B / d2);
        const double gC2 = ag->gQ[0] * (1.0 / d - Cc * A / d2) + ag->gQ[1] * (B * A / d2) + ag->gQ[2] * (-A * A / d2);

        /* cov2 = J Sigc J^T: A = j0 Sigc j0, B = j0 Sigc j1, C = j1 Sigc j1. */
        const double *j0 = &p->J[0], *j1 = &p->J[3];
        double Gc[9];
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l)
                Gc[3 * k + l] = gA2 * j0[k] * j0[l] + gB2 * j0[k] * j1[l] + gC2 * j1[k] * j1[l];
        double Sj0[3], Sj1[3];
        for (int k = 0; k < 3; ++k) {
            Sj0[k] = p->Sigc[3 * k] * j0[0] + p->Sigc[3 * k + 1] * j0[1] + p->Sigc[3 * k + 2] * j0[2];
            Sj1[k] = p->Sigc[3 * k] * j1[0] + p->Sigc[3 * k + 1] * j1[1] + p->Sigc[3 * k + 2] * j1[2];
        }
        double gJ[6];
        for (int k = 0; k < 3; ++k) {
            gJ[k] = gA2 * 2.0 * Sj0[k] + gB2 * Sj1[k];
            gJ[3 + k] = gB2 * Sj0[k] + gC2 * 2.0 * Sj1[k];
        }

        /* Camera-frame centre gradient: projection, Jacobian, depth and pointmap terms. */
        const double fx = V->fx, fy = V->fy, z = p->z, mx = p->m[0], my = p->m[1];
        double gm[3] = {0, 0, 0};
        gm[0] += ag->gu * fx / z;
        gm[2] += ag->gu * (-fx * mx / (z * z));
        gm[1] += ag->gv * fy / z;
        gm[2] += ag->gv * (-fy * my / (z * z));
        gm[2] += ag->gz;
        gm[2] += gJ[0] * (-fx / (z * z)) + gJ[4] * (-fy / (z * z));
        if (!p->clamp_x) {
            gm[0] += gJ[2] * (-fx / (z * z));
            gm[2] += gJ[2] * (2.0 * fx * mx / (z * z * z));
        } else {
            const double cxz = (mx / z < 0.0 ? -1.0 : 1.0) * S->jac_clamp * (double)V->width / (2.0 * fx);
            gm[2] += gJ[2] * (fx * cxz / (z * z));
        }
        if (!p->clamp_y) {
            gm[1] += gJ[5] * (-fy / (z * z));
            gm[2] += gJ[5] * (2.0 * fy * my / (z * z * z));
        } else {
            const double cyz = (my / z < 0.0 ? -1.0 : 1.0) * S->jac_clamp * (double)V->height / (2.0 * fy);
            gm[2] += gJ[5] * (fy * cyz / (z * z));
        }
        for (int c = 0; c < 3; ++c) gm[c] += ag->gpc[c];

        /* mu: m = W mu + t. */
        for (int c = 0; c < 3; ++c)
            out->means[c * n + g] += W[c] * gm[0] + W[3 + c] * gm[1] + W[6 + c] * gm[2] + ag->gpw[c];

        /* Pose: m(xi) = Exp(xi) m, Sigc(xi) = R(phi) Sigc R(phi)^T, to first order. */
        for (int c = 0; c < 3; ++c) pose[c] += gm[c];
        for (int ax = 0; ax < 3; ++ax) {
            double e[3] = {0, 0, 0}, K[9], KS[9], SK[9];
            e[ax] = 1.0;
            skew(e, K);
            /* dm = e x m */
            const double dm[3] = {e[1] * p->m[2] - e[2] * p->m[1], e[2] * p->m[0] - e[0] * p->m[2],
                                  e[0] * p->m[1] - e[1] * p->m[0]};
            double s = gm[0] * dm[0] + gm[1] * dm[1] + gm[2] * dm[2];
            /* dSigc = K Sigc - Sigc K */
            mat3_mul(K, p->Sigc, KS);
            mat3_mul(p->Sigc, K, SK);
            for (int q = 0; q < 9; ++q) s += Gc[q] * (KS[q] - SK[q]);
            pose[3 + ax] += s;
        }

        /* Sigma = W^T Sigc W inverted: dL/dSigma = W^T Gc W. */
        double Wt[9], tmp[9], GS[9];
        mat3_transpose(W, Wt);
        mat3_mul(Wt, Gc, tmp);
        mat3_mul(tmp, W, GS);
        /* Sigma = M M^T with M = Rq diag(s): dL/dM = (GS + GS^T) M. */
        double M[9], gM[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[3 * r + c] = p->Rq[3 * r + c] * p->s[c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc_ = 0.0;
                for (int b = 0; b < 3; ++b) acc_ += (GS[3 * r + b] + GS[3 * b + r]) * M[3 * b + c];
                gM[3 * r + c] = acc_;
            }
        double gRq[9];
        for (int c = 0; c < 3; ++c) {
            double gs = 0.0;
            for (int r = 0; r < 3; ++r) gs += gM[3 * r + c] * p->Rq[3 * r + c];
            out->log_scales[c * n + g] += gs * p->s[c];
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) gRq[3 * r + c] = gM[3 * r + c] * p->s[c];
        double dR[9][4];
        quat_to_rot_jac(p->qn, dR);
        double gqn[4] = {0, 0, 0, 0};
        for (int e = 0; e < 9; ++e)
            for (int k = 0; k < 4; ++k) gqn[k] += gRq[e] * dR[e][k];
        /* q_hat = q / |q|: dL/dq = (g - q_hat (q_hat . g)) / |q|. */
        const double dot = gqn[0] * p->qn[0] + gqn[1] * p->qn[1] + gqn[2] * p->qn[2] + gqn[3] * p->qn[3];
        for (int k = 0; k < 4; ++k) out->quats[k * n + g] += (gqn[k] - p->qn[k] * dot) / p->qnorm;
    }
    for (int c = 0; c < 6; ++c) out->pose[c] += pose[c];
    free(acc);
    free(slot);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Tile lists of the supports (the tile-based rasterization of Sec. 3.1).      */

/* Two definitions, both from the support of O7 alone, for tile size B (tiles numbered
 * row-major, tiles_x = ceil(W / B)):
 *   rect:  Gaussian g is in tile t when t holds a pixel of g's support box;
 *   exact: g is in tile t when t holds a pixel centre (i, j) of the view at which
 *          e = d^T Q d <= q = 2 ln(a / alpha_min), i.e. where the Gaussian's alpha before
 *          the clamp reaches alpha_min.
 * Every pixel centre with e <= q lies in the support box, so exact is a subset of rect,
 * and a fragment the per-pixel compositing keeps always has its Gaussian in the exact
 * list of its pixel's tile.  Writes the rect pairs ordered by (tile, float32 depth,
 * index), the compositing order, and per
 * pair ratio = (min over the tile's pixels of the box of e) / q, so that the pair is in
 * the exact set iff ratio <= 1.  Returns the number of pairs, or -(needed) if cap is
 * short. */
int64_t orc_tile_sets(const orc_proj *P, int64_t n, int32_t width, int32_t height, int32_t B,
                      double alpha_min, int64_t cap, int32_t *tile_out, int64_t *g_out, double *ratio_out)
{
    const int32_t tx = (width + B - 1) / B, ty = (height + B - 1) / B;
    const int64_t ntiles = (int64_t)tx * ty;
    int64_t *cnt = (int64_t *)calloc((size_t)ntiles + 1, sizeof(int64_t));
    if (!cnt) return 0;
    for (int64_t g = 0; g < n; ++g) {
        const orc_proj *p = &P[g];
        if (!p->visible) continue;
        for (int32_t y = p->rect[2] / B; y <= p->rect[3] / B; ++y)
            for (int32_t x = p->rect[0] / B; x <= p->rect[1] / B; ++x) cnt[(int64_t)y * tx + x + 1]++;
    }
    for (int64_t t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
    const int64_t total = cnt[ntiles];
    if (total > cap) {
        free(cnt);
        return -total;
    }
    typedef struct {
        int64_t g;
        double z, ratio;
    } entry_t;
    entry_t *tmp = (entry_t *)malloc(sizeof(entry_t) * (size_t)(total > 0 ? total : 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntiles > 0 ? ntiles : 1));
    if (!tmp || !cur) {
        free(tmp); free(cur); free(cnt);
        return 0;
    }
    memcpy(cur, cnt, sizeof(int64_t) * (size_t)ntiles);
    for (int64_t g = 0; g < n; ++g) {
        const orc_proj *p = &P[g];
        if (!p->visible) continue;
        const double q = 2.0 * log(p->a / alpha_min);
        for (int32_t y = p->rect[2] / B; y <= p->rect[3] / B; ++y)
            for (int32_t x = p->rect[0] / B; x <= p->rect[1] / B; ++x) {
                /* Smallest e over the pixel centres of this tile inside the box. */
                double emin = INFINITY;
                const int32_t ia = x * B > p->rect[0] ? x * B : p->rect[0];
                const int32_t ib = x * B + B - 1 < p->rect[1] ? x * B + B - 1 : p->rect[1];
                const int32_t ja = y * B > p->rect[2] ? y * B : p->rect[2];
                const int32_t jb = y * B + B - 1 < p->rect[3] ? y * B + B - 1 : p->rect[3];
                for (int32_t j = ja; j <= jb; ++j)
                    for (int32_t i = ia; i <= ib; ++i) {
                        const double dx = (double)i - p->u, dy = (double)j - p->v;
                        const double e = p->Q[0] * dx * dx + 2.0 * p->Q[1] * dx * dy + p->Q[2] * dy * dy;
                        if (e < emin) emin = e;
                    }
                const int64_t t = (int64_t)y * tx + x;
                tmp[cur[t]].g = g;
                tmp[cur[t]].z = (double)(float)p->z;
                tmp[cur[t]].ratio = emin / q;
                cur[t]++;
            }
    }
    for (int64_t t = 0; t < ntiles; ++t) {
        /* Order of a tile's list: (float32 depth, index), by insertion (lists are short). */
        for (int64_t k = cnt[t] + 1; k < cnt[t + 1]; ++k) {
            const entry_t e = tmp[k];
            int64_t m = k - 1;
            while (m >= cnt[t] && (tmp[m].z > e.z || (tmp[m].z == e.z && tmp[m].g > e.g))) {
                tmp[m + 1] = tmp[m];
                --m;
            }
            tmp[m + 1] = e;
        }
        for (int64_t k = cnt[t]; k < cnt[t + 1]; ++k) {
            tile_out[k] = (int32_t)t;
            g_out[k] = tmp[k].g;
            ratio_out[k] = tmp[k].ratio;
        }
    }
    free(tmp);
    free(cur);
    free(cnt);
    return total;
}

/* ------------------------------------------------------------------------- */
/* SE(3) exponential: T_out = Exp(xi) T_in, xi = (rho, phi).                    */

void orc_se3_exp_left(const double xi[6], const double T_in[12], double T_out[12])
{
    const double *rho = xi, *phi = xi + 3;
    const double th = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    double K[9], K2[9], R[9], Vm[9];
    skew(phi, K);
    mat3_mul(K, K, K2);
    double A, Bc, Cc;
    if (th < 1e-8) {
        A = 1.0 - th * th / 6.0;
        Bc = 0.5 - th * th / 24.0;
        Cc = 1.0 / 6.0 - th * th / 120.0;
    } else {
        A = sin(th) / th;
        Bc = (1.0 - cos(th)) / (th * th);
        Cc = (th - sin(th)) / (th * th * th);
    }
    for (int q = 0; q < 9; ++q) {
        const double I = (q % 4 == 0) ? 1.0 : 0.0;
        R[q] = I + A * K[q] + Bc * K2[q];
        Vm[q] = I + Bc * K[q] + Cc * K2[q];
    }
    double t[3];
    for (int r = 0; r < 3; ++r) t[r] = Vm[3 * r] * rho[0] + Vm[3 * r + 1] * rho[1] + Vm[3 * r + 2] * rho[2];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            T_out[4 * r + c] = R[3 * r] * T_in[c] + R[3 * r + 1] * T_in[4 + c] + R[3 * r + 2] * T_in[8 + c];
        T_out[4 * r + 3] = R[3 * r] * T_in[3] + R[3 * r + 1] * T_in[7] + R[3 * r + 2] * T_in[11] + t[r];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel regions (the CPU baseline's one-thread run). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
