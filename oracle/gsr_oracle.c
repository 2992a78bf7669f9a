/*
 * FP64 CPU oracle for the differentiable Gaussian-splatting rasterizer of the
 * global map optimisation (paper, Sec. III-C "Optimization": standard
 * differentiable splatting by front-to-back alpha compositing, depth by the
 * same compositing weights (Eq. 8), losses Eq. 9-12, sparse optimizer).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously-correct
 * statement of what the GPU path computes.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or constant table with the HIP library: every formula below is
 * written out from the definition it cites.
 *
 * Everything is double precision.  Inputs are double arrays (callers convert
 * float32 inputs exactly), so finite differences can perturb them.
 *
 * Definitions followed (the paper delegates them to "standard" splatting; the
 * readings are listed with the design notes):
 *   camera   p = R mu + t, pinhole u = fx x/z + cx, v = fy y/z + cy,
 *            pixel (i, j) sampled at its centre (i + 1/2, j + 1/2).
 *   cov      Sigma = Rq S S^T Rq^T, S = diag(exp(log_scale)), Rq from the
 *            normalised (w, x, y, z) quaternion; Sigma_c = R Sigma R^T.
 *   EWA      J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]] with tx = x/z and
 *            ty = y/z clamped to +-1.3 W/(2 fx), +-1.3 H/(2 fy);
 *            Sigma' = J Sigma_c J^T + 0.3 I;  Q = Sigma'^{-1}.
 *   opacity  o = 1 / (1 + exp(-omega)).
 *   colour   rgb = max(0, sum_k Y_k(d) h_k + 1/2), d = (mu - c)/|mu - c|,
 *            c = -R^T t; Y_k real orthonormal SH without Condon-Shortley phase.
 *   alpha    a_raw = o exp(-1/2 D^T Q D), D = pixel centre - (u, v); a pair
 *            contributes iff a_raw >= 1/255; a = min(0.99, a_raw).
 *   order    contributors by ascending (depth key, Gaussian index), the depth key being the
 *            camera depth rounded to float32 (the 32-bit key of the tile binning sort).
 *   blend    T = 1; for each: T' = T (1 - a); stop if T' < 1e-4 (that one is
 *            not composited); C += a T rgb; D += a T z (Eq. 8); T = T'.
 *            Output C + T bg, D, T.
 *   backward exact gradient of the above with every discrete decision held
 *            (visibility, contributor set and order, termination, the 0.99
 *            clamp, the SH clamp and the guard-band clamp), including the
 *            camera pose under a left perturbation T <- Exp(xi) T,
 *            xi = (rho, phi), p -> p + rho + phi x p.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double R[9];      /* world -> camera rotation, row-major */
    double t[3];
    double fx, fy, cx, cy;
    double z_near;
    double bg[3];
    int32_t width, height;
} orc_camera;

typedef struct {
    const double *means;          /* [3][n] */
    const double *log_scales;     /* [3][n] */
    const double *quats;          /* [4][n] (w, x, y, z), not necessarily unit */
    const double *opacity_logits; /* [n] */
    const double *sh;             /* [3K][n], row k*3+ch */
    int64_t n;
    int32_t sh_degree;
} orc_gaussians;

#define ORC_ALPHA_MIN (1.0 / 255.0)
#define ORC_ALPHA_MAX 0.99
#define ORC_T_MIN 1e-4
#define ORC_LOWPASS 0.3
#define ORC_GUARD 1.3

/* ------------------------------------------------------------------------------------------ */
/* Real spherical harmonics, orthonormal on the sphere, no Condon-Shortley phase,             */
/* ordered (l, m = -l..l), written as polynomials of the unit direction (x, y, z).             */
/* ------------------------------------------------------------------------------------------ */
static void sh_consts(double c[10]) {
    c[0] = 0.5 / sqrt(M_PI);              /* l=0 */
    c[1] = sqrt(3.0 / (4.0 * M_PI));      /* l=1 */
    c[2] = 0.5 * sqrt(15.0 / M_PI);       /* xy, yz, xz */
    c[3] = 0.25 * sqrt(5.0 / M_PI);       /* 3z^2-1 */
    c[4] = 0.25 * sqrt(15.0 / M_PI);      /* x^2-y^2 */
    c[5] = 0.25 * sqrt(35.0 / (2 * M_PI));/* y(3x^2-y^2), x(x^2-3y^2) */
    c[6] = 0.5 * sqrt(105.0 / M_PI);      /* xyz */
    c[7] = 0.25 * sqrt(21.0 / (2 * M_PI));/* y(5z^2-1), x(5z^2-1) */
    c[8] = 0.25 * sqrt(7.0 / M_PI);       /* z(5z^2-3) */
    c[9] = 0.25 * sqrt(105.0 / M_PI);     /* z(x^2-y^2) */
}

/* Y[k] and, if dY != NULL, the gradient dY[k][3] of the polynomial in (x, y, z). */
static int sh_eval(int degree, const double d[3], double *Y, double (*dY)[3]) {
    double c[10];
    sh_consts(c);
    const double x = d[0], y = d[1], z = d[2];
    int K = (degree + 1) * (degree + 1);
    double g[16][3];
    memset(g, 0, sizeof g);
    Y[0] = c[0];
    if (degree >= 1) {
        Y[1] = c[1] * y; g[1][1] = c[1];
        Y[2] = c[1] * z; g[2][2] = c[1];
        Y[3] = c[1] * x; g[3][0] = c[1];
    }
    if (degree >= 2) {
        Y[4] = c[2] * x * y;               g[4][0] = c[2] * y; g[4][1] = c[2] * x;
        Y[5] = c[2] * y * z;               g[5][1] = c[2] * z; g[5][2] = c[2] * y;
        Y[6] = c[3] * (3 * z * z - 1);     g[6][2] = 6 * c[3] * z;
        Y[7] = c[2] * x * z;               g[7][0] = c[2] * z; g[7][2] = c[2] * x;
        Y[8] = c[4] * (x * x - y * y);     g[8][0] = 2 * c[4] * x; g[8][1] = -2 * c[4] * y;
    }
    if (degree >= 3) {
        Y[9] = c[5] * y * (3 * x * x - y * y);
        g[9][0] = 6 * c[5] * x * y; g[9][1] = c[5] * (3 * x * x - 3 * y * y);
        Y[10] = c[6] * x * y * z;
        g[10][0] = c[6] * y * z; g[10][1] = c[6] * x * z; g[10][2] = c[6] * x * y;
        Y[11] = c[7] * y * (5 * z * z - 1);
        g[11][1] = c[7] * (5 * z * z - 1); g[11][2] = 10 * c[7] * y * z;
        Y[12] = c[8] * z * (5 * z * z - 3);
        g[12][2] = c[8] * (15 * z * z - 3);
        Y[13] = c[7] * x * (5 * z * z - 1);
        g[13][0] = c[7] * (5 * z * z - 1); g[13][2] = 10 * c[7] * x * z;
        Y[14] = c[9] * z * (x * x - y * y);
        g[14][0] = 2 * c[9] * x * z; g[14][1] = -2 * c[9] * y * z; g[14][2] = c[9] * (x * x - y * y);
        Y[15] = c[5] * x * (x * x - 3 * y * y);
        g[15][0] = c[5] * (3 * x * x - 3 * y * y); g[15][1] = -6 * c[5] * x * y;
    }
    if (dY) memcpy(dY, g, sizeof(double) * 3 * K);
    return K;
}

int orc_sh_basis(int degree, const double *dir, double *Y, double *dY) {
    return sh_eval(degree, dir, Y, (double (*)[3])dY);
}

/* ------------------------------------------------------------------------------------------ */
/* Per (view, Gaussian) projection with the intermediates the backward needs.                 */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int visible;          /* z > z_near and the alpha footprint holds a pixel centre */
    double p[3];          /* camera-frame mean */
    double u, v, z;
    double cov[3];        /* Sigma' (xx, xy, yy) */
    double Q[3];          /* conic (a, b, c) = Sigma'^{-1} entries (xx, xy, yy) */
    double o;             /* opacity */
    double rgb[3], pre[3];
    double r2;            /* footprint: D^T Q D <= r2 = 2 ln(255 o) */
    int x0, x1, y0, y1;   /* inclusive pixel-index bounding box of the footprint */
    double Sc[9], J[6], tx, ty, limx, limy;
    int clampx, clampy;
    double dir[3], dist;
    double Rq[9], s[3], qn[4], qnorm;
    double Y[16];
} orc_pg;

static void quat_to_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void matmul3(const double *A, const double *B, double *C) { /* C = A B */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}
static void matmul3_bt(const double *A, const double *B, double *C) { /* C = A B^T */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * j + k];
            C[3 * i + j] = s;
        }
}
static void matmul3_at(const double *A, const double *B, double *C) { /* C = A^T B */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * k + i] * B[3 * k + j];
            C[3 * i + j] = s;
        }
}

static void project_one(const orc_gaussians *g, int64_t i, const orc_camera *cam, orc_pg *P) {
    const int64_t n = g->n;
    memset(P, 0, sizeof *P);
    double mu[3] = {g->means[i], g->means[n + i], g->means[2 * n + i]};
    const double *R = cam->R;
    for (int r = 0; r < 3; r++) P->p[r] = R[3 * r] * mu[0] + R[3 * r + 1] * mu[1] + R[3 * r + 2] * mu[2] + cam->t[r];
    const double x = P->p[0], y = P->p[1], z = P->p[2];
    P->z = z;
    if (!(z > cam->z_near)) return;

    /* 3-D covariance */
    double q[4] = {g->quats[i], g->quats[n + i], g->quats[2 * n + i], g->quats[3 * n + i]};
    P->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; k++) P->qn[k] = q[k] / P->qnorm;
    quat_to_rot(P->qn, P->Rq);
    for (int k = 0; k < 3; k++) P->s[k] = exp(g->log_scales[k * n + i]);
    double M[9], Sig[9], tmp[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M[3 * r + c] = P->Rq[3 * r + c] * P->s[c];
    matmul3_bt(M, M, Sig);                 /* Sigma = M M^T */
    matmul3(R, Sig, tmp);
    matmul3_bt(tmp, R, P->Sc);             /* Sigma_c = R Sigma R^T */

    /* EWA Jacobian with guard band */
    P->limx = ORC_GUARD * cam->width / (2.0 * cam->fx);
    P->limy = ORC_GUARD * cam->height / (2.0 * cam->fy);
    double tx = x / z, ty = y / z;
    if (tx > P->limx) { tx = P->limx; P->clampx = 1; }
    if (tx < -P->limx) { tx = -P->limx; P->clampx = 1; }
    if (ty > P->limy) { ty = P->limy; P->clampy = 1; }
    if (ty < -P->limy) { ty = -P->limy; P->clampy = 1; }
    P->tx = tx; P->ty = ty;
    double *J = P->J;
    J[0] = cam->fx / z; J[1] = 0; J[2] = -cam->fx * tx / z;
    J[3] = 0; J[4] = cam->fy / z; J[5] = -cam->fy * ty / z;
    double JS[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) JS[3 * r + c] = J[3 * r] * P->Sc[c] + J[3 * r + 1] * P->Sc[3 + c] + J[3 * r + 2] * P->Sc[6 + c];
    double cxx = JS[0] * J[0] + JS[1] * J[1] + JS[2] * J[2] + ORC_LOWPASS;
    double cxy = JS[0] * J[3] + JS[1] * J[4] + JS[2] * J[5];
    double cyy = JS[3] * J[3] + JS[4] * J[4] + JS[5] * J[5] + ORC_LOWPASS;
    P->cov[0] = cxx; P->cov[1] = cxy; P->cov[2] = cyy;
    double det = cxx * cyy - cxy * cxy;
    P->Q[0] = cyy / det; P->Q[1] = -cxy / det; P->Q[2] = cxx / det;

    P->u = cam->fx * x / z + cam->cx;
    P->v = cam->fy * y / z + cam->cy;
    P->o = 1.0 / (1.0 + exp(-g->opacity_logits[i]));

    /* view-dependent colour */
    double c[3];
    for (int r = 0; r < 3; r++) c[r] = -(R[r] * cam->t[0] + R[3 + r] * cam->t[1] + R[6 + r] * cam->t[2]);
    double dv[3] = {mu[0] - c[0], mu[1] - c[1], mu[2] - c[2]};
    P->dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int r = 0; r < 3; r++) P->dir[r] = dv[r] / P->dist;
    int K = sh_eval(g->sh_degree, P->dir, P->Y, NULL);
    for (int ch = 0; ch < 3; ch++) {
        double s = 0.5;
        for (int k = 0; k < K; k++) s += P->Y[k] * g->sh[(int64_t)(3 * k + ch) * n + i];
        P->pre[ch] = s;
        P->rgb[ch] = s > 0 ? s : 0;
    }

    /* footprint: the ellipse D^T Q D <= 2 ln(255 o); its exact bounding box is
       |Dx| <= sqrt(r2 Sigma'_xx), |Dy| <= sqrt(r2 Sigma'_yy). */
    if (255.0 * P->o < 1.0) return;
    P->r2 = 2.0 * log(255.0 * P->o);
    double ex = sqrt(P->r2 * cxx), ey = sqrt(P->r2 * cyy);
    /* pixel i is sampled at i + 1/2; one extra pixel of slack, the alpha test decides */
    P->x0 = (int)floor(P->u - ex - 0.5) - 1; P->x1 = (int)ceil(P->u + ex - 0.5) + 1;
    P->y0 = (int)floor(P->v - ey - 0.5) - 1; P->y1 = (int)ceil(P->v + ey - 0.5) + 1;
    if (P->x0 < 0) P->x0 = 0;
    if (P->y0 < 0) P->y0 = 0;
    if (P->x1 > cam->width - 1) P->x1 = cam->width - 1;
    if (P->y1 > cam->height - 1) P->y1 = cam->height - 1;
    P->visible = (P->x0 <= P->x1 && P->y0 <= P->y1);
}

/* Projection outputs for parity checks: per Gaussian 16 doubles
   {visible, u, v, z, Q_a, Q_b, Q_c, o, r, g, b, cov_xx, cov_xy, cov_yy, x/z margin, min |pre|}. */
void orc_project(const orc_gaussians *g, const orc_camera *cam, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) {
        orc_pg P;
        project_one(g, i, cam, &P);
        double *o = out + 16 * i;
        o[0] = P.visible; o[1] = P.u; o[2] = P.v; o[3] = P.z;
        o[4] = P.Q[0]; o[5] = P.Q[1]; o[6] = P.Q[2]; o[7] = P.o;
        o[8] = P.rgb[0]; o[9] = P.rgb[1]; o[10] = P.rgb[2];
        o[11] = P.cov[0]; o[12] = P.cov[1]; o[13] = P.cov[2];
        double mx = fabs(fabs(P.p[0] / P.z) / P.limx - 1), my = fabs(fabs(P.p[1] / P.z) / P.limy - 1);
        o[14] = mx < my ? mx : my;
        double mp = fabs(P.pre[0]);
        if (fabs(P.pre[1]) < mp) mp = fabs(P.pre[1]);
        if (fabs(P.pre[2]) < mp) mp = fabs(P.pre[2]);
        o[15] = mp;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Candidate lists: the Gaussians whose footprint bounding box holds a pixel.  Only a pruning   */
/* of the "every Gaussian" loop; the per-pixel alpha test decides membership.                 */
/* ------------------------------------------------------------------------------------------ */
#define CELL 16
typedef struct {
    int ncx, ncy;
    int64_t *start;   /* [ncx*ncy + 1] */
    int64_t *ids;
} orc_cells;

static void build_cells(const orc_pg *P, int64_t n, const orc_camera *cam, orc_cells *C) {
    C->ncx = (cam->width + CELL - 1) / CELL;
    C->ncy = (cam->height + CELL - 1) / CELL;
    int64_t nc = (int64_t)C->ncx * C->ncy;
    C->start = calloc(nc + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) {
        if (!P[i].visible) continue;
        for (int cy = P[i].y0 / CELL; cy <= P[i].y1 / CELL; cy++)
            for (int cx = P[i].x0 / CELL; cx <= P[i].x1 / CELL; cx++) C->start[(int64_t)cy * C->ncx + cx + 1]++;
    }
    for (int64_t c = 0; c < nc; c++) C->start[c + 1] += C->start[c];
    C->ids = malloc(sizeof(int64_t) * (C->start[nc] + 1));
    int64_t *fill = malloc(sizeof(int64_t) * (nc + 1));
    memcpy(fill, C->start, sizeof(int64_t) * (nc + 1));
    for (int64_t i = 0; i < n; i++) {
        if (!P[i].visible) continue;
        for (int cy = P[i].y0 / CELL; cy <= P[i].y1 / CELL; cy++)
            for (int cx = P[i].x0 / CELL; cx <= P[i].x1 / CELL; cx++) C->ids[fill[(int64_t)cy * C->ncx + cx]++] = i;
    }
    free(fill);
}

static void free_cells(orc_cells *C) { free(C->start); free(C->ids); }

/* ------------------------------------------------------------------------------------------ */
/* One pixel: collect contributors, order them, composite.                                    */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int64_t id;
    double z, a_raw, a, dx, dy, T;   /* T = transmittance before this contributor */
} orc_contrib;

/* Compositing order: ascending depth key, then Gaussian index.  The depth key is the camera
   depth rounded to float32 (round to nearest), the 32-bit key tile binning sorts on; equal
   keys fall back to the index. */
static int cmp_contrib(const void *pa, const void *pb) {
    const orc_contrib *a = pa, *b = pb;
    const float za = (float)a->z, zb = (float)b->z;
    if (za < zb) return -1;
    if (za > zb) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

static double rel_margin(double v, double ref) { return fabs(v / ref - 1.0); }

/* relative distance of z to the nearest float32 rounding midpoint: below ~1e-13 the depth
   key could round either way under a different (equally exact) evaluation order */
static double f32_round_margin(double z) {
    const float zf = (float)z;
    const double up = 0.5 * ((double)zf + (double)nextafterf(zf, INFINITY));
    const double dn = 0.5 * ((double)zf + (double)nextafterf(zf, -INFINITY));
    const double m = fabs(z - up) < fabs(z - dn) ? fabs(z - up) : fabs(z - dn);
    return m / fabs(z);
}

typedef struct {
    orc_contrib *buf;
    int64_t cap;
} orc_scratch;

static void scratch_reserve(orc_scratch *s, int64_t need) {
    if (need > s->cap) {
        s->cap = need * 2;
        s->buf = realloc(s->buf, sizeof(orc_contrib) * s->cap);
    }
}

/* Returns the number composited; fills rgb, depth, T and margin.  On return s->buf[0..n)
   holds the composited contributors in order, with their pre-blend transmittance. */
static int64_t pixel_composite(const orc_pg *P, const orc_cells *C, const orc_camera *cam, int px, int py,
                               orc_scratch *s, double rgb[3], double *depth, double *Tout, double *margin) {
    int64_t cell = (int64_t)(py / CELL) * C->ncx + (px / CELL);
    int64_t b = C->start[cell], e = C->start[cell + 1];
    scratch_reserve(s, e - b + 1);
    int64_t m = 0;
    double mg = INFINITY;
    const double cxp = px + 0.5, cyp = py + 0.5;
    for (int64_t k = b; k < e; k++) {
        const orc_pg *G = &P[C->ids[k]];
        if (px < G->x0 || px > G->x1 || py < G->y0 || py > G->y1) continue;
        double dx = cxp - G->u, dy = cyp - G->v;
        double q = G->Q[0] * dx * dx + 2 * G->Q[1] * dx * dy + G->Q[2] * dy * dy;
        double ar = G->o * exp(-0.5 * q);
        /* keep near-threshold rejects for the margin test */
        if (ar < ORC_ALPHA_MIN * (1 - 1e-3)) continue;
        orc_contrib *c = &s->buf[m++];
        c->id = C->ids[k]; c->z = G->z; c->a_raw = ar; c->dx = dx; c->dy = dy;
    }
    qsort(s->buf, m, sizeof(orc_contrib), cmp_contrib);
    double T = 1, Cc[3] = {0, 0, 0}, D = 0;
    int64_t n = 0;
    for (int64_t k = 0; k < m; k++) {
        orc_contrib c = s->buf[k];
        double mth = rel_margin(c.a_raw * 255.0, 1.0);
        if (mth < mg) mg = mth;
        if (c.a_raw < ORC_ALPHA_MIN) continue;
        const orc_pg *G = &P[c.id];
        /* depth key at a float32 rounding midpoint */
        if (f32_round_margin(c.z) < 1e-13) mg = 0;
        double mcl = rel_margin(c.a_raw, ORC_ALPHA_MAX);
        if (mcl < mg) mg = mcl;
        double a = c.a_raw < ORC_ALPHA_MAX ? c.a_raw : ORC_ALPHA_MAX;
        double Tn = T * (1 - a);
        double mt = rel_margin(Tn, ORC_T_MIN);
        if (mt < mg) mg = mt;
        if (Tn < ORC_T_MIN) break;
        /* guard-band and SH-clamp decisions of this contributor */
        double mx = fabs(fabs(G->p[0] / G->z) / G->limx - 1), my = fabs(fabs(G->p[1] / G->z) / G->limy - 1);
        if (mx < mg) mg = mx;
        if (my < mg) mg = my;
        for (int ch = 0; ch < 3; ch++)
            if (fabs(G->pre[ch]) < 1e-6) mg = 0;
        double w = a * T;
        for (int ch = 0; ch < 3; ch++) Cc[ch] += w * G->rgb[ch];
        D += w * G->z;
        c.a = a; c.T = T;
        s->buf[n++] = c;
        T = Tn;
    }
    for (int ch = 0; ch < 3; ch++) rgb[ch] = Cc[ch] + T * cam->bg[ch];
    *depth = D;
    *Tout = T;
    *margin = mg;
    return n;
}

static orc_pg *project_all(const orc_gaussians *g, const orc_camera *cam) {
    orc_pg *P = malloc(sizeof(orc_pg) * (g->n > 0 ? g->n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; i++) project_one(g, i, cam, &P[i]);
    return P;
}

/* Forward render.  pix = NULL renders every pixel into [3][H][W] / [H][W] images; otherwise
   pix holds npix (x, y) pairs and the outputs are [npix][3] and [npix]. */
void orc_render(const orc_gaussians *g, const orc_camera *cam, const int32_t *pix, int64_t npix,
                double *rgb, double *depth, double *T, int32_t *ncontrib, double *margin) {
    orc_pg *P = project_all(g, cam);
    orc_cells C;
    build_cells(P, g->n, cam, &C);
    const int W = cam->width, H = cam->height;
    int64_t total = pix ? npix : (int64_t)W * H;
#pragma omp parallel
    {
        orc_scratch s = {NULL, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < total; k++) {
            int px = pix ? pix[2 * k] : (int)(k % W);
            int py = pix ? pix[2 * k + 1] : (int)(k / W);
            double c[3], d, t, mg;
            int64_t n = pixel_composite(P, &C, cam, px, py, &s, c, &d, &t, &mg);
            if (pix) {
                for (int ch = 0; ch < 3; ch++) rgb[3 * k + ch] = c[ch];
            } else {
                for (int ch = 0; ch < 3; ch++) rgb[(int64_t)ch * W * H + k] = c[ch];
            }
            depth[k] = d;
            T[k] = t;
            if (ncontrib) ncontrib[k] = (int32_t)n;
            if (margin) margin[k] = mg;
        }
        free(s.buf);
    }
    free_cells(&C);
    free(P);
}

/* The composited Gaussians of each listed pixel (pix: npix (x, y) pairs), front to back:
   ids[k * cap + j] for j < min(counts[k], cap); counts[k] is the full number. */
void orc_contributors(const orc_gaussians *g, const orc_camera *cam, const int32_t *pix, int64_t npix, int64_t cap,
                      int64_t *ids, int32_t *counts) {
    orc_pg *P = project_all(g, cam);
    orc_cells C;
    build_cells(P, g->n, cam, &C);
#pragma omp parallel
    {
        orc_scratch s = {NULL, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < npix; k++) {
            double c[3], d, t, mg;
            int64_t n = pixel_composite(P, &C, cam, pix[2 * k], pix[2 * k + 1], &s, c, &d, &t, &mg);
            counts[k] = (int32_t)n;
            for (int64_t j = 0; j < n && j < cap; j++) ids[k * cap + j] = s.buf[j].id;
        }
        free(s.buf);
    }
    free_cells(&C);
    free(P);
}

/* ------------------------------------------------------------------------------------------ */
/* Backward.                                                                                  */
/* ------------------------------------------------------------------------------------------ */
/* per (view, Gaussian) screen-space gradient: u, v, Qa, Qb, Qc, o, r, g, b, z */
#define NSG 10

typedef struct {
    double *means, *log_scales, *quats, *opacity_logits, *sh; /* same layouts as the inputs */
} orc_grads;

static void skew_mul_sym(int k, const double *S, double *out) {
    /* out = E_k S - S E_k, E_k = [e_k]_x */
    double E[9] = {0};
    if (k == 0) { E[5] = -1; E[7] = 1; }
    if (k == 1) { E[2] = 1; E[6] = -1; }
    if (k == 2) { E[1] = -1; E[3] = 1; }
    double A[9], B[9];
    matmul3(E, S, A);
    matmul3(S, E, B);
    for (int i = 0; i < 9; i++) out[i] = A[i] - B[i];
}

/* Chain rule of one (view, Gaussian) from its screen-space gradient to the parameters and
   the pose; accumulates into gr (row i) and dpose. */
static void chain_one(const orc_gaussians *g, int64_t i, const orc_camera *cam, const orc_pg *P,
                      const double *gs, orc_grads *gr, double dpose[6]) {
    const int64_t n = g->n;
    const double *R = cam->R;
    const double fx = cam->fx, fy = cam->fy;
    const double x = P->p[0], y = P->p[1], z = P->p[2];
    double Gp[3] = {0, 0, 0};
    double Gmu[3] = {0, 0, 0};

    /* opacity */
    gr->opacity_logits[i] += gs[5] * P->o * (1 - P->o);

    /* colour -> SH coefficients and view direction */
    double Gpre[3];
    for (int ch = 0; ch < 3; ch++) Gpre[ch] = P->pre[ch] > 0 ? gs[6 + ch] : 0.0;
    double Y[16], dY[16][3];
    int K = sh_eval(g->sh_degree, P->dir, Y, dY);
    double Gdir[3] = {0, 0, 0};
    for (int k = 0; k < K; k++)
        for (int ch = 0; ch < 3; ch++) {
            gr->sh[(int64_t)(3 * k + ch) * n + i] += Gpre[ch] * Y[k];
            double h = g->sh[(int64_t)(3 * k + ch) * n + i];
            for (int r = 0; r < 3; r++) Gdir[r] += Gpre[ch] * h * dY[k][r];
        }
    double dd = P->dir[0] * Gdir[0] + P->dir[1] * Gdir[1] + P->dir[2] * Gdir[2];
    double Gdv[3];
    for (int r = 0; r < 3; r++) Gdv[r] = (Gdir[r] - P->dir[r] * dd) / P->dist;
    for (int r = 0; r < 3; r++) Gmu[r] += Gdv[r];
    /* camera centre c = -R^T t moves by -R^T rho: dL/drho += -R dL/dc, dL/dc = -Gdv */
    if (dpose)
        for (int r = 0; r < 3; r++) dpose[r] += R[3 * r] * Gdv[0] + R[3 * r + 1] * Gdv[1] + R[3 * r + 2] * Gdv[2];

    /* conic -> Sigma' : G_S' = -Q G_Q Q, with G_Q symmetric (off-diagonal half each) */
    double Qm[4] = {P->Q[0], P->Q[1], P->Q[1], P->Q[2]};
    double GQ[4] = {gs[2], 0.5 * gs[3], 0.5 * gs[3], gs[4]};
    double T1[4], GSp[4];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) T1[2 * a + b] = Qm[2 * a] * GQ[b] + Qm[2 * a + 1] * GQ[2 + b];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) GSp[2 * a + b] = -(T1[2 * a] * Qm[b] + T1[2 * a + 1] * Qm[2 + b]);

    /* Sigma' = J Sc J^T + 0.3 I : G_Sc = J^T G_S' J, G_J = 2 G_S' J Sc */
    const double *J = P->J;
    double GSc[9];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double s = 0;
            for (int r = 0; r < 2; r++)
                for (int c = 0; c < 2; c++) s += J[3 * r + a] * GSp[2 * r + c] * J[3 * c + b];
            GSc[3 * a + b] = s;
        }
    double GJ[6];
    for (int r = 0; r < 2; r++)
        for (int b = 0; b < 3; b++) {
            double s = 0;
            for (int c = 0; c < 2; c++)
                for (int k = 0; k < 3; k++) s += GSp[2 * r + c] * J[3 * c + k] * P->Sc[3 * k + b];
            GJ[3 * r + b] = 2 * s;
        }
    /* J entries as functions of the camera-frame point */
    Gp[2] += GJ[0] * (-fx / (z * z)) + GJ[4] * (-fy / (z * z));
    if (!P->clampx) {
        Gp[0] += GJ[2] * (-fx / (z * z));
        Gp[2] += GJ[2] * (2 * fx * x / (z * z * z));
    } else {
        Gp[2] += GJ[2] * (fx * P->tx / (z * z));
    }
    if (!P->clampy) {
        Gp[1] += GJ[5] * (-fy / (z * z));
        Gp[2] += GJ[5] * (2 * fy * y / (z * z * z));
    } else {
        Gp[2] += GJ[5] * (fy * P->ty / (z * z));
    }
    /* mean and depth */
    Gp[0] += gs[0] * fx / z;
    Gp[1] += gs[1] * fy / z;
    Gp[2] += gs[0] * (-fx * x / (z * z)) + gs[1] * (-fy * y / (z * z)) + gs[9];

    /* Sc = R Sigma R^T : G_Sigma = R^T G_Sc R; pose rotation through Sc */
    double tmp[9], GSig[9];
    matmul3_at(R, GSc, tmp);
    matmul3(tmp, R, GSig);
    if (dpose)
        for (int k = 0; k < 3; k++) {
            double D[9];
            skew_mul_sym(k, P->Sc, D);
            double s = 0;
            for (int e = 0; e < 9; e++) s += GSc[e] * D[e];
            dpose[3 + k] += s;
        }

    /* p = R mu + t : G_mu += R^T G_p; pose: rho += G_p, phi += p x G_p */
    for (int r = 0; r < 3; r++) Gmu[r] += R[r] * Gp[0] + R[3 + r] * Gp[1] + R[6 + r] * Gp[2];
    if (dpose) {
        for (int r = 0; r < 3; r++) dpose[r] += Gp[r];
        dpose[3] += y * Gp[2] - z * Gp[1];
        dpose[4] += z * Gp[0] - x * Gp[2];
        dpose[5] += x * Gp[1] - y * Gp[0];
    }
    for (int r = 0; r < 3; r++) gr->means[r * n + i] += Gmu[r];

    /* Sigma = M M^T, M = Rq diag(s) : G_M = 2 G_Sigma M */
    double M[9], GM[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M[3 * r + c] = P->Rq[3 * r + c] * P->s[c];
    matmul3(GSig, M, GM);
    for (int e = 0; e < 9; e++) GM[e] *= 2;
    double GRq[9];
    for (int c = 0; c < 3; c++) {
        double gsc = 0;
        for (int r = 0; r < 3; r++) {
            gsc += GM[3 * r + c] * P->Rq[3 * r + c];
            GRq[3 * r + c] = GM[3 * r + c] * P->s[c];
        }
        gr->log_scales[c * n + i] += gsc * P->s[c];
    }
    /* Rq(qn) */
    const double w = P->qn[0], qx = P->qn[1], qy = P->qn[2], qz = P->qn[3];
    const double dw[9] = {0, -2 * qz, 2 * qy, 2 * qz, 0, -2 * qx, -2 * qy, 2 * qx, 0};
    const double dx[9] = {0, 2 * qy, 2 * qz, 2 * qy, -4 * qx, -2 * w, 2 * qz, 2 * w, -4 * qx};
    const double dy[9] = {-4 * qy, 2 * qx, 2 * w, 2 * qx, 0, 2 * qz, -2 * w, 2 * qz, -4 * qy};
    const double dz[9] = {-4 * qz, -2 * w, 2 * qx, 2 * w, -4 * qz, 2 * qy, 2 * qx, 2 * qy, 0};
    double Gqn[4] = {0, 0, 0, 0};
    for (int e = 0; e < 9; e++) {
        Gqn[0] += GRq[e] * dw[e];
        Gqn[1] += GRq[e] * dx[e];
        Gqn[2] += GRq[e] * dy[e];
        Gqn[3] += GRq[e] * dz[e];
    }
    double qd = 0;
    for (int k = 0; k < 4; k++) qd += P->qn[k] * Gqn[k];
    for (int k = 0; k < 4; k++) gr->quats[k * n + i] += (Gqn[k] - P->qn[k] * qd) / P->qnorm;
}

/* Full backward for one view.  dL_drgb [3][H][W], dL_ddepth [H][W] (may be NULL).  Gradients
   are ACCUMULATED into the orc_grads arrays (double, input layouts) and dpose[6] (may be NULL).
   screen (may be NULL) receives the per-Gaussian screen-space gradient [n][10].
   knife_px (may be NULL, [H][W]) marks pixels whose decision margin is below knife_tol;
   knife_g (may be NULL, [n]) is set to 1 for every Gaussian that is a candidate at such a
   pixel.  Returns the number of knife-edge pixels. */
int64_t orc_render_bwd(const orc_gaussians *g, const orc_camera *cam, const double *dL_drgb,
                       const double *dL_ddepth, double *g_means, double *g_log_scales, double *g_quats,
                       double *g_opacity_logits, double *g_sh, double *dpose, double *screen,
                       double knife_tol, uint8_t *knife_px, uint8_t *knife_g) {
    orc_pg *P = project_all(g, cam);
    orc_cells C;
    build_cells(P, g->n, cam, &C);
    const int W = cam->width, H = cam->height;
    const int64_t n = g->n, npx = (int64_t)W * H;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *acc = calloc((size_t)nth * n * NSG + 1, sizeof(double));
    int64_t nknife = 0;
#pragma omp parallel reduction(+ : nknife)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *A = acc + (size_t)tid * n * NSG;
        orc_scratch s = {NULL, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < npx; k++) {
            int px = (int)(k % W), py = (int)(k / W);
            double c[3], d, Tf, mg;
            int64_t m = pixel_composite(P, &C, cam, px, py, &s, c, &d, &Tf, &mg);
            if (mg < knife_tol) {
                nknife++;
                if (knife_px) knife_px[k] = 1;
                if (knife_g) {
                    /* every candidate of this pixel */
                    int64_t cell = (int64_t)(py / CELL) * C.ncx + (px / CELL);
                    for (int64_t e = C.start[cell]; e < C.start[cell + 1]; e++) {
                        const orc_pg *G = &P[C.ids[e]];
                        if (px < G->x0 || px > G->x1 || py < G->y0 || py > G->y1) continue;
                        double dx = px + 0.5 - G->u, dy = py + 0.5 - G->v;
                        double q = G->Q[0] * dx * dx + 2 * G->Q[1] * dx * dy + G->Q[2] * dy * dy;
                        if (G->o * exp(-0.5 * q) >= ORC_ALPHA_MIN * (1 - 1e-3)) knife_g[C.ids[e]] = 1;
                    }
                }
            } else if (knife_px) {
                knife_px[k] = 0;
            }
            double Gc[3];
            for (int ch = 0; ch < 3; ch++) Gc[ch] = dL_drgb ? dL_drgb[(int64_t)ch * npx + k] : 0.0;
            double Gd = dL_ddepth ? dL_ddepth[k] : 0.0;
            /* suffix sums S = sum_{j>k} w_j c_j + T_final bg (colour) and sum_{j>k} w_j z_j */
            double S[3], Sd = 0;
            for (int ch = 0; ch < 3; ch++) S[ch] = Tf * cam->bg[ch];
            for (int64_t j = m - 1; j >= 0; j--) {
                const orc_contrib *cj = &s.buf[j];
                const orc_pg *G = &P[cj->id];
                double w = cj->a * cj->T;
                double *a = A + (size_t)cj->id * NSG;
                double dLda = 0;
                for (int ch = 0; ch < 3; ch++) {
                    a[6 + ch] += Gc[ch] * w;
                    dLda += Gc[ch] * (cj->T * G->rgb[ch] - S[ch] / (1 - cj->a));
                    S[ch] += w * G->rgb[ch];
                }
                a[9] += Gd * w;
                dLda += Gd * (cj->T * G->z - Sd / (1 - cj->a));
                Sd += w * G->z;
                if (cj->a_raw > ORC_ALPHA_MAX) continue; /* clamped: no gradient to a_raw */
                double ar = cj->a_raw;
                double QDx = G->Q[0] * cj->dx + G->Q[1] * cj->dy;
                double QDy = G->Q[1] * cj->dx + G->Q[2] * cj->dy;
                a[0] += dLda * ar * QDx;
                a[1] += dLda * ar * QDy;
                a[2] += dLda * (-0.5 * ar * cj->dx * cj->dx);
                a[3] += dLda * (-ar * cj->dx * cj->dy);
                a[4] += dLda * (-0.5 * ar * cj->dy * cj->dy);
                a[5] += dLda * ar / G->o;
            }
        }
        free(s.buf);
    }
    double *gsum = calloc((size_t)n * NSG + 1, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        for (int t = 0; t < nth; t++)
            for (int e = 0; e < NSG; e++) gsum[i * NSG + e] += acc[((size_t)t * n + i) * NSG + e];
    free(acc);
    if (screen) memcpy(screen, gsum, sizeof(double) * n * NSG);
    orc_grads gr = {g_means, g_log_scales, g_quats, g_opacity_logits, g_sh};
    double dp[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; i++) {
        if (!P[i].visible) continue;
        const double *gs = gsum + i * NSG;
        int any = 0;
        for (int e = 0; e < NSG; e++) any |= gs[e] != 0.0;
        if (!any) continue;
        chain_one(g, i, cam, &P[i], gs, &gr, dp);
    }
    if (dpose)
        for (int k = 0; k < 6; k++) dpose[k] += dp[k];
    free(gsum);
    free_cells(&C);
    free(P);
    return nknife;
}

/* ------------------------------------------------------------------------------------------ */
/* Sparse Adam (paper Sec. III-C: visible, unfrozen Gaussians refined by a sparse gradient     */
/* optimizer).  rows with mask = 0 keep p, m, v; every gradient is zeroed.                    */
/* param/grad/m/v: [cols][rows] component-major.                                              */
/* ------------------------------------------------------------------------------------------ */
void orc_adam(double *param, double *grad, double *m, double *v, int64_t rows, int64_t cols,
              const uint8_t *mask, double lr, double beta1, double beta2, double eps, int step) {
    const double bc1 = 1 - pow(beta1, step), bc2 = 1 - pow(beta2, step);
    for (int64_t c = 0; c < cols; c++)
        for (int64_t r = 0; r < rows; r++) {
            int64_t e = c * rows + r;
            if (!mask || mask[r]) {
                m[e] = beta1 * m[e] + (1 - beta1) * grad[e];
                v[e] = beta2 * v[e] + (1 - beta2) * grad[e] * grad[e];
                param[e] -= lr * (m[e] / bc1) / (sqrt(v[e] / bc2) + eps);
            }
            grad[e] = 0;
        }
}

/* Number of OpenMP threads the oracle's parallel loops use (1 without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
