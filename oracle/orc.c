/*
 * FP64 oracle for the UPSLAM registration path.  TEST INFRASTRUCTURE ONLY
 * (see orc.h).  Single-threaded, plain C, every pixel visited in row-major
 * order, no blocking and no reordering beyond what each definition states.
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 * Parity unpinned: the exact a-trous weights (orc_atrous; the paper gives no
 * parameters) -- pinned only through the filter's invariants and its
 * wide-sigma limit, a plain B3-spline convolution.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Panorama geometry (Section III-A: sweeps are stored as panoramic images).  */
/* Row i looks along elevation el_top - i*d_el, column j along azimuth        */
/* 2*pi*j/cols; the ray is (cos el cos az, cos el sin az, sin el).            */
/* ------------------------------------------------------------------------ */

void orc_ray(const orc_geom *g, int i, int j, double u[3]) {
    double el = g->el_top - (double)i * g->d_el;
    double az = 2.0 * M_PI * (double)j / (double)g->cols;
    u[0] = cos(el) * cos(az);
    u[1] = cos(el) * sin(az);
    u[2] = sin(el);
}

static int range_ok(const orc_geom *g, double r) { return isfinite(r) && r > g->r_min && r <= g->r_max; }

static int normal_ok(const double *s) { return s[0] != 0.0 || s[1] != 0.0 || s[2] != 0.0; }

/* a surfel is usable for association iff it has a valid range and a normal */
static int surfel_ok(const orc_geom *g, const double *s) { return range_ok(g, s[3]) && normal_ok(s); }

/*
 * Spherical projection of a point into a panorama (the projective lookup of
 * Section III-B).  Nearest pixel centre: i = floor(fi + 1/2), j = floor(fj +
 * 1/2) mod cols with fi = (el_top - el)/d_el, fj = az*cols/(2 pi), az in
 * [0, 2 pi).  Returns 0 (no pixel) for the origin or rows outside [0, rows).
 */
int orc_project(const orc_geom *g, const double q[3], int32_t *pi, int32_t *pj) {
    double rho = sqrt(q[0] * q[0] + q[1] * q[1]);
    if (rho == 0.0 && q[2] == 0.0) return 0;
    double el = atan2(q[2], rho);
    double az = atan2(q[1], q[0]);
    if (az < 0.0) az += 2.0 * M_PI;
    double fi = (g->el_top - el) / g->d_el;
    double fj = az * (double)g->cols / (2.0 * M_PI);
    double ii = floor(fi + 0.5);
    if (!(ii >= 0.0 && ii < (double)g->rows)) return 0;
    long jj = (long)floor(fj + 0.5);
    jj %= g->cols;
    if (jj < 0) jj += g->cols;
    *pi = (int32_t)ii;
    *pj = (int32_t)jj;
    return 1;
}

static void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------------ */
/* Section III-A: a rough normal is the cross product of the vectors from a   */
/* pixel's point to two of its image neighbours: the next column (wrapping in */
/* azimuth) and the next row (the previous row for the last row).  It is      */
/* oriented towards the sensor.  Reading: the pixel has no normal when any of */
/* the three ranges is invalid, when a neighbour's range differs from the     */
/* centre's by more than max_rel_jump * r (an occlusion edge), or when the    */
/* cross product is degenerate.                                              */
/* ------------------------------------------------------------------------ */

int orc_raw_normals(const orc_geom *g, const double *depth, double max_rel_jump, double *surfel) {
    const int H = g->rows, W = g->cols;
    for (int i = 0; i < H; i++) {
        for (int j = 0; j < W; j++) {
            double *out = surfel + 4 * ((size_t)i * W + j);
            double rc = depth[(size_t)i * W + j];
            out[0] = out[1] = out[2] = 0.0;
            out[3] = range_ok(g, rc) ? rc : 0.0;
            if (!range_ok(g, rc)) continue;
            int ja = (j + 1) % W;
            int ib = (i + 1 < H) ? i + 1 : i - 1;
            if (ib < 0) continue;
            double ra = depth[(size_t)i * W + ja], rb = depth[(size_t)ib * W + j];
            if (!range_ok(g, ra) || !range_ok(g, rb)) continue;
            if (fabs(ra - rc) > max_rel_jump * rc || fabs(rb - rc) > max_rel_jump * rc) continue;
            double uc[3], ua[3], ub[3], p[3], a[3], b[3], n[3];
            orc_ray(g, i, j, uc);
            orc_ray(g, i, ja, ua);
            orc_ray(g, ib, j, ub);
            for (int k = 0; k < 3; k++) {
                p[k] = rc * uc[k];
                a[k] = ra * ua[k] - p[k];
                b[k] = rb * ub[k] - p[k];
            }
            cross3(a, b, n);
            double nn = norm3(n);
            if (!(nn > 1e-6 * norm3(a) * norm3(b))) continue;
            double s = (dot3(n, p) > 0.0) ? -1.0 / nn : 1.0 / nn;
            out[0] = n[0] * s;
            out[1] = n[1] * s;
            out[2] = n[2] * s;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Section III-A: edge-aware a-trous wavelet smoothing of the normal image    */
/* (the paper cites Dammertz et al. 2010 and gives no parameters).  Reading:  */
/* level l uses the 5x5 B3-spline taps h = (1,4,6,4,1)/16 spaced 2^l apart,   */
/* rows outside the image are skipped and columns wrap; only taps with a      */
/* normal contribute, weighted by h[dy] h[dx] * exp(-((r_q-r_p)/(sigma_r      */
/* r_p))^2) * exp(-(2 - 2 n_p.n_q)/sigma_n^2); the result is renormalised.    */
/* Ranges are not changed.  Each level reads the previous level's output.     */
/* ------------------------------------------------------------------------ */

static void atrous_level(const orc_geom *g, const double *in, int step, double sigma_r, double sigma_n,
                         double *out) {
    static const double h[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    const int H = g->rows, W = g->cols;
    for (int i = 0; i < H; i++) {
        for (int j = 0; j < W; j++) {
            const double *c = in + 4 * ((size_t)i * W + j);
            double *o = out + 4 * ((size_t)i * W + j);
            o[3] = c[3];
            if (!normal_ok(c)) {
                o[0] = o[1] = o[2] = 0.0;
                continue;
            }
            double acc[3] = {0, 0, 0};
            for (int dy = -2; dy <= 2; dy++) {
                int y = i + dy * step;
                if (y < 0 || y >= H) continue;
                for (int dx = -2; dx <= 2; dx++) {
                    int x = ((j + dx * step) % W + W) % W;
                    const double *q = in + 4 * ((size_t)y * W + x);
                    if (!normal_ok(q)) continue;
                    double dr = (q[3] - c[3]) / (sigma_r * c[3]);
                    double dn = 2.0 - 2.0 * dot3(c, q);
                    double w = h[dy + 2] * h[dx + 2] * exp(-dr * dr) * exp(-dn / (sigma_n * sigma_n));
                    acc[0] += w * q[0];
                    acc[1] += w * q[1];
                    acc[2] += w * q[2];
                }
            }
            double nn = norm3(acc);
            if (nn > 0.0) {
                o[0] = acc[0] / nn;
                o[1] = acc[1] / nn;
                o[2] = acc[2] / nn;
            } else {
                o[0] = o[1] = o[2] = 0.0;
            }
        }
    }
}

int orc_atrous(const orc_geom *g, const double *in, int levels, double sigma_r, double sigma_n, double *out) {
    size_t n = (size_t)g->rows * g->cols * 4;
    if (levels <= 0) {
        memcpy(out, in, n * sizeof(double));
        return 0;
    }
    double *tmp = (double *)malloc(n * sizeof(double));
    const double *src = in;
    for (int l = 0; l < levels; l++) {
        /* ping-pong so that the last level lands in out */
        double *dst = ((levels - 1 - l) % 2 == 0) ? out : tmp;
        atrous_level(g, src, 1 << l, sigma_r, sigma_n, dst);
        src = dst;
    }
    free(tmp);
    return 0;
}

int orc_panorama_normals(const orc_geom *g, const double *depth, const orc_normal_params *p, double *surfel) {
    size_t n = (size_t)g->rows * g->cols * 4;
    double *raw = (double *)malloc(n * sizeof(double));
    orc_raw_normals(g, depth, p->max_rel_jump, raw);
    orc_atrous(g, raw, p->atrous_levels, p->sigma_r, p->sigma_n, surfel);
    free(raw);
    return 0;
}

/* Pyramid level l keeps pixel (2^l i, 2^l j) of level 0, normal included.   */
int orc_pyramid_level(const orc_geom *g, const double *surfel, int level, double *out) {
    int s = 1 << level;
    int H = g->rows / s, W = g->cols / s;
    for (int i = 0; i < H; i++)
        for (int j = 0; j < W; j++)
            memcpy(out + 4 * ((size_t)i * W + j), surfel + 4 * ((size_t)(i * s) * g->cols + j * s),
                   4 * sizeof(double));
    return 0;
}

static orc_geom level_geom(const orc_geom *g, int level) {
    orc_geom o = *g;
    o.rows = g->rows >> level;
    o.cols = g->cols >> level;
    o.d_el = g->d_el * (double)(1 << level);
    return o;
}

/* ------------------------------------------------------------------------ */
/* Equation 1 terms.  For scan pixel s2 with point p and normal n2, the       */
/* transformed point is q = R p + t and its normal m = R n2; q is projected   */
/* into the keyframe, the keyframe surfel there gives s1 and N(s1) = n1.      */
/* The similarity filter Omega keeps the pair iff both have a range and a     */
/* normal, |q - s1| <= d_max and m.n1 >= cos(theta_max).  The point-to-plane  */
/* residual is r = (q - s1).n1.  Its derivative under a left perturbation     */
/* T <- Exp(xi) T with xi = (omega, v) is J = [q x n1, n1].                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t idx;
    int inlier;
    double r;
    double J[6];
} pair_t;

static void transform(const double T[12], const double x[3], double y[3]) {
    for (int a = 0; a < 3; a++) y[a] = T[3 * a] * x[0] + T[3 * a + 1] * x[1] + T[3 * a + 2] * x[2] + T[9 + a];
}

static void rotate(const double T[12], const double x[3], double y[3]) {
    for (int a = 0; a < 3; a++) y[a] = T[3 * a] * x[0] + T[3 * a + 1] * x[1] + T[3 * a + 2] * x[2];
}

static void pair_at(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf,
                    const double T[12], double d_max, double cos_theta_max, int i, int j, pair_t *pr) {
    const double *s2 = scan + 4 * ((size_t)i * sg->cols + j);
    pr->idx = -1;
    pr->inlier = 0;
    pr->r = 0.0;
    for (int k = 0; k < 6; k++) pr->J[k] = 0.0;
    if (!surfel_ok(sg, s2)) return;
    double u[3], p[3], q[3], m[3];
    orc_ray(sg, i, j, u);
    for (int k = 0; k < 3; k++) p[k] = s2[3] * u[k];
    transform(T, p, q);
    rotate(T, s2, m);
    int32_t ki, kj;
    if (!orc_project(kg, q, &ki, &kj)) return;
    pr->idx = ki * kg->cols + kj;
    const double *s1 = kf + 4 * (size_t)pr->idx;
    if (!surfel_ok(kg, s1)) return;
    double uk[3], x1[3], d[3];
    orc_ray(kg, ki, kj, uk);
    for (int k = 0; k < 3; k++) {
        x1[k] = s1[3] * uk[k];
        d[k] = q[k] - x1[k];
    }
    if (!(norm3(d) <= d_max)) return;
    if (!(dot3(m, s1) >= cos_theta_max)) return;
    pr->inlier = 1;
    pr->r = dot3(d, s1);
    double qxn[3];
    cross3(q, s1, qxn);
    pr->J[0] = qxn[0];
    pr->J[1] = qxn[1];
    pr->J[2] = qxn[2];
    pr->J[3] = s1[0];
    pr->J[4] = s1[1];
    pr->J[5] = s1[2];
}

int orc_residuals(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf, const double T[12],
                  double d_max, double cos_theta_max, int32_t *kf_index, uint8_t *inlier, double *r, double *J) {
    for (int i = 0; i < sg->rows; i++) {
        for (int j = 0; j < sg->cols; j++) {
            size_t px = (size_t)i * sg->cols + j;
            pair_t pr;
            pair_at(sg, scan, kg, kf, T, d_max, cos_theta_max, i, j, &pr);
            if (kf_index) kf_index[px] = pr.idx;
            if (inlier) inlier[px] = (uint8_t)pr.inlier;
            if (r) r[px] = pr.r;
            if (J)
                for (int k = 0; k < 6; k++) J[6 * px + k] = pr.J[k];
        }
    }
    return 0;
}

/* IRLS weight of one residual for the absolute-value objective of           */
/* Equation 1: w = 1 / max(|r|, delta), so that w r^2 = |r| away from zero;  */
/* below delta the weight stays 1 / delta (the step then minimises Huber's   */
/* function with threshold delta).  delta = 0 selects the squared objective */
/* (w = 1).                                                                  */
static double irls_weight(double r, double delta) {
    if (delta <= 0.0) return 1.0;
    double a = fabs(r);
    return 1.0 / (a > delta ? a : delta);
}

/* Gauss-Newton normal equations of the squared Equation-1 residuals:         */
/* A = sum J^T J (upper triangle, row-major, 21 entries), b = sum J^T r.      */
int orc_normal_equations(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf,
                         const double T[12], double d_max, double cos_theta_max, double A[21], double b[6],
                         double *sum_r2, int64_t *inliers, int64_t *valid) {
    return orc_normal_equations_irls(sg, scan, kg, kf, T, d_max, cos_theta_max, 0.0, A, b, sum_r2, inliers, valid);
}

/* The same with each inlier's terms weighted by irls_weight(r, delta):       */
/* A = sum w J^T J, b = sum w J^T r; sum_r2 stays the unweighted sum of r^2.  */
int orc_normal_equations_irls(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf,
                              const double T[12], double d_max, double cos_theta_max, double delta, double A[21],
                              double b[6], double *sum_r2, int64_t *inliers, int64_t *valid) {
    for (int k = 0; k < 21; k++) A[k] = 0.0;
    for (int k = 0; k < 6; k++) b[k] = 0.0;
    double s2 = 0.0;
    int64_t n_in = 0, n_valid = 0;
    for (int i = 0; i < sg->rows; i++) {
        for (int j = 0; j < sg->cols; j++) {
            const double *sp = scan + 4 * ((size_t)i * sg->cols + j);
            if (range_ok(sg, sp[3])) n_valid++;
            pair_t pr;
            pair_at(sg, scan, kg, kf, T, d_max, cos_theta_max, i, j, &pr);
            if (!pr.inlier) continue;
            n_in++;
            double w = irls_weight(pr.r, delta);
            int e = 0;
            for (int a = 0; a < 6; a++)
                for (int c = a; c < 6; c++) A[e++] += w * pr.J[a] * pr.J[c];
            for (int a = 0; a < 6; a++) b[a] += w * pr.J[a] * pr.r;
            s2 += pr.r * pr.r;
        }
    }
    if (sum_r2) *sum_r2 = s2;
    if (inliers) *inliers = n_in;
    if (valid) *valid = n_valid;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gauss-Newton step: Cholesky factorisation of the 6x6 A, xi = -A^{-1} b.    */
/* A pivot <= 1e-12 * max(diag A) (or a zero matrix) means the correspondence */
/* set does not constrain all six degrees of freedom: returns DEGENERATE.     */
/* ------------------------------------------------------------------------ */

int orc_solve6(const double A21[21], const double b[6], double xi[6]) {
    double A[6][6], L[6][6];
    int e = 0;
    for (int a = 0; a < 6; a++)
        for (int c = a; c < 6; c++) {
            A[a][c] = A21[e];
            A[c][a] = A21[e];
            e++;
        }
    double maxd = 0.0;
    for (int a = 0; a < 6; a++)
        if (A[a][a] > maxd) maxd = A[a][a];
    if (!(maxd > 0.0)) return ORC_DEGENERATE;
    memset(L, 0, sizeof(L));
    for (int c = 0; c < 6; c++) {
        double d = A[c][c];
        for (int k = 0; k < c; k++) d -= L[c][k] * L[c][k];
        if (!(d > 1e-12 * maxd)) return ORC_DEGENERATE;
        L[c][c] = sqrt(d);
        for (int r = c + 1; r < 6; r++) {
            double s = A[r][c];
            for (int k = 0; k < c; k++) s -= L[r][k] * L[c][k];
            L[r][c] = s / L[c][c];
        }
    }
    double y[6];
    for (int r = 0; r < 6; r++) {
        double s = -b[r];
        for (int k = 0; k < r; k++) s -= L[r][k] * y[k];
        y[r] = s / L[r][r];
    }
    for (int r = 5; r >= 0; r--) {
        double s = y[r];
        for (int k = r + 1; k < 6; k++) s -= L[k][r] * xi[k];
        xi[r] = s / L[r][r];
    }
    return ORC_CONVERGED;
}

/* Closed-form exponential of the twist xi = (omega, v) (Rodrigues formula    */
/* for the rotation, the V matrix for the translation), with the series of    */
/* the three coefficients below theta = 1e-4.                                */
void orc_exp_se3(const double xi[6], double T[12]) {
    const double *w = xi, *v = xi + 3;
    double th2 = dot3(w, w), th = sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
    double K2[3][3];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) K2[a][c] = K[a][0] * K[0][c] + K[a][1] * K[1][c] + K[a][2] * K[2][c];
    double V[3][3];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            double I = (a == c) ? 1.0 : 0.0;
            T[3 * a + c] = I + A * K[a][c] + B * K2[a][c];
            V[a][c] = I + B * K[a][c] + C * K2[a][c];
        }
    for (int a = 0; a < 3; a++) T[9 + a] = V[a][0] * v[0] + V[a][1] * v[1] + V[a][2] * v[2];
}

/* out = A * B as rigid transforms (apply B first). */
void orc_compose(const double A[12], const double B[12], double out[12]) {
    double o[12];
    for (int a = 0; a < 3; a++) {
        for (int c = 0; c < 3; c++)
            o[3 * a + c] = A[3 * a] * B[c] + A[3 * a + 1] * B[3 + c] + A[3 * a + 2] * B[6 + c];
        o[9 + a] = A[3 * a] * B[9] + A[3 * a + 1] * B[10] + A[3 * a + 2] * B[11] + A[9 + a];
    }
    memcpy(out, o, sizeof(o));
}

/* ------------------------------------------------------------------------ */
/* Registration (Section III-B): Gauss-Newton on the squared point-to-plane   */
/* residuals of Equation 1 over re-associated projective correspondences,     */
/* coarse-to-fine over a subsampled pyramid, followed by the registration     */
/* quality of Section III-C (inliers over valid scan ranges) at level 0.      */
/* With irls_delta > 0 every step is the reweighted step of the absolute-     */
/* value objective (orc_normal_equations_irls); the quality terms stay        */
/* unweighted and the returned JtJ, Jtr are the weighted ones.               */
/* ------------------------------------------------------------------------ */

int orc_register(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf,
                 const double init[12], const orc_icp_params *p, orc_icp_result *res) {
    double T[12];
    memcpy(T, init, sizeof(T));
    int status = ORC_CONVERGED;
    int iters = 0;
    int level_iters[4] = {0, 0, 0, 0};
    double last_norm = 0.0;
    int stop = 0;
    for (int l = p->levels - 1; l >= 0 && !stop; l--) {
        orc_geom sl = level_geom(sg, l), kl = level_geom(kg, l);
        size_t ns = (size_t)sl.rows * sl.cols * 4, nk = (size_t)kl.rows * kl.cols * 4;
        double *sp = (double *)malloc(ns * sizeof(double));
        double *kp = (double *)malloc(nk * sizeof(double));
        orc_pyramid_level(sg, scan, l, sp);
        orc_pyramid_level(kg, kf, l, kp);
        int converged = 0;
        for (int it = 0; it < p->iters[l]; it++) {
            double A[21], b[6], s2, xi[6], E[12];
            int64_t n_in, n_valid;
            orc_normal_equations_irls(&sl, sp, &kl, kp, T, p->d_max[l], p->cos_theta_max, p->irls_delta, A, b, &s2,
                                      &n_in, &n_valid);
            if (n_in < p->min_inliers) {
                status = ORC_NO_INLIERS;
                stop = 1;
                break;
            }
            if (orc_solve6(A, b, xi) != ORC_CONVERGED) {
                status = ORC_DEGENERATE;
                stop = 1;
                break;
            }
            orc_exp_se3(xi, E);
            orc_compose(E, T, T);
            iters++;
            level_iters[l]++;
            double nrm = 0.0;
            for (int k = 0; k < 6; k++) nrm += xi[k] * xi[k];
            last_norm = sqrt(nrm);
            if (p->stop_update_norm > 0.0 && last_norm < p->stop_update_norm) {
                converged = 1;
                break;
            }
        }
        if (l == 0 && !stop && p->stop_update_norm > 0.0 && !converged) status = ORC_MAX_ITERS;
        free(sp);
        free(kp);
    }
    /* quality at level 0 and the final pose */
    double tau = p->d_max[0];
    double A[21], b[6], s2 = 0.0, trunc = 0.0;
    int64_t n_in = 0, n_valid = 0;
    for (int k = 0; k < 21; k++) A[k] = 0.0;
    for (int k = 0; k < 6; k++) b[k] = 0.0;
    for (int i = 0; i < sg->rows; i++) {
        for (int j = 0; j < sg->cols; j++) {
            const double *s = scan + 4 * ((size_t)i * sg->cols + j);
            if (!range_ok(sg, s[3])) continue;
            n_valid++;
            pair_t pr;
            pair_at(sg, scan, kg, kf, T, p->d_max[0], p->cos_theta_max, i, j, &pr);
            if (!pr.inlier) {
                trunc += tau * tau;
                continue;
            }
            n_in++;
            double r2 = pr.r * pr.r;
            s2 += r2;
            trunc += r2 < tau * tau ? r2 : tau * tau;
            double w = irls_weight(pr.r, p->irls_delta);
            int e = 0;
            for (int a = 0; a < 6; a++)
                for (int c = a; c < 6; c++) A[e++] += w * pr.J[a] * pr.J[c];
            for (int a = 0; a < 6; a++) b[a] += w * pr.J[a] * pr.r;
        }
    }
    memcpy(res->T, T, sizeof(T));
    res->inliers = n_in;
    res->valid = n_valid;
    res->inlier_ratio = n_valid > 0 ? (double)n_in / (double)n_valid : 0.0;
    res->rms = n_in > 0 ? sqrt(s2 / (double)n_in) : 0.0;
    res->trunc_cost = trunc;
    res->iters_run = iters;
    memcpy(res->level_iters, level_iters, sizeof(level_iters));
    res->status = status;
    memcpy(res->JtJ, A, sizeof(A));
    memcpy(res->Jtr, b, sizeof(b));
    res->last_update_norm = last_norm;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Keyframe update (Section III-C).  With the registered pose T (scan ->      */
/* keyframe), each keyframe pixel that already holds samples is mapped back    */
/* into the sweep (x = T^{-1} s1, projected into the scan panorama); if the   */
/* similarity filter passes, the new sample is averaged in with weight 1      */
/* against the pixel's sample count c, and c is incremented, saturating at    */
/* max_count (10 in the paper).  Readings: the new sample's range is where    */
/* the keyframe ray meets the plane through q with normal n1; a grazing       */
/* keyframe ray (|u.n1| < min_cos_incidence) is not updated; empty keyframe   */
/* pixels are filled from the nearest scan surfel that projects onto them    */
/* (smallest |q|, then smallest scan index), starting a count of 1.           */
/* ------------------------------------------------------------------------ */

int orc_fuse(const orc_geom *sg, const double *scan, const orc_geom *kg, double *kf, uint16_t *kf_count,
             const double T[12], const orc_fuse_params *p) {
    const int HK = kg->rows, WK = kg->cols;
    size_t nk = (size_t)HK * WK;
    /* T^{-1} = (R^T, -R^T t) */
    double Ti[12];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) Ti[3 * a + c] = T[3 * c + a];
    for (int a = 0; a < 3; a++) Ti[9 + a] = -(Ti[3 * a] * T[9] + Ti[3 * a + 1] * T[10] + Ti[3 * a + 2] * T[11]);
    uint8_t *was_empty = (uint8_t *)malloc(nk);
    for (size_t k = 0; k < nk; k++) was_empty[k] = kf_count[k] == 0;

    /* update pass over keyframe pixels that hold samples */
    for (int i = 0; i < HK; i++) {
        for (int j = 0; j < WK; j++) {
            size_t px = (size_t)i * WK + j;
            double *s1 = kf + 4 * px;
            int c = kf_count[px];
            if (c == 0 || !surfel_ok(kg, s1)) continue;
            double uk[3], x1[3], x[3];
            orc_ray(kg, i, j, uk);
            for (int k = 0; k < 3; k++) x1[k] = s1[3] * uk[k];
            transform(Ti, x1, x);
            int32_t si, sj;
            if (!orc_project(sg, x, &si, &sj)) continue;
            const double *s2 = scan + 4 * ((size_t)si * sg->cols + sj);
            if (!surfel_ok(sg, s2)) continue;
            double us[3], ps[3], q[3], m[3], d[3];
            orc_ray(sg, si, sj, us);
            for (int k = 0; k < 3; k++) ps[k] = s2[3] * us[k];
            transform(T, ps, q);
            rotate(T, s2, m);
            for (int k = 0; k < 3; k++) d[k] = q[k] - x1[k];
            if (!(norm3(d) <= p->d_max)) continue;
            if (!(dot3(m, s1) >= p->cos_theta_max)) continue;
            double un = dot3(uk, s1);
            if (!(fabs(un) >= p->min_cos_incidence)) continue;
            double r_new = s1[3] + dot3(d, s1) / un;
            double r_avg = ((double)c * s1[3] + r_new) / (double)(c + 1);
            if (!range_ok(kg, r_avg)) continue;
            double n[3];
            for (int k = 0; k < 3; k++) n[k] = (double)c * s1[k] + m[k];
            double nn = norm3(n);
            if (!(nn > 0.0)) continue;
            s1[0] = n[0] / nn;
            s1[1] = n[1] / nn;
            s1[2] = n[2] / nn;
            s1[3] = r_avg;
            kf_count[px] = (uint16_t)(c + 1 < p->max_count ? c + 1 : p->max_count);
        }
    }

    /* fill pass: nearest scan surfel per empty keyframe pixel */
    double *best_r = (double *)malloc(nk * sizeof(double));
    int64_t *best_k = (int64_t *)malloc(nk * sizeof(int64_t));
    for (size_t k = 0; k < nk; k++) {
        best_r[k] = INFINITY;
        best_k[k] = -1;
    }
    for (int i = 0; i < sg->rows; i++) {
        for (int j = 0; j < sg->cols; j++) {
            int64_t sk = (int64_t)i * sg->cols + j;
            const double *s2 = scan + 4 * (size_t)sk;
            if (!surfel_ok(sg, s2)) continue;
            double us[3], ps[3], q[3];
            orc_ray(sg, i, j, us);
            for (int k = 0; k < 3; k++) ps[k] = s2[3] * us[k];
            transform(T, ps, q);
            double rq = norm3(q);
            if (!range_ok(kg, rq)) continue;
            int32_t ki, kj;
            if (!orc_project(kg, q, &ki, &kj)) continue;
            size_t kp = (size_t)ki * WK + kj;
            if (!was_empty[kp]) continue;
            if (rq < best_r[kp] || (rq == best_r[kp] && sk < best_k[kp])) {
                best_r[kp] = rq;
                best_k[kp] = sk;
            }
        }
    }
    for (size_t kp = 0; kp < nk; kp++) {
        if (best_k[kp] < 0) continue;
        const double *s2 = scan + 4 * (size_t)best_k[kp];
        double m[3];
        rotate(T, s2, m);
        double *s1 = kf + 4 * kp;
        s1[0] = m[0];
        s1[1] = m[1];
        s1[2] = m[2];
        s1[3] = best_r[kp];
        kf_count[kp] = 1;
    }
    free(best_r);
    free(best_k);
    free(was_empty);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Moving-object filtering across keyframes (Section III-C: the keyframes    */
/* together hold several hypotheses of occupancy, and a mutual consistency   */
/* check at keyframe switches removes what moved).  Reading: a sample of     */
/* keyframe A is inconsistent with keyframe B when B looked through the      */
/* place where A's sample lies.  A's point x = r u(i, j) is mapped into B    */
/* (y = T_ba x) and projected to B's pixel (i', j'); the sample is marked    */
/* when every pixel of B's 3x3 neighbourhood of (i', j') (columns wrap; a    */
/* row outside the image ends the test) holds a valid range with at least    */
/* min_count samples (any count when b_count is NULL) that exceeds |y| by    */
/* more than max(margin_abs, margin_rel |y|).  The neighbourhood keeps       */
/* samples at B's depth edges, where the nearest pixel can fall on the far   */
/* side of the edge.                                                         */
/* ------------------------------------------------------------------------ */

int orc_free_space_violations(const orc_geom *ga, const double *a, const orc_geom *gb, const double *b,
                              const uint16_t *b_count, const double T_ba[12], const orc_consistency_params *p,
                              uint8_t *mask_a) {
    for (int i = 0; i < ga->rows; i++) {
        for (int j = 0; j < ga->cols; j++) {
            size_t px = (size_t)i * ga->cols + j;
            mask_a[px] = 0;
            double r = a[4 * px + 3];
            if (!range_ok(ga, r)) continue;
            double u[3], x[3], y[3];
            orc_ray(ga, i, j, u);
            for (int k = 0; k < 3; k++) x[k] = r * u[k];
            transform(T_ba, x, y);
            int32_t bi, bj;
            if (!orc_project(gb, y, &bi, &bj)) continue;
            double rho = norm3(y);
            double margin = p->margin_rel * rho > p->margin_abs ? p->margin_rel * rho : p->margin_abs;
            int seen_through = 1;
            for (int di = -1; di <= 1 && seen_through; di++) {
                int ii = bi + di;
                if (ii < 0 || ii >= gb->rows) {
                    seen_through = 0;
                    break;
                }
                for (int dj = -1; dj <= 1; dj++) {
                    int jj = (bj + dj + gb->cols) % gb->cols;
                    size_t q = (size_t)ii * gb->cols + jj;
                    double rb = b[4 * q + 3];
                    int votes = b_count == NULL || b_count[q] >= p->min_count;
                    if (!(range_ok(gb, rb) && votes && rb > rho + margin)) {
                        seen_through = 0;
                        break;
                    }
                }
            }
            mask_a[px] = (uint8_t)seen_through;
        }
    }
    return 0;
}

/* Removal of marked samples: surfel (0, 0, 0, 0), count 0 (count may be NULL). */
int orc_remove_marked(const orc_geom *g, double *surfel, uint16_t *count, const uint8_t *mask) {
    size_t n = (size_t)g->rows * g->cols;
    int removed = 0;
    for (size_t px = 0; px < n; px++) {
        if (!mask[px]) continue;
        for (int k = 0; k < 4; k++) surfel[4 * px + k] = 0.0;
        if (count) count[px] = 0;
        removed++;
    }
    return removed;
}

/* ------------------------------------------------------------------------ */
/* Panorama formation (Section III-A): the measurements of one sweep, each   */
/* taken at its own time, are moved into the frame of a single instant and  */
/* projected into a panoramic image.  raw: the sweep as a range image of     */
/* raw_g (row = beam, column = firing); col_T + 12 j maps column j's frame    */
/* into the reference frame (NULL: identity for every column).  A valid      */
/* measurement r at (i, j) gives x = r u(i, j), y = C_j x; y's pixel of out_g */
/* keeps the nearest |y| (the smaller raw index among equal ranges); pixels   */
/* nothing reaches are 0, and so is every |y| outside out_g's valid ranges.   */
/* ------------------------------------------------------------------------ */

int orc_splat_sweep(const orc_geom *raw_g, const double *raw, const double *col_T, const orc_geom *out_g,
                    double *out) {
    size_t nout = (size_t)out_g->rows * out_g->cols;
    int64_t *win = (int64_t *)malloc(nout * sizeof(int64_t));
    for (size_t k = 0; k < nout; k++) {
        out[k] = 0.0;
        win[k] = -1;
    }
    static const double I12[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
    for (int i = 0; i < raw_g->rows; i++) {
        for (int j = 0; j < raw_g->cols; j++) {
            int64_t k = (int64_t)i * raw_g->cols + j;
            double r = raw[k];
            if (!range_ok(raw_g, r)) continue;
            const double *C = col_T ? col_T + 12 * (size_t)j : I12;
            double u[3], x[3], y[3];
            orc_ray(raw_g, i, j, u);
            for (int a = 0; a < 3; a++) x[a] = r * u[a];
            transform(C, x, y);
            double ry = norm3(y);
            if (!range_ok(out_g, ry)) continue;
            int32_t oi, oj;
            if (!orc_project(out_g, y, &oi, &oj)) continue;
            size_t q = (size_t)oi * out_g->cols + oj;
            if (win[q] < 0 || ry < out[q] || (ry == out[q] && k < win[q])) {
                out[q] = ry;
                win[q] = k;
            }
        }
    }
    free(win);
    return 0;
}

