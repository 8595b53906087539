/*
 * Seeded synthetic lidar scenes: an FP64 ray caster that renders panoramic
 * range images of analytic scenes (a box room with boxes, or an outdoor scene
 * with a gradient-noise ground, vertical cylinders and building facades).
 *
 * This file is input generation only.  It contains none of the registration
 * method's arithmetic: it produces the range images (and, for analytic tests,
 * the exact surface normals of the primitive hit by each ray) that both the
 * CPU oracle and the GPU path consume byte for byte.
 *
 * Scene primitives (all in world coordinates, metres):
 *   room       interior of an axis-aligned box (optional)
 *   boxes      solid axis-aligned boxes                      [nbox][6]  (min xyz, max xyz)
 *   cylinders  vertical cylinders standing on z = zbase       [ncyl][5] (cx, cy, r, zbase, ztop)
 *   facades    vertical rectangles between two xy points      [nfac][6] (x0, y0, x1, y1, z0, z1)
 *   ground     height field z = amp * noise(x / scale, y / scale) (optional)
 *
 * The gradient noise is Perlin's improved noise (SIGGRAPH 2002) restricted to
 * two dimensions: a seeded permutation of 0..255, the quintic fade
 * 6t^5 - 15t^4 + 10t^3, and eight unit-ish gradient directions.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int has_room;
    double room[6];
    int nbox;
    const double *boxes;
    int ncyl;
    const double *cyl;
    int nfac;
    const double *fac;
    int has_ground;
    double g_amp, g_scale;
    const int32_t *perm; /* 512 entries: a permutation of 0..255 repeated twice */
} syn_scene;

typedef struct {
    int rows, cols;
    double el_top, d_el, r_max;
} syn_geom;

/* ---------------- gradient noise ---------------- */

static double fade(double t) { return t * t * t * (t * (t * 6.0 - 15.0) + 10.0); }
static double dfade(double t) { return 30.0 * t * t * (t * (t - 2.0) + 1.0); }

static void grad2(int h, double *gx, double *gy) {
    static const double G[8][2] = {{1, 1}, {-1, 1}, {1, -1}, {-1, -1},
                                   {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    *gx = G[h & 7][0];
    *gy = G[h & 7][1];
}

/* value and gradient of 2-D gradient noise at (x, y) */
static void noise2(const int32_t *p, double x, double y, double *val, double *dx, double *dy) {
    double fx = floor(x), fy = floor(y);
    int X = ((int)fx) & 255, Y = ((int)fy) & 255;
    double xf = x - fx, yf = y - fy;
    int aa = p[p[X] + Y], ab = p[p[X] + Y + 1], ba = p[p[X + 1] + Y], bb = p[p[X + 1] + Y + 1];
    double g[4][2];
    grad2(aa, &g[0][0], &g[0][1]);
    grad2(ba, &g[1][0], &g[1][1]);
    grad2(ab, &g[2][0], &g[2][1]);
    grad2(bb, &g[3][0], &g[3][1]);
    double n00 = g[0][0] * xf + g[0][1] * yf;
    double n10 = g[1][0] * (xf - 1) + g[1][1] * yf;
    double n01 = g[2][0] * xf + g[2][1] * (yf - 1);
    double n11 = g[3][0] * (xf - 1) + g[3][1] * (yf - 1);
    double u = fade(xf), v = fade(yf), du = dfade(xf), dv = dfade(yf);
    double nx0 = n00 + u * (n10 - n00), nx1 = n01 + u * (n11 - n01);
    *val = nx0 + v * (nx1 - nx0);
    /* partial derivatives */
    double dn00x = g[0][0], dn00y = g[0][1], dn10x = g[1][0], dn10y = g[1][1];
    double dn01x = g[2][0], dn01y = g[2][1], dn11x = g[3][0], dn11y = g[3][1];
    double dnx0_dx = dn00x + du * (n10 - n00) + u * (dn10x - dn00x);
    double dnx1_dx = dn01x + du * (n11 - n01) + u * (dn11x - dn01x);
    double dnx0_dy = dn00y + u * (dn10y - dn00y);
    double dnx1_dy = dn01y + u * (dn11y - dn01y);
    *dx = dnx0_dx + v * (dnx1_dx - dnx0_dx);
    *dy = dnx0_dy + dv * (nx1 - nx0) + v * (dnx1_dy - dnx0_dy);
}

void syn_ground_height(const int32_t *perm, double amp, double scale, int n, const double *xy,
                       double *z) {
    for (int k = 0; k < n; k++) {
        double v, dx, dy;
        noise2(perm, xy[2 * k] / scale, xy[2 * k + 1] / scale, &v, &dx, &dy);
        z[k] = amp * v;
    }
}

/* ---------------- ray casting ---------------- */

typedef struct {
    double t;
    double n[3];
    int id;
} hit_t;

static void try_hit(hit_t *h, double t, double nx, double ny, double nz, int id) {
    if (t > 1e-9 && t < h->t) {
        h->t = t;
        h->n[0] = nx;
        h->n[1] = ny;
        h->n[2] = nz;
        h->id = id;
    }
}

static void cast(const syn_scene *sc, const double o[3], const double d[3], hit_t *h,
                 const int *cyl_list, int ncand) {
    /* room interior: leaving distance of the box the ray starts in */
    if (sc->has_room) {
        for (int a = 0; a < 3; a++) {
            if (d[a] > 0) {
                double t = (sc->room[3 + a] - o[a]) / d[a];
                double n[3] = {0, 0, 0};
                n[a] = -1.0;
                try_hit(h, t, n[0], n[1], n[2], 1 + a * 2);
            } else if (d[a] < 0) {
                double t = (sc->room[a] - o[a]) / d[a];
                double n[3] = {0, 0, 0};
                n[a] = 1.0;
                try_hit(h, t, n[0], n[1], n[2], 2 + a * 2);
            }
        }
    }
    /* solid boxes, slab test */
    for (int b = 0; b < sc->nbox; b++) {
        const double *bx = sc->boxes + 6 * b;
        double tn = -INFINITY, tf = INFINITY;
        int ax = -1;
        double sgn = 0;
        int miss = 0;
        for (int a = 0; a < 3; a++) {
            if (d[a] == 0.0) {
                if (o[a] < bx[a] || o[a] > bx[3 + a]) miss = 1;
                continue;
            }
            double t1 = (bx[a] - o[a]) / d[a], t2 = (bx[3 + a] - o[a]) / d[a];
            double lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
            if (lo > tn) {
                tn = lo;
                ax = a;
                sgn = d[a] > 0 ? -1.0 : 1.0;
            }
            if (hi < tf) tf = hi;
        }
        if (!miss && ax >= 0 && tn <= tf && tn > 0) {
            double n[3] = {0, 0, 0};
            n[ax] = sgn;
            try_hit(h, tn, n[0], n[1], n[2], 100 + b);
        }
    }
    /* vertical cylinders */
    double dxy2 = d[0] * d[0] + d[1] * d[1];
    if (dxy2 > 0) {
        for (int k = 0; k < ncand; k++) {
            int c = cyl_list ? cyl_list[k] : k;
            const double *cy = sc->cyl + 5 * c;
            double ox = o[0] - cy[0], oy = o[1] - cy[1];
            double B = ox * d[0] + oy * d[1];
            double C = ox * ox + oy * oy - cy[2] * cy[2];
            double disc = B * B - dxy2 * C;
            if (disc < 0) continue;
            double t = (-B - sqrt(disc)) / dxy2;
            if (t <= 0) continue;
            double z = o[2] + t * d[2];
            if (z < cy[3] || z > cy[4]) continue;
            double hx = ox + t * d[0], hy = oy + t * d[1];
            try_hit(h, t, hx / cy[2], hy / cy[2], 0.0, 10000 + c);
        }
    }
    /* facades */
    for (int f = 0; f < sc->nfac; f++) {
        const double *fc = sc->fac + 6 * f;
        double ex = fc[2] - fc[0], ey = fc[3] - fc[1];
        double len = sqrt(ex * ex + ey * ey);
        double nx = -ey / len, ny = ex / len;
        double den = nx * d[0] + ny * d[1];
        if (den == 0) continue;
        double t = (nx * (fc[0] - o[0]) + ny * (fc[1] - o[1])) / den;
        if (t <= 0) continue;
        double px = o[0] + t * d[0] - fc[0], py = o[1] + t * d[1] - fc[1];
        double s = (px * ex + py * ey) / (len * len);
        double z = o[2] + t * d[2];
        if (s < 0 || s > 1 || z < fc[4] || z > fc[5]) continue;
        double sg = den > 0 ? -1.0 : 1.0;
        try_hit(h, t, sg * nx, sg * ny, 0.0, 20000 + f);
    }
    /* ground height field: Newton from the flat-plane intersection */
    if (sc->has_ground && d[2] < 0) {
        double t = -o[2] / d[2];
        if (t - 4.0 * sc->g_amp / (-d[2]) < h->t) {
            int ok = 0;
            double gx = 0, gy = 0;
            for (int it = 0; it < 30; it++) {
                double x = o[0] + t * d[0], y = o[1] + t * d[1];
                double v, dx, dy;
                noise2(sc->perm, x / sc->g_scale, y / sc->g_scale, &v, &dx, &dy);
                gx = sc->g_amp * dx / sc->g_scale;
                gy = sc->g_amp * dy / sc->g_scale;
                double f = o[2] + t * d[2] - sc->g_amp * v;
                double fp = d[2] - gx * d[0] - gy * d[1];
                if (fp >= 0) break;
                double step = f / fp;
                t -= step;
                if (fabs(step) < 1e-12 * (1.0 + t)) {
                    ok = 1;
                    break;
                }
            }
            if (ok) {
                double nn = sqrt(gx * gx + gy * gy + 1.0);
                try_hit(h, t, -gx / nn, -gy / nn, 1.0 / nn, 30000);
            }
        }
    }
}

typedef struct {
    const syn_scene *sc;
    const syn_geom *g;
    const double *R; /* world <- sensor, row-major */
    const double *o;
    double *range;   /* [rows][cols] */
    double *normal;  /* [rows][cols][3], sensor frame, may be NULL */
    int32_t *hit_id; /* may be NULL */
    int row0, row1;
    const int *bin_start, *bin_items;
    int nbins;
    const double *Rcol, *ocol; /* per-column poses (a sweep taken while moving), or NULL */
} job_t;

static void *render_rows(void *arg) {
    job_t *jb = (job_t *)arg;
    const syn_geom *g = jb->g;
    const double *R = jb->R;
    for (int i = jb->row0; i < jb->row1; i++) {
        double el = g->el_top - i * g->d_el;
        double ce = cos(el), se = sin(el);
        for (int j = 0; j < g->cols; j++) {
            double az = 2.0 * M_PI * (double)j / (double)g->cols;
            double u[3] = {ce * cos(az), ce * sin(az), se};
            double d[3];
            const double *Rj = jb->Rcol ? jb->Rcol + 9 * (size_t)j : R;
            const double *oj = jb->ocol ? jb->ocol + 3 * (size_t)j : jb->o;
            for (int a = 0; a < 3; a++) d[a] = Rj[3 * a] * u[0] + Rj[3 * a + 1] * u[1] + Rj[3 * a + 2] * u[2];
            hit_t h;
            h.t = INFINITY;
            h.id = 0;
            h.n[0] = h.n[1] = h.n[2] = 0;
            const int *list = NULL;
            int ncand = jb->sc->ncyl;
            if (jb->nbins > 0 && jb->sc->ncyl > 0) {
                double a = atan2(d[1], d[0]);
                if (a < 0) a += 2.0 * M_PI;
                int b = (int)(a / (2.0 * M_PI) * jb->nbins);
                if (b >= jb->nbins) b = jb->nbins - 1;
                list = jb->bin_items + jb->bin_start[b];
                ncand = jb->bin_start[b + 1] - jb->bin_start[b];
            }
            cast(jb->sc, oj, d, &h, list, ncand);
            size_t px = (size_t)i * g->cols + j;
            int valid = isfinite(h.t) && h.t <= g->r_max;
            jb->range[px] = valid ? h.t : 0.0;
            if (jb->normal) {
                for (int a = 0; a < 3; a++) {
                    /* sensor-frame normal = R^T n_world */
                    jb->normal[3 * px + a] =
                        valid ? Rj[a] * h.n[0] + Rj[3 + a] * h.n[1] + Rj[6 + a] * h.n[2] : 0.0;
                }
            }
            if (jb->hit_id) jb->hit_id[px] = valid ? h.id : 0;
        }
    }
    return NULL;
}

/* Build an azimuth-bin index of cylinders as seen from the sensor origin. */
static int build_bins(const syn_scene *sc, const double o[3], int nbins, int **start, int **items) {
    int *cnt = (int *)calloc(nbins + 1, sizeof(int));
    int total = 0;
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            *start = (int *)malloc((nbins + 1) * sizeof(int));
            int acc = 0;
            for (int b = 0; b < nbins; b++) {
                (*start)[b] = acc;
                acc += cnt[b];
                cnt[b] = 0;
            }
            (*start)[nbins] = acc;
            total = acc;
            *items = (int *)malloc((total > 0 ? total : 1) * sizeof(int));
        }
        for (int c = 0; c < sc->ncyl; c++) {
            const double *cy = sc->cyl + 5 * c;
            double dx = cy[0] - o[0], dy = cy[1] - o[1];
            double dist = sqrt(dx * dx + dy * dy);
            double half;
            if (dist <= cy[2] * 1.05 + 1e-9) {
                half = M_PI; /* sensor inside or touching: test everywhere */
            } else {
                half = asin(cy[2] / dist) + 2.0 * M_PI / nbins;
            }
            double beta = atan2(dy, dx);
            int nb = (int)ceil(half / (2.0 * M_PI) * nbins) + 1;
            int bc = (int)floor((beta < 0 ? beta + 2 * M_PI : beta) / (2.0 * M_PI) * nbins);
            if (nb * 2 + 1 >= nbins) {
                for (int b = 0; b < nbins; b++) {
                    if (pass == 0) cnt[b]++;
                    else (*items)[(*start)[b] + cnt[b]++] = c;
                }
            } else {
                for (int k = -nb; k <= nb; k++) {
                    int b = ((bc + k) % nbins + nbins) % nbins;
                    if (pass == 0) cnt[b]++;
                    else (*items)[(*start)[b] + cnt[b]++] = c;
                }
            }
        }
    }
    free(cnt);
    return total;
}

/*
 * Render one panorama.  R (world <- sensor, row-major 3x3) and o (sensor origin)
 * give the sensor pose.  Pixel (i, j) looks along elevation el_top - i*d_el and
 * azimuth 2*pi*j/cols.  range[i][j] = distance to the first hit, or 0 when there
 * is none within r_max.  normal (optional) receives the exact normal of the hit
 * primitive in the sensor frame, facing the sensor.
 */
int syn_render(const syn_scene *sc, const syn_geom *g, const double *R, const double *o,
               double *range, double *normal, int32_t *hit_id, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    int nbins = 2048;
    int *bs = NULL, *bi = NULL;
    if (sc->ncyl > 0) build_bins(sc, o, nbins, &bs, &bi);
    else nbins = 0;
    job_t jobs[64];
    pthread_t th[64];
    int per = (g->rows + nthreads - 1) / nthreads;
    int nj = 0;
    for (int k = 0; k < nthreads; k++) {
        int r0 = k * per, r1 = r0 + per;
        if (r1 > g->rows) r1 = g->rows;
        if (r0 >= r1) break;
        jobs[nj] = (job_t){sc, g, R, o, range, normal, hit_id, r0, r1, bs, bi, nbins, NULL, NULL};
        nj++;
    }
    for (int k = 1; k < nj; k++) pthread_create(&th[k], NULL, render_rows, &jobs[k]);
    if (nj > 0) render_rows(&jobs[0]);
    for (int k = 1; k < nj; k++) pthread_join(th[k], NULL);
    free(bs);
    free(bi);
    return 0;
}

/*
 * Render a sweep taken while the sensor moves: column j is captured from its
 * own pose (Rcol + 9 j world <- sensor, ocol + 3 j origin).  No azimuth bins
 * (the origin changes from column to column): every cylinder is tested.
 */
int syn_render_sweep(const syn_scene *sc, const syn_geom *g, const double *Rcol, const double *ocol, double *range,
                     int nthreads) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 64) nthreads = 64;
    job_t jobs[64];
    pthread_t th[64];
    int per = (g->rows + nthreads - 1) / nthreads;
    int nj = 0;
    for (int k = 0; k < nthreads; k++) {
        int r0 = k * per, r1 = r0 + per;
        if (r1 > g->rows) r1 = g->rows;
        if (r0 >= r1) break;
        jobs[nj] = (job_t){sc, g, Rcol, ocol, range, NULL, NULL, r0, r1, NULL, NULL, 0, Rcol, ocol};
        nj++;
    }
    for (int k = 1; k < nj; k++) pthread_create(&th[k], NULL, render_rows, &jobs[k]);
    if (nj > 0) render_rows(&jobs[0]);
    for (int k = 1; k < nj; k++) pthread_join(th[k], NULL);
    return 0;
}

