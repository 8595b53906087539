/*
 * Plain FP64 single-threaded reference ("oracle") for the projective-ICP
 * registration path of UPSLAM (Cowley, Miller, Taylor: "UPSLAM: Union of
 * Panoramas SLAM", arXiv 2101.00585).  TEST INFRASTRUCTURE ONLY: the product
 * library never links, loads or calls this code; only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark do.
 *
 * Everything here is written from the paper's description (Section III-A
 * "Data Intake", Section III-B "Motion Estimation" with Equation 1,
 * Section III-C "Keyframe Update") plus the readings listed where the paper
 * is silent.  It shares no code, header, table or constant generator with the
 * GPU library.
 *
 * Array layouts: a depth image is double[rows][cols] (row-major); a surfel
 * image is double[rows][cols][4] = (nx, ny, nz, range) with a zero normal
 * meaning "no normal" and a zero range meaning "no return"; a keyframe count
 * image is uint16[rows][cols].  A pose is double[12]: a row-major rotation
 * R[9] followed by a translation t[3], mapping scan coordinates into keyframe
 * coordinates (x_kf = R x_scan + t).
 */
#ifndef UPSLAM_ORACLE_H
#define UPSLAM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t rows, cols;
    double el_top, d_el; /* elevation of row 0 and row spacing, radians */
    double r_min, r_max; /* a range r is valid iff finite and r_min < r <= r_max */
} orc_geom;

typedef struct {
    int32_t atrous_levels;
    double sigma_n, sigma_r, max_rel_jump;
} orc_normal_params;

typedef struct {
    int32_t levels;
    int32_t iters[4];
    double d_max[4];
    double cos_theta_max;
    double stop_update_norm;
    int32_t min_inliers;
    double irls_delta; /* 0: squared residuals; > 0: |r| by IRLS, weights 1 / max(|r|, irls_delta) */
} orc_icp_params;

typedef struct {
    double T[12];
    double rms, trunc_cost, inlier_ratio;
    int64_t inliers, valid;
    int32_t iters_run, status;
    int32_t level_iters[4];
    double JtJ[21], Jtr[6];
    double last_update_norm;
} orc_icp_result;

typedef struct {
    double d_max, cos_theta_max, min_cos_incidence;
    int32_t max_count;
} orc_fuse_params;

typedef struct {
    double margin_abs, margin_rel; /* free-space margin max(margin_abs, margin_rel * range) */
    int32_t min_count;             /* samples a pixel of the other keyframe needs to vote */
} orc_consistency_params;

enum { ORC_CONVERGED = 0, ORC_MAX_ITERS = 1, ORC_DEGENERATE = 2, ORC_NO_INLIERS = 3 };

void orc_ray(const orc_geom *g, int i, int j, double u[3]);
int orc_project(const orc_geom *g, const double q[3], int32_t *i, int32_t *j);
int orc_raw_normals(const orc_geom *g, const double *depth, double max_rel_jump, double *surfel);
int orc_atrous(const orc_geom *g, const double *in, int levels, double sigma_r, double sigma_n, double *out);
int orc_panorama_normals(const orc_geom *g, const double *depth, const orc_normal_params *p, double *surfel);
int orc_pyramid_level(const orc_geom *g, const double *surfel, int level, double *out);
int orc_residuals(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf, const double T[12],
                  double d_max, double cos_theta_max, int32_t *kf_index, uint8_t *inlier, double *r, double *J);
int orc_normal_equations(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf,
                         const double T[12], double d_max, double cos_theta_max, double A[21], double b[6],
                         double *sum_r2, int64_t *inliers, int64_t *valid);
int orc_normal_equations_irls(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf,
                              const double T[12], double d_max, double cos_theta_max, double delta, double A[21],
                              double b[6], double *sum_r2, int64_t *inliers, int64_t *valid);
int orc_solve6(const double A[21], const double b[6], double xi[6]);
void orc_exp_se3(const double xi[6], double T[12]);
void orc_compose(const double A[12], const double B[12], double out[12]);
int orc_register(const orc_geom *sg, const double *scan, const orc_geom *kg, const double *kf,
                 const double init[12], const orc_icp_params *p, orc_icp_result *res);
int orc_fuse(const orc_geom *sg, const double *scan, const orc_geom *kg, double *kf, uint16_t *kf_count,
             const double T[12], const orc_fuse_params *p);

int orc_free_space_violations(const orc_geom *ga, const double *a, const orc_geom *gb, const double *b,
                              const uint16_t *b_count, const double T_ba[12], const orc_consistency_params *p,
                              uint8_t *mask_a);
int orc_remove_marked(const orc_geom *g, double *surfel, uint16_t *count, const uint8_t *mask);
int orc_splat_sweep(const orc_geom *raw_g, const double *raw, const double *col_T, const orc_geom *out_g,
                    double *out);

#ifdef __cplusplus
}
#endif
#endif
