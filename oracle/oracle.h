/*
 * Plain CPU oracle of the regression-forest relocalisation path.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. It shares no code,
 * header or table with the GPU library: it exists to say what the GPU path
 * must compute.
 *
 * The paper (Golodetz et al., "Collaborative Large-Scale Dense 3D
 * Reconstruction with Online Inter-Agent Pose Optimisation") trains a
 * regression-forest relocaliser online for each sub-scene (Sec. 3.3) and uses
 * it as a black box that, given an RGB-D frame, either fails or returns a
 * pose (Sec. 3.3.1, Fig. 4). It fixes the success criterion (<= 5 cm and
 * <= 5 deg, Sec. 4.2.2 / Table 2), the number of leaf modes (at most 10 or 50,
 * Sec. 4.2.2), that forests start with empty leaves and train online
 * (Sec. 4.3.1), and that the training data can be deleted once trained
 * (Sec. 4.3.2). Every other rule below (features, reservoirs, mode finding,
 * hypothesis sampling, energies, culls, refinement) is this implementation's
 * own definition of the method, written out step by step.
 *
 * Conventions: depth is uint16 mm [H][W]; rgb is uint8 [H][W][3]; K is
 * {fx, fy, cx, cy} as float; poses are row-major float64 4x4 camera-to-world.
 * All functions return 0 on success, < 0 on an argument error, > 0 for a
 * non-error outcome (relocalisation failure kinds).
 */
#ifndef RELOC_ORACLE_H
#define RELOC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_trees, depth, reservoir_size, max_modes;
    uint64_t seed;
    int32_t depth_min_mm, depth_max_mm, offset_pxmm, f_ref_px16, thr_depth_mm, thr_rgb;
    int32_t dens_radius_mm, link_radius_mm, min_cluster, cov_reg_mm2;
    int32_t n_hypotheses, batch_pixels, max_tries, refine, rgb_tol;
    float rigid_ratio2, min_pair2_m2, min_area2_m4, resid_m, inlier_m;
} oracle_params;

typedef struct {
    float mu[3];        /* metres */
    float sinv[6];      /* inverse covariance, m^-2: xx, xy, xz, yy, yz, zz */
    float kappa;        /* -log(pi) + 0.5 (3 log 2 pi + log det Sigma) */
    int32_t n;          /* points in the cluster */
    uint8_t rgb[3];
    uint8_t pad;
} oracle_mode;

typedef struct {
    int32_t x, y, z;    /* world position, integer mm */
    uint8_t r, g, b, pad;
} oracle_entry;

/* optional per-attempt trace (every pointer may be NULL) */
typedef struct {
    int32_t cap_hyp, cap_rounds;
    int32_t *pool_size;          /* [1] */
    int32_t *hyp_try;            /* [cap_hyp] first passing try, -1 if none */
    double  *hyp_pose;           /* [cap_hyp][12] initial R (row-major) then t */
    int32_t *n_rounds;           /* [1] */
    int32_t *n_alive;            /* [cap_rounds] |H| before the cull of round r */
    int32_t *alive;              /* [cap_rounds][cap_hyp] hypothesis ids scored in round r */
    float   *energy;             /* [cap_rounds][cap_hyp] E_h after round r (by position in alive) */
    int32_t *n_inliers;          /* [cap_rounds][cap_hyp] running inlier counts after round r */
    double  *pose_after;         /* [cap_rounds][cap_hyp][12] pose after refinement (survivors only) */
    int32_t *final_hyp;          /* [1] */
} oracle_trace;

enum {
    ORACLE_OK = 0,
    ORACLE_FAIL_NO_VALID_PIXELS = 1,
    ORACLE_FAIL_NO_MODES = 2,
    ORACLE_FAIL_NO_HYPOTHESIS = 3,
    ORACLE_E_ARG = -1,
    ORACLE_E_NOMEM = -2,
    ORACLE_E_IO = -6,
};

typedef struct oracle_forest oracle_forest;

/* counter-based generator (Philox4x64-10) and integer range mapping */
void     oracle_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
uint64_t oracle_uniform_int(uint64_t u, uint64_t n);

int  oracle_params_default(oracle_params *p);
int  oracle_forest_create(const oracle_params *p, oracle_forest **out);
void oracle_forest_destroy(oracle_forest *f);
/* nodes: [T][L-1] then the 8 extra feature nodes; kind 0 depth, 1..3 rgb channel */
int  oracle_forest_nodes(const oracle_forest *f, int32_t *kind, int32_t *dx, int32_t *dy, int32_t *thr);
int  oracle_set_nodes(oracle_forest *f, const int32_t *kind, const int32_t *dx, const int32_t *dy,
                      const int32_t *thr);

/* split training on posed frames of equal size and intrinsics (n_cand
 * candidates per node, 1..64; every stride-th pixel); replaces the split
 * nodes (not the 8 extra feature nodes) and empties every leaf */
int  oracle_train_forest(oracle_forest *f, int n_frames, const uint16_t *const *depth, const uint8_t *const *rgb,
                         int W, int H, const float K[4], const double *poses /* [n][16] */, int stride, int n_cand);

int  oracle_camera_point(const uint16_t *depth, int W, int H, const float K[4], int u, int v,
                         const oracle_params *p, float out[3]);
int  oracle_leaves(const oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                   const float K[4], int32_t *leaves /* [T][H*W] */);
int  oracle_features8(const oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                      const float K[4], int32_t *feat /* [H*W][8] */);
int  oracle_adapt_frame(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                        const float K[4], const double pose[16]);
int  oracle_reservoir(const oracle_forest *f, int t, int leaf, oracle_entry *entries /* [R] */,
                      uint32_t *count);
int  oracle_leaf_modes(oracle_forest *f, int t, int leaf, oracle_mode *modes /* [M] */, int32_t *n_modes);
int  oracle_modes_from_points(const oracle_params *p, const oracle_entry *pts, int n,
                              oracle_mode *modes, int32_t *n_modes, int32_t *labels /* [n] or NULL */);
int  oracle_modes_bruteforce(const oracle_params *p, const oracle_entry *pts, int n,
                             oracle_mode *modes, int32_t *n_modes, int32_t *labels);
int  oracle_build_all_modes(oracle_forest *f);
/* checkpoint of the whole forest state in the oracle's own file layout;
 * ORACLE_E_IO for a file that cannot be written or read or is not one */
int  oracle_forest_save(const oracle_forest *f, const char *path);
int  oracle_forest_load(const char *path, oracle_forest **out);
int  oracle_drop_reservoirs(oracle_forest *f);
uint64_t oracle_total_samples(const oracle_forest *f);

int  oracle_kabsch(const double *src, const double *dst, int n, double R[9], double t[3]);
int  oracle_svd3(const double A[9], double U[9], double S[3], double V[9]);

int  oracle_relocalise(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                       const float K[4], uint64_t attempt_seed, int n_hyp,
                       const uint32_t *pixel_weights /* [H*W] or NULL */,
                       double pose_out[16], float *score_out, oracle_trace *trace);

int  oracle_pose_success(const double est[16], const double gt[16], double *dt_m, double *dang_deg);

/* ---- single steps of the relocalisation, exported for their pins ---- */
enum {
    ORACLE_TRI_OK = 0,            /* the triple passes every check */
    ORACLE_TRI_SAME_PIXEL = 1,    /* two picks are the same pool pixel */
    ORACLE_TRI_PAIR_DIST = 2,     /* a camera pair is closer than sqrt(min_pair2) */
    ORACLE_TRI_WORLD_LONGER = 3,  /* world squared distance > rigid_ratio2 * camera squared distance */
    ORACLE_TRI_CAMERA_LONGER = 4, /* camera squared distance > rigid_ratio2 * world squared distance */
    ORACLE_TRI_AREA = 5,          /* camera triangle |e1 x e2|^2 < min_area2 */
    ORACLE_TRI_DEGENERATE = 6,    /* the alignment is undetermined (see oracle_pose_from_sums) */
    ORACLE_TRI_RESIDUAL = 7,      /* a residual |R c + t - w| exceeds resid */
};
/* checks of one hypothesis triple: pool indices pi[3], camera points c[3][3]
 * and picked mode means w[3][3]; the pose on ORACLE_TRI_OK */
int  oracle_check_triple(const oracle_params *p, const int32_t pi[3], const float c[9], const float w[9],
                         double R[9], double t[3]);
/* 1 iff the mode's colour is within rgb_tol of the pixel's in every channel */
int  oracle_colour_ok(const oracle_params *p, const uint8_t mode_rgb[3], const uint8_t px[3]);
/* the FP32 energy term kappa + q / 2 of a mode at y */
float oracle_mode_term(const oracle_mode *md, const float y[3]);
/* pose from correspondence sums {n, sum c (3), sum w (3), sum c w^T (9, row
 * a col b), sum c c^T (xx xy xz yy yz zz)}; 0 and (R, t), or 1 when fewer
 * than 3 points or the camera points are degenerate (I2 < 1e-4 n trace) */
int  oracle_pose_from_sums(const double sums[22], double R[9], double t[3]);
/* the preemptive rounds over caller-given hypotheses: poses [n][12] (R
 * row-major then t), valid [n] */
int  oracle_preemptive(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H, const float K[4],
                       uint64_t attempt_seed, int n_hyp, const double *poses, const int32_t *valid,
                       double pose_out[16], float *score_out, oracle_trace *trace);

/* ---- depth-difference verification (Sec. 3.3.1, Eqs. 3-4) ----
 * valid fraction |Omega_a| / |Omega| of the rendered depth da, and the mean
 * absolute depth difference over pixels valid (> 0) in both, in metres;
 * accept iff the fraction exceeds 0.5 and the mean is below 5 cm. */
int  oracle_verify(const uint16_t *da, const uint16_t *db, int W, int H, double *valid_frac, double *mu_m,
                   int *accept);

/* ---- learned proposal: a 24-64-64-1 MLP over per-pixel features ---- */
#define ORACLE_MLP_NPARAM 5825   /* W1[64][24] b1[64] W2[64][64] b2[64] w3[64] b3 */
float oracle_bf16(float x);      /* round to the nearest bfloat16, ties to even */
/* 24 features of each listed valid pixel (FP32, before bfloat16 rounding) */
int  oracle_features24(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H, const float K[4],
                       const int32_t *pix, int n, float *x /* [n][24] */);
/* round(255 x the probability that the pixel's hypothesis pick is correct
 * under `pose`): the fraction of the colour-consistent modes of its leaves
 * within 5 cm of its world point (the labeller of the learned proposal) */
int  oracle_label(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H, const float K[4],
                  const double pose[16], const int32_t *pix, int n, uint8_t *label);
void oracle_mlp_init(uint64_t seed, float *w /* [5825] */);
/* logits of n rows (inputs rounded to bfloat16 here) */
int  oracle_mlp_forward(const float *w, const float *x, int n, double *z);
/* mean binary cross-entropy of n rows against targets y / 255 and its
 * gradient in FP64 */
int  oracle_mlp_grad(const float *w, const float *x, const uint8_t *y, int n, double *grad /* [5825] */,
                     double *loss);

#ifdef __cplusplus
}
#endif
#endif
