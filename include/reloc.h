/*
 * reloc.h -- C ABI of the MI355X (gfx950) regression-forest relocaliser.
 *
 * The operation is the per-sub-scene relocaliser of Golodetz et al.,
 * "Collaborative Large-Scale Dense 3D Reconstruction with Online Inter-Agent
 * Pose Optimisation": a regression forest trained online from the posed
 * RGB-D frames of one agent (Sec. 3.3), which, given an RGB-D frame of
 * another agent's scene, either fails or returns an estimated pose of that
 * frame in its own coordinate system (Sec. 3.3.1, Fig. 4). Its leaves hold a
 * bounded set of 3D modes (at most 10 or 50, Sec. 4.2.2);
 * new forests start with empty leaves and improve as frames arrive
 * (Sec. 4.3.1); their training samples can be deleted once trained
 * (Sec. 4.3.2). A relocalisation is correct within 5 cm and 5 degrees
 * (Table 2). The paper treats the relocaliser as a black box; the rules for
 * features, reservoirs, modes, hypotheses, energies and culls are this
 * library's definition and are the same rules the CPU oracle implements.
 *
 * Conventions
 *  - Every function returns an int status: 0 = RELOC_OK, < 0 = error,
 *    > 0 = a relocalisation outcome that is not an error (RELOC_FAIL_*).
 *    No exception crosses the ABI.
 *  - Frames are caller-owned DEVICE pointers: depth uint16 [H][W] in mm,
 *    rgb uint8 [H][W][3], contiguous, row-major. They are read in stream
 *    order during the call; the library keeps no reference afterwards.
 *  - Poses are host arrays: row-major float64 4x4 camera-to-world; the
 *    translation column is the camera centre.
 *  - Streams are hipStream_t passed as void* (NULL = the null stream).
 *    reloc_relocalise is synchronous on its stream (it writes a host pose);
 *    every other call is stream-asynchronous.
 *  - A forest handle owns all of its device memory and is not thread-safe;
 *    different handles are independent.
 */
#ifndef RELOC_H
#define RELOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum reloc_status {
    RELOC_OK = 0,
    RELOC_FAIL_NO_VALID_PIXELS = 1,  /* the query frame has no depth in [depth_min, depth_max] */
    RELOC_FAIL_NO_MODES = 2,         /* the forest has never received a sample */
    RELOC_FAIL_NO_HYPOTHESIS = 3,    /* no hypothesis passed its checks in max_tries tries */
    RELOC_E_ARG = -1,                /* null pointer, bad size, bad parameter, non-rigid pose */
    RELOC_E_NOMEM = -2,              /* device allocation failed */
    RELOC_E_HIP = -3,                /* a HIP runtime call failed */
    RELOC_E_STATE = -4,              /* operation not valid in this state (e.g. adapt after drop) */
    RELOC_E_RANGE = -5,              /* a value does not fit the packed device layout */
    RELOC_E_IO = -6                  /* a checkpoint file cannot be written or read, or is not one */
};

typedef struct reloc_forest reloc_forest;

/* Intrinsics are rejected (RELOC_E_ARG) unless width and height are in
 * 1..8191, the focal lengths are positive, below 2^20 px with F =
 * round(16 f) below 2^24, |offset| * F < 2^31 and |offset| * F < 2^14 *
 * depth_min_mm * f_ref (per axis; so every probe offset stays below 2^14
 * px), and cx, cy are finite. */
typedef struct {
    int32_t width, height;           /* frame size in pixels */
    float fx, fy, cx, cy;            /* pinhole intrinsics in pixels */
} reloc_intrinsics;

/* Method parameters. reloc_params_default fills the 320x240 single-attempt
 * configuration: 5 trees of depth 10, 256-entry reservoirs, <= 10 modes,
 * 256 hypotheses, 64 pixels per cull round. */
typedef struct {
    int32_t n_trees;          /* T, 1..16 */
    int32_t depth;            /* D: 2^D leaves and 2^D - 1 split nodes per tree, 1..16 */
    int32_t reservoir_size;   /* R samples kept per leaf, 1..1024 */
    int32_t max_modes;        /* M modes per leaf, 1..64 (T * M <= 512) */
    uint64_t seed;            /* forest seed: split parameters and reservoir draws */
    int32_t depth_min_mm, depth_max_mm;   /* valid depth range (inclusive) */
    int32_t offset_pxmm;      /* split offsets uniform in [-O, O] px*mm at the reference focal length */
    int32_t f_ref_px16;       /* reference focal length in 1/16 px */
    int32_t thr_depth_mm;     /* depth-split thresholds uniform in [-thr, thr] mm */
    int32_t thr_rgb;          /* colour-split thresholds uniform in [-thr, thr] */
    int32_t dens_radius_mm;   /* mode finding: density radius */
    int32_t link_radius_mm;   /* mode finding: link radius */
    int32_t min_cluster;      /* minimum cluster size; <= 0 means max(3, R / 64) */
    int32_t cov_reg_mm2;      /* covariance regulariser added to the diagonal */
    int32_t n_hypotheses;     /* N pose hypotheses per attempt, 1..4096 */
    int32_t batch_pixels;     /* B pixels scored per cull round, 1..2048 */
    int32_t max_tries;        /* tries per hypothesis, 1..1024 */
    int32_t refine;           /* 1: Kabsch refinement of the survivors on their inliers */
    int32_t rgb_tol;          /* hypothesis modes must match the pixel colour within this, per channel (>= 0) */
    float rigid_ratio2;       /* squared-distance ratio bound between camera and world triangles */
    float min_pair2_m2;       /* minimum squared distance between hypothesis camera points */
    float min_area2_m4;       /* minimum |e1 x e2|^2 of the hypothesis camera triangle */
    float resid_m;            /* maximum residual of a hypothesis on its own three points */
    float inlier_m;           /* inlier radius around the best mode */
} reloc_params;

/* Fills *out with the defaults described above. */
int reloc_params_default(reloc_params *out);

/* Creates a forest on the current device: draws the split parameters from
 * `p->seed` on the GPU and allocates reservoirs (T * 2^D * R * 16 B), slot
 * stamps (T * 2^D * R * 4 B) and modes (T * 2^D * M * 48 B), all empty.
 * Returns RELOC_E_ARG for out-of-range parameters, RELOC_E_RANGE when the
 * offsets or thresholds do not fit the packed 8-byte split nodes. */
int reloc_forest_create(const reloc_params *p, void *stream, reloc_forest **out);

/* Frees the forest after the work queued on its streams has finished. */
int reloc_forest_destroy(reloc_forest *f);

/* Online adaptation with one posed frame (Sec. 3.3: the relocaliser is
 * trained online from the agent's posed frames). For every tree, the valid
 * pixels are offered to their leaves in raster order; leaf reservoirs follow
 * Algorithm R with counter-based draws keyed by (tree, leaf, k). Leaves that
 * changed are marked for mode extraction. `K->width * K->height` pixels are
 * read from depth_dev / rgb_dev. Asynchronous on `stream`. Errors:
 * RELOC_E_ARG (null pointer, bad intrinsics, pose not a rigid motion),
 * RELOC_E_STATE (reservoirs dropped). */
int reloc_adapt_frame(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                      const reloc_intrinsics *K, const double pose_c2w[16], void *stream);

/* Extracts the modes of every leaf changed since the last call (at most
 * max_modes per leaf; Sec. 4.2.2). Relocalisation calls it implicitly.
 * Asynchronous on `stream`. */
int reloc_update_modes(reloc_forest *f, void *stream);

/* Relocalises one RGB-D frame (Fig. 4): features and traversal of every
 * valid pixel, n_hypotheses three-point Kabsch hypotheses, preemptive
 * scoring with halving culls and inlier refinement. On RELOC_OK writes the
 * pose (camera-to-world, host array) and the inlier fraction of the final
 * hypothesis; on RELOC_FAIL_* writes the identity and 0. n_hypotheses <= 0
 * uses the forest's parameter. pixel_weights_dev (may be NULL) is a device
 * array of H*W uint32 integer sampling weights for the hypothesis pixel
 * picks (learned proposal); NULL picks uniformly over valid pixels.
 * Synchronous on `stream`. */
int reloc_relocalise(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                     const reloc_intrinsics *K, uint64_t attempt_seed, int32_t n_hypotheses,
                     const uint32_t *pixel_weights_dev, double pose_c2w_out[16], float *score_out,
                     void *stream);

/* Everything one attempt reports. */
typedef struct {
    double pose_c2w[16];     /* camera-to-world; identity on failure */
    float score;             /* inlier fraction of the returned hypothesis over all draws scored */
    int32_t status;          /* RELOC_OK or RELOC_FAIL_* */
    int32_t n_rounds;        /* cull rounds run */
    int32_t final_hyp;       /* index of the returned hypothesis, -1 on failure */
    int32_t pool_size;       /* valid pixels of the frame */
    int32_t n_valid;         /* hypotheses that passed their checks */
    uint64_t mode_evals;     /* (hypothesis, draw, mode) energy terms evaluated */
    uint64_t pair_evals;     /* (hypothesis, draw) pairs scored */
} reloc_result;

/* reloc_relocalise with the full result. Synchronous on `stream`. */
int reloc_relocalise_ex(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                        const reloc_intrinsics *K, uint64_t attempt_seed, int32_t n_hypotheses,
                        const uint32_t *pixel_weights_dev, reloc_result *result_out, void *stream);

/* ---- batched relocalisation ----
 * Many attempts, against one or several forests, with frames of different
 * sizes and different hypothesis counts, run as one launch of a captured
 * HIP graph whose kernels walk ragged per-attempt work lists. Each attempt's
 * result is bit-identical to reloc_relocalise_ex on the same arguments (the
 * same kernels run both; the plain call is a batch of one). Not in the
 * paper, which schedules one attempt at a time (Sec. 3.3.1, Sec. 4.3.1). */
typedef struct {
    reloc_forest *forest;              /* target forest */
    const uint16_t *depth_dev;         /* device depth [H][W] mm */
    const uint8_t *rgb_dev;            /* device rgb [H][W][3] */
    reloc_intrinsics K;
    uint64_t seed;                     /* attempt seed (hypothesis and pixel draws) */
    int32_t n_hypotheses;              /* <= 0: the forest's parameter */
    const uint32_t *pixel_weights_dev; /* device [H*W] pick weights, or NULL for uniform picks */
    const struct reloc_mlp *proposal;  /* learned proposal computed inside the batch from the
                                          attempt's own leaves (same weights as
                                          reloc_mlp_pixel_weights), or NULL; not together
                                          with pixel_weights_dev (RELOC_E_ARG) */
} reloc_attempt;

typedef struct reloc_batch reloc_batch;

/* A batch handle caches, per batch shape (attempt count and each attempt's
 * frame size, hypothesis count and forest dimensions), a scratch arena and an
 * instantiated graph. Not thread-safe. */
int reloc_batch_create(reloc_batch **out);
int reloc_batch_destroy(reloc_batch *b);

/* Runs n >= 1 attempts and writes n results to results_host. The first call
 * with a new shape captures its graph and, with tuning on, times a few
 * schedules (draws per scoring unit, persistent grid size, XCD-contiguous
 * unit order) and keeps the fastest; results do not depend on the schedule.
 * Synchronous on `stream`. RELOC_E_ARG for a bad attempt (its index is not
 * reported; check attempts individually with reloc_relocalise_ex). */
int reloc_relocalise_batch(reloc_batch *b, const reloc_attempt *attempts, int32_t n,
                           reloc_result *results_host, void *stream);

/* 1 (default): tune schedules on the first call of each shape; 0: use the
 * fixed default schedule. */
int reloc_batch_set_tuning(reloc_batch *b, int32_t on);

/* Text description of the schedule chosen for the most recent shape. */
int reloc_batch_schedule(const reloc_batch *b, char *desc, int32_t cap);

/* Device bytes held by the batch handle (arenas of cached shapes). */
int reloc_batch_memory(const reloc_batch *b, uint64_t *bytes_out);

/* Builds every pending mode, then frees the reservoirs and slot stamps (the
 * paper deletes a relocaliser's training data once it is trained,
 * Sec. 4.3.2). Relocalisation results are unchanged; further adaptation
 * returns RELOC_E_STATE. */
int reloc_forest_drop_reservoirs(reloc_forest *f, void *stream);

/* Checkpoint of a forest (the paper trains each relocaliser online and can
 * delete its training data once trained, Sec. 4.3.2; a saved forest resumes
 * exactly where it stopped). reloc_forest_save builds every pending mode and
 * writes the split nodes, leaf counters, modes and, unless they were dropped,
 * the reservoirs to the file at `path` (a 640x480-class forest of 5 trees of
 * depth 15 with 1024-entry reservoirs is about 2.8 GB; about 85 MB after
 * reloc_forest_drop_reservoirs). reloc_forest_load creates a new forest on the
 * current device from such a file: adapting it further, or relocalising with
 * it, gives bit for bit what the saved forest would have given. Both are
 * synchronous on `stream`. Errors: RELOC_E_ARG (null pointer), RELOC_E_IO (the
 * file cannot be opened, written or read, or has the wrong magic, version,
 * sizes or trailing bytes), RELOC_E_RANGE (a stored split node does not fit
 * the stored parameters), the errors of reloc_forest_create. */
int reloc_forest_save(reloc_forest *f, const char *path, void *stream);
int reloc_forest_load(const char *path, void *stream, reloc_forest **out);

/* The parameters the forest was created (or loaded) with. */
int reloc_forest_params(const reloc_forest *f, reloc_params *out);

/* One posed training frame: device depth (uint16 mm, [H][W]) and colour
 * (uint8 RGB, [H][W][3]) owned by the caller, its intrinsics and its
 * camera-to-world pose (row-major 4x4, a rigid motion). */
typedef struct {
    const uint16_t *depth_dev;
    const uint8_t *rgb_dev;
    reloc_intrinsics K;
    double pose_c2w[16];
} reloc_train_frame;

/* Split training: replaces the forest's split nodes (not the 8 extra feature
 * nodes of the learned proposal) by splits learned from posed frames of one
 * scene, and empties every leaf; reloc_adapt_frame then fills the leaves
 * from frames of any scene (the paper's forest is pre-trained on one scene
 * and adapted online to the others, Sec. 4.2.2, Table 2). Every node, level
 * by level from the root, takes from n_candidates (1..64) candidate splits,
 * drawn like random ones from the generator keyed by (seed, 8) at counter
 * (tree, node, candidate, 0), the one that minimises the summed squared
 * deviation of its training samples' world points (integer mm, as adaptation
 * stores them) from their child's mean, ties to the lower candidate; a
 * sample is every stride-th pixel in u and v, from stride / 2, of every
 * frame with a valid depth. Synchronous on `stream` (it reads per-level
 * sample counts back); allocates its scratch with hipMallocAsync on
 * `stream` and frees it before returning. Errors: RELOC_E_ARG (null
 * pointers, n_frames < 1, stride < 1, n_candidates outside 1..64, a frame
 * the forest rejects, a pose that is not a rigid motion), RELOC_E_RANGE
 * (more than 2^31 samples over the trees), RELOC_E_STATE (reservoirs
 * dropped), RELOC_E_NOMEM, RELOC_E_HIP. */
int reloc_forest_train(reloc_forest *f, const reloc_train_frame *frames, int32_t n_frames, int32_t stride,
                       int32_t n_candidates, void *stream);

/* Device bytes currently held by the forest. */
int reloc_forest_memory(const reloc_forest *f, uint64_t *bytes_out);

/* A short English description of a status code (static storage). */
const char *reloc_status_string(int code);

/* ---- verification of a proposed pose (Sec. 3.3.1, Eqs. 3-4) ----
 * da_dev, db_dev: device depth images [H][W] in mm. da is the depth of the
 * target sub-scene rendered at the proposed pose (the paper's D_a), db the
 * depth of the frame that was relocalised (D_b); a pixel is valid in an image
 * when its depth is > 0. valid_frac = (pixels valid in da) / (W H), the test
 * that the proposed pose points at the reconstructed sub-scene; mu_m = mean
 * |da - db| over pixels valid in both, in metres (+inf when there are none);
 * accept = valid_frac > 0.5 and mu_m < 0.05. Sums are exact integers.
 * Synchronous on `stream`. */
int reloc_verify(const uint16_t *da_dev, const uint16_t *db_dev, int32_t W, int32_t H, double *valid_frac,
                 double *mu_m, int32_t *accept, void *stream);

/* reloc_verify for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and results, with their partial sums in a 48 KiB array the
 * library holds on each GPU it runs on until the process ends, instead of
 * scratch taken from the stream's allocator. Frames up to 8191 x 8191
 * (RELOC_E_ARG beyond); every frame size fits the array, whose partial pass is
 * capped at 2048 workgroups. Nothing in it needs clearing between calls (each
 * call writes every partial it reads). Calls that overlap in time on one GPU
 * share the array and race: serialise them (one stream, or wait for the
 * previous call). Synchronous on `stream`. */
int reloc_verify_noalloc(const uint16_t *da_dev, const uint16_t *db_dev, int32_t W, int32_t H, double *valid_frac,
                         double *mu_m, int32_t *accept, void *stream);

/* ---- inter-agent scheduling and pose optimisation (Sec. 3.3.1, 3.3.2) ----
 * Host-side steps around the relocaliser; host arrays, no device work.
 * Poses are row-major FP64 4x4 camera-to-world matrices of a frame in one
 * sub-scene's coordinates; relative transforms and global poses map the
 * coordinates of one sub-scene into another's (or the global frame's). */

/* The relative transform sample of a verified relocalisation (Sec. 3.3.1,
 * after Eq. 4): pose_in_a is the frame's relocalised pose in sub-scene a,
 * pose_in_b its own pose in sub-scene b; a_T_b = pose_in_a pose_in_b^-1 maps
 * b's coordinates to a's (the paper's (fT_a)^-1 fT_b, whose poses fT_s map
 * sub-scene coordinates to the camera's). */
int reloc_relative_transform(const double pose_in_a[16], const double pose_in_b[16], double a_T_b[16]);

typedef struct reloc_collab reloc_collab;

/* State of one collaborative session over n_scenes sub-scenes (2..4096);
 * scene 0 is the first agent's, whose global pose is the identity. */
int reloc_collab_create(int32_t n_scenes, uint64_t seed, reloc_collab **out);
int reloc_collab_destroy(reloc_collab *c);
/* the local poses of the frames of one scene: poses [n][16], copied */
int reloc_collab_set_frames(reloc_collab *c, int32_t scene, const double *poses, int32_t n);
/* Chooses the next attempt (Sec. 3.3.1): draws n_cand candidates
 * k = (a, (b, i)), candidate j of scheduling round r from Philox4x64-10 with
 * key (seed, 7) and counter (r, j, 0, 0): the first output picks an ordered
 * pair of distinct scenes uniformly (pair index p over n (n - 1): a = p /
 * (n - 1), then b = the (p mod (n - 1))-th scene other than a), the second a
 * frame of b uniformly (floor(u m / 2^64)). Each is scored by Phi =
 * phi_new - phi_conf - phi_homog (Eqs. 1-2): phi_new = 1 if exactly one of a
 * and b is in the pose graph of the last reloc_collab_optimise, phi_conf =
 * max(0, max over the pair's clusters of (size - 2)), phi_homog = 5 if frame
 * i's local pose is within 5 cm and 5 deg of a frame of b already tried
 * against a (reloc_collab_tried). Writes the first candidate with the largest
 * score; cands_out (may be NULL) receives [n_cand][7] floats (a, b, i, Phi,
 * phi_new, phi_conf, phi_homog). RELOC_E_STATE until every scene has frames. */
int reloc_collab_schedule(reloc_collab *c, int32_t n_cand, int32_t *a_out, int32_t *b_out, int32_t *frame_out,
                          float *cands_out);
/* records that frame `frame` of scene b was relocalised against scene a */
int reloc_collab_tried(reloc_collab *c, int32_t a, int32_t b, int32_t frame);
/* Adds a verified sample a_T_b (Sec. 3.3.2, Sec. 4.2.4): it joins the first
 * cluster of the pair {a, b} that holds a sample within 20 deg and 10 cm of
 * it, or starts a new one; *cluster_size (may be NULL) receives the size of
 * that cluster. Samples of a pair are compared in one orientation (a b_T_a
 * is inverted). */
int reloc_collab_add_sample(reloc_collab *c, int32_t a, int32_t b, const double a_T_b[16], int32_t *cluster_size);
/* the pair's clusters in creation order: sizes [cap], and (may be NULL) the
 * dual-quaternion blend of each as a_T_b, blended [cap][16]; *n_out = count */
int reloc_collab_clusters(const reloc_collab *c, int32_t a, int32_t b, int32_t *sizes, double *blended, int32_t cap,
                          int32_t *n_out);
/* Pose-graph optimisation (Sec. 3.3.2, Eq. 5): G' joins every pair whose
 * largest cluster (the earliest on ties) holds at least 2 samples, with the
 * equal-weight dual-quaternion blend of that cluster (Kavan et al. 2006) as
 * the edge's transform; G is the connected component of G' holding scene 0.
 * Starting from poses chained breadth first from scene 0 (gT_b = gT_a aT_b),
 * Levenberg-Marquardt minimises the sum over G's edges of
 * |v(gT_b^-1 gT_a aT_b)|^2, v(T) = (imaginary part of T's rotation quaternion
 * with non-negative real part, T's translation), with gT_0 = I. Writes
 * in_graph [n] (1 for scenes of G), global_poses [n][16] (gT_s; identity
 * outside G) and the final cost (any of them may be NULL). */
int reloc_collab_optimise(reloc_collab *c, int32_t *in_graph, double *global_poses, double *cost_out);

/* ---- learned proposal (an extension; the paper picks pixels uniformly) ----
 * A 24-64-64-1 MLP (ReLU, ReLU, sigmoid) scores each valid pixel of a query
 * frame with the probability that its hypothesis pick (a mode drawn among the
 * colour-consistent modes of its leaves) lies within 5 cm of its world
 * point. floor(sigma 65536) + 1 becomes the pixel's pick weight for
 * hypothesis generation (reloc_relocalise_ex / reloc_attempt
 * pixel_weights_dev); scoring and culls stay uniform.
 *
 * Parameters: 5825 FP32 values, in this order: W1 [64][24], b1 [64],
 * W2 [64][64], b2 [64], w3 [64], b3 (rows are output units). The products
 * run on bfloat16 copies of the inputs, W1, W2, w3 and the hidden
 * activations (round to nearest even), with FP32 accumulation; biases stay
 * FP32. Rows of inputs are bfloat16 [n][32], the 24 inputs then 8 zeros,
 * 16-byte aligned (RELOC_E_ARG otherwise).
 *
 * Per-pixel inputs (reloc_pixel_features), zeros for a pixel with invalid
 * depth: 0 depth / 5000; 1..8 the 8 extra feature responses (depth ones
 * clamped to +-5000 mm and divided by 1000, colour ones divided by 255);
 * 9..20 for the 3 modes of the pixel's leaves with the largest weight
 * pi = n / min(k, R) (ties: lower (tree, mode)): pi, then -log(Sigma^-1_ii) / 10
 * for i = x, y, z (zeros when there are fewer modes); 21 the mean reservoir
 * fill sum_t min(k_t, R) / (T R); 22, 23 u / W, v / H. */
typedef struct reloc_mlp reloc_mlp;

/* Glorot-uniform weights from Philox (key (seed, 5), counter (k, 0, 0, 0),
 * a = sqrt(6 / (fan_in + fan_out)), w = (2 r - 1) a with r the top 24 bits of
 * the first output over 2^24), zero biases, zero Adam state. */
int reloc_mlp_create(uint64_t seed, void *stream, reloc_mlp **out);
int reloc_mlp_destroy(reloc_mlp *m);
/* synchronous copies of the 5825 FP32 parameters */
int reloc_mlp_get_weights(const reloc_mlp *m, float *w_host);
int reloc_mlp_set_weights(reloc_mlp *m, const float *w_host);
/* Gradient of the mean logistic loss over n rows (x_dev [n][32] bfloat16,
 * y_dev [n] uint8 labels, target y / 255) into grad_host [5825], the mean loss into
 * *loss_host (may be NULL). Synchronous on `stream`. */
int reloc_mlp_gradient(reloc_mlp *m, const uint16_t *x_dev, const uint8_t *y_dev, int32_t n, float *grad_host,
                       float *loss_host, void *stream);
/* Adam (beta 0.9, 0.999, eps 1e-8, learning rate lr) over `epochs` passes of
 * max(1, n_rows / batch_rows) minibatches; minibatch s of epoch e draws its
 * batch_rows rows uniformly with replacement by Philox (key (seed, 6),
 * counter (e, s, j, 0)). epoch_loss_host[e] (may be NULL) receives the mean
 * loss of the last minibatch of epoch e. Synchronous when epoch_loss_host is
 * given, stream-asynchronous otherwise. */
int reloc_mlp_train(reloc_mlp *m, const uint16_t *x_dev, const uint8_t *y_dev, int32_t n_rows, int32_t epochs,
                    int32_t batch_rows, float lr, uint64_t seed, float *epoch_loss_host, void *stream);
/* reloc_relocalise_ex with the learned proposal: the pick weights are
 * computed from the attempt's own leaves inside the same graph (no second
 * traversal); the result equals reloc_relocalise_ex with the weights of
 * reloc_mlp_pixel_weights for the same network and frame. The network must
 * stay alive until the call returns (it is synchronous). */
int reloc_relocalise_learned(reloc_forest *f, const reloc_mlp *m, const uint16_t *depth_dev,
                             const uint8_t *rgb_dev, const reloc_intrinsics *K, uint64_t attempt_seed,
                             int32_t n_hypotheses, reloc_result *result_out, void *stream);

/* logits z_dev [n] of rows x_dev [n][32] */
int reloc_mlp_logits(reloc_mlp *m, const uint16_t *x_dev, int32_t n, float *z_dev, void *stream);
/* pick weights weights_dev [H*W] (0 for invalid pixels) and, if prob_dev is
 * not NULL, sigmoid outputs prob_dev [H*W] of every pixel of a query frame */
int reloc_mlp_pixel_weights(reloc_mlp *m, reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                            const reloc_intrinsics *K, uint32_t *weights_dev, float *prob_dev, void *stream);
/* inputs of the pixels pix_dev [n] (indices v W + u): bfloat16 rows
 * x_dev [n][32] and, if xf_dev is not NULL, the FP32 values xf_dev [n][24] */
int reloc_pixel_features(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                         const reloc_intrinsics *K, const int32_t *pix_dev, int32_t n, uint16_t *x_dev, float *xf_dev,
                         void *stream);
/* The valid pixels of an RGB-D frame given to the relocaliser (Sec. 3.3.1):
 * those whose depth lies in the forest's depth range, the test that the
 * features, the adaptation and the relocaliser's pixel pool apply. Writes
 * their indices v W + u, in raster order, to pix_dev (device memory for W H
 * int32 values, owned by the caller), their number to *n_out (host). The
 * frame is described as for reloc_pixel_features. Allocates a small device
 * buffer of block counts for the call and synchronises `stream` before it
 * returns. Returns RELOC_E_ARG for a null forest, buffer or count pointer or
 * an invalid frame, RELOC_E_NOMEM when the buffer cannot be allocated. */
int reloc_valid_pixels(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev, const reloc_intrinsics *K,
                       int32_t *pix_dev, int32_t *n_out, void *stream);

/* training labels: label_dev[i] = round(255 g / c) for pixel pix_dev[i],
 * where c counts the modes of the pixel's leaves that pass the hypothesis
 * pick's colour test (|mode colour - pixel colour| <= rgb_tol per channel)
 * and g those of them within 5 cm of the pixel's world point under pose_c2w
 * (rounded to FP32; the squared distance is (d0 d0 + d1 d1) + d2 d2 in FP32),
 * 0 when c = 0: the probability that the pixel's pick is correct, the
 * network's target (label / 255) */
int reloc_label_pixels(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev, const reloc_intrinsics *K,
                       const double pose_c2w[16], const int32_t *pix_dev, int32_t n, uint8_t *label_dev,
                       void *stream);

/* ---- per-kernel timing (for measurement; off by default) ----
 * When enabled, a relocalisation runs its kernels one by one instead of as
 * its captured graph, behind a short fixed wait on the GPU (so that the host
 * has queued every launch before the first one runs), and every launch is
 * bracketed by two HIP events recorded on its stream, followed by a bare pair
 * of events recorded back to back. reloc_profile_read sums, over all recorded
 * launches of one kernel, the bracket's elapsed time minus the bare pair's
 * (the events' own cost), waiting for them to finish: the kernels' durations
 * as a profiler's kernel trace gives them (within a few per cent on this
 * path). reloc_profile_read_raw returns both sums separately.
 * reloc_profile_kernels writes the comma-separated kernel names seen so far
 * into `names` (NUL-terminated, truncated to cap - 1 bytes);
 * reloc_profile_reset forgets all launches. Process-wide; not for use while a
 * stream is being captured into a graph. */
int reloc_profile_enable(int on);
int reloc_profile_reset(void);
int reloc_profile_read(const char *kernel, double *total_ms, int64_t *launches);
int reloc_profile_read_raw(const char *kernel, double *bracket_ms, double *pair_ms, int64_t *launches);
int reloc_profile_kernels(char *names, int32_t cap);

/* ---- parity and debug exports: synchronous copies into caller HOST buffers ---- */

/* split nodes [T * (2^D - 1)] followed by the 8 per-pixel feature nodes;
 * kind 0 = depth, 1..3 = colour channel */
int reloc_debug_nodes(const reloc_forest *f, int32_t *kind, int32_t *dx, int32_t *dy, int32_t *thr);
/* replaces the split nodes (same layout); RELOC_E_RANGE if a value does not pack */
int reloc_debug_set_nodes(reloc_forest *f, const int32_t *kind, const int32_t *dx, const int32_t *dy,
                          const int32_t *thr);
/* leaf index per tree and pixel, [T][H*W], -1 for invalid pixels */
int reloc_debug_leaves(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                       const reloc_intrinsics *K, int32_t *leaves_host, void *stream);
/* the 8 per-pixel feature responses, [H*W][8], 0 for invalid pixels */
int reloc_debug_features8(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                          const reloc_intrinsics *K, int32_t *feat_host, void *stream);
/* reservoir entries (16 B: int32 x, y, z mm; uint8 r, g, b, pad) of leaves
 * [leaf0, leaf0 + n) of tree t, [n][R], and their counters [n] */
int reloc_debug_reservoir(const reloc_forest *f, int32_t t, int32_t leaf0, int32_t n, void *entries_host,
                          uint32_t *counters_host);
/* modes (48 B: float mu[3], sinv[6], kappa; int32 n; uint8 rgb[3], pad) of
 * leaves [leaf0, leaf0 + n) of tree t, [n][M], and their counts [n] */
int reloc_debug_modes(reloc_forest *f, int32_t t, int32_t leaf0, int32_t n, void *modes_host,
                      int32_t *n_modes_host);
/* modes of an arbitrary point set (host entries, n <= 4096) computed by the
 * GPU mode kernel with the forest's parameters */
int reloc_debug_modes_from_points(reloc_forest *f, const void *entries_host, int32_t n, void *modes_host,
                                  int32_t *n_modes_host);

/* Trace of the most recent reloc_relocalise on this forest (capacities in
 * elements; any pointer may be NULL):
 *   hyp_try [N]: first passing try or -1;  hyp_pose [N][12]: initial R then t
 *   n_rounds; n_alive [rounds]; alive [rounds][N]; energy [rounds][N];
 *   n_inliers [rounds][N] (by position in alive);  final_hyp; pool_size */
typedef struct {
    int32_t cap_hyp, cap_rounds;
    int32_t *pool_size, *hyp_try;
    double *hyp_pose;
    int32_t *n_rounds, *n_alive, *alive;
    float *energy;
    int32_t *n_inliers, *final_hyp;
} reloc_trace;
int reloc_debug_trace(const reloc_forest *f, reloc_trace *tr);

/* Host run of the work-unit ownership rule of the persistent kernels: for a
 * stage of `total` units on a grid of `grid` workgroups, owners_host[u] =
 * number of workgroups that process unit u (every entry must be 1). */
int reloc_debug_unit_owners(int32_t xcd, int32_t total, int32_t grid, int32_t *owners_host);

/* Host run of the pose solver's eigenvector step: for n cross-covariance
 * matrices h_host [n][3][3] (row a, column b: sum of centred c_a w_b), the
 * unit quaternion (w, x, y, z; sign arbitrary) of the best rotation, or NaNs
 * where the closed-form step declines (H = 0 or an exactly repeated largest
 * eigenvalue) and the device falls back to power iteration. */
int reloc_debug_horn(const double *h_host, int32_t n, double *q_host);

/* Host run of the probe-offset division: the truncating quotient
 * delta F / (d F_ref) of a split feature's depth-adaptive offset (the forest
 * of the relocaliser the paper adopts, Sec. 3.3; the paper does not define
 * the features), formed by multiplication: q_host[i] = trunc(n_host[i] /
 * den_host[i]) for count
 * entries, host arrays. RELOC_E_ARG if a divisor is below 1 or a numerator is
 * -2^31 (the kernels' range is |n| < 2^31, 1 <= den < 2^31). */
int reloc_debug_div(const int32_t *n_host, const int32_t *den_host, int32_t count, int32_t *q_host);

/* The kernels' cross-lane helpers applied on one wavefront to v = 1000 + lane:
 * out_host [12][64] receives, per lane, v of lane ^ 1, 2, 4, 8, 16, 32 (rows
 * 0-5), v of lane - 1, 2, 4, 8 within the lane's row of 16 lanes or 0 below
 * the row's start (rows 6-9), the high word of w = (5000 + lane) << 32 | v of
 * lane ^ 2^(lane mod 6) (row 10) and of lane 37 (row 11). Synchronous; allocates
 * 3 KiB of device memory for the call. Returns RELOC_E_ARG for a null buffer. */
int reloc_debug_lane_probe(uint32_t *out_host);

/* One 16x16 product C = A B on the matrix cores as the MLP kernels issue it
 * (bfloat16 operands, FP32 accumulation): a_host [16][32] row-major A,
 * bt_host [16][32] row-major B^T, c_host [16][16] row-major C. Synchronous. */
int reloc_debug_mfma_probe(const uint16_t *a_host, const uint16_t *bt_host, float *c_host);

/* The float -> bfloat16 conversion of the network's inference kernels (the
 * inputs and the two hidden layers), run on the GPU: y_host[i] = bit pattern
 * of x_host[i] rounded to bfloat16, for n host values. Synchronous. */
int reloc_debug_bf16(const float *x_host, int32_t n, uint16_t *y_host);

#ifdef __cplusplus
}
#endif
#endif
