/* Drives every oracle entry point on small synthetic inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (run by the CPU tests).
 * Exits 0 when every call returns the status it should; the sanitizers abort
 * the run on any memory or undefined-behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                   \
        }                                                               \
    } while (0)

/* a frame of a tilted plane with a box in front, seen from pose T */
static void synth_frame(int W, int H, int shift, uint16_t *depth, uint8_t *rgb)
{
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int p = v * W + u;
            int d = 1500 + 10 * ((u + shift) % 97) + 7 * v;
            if (u > W / 3 && u < W / 2 && v > H / 3 && v < 2 * H / 3) d = 900 + 3 * u;
            if ((u * 7 + v * 3) % 53 == 0) d = 0;     /* holes */
            depth[p] = (uint16_t)d;
            rgb[p * 3 + 0] = (uint8_t)((u * 5 + shift) & 255);
            rgb[p * 3 + 1] = (uint8_t)((v * 3) & 255);
            rgb[p * 3 + 2] = (uint8_t)(((u ^ v) * 11) & 255);
        }
}

int main(int argc, char **argv)
{
    const char *tmp = argc > 1 ? argv[1] : "/tmp/oracle_sanitize.bin";
    const int W = 64, H = 48;
    uint16_t *depth = malloc((size_t)W * H * 2);
    uint8_t *rgb = malloc((size_t)W * H * 3);
    float K[4] = {55.4f, 55.4f, 32.0f, 24.0f};
    oracle_params p;
    CHECK(oracle_params_default(&p) == 0);
    p.n_trees = 3; p.depth = 6; p.reservoir_size = 8; p.max_modes = 5; p.n_hypotheses = 24; p.batch_pixels = 13;
    p.min_cluster = 1; p.rgb_tol = 255;
    oracle_forest *f = NULL;
    CHECK(oracle_forest_create(&p, &f) == 0);
    CHECK(oracle_forest_create(NULL, &f) == ORACLE_E_ARG);
    double pose[16] = {1, 0, 0, 0.1, 0, 1, 0, -0.2, 0, 0, 1, 0.3, 0, 0, 0, 1};
    for (int k = 0; k < 6; ++k) {
        synth_frame(W, H, k, depth, rgb);
        pose[3] = 0.01 * k;
        CHECK(oracle_adapt_frame(f, depth, rgb, W, H, K, pose) == 0);
    }
    double bad[16];
    memcpy(bad, pose, sizeof(bad));
    bad[0] = 2.0;
    CHECK(oracle_adapt_frame(f, depth, rgb, W, H, K, bad) == ORACLE_E_ARG);
    int32_t *leaves = malloc(sizeof(int32_t) * 3 * W * H);
    int32_t *feat = malloc(sizeof(int32_t) * 8 * W * H);
    CHECK(oracle_leaves(f, depth, rgb, W, H, K, leaves) == 0);
    CHECK(oracle_features8(f, depth, rgb, W, H, K, feat) == 0);
    oracle_entry ent[8];
    uint32_t cnt = 0;
    oracle_mode modes[5];
    int32_t nm = 0;
    for (int leaf = 0; leaf < 64; ++leaf) {
        CHECK(oracle_reservoir(f, 1, leaf, ent, &cnt) == 0);
        CHECK(oracle_leaf_modes(f, 1, leaf, modes, &nm) == 0 && nm <= 5);
        if (nm > 0) {
            float y[3] = {modes[0].mu[0] + 0.01f, modes[0].mu[1], modes[0].mu[2]};
            CHECK(isfinite(oracle_mode_term(&modes[0], y)));
        }
    }
    int32_t labels[8];
    CHECK(oracle_modes_bruteforce(&p, ent, 8, modes, &nm, labels) == 0);
    CHECK(oracle_modes_from_points(&p, ent, 8, modes, &nm, labels) == 0);
    double out[16], R[9], t[3];
    float score = 0.0f;
    oracle_trace tr;
    memset(&tr, 0, sizeof(tr));
    int32_t tries[24], n_rounds = 0, n_alive[16], alive[16 * 24], n_inl[16 * 24], final_hyp = -1, pool = 0;
    float energy[16 * 24];
    double hyp_pose[24 * 12], after[16 * 24 * 12];
    tr.cap_hyp = 24; tr.cap_rounds = 16; tr.pool_size = &pool; tr.hyp_try = tries; tr.hyp_pose = hyp_pose;
    tr.n_rounds = &n_rounds; tr.n_alive = n_alive; tr.alive = alive; tr.energy = energy; tr.n_inliers = n_inl;
    tr.pose_after = after; tr.final_hyp = &final_hyp;
    synth_frame(W, H, 2, depth, rgb);
    int st = oracle_relocalise(f, depth, rgb, W, H, K, 77, 0, NULL, out, &score, &tr);
    CHECK(st >= 0);
    uint32_t *wts = malloc(sizeof(uint32_t) * W * H);
    for (int q = 0; q < W * H; ++q) wts[q] = (uint32_t)(q % 7);
    CHECK(oracle_relocalise(f, depth, rgb, W, H, K, 78, 9, wts, out, &score, NULL) >= 0);
    double hp[2 * 12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0.1, -0.2, 0.3, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0.1, -0.2, 0.3};
    int32_t valid[2] = {1, 1};
    CHECK(oracle_preemptive(f, depth, rgb, W, H, K, 5, 2, hp, valid, out, &score, NULL) == 0);
    int32_t pi[3] = {1, 2, 3};
    float c[9] = {0, 0, 2, 0.6f, 0.1f, 2.1f, 0.1f, 0.7f, 2.4f};
    CHECK(oracle_check_triple(&p, pi, c, c, R, t) == ORACLE_TRI_OK);
    double sums[22] = {0};
    CHECK(oracle_pose_from_sums(sums, R, t) == 1);
    uint8_t a3[3] = {1, 2, 3};
    CHECK(oracle_colour_ok(&p, a3, a3) == 1);
    double src[12] = {0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1}, dst[12];
    memcpy(dst, src, sizeof(dst));
    CHECK(oracle_kabsch(src, dst, 4, R, t) == 0);
    double A[9] = {1, 2, 3, 4, 5, 6, 7, 8, 10}, U[9], S[3], V[9];
    CHECK(oracle_svd3(A, U, S, V) == 0);
    double vf, mu;
    int acc;
    CHECK(oracle_verify(depth, depth, W, H, &vf, &mu, &acc) == 0 && mu == 0.0);
    int32_t pix[5] = {0, 100, 200, 300, W * H - 1};
    float x24[5 * 24];
    uint8_t lab[5];
    CHECK(oracle_features24(f, depth, rgb, W, H, K, pix, 5, x24) == 0);
    CHECK(oracle_label(f, depth, rgb, W, H, K, pose, pix, 5, lab) == 0);
    float w[ORACLE_MLP_NPARAM];
    double z[5], grad[ORACLE_MLP_NPARAM], loss;
    oracle_mlp_init(3, w);
    CHECK(oracle_mlp_forward(w, x24, 5, z) == 0);
    CHECK(oracle_mlp_grad(w, x24, lab, 5, grad, &loss) == 0);
    double est[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1}, dt, da;
    CHECK(oracle_pose_success(est, est, &dt, &da) == 1);
    /* checkpoint round trip, then after dropping the reservoirs */
    CHECK(oracle_forest_save(f, tmp) == 0);
    oracle_forest *g = NULL;
    CHECK(oracle_forest_load(tmp, &g) == 0);
    CHECK(oracle_total_samples(g) == oracle_total_samples(f));
    CHECK(oracle_drop_reservoirs(g) == 0);
    CHECK(oracle_forest_save(g, tmp) == 0);
    oracle_forest *h = NULL;
    CHECK(oracle_forest_load(tmp, &h) == 0);
    CHECK(oracle_relocalise(h, depth, rgb, W, H, K, 77, 0, NULL, out, &score, NULL) == st);
    oracle_forest *none = NULL;
    CHECK(oracle_forest_load("/nonexistent/forest.bin", &none) == ORACLE_E_IO && none == NULL);
    oracle_forest_destroy(g);
    oracle_forest_destroy(h);
    oracle_forest_destroy(f);
    free(depth); free(rgb); free(leaves); free(feat); free(wts);
    printf("oracle sanitizer run ok\n");
    return 0;
}
