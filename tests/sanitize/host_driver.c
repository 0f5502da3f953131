/* Drives the library's host-only entry points (argument checks, the offset
 * division, the pose solver's eigenvector step, work-unit ownership, the
 * inter-agent scheduling and pose-graph code, checkpoint file errors) for a
 * build whose host code has AddressSanitizer and UndefinedBehaviorSanitizer
 * (run by the CPU tests; nothing here touches a GPU). Exits 0 when every
 * call returns the status it should. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "reloc.h"

#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            return 1;                                                   \
        }                                                               \
    } while (0)

static void rot(double a, double b, double c, double T[16])
{
    double ca = cos(a), sa = sin(a), cb = cos(b), sb = sin(b), cc = cos(c), sc = sin(c);
    double R[9] = {cb * cc, -cb * sc, sb, sa * sb * cc + ca * sc, -sa * sb * sc + ca * cc, -sa * cb,
                   -ca * sb * cc + sa * sc, ca * sb * sc + sa * cc, ca * cb};
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) T[r * 4 + k] = R[r * 3 + k];
        T[r * 4 + 3] = 0.3 * (r + 1) * a;
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
}

int main(int argc, char **argv)
{
    const char *dir = argc > 1 ? argv[1] : "/tmp";
    char path[512];
    /* parameters and argument errors (no device work is reached) */
    reloc_params p;
    CHECK(reloc_params_default(&p) == RELOC_OK);
    CHECK(reloc_params_default(NULL) == RELOC_E_ARG);
    reloc_forest *f = NULL;
    reloc_params q = p;
    q.depth = 0;
    CHECK(reloc_forest_create(&q, NULL, &f) == RELOC_E_ARG && f == NULL);
    q = p;
    q.max_modes = 65;
    CHECK(reloc_forest_create(&q, NULL, &f) == RELOC_E_ARG);
    CHECK(reloc_forest_destroy(NULL) == RELOC_E_ARG);
    CHECK(reloc_verify(NULL, NULL, 4, 4, NULL, NULL, NULL, NULL) == RELOC_E_ARG);
    CHECK(reloc_verify_noalloc(NULL, NULL, 4, 4, NULL, NULL, NULL, NULL) == RELOC_E_ARG);
    for (int code = -7; code <= 4; ++code) CHECK(strlen(reloc_status_string(code)) > 0);
    /* checkpoint files that are not checkpoints */
    snprintf(path, sizeof(path), "%s/missing_forest.bin", dir);
    CHECK(reloc_forest_load(path, NULL, &f) == RELOC_E_IO && f == NULL);
    snprintf(path, sizeof(path), "%s/junk_forest.bin", dir);
    FILE *fp = fopen(path, "wb");
    CHECK(fp != NULL);
    for (int k = 0; k < 1000; ++k) fputc(k * 37 & 255, fp);
    fclose(fp);
    CHECK(reloc_forest_load(path, NULL, &f) == RELOC_E_IO && f == NULL);
    /* the offset division: exact truncation */
    int32_t n[6] = {-2147483647, -1300, -1, 0, 1300, 2147483647}, den[6] = {1, 1000, 7, 3, 2147483647, 65536};
    int32_t qv[6];
    CHECK(reloc_debug_div(n, den, 6, qv) == RELOC_OK);
    for (int k = 0; k < 6; ++k) CHECK(qv[k] == n[k] / den[k]);
    den[0] = 0;
    CHECK(reloc_debug_div(n, den, 6, qv) == RELOC_E_ARG);
    /* the eigenvector step of the pose solver */
    double H[4 * 9] = {0}, Q[4 * 4];
    for (int k = 0; k < 9; ++k) H[9 + k] = (k % 4 == 0) ? 1.0 : 0.0;
    for (int k = 0; k < 9; ++k) H[18 + k] = sin(1.0 + k);
    for (int k = 0; k < 9; ++k) H[27 + k] = 1e-3 * cos(2.0 * k);
    CHECK(reloc_debug_horn(H, 4, Q) == RELOC_OK);
    CHECK(isnan(Q[0]));                       /* H = 0: the closed form declines */
    CHECK(fabs(fabs(Q[4]) - 1.0) < 1e-12);     /* H = I: the identity rotation */
    /* work-unit ownership of the persistent kernels */
    int32_t *owners = malloc(sizeof(int32_t) * 5000);
    for (int xcd = 0; xcd < 2; ++xcd)
        for (int total = 0; total < 5000; total += 997)
            for (int grid = 1; grid < 300; grid += 37) {
                CHECK(reloc_debug_unit_owners(xcd, total, grid, owners) == RELOC_OK);
                for (int u = 0; u < total; ++u) CHECK(owners[u] == 1);
            }
    free(owners);
    /* inter-agent scheduling, clustering and pose graph */
    double A[16], B[16], T[16], frames[6 * 16];
    rot(0.3, -0.2, 0.5, A);
    rot(-0.7, 0.1, 0.2, B);
    CHECK(reloc_relative_transform(A, B, T) == RELOC_OK);
    reloc_collab *c = NULL;
    CHECK(reloc_collab_create(1, 0, &c) == RELOC_E_ARG);
    CHECK(reloc_collab_create(4, 11, &c) == RELOC_OK);
    int32_t a, b, i, size;
    float cands[10 * 7];
    CHECK(reloc_collab_schedule(c, 10, &a, &b, &i, cands) == RELOC_E_STATE);
    for (int s = 0; s < 4; ++s) {
        for (int k = 0; k < 6; ++k) rot(0.1 * k + s, 0.05 * k, -0.02 * s, frames + 16 * k);
        CHECK(reloc_collab_set_frames(c, s, frames, 6) == RELOC_OK);
    }
    for (int r = 0; r < 30; ++r) {
        CHECK(reloc_collab_schedule(c, 10, &a, &b, &i, cands) == RELOC_OK);
        CHECK(a != b && a >= 0 && b >= 0 && a < 4 && b < 4 && i >= 0 && i < 6);
        CHECK(reloc_collab_tried(c, a, b, i) == RELOC_OK);
        rot(0.01 * (r % 3) + a - b, 0.2, 0.1 * (a + b), T);
        CHECK(reloc_collab_add_sample(c, a, b, T, &size) == RELOC_OK && size >= 1);
        if (r % 5 == 4) {
            int32_t in_graph[4];
            double X[4 * 16], cost = -1.0;
            CHECK(reloc_collab_optimise(c, in_graph, X, &cost) == RELOC_OK && cost >= 0.0 && in_graph[0] == 1);
        }
    }
    int32_t sizes[64], nc = 0;
    double blended[64 * 16];
    CHECK(reloc_collab_clusters(c, 2, 1, sizes, blended, 64, &nc) == RELOC_OK);
    CHECK(reloc_collab_add_sample(c, 1, 1, T, &size) == RELOC_E_ARG);
    CHECK(reloc_collab_destroy(c) == RELOC_OK);
    printf("host sanitizer run ok\n");
    return 0;
}
