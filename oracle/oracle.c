/*
 * Plain CPU oracle of the regression-forest relocalisation path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path. It shares no code
 * with the GPU library. Build: gcc -O2 -ffp-contract=off -fPIC -shared (no
 * fast-math, no FMA contraction: every floating-point operation below is the
 * IEEE operation written, in the order written; fmaf/fma appear only where
 * the method defines a fused multiply-add).
 *
 * What the paper fixes and what is defined here is stated in oracle.h.
 * Parity pins for every function live in the CPU test suite (closed forms,
 * library routines, brute force, invariants).
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

enum { TAG_FOREST = 1, TAG_RESERVOIR = 2, TAG_HYP = 3, TAG_PIX = 4, TAG_TRAIN = 8 };

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers:  */
/* as easy as 1, 2, 3", SC 2011): ten rounds of two 64x64->128 products,    */
/* with a Weyl-sequence key schedule.                                       */
/* ------------------------------------------------------------------------ */

static void mulhilo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo(0xD2E7470EE14C6C93ULL, x0, &hi0, &lo0);
        mulhilo(0xCA5A826395121157ULL, x2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0; x1 = lo1; x2 = n2; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* floor(u * n / 2^64): an integer in [0, n) with no rejection step */
uint64_t oracle_uniform_int(uint64_t u, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)u * (unsigned __int128)n) >> 64);
}

static void draw(uint64_t seed, uint64_t tag, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                 uint64_t out[4])
{
    uint64_t ctr[4] = {c0, c1, c2, c3};
    uint64_t key[2] = {seed, tag};
    oracle_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* forest state                                                             */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t kind, dx, dy, thr; } onode;

struct oracle_forest {
    oracle_params p;
    int T, D, L, R, M;
    onode *nodes;            /* [T][L-1] */
    onode extra[8];          /* the 8 per-pixel feature nodes of the learned proposal */
    uint32_t *counter;       /* [T][L] samples ever offered to the leaf */
    oracle_entry *res;       /* [T][L][R] */
    int32_t *nmodes;         /* [T][L], -1 = not computed since the reservoir changed */
    oracle_mode *modes;      /* [T][L][M] */
    uint64_t total_samples;
    int dropped;
};

int oracle_params_default(oracle_params *p)
{
    if (!p) return ORACLE_E_ARG;
    memset(p, 0, sizeof(*p));
    p->n_trees = 5; p->depth = 10; p->reservoir_size = 256; p->max_modes = 10;
    p->seed = 180108361ULL;
    p->depth_min_mm = 500; p->depth_max_mm = 5000;
    p->offset_pxmm = 130000; p->f_ref_px16 = 277 * 16;
    p->thr_depth_mm = 100; p->thr_rgb = 10;
    p->dens_radius_mm = 50; p->link_radius_mm = 100; p->min_cluster = 0; p->cov_reg_mm2 = 100;
    p->n_hypotheses = 256; p->batch_pixels = 64; p->max_tries = 64; p->refine = 1; p->rgb_tol = 15;
    p->rigid_ratio2 = 1.21f; p->min_pair2_m2 = 0.01f; p->min_area2_m4 = 1e-4f;
    p->resid_m = 0.05f; p->inlier_m = 0.1f;
    return ORACLE_OK;
}

/* a split drawn from the generator keyed by (seed, tag) at counter (c0, c1,
 * c2, 0): kind, offsets and threshold uniform over their ranges */
static void draw_node(uint64_t seed, uint64_t tag, const oracle_params *p, uint64_t c0, uint64_t c1, uint64_t c2,
                      onode *nd)
{
    uint64_t u[4];
    draw(seed, tag, c0, c1, c2, 0, u);
    int k = (int)oracle_uniform_int(u[0], 6);
    nd->kind = k < 3 ? 0 : k - 2;                  /* 0: depth, 1..3: colour channel */
    int64_t O = p->offset_pxmm;
    nd->dx = (int32_t)((int64_t)oracle_uniform_int(u[1], (uint64_t)(2 * O + 1)) - O);
    nd->dy = (int32_t)((int64_t)oracle_uniform_int(u[2], (uint64_t)(2 * O + 1)) - O);
    int64_t Tk = nd->kind == 0 ? p->thr_depth_mm : p->thr_rgb;
    nd->thr = (int32_t)((int64_t)oracle_uniform_int(u[3], (uint64_t)(2 * Tk + 1)) - Tk);
}

/* the random split of node i of tree t (t = T: the extra feature nodes) */
static void gen_node(uint64_t seed, const oracle_params *p, uint64_t t, uint64_t i, onode *nd)
{
    draw_node(seed, TAG_FOREST, p, t, i, 0, nd);
}

int oracle_forest_create(const oracle_params *p, oracle_forest **out)
{
    if (!p || !out) return ORACLE_E_ARG;
    if (p->n_trees < 1 || p->n_trees > 16 || p->depth < 1 || p->depth > 20 || p->reservoir_size < 1 ||
        p->max_modes < 1 || p->max_modes > 64 || p->offset_pxmm < 0 || p->batch_pixels < 1 ||
        p->n_hypotheses < 1 || p->max_tries < 1 || p->cov_reg_mm2 < 1)
        return ORACLE_E_ARG;
    oracle_forest *f = (oracle_forest *)calloc(1, sizeof(*f));
    if (!f) return ORACLE_E_NOMEM;
    f->p = *p;
    f->T = p->n_trees; f->D = p->depth; f->L = 1 << p->depth; f->R = p->reservoir_size; f->M = p->max_modes;
    size_t TL = (size_t)f->T * f->L;
    f->nodes = (onode *)calloc((size_t)f->T * (f->L - 1 > 0 ? f->L - 1 : 1), sizeof(onode));
    f->counter = (uint32_t *)calloc(TL, sizeof(uint32_t));
    f->res = (oracle_entry *)calloc(TL * f->R, sizeof(oracle_entry));
    f->nmodes = (int32_t *)malloc(TL * sizeof(int32_t));
    f->modes = (oracle_mode *)calloc(TL * f->M, sizeof(oracle_mode));
    if (!f->nodes || !f->counter || !f->res || !f->nmodes || !f->modes) {
        oracle_forest_destroy(f);
        return ORACLE_E_NOMEM;
    }
    for (size_t i = 0; i < TL; ++i) f->nmodes[i] = 0;   /* empty leaves hold no modes */
    for (int t = 0; t < f->T; ++t)
        for (int i = 0; i < f->L - 1; ++i)
            gen_node(p->seed, p, (uint64_t)t, (uint64_t)i, &f->nodes[(size_t)t * (f->L - 1) + i]);
    for (int j = 0; j < 8; ++j) gen_node(p->seed, p, (uint64_t)f->T, (uint64_t)j, &f->extra[j]);
    *out = f;
    return ORACLE_OK;
}

void oracle_forest_destroy(oracle_forest *f)
{
    if (!f) return;
    free(f->nodes); free(f->counter); free(f->res); free(f->nmodes); free(f->modes);
    free(f);
}

int oracle_forest_nodes(const oracle_forest *f, int32_t *kind, int32_t *dx, int32_t *dy, int32_t *thr)
{
    if (!f) return ORACLE_E_ARG;
    size_t n = (size_t)f->T * (f->L - 1);
    for (size_t i = 0; i < n + 8; ++i) {
        const onode *nd = i < n ? &f->nodes[i] : &f->extra[i - n];
        if (kind) kind[i] = nd->kind;
        if (dx) dx[i] = nd->dx;
        if (dy) dy[i] = nd->dy;
        if (thr) thr[i] = nd->thr;
    }
    return ORACLE_OK;
}

int oracle_set_nodes(oracle_forest *f, const int32_t *kind, const int32_t *dx, const int32_t *dy,
                     const int32_t *thr)
{
    if (!f || !kind || !dx || !dy || !thr) return ORACLE_E_ARG;
    size_t n = (size_t)f->T * (f->L - 1);
    for (size_t i = 0; i < n + 8; ++i) {
        onode *nd = i < n ? &f->nodes[i] : &f->extra[i - n];
        nd->kind = kind[i]; nd->dx = dx[i]; nd->dy = dy[i]; nd->thr = thr[i];
    }
    return ORACLE_OK;
}

uint64_t oracle_total_samples(const oracle_forest *f) { return f ? f->total_samples : 0; }

/* ------------------------------------------------------------------------ */
/* pixels: validity and back-projection                                     */
/* ------------------------------------------------------------------------ */

static int valid_depth(const oracle_params *p, uint32_t d)
{
    return (int32_t)d >= p->depth_min_mm && (int32_t)d <= p->depth_max_mm;
}

/* camera-frame point in metres, each float operation in the order written */
static void cam_point(int u, int v, uint32_t d, const float K[4], float c[3])
{
    float z = (float)d * 0.001f;
    c[0] = ((float)u - K[2]) * z / K[0];
    c[1] = ((float)v - K[3]) * z / K[1];
    c[2] = z;
}

int oracle_camera_point(const uint16_t *depth, int W, int H, const float K[4], int u, int v,
                        const oracle_params *p, float out[3])
{
    if (!depth || !K || !p || !out || u < 0 || v < 0 || u >= W || v >= H) return ORACLE_E_ARG;
    uint32_t d = depth[(size_t)v * W + u];
    if (!valid_depth(p, d)) return 1;
    cam_point(u, v, d, K, out);
    return ORACLE_OK;
}

/* focal length in 1/16 px, rounded half up */
static int64_t f16(float f) { return (int64_t)floor((double)f * 16.0 + 0.5); }

/* ------------------------------------------------------------------------ */
/* depth-adaptive features and traversal                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint16_t *depth;
    const uint8_t *rgb;
    int W, H;
    int64_t Fx, Fy, Fref;
    const oracle_params *p;
} frame_ctx;

/* Feature response at pixel (u, v) with depth d (mm). The probe offset is the
 * node's metric offset (px mm) scaled by the frame's focal length relative to
 * the reference focal length and divided by the pixel depth, truncated toward
 * zero. Depth probes outside the image or on invalid depth read 65535;
 * colour probes are clamped to the image. */
static int32_t feature(const frame_ctx *fc, const onode *nd, int u, int v, int32_t d)
{
    int64_t den = (int64_t)d * fc->Fref;
    int32_t ox = (int32_t)(((int64_t)nd->dx * fc->Fx) / den);
    int32_t oy = (int32_t)(((int64_t)nd->dy * fc->Fy) / den);
    int qx = u + ox, qy = v + oy;
    if (nd->kind == 0) {
        int32_t dq = 65535;
        if (qx >= 0 && qx < fc->W && qy >= 0 && qy < fc->H) {
            uint32_t z = fc->depth[(size_t)qy * fc->W + qx];
            if (valid_depth(fc->p, z)) dq = (int32_t)z;
        }
        return dq - d;
    }
    int c = nd->kind - 1;
    if (qx < 0) qx = 0;
    if (qx > fc->W - 1) qx = fc->W - 1;
    if (qy < 0) qy = 0;
    if (qy > fc->H - 1) qy = fc->H - 1;
    return (int32_t)fc->rgb[((size_t)qy * fc->W + qx) * 3 + c] - (int32_t)fc->rgb[((size_t)v * fc->W + u) * 3 + c];
}

/* implicit heap: node i has children 2i+1 (left) and 2i+2 (right); a pixel
 * goes right iff its response is >= the node threshold */
static int32_t traverse(const oracle_forest *f, const frame_ctx *fc, int t, int u, int v, int32_t d)
{
    const onode *tree = &f->nodes[(size_t)t * (f->L - 1)];
    int64_t i = 0;
    while (i < f->L - 1) {
        int32_t r = feature(fc, &tree[i], u, v, d);
        i = 2 * i + 1 + (r >= tree[i].thr ? 1 : 0);
    }
    return (int32_t)(i - (f->L - 1));
}

static void make_ctx(const oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                     const float K[4], frame_ctx *fc)
{
    fc->depth = depth; fc->rgb = rgb; fc->W = W; fc->H = H;
    fc->Fx = f16(K[0]); fc->Fy = f16(K[1]); fc->Fref = f->p.f_ref_px16;
    fc->p = &f->p;
}

static int frame_args_ok(const oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                         const float K[4])
{
    if (!f || !depth || !rgb || !K || W < 1 || H < 1) return 0;
    if (!(K[0] > 0.0f) || !(K[1] > 0.0f)) return 0;
    /* the product |offset| * F must fit in 32 bits (the GPU path's contract) */
    if ((int64_t)f->p.offset_pxmm * f16(K[0]) > 2147483647LL) return 0;
    if ((int64_t)f->p.offset_pxmm * f16(K[1]) > 2147483647LL) return 0;
    return 1;
}

int oracle_leaves(const oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                  const float K[4], int32_t *leaves)
{
    if (!frame_args_ok(f, depth, rgb, W, H, K) || !leaves) return ORACLE_E_ARG;
    frame_ctx fc;
    make_ctx(f, depth, rgb, W, H, K, &fc);
    size_t P = (size_t)W * H;
    for (int t = 0; t < f->T; ++t)
        for (int v = 0; v < H; ++v)
            for (int u = 0; u < W; ++u) {
                size_t p = (size_t)v * W + u;
                uint32_t d = depth[p];
                leaves[(size_t)t * P + p] = valid_depth(&f->p, d) ? traverse(f, &fc, t, u, v, (int32_t)d) : -1;
            }
    return ORACLE_OK;
}

int oracle_features8(const oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                     const float K[4], int32_t *feat)
{
    if (!frame_args_ok(f, depth, rgb, W, H, K) || !feat) return ORACLE_E_ARG;
    frame_ctx fc;
    make_ctx(f, depth, rgb, W, H, K, &fc);
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            size_t p = (size_t)v * W + u;
            uint32_t d = depth[p];
            for (int j = 0; j < 8; ++j)
                feat[p * 8 + j] = valid_depth(&f->p, d) ? feature(&fc, &f->extra[j], u, v, (int32_t)d) : 0;
        }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* online leaf reservoirs                                                   */
/* ------------------------------------------------------------------------ */

/* One posed frame. For every tree, the valid pixels are offered to their
 * leaves in raster order. A leaf that has been offered k samples before keeps
 * the new one in slot k while k < R; afterwards it draws j uniform in
 * [0, k] from the counter-based generator keyed by (tree, leaf, k) and
 * replaces slot j if j < R (Vitter's Algorithm R). The stored sample is the
 * world point in integer mm plus the pixel colour. */
/* a camera-to-world pose must be a rigid motion: last row (0, 0, 0, 1) and
 * R^T R = I, det R = +1 to 1e-6 */
static int is_se3(const double T[16])
{
    if (T[12] != 0.0 || T[13] != 0.0 || T[14] != 0.0 || T[15] != 1.0) return 0;
    for (int k = 0; k < 16; ++k)
        if (!isfinite(T[k])) return 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = T[0 * 4 + a] * T[0 * 4 + b] + T[1 * 4 + a] * T[1 * 4 + b] + T[2 * 4 + a] * T[2 * 4 + b];
            if (fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6) return 0;
        }
    double d = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
               T[2] * (T[4] * T[9] - T[5] * T[8]);
    return d > 0.0;
}

int oracle_adapt_frame(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                       const float K[4], const double pose[16])
{
    if (!frame_args_ok(f, depth, rgb, W, H, K) || !pose || !is_se3(pose)) return ORACLE_E_ARG;
    if (f->dropped) return ORACLE_E_ARG;
    frame_ctx fc;
    make_ctx(f, depth, rgb, W, H, K, &fc);
    float R32[9], t32[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R32[r * 3 + c] = (float)pose[r * 4 + c];
        t32[r] = (float)pose[r * 4 + 3];
    }
    for (int t = 0; t < f->T; ++t) {
        for (int v = 0; v < H; ++v)
            for (int u = 0; u < W; ++u) {
                size_t p = (size_t)v * W + u;
                uint32_t d = depth[p];
                if (!valid_depth(&f->p, d)) continue;
                int32_t leaf = traverse(f, &fc, t, u, v, (int32_t)d);
                float c[3], w[3];
                cam_point(u, v, d, K, c);
                for (int k = 0; k < 3; ++k)
                    w[k] = ((R32[k * 3 + 0] * c[0] + R32[k * 3 + 1] * c[1]) + R32[k * 3 + 2] * c[2]) + t32[k];
                size_t li = (size_t)t * f->L + leaf;
                uint32_t k = f->counter[li];
                int64_t slot = -1;
                if (k < (uint32_t)f->R) {
                    slot = k;
                } else {
                    uint64_t rr[4];
                    draw(f->p.seed, TAG_RESERVOIR, (uint64_t)t, (uint64_t)leaf, (uint64_t)k, 0, rr);
                    uint64_t j = oracle_uniform_int(rr[0], (uint64_t)k + 1);
                    if (j < (uint64_t)f->R) slot = (int64_t)j;
                }
                if (slot >= 0) {
                    oracle_entry *e = &f->res[li * f->R + slot];
                    e->x = (int32_t)rintf(w[0] * 1000.0f);
                    e->y = (int32_t)rintf(w[1] * 1000.0f);
                    e->z = (int32_t)rintf(w[2] * 1000.0f);
                    e->r = rgb[p * 3 + 0]; e->g = rgb[p * 3 + 1]; e->b = rgb[p * 3 + 2]; e->pad = 0;
                }
                f->counter[li] = k + 1;
                f->nmodes[li] = -1;
                f->total_samples++;
            }
    }
    return ORACLE_OK;
}

int oracle_reservoir(const oracle_forest *f, int t, int leaf, oracle_entry *entries, uint32_t *count)
{
    if (!f || t < 0 || t >= f->T || leaf < 0 || leaf >= f->L) return ORACLE_E_ARG;
    size_t li = (size_t)t * f->L + leaf;
    if (count) *count = f->counter[li];
    if (entries) memcpy(entries, &f->res[li * f->R], (size_t)f->R * sizeof(oracle_entry));
    return ORACLE_OK;
}

int oracle_drop_reservoirs(oracle_forest *f)
{
    /* the paper deletes each relocaliser's training data once it is fully
     * trained (Sec. 4.3.2): modes are kept, the samples are released */
    if (!f) return ORACLE_E_ARG;
    if (f->dropped) return ORACLE_OK;
    oracle_build_all_modes(f);
    free(f->res);
    f->res = NULL;
    f->dropped = 1;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* checkpoint: the whole forest state in a file of the oracle's own layout  */
/* (parameters, flags, split nodes, counters, lazily built modes and, unless */
/* dropped, the reservoirs), so that a saved forest resumes exactly.        */
/* ------------------------------------------------------------------------ */

static const char ORACLE_MAGIC[8] = {'O', 'R', 'A', 'C', 'L', 'E', 'F', '1'};

int oracle_forest_save(const oracle_forest *f, const char *path)
{
    if (!f || !path) return ORACLE_E_ARG;
    FILE *fp = fopen(path, "wb");
    if (!fp) return ORACLE_E_IO;
    size_t TL = (size_t)f->T * f->L, ns = (size_t)f->T * (f->L - 1);
    int32_t dropped = f->dropped;
    int ok = fwrite(ORACLE_MAGIC, 1, 8, fp) == 8 && fwrite(&f->p, sizeof(f->p), 1, fp) == 1 &&
             fwrite(&dropped, sizeof(dropped), 1, fp) == 1 &&
             fwrite(&f->total_samples, sizeof(f->total_samples), 1, fp) == 1 &&
             fwrite(f->nodes, sizeof(onode), ns, fp) == ns && fwrite(f->extra, sizeof(onode), 8, fp) == 8 &&
             fwrite(f->counter, sizeof(uint32_t), TL, fp) == TL && fwrite(f->nmodes, sizeof(int32_t), TL, fp) == TL &&
             fwrite(f->modes, sizeof(oracle_mode), TL * f->M, fp) == TL * f->M &&
             (f->dropped || fwrite(f->res, sizeof(oracle_entry), TL * f->R, fp) == TL * f->R);
    if (fclose(fp) != 0) ok = 0;
    return ok ? ORACLE_OK : ORACLE_E_IO;
}

int oracle_forest_load(const char *path, oracle_forest **out)
{
    if (!path || !out) return ORACLE_E_ARG;
    *out = NULL;
    FILE *fp = fopen(path, "rb");
    if (!fp) return ORACLE_E_IO;
    char magic[8];
    oracle_params p;
    int32_t dropped = 0;
    uint64_t total = 0;
    if (fread(magic, 1, 8, fp) != 8 || memcmp(magic, ORACLE_MAGIC, 8) != 0 || fread(&p, sizeof(p), 1, fp) != 1 ||
        fread(&dropped, sizeof(dropped), 1, fp) != 1 || fread(&total, sizeof(total), 1, fp) != 1) {
        fclose(fp);
        return ORACLE_E_IO;
    }
    oracle_forest *f = NULL;
    int rc = oracle_forest_create(&p, &f);
    if (rc) { fclose(fp); return rc; }
    size_t TL = (size_t)f->T * f->L, ns = (size_t)f->T * (f->L - 1);
    int ok = fread(f->nodes, sizeof(onode), ns, fp) == ns && fread(f->extra, sizeof(onode), 8, fp) == 8 &&
             fread(f->counter, sizeof(uint32_t), TL, fp) == TL && fread(f->nmodes, sizeof(int32_t), TL, fp) == TL &&
             fread(f->modes, sizeof(oracle_mode), TL * f->M, fp) == TL * f->M &&
             (dropped || fread(f->res, sizeof(oracle_entry), TL * f->R, fp) == TL * f->R) && fgetc(fp) == EOF;
    fclose(fp);
    if (!ok) { oracle_forest_destroy(f); return ORACLE_E_IO; }
    f->total_samples = total;
    if (dropped) {
        free(f->res);
        f->res = NULL;
        f->dropped = 1;
    }
    *out = f;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* leaf modes: integer quick-shift, then Gaussian statistics                */
/* ------------------------------------------------------------------------ */

static int64_t dist2(const oracle_entry *a, const oracle_entry *b)
{
    int64_t dx = (int64_t)a->x - b->x, dy = (int64_t)a->y - b->y, dz = (int64_t)a->z - b->z;
    return dx * dx + dy * dy + dz * dz;
}

typedef struct { int32_t size, root; } cluster_t;

static int cmp_cluster(const void *a, const void *b)
{
    const cluster_t *x = (const cluster_t *)a, *y = (const cluster_t *)b;
    if (x->size != y->size) return x->size > y->size ? -1 : 1;
    return x->root < y->root ? -1 : (x->root > y->root ? 1 : 0);
}

static int min_cluster_size(const oracle_params *p)
{
    if (p->min_cluster > 0) return p->min_cluster;
    int m = p->reservoir_size / 64;
    return m > 3 ? m : 3;
}

/* Given density and parent arrays, form clusters and their statistics.
 * Clusters are the trees of the parent forest; those with at least the
 * minimum size are ordered by (size descending, root index ascending) and the
 * first M become modes. Per mode, from exact integer sums:
 *   mu = sum / (n_m * 1000)                             (metres, FP64 -> FP32)
 *   C  = (n_m * sum xx^T - sum x sum x^T) / n_m^2 + reg I  (mm^2, FP64)
 *   Sigma = C * 1e-6, Sigma^-1 by adjugate / determinant (FP64 -> FP32)
 *   kappa = -log(n_m / n) + 0.5 (3 log 2 pi + log det Sigma)
 * so that kappa + 0.5 q = -log(pi_m N(y; mu, Sigma)) for q the Mahalanobis
 * form. */
static int finish_modes(const oracle_params *p, const oracle_entry *pts, int n, const int32_t *parent,
                        oracle_mode *modes, int32_t *n_modes, int32_t *labels)
{
    int32_t *root = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *size = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *slot = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    cluster_t *cl = (cluster_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(cluster_t));
    if (!root || !size || !slot || !cl) {
        free(root); free(size); free(slot); free(cl);
        return ORACLE_E_NOMEM;
    }
    for (int i = 0; i < n; ++i) {
        int r = i;
        while (parent[r] >= 0) r = parent[r];
        root[i] = r;
        size[r]++;
    }
    int nc = 0, minc = min_cluster_size(p);
    for (int i = 0; i < n; ++i)
        if (parent[i] < 0 && size[i] >= minc) { cl[nc].size = size[i]; cl[nc].root = i; nc++; }
    qsort(cl, (size_t)nc, sizeof(cluster_t), cmp_cluster);
    int M = nc < p->max_modes ? nc : p->max_modes;
    for (int i = 0; i < n; ++i) slot[i] = -1;
    for (int m = 0; m < M; ++m) slot[cl[m].root] = m;
    for (int m = 0; m < M; ++m) {
        int64_t Sx[3] = {0, 0, 0}, Sxx[6] = {0, 0, 0, 0, 0, 0}, Sc[3] = {0, 0, 0};
        int64_t nm = 0;
        for (int i = 0; i < n; ++i) {
            if (slot[root[i]] != m) continue;
            int64_t x = pts[i].x, y = pts[i].y, z = pts[i].z;
            Sx[0] += x; Sx[1] += y; Sx[2] += z;
            Sxx[0] += x * x; Sxx[1] += x * y; Sxx[2] += x * z;
            Sxx[3] += y * y; Sxx[4] += y * z; Sxx[5] += z * z;
            Sc[0] += pts[i].r; Sc[1] += pts[i].g; Sc[2] += pts[i].b;
            nm++;
        }
        oracle_mode *md = &modes[m];
        memset(md, 0, sizeof(*md));
        double dn = (double)nm;
        for (int k = 0; k < 3; ++k) md->mu[k] = (float)((double)Sx[k] / (dn * 1000.0));
        static const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
        double S[6];
        for (int e = 0; e < 6; ++e) {
            int64_t num = nm * Sxx[e] - Sx[ia[e]] * Sx[ib[e]];
            double c = (double)num / (dn * dn);
            if (ia[e] == ib[e]) c = c + (double)p->cov_reg_mm2;
            S[e] = c * 1e-6;
        }
        double a = S[0], b = S[1], c = S[2], d = S[3], e = S[4], g = S[5];
        /* Sigma = [[a b c] [b d e] [c e g]] */
        double A00 = d * g - e * e;
        double A01 = c * e - b * g;
        double A02 = b * e - c * d;
        double A11 = a * g - c * c;
        double A12 = b * c - a * e;
        double A22 = a * d - b * b;
        double det = (a * A00 + b * A01) + c * A02;
        md->sinv[0] = (float)(A00 / det);
        md->sinv[1] = (float)(A01 / det);
        md->sinv[2] = (float)(A02 / det);
        md->sinv[3] = (float)(A11 / det);
        md->sinv[4] = (float)(A12 / det);
        md->sinv[5] = (float)(A22 / det);
        md->kappa = (float)(-log(dn / (double)n) + 0.5 * (3.0 * log(2.0 * M_PI) + log(det)));
        md->n = (int32_t)nm;
        md->rgb[0] = (uint8_t)(Sc[0] / nm);
        md->rgb[1] = (uint8_t)(Sc[1] / nm);
        md->rgb[2] = (uint8_t)(Sc[2] / nm);
    }
    if (labels)
        for (int i = 0; i < n; ++i) labels[i] = slot[root[i]];
    *n_modes = M;
    free(root); free(size); free(slot); free(cl);
    return ORACLE_OK;
}

/* higher density wins; on equal density the lower index wins */
static int denser(const int32_t *rho, int j, int i)
{
    return rho[j] > rho[i] || (rho[j] == rho[i] && j < i);
}

/* The definition: density rho_i = #{j : |p_i - p_j|^2 <= r_d^2} (self
 * included); parent_i = the j minimising (|p_i - p_j|^2, j) among points
 * within the link radius that are denser than i; points with no parent are
 * roots. All in exact integer arithmetic. */
int oracle_modes_bruteforce(const oracle_params *p, const oracle_entry *pts, int n, oracle_mode *modes,
                            int32_t *n_modes, int32_t *labels)
{
    if (!p || (!pts && n > 0) || !modes || !n_modes || n < 0) return ORACLE_E_ARG;
    int64_t rd2 = (int64_t)p->dens_radius_mm * p->dens_radius_mm;
    int64_t rl2 = (int64_t)p->link_radius_mm * p->link_radius_mm;
    int32_t *rho = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *parent = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!rho || !parent) { free(rho); free(parent); return ORACLE_E_NOMEM; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (dist2(&pts[i], &pts[j]) <= rd2) rho[i]++;
    for (int i = 0; i < n; ++i) {
        int best = -1;
        int64_t bd = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i || !denser(rho, j, i)) continue;
            int64_t d2 = dist2(&pts[i], &pts[j]);
            if (d2 > rl2) continue;
            if (best < 0 || d2 < bd || (d2 == bd && j < best)) { best = j; bd = d2; }
        }
        parent[i] = best;
    }
    int rc = finish_modes(p, pts, n, parent, modes, n_modes, labels);
    free(rho); free(parent);
    return rc;
}

/* The same definition with the candidate set pruned by a sweep over points
 * sorted by x: a pair within radius r differs by at most r in x. */
typedef struct { int32_t x, i; } xkey;

static int cmp_xkey(const void *a, const void *b)
{
    const xkey *u = (const xkey *)a, *v = (const xkey *)b;
    if (u->x != v->x) return u->x < v->x ? -1 : 1;
    return u->i < v->i ? -1 : (u->i > v->i ? 1 : 0);
}

int oracle_modes_from_points(const oracle_params *p, const oracle_entry *pts, int n, oracle_mode *modes,
                             int32_t *n_modes, int32_t *labels)
{
    if (!p || (!pts && n > 0) || !modes || !n_modes || n < 0) return ORACLE_E_ARG;
    int64_t rd = p->dens_radius_mm, rl = p->link_radius_mm;
    int64_t rd2 = rd * rd, rl2 = rl * rl;
    int32_t *rho = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *parent = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    xkey *ks = (xkey *)malloc((size_t)(n > 0 ? n : 1) * sizeof(xkey));
    int32_t *pos = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!rho || !parent || !ks || !pos) { free(rho); free(parent); free(ks); free(pos); return ORACLE_E_NOMEM; }
    for (int i = 0; i < n; ++i) { ks[i].x = pts[i].x; ks[i].i = i; }
    qsort(ks, (size_t)n, sizeof(xkey), cmp_xkey);
    for (int s = 0; s < n; ++s) pos[ks[s].i] = s;
    for (int i = 0; i < n; ++i) {
        int s = pos[i];
        int cnt = 1;
        for (int q = s - 1; q >= 0 && (int64_t)pts[i].x - ks[q].x <= rd; --q)
            if (dist2(&pts[i], &pts[ks[q].i]) <= rd2) cnt++;
        for (int q = s + 1; q < n && (int64_t)ks[q].x - pts[i].x <= rd; ++q)
            if (dist2(&pts[i], &pts[ks[q].i]) <= rd2) cnt++;
        rho[i] = cnt;
    }
    for (int i = 0; i < n; ++i) {
        int s = pos[i];
        int best = -1;
        int64_t bd = 0;
        for (int dir = -1; dir <= 1; dir += 2)
            for (int q = s + dir; q >= 0 && q < n; q += dir) {
                int64_t gap = (int64_t)ks[q].x - pts[i].x;
                if (gap > rl || -gap > rl) break;
                int j = ks[q].i;
                if (!denser(rho, j, i)) continue;
                int64_t d2 = dist2(&pts[i], &pts[j]);
                if (d2 > rl2) continue;
                if (best < 0 || d2 < bd || (d2 == bd && j < best)) { best = j; bd = d2; }
            }
        parent[i] = best;
    }
    int rc = finish_modes(p, pts, n, parent, modes, n_modes, labels);
    free(rho); free(parent); free(ks); free(pos);
    return rc;
}

/* modes of one leaf: a pure function of the first min(k, R) reservoir slots */
static int ensure_modes(oracle_forest *f, int t, int leaf)
{
    size_t li = (size_t)t * f->L + leaf;
    if (f->nmodes[li] >= 0) return ORACLE_OK;
    if (f->dropped) return ORACLE_E_ARG;
    uint32_t k = f->counter[li];
    int n = k < (uint32_t)f->R ? (int)k : f->R;
    int32_t nm = 0;
    int rc = oracle_modes_from_points(&f->p, &f->res[li * f->R], n, &f->modes[li * f->M], &nm, NULL);
    if (rc) return rc;
    f->nmodes[li] = nm;
    return ORACLE_OK;
}

int oracle_leaf_modes(oracle_forest *f, int t, int leaf, oracle_mode *modes, int32_t *n_modes)
{
    if (!f || t < 0 || t >= f->T || leaf < 0 || leaf >= f->L) return ORACLE_E_ARG;
    int rc = ensure_modes(f, t, leaf);
    if (rc) return rc;
    size_t li = (size_t)t * f->L + leaf;
    if (n_modes) *n_modes = f->nmodes[li];
    if (modes) memcpy(modes, &f->modes[li * f->M], (size_t)f->nmodes[li] * sizeof(oracle_mode));
    return ORACLE_OK;
}

int oracle_build_all_modes(oracle_forest *f)
{
    if (!f) return ORACLE_E_ARG;
    for (int t = 0; t < f->T; ++t)
        for (int l = 0; l < f->L; ++l) {
            int rc = ensure_modes(f, t, l);
            if (rc) return rc;
        }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* rigid alignment: 3x3 SVD by one-sided Jacobi (Hestenes), then Kabsch     */
/* ------------------------------------------------------------------------ */

int oracle_svd3(const double A[9], double U[9], double S[3], double V[9])
{
    double B[9];
    memcpy(B, A, sizeof(B));
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    static const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int k = 0; k < 3; ++k) {
            int p = P[k], q = Q[k];
            double al = 0, be = 0, ga = 0;
            for (int r = 0; r < 3; ++r) {
                al += B[r * 3 + p] * B[r * 3 + p];
                be += B[r * 3 + q] * B[r * 3 + q];
                ga += B[r * 3 + p] * B[r * 3 + q];
            }
            if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
            rotated = 1;
            double zeta = (be - al) / (2.0 * ga);
            double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            for (int r = 0; r < 3; ++r) {
                double bp = B[r * 3 + p], bq = B[r * 3 + q];
                B[r * 3 + p] = c * bp - s * bq;
                B[r * 3 + q] = s * bp + c * bq;
                double vp = V[r * 3 + p], vq = V[r * 3 + q];
                V[r * 3 + p] = c * vp - s * vq;
                V[r * 3 + q] = s * vp + c * vq;
            }
        }
        if (!rotated) break;
    }
    double sv[3];
    for (int c = 0; c < 3; ++c)
        sv[c] = sqrt(B[0 * 3 + c] * B[0 * 3 + c] + B[1 * 3 + c] * B[1 * 3 + c] + B[2 * 3 + c] * B[2 * 3 + c]);
    int ord[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (sv[ord[b]] > sv[ord[a]]) { int tmp = ord[a]; ord[a] = ord[b]; ord[b] = tmp; }
    double V2[9];
    for (int c = 0; c < 3; ++c) {
        int o = ord[c];
        S[c] = sv[o];
        for (int r = 0; r < 3; ++r) {
            U[r * 3 + c] = sv[o] > 0 ? B[r * 3 + o] / sv[o] : 0.0;
            V2[r * 3 + c] = V[r * 3 + o];
        }
    }
    memcpy(V, V2, sizeof(V2));
    if (!(S[1] > 1e-12 * S[0]) || S[0] == 0.0) return -1;    /* rank < 2: rotation undetermined */
    if (!(S[2] > 1e-12 * S[0])) {                            /* rank 2: complete U by a cross product */
        U[0 * 3 + 2] = U[1 * 3 + 0] * U[2 * 3 + 1] - U[2 * 3 + 0] * U[1 * 3 + 1];
        U[1 * 3 + 2] = U[2 * 3 + 0] * U[0 * 3 + 1] - U[0 * 3 + 0] * U[2 * 3 + 1];
        U[2 * 3 + 2] = U[0 * 3 + 0] * U[1 * 3 + 1] - U[1 * 3 + 0] * U[0 * 3 + 1];
    }
    return 0;
}

static double det3(const double M[9])
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* Kabsch: the proper rotation R maximising tr(R H^T) for the cross-covariance
 * H = sum (c - c_mean)(w - w_mean)^T is R = V diag(1, 1, sign det(V U^T)) U^T
 * with H = U S V^T. */
static int rotation_from_H(const double H[9], double R[9])
{
    double U[9], S[3], V[9];
    if (oracle_svd3(H, U, S, V)) return -1;
    double d = det3(U) * det3(V) < 0 ? -1.0 : 1.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            R[r * 3 + c] = V[r * 3 + 0] * U[c * 3 + 0] + V[r * 3 + 1] * U[c * 3 + 1] + d * V[r * 3 + 2] * U[c * 3 + 2];
    return 0;
}

int oracle_kabsch(const double *src, const double *dst, int n, double R[9], double t[3])
{
    if (!src || !dst || n < 3 || !R || !t) return ORACLE_E_ARG;
    double cs[3] = {0, 0, 0}, cd[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) { cs[k] += src[i * 3 + k]; cd[k] += dst[i * 3 + k]; }
    for (int k = 0; k < 3; ++k) { cs[k] /= n; cd[k] /= n; }
    double H[9] = {0};
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                H[a * 3 + b] += (src[i * 3 + a] - cs[a]) * (dst[i * 3 + b] - cd[b]);
    if (rotation_from_H(H, R)) return 1;
    for (int k = 0; k < 3; ++k) t[k] = cd[k] - (R[k * 3 + 0] * cs[0] + R[k * 3 + 1] * cs[1] + R[k * 3 + 2] * cs[2]);
    return 0;
}

/* Correspondence sums used by hypothesis generation and refinement:
 * n, sum c, sum w, sum c w^T (row a, column b), sum c c^T (xx xy xz yy yz zz). */
typedef struct { double n, c[3], w[3], cw[9], cc[6]; } csums;

static void csums_add_point(csums *s, const float c[3], const float w[3])
{
    double cd[3] = {c[0], c[1], c[2]}, wd[3] = {w[0], w[1], w[2]};
    s->n = s->n + 1.0;
    for (int a = 0; a < 3; ++a) { s->c[a] = s->c[a] + cd[a]; s->w[a] = s->w[a] + wd[a]; }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s->cw[a * 3 + b] = s->cw[a * 3 + b] + cd[a] * wd[b];
    s->cc[0] = s->cc[0] + cd[0] * cd[0]; s->cc[1] = s->cc[1] + cd[0] * cd[1]; s->cc[2] = s->cc[2] + cd[0] * cd[2];
    s->cc[3] = s->cc[3] + cd[1] * cd[1]; s->cc[4] = s->cc[4] + cd[1] * cd[2]; s->cc[5] = s->cc[5] + cd[2] * cd[2];
}

static void csums_add(csums *s, const csums *o)
{
    s->n = s->n + o->n;
    for (int a = 0; a < 3; ++a) { s->c[a] = s->c[a] + o->c[a]; s->w[a] = s->w[a] + o->w[a]; }
    for (int a = 0; a < 9; ++a) s->cw[a] = s->cw[a] + o->cw[a];
    for (int a = 0; a < 6; ++a) s->cc[a] = s->cc[a] + o->cc[a];
}

/* Pose from correspondence sums. Returns 0 and (R, t) when the camera points
 * are spread in at least two directions: with S the centred scatter of the
 * camera points, I2 = the sum of S's principal 2x2 minors must reach
 * 1e-4 * n * trace(S) (about 1 cm of spread across the main axis). */
static int pose_from_sums(const csums *s, double R[9], double t[3])
{
    double n = s->n;
    if (n < 3.0) return 1;
    double H[9], S[6];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H[a * 3 + b] = s->cw[a * 3 + b] - (s->c[a] * s->w[b]) / n;
    S[0] = s->cc[0] - (s->c[0] * s->c[0]) / n;
    S[1] = s->cc[1] - (s->c[0] * s->c[1]) / n;
    S[2] = s->cc[2] - (s->c[0] * s->c[2]) / n;
    S[3] = s->cc[3] - (s->c[1] * s->c[1]) / n;
    S[4] = s->cc[4] - (s->c[1] * s->c[2]) / n;
    S[5] = s->cc[5] - (s->c[2] * s->c[2]) / n;
    double I2 = ((S[0] * S[3] - S[1] * S[1]) + (S[0] * S[5] - S[2] * S[2])) + (S[3] * S[5] - S[4] * S[4]);
    double tr = (S[0] + S[3]) + S[5];
    if (!(I2 >= (1e-4 * n) * tr)) return 1;
    if (rotation_from_H(H, R)) return 1;
    double cm[3], wm[3];
    for (int k = 0; k < 3; ++k) { cm[k] = s->c[k] / n; wm[k] = s->w[k] / n; }
    for (int k = 0; k < 3; ++k) t[k] = wm[k] - ((R[k * 3 + 0] * cm[0] + R[k * 3 + 1] * cm[1]) + R[k * 3 + 2] * cm[2]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* relocalisation: hypotheses, preemptive scoring, culls, refinement        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int valid;
    double R[9], t[3];
    float R32[9], t32[3];
    float E;
    csums inl;
} hyp_t;

typedef struct {
    oracle_forest *f;
    frame_ctx fc;
    const float *K;
    int32_t *pool;           /* pool index -> pixel index */
    int np;
    int32_t *pool_leaf;      /* [np][T] */
} reloc_ctx;

/* number of modes over all trees at a pool pixel, M(p) in (tree, mode) order */
static int modes_at(reloc_ctx *rc, int pi, const oracle_mode **list, int cap)
{
    oracle_forest *f = rc->f;
    int cnt = 0;
    for (int t = 0; t < f->T; ++t) {
        int32_t leaf = rc->pool_leaf[(size_t)pi * f->T + t];
        ensure_modes(f, t, leaf);
        size_t li = (size_t)t * f->L + leaf;
        for (int m = 0; m < f->nmodes[li]; ++m) {
            if (list && cnt < cap) list[cnt] = &f->modes[li * f->M + m];
            cnt++;
        }
    }
    return cnt;
}

static void pool_cam(reloc_ctx *rc, int pi, float c[3])
{
    int p = rc->pool[pi];
    int u = p % rc->fc.W, v = p / rc->fc.W;
    cam_point(u, v, rc->fc.depth[p], rc->K, c);
}

static float sq3(const float a[3], const float b[3])
{
    float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* pick a pool index: uniform, or by the integer weight CDF (upper bound) */
static int pick_pool(reloc_ctx *rc, const uint64_t *cdf, uint64_t u)
{
    if (!cdf) return (int)oracle_uniform_int(u, (uint64_t)rc->np);
    uint64_t r = oracle_uniform_int(u, cdf[rc->np - 1]);
    int lo = 0, hi = rc->np - 1;            /* first i with cdf[i] > r */
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (cdf[mid] > r) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* The checks of one hypothesis triple, in this order: distinct pool pixels;
 * for each pair of points (0,1), (0,2), (1,2): camera squared distance
 * >= min_pair2, world squared distance <= rigid_ratio2 * camera, camera
 * <= rigid_ratio2 * world (all FP32, squared distances summed as
 * (dx dx + dy dy) + dz dz); camera triangle |e1 x e2|^2 >= min_area2; a
 * non-degenerate FP64 alignment of the three pairs; every residual
 * |R c + t - w| <= resid (FP64). Returns ORACLE_TRI_OK with the pose, or the
 * first check that fails. */
int oracle_check_triple(const oracle_params *p, const int32_t pi[3], const float c[9], const float w[9],
                        double R[9], double t[3])
{
    if (!p || !pi || !c || !w || !R || !t) return ORACLE_E_ARG;
    if (pi[0] == pi[1] || pi[0] == pi[2] || pi[1] == pi[2]) return ORACLE_TRI_SAME_PIXEL;
    static const int A[3] = {0, 0, 1}, B[3] = {1, 2, 2};
    for (int e = 0; e < 3; ++e) {
        float dc = sq3(&c[A[e] * 3], &c[B[e] * 3]);
        float dw = sq3(&w[A[e] * 3], &w[B[e] * 3]);
        if (!(dc >= p->min_pair2_m2)) return ORACLE_TRI_PAIR_DIST;
        if (!(dw <= p->rigid_ratio2 * dc)) return ORACLE_TRI_WORLD_LONGER;
        if (!(dc <= p->rigid_ratio2 * dw)) return ORACLE_TRI_CAMERA_LONGER;
    }
    float e1[3] = {c[3] - c[0], c[4] - c[1], c[5] - c[2]};
    float e2[3] = {c[6] - c[0], c[7] - c[1], c[8] - c[2]};
    float cx = e1[1] * e2[2] - e1[2] * e2[1];
    float cy = e1[2] * e2[0] - e1[0] * e2[2];
    float cz = e1[0] * e2[1] - e1[1] * e2[0];
    if (!((cx * cx + cy * cy) + cz * cz >= p->min_area2_m4)) return ORACLE_TRI_AREA;
    csums s;
    memset(&s, 0, sizeof(s));
    for (int j = 0; j < 3; ++j) csums_add_point(&s, &c[j * 3], &w[j * 3]);
    if (pose_from_sums(&s, R, t)) return ORACLE_TRI_DEGENERATE;
    double lim = (double)p->resid_m * (double)p->resid_m;
    for (int j = 0; j < 3; ++j) {
        double r[3];
        for (int k = 0; k < 3; ++k)
            r[k] = (((R[k * 3 + 0] * c[j * 3 + 0] + R[k * 3 + 1] * c[j * 3 + 1]) + R[k * 3 + 2] * c[j * 3 + 2]) + t[k]) -
                   w[j * 3 + k];
        if (!((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2] <= lim)) return ORACLE_TRI_RESIDUAL;
    }
    return ORACLE_TRI_OK;
}

/* a mode may be picked for a pixel when its mean colour is within rgb_tol of
 * the pixel's colour in every channel */
int oracle_colour_ok(const oracle_params *p, const uint8_t mode_rgb[3], const uint8_t px[3])
{
    if (!p || !mode_rgb || !px) return ORACLE_E_ARG;
    for (int ch = 0; ch < 3; ++ch) {
        int dcol = (int)mode_rgb[ch] - (int)px[ch];
        if (dcol < 0) dcol = -dcol;
        if (dcol > p->rgb_tol) return 0;
    }
    return 1;
}

/* One hypothesis: the first of max_tries tries that passes every check.
 * Try tau draws 3 pool pixels and, for each, one mode uniformly among the
 * modes of M(p) that pass the colour test (no such mode fails the try); the
 * triple must then pass oracle_check_triple. */
static int make_hypothesis(reloc_ctx *rc, uint64_t seed, int h, const uint64_t *cdf, hyp_t *hy)
{
    const oracle_params *p = &rc->f->p;
    int cap = rc->f->T * rc->f->M;
    const oracle_mode **lst = (const oracle_mode **)malloc((size_t)cap * sizeof(*lst));
    int found = -1;
    for (int tau = 0; tau < p->max_tries && found < 0; ++tau) {
        uint64_t a[4], b[4];
        draw(seed, TAG_HYP, (uint64_t)h, (uint64_t)tau, 0, 0, a);
        draw(seed, TAG_HYP, (uint64_t)h, (uint64_t)tau, 1, 0, b);
        int32_t pi[3];
        float c[9], w[9];
        int ok = 1;
        for (int j = 0; j < 3 && ok; ++j) {
            pi[j] = pick_pool(rc, cdf, a[j]);
            int cnt = modes_at(rc, pi[j], lst, cap);
            const uint8_t *px = &rc->fc.rgb[(size_t)rc->pool[pi[j]] * 3];
            int nc = 0;
            for (int m = 0; m < cnt; ++m)
                if (oracle_colour_ok(p, lst[m]->rgb, px)) lst[nc++] = lst[m];
            if (nc == 0) { ok = 0; break; }
            int m = (int)oracle_uniform_int(b[j], (uint64_t)nc);
            pool_cam(rc, pi[j], &c[j * 3]);
            for (int k = 0; k < 3; ++k) w[j * 3 + k] = lst[m]->mu[k];
        }
        if (!ok) continue;
        double R[9], t[3];
        if (oracle_check_triple(p, pi, c, w, R, t) != ORACLE_TRI_OK) continue;
        found = tau;
        memcpy(hy->R, R, sizeof(R));
        memcpy(hy->t, t, sizeof(t));
    }
    free(lst);
    hy->valid = found >= 0;
    if (hy->valid) {
        for (int i = 0; i < 9; ++i) hy->R32[i] = (float)hy->R[i];
        for (int i = 0; i < 3; ++i) hy->t32[i] = (float)hy->t[i];
    }
    hy->E = 0.0f;
    memset(&hy->inl, 0, sizeof(hy->inl));
    return found;
}

/* Energy of one mode at the transformed point y (FP32, fused as written):
 *   d = y - mu; a = Sigma^-1 d; q = d . a; term = 0.5 q + kappa
 * which is -log(pi N(y; mu, Sigma)) for the mode's weight pi. */
static float mode_term(const oracle_mode *md, const float y[3], float dd[3])
{
    float d0 = y[0] - md->mu[0], d1 = y[1] - md->mu[1], d2 = y[2] - md->mu[2];
    const float *s = md->sinv;
    float a0 = fmaf(s[2], d2, fmaf(s[1], d1, s[0] * d0));
    float a1 = fmaf(s[4], d2, fmaf(s[3], d1, s[1] * d0));
    float a2 = fmaf(s[5], d2, fmaf(s[4], d1, s[2] * d0));
    float q = fmaf(d2, a2, fmaf(d1, a1, d0 * a0));
    dd[0] = d0; dd[1] = d1; dd[2] = d2;
    return fmaf(0.5f, q, md->kappa);
}

float oracle_mode_term(const oracle_mode *md, const float y[3])
{
    float dd[3];
    return mode_term(md, y, dd);
}

int oracle_pose_from_sums(const double sums[22], double R[9], double t[3])
{
    if (!sums || !R || !t) return ORACLE_E_ARG;
    csums s;
    s.n = sums[0];
    for (int k = 0; k < 3; ++k) { s.c[k] = sums[1 + k]; s.w[k] = sums[4 + k]; }
    for (int k = 0; k < 9; ++k) s.cw[k] = sums[7 + k];
    for (int k = 0; k < 6; ++k) s.cc[k] = sums[16 + k];
    return pose_from_sums(&s, R, t);
}

typedef struct { float E; int32_t h; } ekey;

static int cmp_ekey(const void *a, const void *b)
{
    const ekey *x = (const ekey *)a, *y = (const ekey *)b;
    if (x->E < y->E) return -1;
    if (x->E > y->E) return 1;
    return x->h < y->h ? -1 : (x->h > y->h ? 1 : 0);
}

static void pose_to_mat(const double R[9], const double t[3], double T[16])
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) T[r * 4 + c] = R[r * 3 + c];
        T[r * 4 + 3] = t[r];
    }
    T[12] = 0; T[13] = 0; T[14] = 0; T[15] = 1;
}

static void trace_pose(double *dst, const double R[9], const double t[3])
{
    memcpy(dst, R, 9 * sizeof(double));
    memcpy(dst + 9, t, 3 * sizeof(double));
}

#define GROUP 8   /* energy partial sums run over groups of 8 consecutive draws */
#define LANES 64  /* inlier sums: 64 strided partial sums, then an xor butterfly */

/* the query pool (valid pixels in raster order) and each pool pixel's leaf in
 * every tree */
static int make_pool(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H, const float K[4],
                     reloc_ctx *rc)
{
    memset(rc, 0, sizeof(*rc));
    rc->f = f;
    rc->K = K;
    make_ctx(f, depth, rgb, W, H, K, &rc->fc);
    size_t P = (size_t)W * H;
    rc->pool = (int32_t *)malloc(P * sizeof(int32_t));
    if (!rc->pool) return ORACLE_E_NOMEM;
    for (size_t q = 0; q < P; ++q)
        if (valid_depth(&f->p, depth[q])) rc->pool[rc->np++] = (int32_t)q;
    if (rc->np == 0) return ORACLE_OK;
    rc->pool_leaf = (int32_t *)malloc((size_t)rc->np * f->T * sizeof(int32_t));
    if (!rc->pool_leaf) return ORACLE_E_NOMEM;
    for (int i = 0; i < rc->np; ++i) {
        int q = rc->pool[i];
        for (int t = 0; t < f->T; ++t)
            rc->pool_leaf[(size_t)i * f->T + t] = traverse(f, &rc->fc, t, q % W, q / W, (int32_t)depth[q]);
    }
    return ORACLE_OK;
}

/* The preemptive loop over hypotheses hy[0..N) (at least one valid). Round r
 * draws B pool pixels with replacement; every live hypothesis adds, per draw,
 * min(0, min over the draw's modes of the mode term) to its energy, summed
 * over groups of GROUP consecutive draws (each group in draw order, groups
 * in order); the live list is sorted by (energy, index) and the first half,
 * rounded up, survives; each survivor adds the round's inliers (draws whose
 * best mode is within inlier_m of the transformed point) to its running
 * correspondence sums and, with refinement on, is re-aligned on all of them.
 * Rounds repeat while more than one hypothesis is live (at least one
 * round). The result is the last survivor's pose and its inlier fraction. */
static void run_rounds(reloc_ctx *rc, hyp_t *hy, int N, uint64_t attempt_seed, double pose_out[16],
                       float *score_out, oracle_trace *tr)
{
    oracle_forest *f = rc->f;
    const oracle_params *p = &f->p;
    int B = p->batch_pixels;
    int32_t *alive = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    int na = 0;
    for (int h = 0; h < N; ++h)
        if (hy[h].valid) alive[na++] = h;
    int cap = f->T * f->M;
    const oracle_mode **lst = (const oracle_mode **)malloc((size_t)cap * sizeof(*lst));
    int32_t *dpool = (int32_t *)malloc((size_t)B * sizeof(int32_t));
    float (*dc)[3] = (float (*)[3])malloc((size_t)B * sizeof(*dc));
    ekey *ek = (ekey *)malloc((size_t)N * sizeof(ekey));
    csums *lane = (csums *)malloc(LANES * sizeof(csums));
    csums *tmp = (csums *)malloc(LANES * sizeof(csums));
    float inl2 = p->inlier_m * p->inlier_m;
    int r = 0;
    do {
        /* draw B pool pixels with replacement */
        for (int i = 0; i < B; ++i) {
            uint64_t u[4];
            draw(attempt_seed, TAG_PIX, (uint64_t)r, (uint64_t)i, 0, 0, u);
            dpool[i] = (int)oracle_uniform_int(u[0], (uint64_t)rc->np);
            pool_cam(rc, dpool[i], dc[i]);
        }
        if (tr && tr->n_alive && r < tr->cap_rounds) tr->n_alive[r] = na;
        for (int a = 0; a < na; ++a) {
            hyp_t *x = &hy[alive[a]];
            float S = 0.0f, g = 0.0f;
            memset(lane, 0, LANES * sizeof(csums));
            for (int i = 0; i < B; ++i) {
                const float *c = dc[i];
                float y[3];
                for (int k = 0; k < 3; ++k)
                    y[k] = fmaf(x->R32[k * 3 + 0], c[0], fmaf(x->R32[k * 3 + 1], c[1], fmaf(x->R32[k * 3 + 2], c[2], x->t32[k])));
                int cnt = modes_at(rc, dpool[i], lst, cap);
                float best = 0.0f;
                int bm = -1;
                float bd[3] = {0, 0, 0};
                for (int m = 0; m < cnt; ++m) {
                    float dd[3];
                    float term = mode_term(lst[m], y, dd);
                    if (bm < 0 || term < best) { best = term; bm = m; bd[0] = dd[0]; bd[1] = dd[1]; bd[2] = dd[2]; }
                }
                float e = (bm >= 0 && best < 0.0f) ? best : 0.0f;
                g = g + e;
                if ((i % GROUP) == GROUP - 1 || i == B - 1) { S = S + g; g = 0.0f; }
                if (bm >= 0 && (bd[0] * bd[0] + bd[1] * bd[1]) + bd[2] * bd[2] <= inl2)
                    csums_add_point(&lane[i % LANES], c, lst[bm]->mu);
            }
            x->E = x->E + S;
            /* xor butterfly over the 64 lane sums; lane 0 holds the total */
            for (int o = LANES / 2; o >= 1; o /= 2) {
                for (int l = 0; l < LANES; ++l) { tmp[l] = lane[l]; csums_add(&tmp[l], &lane[l ^ o]); }
                memcpy(lane, tmp, LANES * sizeof(csums));
            }
            csums_add(&x->inl, &lane[0]);
        }
        for (int a = 0; a < na; ++a) { ek[a].E = hy[alive[a]].E; ek[a].h = alive[a]; }
        if (tr && r < tr->cap_rounds) {
            for (int a = 0; a < na && a < tr->cap_hyp; ++a) {
                if (tr->alive) tr->alive[(size_t)r * tr->cap_hyp + a] = alive[a];
                if (tr->energy) tr->energy[(size_t)r * tr->cap_hyp + a] = hy[alive[a]].E;
                if (tr->n_inliers) tr->n_inliers[(size_t)r * tr->cap_hyp + a] = (int32_t)hy[alive[a]].inl.n;
            }
        }
        qsort(ek, (size_t)na, sizeof(ekey), cmp_ekey);
        na = (na + 1) / 2;
        for (int a = 0; a < na; ++a) alive[a] = ek[a].h;
        for (int a = 0; a < na; ++a) {
            hyp_t *x = &hy[alive[a]];
            double R[9], t[3];
            if (p->refine && pose_from_sums(&x->inl, R, t) == 0) {
                memcpy(x->R, R, sizeof(R));
                memcpy(x->t, t, sizeof(t));
                for (int i = 0; i < 9; ++i) x->R32[i] = (float)R[i];
                for (int i = 0; i < 3; ++i) x->t32[i] = (float)t[i];
            }
            if (tr && tr->pose_after && r < tr->cap_rounds && a < tr->cap_hyp)
                trace_pose(&tr->pose_after[((size_t)r * tr->cap_hyp + a) * 12], x->R, x->t);
        }
        r++;
    } while (na > 1);
    int best = alive[0];
    pose_to_mat(hy[best].R, hy[best].t, pose_out);
    *score_out = (float)(hy[best].inl.n / ((double)r * (double)B));
    if (tr && tr->n_rounds) *tr->n_rounds = r;
    if (tr && tr->final_hyp) *tr->final_hyp = best;
    free(alive); free(lst); free(dpool); free(dc); free(ek); free(lane); free(tmp);
}

static void free_ctx(reloc_ctx *rc)
{
    free(rc->pool);
    free(rc->pool_leaf);
}

int oracle_relocalise(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H,
                      const float K[4], uint64_t attempt_seed, int n_hyp, const uint32_t *pixel_weights,
                      double pose_out[16], float *score_out, oracle_trace *tr)
{
    if (!frame_args_ok(f, depth, rgb, W, H, K) || !pose_out || !score_out) return ORACLE_E_ARG;
    const oracle_params *p = &f->p;
    int N = n_hyp > 0 ? n_hyp : p->n_hypotheses;
    for (int k = 0; k < 16; ++k) pose_out[k] = (k % 5 == 0) ? 1.0 : 0.0;
    *score_out = 0.0f;
    reloc_ctx rc;
    int st = make_pool(f, depth, rgb, W, H, K, &rc);
    if (st) { free_ctx(&rc); return st; }
    if (tr && tr->pool_size) *tr->pool_size = rc.np;
    if (rc.np == 0) { free_ctx(&rc); return ORACLE_FAIL_NO_VALID_PIXELS; }
    uint64_t *cdf = NULL;
    if (pixel_weights) {
        cdf = (uint64_t *)malloc((size_t)rc.np * sizeof(uint64_t));
        uint64_t acc = 0;
        for (int i = 0; i < rc.np; ++i) { acc += pixel_weights[rc.pool[i]]; cdf[i] = acc; }
        if (acc == 0) { free(cdf); cdf = NULL; }
    }
    hyp_t *hy = (hyp_t *)calloc((size_t)N, sizeof(hyp_t));
    int na = 0;
    for (int h = 0; h < N; ++h) {
        int tau = make_hypothesis(&rc, attempt_seed, h, cdf, &hy[h]);
        if (tr && tr->hyp_try && h < tr->cap_hyp) tr->hyp_try[h] = tau;
        if (tr && tr->hyp_pose && h < tr->cap_hyp && tau >= 0) trace_pose(&tr->hyp_pose[(size_t)h * 12], hy[h].R, hy[h].t);
        na += hy[h].valid;
    }
    int status = ORACLE_OK;
    if (na == 0) {
        status = f->total_samples == 0 ? ORACLE_FAIL_NO_MODES : ORACLE_FAIL_NO_HYPOTHESIS;
        if (tr && tr->n_rounds) *tr->n_rounds = 0;
    } else {
        run_rounds(&rc, hy, N, attempt_seed, pose_out, score_out, tr);
    }
    free(hy); free(cdf); free_ctx(&rc);
    return status;
}

/* The preemptive loop alone, over caller-given hypotheses: poses [n][12]
 * (R row-major, then t, FP64), valid [n]; the same rounds as
 * oracle_relocalise runs after generating its hypotheses. */
int oracle_preemptive(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H, const float K[4],
                      uint64_t attempt_seed, int n_hyp, const double *poses, const int32_t *valid, double pose_out[16],
                      float *score_out, oracle_trace *tr)
{
    if (!frame_args_ok(f, depth, rgb, W, H, K) || !pose_out || !score_out || n_hyp < 1 || !poses || !valid)
        return ORACLE_E_ARG;
    for (int k = 0; k < 16; ++k) pose_out[k] = (k % 5 == 0) ? 1.0 : 0.0;
    *score_out = 0.0f;
    reloc_ctx rc;
    int st = make_pool(f, depth, rgb, W, H, K, &rc);
    if (st) { free_ctx(&rc); return st; }
    if (tr && tr->pool_size) *tr->pool_size = rc.np;
    if (rc.np == 0) { free_ctx(&rc); return ORACLE_FAIL_NO_VALID_PIXELS; }
    hyp_t *hy = (hyp_t *)calloc((size_t)n_hyp, sizeof(hyp_t));
    int na = 0;
    for (int h = 0; h < n_hyp; ++h) {
        hy[h].valid = valid[h] != 0;
        memcpy(hy[h].R, poses + (size_t)h * 12, 9 * sizeof(double));
        memcpy(hy[h].t, poses + (size_t)h * 12 + 9, 3 * sizeof(double));
        for (int i = 0; i < 9; ++i) hy[h].R32[i] = (float)hy[h].R[i];
        for (int i = 0; i < 3; ++i) hy[h].t32[i] = (float)hy[h].t[i];
        na += hy[h].valid;
    }
    int status = ORACLE_OK;
    if (na == 0) {
        status = ORACLE_FAIL_NO_HYPOTHESIS;
        if (tr && tr->n_rounds) *tr->n_rounds = 0;
    } else {
        run_rounds(&rc, hy, n_hyp, attempt_seed, pose_out, score_out, tr);
    }
    free(hy); free_ctx(&rc);
    return status;
}

/* ------------------------------------------------------------------------ */
/* success criterion: <= 5 cm and <= 5 degrees (Sec. 4.2.2, Table 2)        */
/* ------------------------------------------------------------------------ */

int oracle_pose_success(const double est[16], const double gt[16], double *dt_m, double *dang_deg)
{
    if (!est || !gt) return ORACLE_E_ARG;
    double dx = est[3] - gt[3], dy = est[7] - gt[7], dz = est[11] - gt[11];
    double dt = sqrt(dx * dx + dy * dy + dz * dz);
    /* relative rotation Q = R_est^T R_gt; angle = atan2(|axis vector| / 2, (tr Q - 1) / 2) */
    double Q[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            Q[r * 3 + c] = est[0 * 4 + r] * gt[0 * 4 + c] + est[1 * 4 + r] * gt[1 * 4 + c] + est[2 * 4 + r] * gt[2 * 4 + c];
    double vx = Q[7] - Q[5], vy = Q[2] - Q[6], vz = Q[3] - Q[1];
    double s = 0.5 * sqrt(vx * vx + vy * vy + vz * vz);
    double c = 0.5 * (Q[0] + Q[4] + Q[8] - 1.0);
    double ang = atan2(s, c) * 180.0 / M_PI;
    if (dt_m) *dt_m = dt;
    if (dang_deg) *dang_deg = ang;
    return (dt <= 0.05 && ang <= 5.0) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* depth-difference verification (Sec. 3.3.1, Eqs. 3-4)                    */
/* ------------------------------------------------------------------------ */

/* Omega is every pixel, Omega_s the pixels where D_s > 0; the proposed pose
 * is plausible if |Omega_a| / |Omega| > 0.5, and the mean of |D_a - D_b| over
 * Omega_a intersect Omega_b must be below 5 cm. Sums are exact integers. */
int oracle_verify(const uint16_t *da, const uint16_t *db, int W, int H, double *valid_frac, double *mu_m,
                  int *accept)
{
    if (!da || !db || W < 1 || H < 1 || !valid_frac || !mu_m || !accept) return ORACLE_E_ARG;
    size_t P = (size_t)W * H;
    uint64_t na = 0, nab = 0, sum = 0;
    for (size_t p = 0; p < P; ++p) {
        if (da[p] > 0) na++;
        if (da[p] > 0 && db[p] > 0) {
            nab++;
            sum += (uint64_t)(da[p] > db[p] ? da[p] - db[p] : db[p] - da[p]);
        }
    }
    *valid_frac = (double)na / (double)P;
    *mu_m = nab ? ((double)sum / (double)nab) / 1000.0 : INFINITY;
    *accept = (*valid_frac > 0.5 && *mu_m < 0.05) ? 1 : 0;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* learned proposal                                                         */
/* ------------------------------------------------------------------------ */

enum { TAG_MLP_INIT = 5 };

float oracle_bf16(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7F800000u) == 0x7F800000u) {          /* inf or nan: truncate, keep nan quiet */
        b &= 0xFFFF0000u;
        if ((b & 0x007F0000u) == 0 && (x != x)) b |= 0x00400000u;
    } else {
        b = (b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u;
    }
    float y;
    memcpy(&y, &b, 4);
    return y;
}

/* Per-pixel inputs, in this order:
 *   0      depth / 5000
 *   1..8   the 8 extra feature responses: depth ones clamped to +-5000 mm and
 *          divided by 1000, colour ones divided by 255
 *   9..20  for the 3 modes of M(p) with the largest weight pi = n / min(k, R)
 *          (ties: lower (tree, mode)): pi and -log(Sigma^-1_ii) / 10 for
 *          i = x, y, z; zeros when there are fewer modes
 *   21     mean reservoir fill: sum over trees of min(k, R) / (T R)
 *   22, 23 u / W, v / H */
int oracle_features24(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H, const float K[4],
                      const int32_t *pix, int n, float *x)
{
    if (!frame_args_ok(f, depth, rgb, W, H, K) || (!pix && n > 0) || (!x && n > 0) || n < 0) return ORACLE_E_ARG;
    frame_ctx fc;
    make_ctx(f, depth, rgb, W, H, K, &fc);
    for (int i = 0; i < n; ++i) {
        float *o = x + (size_t)i * 24;
        for (int k = 0; k < 24; ++k) o[k] = 0.0f;
        int p = pix[i];
        if (p < 0 || p >= W * H) return ORACLE_E_ARG;
        uint32_t d = depth[p];
        if (!valid_depth(&f->p, d)) continue;
        int u = p % W, v = p / W;
        o[0] = (float)d / 5000.0f;
        for (int j = 0; j < 8; ++j) {
            int32_t r = feature(&fc, &f->extra[j], u, v, (int32_t)d);
            if (f->extra[j].kind == 0) {
                if (r > 5000) r = 5000;
                if (r < -5000) r = -5000;
                o[1 + j] = (float)r / 1000.0f;
            } else {
                o[1 + j] = (float)r / 255.0f;
            }
        }
        float best_pi[3] = {-1.0f, -1.0f, -1.0f};
        const oracle_mode *best_m[3] = {NULL, NULL, NULL};
        int64_t fill = 0;
        for (int t = 0; t < f->T; ++t) {
            int32_t leaf = traverse(f, &fc, t, u, v, (int32_t)d);
            ensure_modes(f, t, leaf);
            size_t li = (size_t)t * f->L + leaf;
            uint32_t k = f->counter[li];
            uint32_t cap = k < (uint32_t)f->R ? k : (uint32_t)f->R;
            fill += cap;
            for (int m = 0; m < f->nmodes[li]; ++m) {
                const oracle_mode *md = &f->modes[li * f->M + m];
                float pi = (float)md->n / (float)cap;
                /* insert keeping the first (lowest (tree, mode)) among equals */
                for (int s = 0; s < 3; ++s)
                    if (pi > best_pi[s]) {
                        for (int q = 2; q > s; --q) { best_pi[q] = best_pi[q - 1]; best_m[q] = best_m[q - 1]; }
                        best_pi[s] = pi;
                        best_m[s] = md;
                        break;
                    }
            }
        }
        for (int s = 0; s < 3; ++s) {
            if (!best_m[s]) continue;
            o[9 + 4 * s] = best_pi[s];
            o[10 + 4 * s] = -logf(best_m[s]->sinv[0]) / 10.0f;
            o[11 + 4 * s] = -logf(best_m[s]->sinv[3]) / 10.0f;
            o[12 + 4 * s] = -logf(best_m[s]->sinv[5]) / 10.0f;
        }
        o[21] = (float)fill / (float)((int64_t)f->T * f->R);
        o[22] = (float)u / (float)W;
        o[23] = (float)v / (float)H;
    }
    return ORACLE_OK;
}

/* The label of a pixel under `pose` is the probability that its hypothesis
 * pick lands on a correct mode: among the modes of its leaves that pass the
 * pick's colour test (oracle_colour_ok), the fraction within 5 cm of the
 * pixel's world point y = R c + t (the pose rounded to FP32, the same fused
 * chain as scoring; (d0 d0 + d1 d1) + d2 d2 <= 0.05^2 in FP32), as
 * round(255 good / candidates), 0 without candidates. */
int oracle_label(oracle_forest *f, const uint16_t *depth, const uint8_t *rgb, int W, int H, const float K[4],
                 const double pose[16], const int32_t *pix, int n, uint8_t *label)
{
    if (!frame_args_ok(f, depth, rgb, W, H, K) || !pose || (!pix && n > 0) || (!label && n > 0) || n < 0)
        return ORACLE_E_ARG;
    frame_ctx fc;
    make_ctx(f, depth, rgb, W, H, K, &fc);
    float R32[9], t32[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R32[r * 3 + c] = (float)pose[r * 4 + c];
        t32[r] = (float)pose[r * 4 + 3];
    }
    const float lim = 0.05f * 0.05f;
    for (int i = 0; i < n; ++i) {
        label[i] = 0;
        int p = pix[i];
        if (p < 0 || p >= W * H) return ORACLE_E_ARG;
        uint32_t d = depth[p];
        if (!valid_depth(&f->p, d)) continue;
        int u = p % W, v = p / W;
        float c[3], y[3];
        cam_point(u, v, d, K, c);
        for (int k = 0; k < 3; ++k)
            y[k] = fmaf(R32[k * 3 + 0], c[0], fmaf(R32[k * 3 + 1], c[1], fmaf(R32[k * 3 + 2], c[2], t32[k])));
        unsigned cand = 0, good = 0;
        for (int t = 0; t < f->T; ++t) {
            int32_t leaf = traverse(f, &fc, t, u, v, (int32_t)d);
            ensure_modes(f, t, leaf);
            size_t li = (size_t)t * f->L + leaf;
            for (int m = 0; m < f->nmodes[li]; ++m) {
                const oracle_mode *md = &f->modes[li * f->M + m];
                if (!oracle_colour_ok(&f->p, md->rgb, &rgb[(size_t)p * 3])) continue;
                cand++;
                float d0 = y[0] - md->mu[0], d1 = y[1] - md->mu[1], d2 = y[2] - md->mu[2];
                if ((d0 * d0 + d1 * d1) + d2 * d2 <= lim) good++;
            }
        }
        label[i] = cand ? (uint8_t)((255u * good + cand / 2u) / cand) : 0;
    }
    return ORACLE_OK;
}

void oracle_mlp_init(uint64_t seed, float *w)
{
    /* Glorot-uniform weights from Philox (key (seed, 5), counter (k, 0, 0, 0)),
     * zero biases */
    const int fi[3] = {24, 64, 64}, fo[3] = {64, 64, 1};
    const int off[3] = {0, 24 * 64 + 64, 24 * 64 + 64 + 64 * 64 + 64};
    const int cnt[3] = {24 * 64, 64 * 64, 64};
    for (int k = 0; k < ORACLE_MLP_NPARAM; ++k) w[k] = 0.0f;
    for (int l = 0; l < 3; ++l) {
        float a = sqrtf(6.0f / (float)(fi[l] + fo[l]));
        for (int k = 0; k < cnt[l]; ++k) {
            uint64_t u[4];
            draw(seed, TAG_MLP_INIT, (uint64_t)(off[l] + k), 0, 0, 0, u);
            float r = (float)(u[0] >> 40) / 16777216.0f;
            w[off[l] + k] = (2.0f * r - 1.0f) * a;
        }
    }
}

#define O_W1 0
#define O_B1 (24 * 64)
#define O_W2 (O_B1 + 64)
#define O_B2 (O_W2 + 64 * 64)
#define O_W3 (O_B2 + 64)
#define O_B3 (O_W3 + 64)

/* forward of one row; activations are accumulated in FP64, rounded to FP32
 * and then to bfloat16 as the GPU stores them */
static double mlp_row(const float *w, const float *xin, double xb[24], double h1p[64], double h1[64], double h2p[64],
                      double h2[64])
{
    for (int i = 0; i < 24; ++i) xb[i] = oracle_bf16(xin[i]);
    for (int j = 0; j < 64; ++j) {
        double a = 0.0;
        for (int i = 0; i < 24; ++i) a += (double)oracle_bf16(w[O_W1 + j * 24 + i]) * xb[i];
        a += (double)w[O_B1 + j];
        h1p[j] = a;
        h1[j] = a > 0.0 ? (double)oracle_bf16((float)a) : 0.0;
    }
    for (int j = 0; j < 64; ++j) {
        double a = 0.0;
        for (int i = 0; i < 64; ++i) a += (double)oracle_bf16(w[O_W2 + j * 64 + i]) * h1[i];
        a += (double)w[O_B2 + j];
        h2p[j] = a;
        h2[j] = a > 0.0 ? (double)oracle_bf16((float)a) : 0.0;
    }
    double z = 0.0;
    for (int i = 0; i < 64; ++i) z += (double)oracle_bf16(w[O_W3 + i]) * h2[i];
    return z + (double)w[O_B3];
}

int oracle_mlp_forward(const float *w, const float *x, int n, double *z)
{
    if (!w || (!x && n > 0) || (!z && n > 0) || n < 0) return ORACLE_E_ARG;
    double xb[24], h1p[64], h1[64], h2p[64], h2[64];
    for (int r = 0; r < n; ++r) z[r] = mlp_row(w, x + (size_t)r * 24, xb, h1p, h1, h2p, h2);
    return ORACLE_OK;
}

int oracle_mlp_grad(const float *w, const float *x, const uint8_t *y, int n, double *grad, double *loss)
{
    if (!w || !x || !y || !grad || !loss || n < 1) return ORACLE_E_ARG;
    for (int k = 0; k < ORACLE_MLP_NPARAM; ++k) grad[k] = 0.0;
    double L = 0.0;
    double xb[24], h1p[64], h1[64], h2p[64], h2[64], d2[64], d1[64];
    for (int r = 0; r < n; ++r) {
        double z = mlp_row(w, x + (size_t)r * 24, xb, h1p, h1, h2p, h2);
        double t = (double)y[r] / 255.0;
        L += (z > 0 ? z : 0.0) - z * t + log1p(exp(-fabs(z)));
        double dz = (1.0 / (1.0 + exp(-z)) - t) / (double)n;
        for (int i = 0; i < 64; ++i) grad[O_W3 + i] += dz * h2[i];
        grad[O_B3] += dz;
        for (int j = 0; j < 64; ++j) d2[j] = h2p[j] > 0.0 ? dz * (double)oracle_bf16(w[O_W3 + j]) : 0.0;
        for (int j = 0; j < 64; ++j) {
            for (int i = 0; i < 64; ++i) grad[O_W2 + j * 64 + i] += d2[j] * h1[i];
            grad[O_B2 + j] += d2[j];
        }
        for (int i = 0; i < 64; ++i) {
            double a = 0.0;
            for (int j = 0; j < 64; ++j) a += d2[j] * (double)oracle_bf16(w[O_W2 + j * 64 + i]);
            d1[i] = h1p[i] > 0.0 ? a : 0.0;
        }
        for (int j = 0; j < 64; ++j) {
            for (int i = 0; i < 24; ++i) grad[O_W1 + j * 24 + i] += d1[j] * xb[i];
            grad[O_B1 + j] += d1[j];
        }
    }
    *loss = L / (double)n;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* split training: a split structure learned on one scene, whose leaves are */
/* then adapted online to others (Sec. 4.2.2, Table 2: a forest pre-trained */
/* on one scene and adapted to the rest)                                    */
/* ------------------------------------------------------------------------ */

/* Reading (the paper takes the pre-trained forest from its relocaliser's
 * authors and gives no training procedure): every node of every tree, level
 * by level from the root, takes from n_cand candidate splits, drawn like
 * random ones from the generator keyed by (seed, TRAIN) at counter (tree,
 * node, candidate), the one that leaves the training samples reaching it
 * with the smallest summed squared deviation of their world points from
 * their child's mean (the reduction-in-spatial-variance objective of
 * scene-coordinate regression forests); ties go to the lower candidate. A
 * sample is every stride-th pixel in u and v, from stride / 2, of every
 * training frame with a valid depth, with its world point in integer mm as
 * adaptation stores it. The per-child sums (count, coordinate sums, sum of
 * squared norms) are exact integers; the cost of a child with n samples is
 * S2 - |S|^2 / n in FP64, in that order, summed left then right. */

typedef struct {
    int frame, u, v;
    int32_t d;
    int64_t x, y, z;
} tsample;

static double split_cost(const int64_t s[10])
{
    double c = 0.0;
    for (int side = 0; side < 2; ++side) {
        const int64_t *q = s + 5 * side;
        if (q[0] == 0) continue;
        double sx = (double)q[1], sy = (double)q[2], sz = (double)q[3];
        c = c + ((double)q[4] - ((sx * sx + sy * sy) + sz * sz) / (double)q[0]);
    }
    return c;
}

int oracle_train_forest(oracle_forest *f, int n_frames, const uint16_t *const *depth, const uint8_t *const *rgb,
                        int W, int H, const float K[4], const double *poses, int stride, int n_cand)
{
    if (!f || n_frames < 1 || !depth || !rgb || !poses || stride < 1 || n_cand < 1 || n_cand > 64) return ORACLE_E_ARG;
    if (f->dropped) return ORACLE_E_ARG;
    for (int k = 0; k < n_frames; ++k)
        if (!frame_args_ok(f, depth[k], rgb[k], W, H, K) || !is_se3(poses + 16 * k)) return ORACLE_E_ARG;
    /* samples, frame by frame in raster order of the sampling grid */
    size_t cap = (size_t)n_frames * (size_t)((W + stride - 1) / stride) * (size_t)((H + stride - 1) / stride);
    tsample *smp = (tsample *)malloc((cap ? cap : 1) * sizeof(tsample));
    frame_ctx *ctx = (frame_ctx *)malloc((size_t)n_frames * sizeof(frame_ctx));
    if (!smp || !ctx) {
        free(smp); free(ctx);
        return ORACLE_E_NOMEM;
    }
    size_t S = 0;
    for (int k = 0; k < n_frames; ++k) {
        make_ctx(f, depth[k], rgb[k], W, H, K, &ctx[k]);
        const double *P = poses + 16 * k;
        float R32[9], t32[3];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) R32[r * 3 + c] = (float)P[r * 4 + c];
            t32[r] = (float)P[r * 4 + 3];
        }
        for (int v = stride / 2; v < H; v += stride)
            for (int u = stride / 2; u < W; u += stride) {
                uint32_t d = depth[k][(size_t)v * W + u];
                if (!valid_depth(&f->p, d)) continue;
                float c[3], w[3];
                cam_point(u, v, d, K, c);
                for (int a = 0; a < 3; ++a)
                    w[a] = ((R32[a * 3 + 0] * c[0] + R32[a * 3 + 1] * c[1]) + R32[a * 3 + 2] * c[2]) + t32[a];
                tsample *q = &smp[S++];
                q->frame = k; q->u = u; q->v = v; q->d = (int32_t)d;
                q->x = (int32_t)rintf(w[0] * 1000.0f);
                q->y = (int32_t)rintf(w[1] * 1000.0f);
                q->z = (int32_t)rintf(w[2] * 1000.0f);
            }
    }
    int64_t *node = (int64_t *)malloc((S ? S : 1) * sizeof(int64_t));
    size_t *order = (size_t *)malloc((S ? S : 1) * sizeof(size_t));
    size_t *start = (size_t *)malloc(((size_t)f->L + 1) * sizeof(size_t));
    if (!node || !order || !start) {
        free(smp); free(ctx); free(node); free(order); free(start);
        return ORACLE_E_NOMEM;
    }
    for (int t = 0; t < f->T; ++t) {
        onode *tree = &f->nodes[(size_t)t * (f->L - 1)];
        for (size_t s = 0; s < S; ++s) node[s] = 0;
        for (int l = 0; l < f->D; ++l) {
            const int64_t first = ((int64_t)1 << l) - 1, count = (int64_t)1 << l;
            /* the samples of each node of the level together (counting sort) */
            for (int64_t j = 0; j <= count; ++j) start[j] = 0;
            for (size_t s = 0; s < S; ++s) start[node[s] - first + 1]++;
            for (int64_t j = 0; j < count; ++j) start[j + 1] += start[j];
            for (size_t s = 0; s < S; ++s) order[start[node[s] - first]++] = s;
            for (int64_t j = count; j > 0; --j) start[j] = start[j - 1];
            start[0] = 0;
            for (int64_t j = 0; j < count; ++j) {
                const int64_t i = first + j;
                double best_c = INFINITY;
                onode chosen;
                for (int k = 0; k < n_cand; ++k) {
                    onode cand;
                    draw_node(f->p.seed, TAG_TRAIN, &f->p, (uint64_t)t, (uint64_t)i, (uint64_t)k, &cand);
                    int64_t sums[10] = {0};
                    for (size_t o = start[j]; o < start[j + 1]; ++o) {
                        const tsample *q = &smp[order[o]];
                        int32_t r = feature(&ctx[q->frame], &cand, q->u, q->v, q->d);
                        int64_t *a = sums + (r >= cand.thr ? 5 : 0);
                        a[0] += 1;
                        a[1] += q->x; a[2] += q->y; a[3] += q->z;
                        a[4] += q->x * q->x + q->y * q->y + q->z * q->z;
                    }
                    double c = split_cost(sums);
                    if (c < best_c) {
                        best_c = c;
                        chosen = cand;
                    }
                }
                tree[i] = chosen;
            }
            /* route every sample one level down */
            for (size_t s = 0; s < S; ++s) {
                const tsample *q = &smp[s];
                const onode *nd = &tree[node[s]];
                int32_t r = feature(&ctx[q->frame], nd, q->u, q->v, q->d);
                node[s] = 2 * node[s] + 1 + (r >= nd->thr ? 1 : 0);
            }
        }
    }
    free(smp); free(ctx); free(node); free(order); free(start);
    /* the leaves of the new structure start empty */
    size_t TL = (size_t)f->T * f->L;
    memset(f->counter, 0, TL * sizeof(uint32_t));
    memset(f->res, 0, TL * f->R * sizeof(oracle_entry));
    memset(f->modes, 0, TL * f->M * sizeof(oracle_mode));
    for (size_t i = 0; i < TL; ++i) f->nmodes[i] = 0;
    f->total_samples = 0;
    return ORACLE_OK;
}
