// Learned proposal on the GPU: a 24-64-64-1 MLP (ReLU, ReLU, sigmoid) that
// predicts, per pixel, the probability that its hypothesis pick (a mode drawn
// among the colour-consistent modes of its leaves) lies within 5 cm of its
// true world point. Its output becomes integer pick weights for
// the three pixel picks of every hypothesis try; uniform preemptive scoring
// stays the judge.
//
// Matrix products run on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16:
// bfloat16 operands, FP32 accumulation). One wavefront owns a tile of 64 rows:
// forward (two MFMA layers and an FP32 output dot), loss, and backward (weight
// gradients and the hidden-layer input gradient are MFMA as well), staged in
// LDS; per-tile gradient partials are summed in a fixed order, then Adam
// updates the FP32 master weights and their bfloat16 copies are refreshed.
//
// Also here: the per-pixel inputs and the inlier labeller that trains the MLP
// from poses accepted by the depth-difference check of Sec. 3.3.1, Eqs. 3-4
// (verify.hip).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mlp_dev.h"

namespace rl {

int update_modes(Forest *f, hipStream_t s);
int frame_from(const Forest *f, const uint16_t *depth, const uint8_t *rgb, const reloc_intrinsics *K, Frame &fr);

}  // namespace rl

struct reloc_mlp {
    float *w = nullptr;          // [NP] FP32 master weights
    float *m = nullptr, *v = nullptr;
    float *grad = nullptr;       // [NP + 1]: gradient, then the loss
    float *partial = nullptr;    // [cap_tiles][NP + 1]
    int cap_tiles = 0;
    uint16_t *q = nullptr;       // [NQ] bfloat16 copies
    int32_t *rows = nullptr;     // [cap_rows] minibatch row indices
    int cap_rows = 0;
    int step = 0;
};

namespace rl {

// one 16x32 by 32x16 product of host-given tiles (checks the lane layout)
__global__ void __launch_bounds__(64) k_mfma_probe(const uint16_t *__restrict__ A, const uint16_t *__restrict__ Bt,
                                                   float *__restrict__ C)
{
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mfma_tile(A, 32, Bt, 32, 32, acc);
    const int l = __lane_id();
    for (int i = 0; i < 4; ++i) C[(4 * (l >> 4) + i) * 16 + (l & 15)] = acc[i];
}

// ---------------------------------------------------------------------------
// initialisation and bfloat16 copies
// ---------------------------------------------------------------------------

// Glorot-uniform weights from Philox (key (seed, 5), counter (k, 0, 0, 0)),
// zero biases
__global__ void k_mlp_init(float *__restrict__ w, uint64_t seed)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NP) return;
    int fi = 0, fo = 0;
    if (k < OB1) { fi = 24; fo = 64; }
    else if (k >= OW2 && k < OB2) { fi = 64; fo = 64; }
    else if (k >= OW3 && k < OB3) { fi = 64; fo = 1; }
    if (!fi) {
        w[k] = 0.0f;
        return;
    }
    const float a = sqrtf(6.0f / (float)(fi + fo));
    const U4 u = philox((uint64_t)k, 0, 0, 0, seed, TAG_MLP_INIT);
    const float r = (float)(u.x[0] >> 40) / 16777216.0f;
    w[k] = (2.0f * r - 1.0f) * a;
}

__global__ void k_mlp_pack(const float *__restrict__ w, uint16_t *__restrict__ q)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 64 * 32) {
        const int j = k / 32, i = k % 32;
        q[QW1 + k] = i < 24 ? f2bf(w[OW1 + j * 24 + i]) : (uint16_t)0;
    }
    if (k < 64 * 64) {
        const int j = k / 64, i = k % 64;
        const uint16_t h = f2bf(w[OW2 + k]);
        q[QW2 + k] = h;
        q[QW2T + i * 64 + j] = h;
    }
    if (k < 64) q[QW3 + k] = f2bf(w[OW3 + k]);
}

// ---------------------------------------------------------------------------
// one 64-row tile in LDS
// ---------------------------------------------------------------------------

struct __align__(16) TileLds {
    uint16_t X[ROWS * 32], XT[32 * ROWS];
    uint16_t H1[ROWS * 64], H1T[64 * ROWS];
    uint16_t H2[ROWS * 64];
    uint16_t Db[ROWS * 64], DT[64 * ROWS];
    float z[ROWS], dz[ROWS];
};

// X (row-major) -> XT
__device__ __forceinline__ void tile_transpose_x(TileLds &S)
{
    const int l = __lane_id();
    for (int k = 0; k < 32; ++k) S.XT[k * ROWS + l] = S.X[l * 32 + k];
    __syncthreads();
}

// column sums of a 4-row-per-lane tile value over the 4 row groups of a wave
__device__ __forceinline__ float col_sum(float s)
{
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    return s;
}

// backward of the tile: gradient partial (NP values) and the loss sum of the
// valid rows (entry NP) into `out`; the target of label q is q / 255 and
// dz = (sigmoid(z) - q / 255) * inv_n
__device__ void tile_backward(TileLds &S, const uint16_t *__restrict__ q, const uint8_t *ys, int nvalid, float inv_n,
                              float *__restrict__ out)
{
    const int l = __lane_id(), col = l & 15, r0 = (l >> 4) * 4;
    {
        const float z = S.z[l];
        float dz = 0.0f, loss = 0.0f;
        if (l < nvalid) {
            const float y = (float)ys[l] / 255.0f;
            dz = (1.0f / (1.0f + expf(-z)) - y) * inv_n;
            loss = fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
        }
        S.dz[l] = dz;
        for (int o = 32; o >= 1; o >>= 1) loss += __shfl_xor(loss, o, 64);
        if (l == 0) out[NP] = loss;
    }
    __syncthreads();
    {   // dw3[j] = sum_rows dz h2 (lane = j), db3 = sum dz
        float g = 0.0f, b = 0.0f;
        for (int row = 0; row < ROWS; ++row) {
            g = fmaf(S.dz[row], bf2f(S.H2[row * 64 + l]), g);
            b += S.dz[row];
        }
        out[OW3 + l] = g;
        if (l == 0) out[OB3] = b;
    }
    // dH2 = dz w3 [h2 > 0]; db2 = column sums
    for (int tj = 0; tj < 4; ++tj) {
        const int c = 16 * tj + col;
        const float w3 = bf2f(q[QW3 + c]);
        float bs = 0.0f;
        for (int ti = 0; ti < 4; ++ti)
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * ti + r0 + i;
                const float d = S.H2[row * 64 + c] ? S.dz[row] * w3 : 0.0f;
                bs += d;
                const uint16_t h = f2bf(d);
                S.Db[row * 64 + c] = h;
                S.DT[c * ROWS + row] = h;
            }
        bs = col_sum(bs);
        if (l < 16) out[OB2 + c] = bs;
    }
    __syncthreads();
    // dW2 = dH2^T H1
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 4; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_tile(S.DT + 16 * ti * ROWS, ROWS, S.H1T + 16 * tj * ROWS, ROWS, ROWS, acc);
            for (int i = 0; i < 4; ++i) out[OW2 + (16 * ti + r0 + i) * 64 + 16 * tj + col] = acc[i];
        }
    __syncthreads();
    // dH1 = dH2 W2 [h1 > 0] (into DT, transposed); db1 = column sums
    for (int tj = 0; tj < 4; ++tj) {
        const int c = 16 * tj + col;
        float bs = 0.0f;
        floatx4 acc[4];
        for (int ti = 0; ti < 4; ++ti) {
            floatx4 a0 = {0.0f, 0.0f, 0.0f, 0.0f};
            acc[ti] = mfma_tile(S.Db + 16 * ti * 64, 64, q + QW2T + 16 * tj * 64, 64, 64, a0);
        }
        __syncthreads();
        for (int ti = 0; ti < 4; ++ti)
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * ti + r0 + i;
                const float d = S.H1[row * 64 + c] ? acc[ti][i] : 0.0f;
                bs += d;
                S.DT[c * ROWS + row] = f2bf(d);
            }
        bs = col_sum(bs);
        if (l < 16) out[OB1 + c] = bs;
    }
    __syncthreads();
    // dW1 = dH1^T X (input columns 24..31 are padding)
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 2; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_tile(S.DT + 16 * ti * ROWS, ROWS, S.XT + 16 * tj * ROWS, ROWS, ROWS, acc);
            const int c = 16 * tj + col;
            if (c < 24)
                for (int i = 0; i < 4; ++i) out[OW1 + (16 * ti + r0 + i) * 24 + c] = acc[i];
        }
    __syncthreads();
}

// rows r0.. of X (or the rows listed in idx) into the tile
__device__ void tile_load(TileLds &S, const uint16_t *__restrict__ X, const int32_t *__restrict__ idx, int r0, int n)
{
    const int l = __lane_id();
    const int row = r0 + l;
    uint4 *d = (uint4 *)(S.X + l * 32);
    if (row < n) {
        const int64_t src = idx ? idx[row] : row;
        const uint4 *s = (const uint4 *)(X + src * 32);
        for (int k = 0; k < 4; ++k) d[k] = s[k];
    } else {
        for (int k = 0; k < 4; ++k) d[k] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    tile_transpose_x(S);
}

__global__ void __launch_bounds__(64) k_mlp_fwd_bwd(const uint16_t *__restrict__ X, const uint8_t *__restrict__ Y,
                                                    const int32_t *__restrict__ idx, int n, float inv_n,
                                                    const uint16_t *__restrict__ q, const float *__restrict__ w,
                                                    float *__restrict__ partial)
{
    __shared__ TileLds S;
    __shared__ uint8_t ys[ROWS];
    const int tile = blockIdx.x, r0 = tile * ROWS, l = __lane_id();
    tile_load(S, X, idx, r0, n);
    const int row = r0 + l;
    ys[l] = row < n ? Y[idx ? idx[row] : row] : 0;
    __syncthreads();
    tile_forward<TileLds, true>(S, q, w);
    tile_backward(S, q, ys, min(ROWS, n - r0), inv_n, partial + (int64_t)tile * (NP + 1));
}

// fixed-order sum of the tile partials (gradient and loss)
__global__ void k_mlp_reduce(const float *__restrict__ partial, int tiles, float *__restrict__ grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > NP) return;
    float s = 0.0f;
    for (int t = 0; t < tiles; ++t) s += partial[(int64_t)t * (NP + 1) + k];
    grad[k] = s;
}

__global__ void k_mlp_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ grad, float lr, float c1, float c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NP) return;
    const float g = grad[k];
    const float mk = 0.9f * m[k] + 0.1f * g;
    const float vk = 0.999f * v[k] + 0.001f * g * g;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
}

// rows of minibatch `step` of `epoch`: uniform with replacement (Philox key
// (seed, 6), counter (epoch, step, j, 0))
__global__ void k_mlp_rows(int32_t *__restrict__ rows, int nb, int n_rows, uint64_t seed, int epoch, int step)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const U4 u = philox((uint64_t)epoch, (uint64_t)step, (uint64_t)j, 0, seed, TAG_MLP_BATCH);
    rows[j] = (int32_t)uniform_int(u.x[0], (uint64_t)n_rows);
}

__global__ void __launch_bounds__(64) k_mlp_logits(const uint16_t *__restrict__ X, int n,
                                                   const uint16_t *__restrict__ q, const float *__restrict__ w,
                                                   float *__restrict__ z)
{
    __shared__ InTile S;
    const int r0 = blockIdx.x * ROWS, l = __lane_id();
    uint4 *d = (uint4 *)(S.X + l * 32);
    if (r0 + l < n) {
        const uint4 *src = (const uint4 *)(X + (int64_t)(r0 + l) * 32);
        for (int k = 0; k < 4; ++k) d[k] = src[k];
    } else {
        for (int k = 0; k < 4; ++k) d[k] = make_uint4(0, 0, 0, 0);
    }
    stage_head(S, q, w);
    __syncthreads();
    const float zl = tile_forward_regs(S, q, w);
    if (r0 + l < n) z[r0 + l] = zl;
}

// ---------------------------------------------------------------------------
// per-pixel inputs, labels, verification
// ---------------------------------------------------------------------------

__global__ void k_pixel_features(FeatArgs A, const int32_t *__restrict__ pix, int n, uint16_t *__restrict__ X,
                                 float *__restrict__ XF)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int p = pix[i];
    float x[24];
    if (p >= 0 && p < A.fr.W * A.fr.H) pixel_features(A, p, x);
    else
        for (int k = 0; k < 24; ++k) x[k] = 0.0f;
    for (int k = 0; k < 32; ++k) X[(int64_t)i * 32 + k] = k < 24 ? f2bf(x[k]) : (uint16_t)0;
    if (XF)
        for (int k = 0; k < 24; ++k) XF[(int64_t)i * 24 + k] = x[k];
}

struct PoseF {
    float R[9], t[3];
};

// The probability that the pixel's hypothesis pick is correct under the
// pose: among the modes of the pixel's leaves whose colour passes the pick's
// colour test (|mode - pixel| <= rgb_tol in every channel), the fraction that
// lie within 5 cm of y = R c + t (FP32, the scoring transform), as
// round(255 good / candidates) (0 without candidates)
__global__ void k_label(FeatArgs A, PoseF P, int rgb_tol, const int32_t *__restrict__ pix, int n,
                        uint8_t *__restrict__ lab)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int p = pix[i];
    uint32_t cand = 0, good = 0;
    if (p >= 0 && p < A.fr.W * A.fr.H) {
        const uint32_t d = A.fr.depth[p];
        if (valid_depth(A.fr, d)) {
            const int u = p % A.fr.W, v = p / A.fr.W;
            float c[3];
            cam_point(A.fr, u, v, d, c);
            float y[3];
            for (int k = 0; k < 3; ++k)
                y[k] = fmaf(P.R[k * 3 + 0], c[0], fmaf(P.R[k * 3 + 1], c[1], fmaf(P.R[k * 3 + 2], c[2], P.t[k])));
            const int pr = A.fr.rgb[(int64_t)p * 3], pg = A.fr.rgb[(int64_t)p * 3 + 1], pb = A.fr.rgb[(int64_t)p * 3 + 2];
            const float lim = 0.05f * 0.05f;
            for (int t = 0; t < A.T; ++t) {
                const int32_t leaf = traverse(A.nodes + (int64_t)t * (A.L - 1), A.L, A.fr, u, v, (int32_t)d);
                const int64_t li = (int64_t)t * A.L + leaf;
                for (int m = 0; m < A.nmodes[li]; ++m) {
                    const Mode &md = A.modes[li * A.M + m];
                    const int mr = (int)(md.rgb & 255u), mg = (int)((md.rgb >> 8) & 255u), mb = (int)((md.rgb >> 16) & 255u);
                    if (abs(mr - pr) > rgb_tol || abs(mg - pg) > rgb_tol || abs(mb - pb) > rgb_tol) continue;
                    cand++;
                    const float d0 = y[0] - md.mu[0], d1 = y[1] - md.mu[1], d2 = y[2] - md.mu[2];
                    if ((d0 * d0 + d1 * d1) + d2 * d2 <= lim) good++;
                }
            }
        }
    }
    lab[i] = cand ? (uint8_t)((255u * good + cand / 2u) / cand) : (uint8_t)0;
}

// every pixel of a frame: inputs, forward, pick weight floor(sigma 65536) + 1
// for valid pixels, 0 otherwise
__global__ void __launch_bounds__(64) k_mlp_pixels(FeatArgs A, const uint16_t *__restrict__ q,
                                                   const float *__restrict__ w, uint32_t *__restrict__ weights,
                                                   float *__restrict__ prob)
{
    __shared__ InTile S;
    const int P = A.fr.W * A.fr.H;
    const int l = __lane_id();
    const int p = blockIdx.x * ROWS + l;
    float x[24];
    if (p < P) pixel_features(A, p, x);
    else
        for (int k = 0; k < 24; ++k) x[k] = 0.0f;
    store_row(S.X, x);
    stage_head(S, q, w);
    __syncthreads();
    const float zl = tile_forward_regs(S, q, w);
    if (p < P) {
        const bool ok = valid_depth(A.fr, A.fr.depth[p]);
        float sg = 0.0f;
        const uint32_t wt = pick_weight(zl, &sg);
        weights[p] = ok ? wt : 0u;
        if (prob) prob[p] = ok ? sg : 0.0f;
    }
}

static FeatArgs feat_args(const Forest *f, const Frame &fr)
{
    FeatArgs A;
    A.fr = fr;
    A.nodes = f->nodes;
    A.nmodes = f->nmodes;
    A.modes = f->modes;
    A.leaf_in = f->leaf_in;
    A.packed = nullptr;
    A.xnodes = nullptr;
    A.T = f->T; A.L = f->L; A.M = f->M; A.R = f->R;
    return A;
}

static int ensure_tiles(reloc_mlp *m, int tiles)
{
    if (tiles <= m->cap_tiles) return RELOC_OK;
    if (m->partial) (void)hipFree(m->partial);
    m->partial = nullptr;
    m->cap_tiles = 0;
    RL_HIP(hipMalloc((void **)&m->partial, (size_t)tiles * (NP + 1) * sizeof(float)));
    m->cap_tiles = tiles;
    return RELOC_OK;
}

static int ensure_rows(reloc_mlp *m, int n)
{
    if (n <= m->cap_rows) return RELOC_OK;
    if (m->rows) (void)hipFree(m->rows);
    m->rows = nullptr;
    m->cap_rows = 0;
    RL_HIP(hipMalloc((void **)&m->rows, (size_t)n * sizeof(int32_t)));
    m->cap_rows = n;
    return RELOC_OK;
}

// gradient of the mean loss over rows (idx or 0..n-1) into m->grad
static int mlp_gradient(reloc_mlp *m, const uint16_t *X, const uint8_t *Y, const int32_t *idx, int n, hipStream_t s)
{
    const int tiles = (n + ROWS - 1) / ROWS;
    int rc = ensure_tiles(m, tiles);
    if (rc) return rc;
    RL_LAUNCH("k_mlp_fwd_bwd", k_mlp_fwd_bwd, dim3(tiles), dim3(64), 0, s, X, Y, idx, n, 1.0f / (float)n, m->q, m->w,
              m->partial);
    RL_LAUNCH("k_mlp_reduce", k_mlp_reduce, dim3((NP + 1 + 255) / 256), dim3(256), 0, s, m->partial, tiles, m->grad);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

// Valid pixels of a frame (the depth test of the features and of the
// relocaliser's pool) as indices v W + u in raster order: per block of
// VP_BLOCK pixels a count, one workgroup's exclusive scan of the counts, then
// each block's indices at its offset. Each of VP_THREADS threads takes
// pixels t + j VP_THREADS of its block, so its wavefront's 64-pixel chunks
// c = j (VP_THREADS / 64) + wave run in raster order.
constexpr int VP_BLOCK = 1024, VP_THREADS = 256, VP_CH = VP_BLOCK / 64;

__global__ void __launch_bounds__(VP_THREADS) k_valid_count(Frame fr, int P, int32_t *__restrict__ cnt)
{
    __shared__ int32_t wc[VP_THREADS / 64];
    const int b = blockIdx.x, t = threadIdx.x;
    int n = 0;
    for (int j = 0; j < VP_BLOCK / VP_THREADS; ++j) {
        const int p = b * VP_BLOCK + j * VP_THREADS + t;
        n += __popcll(__ballot(p < P && valid_depth(fr, fr.depth[p])));
    }
    if (__lane_id() == 0) wc[t >> 6] = n;
    __syncthreads();
    if (t == 0) {
        int s = 0;
        for (int w = 0; w < VP_THREADS / 64; ++w) s += wc[w];
        cnt[b] = s;
    }
}

// exclusive scan of nb counts in place; the total to cnt[nb]
__global__ void __launch_bounds__(1024) k_valid_scan(int32_t *__restrict__ cnt, int nb)
{
    __shared__ int32_t ws[16];
    __shared__ int32_t carry;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const int v = i < nb ? cnt[i] : 0;
        int x = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) ws[wave] = x;
        __syncthreads();
        int off = carry;
        for (int w = 0; w < wave; ++w) off += ws[w];
        __syncthreads();
        if (i < nb) cnt[i] = off + x - v;
        if (threadIdx.x == 1023) carry = off + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[nb] = carry;
}

__global__ void __launch_bounds__(VP_THREADS) k_valid_emit(Frame fr, int P, const int32_t *__restrict__ off,
                                                           int32_t *__restrict__ pix)
{
    __shared__ int32_t wc[VP_CH];
    const int b = blockIdx.x, t = threadIdx.x, wave = t >> 6;
    constexpr int J = VP_BLOCK / VP_THREADS;
    bool ok[J];
    uint64_t m[J];
    for (int j = 0; j < J; ++j) {
        const int p = b * VP_BLOCK + j * VP_THREADS + t;
        ok[j] = p < P && valid_depth(fr, fr.depth[p]);
        m[j] = __ballot(ok[j]);
        if (__lane_id() == 0) wc[j * (VP_THREADS / 64) + wave] = __popcll(m[j]);
    }
    __syncthreads();
    for (int j = 0; j < J; ++j) {
        const int c = j * (VP_THREADS / 64) + wave;
        int o = off[b];
        for (int k = 0; k < c; ++k) o += wc[k];
        if (ok[j]) pix[o + __popcll(m[j] & ((1ull << __lane_id()) - 1ull))] = b * VP_BLOCK + j * VP_THREADS + t;
    }
}

static int mlp_pack(reloc_mlp *m, hipStream_t s)
{
    RL_LAUNCH("k_mlp_pack", k_mlp_pack, dim3(16), dim3(256), 0, s, m->w, m->q);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

}  // namespace rl

using namespace rl;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

const uint16_t *rl_mlp_q(const reloc_mlp *m) { return m->q; }
const float *rl_mlp_w(const reloc_mlp *m) { return m->w; }

static void mlp_free(reloc_mlp *m)
{
    (void)hipFree(m->w);
    (void)hipFree(m->m);
    (void)hipFree(m->v);
    (void)hipFree(m->grad);
    (void)hipFree(m->partial);
    (void)hipFree(m->q);
    (void)hipFree(m->rows);
}

extern "C" int reloc_mlp_create(uint64_t seed, void *stream, reloc_mlp **out)
{
    if (!out) return RELOC_E_ARG;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    reloc_mlp *m = new (std::nothrow) reloc_mlp();
    if (!m) return RELOC_E_NOMEM;
    if (hipMalloc((void **)&m->w, NP * 4) != hipSuccess || hipMalloc((void **)&m->m, NP * 4) != hipSuccess ||
        hipMalloc((void **)&m->v, NP * 4) != hipSuccess || hipMalloc((void **)&m->grad, (NP + 1) * 4) != hipSuccess ||
        hipMalloc((void **)&m->q, NQ * 2) != hipSuccess) {
        mlp_free(m);
        delete m;
        return RELOC_E_NOMEM;
    }
    if (hipMemsetAsync(m->m, 0, NP * 4, s) != hipSuccess || hipMemsetAsync(m->v, 0, NP * 4, s) != hipSuccess) {
        mlp_free(m);
        delete m;
        return RELOC_E_HIP;
    }
    RL_LAUNCH("k_mlp_init", k_mlp_init, dim3((NP + 255) / 256), dim3(256), 0, s, m->w, seed);
    if (mlp_pack(m, s)) {
        mlp_free(m);
        delete m;
        return RELOC_E_HIP;
    }
    *out = m;
    return RELOC_OK;
}

extern "C" int reloc_mlp_destroy(reloc_mlp *m)
{
    if (!m) return RELOC_E_ARG;
    (void)hipDeviceSynchronize();
    mlp_free(m);
    delete m;
    return RELOC_OK;
}

extern "C" int reloc_mlp_get_weights(const reloc_mlp *m, float *w_host)
{
    if (!m || !w_host) return RELOC_E_ARG;
    RL_HIP(hipDeviceSynchronize());
    RL_HIP(hipMemcpy(w_host, m->w, NP * 4, hipMemcpyDeviceToHost));
    return RELOC_OK;
}

extern "C" int reloc_mlp_set_weights(reloc_mlp *m, const float *w_host)
{
    if (!m || !w_host) return RELOC_E_ARG;
    RL_HIP(hipDeviceSynchronize());
    RL_HIP(hipMemcpy(m->w, w_host, NP * 4, hipMemcpyHostToDevice));
    int rc = mlp_pack(m, 0);
    if (rc) return rc;
    RL_HIP(hipDeviceSynchronize());
    return RELOC_OK;
}

extern "C" int reloc_mlp_gradient(reloc_mlp *m, const uint16_t *x_dev, const uint8_t *y_dev, int32_t n,
                                  float *grad_host, float *loss_host, void *stream)
{
    if (!m || !x_dev || !y_dev || n < 1 || !grad_host || ((uintptr_t)x_dev & 15)) return RELOC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    int rc = mlp_gradient(m, x_dev, y_dev, nullptr, n, s);
    if (rc) return rc;
    std::vector<float> g(NP + 1);
    RL_HIP(hipMemcpyAsync(g.data(), m->grad, (NP + 1) * 4, hipMemcpyDeviceToHost, s));
    RL_HIP(hipStreamSynchronize(s));
    memcpy(grad_host, g.data(), NP * 4);
    if (loss_host) *loss_host = g[NP] / (float)n;
    return RELOC_OK;
}

extern "C" int reloc_mlp_train(reloc_mlp *m, const uint16_t *x_dev, const uint8_t *y_dev, int32_t n_rows,
                               int32_t epochs, int32_t batch_rows, float lr, uint64_t seed, float *epoch_loss_host,
                               void *stream)
{
    if (!m || !x_dev || !y_dev || n_rows < 1 || epochs < 0 || batch_rows < 1 || !(lr > 0.0f) ||
        ((uintptr_t)x_dev & 15))
        return RELOC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_rows(m, batch_rows);
    if (rc) return rc;
    const int steps = std::max(1, n_rows / batch_rows);
    std::vector<float> g(NP + 1);
    for (int e = 0; e < epochs; ++e) {
        double loss = 0.0;
        for (int st = 0; st < steps; ++st) {
            RL_LAUNCH("k_mlp_rows", k_mlp_rows, dim3((batch_rows + 255) / 256), dim3(256), 0, s, m->rows, batch_rows,
                      n_rows, seed, e, st);
            rc = mlp_gradient(m, x_dev, y_dev, m->rows, batch_rows, s);
            if (rc) return rc;
            m->step++;
            const float c1 = 1.0f - powf(0.9f, (float)m->step), c2 = 1.0f - powf(0.999f, (float)m->step);
            RL_LAUNCH("k_mlp_adam", k_mlp_adam, dim3((NP + 255) / 256), dim3(256), 0, s, m->w, m->m, m->v, m->grad, lr,
                      c1, c2);
            rc = mlp_pack(m, s);
            if (rc) return rc;
            if (epoch_loss_host && st == steps - 1) {
                RL_HIP(hipMemcpyAsync(g.data(), m->grad, (NP + 1) * 4, hipMemcpyDeviceToHost, s));
                RL_HIP(hipStreamSynchronize(s));
                loss = g[NP] / (double)batch_rows;
            }
        }
        if (epoch_loss_host) epoch_loss_host[e] = (float)loss;
    }
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

extern "C" int reloc_mlp_logits(reloc_mlp *m, const uint16_t *x_dev, int32_t n, float *z_dev, void *stream)
{
    if (!m || !x_dev || !z_dev || n < 1 || ((uintptr_t)x_dev & 15)) return RELOC_E_ARG;
    RL_LAUNCH("k_mlp_logits", k_mlp_logits, dim3((n + ROWS - 1) / ROWS), dim3(64), 0, (hipStream_t)stream, x_dev, n,
              m->q, m->w, z_dev);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

extern "C" int reloc_mlp_pixel_weights(reloc_mlp *m, reloc_forest *f, const uint16_t *depth_dev,
                                       const uint8_t *rgb_dev, const reloc_intrinsics *K, uint32_t *weights_dev,
                                       float *prob_dev, void *stream)
{
    if (!m || !f || !weights_dev) return RELOC_E_ARG;
    Frame fr;
    int rc = frame_from(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = update_modes(f, s);
    if (rc) return rc;
    const int P = fr.W * fr.H;
    RL_LAUNCH("k_mlp_pixels", k_mlp_pixels, dim3((P + ROWS - 1) / ROWS), dim3(64), 0, s, feat_args(f, fr), m->q, m->w,
              weights_dev, prob_dev);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

extern "C" int reloc_pixel_features(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                    const reloc_intrinsics *K, const int32_t *pix_dev, int32_t n, uint16_t *x_dev,
                                    float *xf_dev, void *stream)
{
    if (!f || n < 0 || (n > 0 && (!pix_dev || !x_dev))) return RELOC_E_ARG;
    Frame fr;
    int rc = frame_from(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = update_modes(f, s);
    if (rc) return rc;
    if (n == 0) return RELOC_OK;
    RL_LAUNCH("k_pixel_features", k_pixel_features, dim3((n + 127) / 128), dim3(128), 0, s, feat_args(f, fr), pix_dev,
              n, x_dev, xf_dev);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

extern "C" int reloc_valid_pixels(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                  const reloc_intrinsics *K, int32_t *pix_dev, int32_t *n_out, void *stream)
{
    if (!f || !pix_dev || !n_out) return RELOC_E_ARG;
    Frame fr;
    int rc = frame_from(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int P = fr.W * fr.H, nb = (P + VP_BLOCK - 1) / VP_BLOCK;
    int32_t *cnt = nullptr;
    if (hipMalloc((void **)&cnt, (size_t)(nb + 1) * 4) != hipSuccess) return RELOC_E_NOMEM;
    RL_LAUNCH("k_valid_count", k_valid_count, dim3(nb), dim3(VP_THREADS), 0, s, fr, P, cnt);
    RL_LAUNCH("k_valid_scan", k_valid_scan, dim3(1), dim3(1024), 0, s, cnt, nb);
    RL_LAUNCH("k_valid_emit", k_valid_emit, dim3(nb), dim3(VP_THREADS), 0, s, fr, P, cnt, pix_dev);
    int32_t n = 0;
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&n, cnt + nb, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        rc = RELOC_E_HIP;
    (void)hipFree(cnt);
    if (rc) return rc;
    *n_out = n;
    return RELOC_OK;
}

extern "C" int reloc_label_pixels(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                  const reloc_intrinsics *K, const double pose_c2w[16], const int32_t *pix_dev,
                                  int32_t n, uint8_t *label_dev, void *stream)
{
    if (!f || !pose_c2w || n < 0 || (n > 0 && (!pix_dev || !label_dev))) return RELOC_E_ARG;
    Frame fr;
    int rc = frame_from(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = update_modes(f, s);
    if (rc) return rc;
    if (n == 0) return RELOC_OK;
    PoseF P;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) P.R[r * 3 + c] = (float)pose_c2w[r * 4 + c];
        P.t[r] = (float)pose_c2w[r * 4 + 3];
    }
    RL_LAUNCH("k_label", k_label, dim3((n + 127) / 128), dim3(128), 0, s, feat_args(f, fr), P, f->p.rgb_tol, pix_dev,
              n, label_dev);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}


__global__ void k_bf16_probe(const float *__restrict__ x, int n, uint16_t *__restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * i + 1 < n) {
        const uint32_t p = bf16_pair(x[2 * i], x[2 * i + 1]);
        y[2 * i] = (uint16_t)(p & 0xFFFFu);
        y[2 * i + 1] = (uint16_t)(p >> 16);
    } else if (2 * i < n) {
        y[2 * i] = (uint16_t)(bf16_pair(x[2 * i], 0.0f) & 0xFFFFu);
    }
}

extern "C" int reloc_debug_bf16(const float *x_host, int32_t n, uint16_t *y_host)
{
    if (n < 0 || (n > 0 && (!x_host || !y_host))) return RELOC_E_ARG;
    if (n == 0) return RELOC_OK;
    float *x = nullptr;
    uint16_t *y = nullptr;
    if (hipMalloc((void **)&x, (size_t)n * 4) != hipSuccess) return RELOC_E_NOMEM;
    if (hipMalloc((void **)&y, (size_t)n * 2) != hipSuccess) {
        (void)hipFree(x);
        return RELOC_E_NOMEM;
    }
    int rc = RELOC_OK;
    if (hipMemcpy(x, x_host, (size_t)n * 4, hipMemcpyHostToDevice) != hipSuccess) rc = RELOC_E_HIP;
    if (!rc) {
        const int pairs = (n + 1) / 2;
        hipLaunchKernelGGL(k_bf16_probe, dim3((pairs + 255) / 256), dim3(256), 0, 0, x, n, y);
        if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(y_host, y, (size_t)n * 2, hipMemcpyDeviceToHost) != hipSuccess)
            rc = RELOC_E_HIP;
    }
    (void)hipFree(x);
    (void)hipFree(y);
    return rc;
}

extern "C" int reloc_debug_mfma_probe(const uint16_t *a_host, const uint16_t *bt_host, float *c_host)
{
    if (!a_host || !bt_host || !c_host) return RELOC_E_ARG;
    uint16_t *a = nullptr, *b = nullptr;
    float *c = nullptr;
    if (hipMalloc((void **)&a, 16 * 32 * 2) != hipSuccess) return RELOC_E_NOMEM;
    if (hipMalloc((void **)&b, 16 * 32 * 2) != hipSuccess || hipMalloc((void **)&c, 256 * 4) != hipSuccess) {
        (void)hipFree(a);
        (void)hipFree(b);
        return RELOC_E_NOMEM;
    }
    int rc = RELOC_OK;
    if (hipMemcpy(a, a_host, 16 * 32 * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b, bt_host, 16 * 32 * 2, hipMemcpyHostToDevice) != hipSuccess)
        rc = RELOC_E_HIP;
    if (!rc) {
        hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, 0, a, b, c);
        if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(c_host, c, 256 * 4, hipMemcpyDeviceToHost) != hipSuccess)
            rc = RELOC_E_HIP;
    }
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(c);
    return rc;
}
