// Learned proposal on the GPU: a 24-64-64-1 MLP (ReLU, ReLU, sigmoid) that
// predicts, per pixel, the probability that one of its leaf modes lies within
// 5 cm of its true world point. Its output becomes integer pick weights for
// the three pixel picks of every hypothesis try; the uniform preemptive
// scoring stays the judge.
//
// Matrix products run on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16:
// bfloat16 operands, FP32 accumulation). One wavefront owns a tile of 64 rows:
// forward (two MFMA layers and a VALU output dot), loss, and backward (the
// weight-gradient and input-gradient products are MFMA as well), all staged
// in LDS; per-wavefront gradient partials are summed in a fixed order, then
// Adam updates the FP32 master weights and refreshes their bfloat16 copies.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "common.h"

namespace rl {

int update_modes(Forest *f, hipStream_t s);
int frame_from(const Forest *f, const uint16_t *depth, const uint8_t *rgb, const reloc_intrinsics *K, Frame &fr);

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int NP = 5825;
constexpr int OW1 = 0, OB1 = 1536, OW2 = 1600, OB2 = 5696, OW3 = 5760, OB3 = 5824;
// bfloat16 copies: W1 padded to [64][32], W2 [64][64], W2^T [64][64], w3 [64]
constexpr int QW1 = 0, QW2 = 2048, QW2T = 2048 + 4096, QW3 = 2048 + 8192, NQ = 2048 + 8192 + 64;
constexpr uint64_t TAG_MLP_INIT = 5, TAG_MLP_BATCH = 6;
constexpr int ROWS = 64;         // rows per wavefront tile

struct Mlp {
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

}  // namespace rl

struct reloc_mlp : public rl::Mlp {};

namespace rl {

__host__ __device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7F800000u) == 0x7F800000u) {
        uint16_t h = (uint16_t)(b >> 16);
        if ((b & 0x007FFFFFu) && !(h & 0x7F)) h |= 0x40;
        return h;
    }
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    const uint4 v = *(const uint4 *)p;
    return __builtin_bit_cast(bf16x8, v);
}

// 16x16 tile of A (16 rows, K-contiguous, stride lda) times B given as B^T
// (16 columns, K-contiguous, stride ldb), K a multiple of 32, accumulated into
// acc. Lane l supplies row / column (l & 15) and k-block 8 (l >> 4); the
// result holds column (l & 15), rows 4 (l >> 4) + i.
__device__ __forceinline__ floatx4 mfma_tile(const uint16_t *A, int lda, const uint16_t *Bt, int ldb, int K,
                                             floatx4 acc)
{
    const int l = __lane_id(), r = l & 15, kb = (l >> 4) * 8;
    for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 a = load8(A + r * lda + k0 + kb);
        const bf16x8 b = load8(Bt + r * ldb + k0 + kb);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// ---------------------------------------------------------------------------
// initialisation and bfloat16 copies
// ---------------------------------------------------------------------------

__global__ void k_mlp_init(float *__restrict__ w, uint64_t seed)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NP) return;
    int l = -1, o = 0, fi = 0, fo = 0;
    if (k < OB1) { l = 0; o = OW1; fi = 24; fo = 64; }
    else if (k >= OW2 && k < OB2) { l = 1; o = OW2; fi = 64; fo = 64; }
    else if (k >= OW3 && k < OB3) { l = 2; o = OW3; fi = 64; fo = 1; }
    if (l < 0) {
        w[k] = 0.0f;
        return;
    }
    (void)o;
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
// forward of one 64-row tile held in LDS (sX row-major [64][32])
// ---------------------------------------------------------------------------

struct TileLds {
    uint16_t X[ROWS * 32], XT[32 * ROWS];
    uint16_t H1[ROWS * 64], H1T[64 * ROWS];
    uint16_t H2[ROWS * 64], H2T[64 * ROWS];
    uint16_t Db[ROWS * 64], DT[64 * ROWS];
    float D[ROWS * 65];
    float z[ROWS], dz[ROWS];
};

__device__ void tile_forward(TileLds &S, const uint16_t *__restrict__ q, const float *__restrict__ w)
{
    const int l = __lane_id(), col = l & 15, r0 = (l >> 4) * 4;
    // layer 1: H1 = relu(X W1^T + b1)
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 4; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_tile(S.X + 16 * ti * 32, 32, q + QW1 + 16 * tj * 32, 32, 32, acc);
            const int c = 16 * tj + col;
            const float b = w[OB1 + c];
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * ti + r0 + i;
                const float hv = acc[i] + b;
                const uint16_t h = hv > 0.0f ? f2bf(hv) : (uint16_t)0;
                S.H1[row * 64 + c] = h;
                S.H1T[c * ROWS + row] = h;
            }
        }
    __syncthreads();
    // layer 2: H2 = relu(H1 W2^T + b2)
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 4; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_tile(S.H1 + 16 * ti * 64, 64, q + QW2 + 16 * tj * 64, 64, 64, acc);
            const int c = 16 * tj + col;
            const float b = w[OB2 + c];
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * ti + r0 + i;
                const float hv = acc[i] + b;
                const uint16_t h = hv > 0.0f ? f2bf(hv) : (uint16_t)0;
                S.H2[row * 64 + c] = h;
                S.H2T[c * ROWS + row] = h;
            }
        }
    __syncthreads();
    // output: z = w3 . h2 + b3 (FP32, lane = row)
    float z = 0.0f;
    for (int j = 0; j < 64; ++j) z = fmaf(bf2f(q[QW3 + j]), bf2f(S.H2T[j * ROWS + l]), z);
    S.z[l] = z + w[OB3];
    __syncthreads();
}

// backward of the tile: gradient partials (NP values) and the loss sum of the
// valid rows into `out`; dz = (sigmoid(z) - y) * inv_n
__device__ void tile_backward(TileLds &S, const uint16_t *__restrict__ q, const uint8_t *yrow, int nvalid,
                              float inv_n, float *__restrict__ out)
{
    const int l = __lane_id(), col = l & 15, r0 = (l >> 4) * 4;
    {
        const float z = S.z[l];
        float dz = 0.0f, loss = 0.0f;
        if (l < nvalid) {
            const float y = yrow[l] ? 1.0f : 0.0f;
            dz = (1.0f / (1.0f + expf(-z)) - y) * inv_n;
            loss = fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
        }
        S.dz[l] = dz;
        // loss of the tile: wave sum in lane order
        for (int o = 32; o >= 1; o >>= 1) loss += __shfl_xor(loss, o, 64);
        if (l == 0) out[NP] = loss;
    }
    __syncthreads();
    // dw3[j] = sum_rows dz h2, db3 = sum dz (lane = j)
    {
        float g = 0.0f;
        for (int row = 0; row < ROWS; ++row) g = fmaf(S.dz[row], bf2f(S.H2[row * 64 + l]), g);
        out[OW3 + l] = g;
        float b = 0.0f;
        for (int row = 0; row < ROWS; ++row) b += S.dz[row];
        if (l == 0) out[OB3] = b;
    }
    // dH2 = dz w3 [h2 > 0]
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 4; ++tj) {
            const int c = 16 * tj + col;
            const float w3 = bf2f(q[QW3 + c]);
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * ti + r0 + i;
                const float d = S.H2[row * 64 + c] ? S.dz[row] * w3 : 0.0f;
                S.D[row * 65 + c] = d;
                const uint16_t h = f2bf(d);
                S.Db[row * 64 + c] = h;
                S.DT[c * ROWS + row] = h;
            }
        }
    __syncthreads();
    {   // db2 (lane = output unit)
        float b = 0.0f;
        for (int row = 0; row < ROWS; ++row) b += S.D[row * 65 + l];
        out[OB2 + l] = b;
    }
    // dW2 = dH2^T H1
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 4; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_tile(S.DT + 16 * ti * ROWS, ROWS, S.H1T + 16 * tj * ROWS, ROWS, ROWS, acc);
            for (int i = 0; i < 4; ++i) out[OW2 + (16 * ti + r0 + i) * 64 + 16 * tj + col] = acc[i];
        }
    __syncthreads();
    // dH1 = dH2 W2 [h1 > 0]
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 4; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_tile(S.Db + 16 * ti * 64, 64, q + QW2T + 16 * tj * 64, 64, 64, acc);
            const int c = 16 * tj + col;
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * ti + r0 + i;
                const float d = S.H1[row * 64 + c] ? acc[i] : 0.0f;
                S.D[row * 65 + c] = d;
                S.DT[c * ROWS + row] = f2bf(d);
            }
        }
    __syncthreads();
    {   // db1
        float b = 0.0f;
        for (int row = 0; row < ROWS; ++row) b += S.D[row * 65 + l];
        out[OB1 + l] = b;
    }
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

// loads rows (row indices, or r0 + t when idx is null) into the tile
__device__ void tile_load(TileLds &S, const uint16_t *__restrict__ X, const int32_t *__restrict__ idx, int r0, int n)
{
    const int l = __lane_id();
    const int row = r0 + l;
    if (row < n) {
        const int64_t src = idx ? idx[row] : row;
        const uint4 *s = (const uint4 *)(X + src * 32);
        uint4 *d = (uint4 *)(S.X + l * 32);
        for (int k = 0; k < 4; ++k) d[k] = s[k];
    } else {
        uint4 *d = (uint4 *)(S.X + l * 32);
        for (int k = 0; k < 4; ++k) d[k] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k) S.XT[k * ROWS + l] = S.X[l * 32 + k];
    __syncthreads();
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
    tile_forward(S, q, w);
    tile_backward(S, q, ys, min(ROWS, n - r0), inv_n, partial + (int64_t)tile * (NP + 1));
}

// fixed-order sum of the tile partials
__global__ void k_mlp_reduce(const float *__restrict__ partial, int tiles, float *__restrict__ grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > NP) return;
    float s = 0.0f;
    for (int t = 0; t < tiles; ++t) s += partial[(int64_t)t * (NP + 1) + k];
    grad[k] = s;
}

__global__ void k_mlp_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ grad, float lr, float c1, float c2, int clear)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NP) return;
    if (clear) {
        m[k] = 0.0f;
        v[k] = 0.0f;
        return;
    }
    const float g = grad[k];
    const float mk = 0.9f * m[k] + 0.1f * g;
    const float vk = 0.999f * v[k] + 0.001f * g * g;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
}

// minibatch rows of step s: uniform with replacement from Philox
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
    __shared__ TileLds S;
    const int r0 = blockIdx.x * ROWS, l = __lane_id();
    tile_load(S, X, nullptr, r0, n);
    tile_forward(S, q, w);
    if (r0 + l < n) z[r0 + l] = S.z[l];
}

// ---------------------------------------------------------------------------
// per-pixel features (the MLP input)
// ---------------------------------------------------------------------------

struct FeatArgs {
    Frame fr;
    const uint64_t *nodes;       // [T][L-1] then 8 extra
    const int32_t *nmodes;
    const Mode *modes;
    const uint32_t *counter;
    int T, L, M, R;
};

// The 24 inputs of one valid pixel, FP32, in the order and with the scales
// documented in the oracle (depth / 5000; the 8 extra responses; pi and
// -log(Sigma^-1_ii) / 10 of the 3 heaviest modes; mean reservoir fill; u / W,
// v / H).
__device__ void pixel_features(const FeatArgs &A, int p, float x[24])
{
    for (int k = 0; k < 24; ++k) x[k] = 0.0f;
    const uint32_t d = A.fr.depth[p];
    if (!valid_depth(A.fr, d)) return;
    const int u = p % A.fr.W, v = p / A.fr.W;
    x[0] = (float)d / 5000.0f;
    const uint64_t *extra = A.nodes + (int64_t)A.T * (A.L - 1);
    for (int j = 0; j < 8; ++j) {
        int32_t thr;
        int32_t r = node_response(A.fr, extra[j], u, v, (int32_t)d, thr);
        if ((extra[j] & 3u) == 0) {
            r = r > 5000 ? 5000 : (r < -5000 ? -5000 : r);
            x[1 + j] = (float)r / 1000.0f;
        } else {
            x[1 + j] = (float)r / 255.0f;
        }
    }
    float best_pi[3] = {-1.0f, -1.0f, -1.0f};
    int64_t best_m[3] = {-1, -1, -1};
    int64_t fill = 0;
    for (int t = 0; t < A.T; ++t) {
        const int32_t leaf = traverse(A.nodes + (int64_t)t * (A.L - 1), A.L, A.fr, u, v, (int32_t)d);
        const int64_t li = (int64_t)t * A.L + leaf;
        const uint32_t k = A.counter[li];
        const uint32_t cap = k < (uint32_t)A.R ? k : (uint32_t)A.R;
        fill += cap;
        const int nm = A.nmodes[li];
        for (int m = 0; m < nm; ++m) {
            const float pi = (float)A.modes[li * A.M + m].n / (float)cap;
            for (int s = 0; s < 3; ++s)
                if (pi > best_pi[s]) {
                    for (int qq = 2; qq > s; --qq) {
                        best_pi[qq] = best_pi[qq - 1];
                        best_m[qq] = best_m[qq - 1];
                    }
                    best_pi[s] = pi;
                    best_m[s] = li * A.M + m;
                    break;
                }
        }
    }
    for (int s = 0; s < 3; ++s) {
        if (best_m[s] < 0) continue;
        const Mode &md = A.modes[best_m[s]];
        x[9 + 4 * s] = best_pi[s];
        x[10 + 4 * s] = -logf(md.sinv[0]) / 10.0f;
        x[11 + 4 * s] = -logf(md.sinv[3]) / 10.0f;
        x[12 + 4 * s] = -logf(md.sinv[5]) / 10.0f;
    }
    x[21] = (float)fill / (float)((int64_t)A.T * A.R);
    x[22] = (float)u / (float)A.fr.W;
    x[23] = (float)v / (float)A.fr.H;
}

__global__ void k_pixel_features(FeatArgs A, const int32_t *__restrict__ pix, int n, uint16_t *__restrict__ X,
                                 float *__restrict__ XF)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[24];
    pixel_features(A, pix[i], x);
    for (int k = 0; k < 32; ++k) X[(int64_t)i * 32 + k] = k < 24 ? f2bf(x[k]) : (uint16_t)0;
    if (XF)
        for (int k = 0; k < 24; ++k) XF[(int64_t)i * 24 + k] = x[k];
}

// inlier labels of listed pixels under a pose (FP32, the scoring transform)
__global__ void k_label(FeatArgs A, Pose32Args pose, const int32_t *__restrict__ pix, int n, uint8_t *__restrict__ lab);

// every pixel of a frame: features, forward, pick weight floor(sigma 65536) + 1
// for valid pixels, 0 otherwise
__global__ void __launch_bounds__(64) k_mlp_pixels(FeatArgs A, const uint16_t *__restrict__ q,
                                                   const float *__restrict__ w, uint32_t *__restrict__ weights,
                                                   float *__restrict__ prob)
{
    __shared__ TileLds S;
    const int P = A.fr.W * A.fr.H;
    const int l = __lane_id();
    const int p = blockIdx.x * ROWS + l;
    float x[24];
    if (p < P) pixel_features(A, p, x);
    else
        for (int k = 0; k < 24; ++k) x[k] = 0.0f;
    for (int k = 0; k < 32; ++k) S.X[l * 32 + k] = k < 24 ? f2bf(x[k]) : (uint16_t)0;
    __syncthreads();
    for (int k = 0; k < 32; ++k) S.XT[k * ROWS + l] = S.X[l * 32 + k];
    __syncthreads();
    tile_forward(S, q, w);
    if (p < P) {
        const bool ok = valid_depth(A.fr, A.fr.depth[p]);
        const float sg = 1.0f / (1.0f + expf(-S.z[l]));
        weights[p] = ok ? (uint32_t)floorf(sg * 65536.0f) + 1u : 0u;
        if (prob) prob[p] = ok ? sg : 0.0f;
    }
}

}  // namespace rl
