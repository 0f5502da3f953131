// Device code of the learned proposal shared by the MLP kernels and the
// relocalisation graph: bfloat16 helpers, the 16x16x32 matrix-core tile, the
// forward pass of a 64-row tile, and the 24 per-pixel inputs.
#pragma once

#include "common.h"

namespace rl {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// parameters (FP32): W1 [64][24], b1 [64], W2 [64][64], b2 [64], w3 [64], b3
constexpr int NP = 5825;
constexpr int OW1 = 0, OB1 = 1536, OW2 = 1600, OB2 = 5696, OW3 = 5760, OB3 = 5824;
// bfloat16 copies: W1 padded to [64][32], W2 [64][64], W2^T [64][64], w3 [64]
constexpr int QW1 = 0, QW2 = 2048, QW2T = 2048 + 4096, QW3 = 2048 + 8192, NQ = 2048 + 8192 + 64;
constexpr uint64_t TAG_MLP_INIT = 5, TAG_MLP_BATCH = 6;
constexpr int ROWS = 64;         // rows per wavefront tile

// round to nearest even; NaN stays a quiet NaN
__device__ __forceinline__ uint16_t f2bf(float x)
{
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u) {
        uint16_t h = (uint16_t)(b >> 16);
        if ((b & 0x007FFFFFu) && !(h & 0x7F)) h |= 0x40;
        return h;
    }
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// two floats to a bfloat16 pair (lo in bits 0-15) by the conversion
// instruction, which rounds to nearest even like f2bf
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi)
{
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    const uint4 v = *(const uint4 *)p;
    return __builtin_bit_cast(bf16x8, v);
}

// 16x16 tile of A (16 rows, K-contiguous, stride lda) times B given as B^T
// (16 columns, K-contiguous, stride ldb), K a multiple of 32, accumulated into
// acc. Lane l supplies row / column (l & 15) and the k-block 8 (l >> 4) .. +7;
// the result holds column (l & 15), rows 4 (l >> 4) + i, i < 4.
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

// LDS of an inference tile: the rows' inputs (the activations stay in
// registers, tile_forward_regs)
struct __align__(16) InTile {
    uint16_t X[ROWS * 32];
    float b1[64], b2[64], w3[64];   // biases and output weights (w3 from its bfloat16 copy)
};

// the tile's copy of the network's biases and output weights (every thread
// of the workgroup takes part; a barrier must follow before they are read)
__device__ __forceinline__ void stage_head(InTile &S, const uint16_t *__restrict__ q, const float *__restrict__ w)
{
    for (int k = threadIdx.x; k < 64; k += blockDim.x) {
        S.b1[k] = w[OB1 + k];
        S.b2[k] = w[OB2 + k];
        S.w3[k] = bf2f(q[QW3 + k]);
    }
}

// Forward pass of the 64 rows in S.X (bfloat16, 24 inputs + 8 zeros): H1, H2
// in bfloat16, logits in S.z. With kTrans the tile also keeps H1 transposed
// (for the weight gradient of layer 2).
template <class Tile, bool kTrans>
__device__ void tile_forward(Tile &S, const uint16_t *__restrict__ q, const float *__restrict__ w)
{
    const int l = __lane_id(), col = l & 15, r0 = (l >> 4) * 4;
    // layer 1: H1 = relu(X W1^T + b1), stored bfloat16
#pragma unroll 1
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
                if constexpr (kTrans) S.H1T[c * ROWS + row] = h;
            }
        }
    __syncthreads();
    // layer 2: H2 = relu(H1 W2^T + b2)
#pragma unroll 1
    for (int ti = 0; ti < 4; ++ti)
        for (int tj = 0; tj < 4; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = mfma_tile(S.H1 + 16 * ti * 64, 64, q + QW2 + 16 * tj * 64, 64, 64, acc);
            const int c = 16 * tj + col;
            const float b = w[OB2 + c];
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * ti + r0 + i;
                const float hv = acc[i] + b;
                S.H2[row * 64 + c] = hv > 0.0f ? f2bf(hv) : (uint16_t)0;
            }
        }
    __syncthreads();
    // output: z = w3 . h2 + b3 (FP32, lane = row)
    float z = 0.0f;
    for (int j = 0; j < 64; ++j) z = fmaf(bf2f(q[QW3 + j]), bf2f(S.H2[l * 64 + j]), z);
    S.z[l] = z + w[OB3];
    __syncthreads();
}

// Layer 1's A operand for hidden rows 16 tj .. + 15 as lane l supplies it:
// row 16 tj + (l & 15) of W1 (bfloat16, [64][32]), k-block 8 (l >> 4) .. + 7.
__device__ __forceinline__ bf16x8 w1_operand(const uint16_t *__restrict__ q, int tj, int l)
{
    return load8(q + QW1 + (16 * tj + (l & 15)) * 32 + 8 * (l >> 4));
}

// Layer 2's A operand for hidden rows 16 tk .. + 15 and k-chunk c as lane l
// supplies it: row 16 tk + (l & 15) of W2, k-slot s of lane group g = l >> 4
// standing for hidden unit 32 c + 16 (s >> 2) + 4 g + (s & 3)
__device__ __forceinline__ bf16x8 w2_operand(const uint16_t *__restrict__ q, int tk, int c, int l)
{
    const uint16_t *row = q + QW2 + (16 * tk + (l & 15)) * 64 + 32 * c + 4 * (l >> 4);
    const uint2 lo = *(const uint2 *)row;          // hidden 32 c + 4 g .. + 3
    const uint2 hi = *(const uint2 *)(row + 16);   // hidden 32 c + 16 + 4 g .. + 3
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

// Forward pass of a 64-row tile for inference, with the activations kept in
// registers. Row i's 32 inputs (bfloat16: 24 and 8 zeros) are X[32 i ..]
// (LDS); a1, a2 are the lane's weight operands (w1_operand, w2_operand);
// returns the logit of row `lane` without the output bias. The layers are
// computed transposed (hidden units x rows), 16 rows at a time: layer 1
// leaves lane l holding row (l & 15) and hidden units 16 tj + 4 (l >> 4) + i
// (tj, i < 4), which are the 8 + 8 k-values that layer 2's B operand needs
// from that lane for its two 32-wide k-chunks, once W2's columns are taken in
// the same order (w2_operand; an MFMA sums the same products whatever the
// slot order). H1 and H2 are rounded to bfloat16 (nearest even, by the
// conversion instruction) after bias and ReLU as in tile_forward; the output
// dot w3 . h2 is summed per lane over its 16 hidden units, then over the four
// lane groups.
__device__ __forceinline__ float tile_forward_core(const uint16_t *X, const bf16x8 a1[4], const bf16x8 a2[4][2],
                                                   const float *b1, const float *b2, const float *w3)
{
    const int l = __lane_id(), col = l & 15, g = l >> 4;
    float zrow = 0.0f;
#pragma unroll 1
    for (int ti = 0; ti < 4; ++ti) {
        const bf16x8 xb = load8(X + (16 * ti + col) * 32 + 8 * g);
        uint32_t h1[8];   // bfloat16 pairs: h1 unit 16 tj + 4 g + i at half 4 tj + i
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[tj], xb, acc, 0, 0, 0);
            const float4 bb = *(const float4 *)(b1 + 16 * tj + 4 * g);
            float hv[4] = {acc[0] + bb.x, acc[1] + bb.y, acc[2] + bb.z, acc[3] + bb.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) hv[i] = hv[i] > 0.0f ? hv[i] : 0.0f;
            h1[2 * tj] = bf16_pair(hv[0], hv[1]);
            h1[2 * tj + 1] = bf16_pair(hv[2], hv[3]);
        }
        const bf16x8 b2lo = __builtin_bit_cast(bf16x8, make_uint4(h1[0], h1[1], h1[2], h1[3]));
        const bf16x8 b2hi = __builtin_bit_cast(bf16x8, make_uint4(h1[4], h1[5], h1[6], h1[7]));
        float z = 0.0f;
#pragma unroll
        for (int tk = 0; tk < 4; ++tk) {
            floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[tk][0], b2lo, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[tk][1], b2hi, acc, 0, 0, 0);
            const float4 bb = *(const float4 *)(b2 + 16 * tk + 4 * g);
            float hv[4] = {acc[0] + bb.x, acc[1] + bb.y, acc[2] + bb.z, acc[3] + bb.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) hv[i] = hv[i] > 0.0f ? hv[i] : 0.0f;
            const uint32_t p01 = bf16_pair(hv[0], hv[1]), p23 = bf16_pair(hv[2], hv[3]);
            const float h2[4] = {__uint_as_float(p01 << 16), __uint_as_float(p01 & 0xFFFF0000u),
                                 __uint_as_float(p23 << 16), __uint_as_float(p23 & 0xFFFF0000u)};
            const float4 ww = *(const float4 *)(w3 + 16 * tk + 4 * g);
            z = fmaf(ww.x, h2[0], z);
            z = fmaf(ww.y, h2[1], z);
            z = fmaf(ww.z, h2[2], z);
            z = fmaf(ww.w, h2[3], z);
        }
        z = z + __shfl_xor(z, 16, 64);
        z = z + __shfl_xor(z, 32, 64);
        if (ti == g) zrow = z;   // lane 16 g + col is row 16 ti + col
    }
    return zrow;
}

// tile_forward_core with the weight operands loaded from the network's
// bfloat16 copy and the head from S
__device__ __forceinline__ float tile_forward_regs(const InTile &S, const uint16_t *__restrict__ q,
                                                   const float *__restrict__ w)
{
    const int l = __lane_id();
    bf16x8 a1[4], a2[4][2];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) a1[tj] = w1_operand(q, tj, l);
#pragma unroll
    for (int tk = 0; tk < 4; ++tk)
#pragma unroll
        for (int c = 0; c < 2; ++c) a2[tk][c] = w2_operand(q, tk, c, l);
    return tile_forward_core(S.X, a1, a2, S.b1, S.b2, S.w3) + w[OB3];
}

// The network as inference tiles read it, staged once per workgroup in LDS:
// every lane's weight operands (w1_operand, w2_operand) in lane order, the
// biases, the output weights (from their bfloat16 copy) and the output bias.
struct __align__(16) WTile {
    bf16x8 a1[4][64];
    bf16x8 a2[4][2][64];
    float b1[64], b2[64], w3[64];
    float b3;
};

// every thread of the workgroup takes part; a barrier must follow
__device__ __forceinline__ void stage_weights(WTile &W, const uint16_t *__restrict__ q, const float *__restrict__ w)
{
    for (int k = threadIdx.x; k < 4 * 64; k += blockDim.x) W.a1[k >> 6][k & 63] = w1_operand(q, k >> 6, k & 63);
    for (int k = threadIdx.x; k < 8 * 64; k += blockDim.x)
        W.a2[k >> 7][(k >> 6) & 1][k & 63] = w2_operand(q, k >> 7, (k >> 6) & 1, k & 63);
    for (int k = threadIdx.x; k < 64; k += blockDim.x) {
        W.b1[k] = w[OB1 + k];
        W.b2[k] = w[OB2 + k];
        W.w3[k] = bf2f(q[QW3 + k]);
    }
    if (threadIdx.x == 0) W.b3 = w[OB3];
}

// tile_forward_regs with the weights from a staged WTile (the same operands,
// so the same logits)
__device__ __forceinline__ float tile_forward_staged(const uint16_t *X, const WTile &W)
{
    const int l = __lane_id();
    bf16x8 a1[4], a2[4][2];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) a1[tj] = W.a1[tj][l];
#pragma unroll
    for (int tk = 0; tk < 4; ++tk)
#pragma unroll
        for (int c = 0; c < 2; ++c) a2[tk][c] = W.a2[tk][c][l];
    return tile_forward_core(X, a1, a2, W.b1, W.b2, W.w3) + W.b3;
}

// what the per-pixel inputs need from a forest and a frame
struct FeatArgs {
    Frame fr;
    const uint64_t *nodes;       // [T][L-1] then 8 extra
    const int32_t *nmodes;
    const Mode *modes;
    const float4 *leaf_in;       // [T][L][4] per-leaf summaries written with the modes
    const uint64_t *packed;      // the frame packed for probes, or null (probes read the frame)
    const ProbeNode *xnodes;     // the 8 extra nodes prepared for the frame (with packed), or null
    int T, L, M, R;
};

// The 24 inputs of valid pixel (u, v) with depth d, FP32: depth / 5000; the 8
// extra responses (depth clamped to +-5000 mm over 1000, colour over 255);
// pi = n / min(k, R) and -log(Sigma^-1_ii) / 10 of the 3 heaviest modes of the
// pixel's leaves (ties: lower (tree, mode)); mean reservoir fill; u / W,
// v / H. leaf_of(t) gives the pixel's leaf in tree t. A leaf's modes are
// ranked by size, so its pi never increase with the mode index and only its
// first three modes can be among the three heaviest; their values come from
// the leaf's summary, computed with the same operations when the modes are
// built.
template <class LeafOf>
__device__ __forceinline__ void pixel_inputs(const FeatArgs &A, int u, int v, uint32_t d, LeafOf leaf_of,
                                             float x[24])
{
    for (int k = 0; k < 24; ++k) x[k] = 0.0f;
    x[0] = (float)d / 5000.0f;
    const PixelDen pd = pixel_den(A.fr, (int32_t)d);
    const uint64_t *extra = A.nodes + (int64_t)A.T * (A.L - 1);
    const uint64_t own = A.packed ? A.packed[v * A.fr.W + u] : 0ull;
    if (A.packed && A.xnodes) {
        // prepared nodes: the 8 probes are independent loads issued together
        const __amdgpu_buffer_rsrc_t rs = packed_rsrc(A.packed, A.fr.W * A.fr.H);
        int32_t rr[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) rr[j] = probe_response(rs, A.fr.W, A.fr.H, u, v, own, pd, A.xnodes[j]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            int32_t r = rr[j];
            if ((A.xnodes[j].sh & 63u) == 0) {
                r = r > 5000 ? 5000 : (r < -5000 ? -5000 : r);
                x[1 + j] = (float)r / 1000.0f;
            } else {
                x[1 + j] = (float)r / 255.0f;
            }
        }
    } else {
        for (int j = 0; j < 8; ++j) {
            int32_t r;
            if (A.packed) {
                r = probe_response(packed_rsrc(A.packed, A.fr.W * A.fr.H), A.fr.W, A.fr.H, u, v, own, pd,
                                   probe_node(extra[j], A.fr));
            } else {
                int32_t thr;
                r = node_response_d(A.fr, extra[j], u, v, (int32_t)d, pd, thr);
            }
            if ((extra[j] & 3u) == 0) {
                r = r > 5000 ? 5000 : (r < -5000 ? -5000 : r);
                x[1 + j] = (float)r / 1000.0f;
            } else {
                x[1 + j] = (float)r / 255.0f;
            }
        }
    }
    // the heaviest three over the leaves' first three modes, ties to the lower
    // (tree, mode): each leaf's summary holds min(k, R), its mode count (<= 3)
    // and (pi, -log(Sigma^-1_ii) / 10) of those modes
    float4 b0 = make_float4(-1.0f, 0.0f, 0.0f, 0.0f), b1 = b0, b2 = b0;
    bool h0 = false, h1 = false, h2 = false;
    int64_t fill = 0;
    // the first 8 trees' leaf indices loaded together, ahead of the summaries
    int32_t lv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) lv[t] = t < A.T ? leaf_of(t) : 0;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        if (t >= A.T) break;
        // the whole summary at once (the mode count selects what is used)
        const float4 *S = A.leaf_in + ((int64_t)t * A.L + (t < 8 ? lv[t] : leaf_of(t))) * 4;
        const float4 head = S[0], m3[3] = {S[1], S[2], S[3]};
        fill += (int64_t)__float_as_uint(head.x);
        const int n3 = __float_as_int(head.y);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            if (m >= n3) break;
            const float4 c = m3[m];
            if (c.x > b0.x) {
                b2 = b1; h2 = h1; b1 = b0; h1 = h0; b0 = c; h0 = true;
            } else if (c.x > b1.x) {
                b2 = b1; h2 = h1; b1 = c; h1 = true;
            } else if (c.x > b2.x) {
                b2 = c; h2 = true;
            }
        }
    }
    if (h0) { x[9] = b0.x; x[10] = b0.y; x[11] = b0.z; x[12] = b0.w; }
    if (h1) { x[13] = b1.x; x[14] = b1.y; x[15] = b1.z; x[16] = b1.w; }
    if (h2) { x[17] = b2.x; x[18] = b2.y; x[19] = b2.z; x[20] = b2.w; }
    x[21] = (float)fill / (float)((int64_t)A.T * A.R);
    x[22] = (float)u / (float)A.fr.W;
    x[23] = (float)v / (float)A.fr.H;
}

// the same with the leaves found by traversal (zeros for an invalid pixel)
__device__ __forceinline__ void pixel_features(const FeatArgs &A, int p, float x[24])
{
    const uint32_t d = A.fr.depth[p];
    if (!valid_depth(A.fr, d)) {
        for (int k = 0; k < 24; ++k) x[k] = 0.0f;
        return;
    }
    const int u = p % A.fr.W, v = p / A.fr.W;
    const PixelDen pd = pixel_den(A.fr, (int32_t)d);
    pixel_inputs(A, u, v, d,
                 [&](int t) { return traverse_d(A.nodes + (int64_t)t * (A.L - 1), A.L, A.fr, u, v, (int32_t)d, pd); },
                 x);
}

// lane l's inputs as row l of a tile's inputs X (bfloat16, 8 zeros of
// padding)
__device__ __forceinline__ void store_row(uint16_t *X, const float x[24])
{
    const int l = __lane_id();
    uint4 *row = (uint4 *)(X + l * 32);
#pragma unroll
    for (int k = 0; k < 3; ++k)
        row[k] = make_uint4(bf16_pair(x[8 * k], x[8 * k + 1]), bf16_pair(x[8 * k + 2], x[8 * k + 3]),
                            bf16_pair(x[8 * k + 4], x[8 * k + 5]), bf16_pair(x[8 * k + 6], x[8 * k + 7]));
    row[3] = make_uint4(0u, 0u, 0u, 0u);
}

// pick weight of a valid pixel from its logit: floor(sigmoid(z) 65536) + 1
__device__ __forceinline__ uint32_t pick_weight(float z, float *prob)
{
    const float sg = 1.0f / (1.0f + expf(-z));
    if (prob) *prob = sg;
    return (uint32_t)floorf(sg * 65536.0f) + 1u;
}

}  // namespace rl
