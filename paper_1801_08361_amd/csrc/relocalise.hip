// Relocalisation on the GPU: query pool, three-point Kabsch hypotheses,
// preemptive scoring with halving culls and inlier refinement, for a ragged
// batch of attempts (the plain call is a batch of one).
//
// Every stage is a persistent kernel over the stage's work units; attempt a
// owns units [off[a], off[a+1]) (frame blocks, hypotheses, (hypothesis block,
// draw chunk) pairs, survivors). A whole batch is one captured HIP graph.
// Layout of the work inside an attempt:
//  - hypotheses: one wavefront per hypothesis, one lane per try; the first
//    passing try (lowest lane, then lowest chunk of 64 tries) defines it; the
//    same launch stages every round's draws (pixel, camera point, each tree's
//    leaf modes), one lane per draw;
//  - scoring: a workgroup holds 64 live hypotheses (one per lane) and a chunk
//    of draws spread over its wavefronts; each wavefront takes its draw,
//    stages the draw's modes once in LDS and reads them back as broadcasts
//    while every lane evaluates its own pose; energies are summed per group
//    of 8 draws in draw order and the group sums go to memory;
//  - cull: the group sums are added in group order and the live hypotheses
//    ordered by (energy, index); the first half, rounded up, survives. Rounds
//    of at most 1024 live hypotheses (in batches needing few workgroups) rank
//    each key by counting the smaller ones, a workgroup per 64 keys; other
//    rounds sort the keys in LDS, one workgroup per attempt;
//  - refinement: one wavefront per survivor sums its inliers of the round
//    (lanes over draws, xor butterfly) into its running sums and the pose is
//    re-aligned from them (Horn's method, FP64), by lane 0 of that wavefront
//    in small rounds or by one lane per survivor in a second kernel in large
//    ones.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "mlp_dev.h"

namespace rl {

int update_modes(Forest *f, hipStream_t s);
int frame_from(const Forest *f, const uint16_t *depth, const uint8_t *rgb, const reloc_intrinsics *K, Frame &fr);

constexpr int PIX_BLOCK = 256;
constexpr int POOL_BLOCK = 1024;
constexpr int PB_PIX = 4;   // pixels per thread in the pixel-block kernels (pack, pool write)

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

#define FOR_UNITS(S, u)                 \
    int u##0_, u##1_, u##s_;            \
    unit_range(S, u##0_, u##1_, u##s_); \
    for (int u = u##0_; u < u##1_; u += u##s_)

// Orders one wavefront's LDS writes before its later LDS reads of other
// lanes' data, and its reads before its later writes: a wavefront's LDS
// operations are performed in issue order, so only the compiler must keep
// them in place.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// round r of attempt A runs when at least one (r = 0) or more than one
// (r > 0) hypothesis is live at its start
__device__ __forceinline__ bool round_active(const Attempt &A, int r)
{
    const int na = A.rl[r];
    return r == 0 ? na >= 1 : na > 1;
}

// the live list scored in round r (buffer r & 1) and the one its cull writes
__device__ __forceinline__ int32_t *live_list(const Attempt &A, int r) { return A.alive + (int64_t)(r & 1) * A.N; }
__device__ __forceinline__ float *live_energy(const Attempt &A, int r) { return A.energy + (int64_t)(r & 1) * A.N; }

// ---------------------------------------------------------------------------
// features and traversal of every pixel
// ---------------------------------------------------------------------------

// The pool entries of pool block b for uniform picks, by the PIX_BLOCK
// threads of a traversal workgroup (thread tid holds pixels
// b POOL_BLOCK + j PIX_BLOCK + tid, j < 4, valid where ok[j]): each wavefront
// adds up the valid counts of the blocks before this one and of all blocks
// itself (integer sums), the wavefronts share only their 64-pixel chunks'
// counts (16 bytes of LDS, so that the traversal keeps five workgroups per
// CU), and the valid pixels are placed in raster order; block 0 stores the
// pool size and resets the attempt's counters. Every thread of the
// workgroup takes part (barriers).
static_assert(POOL_BLOCK == 4 * PIX_BLOCK, "a pool block is four traversal rows of a workgroup");

__device__ void pool_block_uniform(const Attempt &A, int b, const bool ok[4], uint8_t *wcnt)
{
    const int tid = (int)threadIdx.x, wave = tid >> 6, lane = __lane_id();
    const int nb = (A.P + POOL_BLOCK - 1) / POOL_BLOCK;
    unsigned long long pc = 0ull, tc = 0ull;
    for (int i = lane; i < nb; i += 64) {
        const unsigned long long c = (unsigned long long)A.blockcnt[i];
        tc += c;
        if (i < b) pc += c;
    }
    for (int o = 32; o > 0; o >>= 1) {
        pc += __shfl_xor(pc, o, 64);
        tc += __shfl_xor(tc, o, 64);
    }
    uint64_t m[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) m[j] = __ballot(ok[j]);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) wcnt[j * (PIX_BLOCK / 64) + wave] = (uint8_t)__popcll(m[j]);
    }
    __syncthreads();
    if (b == 0 && tid == 0) {
        A.misc[0] = (int32_t)tc;
        A.misc[2] = 0;
        A.stats[0] = 0ull;
        A.stats[1] = 0ull;
        A.stats[2] = 0ull;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = j * (PIX_BLOCK / 64) + wave;
        int off = (int)pc;
        for (int k = 0; k < c; ++k) off += wcnt[k];
        const int idx = off + __popcll(m[j] & lanemask_lt());
        if (ok[j] && idx < A.P) A.pool[idx] = b * POOL_BLOCK + j * PIX_BLOCK + tid;
    }
    __syncthreads();
}

// unit = (tree, block of K x PIX_BLOCK pixels): each thread walks K pixels of
// one tree together (pixels tid, tid + PIX_BLOCK, ...), so that several
// chains of dependent probe loads are in flight per thread and the trees'
// units run side by side. K = 4 keeps a single frame's units numerous enough
// to fill the chip; K = 8 (more chains per wavefront, fewer wavefronts) suits
// large batches.
// The workgroup keeps the top levels of its unit's tree in LDS, scaled for
// the attempt's frame (restaged only when the (attempt, tree) pair changes
// between its units).
template <int K>
__global__ void __launch_bounds__(PIX_BLOCK) k_b_leaves(const Attempt *__restrict__ att, Stage S, int do_pool)
{
    __shared__ ProbeNode top[TOP_NODES];
    __shared__ uint8_t p_wcnt[K == 4 ? 4 * (PIX_BLOCK / 64) : 1];
    int cached_a = -1, cached_t = -1;
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        constexpr int PU = K * PIX_BLOCK;
        const int nb = (A.P + PU - 1) / PU;
        const int local = u - S.off[a];
        const int t = local / nb;
        const uint64_t *tree = A.nodes + (int64_t)t * (A.L - 1);
        const int ntop = A.L - 1 < TOP_NODES ? A.L - 1 : TOP_NODES;
        const Frame fr = A.fr;
        if (a != cached_a || t != cached_t) {
            __syncthreads();
            stage_top(top, tree, ntop, fr, (int)threadIdx.x, PIX_BLOCK);
            __syncthreads();
            cached_a = a;
            cached_t = t;
        }
        const int base = (local % nb) * PU + (int)threadIdx.x;
        if constexpr (K == 4) {
            // the units of tree 0 also write the pool of their pixel block
            // when no attempt of the plan has pick weights (uniform per
            // workgroup; every thread takes part)
            if (do_pool && t == 0) {
                bool okp[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int q = base + k * PIX_BLOCK;
                    okp[k] = q < A.P && packed_valid(A.packed[q < A.P ? q : A.P - 1]);
                }
                pool_block_uniform(A, local % nb, okp, p_wcnt);
            }
        }
        if (base >= A.P) continue;
        int p[K];
        uint64_t own[K];
        bool ok[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int q = base + k * PIX_BLOCK;
            p[k] = q < A.P ? q : A.P - 1;
            own[k] = A.packed[p[k]];
            ok[k] = q < A.P && packed_valid(own[k]);
        }
        int32_t leaf[K];
        traverse_packed_k<K>(top, ntop, A.deep + (int64_t)t * (A.L - 1), A.L, fr, A.packed, p, own,
                                          ok, leaf);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (base + k * PIX_BLOCK < A.P) A.leaves[(int64_t)t * A.P + base + k * PIX_BLOCK] = leaf[k];
    }
}

// Learned pick weights from the attempt's own leaves (attempts with a
// proposal network only): a unit is WT_WAVES tiles of 64 pixels, one per
// wavefront; the 24 inputs of each valid pixel, the network's forward pass on
// the matrix cores, and floor(sigmoid 65536) + 1 (0 for an invalid pixel),
// exactly as the stand-alone weight kernel computes them after its own
// traversal. The workgroup keeps the attempt's network in LDS (restaged when
// the attempt changes between its units); each wavefront's input tile is its
// own. (At least 4 wavefronts per SIMD: the kernel waits on gathers most of
// the time, and 4 resident wavefronts with a few spilled registers beat 3
// without.)
constexpr int WT_WAVES = 4;

__global__ void __launch_bounds__(64 * WT_WAVES, 4) k_b_weights(const Attempt *__restrict__ att, Stage S)
{
    __shared__ WTile W;
    __shared__ ProbeNode xn[8];
    __shared__ __align__(16) uint16_t X[WT_WAVES][ROWS * 32];
    const int l = __lane_id(), wv = (int)threadIdx.x >> 6;
    int cached = -1;
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        if (a != cached) {
            // the attempt's network and its 8 extra nodes prepared for its frame
            __syncthreads();
            stage_weights(W, A.mq, A.mw);
            if (threadIdx.x < 8) xn[threadIdx.x] = probe_node(A.nodes[(int64_t)A.T * (A.L - 1) + threadIdx.x], A.fr);
            __syncthreads();
            cached = a;
        }
        const int p = (u - S.off[a]) * (ROWS * WT_WAVES) + wv * ROWS + l;
        FeatArgs F;
        F.fr = A.fr;
        F.nodes = A.nodes;
        F.nmodes = A.nmodes;
        F.modes = A.modes;
        F.leaf_in = A.leaf_in;
        F.packed = A.packed;
        F.xnodes = xn;
        F.T = A.T; F.L = A.L; F.M = A.M; F.R = A.R;
        float x[24];
        for (int k = 0; k < 24; ++k) x[k] = 0.0f;
        bool ok = false;
        if (p < A.P) {
            const uint64_t own = A.packed[p];
            ok = packed_valid(own);
            if (ok)
                pixel_inputs(F, p % A.fr.W, p / A.fr.W, packed_depth(own),
                             [&](int t) { return A.leaves[(int64_t)t * A.P + p]; }, x);
        }
        // the tile is this wavefront's alone
        wave_lds_sync();
        store_row(X[wv], x);
        wave_lds_sync();
        const float zl = tile_forward_staged(X[wv], W);
        const uint32_t w = (p < A.P && ok) ? pick_weight(zl, nullptr) : 0u;
        if (p < A.P) A.wbuf[p] = w;
        // the tile's weight sum into its pixel block's (zeroed by k_b_pack;
        // integer sums, so the order of the additions does not matter)
        unsigned long long ws = w;
        for (int o = 32; o > 0; o >>= 1) ws += __shfl_xor(ws, o, 64);
        if (l == 0 && ws) atomicAdd(&A.blockw[(p - l) / POOL_BLOCK], ws);
    }
}

// ---------------------------------------------------------------------------
// query pool (valid pixels in raster order) and the pick-weight prefix
// ---------------------------------------------------------------------------

// Weighted picks find the first pool entry whose inclusive weight prefix
// exceeds a draw r < total. A guide table narrows that search: draw r falls in
// bucket f(r) = umulhi(r, M), M = min(floor(G 2^64 / total), 2^64 - 1) with
// G = min(pool size, total) buckets, so f never decreases and steps by at
// most 1; guide[g] is the entry whose weight range [prefix - w, prefix)
// holds the first draw of bucket g. The entry sought for r then lies between
// guide[f(r)] and guide[f(r) + 1] (the last entry for the last bucket in
// use), and a binary search over that span returns exactly the entry the
// search over the whole prefix would.
__device__ __forceinline__ uint32_t guide_bucket(unsigned long long r, unsigned long long M)
{
    return (uint32_t)__umul64hi(r, M);
}

// floor(G 2^64 / total) for 1 <= G <= total, saturated at 2^64 - 1 (restoring
// division of G 2^64, one quotient bit at a time)
__device__ __forceinline__ unsigned long long guide_multiplier(unsigned long long G, unsigned long long total)
{
    if (G >= total) return ~0ull;
    unsigned long long rem = G, q = 0ull;
    for (int i = 0; i < 64; ++i) {
        const bool top = (rem >> 63) != 0ull;
        rem <<= 1;
        q <<= 1;
        if (top || rem >= total) {
            rem -= total;
            q |= 1ull;
        }
    }
    return q;
}

__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long x)
{
    const int lane = __lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// unit = block of POOL_BLOCK pixels: the frame packed for probing (one word
// per pixel), the block's count of valid pixels and, for pick weights given
// by the caller, the block's weight sum (learned weights computed in the
// batch add theirs in k_b_weights, onto the zero written here)
// (POOL_BLOCK / PB_PIX threads per block: thread t handles pixels
// t + j POOL_BLOCK / PB_PIX of it, all loads first)
__global__ void __launch_bounds__(POOL_BLOCK / PB_PIX) k_b_pack(const Attempt *__restrict__ att, Stage S)
{
    constexpr int NT = POOL_BLOCK / PB_PIX;
    __shared__ int32_t wcnt[NT / 64];
    __shared__ unsigned long long wsum[NT / 64];
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int b = u - S.off[a];
        uint64_t w[PB_PIX];
        bool ok[PB_PIX];
#pragma unroll
        for (int j = 0; j < PB_PIX; ++j) {
            const int p = b * POOL_BLOCK + j * NT + tid;
            w[j] = p < A.P ? pack_pixel(A.fr, p) : 0ull;
        }
        int n = 0;
        unsigned long long ws = 0ull;
#pragma unroll
        for (int j = 0; j < PB_PIX; ++j) {
            const int p = b * POOL_BLOCK + j * NT + tid;
            ok[j] = p < A.P && packed_valid(w[j]);
            if (p < A.P) A.packed[p] = w[j];
            n += __popcll(__ballot(ok[j]));
            if (A.weights && !A.mq && ok[j]) ws += (unsigned long long)A.weights[p];
        }
        // the block's valid pixels and, for given weights, their weight sum
        if (A.weights && !A.mq)
            for (int o = 32; o > 0; o >>= 1) ws += __shfl_xor(ws, o, 64);
        if (__lane_id() == 0) {
            wcnt[wave] = n;
            wsum[wave] = ws;
        }
        __syncthreads();
        if (tid == 0) {
            int tn = 0;
            unsigned long long tw = 0ull;
            for (int k = 0; k < NT / 64; ++k) {
                tn += wcnt[k];
                tw += wsum[k];
            }
            A.blockcnt[b] = tn;
            // learned weights computed in the batch add theirs onto this zero
            if (A.weights) A.blockw[b] = A.mq ? 0ull : tw;
        }
        __syncthreads();
    }
}

// unit = block of POOL_BLOCK pixels: its valid pixels' indices into the
// pool (valid pixels in raster order) and, with pick weights, their inclusive
// weight prefix and guide-table entries. Each block adds up the counts and
// weight sums of the blocks before it and of all blocks itself (integer
// sums, exact in any order), so no separate scan launch is needed; block 0
// stores the pool size and the guide table's parameters and resets the
// attempt's counters. (POOL_BLOCK / PB_PIX threads per block, as k_b_pack:
// the block's 64-pixel chunks c = j (POOL_BLOCK / PB_PIX / 64) + wave,
// counted and summed in chunk order, which is raster order.)
__global__ void __launch_bounds__(POOL_BLOCK / PB_PIX) k_b_pool_write(const Attempt *__restrict__ att, Stage S)
{
    constexpr int NT = POOL_BLOCK / PB_PIX, NC = POOL_BLOCK / 64;
    __shared__ int32_t wcnt[NC];
    __shared__ unsigned long long wsw[NC];
    __shared__ unsigned long long s_part[4][NT / 64];
    const int tid = (int)threadIdx.x, wave = tid >> 6;
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int b = u - S.off[a];
        const int nb = (A.P + POOL_BLOCK - 1) / POOL_BLOCK;
        // the blocks' counts and weight sums: before this block, and in all
        unsigned long long pc = 0ull, pw = 0ull, tc = 0ull, tw = 0ull;
        for (int i = tid; i < nb; i += NT) {
            const unsigned long long c = (unsigned long long)A.blockcnt[i];
            const unsigned long long w = A.weights ? A.blockw[i] : 0ull;
            tc += c;
            tw += w;
            if (i < b) {
                pc += c;
                pw += w;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            pc += __shfl_xor(pc, o, 64);
            pw += __shfl_xor(pw, o, 64);
            tc += __shfl_xor(tc, o, 64);
            tw += __shfl_xor(tw, o, 64);
        }
        if (__lane_id() == 0) {
            s_part[0][wave] = pc;
            s_part[1][wave] = pw;
            s_part[2][wave] = tc;
            s_part[3][wave] = tw;
        }
        __syncthreads();
        unsigned long long blk_c = 0ull, blk_w = 0ull, tot_c = 0ull, tot_w = 0ull;
        for (int w = 0; w < NT / 64; ++w) {
            blk_c += s_part[0][w];
            blk_w += s_part[1][w];
            tot_c += s_part[2][w];
            tot_w += s_part[3][w];
        }
        // the guide table's multiplier (no buckets without weight)
        const unsigned long long G = tot_w < tot_c ? tot_w : tot_c;
        const unsigned long long gM = (A.weights && G) ? guide_multiplier(G, tot_w) : 0ull;
        if (b == 0 && tid == 0) {
            if (A.weights) {
                A.gsel[0] = tot_w;
                A.gsel[1] = gM;
                A.gsel[2] = tot_w ? (unsigned long long)guide_bucket(tot_w - 1ull, gM) + 1ull : 0ull;
            }
            A.misc[0] = (int32_t)tot_c;
            A.misc[2] = 0;
            A.stats[0] = 0ull;
            A.stats[1] = 0ull;
            A.stats[2] = 0ull;
        }
        uint32_t dep[PB_PIX];
#pragma unroll
        for (int j = 0; j < PB_PIX; ++j) {
            const int p = b * POOL_BLOCK + j * NT + tid;
            dep[j] = p < A.P ? (uint32_t)A.fr.depth[p] : 0u;
        }
        bool ok[PB_PIX];
        uint64_t m[PB_PIX];
        unsigned long long w[PB_PIX], wi[PB_PIX];
#pragma unroll
        for (int j = 0; j < PB_PIX; ++j) {
            const int p = b * POOL_BLOCK + j * NT + tid;
            ok[j] = p < A.P && valid_depth(A.fr, dep[j]);
            m[j] = __ballot(ok[j]);
            w[j] = (ok[j] && A.weights) ? (unsigned long long)A.weights[p] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < PB_PIX; ++j) {
            wi[j] = wave_incl_scan_u64(w[j]);
            if (__lane_id() == 63) {
                wcnt[j * (NT / 64) + wave] = __popcll(m[j]);
                wsw[j * (NT / 64) + wave] = wi[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PB_PIX; ++j) {
            const int p = b * POOL_BLOCK + j * NT + tid;
            const int c = j * (NT / 64) + wave;
            int off = (int)blk_c;
            unsigned long long offw = blk_w;
            for (int k = 0; k < c; ++k) {
                off += wcnt[k];
                offw += wsw[k];
            }
            const int idx = off + __popcll(m[j] & lanemask_lt());
            if (ok[j] && idx < A.P) {
                A.pool[idx] = p;
                if (A.weights) {
                    const unsigned long long c1 = offw + wi[j], c0 = c1 - w[j];
                    A.cdf[idx] = c1;
                    if (w[j]) {
                        // the buckets whose first draw lies in [c0, c1)
                        const unsigned long long M = gM;
                        const uint32_t g1 = guide_bucket(c1 - 1ull, M);
                        for (uint32_t g = c0 ? guide_bucket(c0 - 1ull, M) + 1u : 0u; g <= g1; ++g) A.guide[g] = idx;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// hypotheses
// ---------------------------------------------------------------------------

__device__ __forceinline__ float sq3(const float a[3], const float b[3])
{
    float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz;
}

// The colour test of a hypothesis pick, |a_c - p_c| <= tol in each channel,
// as a window per channel: max(p_c - tol, 0) <= a_c <= min(p_c + tol, 255)
// (equivalent for colours 0..255 and tol >= 0). Red and green are tested
// together as two 16-bit lanes; blue is tested with the byte above it, which
// is 0 for a mode's colour and 0xFF in an empty slot, so empty slots fail.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
struct ColourWin {
    u16x2 lo, hi;       // red, green
    uint32_t blo, bhi;  // blue
};

__device__ __forceinline__ ColourWin colour_win(uint32_t r, uint32_t g, uint32_t b, int tol)
{
    auto lo = [&](uint32_t c) { return (unsigned short)((int)c - tol < 0 ? 0 : (int)c - tol); };
    auto hi = [&](uint32_t c) { return (unsigned short)((int)c + tol > 255 ? 255 : (int)c + tol); };
    ColourWin w;
    w.lo = u16x2{lo(r), lo(g)};
    w.hi = u16x2{hi(r), hi(g)};
    w.blo = lo(b);
    w.bhi = hi(b);
    return w;
}

__device__ __forceinline__ bool colour_in(uint32_t a, const ColourWin &w)
{
    const uint32_t rg = (a & 0xFFu) | ((a << 8) & 0xFF0000u);
    const u16x2 x = __builtin_bit_cast(u16x2, rg);
    const u16x2 c = __builtin_elementwise_min(__builtin_elementwise_max(x, w.lo), w.hi);
    const uint32_t bt = a >> 16;
    return __builtin_bit_cast(uint32_t, c) == rg && min(max(bt, w.blo), w.bhi) == bt;
}

// pool index for draw u: uniform, or the first pool entry whose inclusive
// weight prefix exceeds floor(u * total / 2^64)
__device__ __forceinline__ int pick_pool(const Attempt &A, int np, uint64_t u)
{
    if (!A.weights) return (int)uniform_int(u, (uint64_t)np);
    const unsigned long long total = A.gsel[0];
    if (total == 0ull) return (int)uniform_int(u, (uint64_t)np);
    const unsigned long long r = uniform_int(u, total);
    // the span the guide table leaves (see guide_bucket)
    const uint32_t g = guide_bucket(r, A.gsel[1]);
    int lo = A.guide[g];
    int hi = (unsigned long long)g + 1ull < A.gsel[2] ? A.guide[g + 1] : np - 1;
    while (lo < hi) {
        int mid = lo + ((hi - lo) >> 1);
        if (A.cdf[mid] > r) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Colour-consistent modes of one leaf as a bit mask: bit m is set when slot m
// holds a mode whose colour is within tol of (pr, pg, pb) in every channel.
// The row is read with 16-byte loads (rgb_stride(M) colours). Mask is a
// 32-bit word for up to 32 modes per leaf, else a 64-bit one.
template <typename Mask>
__device__ __forceinline__ Mask colour_mask(const uint32_t *__restrict__ row, int Mp, const ColourWin &w)
{
    Mask mask = 0;
    for (int q = 0; q < Mp; q += 4) {
        const uint4 v = *(const uint4 *)(row + q);
        const uint32_t c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (colour_in(c[e], w)) mask |= (Mask)1 << (q + e);
    }
    return mask;
}

__device__ __forceinline__ int popc_mask(uint32_t m) { return __popc(m); }
__device__ __forceinline__ int popc_mask(uint64_t m) { return __popcll((unsigned long long)m); }
__device__ __forceinline__ int ffs_mask(uint32_t m) { return __ffs(m); }
__device__ __forceinline__ int ffs_mask(uint64_t m) { return __ffsll((unsigned long long)m); }

// the same for rows of at most 12 colours, with the row's loads issued
// before any test
__device__ __forceinline__ uint32_t colour_mask12(const uint32_t *__restrict__ row, int Mp, const ColourWin &w)
{
    const uint4 none = make_uint4(RGB_NONE, RGB_NONE, RGB_NONE, RGB_NONE);
    const uint4 *r4 = (const uint4 *)row;
    const uint4 v0 = r4[0];
    const uint4 v1 = Mp > 4 ? r4[1] : none;
    const uint4 v2 = Mp > 8 ? r4[2] : none;
    const uint32_t c[12] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x, v2.y, v2.z, v2.w};
    uint32_t mask = 0;
#pragma unroll
    for (int e = 0; e < 12; ++e)
        if (colour_in(c[e], w)) mask |= 1u << e;
    return mask;
}

// one try: draws, colour-consistent mode picks, FP32 checks, FP64 alignment
// and residuals. The pick of pixel j is the sel-th colour-consistent mode in
// (tree, mode) order, sel = uniform_int(u, count). Loads are issued a stage at
// a time (pool entries; pixel colours and depths; per pixel, its leaves and
// then its mode colour rows; the three picked modes) so that each stage
// waits once.
template <typename Mask>
__device__ bool try_hypothesis(const Attempt &A, int np, uint64_t h, uint64_t tau, double R[9], double t[3],
                               int32_t *__restrict__ s_li, Mask *__restrict__ s_mask, int ps)
{
    const U4 a = philox(h, tau, 0, 0, A.seed, TAG_HYP);
    const U4 b = philox(h, tau, 1, 0, A.seed, TAG_HYP);
    const int Mp = rgb_stride(A.M);
    int pi[3], p[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) pi[j] = pick_pool(A, np, a.x[j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) p[j] = A.pool[pi[j]];
    uint32_t pr[3], pg[3], pb[3], dep[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint64_t pw = A.packed[p[j]];   // pool pixels are valid: the word holds their depth
        dep[j] = packed_depth(pw);
        pr[j] = packed_colour(pw, 0);
        pg[j] = packed_colour(pw, 1);
        pb[j] = packed_colour(pw, 2);
    }
    int64_t pick[3];
    float c[3][3], w[3][3];
    // The colour-consistent modes of pixels q0 .. q0 + NJ - 1, held in LDS
    // slots j0 .. j0 + NJ - 1, tree by tree (all of the pixels' rows of a tree loaded before their
    // tests): the leaf indices are in s_li, the masks go to s_mask (slot
    // stride ps, one row of 64 lanes per tree); cnt[j] receives the count
    auto masks = [&](auto nj, int j0, int q0, int *cnt) {
        constexpr int NJ = decltype(nj)::value;
        ColourWin win[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            win[j] = colour_win(pr[q0 + j], pg[q0 + j], pb[q0 + j], A.rgb_tol);
            cnt[j] = 0;
        }
        if (Mp <= 12) {
            // up to 12 modes per leaf: each row's three 16-byte loads are
            // issued together, four trees at a time
#pragma unroll 4
            for (int tt = 0; tt < A.T; ++tt) {
                Mask mk[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j)
                    mk[j] = colour_mask12(A.mode_rgb + (int64_t)s_li[(j0 + j) * ps + tt * 64] * Mp, Mp, win[j]);
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    s_mask[(j0 + j) * ps + tt * 64] = mk[j];
                    cnt[j] += popc_mask(mk[j]);
                }
            }
        } else {
            for (int tt = 0; tt < A.T; ++tt) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const Mask mk = colour_mask<Mask>(A.mode_rgb + (int64_t)s_li[(j0 + j) * ps + tt * 64] * Mp, Mp,
                                                      win[j]);
                    s_mask[(j0 + j) * ps + tt * 64] = mk;
                    cnt[j] += popc_mask(mk);
                }
            }
        }
    };
    // the sel-th colour-consistent mode of the pixel in slot j, in (tree,
    // mode) order
    auto pick_of = [&](int j, int sel) {
        int64_t pk = 0;
        for (int tt = 0; tt < A.T; ++tt) {
            const Mask mk = s_mask[j * ps + tt * 64];
            const int k = popc_mask(mk);
            if (sel >= 0 && sel < k) {
                Mask mm = mk;
                for (int q = 0; q < sel; ++q) mm &= mm - (Mask)1;
                pk = (int64_t)s_li[j * ps + tt * 64] * A.M + (ffs_mask(mm) - 1);
            }
            sel -= k;
        }
        return pk;
    };
    // pixels 0 and 1 stage by stage together (their leaves, then their mode
    // colour rows, then their picked modes), then the first pair's checks
    // before any load of pixel 2 (every check is a plain predicate, so their
    // order does not change the result; lanes that fail load nothing more)
#pragma unroll 4
    for (int tt = 0; tt < A.T; ++tt) {
        const int32_t l0 = A.leaves[(int64_t)tt * A.P + p[0]], l1 = A.leaves[(int64_t)tt * A.P + p[1]];
        s_li[tt * 64] = tt * A.L + l0;
        s_li[ps + tt * 64] = tt * A.L + l1;
    }
    int cnt01[2];
    masks(std::integral_constant<int, 2>(), 0, 0, cnt01);
    if (cnt01[0] == 0 || cnt01[1] == 0) return false;
    pick[0] = pick_of(0, (int)uniform_int(b.x[0], (uint64_t)cnt01[0]));
    pick[1] = pick_of(1, (int)uniform_int(b.x[1], (uint64_t)cnt01[1]));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        cam_point(A.fr, p[j] % A.fr.W, p[j] / A.fr.W, dep[j], c[j]);
        const Mode &md = A.modes[pick[j]];
        w[j][0] = md.mu[0];
        w[j][1] = md.mu[1];
        w[j][2] = md.mu[2];
    }
    {
        if (pi[0] == pi[1]) return false;
        const float dc = sq3(c[0], c[1]);
        const float dw = sq3(w[0], w[1]);
        if (!(dc >= A.min_pair2) || !(dw <= A.ratio2 * dc) || !(dc <= A.ratio2 * dw)) return false;
    }
    // pixel 2, in slot 0 (the first two pixels' picks are done)
#pragma unroll 4
    for (int tt = 0; tt < A.T; ++tt) s_li[tt * 64] = tt * A.L + A.leaves[(int64_t)tt * A.P + p[2]];
    int cnt2[1];
    masks(std::integral_constant<int, 1>(), 0, 2, cnt2);
    if (cnt2[0] == 0) return false;
    pick[2] = pick_of(0, (int)uniform_int(b.x[2], (uint64_t)cnt2[0]));
    cam_point(A.fr, p[2] % A.fr.W, p[2] / A.fr.W, dep[2], c[2]);
    {
        const Mode &md = A.modes[pick[2]];
        w[2][0] = md.mu[0];
        w[2][1] = md.mu[1];
        w[2][2] = md.mu[2];
    }
    if (pi[0] == pi[1] || pi[0] == pi[2] || pi[1] == pi[2]) return false;
    const int EA[3] = {0, 0, 1}, EB[3] = {1, 2, 2};
    for (int e = 0; e < 3; ++e) {
        const float dc = sq3(c[EA[e]], c[EB[e]]);
        const float dw = sq3(w[EA[e]], w[EB[e]]);
        if (!(dc >= A.min_pair2)) return false;
        if (!(dw <= A.ratio2 * dc)) return false;
        if (!(dc <= A.ratio2 * dw)) return false;
    }
    const float e1[3] = {c[1][0] - c[0][0], c[1][1] - c[0][1], c[1][2] - c[0][2]};
    const float e2[3] = {c[2][0] - c[0][0], c[2][1] - c[0][1], c[2][2] - c[0][2]};
    const float cx = e1[1] * e2[2] - e1[2] * e2[1];
    const float cy = e1[2] * e2[0] - e1[0] * e2[2];
    const float cz = e1[0] * e2[1] - e1[1] * e2[0];
    if (!((cx * cx + cy * cy) + cz * cz >= A.min_area2)) return false;
    double s[NSUM];
    for (int k = 0; k < NSUM; ++k) s[k] = 0.0;
    for (int j = 0; j < 3; ++j) sums_add_point(s, c[j], w[j]);
    if (!pose_from_sums(s, R, t)) return false;
    for (int j = 0; j < 3; ++j) {
        double r[3];
        for (int k = 0; k < 3; ++k)
            r[k] = (((R[k * 3 + 0] * c[j][0] + R[k * 3 + 1] * c[j][1]) + R[k * 3 + 2] * c[j][2]) + t[k]) - w[j][k];
        if (!((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2] <= A.resid2)) return false;
    }
    return true;
}

// (Mask: uint32_t when every attempt's forest keeps at most 32 modes per
// leaf, uint64_t up to 64)
// LDS: per lane (column) and tree (row) the leaf index and the colour mask of
// the pixels being picked, two pixel slots of tmax rows (the plan's largest
// tree count)
template <typename Mask>
__global__ void __launch_bounds__(64) k_b_hypgen(const Attempt *__restrict__ att, Stage S, int tmax)
{
    extern __shared__ __align__(16) char hg_lds[];
    const int ps = tmax * 64;
    int32_t *s_li = (int32_t *)hg_lds;
    Mask *s_mask = (Mask *)(hg_lds + (size_t)2 * ps * sizeof(int32_t));
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int h = u - S.off[a];
        const int lane = __lane_id();
        const int np = A.misc[0];
        if (h >= A.N) {
            // units past the hypotheses: every round's draws, one per lane
            // (Philox counter (round, draw)), with each tree's leaf modes
            const int gi = (h - A.N) * 64 + lane;
            if (gi < A.rounds * A.B && np > 0) {
                const int rr = gi / A.B, i = gi - rr * A.B;
                const U4 x = philox((uint64_t)rr, (uint64_t)i, 0, 0, A.seed, TAG_PIX);
                const int p = A.pool[uniform_int(x.x[0], (uint64_t)np)];
                float c[3];
                cam_point(A.fr, p % A.fr.W, p / A.fr.W, packed_depth(A.packed[p]), c);
                A.draws[gi] = make_float4(c[0], c[1], c[2], __int_as_float(p));
                for (int t = 0; t < A.T; ++t) {
                    const int li = t * A.L + A.leaves[(int64_t)t * A.P + p];
                    A.dtree[(int64_t)gi * A.T + t] = make_int2(li * A.M, A.nmodes[li]);
                }
            }
            continue;
        }
        int found = -1;
        double R[9], t[3];
        for (int chunk = 0; chunk * 64 < A.max_tries && found < 0; ++chunk) {
            const int tau = chunk * 64 + lane;
            const bool ok = tau < A.max_tries && np > 0 &&
                            try_hypothesis(A, np, (uint64_t)h, (uint64_t)tau, R, t, s_li + lane, s_mask + lane, ps);
            const uint64_t m = __ballot(ok);
            if (m) {
                const int first = __ffsll((unsigned long long)m) - 1;
                found = chunk * 64 + first;
                if (lane == first) {
                    Hyp hy;
                    for (int k = 0; k < 9; ++k) {
                        hy.R[k] = R[k];
                        hy.R32[k] = (float)R[k];
                    }
                    for (int k = 0; k < 3; ++k) {
                        hy.t[k] = t[k];
                        hy.t32[k] = (float)t[k];
                    }
                    A.hyp[h] = hy;
                    for (int k = 0; k < 9; ++k) A.hyp_init[(int64_t)h * 12 + k] = R[k];
                    for (int k = 0; k < 3; ++k) A.hyp_init[(int64_t)h * 12 + 9 + k] = t[k];
                }
            }
        }
        if (lane == 0) {
            A.hyp_try[h] = found;
        }
        if (lane < NSUM) A.sums[(int64_t)h * NSUM + lane] = 0.0;
    }
}

// live list = valid hypotheses in index order, with their FP32 poses
__global__ void __launch_bounds__(1024) k_b_alive_init(const Attempt *__restrict__ att, Stage S)
{
    __shared__ int32_t wcnt[16];
    __shared__ int32_t carry;
    const int wave = threadIdx.x / 64;
    FOR_UNITS(S, u) {
        const Attempt &A = att[u];
        if (threadIdx.x == 0) carry = 0;
        __syncthreads();
        for (int base = 0; base < A.N; base += 1024) {
            const int h = base + (int)threadIdx.x;
            // the pose is loaded together with the try index (one round trip)
            float pz[12];
            bool ok = false;
            if (h < A.N) {
                const Hyp &hy = A.hyp[h];
                for (int k = 0; k < 9; ++k) pz[k] = hy.R32[k];
                for (int k = 0; k < 3; ++k) pz[9 + k] = hy.t32[k];
                ok = A.hyp_try[h] >= 0;
            }
            const uint64_t m = __ballot(ok);
            if (__lane_id() == 0) wcnt[wave] = __popcll(m);
            __syncthreads();
            int off = carry;
            for (int w = 0; w < wave; ++w) off += wcnt[w];
            if (ok) {
                const int pos = off + __popcll(m & lanemask_lt());
                A.alive[pos] = h;     // buffer 0: the list of round 0
                A.energy[pos] = 0.0f;
                for (int k = 0; k < 12; ++k) A.lpose[pos * 12 + k] = pz[k];
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                int tot = 0;
                for (int w = 0; w < 16; ++w) tot += wcnt[w];
                carry += tot;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            A.misc[2] = carry;
            A.rl[0] = carry;
        }
        if (threadIdx.x >= 1 && threadIdx.x <= MAX_ROUNDS) A.rl[threadIdx.x] = 0;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// preemptive rounds
// ---------------------------------------------------------------------------

// LDS image of one mode: mu (3), sinv (6), kappa, global mode index, pad
constexpr int SMODE = 12;
// LDS budget of the modes staged by one scoring workgroup
constexpr size_t SCORE_LDS = 64 * 1024;

// wavefronts per scoring workgroup when one draw can have up to tm modes
static int score_waves(int tm)
{
    int w = GROUP;
    while (w > 1 && (size_t)w * (size_t)tm * SMODE * sizeof(float) > SCORE_LDS) w >>= 1;
    return w;
}

// Cull of round r of one attempt, by the whole workgroup: energies in the
// defined order, bitonic sort of keys (energy key << 32 | index << 12 |
// position), which orders by (energy, index); keep the first ceil(n / 2),
// with each survivor's position in this round's list (where its inliers were
// stored) and its energy at its new position. Compare-exchange distances of 64 and more go through LDS (`keys`,
// room for the attempt's hypothesis count rounded up to a power of two, at
// least 64) with a barrier; shorter ones run in registers across the lanes of
// a wavefront.
__device__ __forceinline__ unsigned long long cull_key(float E, int h, int ap)
{
    return ((unsigned long long)float_key(E) << 32) | ((unsigned long long)(uint32_t)h << 12) | (uint32_t)ap;
}

// Live position ap's energy over a round's groups: its group sums (rows of
// `stride` floats) added in group order, CH loaded at a time. Loads past the
// last group read the last one again and add +0 instead (a group sum is
// never -0, so the total is the same), which keeps them free of branches.
template <int CH>
__device__ __forceinline__ float group_total(const float RL_GLOBAL *gs, int ap, int ng, int stride)
{
    float S = 0.0f;
    for (int k0 = 0; k0 < ng; k0 += CH) {
        float v[CH];
        const float RL_GLOBAL *row = gs + (int64_t)k0 * stride + ap;
        const int last = ng - 1 - k0;
#pragma unroll
        for (int k = 0; k < CH; ++k) v[k] = row[(int64_t)min(k, last) * stride];
#pragma unroll
        for (int k = 0; k < CH; ++k) S = S + (k <= last ? v[k] : 0.0f);
    }
    return S;
}

__device__ void cull_round(const Attempt &A, int r, unsigned long long *__restrict__ keys)
{
    const int nt = (int)blockDim.x;
    const int lane = __lane_id(), wave = (int)(threadIdx.x >> 6);
    const int na = A.rl[r];
    const int32_t *al = live_list(A, r);
    const float *en = live_energy(A, r);
    int n2 = 64;
    while (n2 < na) n2 <<= 1;
    for (int ap = threadIdx.x; ap < n2; ap += nt) {
        if (ap < na) {
            const int h = al[ap];
            const int ng = (A.B + GROUP - 1) / GROUP;
            const float E = en[ap] + group_total<32>(A.gs, ap, ng, A.N);
            keys[ap] = cull_key(E, h, ap);
            if (r < MAX_ROUNDS) {
                A.tr_alive[r * A.N + ap] = h;
                A.tr_energy[r * A.N + ap] = E;
            }
        } else {
            keys[ap] = ~0ull;
        }
    }
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        int j = k >> 1;
        for (; j >= 64; j >>= 1) {
            for (int i = threadIdx.x; i < n2; i += nt) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long x = keys[i], y = keys[ixj];
                    const bool asc = (i & k) == 0;
                    if ((x > y) == asc) {
                        keys[i] = y;
                        keys[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
        // j < 64: partners are lanes of the same wavefront (n2 is a multiple
        // of 64, so every wavefront's block is whole)
        for (int base = wave * 64; base < n2; base += nt) {
            const int i = base + lane;
            unsigned long long x = keys[i];
            const bool asc = (i & k) == 0;
            for (int jj = j; jj > 0; jj >>= 1) {
                const unsigned long long y = __shfl_xor(x, jj, 64);
                const bool lower = (lane & jj) == 0;
                const unsigned long long lo = x < y ? x : y, hi = x < y ? y : x;
                x = (lower == asc) ? lo : hi;
            }
            keys[i] = x;
        }
        __syncthreads();
    }
    const int keep = (na + 1) / 2;
    int32_t *al_next = live_list(A, r + 1);
    float *en_next = live_energy(A, r + 1);
    for (int i = threadIdx.x; i < keep; i += nt) {
        const unsigned long long key = keys[i];
        al_next[i] = (int32_t)((key >> 12) & 0xFFFFFull);
        A.pos[i] = (int32_t)(key & 0xFFFull);
        en_next[i] = key_float((uint32_t)(key >> 32));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (r < MAX_ROUNDS) A.tr_n_alive[r] = na;
        A.stats[0] += (unsigned long long)na * A.stats[2];
        A.stats[1] += (unsigned long long)na * (unsigned long long)A.B;
        A.stats[2] = 0ull;
        A.rl[r + 1] = keep;
    }
    __syncthreads();
}

constexpr int CULL_THREADS = 1024;

// one workgroup per attempt
__global__ void __launch_bounds__(CULL_THREADS) k_b_cull(const Attempt *__restrict__ att, Stage S, int r)
{
    __shared__ unsigned long long keys[MAX_HYP];
    FOR_UNITS(S, u) {
        const Attempt &A = att[u];
        if (round_active(A, r)) cull_round(A, r, keys);
    }
}

// The same cull with ranks counted instead of sorted, for rounds of at most
// RANK_MAX live hypotheses: unit = (attempt, block of 64 live positions).
// Every workgroup forms all of the round's keys in LDS as cull_round does,
// then ranks its block's keys, 16 threads per key, each counting the smaller
// keys among every 16th one (the counts added across the 16 lanes). Keys are
// distinct, so a key's rank is its position in cull_round's sorted order: the
// survivors, their order, positions and energies are the same. The work is
// spread over a workgroup per 64 live hypotheses instead of one per attempt,
// and there is no sorting network.
constexpr int RANK_MAX = 1024;
constexpr int RANK_UNITS = 64;   // rank workgroups of a round up to which it culls by ranks

__global__ void __launch_bounds__(CULL_THREADS) k_b_cull_rank(const Attempt *__restrict__ att, Stage S, int r)
{
    __shared__ unsigned long long keys[RANK_MAX];
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int blk = u - S.off[a];
        const int na = A.rl[r];
        // (uniform over the workgroup: the round did not run, or the block
        // lies past the live list)
        if (!round_active(A, r) || blk * 64 >= na) continue;
        __syncthreads();   // the previous unit's reads of `keys` are done
        const int32_t *al = live_list(A, r);
        const float *en = live_energy(A, r);
        const int ng = (A.B + GROUP - 1) / GROUP;
        for (int ap = (int)threadIdx.x; ap < na; ap += CULL_THREADS)
            keys[ap] = cull_key(en[ap] + group_total<32>(A.gs, ap, ng, A.N), al[ap], ap);
        __syncthreads();
        const int i = blk * 64 + (int)(threadIdx.x >> 4), sl = (int)(threadIdx.x & 15);
        const unsigned long long key = keys[i < na ? i : na - 1];
        uint32_t cnt = 0;
        for (int q = sl; q < na; q += 16) cnt += keys[q] < key ? 1u : 0u;
        // every lane is active here (the 16 lanes of a key form one DPP row)
        cnt += xor_lane<8>(cnt);
        cnt += xor_lane<4>(cnt);
        cnt += xor_lane<2>(cnt);
        cnt += xor_lane<1>(cnt);
        const int keep = (na + 1) / 2;
        if (sl == 0 && i < na) {
            const int h = (int)((key >> 12) & 0xFFFFFull);
            const float E = key_float((uint32_t)(key >> 32));
            if (r < MAX_ROUNDS) {
                A.tr_alive[r * A.N + i] = h;
                A.tr_energy[r * A.N + i] = E;
            }
            if ((int)cnt < keep) {
                live_list(A, r + 1)[cnt] = h;
                A.pos[cnt] = i;
                live_energy(A, r + 1)[cnt] = E;
            }
        }
        if (blk == 0 && threadIdx.x == 0) {
            if (r < MAX_ROUNDS) A.tr_n_alive[r] = na;
            A.stats[0] += (unsigned long long)na * A.stats[2];
            A.stats[1] += (unsigned long long)na * (unsigned long long)A.B;
            A.stats[2] = 0ull;
            A.rl[r + 1] = keep;
        }
    }
}

// One unit: 64 live hypotheses (lanes) x `dpu` consecutive draws (a multiple
// of GROUP). The draws of a group are spread over the workgroup's wavefronts;
// each wavefront takes its draw (pixel and leaves, staged for every round by
// the hypothesis kernel), stages the draw's modes in (tree, mode) order in
// its own LDS slice, and scores them against its lanes' hypotheses (only
// the wavefront itself touches its slice, so the wavefronts do not wait for
// each other between draws). The group's energies are then summed per lane
// in draw order and stored; the cull adds the group sums in group order. The
// units of hypothesis block 0 also count their draws' modes.
// With lph > 0 (rounds in which every attempt has at most 64 >> lph live
// hypotheses) each hypothesis takes 2^lph lanes, which split the draw's modes
// (lane j of the group takes modes j, j + 2^lph, ...) and then combine their
// first minima, ties to the lower mode, which is the first minimum in mode
// order: the same best mode and energy as one lane looping over all modes.
template <int U>
__global__ void __launch_bounds__(64 * GROUP) k_b_score(const Attempt *__restrict__ att, Stage S, int r, int dpu,
                                                        int tm, int lph)
{
    extern __shared__ __align__(16) float smode[];
    __shared__ int32_t s_ex[GROUP][16], s_base[GROUP][16];
    __shared__ float s_e[GROUP][64];
    __shared__ uint32_t s_cnt[GROUP];
    const int lane = __lane_id(), wv = (int)(threadIdx.x >> 6), nw = (int)(blockDim.x >> 6);
    float *sm = smode + (size_t)wv * tm * SMODE;
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int local = u - S.off[a];
        const int na = A.rl[r];
        const int nch = (A.B + dpu - 1) / dpu;
        const int a0 = (local / nch) * 64;
        const int ch = local % nch;
        // the lane's pose and the wavefront's first draw are loaded together
        // with the live count (a lane past the live list reads a row it does
        // not use; the addresses are within the arrays either way)
        const int sub = lane & ((1 << lph) - 1);
        const int ap = a0 + (lane >> lph);
        const float *lp = A.lpose + (int64_t)min(ap, A.N - 1) * 12;
        const float R0 = lp[0], R1 = lp[1], R2 = lp[2], R3 = lp[3], R4 = lp[4], R5 = lp[5], R6 = lp[6],
                    R7 = lp[7], R8 = lp[8];
        const float t0 = lp[9], t1 = lp[10], t2 = lp[11];
        const int i1 = min((ch + 1) * dpu, A.B);
        const int64_t rb = (int64_t)r * A.B;
        const int i_first = ch * dpu + wv;
        float4 dr_first = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        int2 e_first = make_int2(0, 0);
        if (i_first < i1) {
            dr_first = A.draws[rb + i_first];
            if (lane < A.T) e_first = A.dtree[(rb + i_first) * A.T + lane];
        }
        if (round_active(A, r) && a0 < na) {
            const bool act = ap < na;
            const bool publish = a0 == 0;
            uint32_t wcnt = 0;   // this wavefront's mode count over its draws
            for (int g0 = ch * dpu; g0 < i1; g0 += GROUP) {
                for (int k = 0; k < GROUP / nw; ++k) {
                    const int slot = k * nw + wv;
                    const int i = g0 + slot;
                    const bool has = i < i1;
                    float4 dr = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    int base = 0, nm = 0;
                    if (i == i_first) {
                        dr = dr_first;
                        base = e_first.x;
                        nm = e_first.y;
                    } else if (has) {
                        dr = A.draws[rb + i];
                        if (lane < A.T) {
                            const int2 e = A.dtree[(rb + i) * A.T + lane];
                            base = e.x;
                            nm = e.y;
                        }
                    }
                    // inclusive scan of the mode counts over the trees (lanes
                    // 0 .. T - 1 of the first row)
                    int incl = nm;
                    incl += row_up<1>(incl);
                    incl += row_up<2>(incl);
                    incl += row_up<4>(incl);
                    incl += row_up<8>(incl);
                    const int cnt = __builtin_amdgcn_readlane(incl, A.T - 1);
                    if (lane < A.T) {
                        s_ex[wv][lane] = incl - nm;
                        s_base[wv][lane] = base;
                    }
                    wcnt += has ? (uint32_t)cnt : 0u;
                    wave_lds_sync();
                    // staged up to a multiple of 4 modes: the padding slots
                    // hold a zero form and kappa = +inf, so their term is +inf
                    // and never below the best (which starts at +inf)
                    const int cnt4 = (cnt + 3) & ~3;
                    for (int j = lane; j < cnt4; j += 64) {
                        float *dst = sm + j * SMODE;
                        if (j < cnt) {
                            // the mode's tree: the last tree whose first mode index is <= j
                            int tj = 0;
                            for (int t = 1; t < A.T; ++t)
                                if (j >= s_ex[wv][t]) tj = t;
                            const int gidx = s_base[wv][tj] + (j - s_ex[wv][tj]);
                            const Mode md = A.modes[gidx];
                            dst[0] = md.mu[0]; dst[1] = md.mu[1]; dst[2] = md.mu[2];
                            dst[3] = md.sinv[0]; dst[4] = md.sinv[1]; dst[5] = md.sinv[2];
                            dst[6] = md.sinv[3]; dst[7] = md.sinv[4]; dst[8] = md.sinv[5];
                            dst[9] = md.kappa;
                            dst[10] = __int_as_float(gidx);
                        } else {
                            for (int k = 0; k < 9; ++k) dst[k] = 0.0f;
                            dst[9] = INFINITY;
                            dst[10] = __int_as_float(-1);
                        }
                        dst[11] = 0.0f;
                    }
                    wave_lds_sync();
                    const float y0 = fmaf(R0, dr.x, fmaf(R1, dr.y, fmaf(R2, dr.z, t0)));
                    const float y1 = fmaf(R3, dr.x, fmaf(R4, dr.y, fmaf(R5, dr.z, t1)));
                    const float y2 = fmaf(R6, dr.x, fmaf(R7, dr.y, fmaf(R8, dr.z, t2)));
                    float best = INFINITY;
                    int bj = -1;
                    // modes j0, j0 + js, ... of the draw against the lane's pose
                    // (unrolled U times: U modes' LDS reads in flight at once; the
                    // comparisons still run in mode order)
                    auto term_of = [&](int j) {
                        const float4 q0 = *(const float4 *)(sm + j * SMODE);
                        const float4 q1 = *(const float4 *)(sm + j * SMODE + 4);
                        const float2 q2 = *(const float2 *)(sm + j * SMODE + 8);
                        const float d0 = y0 - q0.x, d1 = y1 - q0.y, d2 = y2 - q0.z;
                        const float s0 = q0.w, s1 = q1.x, s2 = q1.y, s3 = q1.z, s4 = q1.w, s5 = q2.x;
                        const float a0v = fmaf(s2, d2, fmaf(s1, d1, s0 * d0));
                        const float a1v = fmaf(s4, d2, fmaf(s3, d1, s1 * d0));
                        const float a2v = fmaf(s5, d2, fmaf(s4, d1, s2 * d0));
                        const float q = fmaf(d2, a2v, fmaf(d1, a1v, d0 * a0v));
                        return fmaf(0.5f, q, q2.y);
                    };
                    if (lph == 0 && U == 4) {
                        // every staged mode, four at a time over the padded
                        // count (no bounds test per mode; the comparisons run
                        // in mode order)
                        for (int j = 0; j < cnt4; j += 4) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const float term = term_of(j + e);
                                if (term < best) {
                                    best = term;
                                    bj = j + e;
                                }
                            }
                        }
                    } else if (lph == 0) {
                        for (int j = 0; j < cnt; ++j) {
                            const float term = term_of(j);
                            if (term < best) {
                                best = term;
                                bj = j;
                            }
                        }
                    } else {
                        for (int j = sub; j < cnt; j += 1 << lph) {
                            const float term = term_of(j);
                            if (term < best) {
                                best = term;
                                bj = j;
                            }
                        }
                    }
                    // the lanes of a hypothesis combine their minima (every
                    // lane is active here; best is +inf exactly when bj < 0)
                    for (int o = 1; o < (1 << lph); o <<= 1) {
                        const float ob = __shfl_xor(best, o, 64);
                        const int oj = __shfl_xor(bj, o, 64);
                        if (ob < best || (ob == best && oj < bj)) {
                            best = ob;
                            bj = oj;
                        }
                    }
                    int32_t gid = -1;
                    if (bj >= 0) {
                        const float *mb = sm + bj * SMODE;
                        const float d0 = y0 - mb[0], d1 = y1 - mb[1], d2 = y2 - mb[2];
                        if ((d0 * d0 + d1 * d1) + d2 * d2 <= A.inl2) gid = __float_as_int(mb[10]);
                    }
                    if (sub == 0) s_e[slot][lane >> lph] = best < 0.0f ? best : 0.0f;
                    if (act && has && sub == 0) A.inl[inl_at(A, i, ap)] = gid;
                    // this wavefront's next draw restages its own LDS slice
                    wave_lds_sync();
                }
                __syncthreads();
                // the group's energy sum per lane, in draw order
                if (wv == 0) {
                    // lane = hypothesis of the block here
                    float g = 0.0f;
                    for (int w = 0; w < GROUP && g0 + w < i1; ++w) g = g + s_e[w][lane];
                    if (lane < (64 >> lph) && a0 + lane < na) A.gs[(int64_t)(g0 / GROUP) * A.N + a0 + lane] = g;
                }
                __syncthreads();
            }
            // one count per unit: the units of hypothesis block 0 add their
            // draws' modes to the round's count (one atomic per workgroup
            // instead of one per draw, all on the same counter)
            if (publish) {
                if (lane == 0) s_cnt[wv] = wcnt;
                __syncthreads();
                if (threadIdx.x == 0) {
                    uint32_t c = 0;
                    for (int w = 0; w < nw; ++w) c += s_cnt[w];
                    if (c) atomicAdd(&A.stats[2], (unsigned long long)c);
                }
            }
        }
    }
}

// Refinement of the survivors of round r. A survivor's inliers of the round
// are summed by one wavefront: lane-strided in draw order, combined with the
// values of an xor butterfly (each total then sits in its own lane, which
// adds it to the survivor's running sum and stores it). With refinement on, the pose is then re-solved
// from the running sums (Kabsch on all of its inliers so far). Small rounds
// run both steps in one kernel (the solve on lane 0 of each wavefront); large
// rounds (batches) solve in a second kernel with one lane per survivor, so
// that the solver's registers do not limit the occupancy of the sums. Both
// forms do the same arithmetic.
constexpr int RB = 8;              // draws per lane per load batch in refinement
constexpr int FUSED_REFINE = 1024; // survivors up to which a round refines in one kernel

// The lane-sum combination below is the xor butterfly (offsets 32, 16, ...,
// 1) with every lane keeping only the values it still needs (a
// reduce-scatter): at offset o the lanes with bit o clear keep the first half
// of their values and the others the second half, and each kept value is the
// lane's own plus its partner's, exactly as in the full butterfly (whose
// lanes all end with the same totals). Lane L ends with the total of sum
// rs_sum_of(L) (-1: a padding slot); lane rs_lane_of(k) holds sum k.
__host__ __device__ constexpr int rs_sum_of(int L)
{
    // 22 sums -> 11 (offset 32) -> 12 with one zero -> 6 (16) -> 3 (8) -> 4
    // with one zero -> 2 (4) -> 1 (2); offset 1 adds the last pair whole
    return (((L >> 1) & 1) + 2 * ((L >> 2) & 1) < 3 &&
            ((L >> 1) & 1) + 2 * ((L >> 2) & 1) + 3 * ((L >> 3) & 1) + 6 * ((L >> 4) & 1) < 11)
               ? ((L >> 1) & 1) + 2 * ((L >> 2) & 1) + 3 * ((L >> 3) & 1) + 6 * ((L >> 4) & 1) + 11 * ((L >> 5) & 1)
               : -1;
}
__host__ __device__ constexpr int rs_lane_of(int k)
{
    return (k >= 11 ? 32 : 0) + ((k % 11) >= 6 ? 16 : 0) + (((k % 11) % 6) >= 3 ? 8 : 0) +
           ((((k % 11) % 6) % 3) >= 2 ? 4 : 0) + ((((k % 11) % 6) % 3) % 2 == 1 ? 2 : 0);
}
static_assert(NSUM == 22, "the reduce-scatter below is laid out for 22 sums");
// every sum has exactly one even lane (and its odd neighbour) holding it
__host__ __device__ constexpr bool rs_maps_agree()
{
    int held = 0;
    for (int L = 0; L < 64; L += 2) {
        const int k = rs_sum_of(L);
        if (k >= NSUM || rs_sum_of(L + 1) != k) return false;
        if (k >= 0) {
            if (rs_lane_of(k) != L) return false;
            ++held;
        }
    }
    return held == NSUM;
}
static_assert(rs_maps_agree(), "lane and sum maps of the reduce-scatter disagree");

// one reduce-scatter step at offset M: lanes with bit M clear return a plus
// their partner's a, the others their partner's b plus b
template <int M>
__device__ __forceinline__ double rs_pair(double a, double b)
{
    if constexpr (M == 32 || M == 16) {
        // gfx950 permlane swaps: the upper half (M = 32) or the odd rows of
        // 16 (M = 16) of the first operand trade places with the lower half
        // or even rows of the second, which is each lane's partner exchange
        const uint64_t ai = (uint64_t)__double_as_longlong(a), bi = (uint64_t)__double_as_longlong(b);
        const auto lo = M == 32 ? __builtin_amdgcn_permlane32_swap((uint32_t)ai, (uint32_t)bi, false, false)
                                : __builtin_amdgcn_permlane16_swap((uint32_t)ai, (uint32_t)bi, false, false);
        const auto hi = M == 32 ? __builtin_amdgcn_permlane32_swap((uint32_t)(ai >> 32), (uint32_t)(bi >> 32), false, false)
                                : __builtin_amdgcn_permlane16_swap((uint32_t)(ai >> 32), (uint32_t)(bi >> 32), false, false);
        const double p0 = __longlong_as_double((long long)(((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]));
        const double p1 = __longlong_as_double((long long)(((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]));
        return p0 + p1;
    } else {
        const bool up = (__lane_id() & M) != 0;
        const double keep = up ? b : a, send = up ? a : b;
        return keep + xor_lane_f64<M>(send);
    }
}

// one batch of RB draws per lane of live position ap's round-r inliers: the
// inlier ids (global mode index, -1: not an inlier) and the draws' camera
// points
struct RefBatch {
    int32_t gid[RB];
    float4 dr[RB];
};

__device__ __forceinline__ void refine_batch_load(const Attempt &A, int r, int ap, int base, RefBatch &q)
{
    const int lane = __lane_id();
#pragma unroll
    for (int k = 0; k < RB; ++k) {
        const int i = base + k * 64 + lane;
        q.gid[k] = i < A.B ? A.inl[inl_at(A, i, ap)] : -1;
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
        const int i = base + k * 64 + lane;
        q.dr[k] = i < A.B ? A.draws[(int64_t)r * A.B + i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

// this round's inlier sums of hypothesis h (scored at live position ap), its
// first batch already loaded, added to its running sums and stored; s
// receives the totals (wavefront-uniform values)
__device__ __forceinline__ void refine_sums_pre(const Attempt &A, int r, int h, int ap, const RefBatch &q0,
                                                double s[NSUM])
{
    const int lane = __lane_id();
    const int mine = rs_sum_of(lane);
    // the running sum of the lane's own total, fetched while this round's are
    // formed
    const double runk = mine >= 0 ? A.sums[(int64_t)h * NSUM + mine] : 0.0;
#pragma unroll
    for (int k = 0; k < NSUM; ++k) s[k] = 0.0;
    // lane-strided draws, RB per lane at a time: all inlier ids first, then the
    // camera points and mode means of the inliers, then the sums in draw order
    for (int base = 0; base < A.B; base += 64 * RB) {
        RefBatch q;
        if (base == 0)
            q = q0;
        else
            refine_batch_load(A, r, ap, base, q);
        float c[RB][3], w[RB][3];
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            if (q.gid[k] >= 0) {
                const Mode &md = A.modes[q.gid[k]];
                c[k][0] = q.dr[k].x; c[k][1] = q.dr[k].y; c[k][2] = q.dr[k].z;
                w[k][0] = md.mu[0]; w[k][1] = md.mu[1]; w[k][2] = md.mu[2];
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (q.gid[k] >= 0) sums_add_point(s, c[k], w[k]);
    }
    // reduce-scatter of the 64 lane sums (every lane active)
    double w11[12], x6[6], y4[4], z2[2];
#pragma unroll
    for (int i = 0; i < 11; ++i) w11[i] = rs_pair<32>(s[i], s[i + 11]);
    w11[11] = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) x6[i] = rs_pair<16>(w11[i], w11[i + 6]);
#pragma unroll
    for (int i = 0; i < 3; ++i) y4[i] = rs_pair<8>(x6[i], x6[i + 3]);
    y4[3] = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i) z2[i] = rs_pair<4>(y4[i], y4[i + 2]);
    double u = rs_pair<2>(z2[0], z2[1]);
    u = u + xor_lane_f64<1>(u);
    const double tot = runk + u;
    if (mine >= 0 && (lane & 1) == 0) A.sums[(int64_t)h * NSUM + mine] = tot;
#pragma unroll
    for (int k = 0; k < NSUM; ++k) s[k] = lane_f64(tot, rs_lane_of(k));
}

__device__ __forceinline__ void refine_sums_at(const Attempt &A, int r, int h, int ap, double s[NSUM])
{
    RefBatch q0;
    refine_batch_load(A, r, ap, 0, q0);
    refine_sums_pre(A, r, h, ap, q0, s);
}

// the same for survivor position sidx of round r; returns the hypothesis index
__device__ __forceinline__ int refine_sums_of(const Attempt &A, int r, int sidx, double s[NSUM])
{
    const int h = live_list(A, r + 1)[sidx];
    refine_sums_at(A, r, h, A.pos[sidx], s);
    return h;
}

// re-solves hypothesis h, survivor sidx, from its running sums s when
// refinement is on, and stores its FP32 pose at its live position
__device__ __forceinline__ void refine_solve_of(const Attempt &A, int sidx, int h, const double s[NSUM])
{
    double R[9], t[3];
    float *lp = A.lpose + sidx * 12;
    Hyp &hy = A.hyp[h];
    if (A.refine && pose_from_sums(s, R, t)) {
        for (int k = 0; k < 9; ++k) {
            hy.R[k] = R[k];
            hy.R32[k] = (float)R[k];
            lp[k] = (float)R[k];
        }
        for (int k = 0; k < 3; ++k) {
            hy.t[k] = t[k];
            hy.t32[k] = (float)t[k];
            lp[9 + k] = (float)t[k];
        }
    } else {
        for (int k = 0; k < 9; ++k) lp[k] = hy.R32[k];
        for (int k = 0; k < 3; ++k) lp[9 + k] = hy.t32[k];
    }
}

// sums and solve in one kernel: one wavefront per survivor
__global__ void __launch_bounds__(64) k_b_refine(const Attempt *__restrict__ att, Stage S, int r)
{
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int sidx = u - S.off[a];
        // the survivor count and the survivor's slot loaded together (sidx is
        // below the planned survivor bound, so within the live arrays; a slot
        // past the survivor count is read but not used; the count is 0 when
        // round r did not run)
        const int keep = A.rl[r + 1];
        const int h = live_list(A, r + 1)[sidx], ap = A.pos[sidx];
        if ((sidx >= keep) | (h < 0) | (ap < 0)) continue;
        double s[NSUM];
        refine_sums_at(A, r, h, ap, s);
        if (__lane_id() == 0) refine_solve_of(A, sidx, h, s);
    }
}

// sums only: one wavefront per survivor
__global__ void __launch_bounds__(64) k_b_refine_sums(const Attempt *__restrict__ att, Stage S, int r)
{
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int sidx = u - S.off[a];
        if (sidx >= A.rl[r + 1]) continue;
        double s[NSUM];
        refine_sums_of(A, r, sidx, s);
    }
}

// solve only: one lane per survivor
__global__ void __launch_bounds__(64) k_b_refine_solve(const Attempt *__restrict__ att, Stage S, int r)
{
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int sidx = (u - S.off[a]) * 64 + __lane_id();
        if (sidx >= A.rl[r + 1]) continue;
        const int h = live_list(A, r + 1)[sidx];
        double s[NSUM];
        const double *run = A.sums + (int64_t)h * NSUM;
#pragma unroll
        for (int k = 0; k < NSUM; ++k) s[k] = run[k];
        refine_solve_of(A, sidx, h, s);
    }
}

// The attempt's result, from its final live list, into its slot of the
// plan's results (mapped host memory); by one thread
__device__ void finish_attempt(const Attempt &A)
{
    Result o;
    for (int k = 0; k < 16; ++k) o.pose_c2w[k] = (k % 5 == 0) ? 1.0 : 0.0;
    o.score = 0.0f;
    o.pool_size = A.misc[0];
    o.n_valid = A.misc[2];
    // rounds run: the first r >= 1 that starts with at most one live
    // hypothesis (none when no hypothesis is valid)
    int nr = 0;
    if (A.rl[0] >= 1) {
        nr = 1;
        while (nr < MAX_ROUNDS && A.rl[nr] > 1) ++nr;
    }
    o.n_rounds = nr;
    o.final_hyp = -1;
    o.mode_evals = A.stats[0];
    o.pair_evals = A.stats[1];
    if (o.pool_size == 0) {
        o.status = RELOC_FAIL_NO_VALID_PIXELS;
    } else if (o.n_valid == 0) {
        o.status = *A.total_samples == 0ull ? RELOC_FAIL_NO_MODES : RELOC_FAIL_NO_HYPOTHESIS;
    } else {
        const int h = live_list(A, nr)[0];
        const Hyp &hy = A.hyp[h];
        for (int rr = 0; rr < 3; ++rr) {
            for (int c = 0; c < 3; ++c) o.pose_c2w[rr * 4 + c] = hy.R[rr * 3 + c];
            o.pose_c2w[rr * 4 + 3] = hy.t[rr];
        }
        o.score = (float)(A.sums[(int64_t)h * NSUM] / ((double)o.n_rounds * (double)A.B));
        o.status = RELOC_OK;
        o.final_hyp = h;
    }
    *A.result = o;
}

__global__ void __launch_bounds__(64) k_b_finish(const Attempt *__restrict__ att, Stage S)
{
    FOR_UNITS(S, u) {
        if (threadIdx.x == 0) finish_attempt(att[u]);
    }
}

// Cull and refinement of a small round (at most FUSED_LIVE live hypotheses
// per attempt) in one kernel: one wavefront per live position w. Each
// wavefront forms every live hypothesis's energy exactly as the cull does
// (group sums in group order, added to the accumulated energy, one position
// per lane) and counts the keys (energy, index) below position w's: that
// rank is w's place in the sorted order, so the positions of rank below
// ceil(n / 2) survive, each into the slot of its rank, and are refined by
// their own wavefront (whose inlier ids and draws, indexed by w, were
// loaded together with the group sums). The wavefront of slot 0 writes the
// round's trace, statistics and survivor count. The lists are
// double-buffered by round parity, so no wavefront overwrites what another
// reads. With `fin` (the plan's last round, a lone attempt) lane 0 of slot 0
// then writes the attempt's result too, after its own refinement (all that
// the result reads was written by that lane or by earlier launches), in
// place of a separate finishing launch.
constexpr int FUSED_LIVE = 64;    // live hypotheses per attempt up to which a round culls in its refinement

__global__ void __launch_bounds__(64) k_b_cull_refine(const Attempt *__restrict__ att, Stage S, int r, int fin)
{
    FOR_UNITS(S, u) {
        const int a = attempt_of(S, u);
        const Attempt &A = att[a];
        const int w = u - S.off[a];    // below the planned live bound, so within the lists
        const int lane = __lane_id();
        const int na = A.rl[r];        // <= FUSED_LIVE: one live position per lane
        // positions clamped into the lists, so that these loads issue with
        // the live count, and position w's first batch of inlier ids and
        // draws with them
        const int apl = min(lane, A.N - 1);
        const int hl = live_list(A, r)[apl];
        const float El = live_energy(A, r)[apl];
        RefBatch q0;
        refine_batch_load(A, r, w, 0, q0);
        const int ng = (A.B + GROUP - 1) / GROUP;
        // the group sums in group order, 64 loads at a time
        const float Ssum = group_total<64>(A.gs, apl, ng, A.N);
        if (!round_active(A, r)) {
            if (fin && w == 0 && lane == 0) finish_attempt(A);
            continue;
        }
        if (w >= na) continue;
        const int keep = (na + 1) / 2;
        const bool live = lane < na;
        const float E = El + Ssum;
        const unsigned long long key = live ? cull_key(E, hl, lane) : ~0ull;
        // rank of position w: how many live keys are smaller (keys are distinct)
        const unsigned long long kw = lane_u64(key, w);
        const int sidx = __popcll(__ballot(live && key < kw));
        if (sidx >= keep) continue;
        const int h = (int)((kw >> 12) & 0xFFFFFull);
        if (lane == 0) {
            live_list(A, r + 1)[sidx] = h;
            live_energy(A, r + 1)[sidx] = key_float((uint32_t)(kw >> 32));
            A.pos[sidx] = w;
        }
        if (sidx == 0) {
            if (r < MAX_ROUNDS && live) {
                A.tr_alive[r * A.N + lane] = hl;
                A.tr_energy[r * A.N + lane] = E;
            }
            if (lane == 0) {
                if (r < MAX_ROUNDS) A.tr_n_alive[r] = na;
                A.stats[0] += (unsigned long long)na * A.stats[2];
                A.stats[1] += (unsigned long long)na * (unsigned long long)A.B;
                A.stats[2] = 0ull;
                A.rl[r + 1] = keep;
            }
        }
        double sm[NSUM];
        refine_sums_pre(A, r, h, w, q0, sm);
        if (lane == 0) refine_solve_of(A, sidx, h, sm);
        if (fin && sidx == 0 && lane == 0) finish_attempt(A);
    }
}

// ---------------------------------------------------------------------------
// host: batch plans, graphs and schedules
// ---------------------------------------------------------------------------

static int rounds_for(int N)
{
    int r = 0;
    while ((1 << r) < N) ++r;
    return r < 1 ? 1 : r;
}

struct Sched {
    int dpu[MAX_ROUNDS];   // per round: draws per scoring unit, a multiple of GROUP
    int grid;              // persistent grid of the scoring kernel (0: one workgroup per unit)
    int xcd;               // XCD-contiguous unit order
    int pix;               // pixels per traversal thread (4 or 8)
    int su;                // scoring mode-loop unroll (4 for a single attempt, else 1)
};

// a schedule with the same draws per unit in every round
static Sched uniform_sched(int dpu, int grid, int xcd, int pix, int su)
{
    Sched s;
    for (int r = 0; r < MAX_ROUNDS; ++r) s.dpu[r] = dpu;
    s.grid = grid;
    s.xcd = xcd;
    s.pix = pix;
    s.su = su;
    return s;
}

struct Shape {
    int W, H, N, B, T, L, M, weights;   // weights: 0 uniform, 1 given, 2 learned in the graph
    bool operator==(const Shape &o) const
    {
        return W == o.W && H == o.H && N == o.N && B == o.B && T == o.T && L == o.L && M == o.M &&
               weights == o.weights;
    }
};

struct Plan {
    std::vector<Shape> shape;
    int n = 0, rounds = 0, tm_max = 1, m_max = 1;
    int fused_from = 0;             // rounds from here on cull inside their refinement (k_b_cull_refine)
    char *arena = nullptr;
    size_t arena_bytes = 0;
    Attempt *d_att = nullptr;
    Attempt *h_att = nullptr;       // pinned, mapped: the graph's first kernel copies it to d_att
    const Attempt *h_att_dev = nullptr;   // its device address
    Result *h_res = nullptr;        // pinned
    std::vector<Attempt> slices;    // scratch pointers per attempt
    int32_t *d_off = nullptr;       // stage offsets of the chosen schedule
    hipGraphExec_t exec = nullptr;
    Sched sched = uniform_sched(GROUP, 0, 0, 4, 1);
    std::string desc;
    uint64_t last_use = 0;
};

}  // namespace rl

struct reloc_batch {
    std::vector<rl::Plan *> plans;
    int tune = 1;
    uint64_t clock = 0;
    uint64_t bytes = 0;
    hipStream_t cap = nullptr;
    std::string last_desc;
};

namespace rl {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// scratch of one attempt, carved from `base` (nullptr: sizing pass)
static size_t carve(const Shape &s, char *base, Attempt &A)
{
    const int64_t P = (int64_t)s.W * s.H;
    const int nb = (int)((P + POOL_BLOCK - 1) / POOL_BLOCK);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    A.leaves = (decltype(A.leaves))take((size_t)s.T * P * 4);
    A.packed = (decltype(A.packed))take((size_t)P * 8);
    A.pool = (decltype(A.pool))take((size_t)P * 4);
    A.blockcnt = (decltype(A.blockcnt))take((size_t)nb * 4);
    A.blockw = (decltype(A.blockw))take((size_t)nb * 8);
    A.cdf = (decltype(A.cdf))take(s.weights ? (size_t)P * 8 : 8);
    A.guide = (decltype(A.guide))take(s.weights ? (size_t)P * 4 : 4);
    A.gsel = (decltype(A.gsel))take(3 * 8);
    A.wbuf = (decltype(A.wbuf))take(s.weights == 2 ? (size_t)P * 4 : 4);
    A.misc = (decltype(A.misc))take(16);
    A.rl = (decltype(A.rl))take((size_t)(MAX_ROUNDS + 1) * 4);
    A.hyp = (decltype(A.hyp))take((size_t)s.N * sizeof(Hyp));
    A.hyp_init = (decltype(A.hyp_init))take((size_t)s.N * 12 * 8);
    A.hyp_try = (decltype(A.hyp_try))take((size_t)s.N * 4);
    A.energy = (decltype(A.energy))take((size_t)2 * s.N * 4);
    A.sums = (decltype(A.sums))take((size_t)s.N * NSUM * 8);
    A.alive = (decltype(A.alive))take((size_t)2 * s.N * 4);
    A.pos = (decltype(A.pos))take((size_t)s.N * 4);
    A.lpose = (decltype(A.lpose))take((size_t)s.N * 12 * 4);
    const int rounds = rounds_for(s.N);
    A.draws = (decltype(A.draws))take((size_t)rounds * s.B * 16);
    A.dtree = (decltype(A.dtree))take((size_t)rounds * s.B * s.T * 8);
    A.gs = (decltype(A.gs))take((size_t)((s.B + GROUP - 1) / GROUP) * s.N * 4);
    A.inl = (decltype(A.inl))take((size_t)((s.B + INL_TILE - 1) / INL_TILE) * INL_TILE * s.N * 4);
    A.stats = (decltype(A.stats))take(3 * 8);
    A.tr_alive = (decltype(A.tr_alive))take((size_t)MAX_ROUNDS * s.N * 4);
    A.tr_energy = (decltype(A.tr_energy))take((size_t)MAX_ROUNDS * s.N * 4);
    A.tr_n_alive = (decltype(A.tr_n_alive))take((size_t)MAX_ROUNDS * 4);
    A.result = nullptr;   // a slot of the plan's pinned host results, written by k_b_finish
    return off;
}

static void free_plan(reloc_batch *b, Plan *pl)
{
    if (!pl) return;
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->arena) (void)hipFree(pl->arena);
    if (pl->d_att) (void)hipFree(pl->d_att);
    if (pl->d_off) (void)hipFree(pl->d_off);
    if (pl->h_att) (void)hipHostFree(pl->h_att);
    if (pl->h_res) (void)hipHostFree(pl->h_res);
    b->bytes -= pl->arena_bytes;
    delete pl;
}

// copies n8 8-byte words (the batch's descriptors) from host-mapped memory
__global__ void __launch_bounds__(256) k_b_desc(const uint2 *__restrict__ src, uint2 *__restrict__ dst, int n8)
{
    for (int i = (int)threadIdx.x; i < n8; i += 256) dst[i] = src[i];
}

// stages of one schedule in launch order
struct Stages {
    Stage pix, pb, att, hyp, wts;
    std::vector<Stage> score, refine, solve, cull, live;
};

// host offsets of every stage for schedule `sc`: pix, pb, att, hyp, wts, then
// per round (score, refine, solve, cull by ranks, live positions)
static std::vector<int32_t> offsets(const Plan *pl, const Sched &sc)
{
    const int n = pl->n, R = pl->rounds;
    const int n_stage = 5 + 5 * R;
    std::vector<int32_t> off((size_t)n_stage * (n + 1), 0);
    auto fill = [&](int k, auto units) {
        int32_t *o = off.data() + (size_t)k * (n + 1);
        o[0] = 0;
        for (int a = 0; a < n; ++a) o[a + 1] = o[a] + units(a);
    };
    auto P = [&](int a) { return (int64_t)pl->shape[a].W * pl->shape[a].H; };
    fill(0, [&](int a) {
        return pl->shape[a].T * (int)((P(a) + sc.pix * PIX_BLOCK - 1) / (sc.pix * PIX_BLOCK));
    });
    fill(1, [&](int a) { return (int)((P(a) + POOL_BLOCK - 1) / POOL_BLOCK); });
    fill(2, [&](int) { return 1; });
    fill(3, [&](int a) { return pl->shape[a].N + (rounds_for(pl->shape[a].N) * pl->shape[a].B + 63) / 64; });
    fill(4, [&](int a) {
        return pl->shape[a].weights == 2 ? (int)((P(a) + ROWS * WT_WAVES - 1) / (ROWS * WT_WAVES)) : 0;
    });
    auto bound = [&](int a, int rr) {
        int bnd = pl->shape[a].N;
        for (int k = 0; k < rr; ++k) bnd = (bnd + 1) / 2;
        return bnd;
    };
    for (int r = 0; r < R; ++r) {
        fill(5 + 5 * r, [&](int a) {
            if (r >= rounds_for(pl->shape[a].N)) return 0;
            return ((bound(a, r) + 63) / 64) * ((pl->shape[a].B + sc.dpu[r] - 1) / sc.dpu[r]);
        });
        fill(6 + 5 * r, [&](int a) { return r >= rounds_for(pl->shape[a].N) ? 0 : bound(a, r + 1); });
        fill(7 + 5 * r, [&](int a) { return r >= rounds_for(pl->shape[a].N) ? 0 : (bound(a, r + 1) + 63) / 64; });
        fill(8 + 5 * r, [&](int a) { return r >= rounds_for(pl->shape[a].N) ? 0 : (bound(a, r) + 63) / 64; });
        fill(9 + 5 * r, [&](int a) { return r >= rounds_for(pl->shape[a].N) ? 0 : bound(a, r); });
    }
    return off;
}

static Stages stages_of(const Plan *pl, const Sched &sc, const int32_t *d_off, const std::vector<int32_t> &off)
{
    const int n = pl->n;
    auto mk = [&](int k) {
        Stage s;
        s.off = d_off + (size_t)k * (n + 1);
        s.n = n;
        s.total = off[(size_t)k * (n + 1) + n];
        s.xcd = sc.xcd;
        return s;
    };
    Stages st;
    st.pix = mk(0); st.pb = mk(1); st.att = mk(2); st.hyp = mk(3); st.wts = mk(4);
    for (int r = 0; r < pl->rounds; ++r) {
        st.score.push_back(mk(5 + 5 * r));
        st.refine.push_back(mk(6 + 5 * r));
        st.solve.push_back(mk(7 + 5 * r));
        st.cull.push_back(mk(8 + 5 * r));
        st.live.push_back(mk(9 + 5 * r));
    }
    return st;
}

static unsigned grid_of(const Stage &s, int cap, int xcd)
{
    int g = s.total < 1 ? 1 : s.total;
    if (cap > 0 && g > cap) g = cap;
    if (xcd) g = ((g + 7) / 8) * 8;
    return (unsigned)g;
}

static void launch_leaves(const Sched &sc, const Stages &st, int cap, const Attempt *d, hipStream_t s, int do_pool)
{
    if (sc.pix == 8)
        RL_LAUNCH("k_b_leaves", k_b_leaves<8>, dim3(grid_of(st.pix, cap, sc.xcd)), dim3(PIX_BLOCK), 0, s, d, st.pix,
                  do_pool);
    else
        RL_LAUNCH("k_b_leaves", k_b_leaves<4>, dim3(grid_of(st.pix, cap, sc.xcd)), dim3(PIX_BLOCK), 0, s, d, st.pix,
                  do_pool);
}

// Per-launch timing for the tuner: events around the traversal launch and
// each round's scoring launch, each pair followed by a bare pair whose
// elapsed time (the events' own cost) is subtracted
struct LaunchTimer {
    hipEvent_t ev[2 * (MAX_ROUNDS + 1)][4] = {};
    bool ok = false;
    LaunchTimer()
    {
        ok = true;
        for (auto &e : ev)
            for (auto &x : e)
                if (hipEventCreate(&x) != hipSuccess) ok = false;
    }
    ~LaunchTimer()
    {
        for (auto &e : ev)
            for (auto &x : e)
                if (x) (void)hipEventDestroy(x);
    }
    // slot 0: traversal; slot 1 + r: scoring of round r
    void begin(int slot, hipStream_t s) { (void)hipEventRecord(ev[slot][0], s); }
    void end(int slot, hipStream_t s)
    {
        (void)hipEventRecord(ev[slot][1], s);
        (void)hipEventRecord(ev[slot][2], s);
        (void)hipEventRecord(ev[slot][3], s);
    }
    // milliseconds of slot (at least 0: a launch with nothing to do can take
    // less than the spread of the events' own cost), < 0 on error
    float ms(int slot)
    {
        float a = 0.0f, b = 0.0f;
        if (hipEventSynchronize(ev[slot][3]) != hipSuccess || hipEventElapsedTime(&a, ev[slot][0], ev[slot][1]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[slot][2], ev[slot][3]) != hipSuccess)
            return -1.0f;
        return a > b ? a - b : 0.0f;
    }
};

// enqueues every kernel of the batch on `s` (with `tm`, the traversal and
// the scoring launches are timed)
static int enqueue(const Plan *pl, const Sched &sc, const Stages &st, hipStream_t s, LaunchTimer *tm = nullptr)
{
    const Attempt *d = pl->d_att;
    const int cap = 4096;
    // the attempts' descriptors, written by the host into mapped pinned
    // memory before each launch, copied to device memory by the first kernel
    static_assert(sizeof(Attempt) % 8 == 0, "descriptor copied in 8-byte words");
    RL_LAUNCH("k_b_desc", k_b_desc, dim3(1), dim3(256), 0, s, (const uint2 *)pl->h_att_dev, (uint2 *)pl->d_att,
              (int)(sizeof(Attempt) / 8) * pl->n);
    // one workgroup per attempt: plain round-robin ownership
    Stage att = st.att;
    att.xcd = 0;
    RL_LAUNCH("k_b_pack", k_b_pack, dim3(grid_of(st.pb, cap, sc.xcd)), dim3(POOL_BLOCK / PB_PIX), 0, s, d, st.pb);
    // without pick weights the 4-pixel traversal's tree-0 units write the
    // pool; otherwise the pool (and its weight prefix) follows the weights
    bool weighted = false;
    for (const Shape &sh : pl->shape) weighted |= sh.weights != 0;
    const bool pool_in_leaves = !weighted && sc.pix == 4;
    if (tm) tm->begin(0, s);
    launch_leaves(sc, st, cap, d, s, pool_in_leaves ? 1 : 0);
    if (tm) tm->end(0, s);
    // learned weights feed the pool's weight prefix
    if (st.wts.total > 0)
        RL_LAUNCH("k_b_weights", k_b_weights, dim3(grid_of(st.wts, cap / WT_WAVES, sc.xcd)), dim3(64 * WT_WAVES), 0,
                  s, d, st.wts);
    if (!pool_in_leaves)
        RL_LAUNCH("k_b_pool_write", k_b_pool_write, dim3(grid_of(st.pb, cap, sc.xcd)), dim3(POOL_BLOCK / PB_PIX), 0,
                  s, d, st.pb);
    int t_max = 1;
    for (const Shape &sh : pl->shape) t_max = sh.T > t_max ? sh.T : t_max;
    if (pl->m_max > 32)
        RL_LAUNCH("k_b_hypgen", k_b_hypgen<uint64_t>, dim3(grid_of(st.hyp, 0, sc.xcd)), dim3(64),
                  (size_t)2 * t_max * 64 * (4 + 8), s, d, st.hyp, t_max);
    else
        RL_LAUNCH("k_b_hypgen", k_b_hypgen<uint32_t>, dim3(grid_of(st.hyp, 0, sc.xcd)), dim3(64),
                  (size_t)2 * t_max * 64 * (4 + 4), s, d, st.hyp, t_max);
    RL_LAUNCH("k_b_alive_init", k_b_alive_init, dim3(grid_of(att, cap, 0)), dim3(1024), 0, s, d, att);
    // the LDS slice of a wavefront holds a draw's modes padded to a multiple of 4
    const int tm4 = (pl->tm_max + 3) & ~3;
    const int nw = score_waves(tm4);
    const size_t smem = (size_t)nw * tm4 * SMODE * sizeof(float);
    // a round culls by ranks when every attempt's live list fits RANK_MAX and
    // the round needs few rank workgroups (each one reads all of its
    // attempt's group sums); otherwise by one sorting workgroup per attempt
    auto rank_cull = [&](int r) {
        if (st.cull[r].total > RANK_UNITS) return false;
        for (const Shape &sh : pl->shape) {
            int bnd = sh.N;
            for (int k = 0; k < r; ++k) bnd = (bnd + 1) / 2;
            if (bnd > RANK_MAX) return false;
        }
        return true;
    };
    // lanes per hypothesis (log2) in the scoring of round r: the largest
    // planned live count of the round's attempts, rounded up to a power of
    // two, takes 64 >> lph lanes (at least 2 hypotheses per block)
    auto lph_of = [&](int r) {
        int mx = 0;
        for (const Shape &sh : pl->shape) {
            int bnd = sh.N;
            for (int k = 0; k < r; ++k) bnd = (bnd + 1) / 2;
            mx = bnd > mx ? bnd : mx;
        }
        int l = 0;
        while (l < 5 && (64 >> (l + 1)) >= mx) ++l;
        return l;
    };
    bool finished = false;
    for (int r = 0; r < pl->rounds; ++r) {
        if (tm) tm->begin(1 + r, s);
        if (sc.su == 4)
            RL_LAUNCH("k_b_score", k_b_score<4>, dim3(grid_of(st.score[r], sc.grid, sc.xcd)), dim3(64 * nw), smem,
                      s, d, st.score[r], r, sc.dpu[r], tm4, lph_of(r));
        else
            RL_LAUNCH("k_b_score", k_b_score<1>, dim3(grid_of(st.score[r], sc.grid, sc.xcd)), dim3(64 * nw), smem,
                      s, d, st.score[r], r, sc.dpu[r], tm4, lph_of(r));
        if (tm) tm->end(1 + r, s);
        if (r >= pl->fused_from && st.refine[r].total <= FUSED_REFINE) {
            // a lone attempt's last round also writes its result
            const int fin = (pl->n == 1 && r == pl->rounds - 1) ? 1 : 0;
            RL_LAUNCH("k_b_cull_refine", k_b_cull_refine, dim3(grid_of(st.live[r], 0, sc.xcd)), dim3(64), 0, s, d,
                      st.live[r], r, fin);
            finished |= fin != 0;
            continue;
        }
        if (rank_cull(r))
            RL_LAUNCH("k_b_cull_rank", k_b_cull_rank, dim3(grid_of(st.cull[r], 0, sc.xcd)), dim3(CULL_THREADS), 0, s,
                      d, st.cull[r], r);
        else
            RL_LAUNCH("k_b_cull", k_b_cull, dim3(grid_of(att, cap, 0)), dim3(CULL_THREADS), 0, s, d, att, r);
        if (st.refine[r].total <= FUSED_REFINE) {
            RL_LAUNCH("k_b_refine", k_b_refine, dim3(grid_of(st.refine[r], 0, sc.xcd)), dim3(64), 0, s, d,
                      st.refine[r], r);
        } else {
            RL_LAUNCH("k_b_refine_sums", k_b_refine_sums, dim3(grid_of(st.refine[r], 0, sc.xcd)), dim3(64), 0, s, d,
                      st.refine[r], r);
            RL_LAUNCH("k_b_refine_solve", k_b_refine_solve, dim3(grid_of(st.solve[r], 0, sc.xcd)), dim3(64), 0, s,
                      d, st.solve[r], r);
        }
    }
    if (!finished) RL_LAUNCH("k_b_finish", k_b_finish, dim3(grid_of(att, cap, 0)), dim3(64), 0, s, d, att);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

// captures the batch for schedule `sc` with its own offsets buffer
static int capture(reloc_batch *b, const Plan *pl, const Sched &sc, int32_t **d_off_out, hipGraphExec_t *out)
{
    const std::vector<int32_t> off = offsets(pl, sc);
    int32_t *d_off = nullptr;
    RL_HIP(hipMalloc((void **)&d_off, off.size() * 4));
    if (hipMemcpy(d_off, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d_off);
        return RELOC_E_HIP;
    }
    const Stages st = stages_of(pl, sc, d_off, off);
    if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(d_off);
        return RELOC_E_HIP;
    }
    const bool was_on = prof_on();
    if (was_on) reloc_profile_enable(0);
    hipGraph_t g = nullptr;
    int rc = RELOC_OK;
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = RELOC_E_HIP;
    if (!rc) {
        rc = enqueue(pl, sc, st, b->cap);
        if (hipStreamEndCapture(b->cap, &g) != hipSuccess && !rc) rc = RELOC_E_HIP;
    }
    if (was_on) reloc_profile_enable(1);
    if (!rc && hipGraphInstantiate(out, g, nullptr, nullptr, 0) != hipSuccess) rc = RELOC_E_HIP;
    if (g) (void)hipGraphDestroy(g);
    if (rc) {
        (void)hipFree(d_off);
        return rc;
    }
    *d_off_out = d_off;
    return RELOC_OK;
}

static std::string sched_desc(const Sched &s, int rounds)
{
    std::string dpu;
    for (int r = 0; r < rounds && r < MAX_ROUNDS; ++r) dpu += (r ? "/" : "") + std::to_string(s.dpu[r]);
    char buf[200];
    if (s.grid)
        snprintf(buf, sizeof(buf), "draws_per_unit=%s score_grid=%d xcd_contiguous=%d pix_per_thread=%d score_unroll=%d",
                 dpu.c_str(), s.grid, s.xcd, s.pix, s.su);
    else
        snprintf(buf, sizeof(buf),
                 "draws_per_unit=%s score_grid=per-unit xcd_contiguous=%d pix_per_thread=%d score_unroll=%d",
                 dpu.c_str(), s.xcd, s.pix, s.su);
    return buf;
}

// runs the plan once: the graph, or, while per-kernel timing is on, the same
// kernels launched one by one so that each launch can be timed
static int run_plan(Plan *pl, hipStream_t s)
{
    if (prof_on()) {
        const std::vector<int32_t> off = offsets(pl, pl->sched);
        prof_delay(s, 8 + 3 * pl->rounds);
        return enqueue(pl, pl->sched, stages_of(pl, pl->sched, pl->d_off, off), s);
    }
    RL_HIP(hipGraphLaunch(pl->exec, s));
    return RELOC_OK;
}

// times one uncaptured run of schedule `sc` (launches one by one behind the
// timing delay): per round, the scoring kernel's duration into t_round[r]
// (ms); the second of two runs counts (the first warms the caches)
static int time_rounds(Plan *pl, const Sched &sc, hipStream_t s, LaunchTimer &tm, float *t_round)
{
    const std::vector<int32_t> off = offsets(pl, sc);
    int32_t *d_off = nullptr;
    RL_HIP(hipMalloc((void **)&d_off, off.size() * 4));
    int rc = RELOC_OK;
    if (hipMemcpy(d_off, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess) rc = RELOC_E_HIP;
    const Stages st = stages_of(pl, sc, d_off, off);
    for (int run = 0; run < 2 && !rc; ++run) {
        prof_delay(s, 8 + 3 * pl->rounds);
        rc = enqueue(pl, sc, st, s, &tm);
        if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = RELOC_E_HIP;
    }
    for (int r = 0; r < pl->rounds && !rc; ++r) {
        t_round[r] = tm.ms(1 + r);
        if (t_round[r] < 0.0f) rc = RELOC_E_HIP;
    }
    (void)hipFree(d_off);
    return rc;
}

// Chooses the batch's schedule. Without tuning: every round 8 draws per
// scoring unit, one workgroup per unit. With tuning: (1) per round, the
// draws per scoring unit (8, 16, 32 or 64) whose scoring launch was
// fastest in per-launch timings of uncaptured runs (the lower of two
// passes); (2) over that per-round schedule and six uniform ones, with and
// without a persistent scoring grid and the XCD-contiguous unit order, the
// captured graph with the lowest of three timed launches, the candidates
// launched in turn after three warm launches. Every schedule computes the
// same results. Traversal width and the scoring unroll follow fixed rules.
static int tune(reloc_batch *b, Plan *pl, hipStream_t s)
{
    // traversal work of the batch (pixels x trees): 8 pixels per thread from
    // about five full-size frames of five trees on, where the units still
    // fill the chip several times over
    int64_t work = 0;
    int max_B = 1;
    for (const Shape &sh : pl->shape) {
        work += (int64_t)sh.W * sh.H * sh.T;
        max_B = std::max(max_B, sh.B);
    }
    const int pix = work >= 8000000 ? 8 : 4;
    // a single attempt's rounds are short latency chains: the scoring
    // kernel's mode loop unrolled (more registers, fewer resident
    // wavefronts) shortens them; batches keep the leaner loop
    const int su = pl->n == 1 ? 4 : 1;
    std::vector<Sched> cands;
    cands.push_back(uniform_sched(GROUP, 0, 0, pix, su));
    if (b->tune) {
        // (1) per-round draws per unit from per-launch timings
        const bool was_on = prof_on();
        if (was_on) reloc_profile_enable(0);
        Sched per = uniform_sched(GROUP, 0, 1, pix, su);
        float best_t[MAX_ROUNDS];
        for (float &x : best_t) x = 1e30f;
        int rc = RELOC_OK;
        {
            // two passes over the candidates (the first also warms the chip),
            // the lower time of each (candidate, round) counting
            LaunchTimer tm;
            if (!tm.ok) rc = RELOC_E_HIP;
            float t_dpu[4][MAX_ROUNDS];
            for (auto &row : t_dpu)
                for (float &x : row) x = 1e30f;
            int n_dpu = 0;
            for (int d = GROUP; d <= 8 * GROUP; d *= 2) {
                if (d > GROUP && d / 2 >= max_B) break;
                ++n_dpu;
            }
            for (int pass = 0; pass < 2 && !rc; ++pass)
                for (int j = 0; j < n_dpu && !rc; ++j) {
                    float t[MAX_ROUNDS];
                    rc = time_rounds(pl, uniform_sched(GROUP << j, 0, 1, pix, su), s, tm, t);
                    for (int r = 0; r < pl->rounds && !rc; ++r) t_dpu[j][r] = std::min(t_dpu[j][r], t[r]);
                }
            for (int j = 0; j < n_dpu && !rc; ++j)
                for (int r = 0; r < pl->rounds; ++r)
                    if (t_dpu[j][r] < best_t[r]) {
                        best_t[r] = t_dpu[j][r];
                        per.dpu[r] = GROUP << j;
                    }
        }
        if (was_on) reloc_profile_enable(1);
        if (rc) return rc;
        // (2) whole graphs
        for (int xcd = 0; xcd < 2; ++xcd) {
            Sched c = per;
            c.xcd = xcd;
            cands.push_back(c);
        }
        Sched c = per;
        c.grid = 2048;
        cands.push_back(c);
        cands.push_back(uniform_sched(GROUP, 0, 1, pix, su));
        cands.push_back(uniform_sched(2 * GROUP, 0, 1, pix, su));
        cands.push_back(uniform_sched(4 * GROUP, 0, 1, pix, su));
        cands.push_back(uniform_sched(GROUP, 2048, 1, pix, su));
        cands.push_back(uniform_sched(2 * GROUP, 1024, 1, pix, su));
    }
    // every candidate captured; then, after three warm launches, three passes
    // that launch each candidate once, the lowest of its three times counting
    const size_t nc = cands.size();
    std::vector<hipGraphExec_t> ex(nc, nullptr);
    std::vector<int32_t *> offs(nc, nullptr);
    std::vector<float> t_min(nc, 1e30f);
    int rc = RELOC_OK;
    for (size_t i = 0; i < nc && !rc; ++i) rc = capture(b, pl, cands[i], &offs[i], &ex[i]);
    if (!rc && nc > 1) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = RELOC_E_HIP;
        for (int w = 0; w < 3 && !rc; ++w)
            if (hipGraphLaunch(ex[0], s) != hipSuccess) rc = RELOC_E_HIP;
        for (int pass = 0; pass < 3 && !rc; ++pass)
            for (size_t i = 0; i < nc && !rc; ++i) {
                float ms = 0.0f;
                if (hipEventRecord(e0, s) != hipSuccess || hipGraphLaunch(ex[i], s) != hipSuccess ||
                    hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                    rc = RELOC_E_HIP;
                else
                    t_min[i] = std::min(t_min[i], ms);
            }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    size_t pick = 0;
    for (size_t i = 1; i < nc; ++i)
        if (t_min[i] < t_min[pick]) pick = i;
    for (size_t i = 0; i < nc; ++i)
        if (rc || i != pick) {
            if (ex[i]) (void)hipGraphExecDestroy(ex[i]);
            if (offs[i]) (void)hipFree(offs[i]);
        }
    if (rc) return rc;
    hipGraphExec_t best = ex[pick];
    int32_t *best_off = offs[pick];
    const Sched best_s = cands[pick];
    pl->exec = best;
    pl->d_off = best_off;
    pl->sched = best_s;
    pl->desc = sched_desc(best_s, pl->rounds) + (cands.size() > 1 ? " (tuned)" : " (fixed)");
    return RELOC_OK;
}

static Plan *find_or_make_plan(reloc_batch *b, const std::vector<Shape> &shape, int tm_max, int *rc)
{
    for (Plan *p : b->plans)
        if (p->shape.size() == shape.size() && std::equal(shape.begin(), shape.end(), p->shape.begin()) &&
            p->tm_max == tm_max) {
            p->last_use = ++b->clock;
            return p;
        }
    if (b->plans.size() >= 8) {     // evict the least recently used shape
        auto it = std::min_element(b->plans.begin(), b->plans.end(),
                                   [](Plan *x, Plan *y) { return x->last_use < y->last_use; });
        free_plan(b, *it);
        b->plans.erase(it);
    }
    Plan *pl = new (std::nothrow) Plan();
    if (!pl) {
        *rc = RELOC_E_NOMEM;
        return nullptr;
    }
    pl->shape = shape;
    pl->n = (int)shape.size();
    pl->tm_max = tm_max;
    for (const Shape &s : shape) {
        pl->rounds = std::max(pl->rounds, rounds_for(s.N));
        pl->m_max = std::max(pl->m_max, s.M);
        // the first round whose live list is at most FUSED_LIVE long whatever
        // the number of valid hypotheses (N halved once per round)
        int r = 0, bound = s.N;
        while (bound > FUSED_LIVE) {
            bound = (bound + 1) / 2;
            ++r;
        }
        pl->fused_from = std::max(pl->fused_from, r);
    }
    size_t total = 0;
    pl->slices.resize(pl->n);
    std::vector<size_t> at(pl->n);
    for (int a = 0; a < pl->n; ++a) {
        at[a] = total;
        total += carve(shape[a], nullptr, pl->slices[a]);
    }
    pl->arena_bytes = total;
    if (hipMalloc((void **)&pl->arena, total) != hipSuccess ||
        hipMalloc((void **)&pl->d_att, sizeof(Attempt) * pl->n) != hipSuccess ||
        hipHostMalloc((void **)&pl->h_att, sizeof(Attempt) * pl->n, hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&pl->h_res, sizeof(Result) * pl->n, hipHostMallocCoherent) != hipSuccess) {
        pl->arena_bytes = 0;
        free_plan(b, pl);
        *rc = RELOC_E_NOMEM;
        return nullptr;
    }
    b->bytes += total;
    // results go straight from k_b_finish into coherent pinned host memory (no
    // copy per attempt after the graph)
    Result *d_res = nullptr;
    if (hipHostGetDevicePointer((void **)&d_res, pl->h_res, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&pl->h_att_dev, pl->h_att, 0) != hipSuccess) {
        free_plan(b, pl);
        *rc = RELOC_E_HIP;
        return nullptr;
    }
    for (int a = 0; a < pl->n; ++a) {
        carve(shape[a], pl->arena + at[a], pl->slices[a]);
        pl->slices[a].result = (decltype(pl->slices[a].result))(d_res + a);
    }
    pl->last_use = ++b->clock;
    b->plans.push_back(pl);
    return pl;
}

// validates and runs a batch; results land in pl->h_res (pinned)
static int run_batch(reloc_batch *b, const reloc_attempt *att, int n, hipStream_t s, Plan **plan_out)
{
    if (!b || !att || n < 1) return RELOC_E_ARG;
    std::vector<Shape> shape(n);
    std::vector<Frame> frames(n);
    int tm_max = 1;
    for (int a = 0; a < n; ++a) {
        const reloc_attempt &x = att[a];
        Forest *f = x.forest;
        if (!f || (x.proposal && x.pixel_weights_dev)) return RELOC_E_ARG;
        int rc = frame_from(f, x.depth_dev, x.rgb_dev, &x.K, frames[a]);
        if (rc) return rc;
        const int N = x.n_hypotheses > 0 ? x.n_hypotheses : f->p.n_hypotheses;
        if (N > MAX_HYP || f->T * f->M > MAX_TM) return RELOC_E_ARG;
        shape[a] = Shape{frames[a].W, frames[a].H, N, f->p.batch_pixels, f->T, f->L, f->M,
                         x.proposal ? 2 : (x.pixel_weights_dev ? 1 : 0)};
        tm_max = std::max(tm_max, f->T * f->M);
    }
    for (int a = 0; a < n; ++a) {   // pending modes of every forest involved
        int rc = update_modes(att[a].forest, s);
        if (rc) return rc;
    }
    int rc = RELOC_OK;
    Plan *pl = find_or_make_plan(b, shape, tm_max, &rc);
    if (!pl) return rc;
    for (int a = 0; a < n; ++a) {
        const reloc_attempt &x = att[a];
        const Forest *f = x.forest;
        Attempt A = pl->slices[a];
        A.fr = frames[a];
        A.nodes = (decltype(A.nodes))f->nodes;
        A.deep = (decltype(A.deep))f->deep;
        A.nmodes = (decltype(A.nmodes))f->nmodes;
        A.modes = (decltype(A.modes))f->modes;
        A.mode_rgb = (decltype(A.mode_rgb))f->mode_rgb;
        A.total_samples = (decltype(A.total_samples))f->total_samples;
        A.weights = x.proposal ? (decltype(A.weights))A.wbuf : (decltype(A.weights))x.pixel_weights_dev;
        A.leaf_in = (decltype(A.leaf_in))f->leaf_in;
        A.R = f->R;
        A.mq = x.proposal ? (decltype(A.mq))rl_mlp_q(x.proposal) : nullptr;
        A.mw = x.proposal ? (decltype(A.mw))rl_mlp_w(x.proposal) : nullptr;
        A.T = f->T; A.L = f->L; A.M = f->M; A.P = frames[a].W * frames[a].H;
        A.N = shape[a].N; A.B = f->p.batch_pixels; A.max_tries = f->p.max_tries; A.rgb_tol = f->p.rgb_tol;
        A.refine = f->p.refine; A.rounds = rounds_for(A.N);
        A.ratio2 = f->p.rigid_ratio2; A.min_pair2 = f->p.min_pair2_m2; A.min_area2 = f->p.min_area2_m4;
        A.inl2 = f->p.inlier_m * f->p.inlier_m;
        A.resid2 = (double)f->p.resid_m * (double)f->p.resid_m;
        A.seed = x.seed;
        pl->h_att[a] = A;
    }
    if (!pl->exec) {
        rc = tune(b, pl, s);
        if (rc) return rc;
    }
    b->last_desc = pl->desc;
    rc = run_plan(pl, s);
    if (rc) return rc;
    RL_HIP(hipStreamSynchronize(s));
    if (plan_out) *plan_out = pl;
    return RELOC_OK;
}

}  // namespace rl

using namespace rl;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" int reloc_batch_create(reloc_batch **out)
{
    if (!out) return RELOC_E_ARG;
    *out = new (std::nothrow) reloc_batch();
    return *out ? RELOC_OK : RELOC_E_NOMEM;
}

extern "C" int reloc_batch_destroy(reloc_batch *b)
{
    if (!b) return RELOC_E_ARG;
    (void)hipDeviceSynchronize();
    for (Plan *p : b->plans) free_plan(b, p);
    b->plans.clear();
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return RELOC_OK;
}

extern "C" int reloc_batch_set_tuning(reloc_batch *b, int32_t on)
{
    if (!b) return RELOC_E_ARG;
    b->tune = on ? 1 : 0;
    return RELOC_OK;
}

extern "C" int reloc_batch_schedule(const reloc_batch *b, char *desc, int32_t cap)
{
    if (!b || !desc || cap < 1) return RELOC_E_ARG;
    const int n = (int)b->last_desc.size() < cap - 1 ? (int)b->last_desc.size() : cap - 1;
    memcpy(desc, b->last_desc.data(), (size_t)n);
    desc[n] = 0;
    return RELOC_OK;
}

extern "C" int reloc_batch_memory(const reloc_batch *b, uint64_t *bytes_out)
{
    if (!b || !bytes_out) return RELOC_E_ARG;
    *bytes_out = b->bytes;
    return RELOC_OK;
}

extern "C" int reloc_relocalise_batch(reloc_batch *b, const reloc_attempt *attempts, int32_t n,
                                      reloc_result *results_host, void *stream)
{
    if (!results_host) return RELOC_E_ARG;
    Plan *pl = nullptr;
    const int rc = run_batch(b, attempts, n, (hipStream_t)stream, &pl);
    if (rc) return rc;
    memcpy(results_host, pl->h_res, sizeof(Result) * n);
    return RELOC_OK;
}

static int plain(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev, const reloc_intrinsics *K,
                 uint64_t seed, int32_t n_hypotheses, const uint32_t *weights, const reloc_mlp *proposal,
                 reloc_result *out, void *stream)
{
    if (!f || !K || !out) return RELOC_E_ARG;
    if (!f->plain) {
        reloc_batch *b = nullptr;
        const int rc = reloc_batch_create(&b);
        if (rc) return rc;
        b->tune = 0;
        f->plain = b;
    }
    reloc_attempt x;
    x.forest = f;
    x.depth_dev = depth_dev;
    x.rgb_dev = rgb_dev;
    x.K = *K;
    x.seed = seed;
    x.n_hypotheses = n_hypotheses;
    x.pixel_weights_dev = weights;
    x.proposal = proposal;
    return reloc_relocalise_batch(f->plain, &x, 1, out, stream);
}

extern "C" int reloc_relocalise_ex(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                   const reloc_intrinsics *K, uint64_t attempt_seed, int32_t n_hypotheses,
                                   const uint32_t *pixel_weights_dev, reloc_result *result_out, void *stream)
{
    const int rc = plain(f, depth_dev, rgb_dev, K, attempt_seed, n_hypotheses, pixel_weights_dev, nullptr, result_out,
                         stream);
    if (rc) return rc;
    return result_out->status;
}

extern "C" int reloc_relocalise_learned(reloc_forest *f, const reloc_mlp *m, const uint16_t *depth_dev,
                                        const uint8_t *rgb_dev, const reloc_intrinsics *K, uint64_t attempt_seed,
                                        int32_t n_hypotheses, reloc_result *result_out, void *stream)
{
    if (!m) return RELOC_E_ARG;
    const int rc = plain(f, depth_dev, rgb_dev, K, attempt_seed, n_hypotheses, nullptr, m, result_out, stream);
    if (rc) return rc;
    return result_out->status;
}

extern "C" int reloc_relocalise(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                const reloc_intrinsics *K, uint64_t attempt_seed, int32_t n_hypotheses,
                                const uint32_t *pixel_weights_dev, double pose_c2w_out[16], float *score_out,
                                void *stream)
{
    if (!pose_c2w_out || !score_out) return RELOC_E_ARG;
    reloc_result r;
    const int rc = plain(f, depth_dev, rgb_dev, K, attempt_seed, n_hypotheses, pixel_weights_dev, nullptr, &r, stream);
    if (rc) return rc;
    memcpy(pose_c2w_out, r.pose_c2w, sizeof(r.pose_c2w));
    *score_out = r.score;
    return r.status;
}

extern "C" int reloc_debug_trace(const reloc_forest *f, reloc_trace *tr)
{
    if (!f || !tr) return RELOC_E_ARG;
    const reloc_batch *b = f->plain;
    if (!b || b->plans.empty()) return RELOC_E_STATE;
    const Plan *pl = *std::max_element(b->plans.begin(), b->plans.end(),
                                       [](Plan *x, Plan *y) { return x->last_use < y->last_use; });
    RL_HIP(hipDeviceSynchronize());
    const Attempt &A = pl->slices[0];
    const Result &o = pl->h_res[0];
    const int N = pl->shape[0].N;
    if (tr->pool_size) *tr->pool_size = o.pool_size;
    if (tr->final_hyp) *tr->final_hyp = o.final_hyp;
    if (tr->n_rounds) *tr->n_rounds = o.n_rounds;
    const int nh = std::min(N, tr->cap_hyp);
    if (tr->hyp_try) RL_HIP(hipMemcpy(tr->hyp_try, A.hyp_try, (size_t)nh * 4, hipMemcpyDeviceToHost));
    if (tr->hyp_pose) RL_HIP(hipMemcpy(tr->hyp_pose, A.hyp_init, (size_t)nh * 12 * 8, hipMemcpyDeviceToHost));
    const int nr = std::min(std::min(o.n_rounds, tr->cap_rounds), MAX_ROUNDS);
    if (tr->n_alive) RL_HIP(hipMemcpy(tr->n_alive, A.tr_n_alive, (size_t)nr * 4, hipMemcpyDeviceToHost));
    for (int r = 0; r < nr; ++r) {
        if (tr->alive)
            RL_HIP(hipMemcpy(tr->alive + (size_t)r * tr->cap_hyp, A.tr_alive + (size_t)r * N, (size_t)nh * 4,
                             hipMemcpyDeviceToHost));
        if (tr->energy)
            RL_HIP(hipMemcpy(tr->energy + (size_t)r * tr->cap_hyp, A.tr_energy + (size_t)r * N, (size_t)nh * 4,
                             hipMemcpyDeviceToHost));
    }
    return RELOC_OK;
}

// each cross-lane helper of the kernels applied to v = 1000 + lane
__global__ void __launch_bounds__(64) k_lane_probe(uint32_t *out)
{
    const int lane = __lane_id();
    const uint32_t v = 1000u + (uint32_t)lane;
    out[0 * 64 + lane] = xor_lane<1>(v);
    out[1 * 64 + lane] = xor_lane<2>(v);
    out[2 * 64 + lane] = xor_lane<4>(v);
    out[3 * 64 + lane] = xor_lane<8>(v);
    out[4 * 64 + lane] = xor_lane<16>(v);
    out[5 * 64 + lane] = xor_lane<32>(v);
    out[6 * 64 + lane] = (uint32_t)row_up<1>((int)v);
    out[7 * 64 + lane] = (uint32_t)row_up<2>((int)v);
    out[8 * 64 + lane] = (uint32_t)row_up<4>((int)v);
    out[9 * 64 + lane] = (uint32_t)row_up<8>((int)v);
    const uint64_t w = ((uint64_t)(5000u + (uint32_t)lane) << 32) | v;
    const uint64_t y[6] = {xor_lane64<1>(w), xor_lane64<2>(w), xor_lane64<4>(w),
                           xor_lane64<8>(w), xor_lane64<16>(w), xor_lane64<32>(w)};
    out[10 * 64 + lane] = (uint32_t)(y[lane % 6] >> 32);
    out[11 * 64 + lane] = (uint32_t)(lane_u64(w, 37) >> 32);
}

extern "C" int reloc_debug_lane_probe(uint32_t *out_host)
{
    if (!out_host) return RELOC_E_ARG;
    uint32_t *d = nullptr;
    if (hipMalloc((void **)&d, 12 * 64 * 4) != hipSuccess) return RELOC_E_NOMEM;
    int rc = RELOC_OK;
    hipLaunchKernelGGL(k_lane_probe, dim3(1), dim3(64), 0, 0, d);
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(out_host, d, 12 * 64 * 4, hipMemcpyDeviceToHost) != hipSuccess)
        rc = RELOC_E_HIP;
    (void)hipFree(d);
    return rc;
}

extern "C" int reloc_debug_unit_owners(int32_t xcd, int32_t total, int32_t grid, int32_t *owners_host)
{
    if (!owners_host || total < 0 || grid < 1) return RELOC_E_ARG;
    for (int u = 0; u < total; ++u) owners_host[u] = 0;
    for (int b = 0; b < grid; ++b) {
        int start, end, step;
        unit_range_of(xcd, total, (unsigned)b, (unsigned)grid, start, end, step);
        if (step < 1) return RELOC_E_STATE;
        for (int u = start; u < end; u += step) {
            if (u < 0 || u >= total) return RELOC_E_STATE;
            owners_host[u]++;
        }
    }
    return RELOC_OK;
}

extern "C" int reloc_debug_horn(const double *h_host, int32_t n, double *q_host)
{
    if (n < 0 || (n > 0 && (!h_host || !q_host))) return RELOC_E_ARG;
    for (int i = 0; i < n; ++i) {
        const double *H = h_host + (size_t)i * 9;
        double N[16];
        horn_matrix(H, N);
        double q[4];
        if (top_eigvec_horn(N, H, q)) {
            const double qn = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
            for (int k = 0; k < 4; ++k) q[k] = q[k] / qn;
        } else {
            for (int k = 0; k < 4; ++k) q[k] = NAN;
        }
        for (int k = 0; k < 4; ++k) q_host[(size_t)i * 4 + k] = q[k];
    }
    return RELOC_OK;
}

extern "C" int reloc_debug_div(const int32_t *n_host, const int32_t *den_host, int32_t count, int32_t *q_host)
{
    if (count < 0 || (count > 0 && (!n_host || !den_host || !q_host))) return RELOC_E_ARG;
    for (int32_t i = 0; i < count; ++i)
        if (den_host[i] < 1 || n_host[i] == INT32_MIN) return RELOC_E_ARG;
    for (int32_t i = 0; i < count; ++i) q_host[i] = div_trunc(n_host[i], pixel_den_of((uint32_t)den_host[i]));
    return RELOC_OK;
}

// releases a forest's plain-path batch (called when the forest is destroyed)
void rl_free_plain(Forest *f)
{
    if (f->plain) {
        reloc_batch_destroy(f->plain);
        f->plain = nullptr;
    }
}
