// Forest state on the GPU: split-node generation, features and traversal,
// online reservoir adaptation and leaf-mode extraction.
//
// Reservoir adaptation keeps the sequential definition (per tree, pixels
// offered to their leaves in raster order; Algorithm R with draws keyed by
// (tree, leaf, k)) while running every pixel in parallel: a pixel's k is its
// leaf's counter plus its stable rank among the frame's pixels in the same
// leaf, and because a slot depends only on k, each slot keeps the sample with
// the largest k that maps to it. Ranks come from an LDS sort of each 4096-pixel
// chunk plus a per-leaf prefix over chunks; "largest k wins" is an atomicMax
// on a per-slot stamp followed by the write of the single winner.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "common.h"

namespace rl {

// ---------------------------------------------------------------------------
// parameters
// ---------------------------------------------------------------------------

static void params_default(reloc_params *p)
{
    memset(p, 0, sizeof(*p));
    p->n_trees = 5; p->depth = 10; p->reservoir_size = 256; p->max_modes = 10;
    p->seed = 180108361ull;
    p->depth_min_mm = 500; p->depth_max_mm = 5000;
    p->offset_pxmm = 130000; p->f_ref_px16 = 277 * 16;
    p->thr_depth_mm = 100; p->thr_rgb = 10;
    p->dens_radius_mm = 50; p->link_radius_mm = 100; p->min_cluster = 0; p->cov_reg_mm2 = 100;
    p->n_hypotheses = 256; p->batch_pixels = 64; p->max_tries = 64; p->refine = 1; p->rgb_tol = 15;
    p->rigid_ratio2 = 1.21f; p->min_pair2_m2 = 0.01f; p->min_area2_m4 = 1e-4f;
    p->resid_m = 0.05f; p->inlier_m = 0.1f;
}

static int params_check(const reloc_params *p)
{
    if (p->n_trees < 1 || p->n_trees > 16 || p->depth < 1 || p->depth > 16) return RELOC_E_ARG;
    if (p->reservoir_size < 1 || p->reservoir_size > MAX_R || p->max_modes < 1 || p->max_modes > MAX_M ||
        p->n_trees * p->max_modes > MAX_TM)
        return RELOC_E_ARG;
    if (p->n_hypotheses < 1 || p->n_hypotheses > MAX_HYP || p->batch_pixels < 1 || p->batch_pixels > MAX_B)
        return RELOC_E_ARG;
    if (p->max_tries < 1 || p->max_tries > 1024 || p->rgb_tol < 0 || p->depth_min_mm < 1 || p->depth_max_mm > 65534 ||
        p->depth_min_mm > p->depth_max_mm || p->f_ref_px16 < 1)
        return RELOC_E_ARG;
    if (p->offset_pxmm < 0 || p->thr_depth_mm < 0 || p->thr_rgb < 0 || p->dens_radius_mm < 0 ||
        p->link_radius_mm < 0 || p->dens_radius_mm > 20000 || p->link_radius_mm > 20000 || p->cov_reg_mm2 < 1)
        return RELOC_E_ARG;
    if (p->offset_pxmm > NODE_OFF_MAX || p->thr_depth_mm > NODE_THR_MAX || p->thr_rgb > NODE_THR_MAX)
        return RELOC_E_RANGE;
    // depth denominators d * F_ref must fit 32 bits
    if ((int64_t)p->depth_max_mm * p->f_ref_px16 > 2147483647LL) return RELOC_E_RANGE;
    return RELOC_OK;
}

static int32_t focal16(float f) { return (int32_t)floor((double)f * 16.0 + 0.5); }

// intrinsics valid, width and height at most 8191, the focal lengths F in
// 1/16 px below 2^24, and |offset| * F fits 32 bits (so features stay exact)
static int frame_of(const Forest *f, const uint16_t *depth, const uint8_t *rgb, const reloc_intrinsics *K,
                    Frame &fr)
{
    if (!depth || !rgb || !K) return RELOC_E_ARG;
    if (K->width < 1 || K->height < 1 || K->width > 8191 || K->height > 8191) return RELOC_E_ARG;
    if (!(K->fx > 0.0f) || !(K->fy > 0.0f) || !isfinite(K->cx) || !isfinite(K->cy) || !isfinite(K->fx) ||
        !isfinite(K->fy))
        return RELOC_E_ARG;
    fr.depth = (decltype(fr.depth))depth; fr.rgb = (decltype(fr.rgb))rgb; fr.W = K->width; fr.H = K->height;
    fr.fx = K->fx; fr.fy = K->fy; fr.cx = K->cx; fr.cy = K->cy;
    if (!(K->fx < 1048576.0f) || !(K->fy < 1048576.0f)) return RELOC_E_ARG;
    int64_t Fx = focal16(K->fx), Fy = focal16(K->fy);
    if ((int64_t)f->p.offset_pxmm * Fx > 2147483647LL || (int64_t)f->p.offset_pxmm * Fy > 2147483647LL)
        return RELOC_E_ARG;
    // and every probe offset, at most |offset| * F / (d_min * F_ref) pixels,
    // stays below 2^14
    const int64_t den14 = ((int64_t)f->p.depth_min_mm * f->p.f_ref_px16) << 14;
    if ((int64_t)f->p.offset_pxmm * Fx >= den14 || (int64_t)f->p.offset_pxmm * Fy >= den14) return RELOC_E_ARG;
    if (Fx >= (1 << 24) || Fy >= (1 << 24)) return RELOC_E_ARG;
    fr.Fx = (int32_t)Fx; fr.Fy = (int32_t)Fy;
    fr.dmin = f->p.depth_min_mm; fr.dmax = f->p.depth_max_mm; fr.Fref = f->p.f_ref_px16;
    return RELOC_OK;
}

static bool is_se3(const double T[16])
{
    if (T[12] != 0.0 || T[13] != 0.0 || T[14] != 0.0 || T[15] != 1.0) return false;
    for (int k = 0; k < 16; ++k)
        if (!isfinite(T[k])) return false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = T[0 * 4 + a] * T[0 * 4 + b] + T[1 * 4 + a] * T[1 * 4 + b] + T[2 * 4 + a] * T[2 * 4 + b];
            if (fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6) return false;
        }
    double d = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
               T[2] * (T[4] * T[9] - T[5] * T[8]);
    return d > 0.0;
}

template <typename T>
static int dalloc(Forest *f, T **ptr, size_t count, hipStream_t s)
{
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    (void)s;
    if (hipMalloc((void **)ptr, bytes) != hipSuccess) {
        *ptr = nullptr;
        return RELOC_E_NOMEM;
    }
    f->bytes += bytes;
    return RELOC_OK;
}

template <typename T>
static void dfree(Forest *f, T **ptr, size_t count)
{
    if (*ptr) {
        (void)hipFree(*ptr);
        f->bytes -= std::max<size_t>(count * sizeof(T), sizeof(T));
        *ptr = nullptr;
    }
}

// ---------------------------------------------------------------------------
// kernels: node generation
// ---------------------------------------------------------------------------

__global__ void k_gen_nodes(uint64_t *nodes, DeepNode *deep, int T, int L, uint64_t seed, int32_t O, int32_t thr_d,
                            int32_t thr_c)
{
    int64_t n_split = (int64_t)T * (L - 1);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_split + 8) return;
    uint64_t t, node;
    if (i < n_split) {
        t = (uint64_t)(i / (L - 1));
        node = (uint64_t)(i % (L - 1));
    } else {
        t = (uint64_t)T;
        node = (uint64_t)(i - n_split);
    }
    nodes[i] = split_from_draw(philox(t, node, 0, 0, seed, TAG_FOREST), O, thr_d, thr_c);
    if (i < n_split) deep[i] = deep_node(nodes[i]);
}

// ---------------------------------------------------------------------------
// kernels: features and traversal
// ---------------------------------------------------------------------------

// one thread per (pixel, tree): blockIdx.y is the tree, so the trees' node
// chains run side by side instead of one after another
__global__ void __launch_bounds__(256) k_pack(Frame fr, uint64_t *__restrict__ packed)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < (int64_t)fr.W * fr.H) packed[p] = pack_pixel(fr, p);
}

// block (x) of 4 x 256 pixels and tree (y): each thread walks 4 pixels of
// the tree together (tid, tid + 256, ...)
constexpr int LEAF_PIX = 4;

__global__ void __launch_bounds__(256) k_leaves(const uint64_t *__restrict__ nodes, const DeepNode *__restrict__ deep,
                                                int T, int L, Frame fr, const uint64_t *__restrict__ packed,
                                                int32_t *__restrict__ leaves)
{
    __shared__ ProbeNode top[TOP_NODES];
    const int P = fr.W * fr.H;
    const int base = blockIdx.x * (LEAF_PIX * 256) + threadIdx.x;
    const int t = blockIdx.y;
    const uint64_t *tree = nodes + (int64_t)t * (L - 1);
    const int ntop = L - 1 < TOP_NODES ? L - 1 : TOP_NODES;
    stage_top(top, tree, ntop, fr, (int)threadIdx.x, (int)blockDim.x);
    __syncthreads();
    if (base >= P || t >= T) return;
    int p[LEAF_PIX];
    uint64_t own[LEAF_PIX];
    bool ok[LEAF_PIX];
#pragma unroll
    for (int k = 0; k < LEAF_PIX; ++k) {
        const int q = base + k * 256;
        p[k] = q < P ? q : P - 1;
        own[k] = packed[p[k]];
        ok[k] = q < P && packed_valid(own[k]);
    }
    int32_t leaf[LEAF_PIX];
    traverse_packed_k<LEAF_PIX>(top, ntop, deep + (int64_t)t * (L - 1), L, fr, packed, p, own, ok, leaf);
#pragma unroll
    for (int k = 0; k < LEAF_PIX; ++k)
        if (base + k * 256 < P) leaves[(int64_t)t * P + base + k * 256] = leaf[k];
}

__global__ void k_features8(const uint64_t *__restrict__ extra, Frame fr, int32_t *__restrict__ feat)
{
    int P = fr.W * fr.H;
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int u = p % fr.W, v = p / fr.W;
    uint32_t d = fr.depth[p];
    bool ok = valid_depth(fr, d);
    if (!ok) {
        for (int j = 0; j < 8; ++j) feat[(int64_t)p * 8 + j] = 0;
        return;
    }
    const PixelDen pd = pixel_den(fr, (int32_t)d);
    for (int j = 0; j < 8; ++j) {
        int32_t thr;
        feat[(int64_t)p * 8 + j] = node_response_d(fr, extra[j], u, v, (int32_t)d, pd, thr);
    }
}

// ---------------------------------------------------------------------------
// kernels: reservoir adaptation
// ---------------------------------------------------------------------------

constexpr int RANK_THREADS = 512;

// Per (chunk, tree): stable rank of each valid pixel among the chunk's pixels
// in the same leaf (bitonic sort of (leaf, local index) keys in LDS), and the
// chunk's per-leaf counts into the dense [T][C][L] table (kept zero elsewhere).
// one bitonic step at distance D < 8 over a thread's eight keys (key i = 8
// tid + e in register e), for the merge of size k
template <int D>
__device__ __forceinline__ void bitonic_in_thread(uint32_t v[8], int tid, int k)
{
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if ((e & D) == 0) {
            const bool asc = ((8 * tid + e) & k) == 0;
            const uint32_t a = v[e], b = v[e + D];
            if ((a > b) == asc) {
                v[e] = b;
                v[e + D] = a;
            }
        }
}

// the same in the strided layout (key tid + RANK_THREADS e in register e),
// for distance D RANK_THREADS
template <int D>
__device__ __forceinline__ void bitonic_strided(uint32_t v[8], int tid, int k)
{
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if ((e & D) == 0) {
            const bool asc = ((tid + RANK_THREADS * e) & k) == 0;
            const uint32_t a = v[e], b = v[e + D];
            if ((a > b) == asc) {
                v[e] = b;
                v[e + D] = a;
            }
        }
}

__global__ void __launch_bounds__(RANK_THREADS) k_chunk_rank(const int32_t *__restrict__ leaves, int P, int L,
                                                             int C, uint16_t *__restrict__ rank,
                                                             uint16_t *__restrict__ cnt)
{
    __shared__ uint32_t keys[CHUNK];
    const int c = blockIdx.x, t = blockIdx.y, tid = threadIdx.x;
    const int64_t base = (int64_t)c * CHUNK;
    // Bitonic sort with key i (of CHUNK) in register e of thread tid for
    // i = E tid + e: exchanges at distance j < E stay in the thread, those at
    // E <= j < 64 E are between lanes of one wavefront (xor shuffles), and
    // only those at j >= 64 E go through LDS between barriers.
    constexpr int E = CHUNK / RANK_THREADS;
    static_assert(E == 8, "eight keys per thread");
    uint32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = E * tid + e;
        const int64_t p = base + j;
        const int32_t leaf = p < P ? leaves[(int64_t)t * P + p] : -1;
        v[e] = leaf >= 0 ? (((uint32_t)leaf << 12) | (uint32_t)j) : 0xFFFFFFFFu;
    }
    for (int k = 2; k <= CHUNK; k <<= 1) {
        int j = k >> 1;
        if (j >= 64 * E) {
            // distances of 512 and more: through LDS into the strided layout
            // (key tid + 512 e in register e), where they are exchanges
            // inside the thread, and back
#pragma unroll
            for (int e = 0; e < E; ++e) keys[E * tid + e] = v[e];
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = keys[tid + RANK_THREADS * e];
            for (; j >= 64 * E; j >>= 1) {
                if (j == 4 * RANK_THREADS)
                    bitonic_strided<4>(v, tid, k);
                else if (j == 2 * RANK_THREADS)
                    bitonic_strided<2>(v, tid, k);
                else
                    bitonic_strided<1>(v, tid, k);
            }
#pragma unroll
            for (int e = 0; e < E; ++e) keys[tid + RANK_THREADS * e] = v[e];
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = keys[E * tid + e];
            __syncthreads();
        }
        for (; j >= E; j >>= 1) {
            const int m = j / E;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int i = E * tid + e;
                const uint32_t o = __shfl_xor(v[e], m, 64);
                v[e] = (((i & j) == 0) == ((i & k) == 0)) ? min(v[e], o) : max(v[e], o);
            }
        }
        for (; j > 0; j >>= 1) {
            if (j == 4)
                bitonic_in_thread<4>(v, tid, k);
            else if (j == 2)
                bitonic_in_thread<2>(v, tid, k);
            else
                bitonic_in_thread<1>(v, tid, k);
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) keys[E * tid + e] = v[e];
    __syncthreads();
    // A key's rank is its sorted position s minus the first position of its
    // leaf's run: the running maximum of the run starts (positions whose leaf
    // differs from the previous key's), in the thread, over the wavefront's
    // lanes and over the wavefronts.
    __shared__ uint32_t wmax[RANK_THREADS / 64];
    const int lane = tid & 63, wave = tid >> 6;
    uint32_t m[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int s = E * tid + e;
        const uint32_t prev = e > 0 ? v[e - 1] >> 12 : (s > 0 ? keys[s - 1] >> 12 : 0xFFFFFFFFu);
        const uint32_t start = (s == 0 || (v[e] >> 12) != prev) ? (uint32_t)s : 0u;
        m[e] = e > 0 ? max(m[e - 1], start) : start;
    }
    uint32_t x = m[E - 1];
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x = max(x, y);
    }
    uint32_t before = __shfl_up(x, 1, 64);
    if (lane == 0) before = 0u;
    if (lane == 63) wmax[wave] = x;
    __syncthreads();
    for (int w = 0; w < wave; ++w) before = max(before, wmax[w]);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int s = E * tid + e;
        const uint32_t key = v[e];
        if (key == 0xFFFFFFFFu) continue;
        const uint32_t leaf = key >> 12;
        const int r = s - (int)max(m[e], before);
        rank[(int64_t)t * P + base + (key & 4095u)] = (uint16_t)r;
        const uint32_t next = e + 1 < E ? v[e + 1] >> 12 : (s + 1 < CHUNK ? keys[s + 1] >> 12 : 0xFFFFFFFFu);
        if (next != leaf) cnt[((int64_t)t * C + c) * L + leaf] = (uint16_t)(r + 1);
    }
}

// Per (tree, leaf): prefix of chunk counts in chunk order, reset of the
// table, counter update, and marking of the leaf for mode extraction.
__global__ void k_leaf_scan(int T, int L, int C, uint16_t *__restrict__ cnt, uint32_t *__restrict__ pref,
                            uint32_t *__restrict__ counter, uint32_t *__restrict__ base,
                            uint32_t *__restrict__ dirty, uint32_t *__restrict__ dirty_list,
                            uint32_t *__restrict__ dirty_count, unsigned long long *__restrict__ total)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)T * L) return;
    int t = (int)(i / L), leaf = (int)(i % L);
    uint32_t run = 0;
    // chunks 16 at a time: their counts are loaded before any of them is
    // cleared (the clears would otherwise order every load after the last)
    constexpr int CB = 16;
    for (int c0 = 0; c0 < C; c0 += CB) {
        uint32_t v[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q)
            v[q] = c0 + q < C ? (uint32_t)cnt[((int64_t)t * C + c0 + q) * L + leaf] : 0u;
#pragma unroll
        for (int q = 0; q < CB; ++q)
            if (v[q]) {
                const int64_t idx = ((int64_t)t * C + c0 + q) * L + leaf;
                pref[idx] = run;
                cnt[idx] = 0;
                run += v[q];
            }
    }
    uint32_t k0 = counter[i];
    base[i] = k0;
    if (run) {
        counter[i] = k0 + run;
        if (atomicExch(&dirty[i], 1u) == 0u) {
            uint32_t pos = atomicAdd(dirty_count, 1u);
            dirty_list[pos] = (uint32_t)i;
        }
        if (t == 0) atomicAdd(total, (unsigned long long)run);
    }
}

// Per pixel: k and slot for every tree; the stamp of the slot takes the
// largest k + 1 that maps to it.
__global__ void k_slots(const int32_t *__restrict__ leaves, const uint16_t *__restrict__ rank,
                        const uint32_t *__restrict__ pref, const uint32_t *__restrict__ base, int T, int L, int R,
                        int C, int P, uint64_t seed, int32_t *__restrict__ slot, uint32_t *__restrict__ kval,
                        uint32_t *__restrict__ stamp)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int c = p / CHUNK;
    for (int t = 0; t < T; ++t) {
        int64_t ti = (int64_t)t * P + p;
        int32_t leaf = leaves[ti];
        int32_t s = -1;
        uint32_t k = 0;
        if (leaf >= 0) {
            int64_t li = (int64_t)t * L + leaf;
            k = base[li] + pref[((int64_t)t * C + c) * L + leaf] + rank[ti];
            if (k < (uint32_t)R) {
                s = (int32_t)k;
            } else {
                U4 u = philox((uint64_t)t, (uint64_t)leaf, (uint64_t)k, 0, seed, TAG_RESERVOIR);
                uint64_t j = uniform_int(u.x[0], (uint64_t)k + 1);
                if (j < (uint64_t)R) s = (int32_t)j;
            }
            if (s >= 0) atomicMax(&stamp[li * R + s], k + 1u);
        }
        slot[ti] = s;
        kval[ti] = k;
    }
}

struct Pose32 {
    float R[9], t[3];
};

// Per pixel: the winner of each slot writes the world point (integer mm,
// FP32 transform then round-half-even) and the colour.
__global__ void k_write(const int32_t *__restrict__ leaves, const int32_t *__restrict__ slot,
                        const uint32_t *__restrict__ kval, const uint32_t *__restrict__ stamp, int T, int L, int R,
                        Frame fr, Pose32 pose, Entry *__restrict__ res)
{
    int P = fr.W * fr.H;
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint32_t d = fr.depth[p];
    if (!valid_depth(fr, d)) return;
    int u = p % fr.W, v = p / fr.W;
    float c[3];
    cam_point(fr, u, v, d, c);
    Entry e;
    float w0 = ((pose.R[0] * c[0] + pose.R[1] * c[1]) + pose.R[2] * c[2]) + pose.t[0];
    float w1 = ((pose.R[3] * c[0] + pose.R[4] * c[1]) + pose.R[5] * c[2]) + pose.t[1];
    float w2 = ((pose.R[6] * c[0] + pose.R[7] * c[1]) + pose.R[8] * c[2]) + pose.t[2];
    e.x = (int32_t)rintf(w0 * 1000.0f);
    e.y = (int32_t)rintf(w1 * 1000.0f);
    e.z = (int32_t)rintf(w2 * 1000.0f);
    e.rgb = (uint32_t)fr.rgb[p * 3] | ((uint32_t)fr.rgb[p * 3 + 1] << 8) | ((uint32_t)fr.rgb[p * 3 + 2] << 16);
    for (int t = 0; t < T; ++t) {
        int64_t ti = (int64_t)t * P + p;
        int32_t s = slot[ti];
        if (s < 0) continue;
        int64_t si = ((int64_t)t * L + leaves[ti]) * R + s;
        if (stamp[si] == kval[ti] + 1u) res[si] = e;
    }
}

// ---------------------------------------------------------------------------
// kernels: leaf modes (integer quick-shift, then Gaussian statistics)
// ---------------------------------------------------------------------------

constexpr int MODE_THREADS = 256;

struct ModeParams {
    int32_t R, M, minc, rd, rl, reg;
};

// dynamic LDS of the mode kernel: 7 int32 arrays of `cap` points
static inline size_t mode_smem(int cap) { return (size_t)7 * 4 * (cap > 0 ? cap : 1); }

// One workgroup per leaf. Density and parent searches are exact integer
// comparisons on LDS-resident points; clusters are the trees of the parent
// forest (roots by pointer jumping); clusters of at least `minc` points are
// ranked by (size descending, root ascending) and the first M become modes.
__device__ void leaf_modes(const Entry *__restrict__ pts, int n, int n_total, int cap, const ModeParams mp,
                           Mode *__restrict__ out, uint32_t *__restrict__ rgb_out, int rgb_len,
                           int32_t *__restrict__ n_out, char *smem)
{
    int32_t *X = (int32_t *)smem;
    int32_t *Y = X + cap;
    int32_t *Z = Y + cap;
    int32_t *rho = Z + cap;
    int32_t *par = rho + cap;
    int32_t *size = par + cap;
    uint32_t *col = (uint32_t *)(size + cap);
    __shared__ int32_t cand_root[MAX_R];
    __shared__ int32_t n_cand;
    __shared__ unsigned long long acc[MAX_M][13];
    __shared__ int32_t n_modes;
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += MODE_THREADS) {
        Entry e = pts[i];
        X[i] = e.x; Y[i] = e.y; Z[i] = e.z; col[i] = e.rgb;
        size[i] = 0;
    }
    if (tid == 0) n_cand = 0;
    for (int i = tid; i < MAX_M * 13; i += MODE_THREADS) acc[i / 13][i % 13] = 0ull;
    __syncthreads();
    const int rd = mp.rd, rl = mp.rl;
    const int rd2 = rd * rd, rl2 = rl * rl;
    for (int i = tid; i < n; i += MODE_THREADS) {
        int xi = X[i], yi = Y[i], zi = Z[i], cnt = 0;
        for (int j = 0; j < n; ++j) {
            int dx = X[j] - xi, dy = Y[j] - yi, dz = Z[j] - zi;
            if (abs(dx) <= rd && abs(dy) <= rd && abs(dz) <= rd && dx * dx + dy * dy + dz * dz <= rd2) cnt++;
        }
        rho[i] = cnt;
    }
    __syncthreads();
    for (int i = tid; i < n; i += MODE_THREADS) {
        int xi = X[i], yi = Y[i], zi = Z[i], ri = rho[i];
        int best = -1, bd = 0;
        for (int j = 0; j < n; ++j) {
            int dx = X[j] - xi, dy = Y[j] - yi, dz = Z[j] - zi;
            if (abs(dx) > rl || abs(dy) > rl || abs(dz) > rl) continue;
            int d2 = dx * dx + dy * dy + dz * dz;
            if (d2 > rl2 || j == i) continue;
            int rj = rho[j];
            if (!(rj > ri || (rj == ri && j < i))) continue;
            if (best < 0 || d2 < bd || (d2 == bd && j < best)) {
                best = j;
                bd = d2;
            }
        }
        par[i] = best;
    }
    __syncthreads();
    // pointer jumping: par[i] becomes the root of i
    for (int it = 0; it < 13; ++it) {
        for (int i = tid; i < n; i += MODE_THREADS) {
            int a = par[i];
            if (a >= 0) {
                int b = par[a];
                if (b >= 0) par[i] = b;
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += MODE_THREADS) {
        int r = par[i] < 0 ? i : par[i];
        atomicAdd(&size[r], 1);
    }
    __syncthreads();
    for (int i = tid; i < n; i += MODE_THREADS)
        if (par[i] < 0 && size[i] >= mp.minc) {
            int k = atomicAdd(&n_cand, 1);
            cand_root[k] = i;
        }
    __syncthreads();
    // rank candidates by (size desc, root asc); rank < M becomes the mode slot
    // (stored in rho[], which is no longer needed)
    int nc = n_cand;
    for (int i = tid; i < n; i += MODE_THREADS) rho[i] = -1;
    __syncthreads();
    for (int a = tid; a < nc; a += MODE_THREADS) {
        int ra = cand_root[a], sa = size[ra], rank = 0;
        for (int b = 0; b < nc; ++b) {
            int rb = cand_root[b], sb = size[rb];
            if (sb > sa || (sb == sa && rb < ra)) rank++;
        }
        if (rank < mp.M) rho[ra] = rank;
    }
    if (tid == 0) n_modes = nc < mp.M ? nc : mp.M;
    __syncthreads();
    for (int i = tid; i < n; i += MODE_THREADS) {
        int r = par[i] < 0 ? i : par[i];
        int m = rho[r];
        if (m < 0) continue;
        int64_t x = X[i], y = Y[i], z = Z[i];
        uint32_t cl = col[i];
        atomicAdd(&acc[m][0], (unsigned long long)x);
        atomicAdd(&acc[m][1], (unsigned long long)y);
        atomicAdd(&acc[m][2], (unsigned long long)z);
        atomicAdd(&acc[m][3], (unsigned long long)(x * x));
        atomicAdd(&acc[m][4], (unsigned long long)(x * y));
        atomicAdd(&acc[m][5], (unsigned long long)(x * z));
        atomicAdd(&acc[m][6], (unsigned long long)(y * y));
        atomicAdd(&acc[m][7], (unsigned long long)(y * z));
        atomicAdd(&acc[m][8], (unsigned long long)(z * z));
        atomicAdd(&acc[m][9], (unsigned long long)(cl & 255u));
        atomicAdd(&acc[m][10], (unsigned long long)((cl >> 8) & 255u));
        atomicAdd(&acc[m][11], (unsigned long long)((cl >> 16) & 255u));
        atomicAdd(&acc[m][12], 1ull);
    }
    __syncthreads();
    int nm = n_modes;
    if (tid < nm) {
        const unsigned long long *a = acc[tid];
        int64_t Sx[3] = {(int64_t)a[0], (int64_t)a[1], (int64_t)a[2]};
        int64_t Sxx[6] = {(int64_t)a[3], (int64_t)a[4], (int64_t)a[5], (int64_t)a[6], (int64_t)a[7], (int64_t)a[8]};
        int64_t nmm = (int64_t)a[12];
        Mode md;
        double dn = (double)nmm;
        for (int k = 0; k < 3; ++k) md.mu[k] = (float)((double)Sx[k] / (dn * 1000.0));
        const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
        double S[6];
        for (int e = 0; e < 6; ++e) {
            int64_t num = nmm * Sxx[e] - Sx[ia[e]] * Sx[ib[e]];
            double cv = (double)num / (dn * dn);
            if (ia[e] == ib[e]) cv = cv + (double)mp.reg;
            S[e] = cv * 1e-6;
        }
        double A = S[0], B = S[1], Cc = S[2], Dd = S[3], E = S[4], G = S[5];
        double A00 = Dd * G - E * E;
        double A01 = Cc * E - B * G;
        double A02 = B * E - Cc * Dd;
        double A11 = A * G - Cc * Cc;
        double A12 = B * Cc - A * E;
        double A22 = A * Dd - B * B;
        double det = (A * A00 + B * A01) + Cc * A02;
        md.sinv[0] = (float)(A00 / det);
        md.sinv[1] = (float)(A01 / det);
        md.sinv[2] = (float)(A02 / det);
        md.sinv[3] = (float)(A11 / det);
        md.sinv[4] = (float)(A12 / det);
        md.sinv[5] = (float)(A22 / det);
        md.kappa = (float)(-log(dn / (double)n_total) + 0.5 * (3.0 * log(2.0 * M_PI) + log(det)));
        md.n = (int32_t)nmm;
        md.rgb = (uint32_t)(a[9] / (unsigned long long)nmm) | ((uint32_t)(a[10] / (unsigned long long)nmm) << 8) |
                 ((uint32_t)(a[11] / (unsigned long long)nmm) << 16);
        out[tid] = md;
        if (rgb_out) rgb_out[tid] = md.rgb;
    } else if (rgb_out && tid < rgb_len) {
        rgb_out[tid] = RGB_NONE;
    }
    if (tid == 0) *n_out = nm;
    __syncthreads();
}

// persistent over the dirty-leaf list; also refreshes each leaf's summary
// for the learned proposal's inputs: {min(k, R), number of modes kept (<= 3)}
// and, for its first three modes (the heaviest: modes are ranked by size),
// {pi = n / min(k, R), -log(Sigma^-1_xx) / 10, -log(Sigma^-1_yy) / 10,
// -log(Sigma^-1_zz) / 10}
__global__ void __launch_bounds__(MODE_THREADS) k_modes(const uint32_t *__restrict__ list,
                                                        const uint32_t *__restrict__ count,
                                                        const uint32_t *__restrict__ counter,
                                                        const Entry *__restrict__ res, ModeParams mp,
                                                        Mode *__restrict__ modes, uint32_t *__restrict__ mode_rgb,
                                                        int32_t *__restrict__ nmodes, float4 *__restrict__ leaf_in)
{
    extern __shared__ char smem[];
    uint32_t n_list = *count;
    for (uint32_t it = blockIdx.x; it < n_list; it += gridDim.x) {
        uint32_t li = list[it];
        uint32_t k = counter[li];
        int n = k < (uint32_t)mp.R ? (int)k : mp.R;
        const int ms = rgb_stride(mp.M);
        leaf_modes(res + (int64_t)li * mp.R, n, n, mp.R, mp, modes + (int64_t)li * mp.M, mode_rgb + (int64_t)li * ms, ms,
                   nmodes + li, smem);
        // leaf_modes ends with a barrier: the modes and their count are visible
        const int tid = (int)threadIdx.x;
        if (tid < 4) {
            const int nm = nmodes[li];
            const int n3 = nm < 3 ? nm : 3;
            float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (tid == 0) {
                q.x = __uint_as_float((uint32_t)n);
                q.y = __int_as_float(n3);
            } else if (tid - 1 < n3) {
                const Mode md = modes[(int64_t)li * mp.M + tid - 1];
                q.x = (float)md.n / (float)n;
                q.y = -logf(md.sinv[0]) / 10.0f;
                q.z = -logf(md.sinv[3]) / 10.0f;
                q.w = -logf(md.sinv[5]) / 10.0f;
            }
            leaf_in[(int64_t)li * 4 + tid] = q;
        }
        __syncthreads();
    }
}

__global__ void k_modes_done(const uint32_t *__restrict__ list, uint32_t *__restrict__ count,
                             uint32_t *__restrict__ dirty)
{
    uint32_t n = *count;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dirty[list[i]] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) *count = 0u;
}

__global__ void __launch_bounds__(MODE_THREADS) k_modes_points(const Entry *__restrict__ pts, int n, ModeParams mp,
                                                               Mode *__restrict__ out, int32_t *__restrict__ n_out)
{
    extern __shared__ char smem[];
    leaf_modes(pts, n, n, n, mp, out, nullptr, 0, n_out, smem);
}

static ModeParams mode_params(const Forest *f)
{
    ModeParams mp;
    mp.R = f->R;
    mp.M = f->M;
    mp.minc = f->p.min_cluster > 0 ? f->p.min_cluster : std::max(3, f->R / 64);
    mp.rd = f->p.dens_radius_mm;
    mp.rl = f->p.link_radius_mm;
    mp.reg = f->p.cov_reg_mm2;
    return mp;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int ensure_frame_scratch(Forest *f, int64_t P, hipStream_t s)
{
    if (P <= f->cap_P) return RELOC_OK;
    int64_t C_old = (f->cap_P + CHUNK - 1) / CHUNK;
    dfree(f, &f->leaves, (size_t)f->T * f->cap_P);
    dfree(f, &f->packed, (size_t)f->cap_P);
    dfree(f, &f->rank, (size_t)f->T * f->cap_P);
    dfree(f, &f->slot, (size_t)f->T * f->cap_P);
    dfree(f, &f->kval, (size_t)f->T * f->cap_P);
    dfree(f, &f->chunk_cnt, (size_t)f->T * C_old * f->L);
    dfree(f, &f->chunk_pref, (size_t)f->T * C_old * f->L);
    f->cap_P = 0;
    int64_t C = (P + CHUNK - 1) / CHUNK;
    int rc = RELOC_OK;
    rc |= dalloc(f, &f->leaves, (size_t)f->T * P, s);
    rc |= dalloc(f, &f->packed, (size_t)P, s);
    rc |= dalloc(f, &f->rank, (size_t)f->T * P, s);
    rc |= dalloc(f, &f->slot, (size_t)f->T * P, s);
    rc |= dalloc(f, &f->kval, (size_t)f->T * P, s);
    rc |= dalloc(f, &f->chunk_cnt, (size_t)f->T * C * f->L, s);
    rc |= dalloc(f, &f->chunk_pref, (size_t)f->T * C * f->L, s);
    if (rc) return RELOC_E_NOMEM;
    RL_HIP(hipMemsetAsync(f->chunk_cnt, 0, (size_t)f->T * C * f->L * sizeof(uint16_t), s));
    f->cap_P = P;
    return RELOC_OK;
}

int update_modes(Forest *f, hipStream_t s)
{
    if (!f->maybe_dirty) return RELOC_OK;
    if (!f->res) return RELOC_E_STATE;
    ModeParams mp = mode_params(f);
    int grid = std::min(f->T * f->L, 4096);
    RL_LAUNCH("k_modes", k_modes, dim3(grid), dim3(MODE_THREADS), mode_smem(f->R), s, f->dirty_list, f->dirty_count,
                       f->counter, f->res, mp, f->modes, f->mode_rgb, f->nmodes, f->leaf_in);
    RL_LAUNCH("k_modes_done", k_modes_done, dim3(1), dim3(1024), 0, s, f->dirty_list, f->dirty_count, f->dirty);
    RL_HIP(hipGetLastError());
    f->maybe_dirty = false;
    return RELOC_OK;
}

int traverse_frame(Forest *f, const Frame &fr, hipStream_t s)
{
    int64_t P = (int64_t)fr.W * fr.H;
    int rc = ensure_frame_scratch(f, P, s);
    if (rc) return rc;
    RL_LAUNCH("k_pack", k_pack, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, fr, f->packed);
    RL_LAUNCH("k_leaves", k_leaves, dim3((unsigned)((P + LEAF_PIX * 256 - 1) / (LEAF_PIX * 256)), (unsigned)f->T),
              dim3(256), 0, s, f->nodes, f->deep, f->T, f->L, fr, f->packed, f->leaves);
    RL_HIP(hipGetLastError());
    return RELOC_OK;
}

int frame_from(const Forest *f, const uint16_t *depth, const uint8_t *rgb, const reloc_intrinsics *K, Frame &fr)
{
    return frame_of(f, depth, rgb, K, fr);
}

bool pose_is_se3(const double T[16]) { return is_se3(T); }

// every leaf of a forest empty again (the state of a new forest): counters,
// reservoirs, slot stamps, modes, the learned proposal's leaf summaries,
// the dirty list and the sample count
int forest_empty_leaves(Forest *f, hipStream_t s)
{
    const size_t TL = (size_t)f->T * f->L;
    if (f->dropped) return RELOC_E_STATE;
    if (hipMemsetAsync(f->counter, 0, TL * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->stamp, 0, TL * f->R * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->res, 0, TL * f->R * sizeof(Entry), s) != hipSuccess ||
        hipMemsetAsync(f->nmodes, 0, TL * sizeof(int32_t), s) != hipSuccess ||
        hipMemsetAsync(f->mode_rgb, 0xFF, TL * rgb_stride(f->M) * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->leaf_in, 0, TL * 4 * sizeof(float4), s) != hipSuccess ||
        hipMemsetAsync(f->dirty, 0, TL * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->dirty_count, 0, sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->total_samples, 0, sizeof(unsigned long long), s) != hipSuccess)
        return RELOC_E_HIP;
    f->maybe_dirty = false;
    return RELOC_OK;
}

}  // namespace rl

using namespace rl;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" int reloc_params_default(reloc_params *out)
{
    if (!out) return RELOC_E_ARG;
    params_default(out);
    return RELOC_OK;
}

extern "C" const char *reloc_status_string(int code)
{
    switch (code) {
    case RELOC_OK: return "ok";
    case RELOC_FAIL_NO_VALID_PIXELS: return "relocalisation failed: no valid depth in the frame";
    case RELOC_FAIL_NO_MODES: return "relocalisation failed: the forest has never been adapted";
    case RELOC_FAIL_NO_HYPOTHESIS: return "relocalisation failed: no hypothesis passed its checks";
    case RELOC_E_ARG: return "invalid argument";
    case RELOC_E_NOMEM: return "device allocation failed";
    case RELOC_E_HIP: return "HIP runtime error";
    case RELOC_E_STATE: return "operation not valid in this state";
    case RELOC_E_RANGE: return "value does not fit the packed device layout";
    case RELOC_E_IO: return "checkpoint file cannot be written or read, or is not a forest checkpoint";
    default: return "unknown status";
    }
}

static void forest_free(Forest *f)
{
    int64_t C = (f->cap_P + CHUNK - 1) / CHUNK;
    size_t TL = (size_t)f->T * f->L;
    dfree(f, &f->nodes, (size_t)f->T * (f->L - 1) + 8);
    dfree(f, &f->deep, (size_t)f->T * (f->L - 1));
    dfree(f, &f->counter, TL);
    dfree(f, &f->base, TL);
    dfree(f, &f->res, TL * f->R);
    dfree(f, &f->stamp, TL * f->R);
    dfree(f, &f->modes, TL * f->M);
    dfree(f, &f->nmodes, TL);
    dfree(f, &f->dirty, TL);
    dfree(f, &f->dirty_list, TL);
    dfree(f, &f->dirty_count, 1);
    dfree(f, &f->total_samples, 1);
    dfree(f, &f->leaves, (size_t)f->T * f->cap_P);
    dfree(f, &f->packed, (size_t)f->cap_P);
    dfree(f, &f->rank, (size_t)f->T * f->cap_P);
    dfree(f, &f->slot, (size_t)f->T * f->cap_P);
    dfree(f, &f->kval, (size_t)f->T * f->cap_P);
    dfree(f, &f->chunk_cnt, (size_t)f->T * C * f->L);
    dfree(f, &f->chunk_pref, (size_t)f->T * C * f->L);
    dfree(f, &f->mode_rgb, TL * rgb_stride(f->M));
    dfree(f, &f->leaf_in, TL * 4);
}

extern "C" int reloc_forest_create(const reloc_params *p, void *stream, reloc_forest **out)
{
    if (!p || !out) return RELOC_E_ARG;
    *out = nullptr;
    int rc = params_check(p);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    reloc_forest *f = new (std::nothrow) reloc_forest();
    if (!f) return RELOC_E_NOMEM;
    f->p = *p;
    f->T = p->n_trees; f->D = p->depth; f->L = 1 << p->depth; f->R = p->reservoir_size; f->M = p->max_modes;
    if (hipGetDevice(&f->device) != hipSuccess) { delete f; return RELOC_E_HIP; }
    size_t TL = (size_t)f->T * f->L;
    rc = RELOC_OK;
    rc |= dalloc(f, &f->nodes, (size_t)f->T * (f->L - 1) + 8, s);
    rc |= dalloc(f, &f->deep, (size_t)f->T * (f->L - 1), s);
    rc |= dalloc(f, &f->counter, TL, s);
    rc |= dalloc(f, &f->base, TL, s);
    rc |= dalloc(f, &f->res, TL * f->R, s);
    rc |= dalloc(f, &f->stamp, TL * f->R, s);
    rc |= dalloc(f, &f->modes, TL * f->M, s);
    rc |= dalloc(f, &f->nmodes, TL, s);
    rc |= dalloc(f, &f->dirty, TL, s);
    rc |= dalloc(f, &f->dirty_list, TL, s);
    rc |= dalloc(f, &f->dirty_count, 1, s);
    rc |= dalloc(f, &f->total_samples, 1, s);
    rc |= dalloc(f, &f->mode_rgb, TL * rgb_stride(f->M), s);
    rc |= dalloc(f, &f->leaf_in, TL * 4, s);
    if (rc) {
        forest_free(f);
        delete f;
        return RELOC_E_NOMEM;
    }
    if (hipMemsetAsync(f->counter, 0, TL * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->stamp, 0, TL * f->R * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->res, 0, TL * f->R * sizeof(Entry), s) != hipSuccess ||
        hipMemsetAsync(f->nmodes, 0, TL * sizeof(int32_t), s) != hipSuccess ||
        hipMemsetAsync(f->mode_rgb, 0xFF, TL * rgb_stride(f->M) * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->leaf_in, 0, TL * 4 * sizeof(float4), s) != hipSuccess ||
        hipMemsetAsync(f->dirty, 0, TL * sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->dirty_count, 0, sizeof(uint32_t), s) != hipSuccess ||
        hipMemsetAsync(f->total_samples, 0, sizeof(unsigned long long), s) != hipSuccess) {
        forest_free(f);
        delete f;
        return RELOC_E_HIP;
    }
    int64_t nn = (int64_t)f->T * (f->L - 1) + 8;
    RL_LAUNCH("k_gen_nodes", k_gen_nodes, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, f->nodes, f->deep, f->T, f->L,
                       p->seed, p->offset_pxmm, p->thr_depth_mm, p->thr_rgb);
    if (hipGetLastError() != hipSuccess) {
        forest_free(f);
        delete f;
        return RELOC_E_HIP;
    }
    *out = f;
    return RELOC_OK;
}

extern "C" int reloc_forest_destroy(reloc_forest *f)
{
    if (!f) return RELOC_E_ARG;
    (void)hipDeviceSynchronize();
    rl_free_plain(f);
    forest_free(f);
    delete f;
    return RELOC_OK;
}

extern "C" int reloc_forest_params(const reloc_forest *f, reloc_params *out)
{
    if (!f || !out) return RELOC_E_ARG;
    *out = f->p;
    return RELOC_OK;
}

extern "C" int reloc_forest_memory(const reloc_forest *f, uint64_t *bytes_out)
{
    if (!f || !bytes_out) return RELOC_E_ARG;
    *bytes_out = f->bytes;
    return RELOC_OK;
}

extern "C" int reloc_adapt_frame(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                 const reloc_intrinsics *K, const double pose_c2w[16], void *stream)
{
    if (!f || !pose_c2w) return RELOC_E_ARG;
    if (f->dropped) return RELOC_E_STATE;
    Frame fr;
    int rc = frame_of(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    if (!is_se3(pose_c2w)) return RELOC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    int64_t P = (int64_t)fr.W * fr.H;
    rc = traverse_frame(f, fr, s);
    if (rc) return rc;
    int C = (int)((P + CHUNK - 1) / CHUNK);
    RL_LAUNCH("k_chunk_rank", k_chunk_rank, dim3(C, f->T), dim3(RANK_THREADS), 0, s, f->leaves, (int)P, f->L, C, f->rank,
                       f->chunk_cnt);
    int64_t TL = (int64_t)f->T * f->L;
    RL_LAUNCH("k_leaf_scan", k_leaf_scan, dim3((unsigned)((TL + 255) / 256)), dim3(256), 0, s, f->T, f->L, C,
                       f->chunk_cnt, f->chunk_pref, f->counter, f->base, f->dirty, f->dirty_list, f->dirty_count,
                       f->total_samples);
    RL_LAUNCH("k_slots", k_slots, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, f->leaves, f->rank,
                       f->chunk_pref, f->base, f->T, f->L, f->R, C, (int)P, f->p.seed, f->slot, f->kval, f->stamp);
    Pose32 ps;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) ps.R[r * 3 + c] = (float)pose_c2w[r * 4 + c];
        ps.t[r] = (float)pose_c2w[r * 4 + 3];
    }
    RL_LAUNCH("k_write", k_write, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, f->leaves, f->slot, f->kval,
                       f->stamp, f->T, f->L, f->R, fr, ps, f->res);
    RL_HIP(hipGetLastError());
    f->maybe_dirty = true;
    return RELOC_OK;
}

extern "C" int reloc_update_modes(reloc_forest *f, void *stream)
{
    if (!f) return RELOC_E_ARG;
    return update_modes(f, (hipStream_t)stream);
}

extern "C" int reloc_forest_drop_reservoirs(reloc_forest *f, void *stream)
{
    if (!f) return RELOC_E_ARG;
    if (f->dropped) return RELOC_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc = update_modes(f, s);
    if (rc) return rc;
    RL_HIP(hipStreamSynchronize(s));
    size_t TLR = (size_t)f->T * f->L * f->R;
    dfree(f, &f->res, TLR);
    dfree(f, &f->stamp, TLR);
    f->dropped = true;
    return RELOC_OK;
}

// ---- checkpoint: save and load ---------------------------------------------
//
// File layout (little-endian, this library's own format): a FileHeader, then
// the split nodes (u64 [T (L - 1) + 8]), leaf counters (u32 [T L]), mode
// counts (i32 [T L]), modes (Mode [T L M]), mode colour rows
// (u32 [T L rgb_stride(M)]), learned-input leaf summaries (float4 [T L 4])
// and, unless the reservoirs were dropped, the reservoirs (Entry [T L R]).
// Slot stamps are not stored: a stamp only has to be below every k + 1 that
// later frames can produce, and every later k is at least the leaf's counter,
// so the zero stamps of a new forest select the same winners.

namespace {

struct FileHeader {
    char magic[8];
    uint32_t version;
    uint32_t dropped;
    reloc_params p;
    uint64_t total_samples;
    uint64_t n_nodes, n_leaves, n_mode_slots, n_rgb, n_res;
};

constexpr char FILE_MAGIC[8] = {'R', 'L', 'F', 'O', 'R', 'E', 'S', 'T'};
constexpr uint32_t FILE_VERSION = 1;
constexpr size_t STAGE_BYTES = (size_t)64 << 20;

struct Staging {
    void *buf = nullptr;
    ~Staging()
    {
        if (buf) (void)hipHostFree(buf);
    }
};

// device -> file in chunks through pinned host memory
int save_section(FILE *fp, const void *dev, size_t bytes, Staging &st, hipStream_t s)
{
    const char *src = (const char *)dev;
    for (size_t off = 0; off < bytes; off += STAGE_BYTES) {
        const size_t n = std::min(STAGE_BYTES, bytes - off);
        RL_HIP(hipMemcpyAsync(st.buf, src + off, n, hipMemcpyDeviceToHost, s));
        RL_HIP(hipStreamSynchronize(s));
        if (fwrite(st.buf, 1, n, fp) != n) return RELOC_E_IO;
    }
    return RELOC_OK;
}

// file -> device in chunks through pinned host memory
int load_section(FILE *fp, void *dev, size_t bytes, Staging &st, hipStream_t s)
{
    char *dst = (char *)dev;
    for (size_t off = 0; off < bytes; off += STAGE_BYTES) {
        const size_t n = std::min(STAGE_BYTES, bytes - off);
        RL_HIP(hipStreamSynchronize(s));   // the previous chunk has left the staging buffer
        if (fread(st.buf, 1, n, fp) != n) return RELOC_E_IO;
        RL_HIP(hipMemcpyAsync(dst + off, st.buf, n, hipMemcpyHostToDevice, s));
    }
    RL_HIP(hipStreamSynchronize(s));
    return RELOC_OK;
}

FileHeader header_of(const Forest *f)
{
    FileHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, FILE_MAGIC, sizeof(FILE_MAGIC));
    h.version = FILE_VERSION;
    h.dropped = f->dropped ? 1u : 0u;
    h.p = f->p;
    const uint64_t TL = (uint64_t)f->T * f->L;
    h.n_nodes = (uint64_t)f->T * (f->L - 1) + 8;
    h.n_leaves = TL;
    h.n_mode_slots = TL * f->M;
    h.n_rgb = TL * rgb_stride(f->M);
    h.n_res = f->dropped ? 0 : TL * f->R;
    return h;
}

int save_forest(Forest *f, FILE *fp, hipStream_t s)
{
    int rc = update_modes(f, s);
    if (rc) return rc;
    Staging st;
    RL_HIP(hipHostMalloc(&st.buf, STAGE_BYTES, hipHostMallocDefault));
    FileHeader h = header_of(f);
    RL_HIP(hipMemcpyAsync(&h.total_samples, f->total_samples, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    RL_HIP(hipStreamSynchronize(s));
    if (fwrite(&h, sizeof(h), 1, fp) != 1) return RELOC_E_IO;
    if ((rc = save_section(fp, f->nodes, h.n_nodes * sizeof(uint64_t), st, s))) return rc;
    if ((rc = save_section(fp, f->counter, h.n_leaves * sizeof(uint32_t), st, s))) return rc;
    if ((rc = save_section(fp, f->nmodes, h.n_leaves * sizeof(int32_t), st, s))) return rc;
    if ((rc = save_section(fp, f->modes, h.n_mode_slots * sizeof(Mode), st, s))) return rc;
    if ((rc = save_section(fp, f->mode_rgb, h.n_rgb * sizeof(uint32_t), st, s))) return rc;
    if ((rc = save_section(fp, f->leaf_in, h.n_leaves * 4 * sizeof(float4), st, s))) return rc;
    if (!f->dropped && (rc = save_section(fp, f->res, h.n_res * sizeof(Entry), st, s))) return rc;
    return RELOC_OK;
}

int load_forest(FILE *fp, hipStream_t s, reloc_forest **out)
{
    FileHeader h;
    if (fread(&h, sizeof(h), 1, fp) != 1) return RELOC_E_IO;
    if (memcmp(h.magic, FILE_MAGIC, sizeof(FILE_MAGIC)) != 0 || h.version != FILE_VERSION || h.dropped > 1u)
        return RELOC_E_IO;
    reloc_forest *f = nullptr;
    int rc = reloc_forest_create(&h.p, s, &f);
    if (rc) return rc;
    const FileHeader want = [&] {
        FileHeader w = header_of(f);
        if (h.dropped) w.n_res = 0;
        return w;
    }();
    if (h.n_nodes != want.n_nodes || h.n_leaves != want.n_leaves || h.n_mode_slots != want.n_mode_slots ||
        h.n_rgb != want.n_rgb || h.n_res != want.n_res) {
        reloc_forest_destroy(f);
        return RELOC_E_IO;
    }
    Staging st;
    std::vector<uint64_t> nodes(h.n_nodes);
    std::vector<DeepNode> deep((size_t)f->T * (f->L - 1));
    rc = hipHostMalloc(&st.buf, STAGE_BYTES, hipHostMallocDefault) == hipSuccess ? RELOC_OK : RELOC_E_NOMEM;
    if (!rc && fread(nodes.data(), sizeof(uint64_t), nodes.size(), fp) != nodes.size()) rc = RELOC_E_IO;
    if (!rc) {
        // split nodes are checked like reloc_debug_set_nodes checks them
        for (size_t i = 0; i < nodes.size() && !rc; ++i) {
            int32_t kind, dx, dy, thr;
            unpack_node(nodes[i], kind, dx, dy, thr);
            if (kind < 0 || kind > 3 || (int64_t)std::abs((int64_t)dx) > f->p.offset_pxmm ||
                (int64_t)std::abs((int64_t)dy) > f->p.offset_pxmm || pack_node(kind, dx, dy, thr) != nodes[i])
                rc = RELOC_E_RANGE;
        }
        for (size_t i = 0; i < deep.size() && !rc; ++i) deep[i] = deep_node(nodes[i]);
    }
    if (!rc && (hipMemcpyAsync(f->nodes, nodes.data(), nodes.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s) !=
                    hipSuccess ||
                hipMemcpyAsync(f->deep, deep.data(), deep.size() * sizeof(DeepNode), hipMemcpyHostToDevice, s) !=
                    hipSuccess ||
                hipMemcpyAsync(f->total_samples, &h.total_samples, sizeof(uint64_t), hipMemcpyHostToDevice, s) !=
                    hipSuccess))
        rc = RELOC_E_HIP;
    if (!rc) rc = load_section(fp, f->counter, h.n_leaves * sizeof(uint32_t), st, s);
    if (!rc) rc = load_section(fp, f->nmodes, h.n_leaves * sizeof(int32_t), st, s);
    if (!rc) rc = load_section(fp, f->modes, h.n_mode_slots * sizeof(Mode), st, s);
    if (!rc) rc = load_section(fp, f->mode_rgb, h.n_rgb * sizeof(uint32_t), st, s);
    if (!rc) rc = load_section(fp, f->leaf_in, h.n_leaves * 4 * sizeof(float4), st, s);
    if (!rc && !h.dropped) rc = load_section(fp, f->res, h.n_res * sizeof(Entry), st, s);
    if (!rc && fgetc(fp) != EOF) rc = RELOC_E_IO;   // trailing bytes: not a file this version wrote
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = RELOC_E_HIP;
    if (!rc && h.dropped) {
        const size_t TLR = (size_t)f->T * f->L * f->R;
        dfree(f, &f->res, TLR);
        dfree(f, &f->stamp, TLR);
        f->dropped = true;
    }
    if (rc) {
        reloc_forest_destroy(f);
        return rc;
    }
    f->maybe_dirty = false;
    *out = f;
    return RELOC_OK;
}

}  // namespace

extern "C" int reloc_forest_save(reloc_forest *f, const char *path, void *stream)
{
    if (!f || !path) return RELOC_E_ARG;
    FILE *fp = fopen(path, "wb");
    if (!fp) return RELOC_E_IO;
    int rc = save_forest(f, fp, (hipStream_t)stream);
    if (fclose(fp) != 0 && !rc) rc = RELOC_E_IO;
    return rc;
}

extern "C" int reloc_forest_load(const char *path, void *stream, reloc_forest **out)
{
    if (!path || !out) return RELOC_E_ARG;
    *out = nullptr;
    FILE *fp = fopen(path, "rb");
    if (!fp) return RELOC_E_IO;
    const int rc = load_forest(fp, (hipStream_t)stream, out);
    fclose(fp);
    return rc;
}

// ---- debug exports --------------------------------------------------------

extern "C" int reloc_debug_nodes(const reloc_forest *f, int32_t *kind, int32_t *dx, int32_t *dy, int32_t *thr)
{
    if (!f) return RELOC_E_ARG;
    size_t n = (size_t)f->T * (f->L - 1) + 8;
    uint64_t *h = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (!h) return RELOC_E_NOMEM;
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(h, f->nodes, n * 8, hipMemcpyDeviceToHost) != hipSuccess) {
        free(h);
        return RELOC_E_HIP;
    }
    for (size_t i = 0; i < n; ++i) {
        int32_t a, b, c, d;
        unpack_node(h[i], a, b, c, d);
        if (kind) kind[i] = a;
        if (dx) dx[i] = b;
        if (dy) dy[i] = c;
        if (thr) thr[i] = d;
    }
    free(h);
    return RELOC_OK;
}

extern "C" int reloc_debug_set_nodes(reloc_forest *f, const int32_t *kind, const int32_t *dx, const int32_t *dy,
                                     const int32_t *thr)
{
    if (!f || !kind || !dx || !dy || !thr) return RELOC_E_ARG;
    size_t n = (size_t)f->T * (f->L - 1) + 8;
    uint64_t *h = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (!h) return RELOC_E_NOMEM;
    for (size_t i = 0; i < n; ++i) {
        if (kind[i] < 0 || kind[i] > 3 || dx[i] < -NODE_OFF_MAX - 1 || dx[i] > NODE_OFF_MAX ||
            dy[i] < -NODE_OFF_MAX - 1 || dy[i] > NODE_OFF_MAX || thr[i] < -NODE_THR_MAX - 1 || thr[i] > NODE_THR_MAX ||
            (int64_t)std::abs((int64_t)dx[i]) > f->p.offset_pxmm || (int64_t)std::abs((int64_t)dy[i]) > f->p.offset_pxmm) {
            free(h);
            return RELOC_E_RANGE;
        }
        h[i] = pack_node(kind[i], dx[i], dy[i], thr[i]);
    }
    const size_t ns = (size_t)f->T * (f->L - 1);
    DeepNode *hd = (DeepNode *)malloc(ns * sizeof(DeepNode));
    if (!hd) {
        free(h);
        return RELOC_E_NOMEM;
    }
    for (size_t i = 0; i < ns; ++i) hd[i] = deep_node(h[i]);
    int rc = RELOC_OK;
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(f->nodes, h, n * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(f->deep, hd, ns * sizeof(DeepNode), hipMemcpyHostToDevice) != hipSuccess)
        rc = RELOC_E_HIP;
    free(hd);
    free(h);
    return rc;
}

extern "C" int reloc_debug_leaves(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                  const reloc_intrinsics *K, int32_t *leaves_host, void *stream)
{
    if (!f || !leaves_host) return RELOC_E_ARG;
    Frame fr;
    int rc = frame_of(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    rc = traverse_frame(f, fr, s);
    if (rc) return rc;
    int64_t P = (int64_t)fr.W * fr.H;
    RL_HIP(hipMemcpyAsync(leaves_host, f->leaves, (size_t)f->T * P * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RL_HIP(hipStreamSynchronize(s));
    return RELOC_OK;
}

extern "C" int reloc_debug_features8(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                     const reloc_intrinsics *K, int32_t *feat_host, void *stream)
{
    if (!f || !feat_host) return RELOC_E_ARG;
    Frame fr;
    int rc = frame_of(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    int64_t P = (int64_t)fr.W * fr.H;
    int32_t *d = nullptr;
    RL_HIP(hipMallocAsync((void **)&d, (size_t)P * 8 * sizeof(int32_t), s));
    RL_LAUNCH("k_features8", k_features8, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s,
                       f->nodes + (int64_t)f->T * (f->L - 1), fr, d);
    hipError_t e = hipMemcpyAsync(feat_host, d, (size_t)P * 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(d, s);
    RL_HIP(e);
    RL_HIP(hipStreamSynchronize(s));
    return RELOC_OK;
}

extern "C" int reloc_debug_reservoir(const reloc_forest *f, int32_t t, int32_t leaf0, int32_t n, void *entries_host,
                                     uint32_t *counters_host)
{
    if (!f || t < 0 || t >= f->T || leaf0 < 0 || n < 0 || leaf0 + n > f->L) return RELOC_E_ARG;
    if (f->dropped && entries_host) return RELOC_E_STATE;
    RL_HIP(hipDeviceSynchronize());
    int64_t li = (int64_t)t * f->L + leaf0;
    if (entries_host)
        RL_HIP(hipMemcpy(entries_host, f->res + li * f->R, (size_t)n * f->R * sizeof(Entry), hipMemcpyDeviceToHost));
    if (counters_host)
        RL_HIP(hipMemcpy(counters_host, f->counter + li, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return RELOC_OK;
}

extern "C" int reloc_debug_modes(reloc_forest *f, int32_t t, int32_t leaf0, int32_t n, void *modes_host,
                                 int32_t *n_modes_host)
{
    if (!f || t < 0 || t >= f->T || leaf0 < 0 || n < 0 || leaf0 + n > f->L) return RELOC_E_ARG;
    int rc = update_modes(f, 0);
    if (rc) return rc;
    RL_HIP(hipDeviceSynchronize());
    int64_t li = (int64_t)t * f->L + leaf0;
    if (modes_host)
        RL_HIP(hipMemcpy(modes_host, f->modes + li * f->M, (size_t)n * f->M * sizeof(Mode), hipMemcpyDeviceToHost));
    if (n_modes_host)
        RL_HIP(hipMemcpy(n_modes_host, f->nmodes + li, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost));
    return RELOC_OK;
}

extern "C" int reloc_debug_modes_from_points(reloc_forest *f, const void *entries_host, int32_t n, void *modes_host,
                                             int32_t *n_modes_host)
{
    if (!f || (!entries_host && n > 0) || !modes_host || !n_modes_host || n < 0 || n > MAX_R) return RELOC_E_ARG;
    Entry *d_pts = nullptr;
    Mode *d_modes = nullptr;
    int32_t *d_n = nullptr;
    RL_HIP(hipDeviceSynchronize());
    if (hipMalloc((void **)&d_pts, (size_t)std::max(n, 1) * sizeof(Entry)) != hipSuccess) return RELOC_E_NOMEM;
    if (hipMalloc((void **)&d_modes, (size_t)f->M * sizeof(Mode)) != hipSuccess ||
        hipMalloc((void **)&d_n, sizeof(int32_t)) != hipSuccess) {
        (void)hipFree(d_pts);
        (void)hipFree(d_modes);
        return RELOC_E_NOMEM;
    }
    int rc = RELOC_OK;
    if (n > 0 && hipMemcpy(d_pts, entries_host, (size_t)n * sizeof(Entry), hipMemcpyHostToDevice) != hipSuccess)
        rc = RELOC_E_HIP;
    if (!rc) {
        ModeParams mp = mode_params(f);
        RL_LAUNCH("k_modes_points", k_modes_points, dim3(1), dim3(MODE_THREADS), mode_smem(n), 0, d_pts, (int)n, mp, d_modes,
                           d_n);
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemcpy(n_modes_host, d_n, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(modes_host, d_modes, (size_t)f->M * sizeof(Mode), hipMemcpyDeviceToHost) != hipSuccess)
            rc = RELOC_E_HIP;
    }
    (void)hipFree(d_pts);
    (void)hipFree(d_modes);
    (void)hipFree(d_n);
    return rc;
}
