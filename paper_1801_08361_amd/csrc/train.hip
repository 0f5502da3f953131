// Split training: a split structure learned from posed frames of one scene,
// whose leaves are then adapted online to others (Sec. 4.2.2, Table 2: a
// forest pre-trained on one scene and adapted to the rest).
//
// Every node of every tree, level by level from the root, takes from n_cand
// candidate splits (drawn like random splits, from the generator keyed by
// (seed, TRAIN) at counter (tree, node, candidate)) the one that leaves the
// training samples reaching it with the smallest summed squared deviation of
// their world points (integer mm) from their child's mean; ties go to the
// lower candidate. A sample is every stride-th pixel in u and v, from
// stride / 2, of every training frame with a valid depth, with its world
// point as adaptation stores it. The per-child sums (count, coordinate sums,
// sum of squared norms) are exact 64-bit integers, so any grouping of the
// samples gives the same sums; the cost of a child with n samples is
// S2 - |S|^2 / n in FP64, in that order, summed left then right.
//
// Layout: the samples of all frames in one array (frame, pixel, packed word,
// world point); per tree, each sample's node and a permutation that groups
// the samples of each node of the current level. Per level:
//   k_tr_count    samples per (tree, node)                   (host reads them)
//   k_tr_scatter  the grouping permutation                   (host offsets)
//   k_tr_eval     one wavefront per unit of at most TR_CHUNK samples of one node,
//                 one lane per candidate: the candidate's response for each
//                 sample, its two children's sums in registers; a node of one
//                 unit picks its split there, larger nodes store partial sums
//   k_tr_pick     one wavefront per node of several units: the partials'
//                 sums (exact), the costs and the split
//   k_tr_route    every sample one level down
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace rl {

int frame_from(const Forest *f, const uint16_t *depth, const uint8_t *rgb, const reloc_intrinsics *K, Frame &fr);
bool pose_is_se3(const double T[16]);
int forest_empty_leaves(Forest *f, hipStream_t s);

namespace {

constexpr int TR_CHUNK = 64;      // samples per evaluation unit
constexpr int NSPLIT = 10;     // per candidate: (n, Sx, Sy, Sz, S2) left, then right

struct TrainPose {
    float R[9], t[3];
};

struct Unit {
    int32_t t, j;        // tree, node index within the level
    int32_t start, len;  // range of the node's samples in the tree's permutation
    int32_t slot;        // partial-sum slot, or -1: the unit is its node's only one
};

struct Samples {
    int32_t *frame;      // [S]
    int32_t *pix;        // [S] pixel index in its frame
    uint64_t *own;       // [S] packed word of the pixel
    int4 *q;             // [S] world point (mm)
    int32_t *count;      // [1]
};

__global__ void __launch_bounds__(256) k_tr_pack(Frame fr, uint64_t *__restrict__ packed)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < (int64_t)fr.W * fr.H) packed[p] = pack_pixel(fr, p);
}

// one thread per point of the sampling grid of frame `fi`
__global__ void __launch_bounds__(256) k_tr_samples(Frame fr, TrainPose pose, int fi, int stride, int gw, int gh,
                                                    const uint64_t *__restrict__ packed, Samples smp)
{
    const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (g >= gw * gh) return;
    const int u = stride / 2 + (g % gw) * stride, v = stride / 2 + (g / gw) * stride;
    const int p = v * fr.W + u;
    const uint32_t d = fr.depth[p];
    if (!valid_depth(fr, d)) return;
    float c[3];
    cam_point(fr, u, v, d, c);
    const float w0 = ((pose.R[0] * c[0] + pose.R[1] * c[1]) + pose.R[2] * c[2]) + pose.t[0];
    const float w1 = ((pose.R[3] * c[0] + pose.R[4] * c[1]) + pose.R[5] * c[2]) + pose.t[1];
    const float w2 = ((pose.R[6] * c[0] + pose.R[7] * c[1]) + pose.R[8] * c[2]) + pose.t[2];
    const int s = atomicAdd(smp.count, 1);
    smp.frame[s] = fi;
    smp.pix[s] = p;
    smp.own[s] = packed[p];
    smp.q[s] = make_int4((int32_t)rintf(w0 * 1000.0f), (int32_t)rintf(w1 * 1000.0f), (int32_t)rintf(w2 * 1000.0f), 0);
}

struct TrainArgs {
    const Frame *frames;          // [n_frames]
    const int64_t *poff;          // [n_frames] offset of each frame's packed words
    const uint64_t *packed;
    Samples smp;
    int32_t S;                    // samples
    int32_t T, L;
    int32_t level_first;          // heap index of the level's first node
    int32_t n_level;              // nodes in the level
    int32_t n_cand;
    uint64_t seed;
    int32_t O, thr_d, thr_c;
    int32_t *node;                // [T][S] heap index of each sample's node
    int32_t *perm;                // [T][S]
    int32_t *count;               // [T][n_level]
    int32_t *cursor;              // [T][n_level]
    uint64_t *nodes;              // the forest's split nodes [T][L - 1]
    DeepNode *deep;
};

// the response of sample s to the split in packed word w
__device__ __forceinline__ int32_t sample_response(const TrainArgs &A, int s, uint64_t w, int32_t *thr)
{
    const int fi = A.smp.frame[s];
    const Frame fr = A.frames[fi];
    const int p = A.smp.pix[s];
    const uint64_t own = A.smp.own[s];
    const ProbeNode n = probe_node(w, fr);
    *thr = n.thr;
    const __amdgpu_buffer_rsrc_t rs = packed_rsrc(A.packed + A.poff[fi], fr.W * fr.H);
    return probe_response(rs, fr.W, fr.H, p % fr.W, p / fr.W, own, pixel_den(fr, (int32_t)packed_depth(own)), n);
}

__global__ void __launch_bounds__(256) k_tr_count(TrainArgs A)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)A.T * A.S) return;
    const int t = (int)(g / A.S);
    atomicAdd(&A.count[(int64_t)t * A.n_level + (A.node[g] - A.level_first)], 1);
}

__global__ void __launch_bounds__(256) k_tr_scatter(TrainArgs A)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)A.T * A.S) return;
    const int t = (int)(g / A.S);
    const int at = atomicAdd(&A.cursor[(int64_t)t * A.n_level + (A.node[g] - A.level_first)], 1);
    A.perm[(int64_t)t * A.S + at] = (int32_t)(g - (int64_t)t * A.S);
}

// the cost of one candidate's sums (as the oracle defines it)
__device__ __forceinline__ double split_cost(const long long v[NSPLIT])
{
    double c = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const long long *q = v + 5 * side;
        if (q[0] == 0) continue;
        const double sx = (double)q[1], sy = (double)q[2], sz = (double)q[3];
        c = c + ((double)q[4] - ((sx * sx + sy * sy) + sz * sz) / (double)q[0]);
    }
    return c;
}

// lane k's candidate, or the first of equal lowest costs over the lanes: the
// lane of the chosen candidate
__device__ __forceinline__ int wave_argmin(double c, int k)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double co = __shfl_xor(c, o, 64);
        const int ko = __shfl_xor(k, o, 64);
        if (co < c || (co == c && ko < k)) {
            c = co;
            k = ko;
        }
    }
    return k;
}

__device__ __forceinline__ void write_split(const TrainArgs &A, int t, int j, uint64_t w)
{
    const int64_t at = (int64_t)t * (A.L - 1) + A.level_first + j;
    A.nodes[at] = w;
    A.deep[at] = deep_node(w);
}

__global__ void __launch_bounds__(64) k_tr_eval(TrainArgs A, const Unit *__restrict__ units, int n_units,
                                                long long *__restrict__ partial)
{
    for (int ui = (int)blockIdx.x; ui < n_units; ui += (int)gridDim.x) {
        const Unit U = units[ui];
        const int k = __lane_id();
        const bool cand = k < A.n_cand;
        const uint64_t i = (uint64_t)(A.level_first + U.j);
        const uint64_t w = split_from_draw(philox((uint64_t)U.t, i, (uint64_t)(cand ? k : 0), 0, A.seed, TAG_TRAIN),
                                           A.O, A.thr_d, A.thr_c);
        long long v[NSPLIT];
#pragma unroll
        for (int e = 0; e < NSPLIT; ++e) v[e] = 0;
        const int32_t *perm = A.perm + (int64_t)U.t * A.S + U.start;
        for (int o = 0; o < U.len; ++o) {
            const int s = perm[o];
            int32_t thr;
            const int32_t r = sample_response(A, s, w, &thr);
            const int4 q = A.smp.q[s];
            const long long x = q.x, y = q.y, z = q.z;
            const long long q2 = x * x + y * y + z * z;
            const bool right = r >= thr;
            v[0] += right ? 0 : 1;
            v[1] += right ? 0 : x;
            v[2] += right ? 0 : y;
            v[3] += right ? 0 : z;
            v[4] += right ? 0 : q2;
            v[5] += right ? 1 : 0;
            v[6] += right ? x : 0;
            v[7] += right ? y : 0;
            v[8] += right ? z : 0;
            v[9] += right ? q2 : 0;
        }
        if (U.slot < 0) {
            const double c = cand ? split_cost(v) : INFINITY;
            const int best = wave_argmin(c, k);
            if (k == best) write_split(A, U.t, U.j, w);
        } else if (cand) {
            long long *dst = partial + ((int64_t)U.slot * 64 + k) * NSPLIT;
#pragma unroll
            for (int e = 0; e < NSPLIT; ++e) dst[e] = v[e];
        }
    }
}

// nodes of several units: picks[n] = (tree, node in level, first slot, slots)
__global__ void __launch_bounds__(64) k_tr_pick(TrainArgs A, const int4 *__restrict__ picks, int n_picks,
                                                const long long *__restrict__ partial)
{
    for (int pi = (int)blockIdx.x; pi < n_picks; pi += (int)gridDim.x) {
        const int4 P = picks[pi];
        const int k = __lane_id();
        const bool cand = k < A.n_cand;
        long long v[NSPLIT];
#pragma unroll
        for (int e = 0; e < NSPLIT; ++e) v[e] = 0;
        if (cand)
            for (int sl = P.z; sl < P.z + P.w; ++sl) {
                const long long *src = partial + ((int64_t)sl * 64 + k) * NSPLIT;
#pragma unroll
                for (int e = 0; e < NSPLIT; ++e) v[e] += src[e];
            }
        const double c = cand ? split_cost(v) : INFINITY;
        const int best = wave_argmin(c, k);
        if (k == best) {
            const uint64_t i = (uint64_t)(A.level_first + P.y);
            write_split(A, P.x, P.y,
                        split_from_draw(philox((uint64_t)P.x, i, (uint64_t)k, 0, A.seed, TAG_TRAIN), A.O, A.thr_d,
                                        A.thr_c));
        }
    }
}

__global__ void __launch_bounds__(256) k_tr_route(TrainArgs A)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)A.T * A.S) return;
    const int t = (int)(g / A.S);
    const int s = (int)(g - (int64_t)t * A.S);
    const int i = A.node[g];
    int32_t thr;
    const int32_t r = sample_response(A, s, A.nodes[(int64_t)t * (A.L - 1) + i], &thr);
    A.node[g] = 2 * i + 1 + (r >= thr ? 1 : 0);
}

__global__ void __launch_bounds__(256) k_tr_root(int32_t *node, int64_t n)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) node[g] = 0;
}

// device scratch of one training call, freed in stream order
struct Scratch {
    std::vector<void *> ptrs;
    hipStream_t s;
    explicit Scratch(hipStream_t st) : s(st) {}
    template <typename X>
    bool get(X **p, size_t count)
    {
        *p = nullptr;
        if (hipMallocAsync((void **)p, std::max<size_t>(count, 1) * sizeof(X), s) != hipSuccess) return false;
        ptrs.push_back((void *)*p);
        return true;
    }
    ~Scratch()
    {
        for (void *p : ptrs) (void)hipFreeAsync(p, s);
        (void)hipStreamSynchronize(s);
    }
};

unsigned blocks_of(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace
}  // namespace rl

using namespace rl;

extern "C" int reloc_forest_train(reloc_forest *f, const reloc_train_frame *frames, int32_t n_frames, int32_t stride,
                                  int32_t n_candidates, void *stream)
{
    if (!f || !frames || n_frames < 1 || stride < 1 || n_candidates < 1 || n_candidates > 64) return RELOC_E_ARG;
    if (f->dropped) return RELOC_E_STATE;
    hipStream_t s = (hipStream_t)stream;
    std::vector<Frame> fr(n_frames);
    std::vector<int64_t> poff(n_frames + 1, 0);
    int64_t S_cap = 0;
    for (int k = 0; k < n_frames; ++k) {
        int rc = frame_from(f, frames[k].depth_dev, frames[k].rgb_dev, &frames[k].K, fr[k]);
        if (rc) return rc;
        if (!pose_is_se3(frames[k].pose_c2w)) return RELOC_E_ARG;
        poff[k + 1] = poff[k] + (int64_t)fr[k].W * fr[k].H;
        S_cap += (int64_t)((fr[k].W - stride / 2 + stride - 1) / stride) * ((fr[k].H - stride / 2 + stride - 1) / stride);
    }
    if (S_cap > (int64_t)INT32_MAX / std::max(f->T, 1)) return RELOC_E_RANGE;
    Scratch sc(s);
    Frame *d_frames;
    int64_t *d_poff;
    uint64_t *packed;
    Samples smp;
    if (!sc.get(&d_frames, n_frames) || !sc.get(&d_poff, n_frames) || !sc.get(&packed, poff[n_frames]) ||
        !sc.get(&smp.frame, S_cap) || !sc.get(&smp.pix, S_cap) || !sc.get(&smp.own, S_cap) || !sc.get(&smp.q, S_cap) ||
        !sc.get(&smp.count, 1))
        return RELOC_E_NOMEM;
    RL_HIP(hipMemcpyAsync(d_frames, fr.data(), sizeof(Frame) * n_frames, hipMemcpyHostToDevice, s));
    RL_HIP(hipMemcpyAsync(d_poff, poff.data(), sizeof(int64_t) * n_frames, hipMemcpyHostToDevice, s));
    RL_HIP(hipMemsetAsync(smp.count, 0, sizeof(int32_t), s));
    for (int k = 0; k < n_frames; ++k) {
        const int64_t P = (int64_t)fr[k].W * fr[k].H;
        RL_LAUNCH("k_tr_pack", k_tr_pack, dim3(blocks_of(P, 256)), dim3(256), 0, s, fr[k], packed + poff[k]);
        TrainPose ps;
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) ps.R[r * 3 + c] = (float)frames[k].pose_c2w[r * 4 + c];
            ps.t[r] = (float)frames[k].pose_c2w[r * 4 + 3];
        }
        const int gw = (fr[k].W - stride / 2 + stride - 1) / stride, gh = (fr[k].H - stride / 2 + stride - 1) / stride;
        if (gw > 0 && gh > 0)
            RL_LAUNCH("k_tr_samples", k_tr_samples, dim3(blocks_of((int64_t)gw * gh, 256)), dim3(256), 0, s, fr[k], ps,
                      k, stride, gw, gh, (const uint64_t *)(packed + poff[k]), smp);
    }
    int32_t S = 0;
    RL_HIP(hipMemcpyAsync(&S, smp.count, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RL_HIP(hipStreamSynchronize(s));
    TrainArgs A;
    A.frames = d_frames;
    A.poff = d_poff;
    A.packed = packed;
    A.smp = smp;
    A.S = S;
    A.T = f->T;
    A.L = f->L;
    A.n_cand = n_candidates;
    A.seed = f->p.seed;
    A.O = f->p.offset_pxmm;
    A.thr_d = f->p.thr_depth_mm;
    A.thr_c = f->p.thr_rgb;
    A.nodes = f->nodes;
    A.deep = f->deep;
    const int64_t TS = (int64_t)f->T * S;
    const int64_t max_level = (int64_t)1 << (f->D - 1);
    const int64_t max_units = (int64_t)f->T * max_level + TS / TR_CHUNK + 1;
    // partial slots: only nodes of more than TR_CHUNK samples use them, ceil(n / TR_CHUNK) < 2 n / TR_CHUNK each
    const int64_t max_slots = 2 * TS / TR_CHUNK + 1;
    Unit *d_units;
    int4 *d_picks;
    long long *partial;
    if (!sc.get(&A.node, TS) || !sc.get(&A.perm, TS) || !sc.get(&A.count, f->T * max_level) ||
        !sc.get(&A.cursor, f->T * max_level) || !sc.get(&d_units, max_units) || !sc.get(&d_picks, f->T * max_level) ||
        !sc.get(&partial, max_slots * 64 * NSPLIT))
        return RELOC_E_NOMEM;
    if (TS > 0) RL_LAUNCH("k_tr_root", k_tr_root, dim3(blocks_of(TS, 256)), dim3(256), 0, s, A.node, TS);
    std::vector<int32_t> cnt, off;
    std::vector<Unit> units;
    std::vector<int4> picks;
    for (int l = 0; l < f->D; ++l) {
        A.level_first = (1 << l) - 1;
        A.n_level = 1 << l;
        const int64_t TN = (int64_t)f->T * A.n_level;
        cnt.assign(TN, 0);
        if (TS > 0) {
            RL_HIP(hipMemsetAsync(A.count, 0, TN * sizeof(int32_t), s));
            RL_LAUNCH("k_tr_count", k_tr_count, dim3(blocks_of(TS, 256)), dim3(256), 0, s, A);
            RL_HIP(hipMemcpyAsync(cnt.data(), A.count, TN * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            RL_HIP(hipStreamSynchronize(s));
        }
        // offsets within each tree's permutation, the units and the picks
        off.assign(TN, 0);
        units.clear();
        picks.clear();
        int32_t slots = 0;
        for (int t = 0; t < f->T; ++t) {
            int32_t at = 0;
            for (int j = 0; j < A.n_level; ++j) {
                const int32_t n = cnt[(int64_t)t * A.n_level + j];
                off[(int64_t)t * A.n_level + j] = at;
                if (n <= TR_CHUNK) {
                    units.push_back(Unit{t, j, at, n, -1});
                } else {
                    const int32_t first = slots;
                    for (int32_t o = 0; o < n; o += TR_CHUNK)
                        units.push_back(Unit{t, j, at + o, std::min(TR_CHUNK, n - o), slots++});
                    picks.push_back(make_int4(t, j, first, slots - first));
                }
                at += n;
            }
        }
        if ((int64_t)units.size() > max_units || slots > max_slots) return RELOC_E_STATE;
        RL_HIP(hipMemcpyAsync(A.cursor, off.data(), TN * sizeof(int32_t), hipMemcpyHostToDevice, s));
        RL_HIP(hipMemcpyAsync(d_units, units.data(), units.size() * sizeof(Unit), hipMemcpyHostToDevice, s));
        if (!picks.empty())
            RL_HIP(hipMemcpyAsync(d_picks, picks.data(), picks.size() * sizeof(int4), hipMemcpyHostToDevice, s));
        if (TS > 0) RL_LAUNCH("k_tr_scatter", k_tr_scatter, dim3(blocks_of(TS, 256)), dim3(256), 0, s, A);
        const int nu = (int)units.size();
        RL_LAUNCH("k_tr_eval", k_tr_eval, dim3((unsigned)std::min(nu, 65536)), dim3(64), 0, s, A,
                  (const Unit *)d_units, nu, partial);
        if (!picks.empty())
            RL_LAUNCH("k_tr_pick", k_tr_pick, dim3((unsigned)std::min<size_t>(picks.size(), 65536)), dim3(64), 0, s, A,
                      (const int4 *)d_picks, (int)picks.size(), (const long long *)partial);
        if (TS > 0 && l + 1 < f->D) RL_LAUNCH("k_tr_route", k_tr_route, dim3(blocks_of(TS, 256)), dim3(256), 0, s, A);
        // the host vectors are reused by the next level: the copies above
        // must have read them
        RL_HIP(hipStreamSynchronize(s));
    }
    RL_HIP(hipGetLastError());
    return forest_empty_leaves(f, s);
}
