// Relocalisation of one RGB-D frame on the GPU: query pool, three-point
// Kabsch hypotheses, preemptive scoring with halving culls and inlier
// refinement.
//
// Layout of the work:
//  - hypotheses: one wavefront per hypothesis, one lane per try; the first
//    passing try (lowest lane, then lowest chunk of 64 tries) defines it;
//  - scoring: one wavefront holds 64 live hypotheses (one per lane) and one
//    group of 8 consecutive draws; the draw's modes are wave-uniform, so they
//    come through scalar loads and every lane evaluates its own pose against
//    them; partial energies are written per (group, hypothesis) and summed in
//    group order by the cull;
//  - cull: one workgroup sorts the live hypotheses by (energy, index) in LDS
//    and keeps the first half (rounded up);
//  - refinement: one wavefront per survivor, lanes over the round's draws,
//    FP64 inlier sums combined by an xor butterfly, then Horn's method.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "common.h"

namespace rl {

int update_modes(Forest *f, hipStream_t s);
int traverse_frame(Forest *f, const Frame &fr, hipStream_t s);
int frame_from(const Forest *f, const uint16_t *depth, const uint8_t *rgb, const reloc_intrinsics *K, Frame &fr);

// ---------------------------------------------------------------------------
// query pool: valid pixels in raster order
// ---------------------------------------------------------------------------

constexpr int POOL_BLOCK = 1024;

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

__global__ void __launch_bounds__(POOL_BLOCK) k_pool_count(Frame fr, int32_t *__restrict__ blockcnt)
{
    int P = fr.W * fr.H;
    int p = blockIdx.x * POOL_BLOCK + threadIdx.x;
    bool ok = p < P && valid_depth(fr, fr.depth[p]);
    int n = __syncthreads_count(ok);
    if (threadIdx.x == 0) blockcnt[blockIdx.x] = n;
}

// exclusive scan of the block counts (one workgroup), pool size
__global__ void __launch_bounds__(1024) k_pool_scan(int32_t *__restrict__ blockcnt, int nb,
                                                    int32_t *__restrict__ pool_size)
{
    __shared__ int32_t wsum[16];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    for (int base = 0; base < nb; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < nb ? blockcnt[i] : 0;
        int x = v;
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int woff = 0;
        for (int w = 0; w < wave; ++w) woff += wsum[w];
        int excl = carry + woff + x - v;
        __syncthreads();
        if (i < nb) blockcnt[i] = excl;
        if (threadIdx.x == 1023) carry = excl + v;
        __syncthreads();
    }
    if (threadIdx.x == 0) *pool_size = carry;
}

__global__ void __launch_bounds__(POOL_BLOCK) k_pool_write(Frame fr, const int32_t *__restrict__ blockoff,
                                                           int32_t *__restrict__ pool)
{
    __shared__ int32_t wcnt[POOL_BLOCK / 64];
    int P = fr.W * fr.H;
    int p = blockIdx.x * POOL_BLOCK + threadIdx.x;
    bool ok = p < P && valid_depth(fr, fr.depth[p]);
    uint64_t m = __ballot(ok);
    const int wave = threadIdx.x / 64;
    if (__lane_id() == 0) wcnt[wave] = __popcll(m);
    __syncthreads();
    int off = blockoff[blockIdx.x];
    for (int w = 0; w < wave; ++w) off += wcnt[w];
    if (ok) pool[off + __popcll(m & lanemask_lt())] = p;
}

// ---------------------------------------------------------------------------
// hypotheses
// ---------------------------------------------------------------------------

struct HypArgs {
    Frame fr;
    const int32_t *__restrict__ pool;
    const int32_t *__restrict__ pool_size;
    const int32_t *__restrict__ leaves;
    const int32_t *__restrict__ nmodes;
    const Mode *__restrict__ modes;
    int T, L, M, P;
    int max_tries, rgb_tol;
    float ratio2, min_pair2, min_area2;
    double resid2;
    uint64_t seed;
    Hyp *__restrict__ hyp;
    double *__restrict__ hyp_init;
    int32_t *__restrict__ hyp_try;
    float *__restrict__ energy;
    double *__restrict__ sums;
};

__device__ __forceinline__ float sq3(const float a[3], const float b[3])
{
    float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ bool rgb_close(uint32_t a, uint32_t r, uint32_t g, uint32_t b, int tol)
{
    int dr = (int)(a & 255u) - (int)r, dg = (int)((a >> 8) & 255u) - (int)g, db = (int)((a >> 16) & 255u) - (int)b;
    return abs(dr) <= tol && abs(dg) <= tol && abs(db) <= tol;
}

// one try: draws, mode picks, FP32 checks, FP64 alignment and residuals
__device__ bool try_hypothesis(const HypArgs &A, int np, uint64_t h, uint64_t tau, double R[9], double t[3])
{
    U4 a = philox(h, tau, 0, 0, A.seed, TAG_HYP);
    U4 b = philox(h, tau, 1, 0, A.seed, TAG_HYP);
    int pi[3];
    float c[3][3], w[3][3];
    for (int j = 0; j < 3; ++j) {
        pi[j] = (int)uniform_int(a.x[j], (uint64_t)np);
        int p = A.pool[pi[j]];
        uint32_t pr = A.fr.rgb[p * 3], pg = A.fr.rgb[p * 3 + 1], pb = A.fr.rgb[p * 3 + 2];
        int cnt = 0;
        for (int tt = 0; tt < A.T; ++tt) {
            int li = tt * A.L + A.leaves[(int64_t)tt * A.P + p];
            int nm = A.nmodes[li];
            const Mode *mb = A.modes + (int64_t)li * A.M;
            for (int m = 0; m < nm; ++m) cnt += rgb_close(mb[m].rgb, pr, pg, pb, A.rgb_tol) ? 1 : 0;
        }
        if (cnt == 0) return false;
        int sel = (int)uniform_int(b.x[j], (uint64_t)cnt);
        const Mode *pick = nullptr;
        for (int tt = 0; tt < A.T && !pick; ++tt) {
            int li = tt * A.L + A.leaves[(int64_t)tt * A.P + p];
            int nm = A.nmodes[li];
            const Mode *mb = A.modes + (int64_t)li * A.M;
            for (int m = 0; m < nm; ++m)
                if (rgb_close(mb[m].rgb, pr, pg, pb, A.rgb_tol)) {
                    if (sel == 0) {
                        pick = &mb[m];
                        break;
                    }
                    sel--;
                }
        }
        int u = p % A.fr.W, v = p / A.fr.W;
        cam_point(A.fr, u, v, A.fr.depth[p], c[j]);
        w[j][0] = pick->mu[0];
        w[j][1] = pick->mu[1];
        w[j][2] = pick->mu[2];
    }
    if (pi[0] == pi[1] || pi[0] == pi[2] || pi[1] == pi[2]) return false;
    const int EA[3] = {0, 0, 1}, EB[3] = {1, 2, 2};
    for (int e = 0; e < 3; ++e) {
        float dc = sq3(c[EA[e]], c[EB[e]]);
        float dw = sq3(w[EA[e]], w[EB[e]]);
        if (!(dc >= A.min_pair2)) return false;
        if (!(dw <= A.ratio2 * dc)) return false;
        if (!(dc <= A.ratio2 * dw)) return false;
    }
    float e1[3] = {c[1][0] - c[0][0], c[1][1] - c[0][1], c[1][2] - c[0][2]};
    float e2[3] = {c[2][0] - c[0][0], c[2][1] - c[0][1], c[2][2] - c[0][2]};
    float cx = e1[1] * e2[2] - e1[2] * e2[1];
    float cy = e1[2] * e2[0] - e1[0] * e2[2];
    float cz = e1[0] * e2[1] - e1[1] * e2[0];
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

__global__ void __launch_bounds__(64) k_hypgen(HypArgs A)
{
    const int h = blockIdx.x, lane = __lane_id();
    const int np = *A.pool_size;
    int found = -1;
    double R[9], t[3];
    for (int chunk = 0; chunk * 64 < A.max_tries && found < 0; ++chunk) {
        int tau = chunk * 64 + lane;
        bool ok = tau < A.max_tries && np > 0 && try_hypothesis(A, np, (uint64_t)h, (uint64_t)tau, R, t);
        uint64_t m = __ballot(ok);
        if (m) {
            int first = __ffsll((unsigned long long)m) - 1;
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
        A.energy[h] = 0.0f;
    }
    if (lane < NSUM) A.sums[(int64_t)h * NSUM + lane] = 0.0;
}

// live list = valid hypotheses in index order
__global__ void __launch_bounds__(1024) k_alive_init(const int32_t *__restrict__ hyp_try, int N,
                                                     int32_t *__restrict__ alive, int32_t *__restrict__ n_alive,
                                                     int32_t *__restrict__ rounds_done)
{
    __shared__ int32_t wcnt[16];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int wave = threadIdx.x / 64;
    for (int base = 0; base < N; base += 1024) {
        int h = base + threadIdx.x;
        bool ok = h < N && hyp_try[h] >= 0;
        uint64_t m = __ballot(ok);
        if (__lane_id() == 0) wcnt[wave] = __popcll(m);
        __syncthreads();
        int off = carry;
        for (int w = 0; w < wave; ++w) off += wcnt[w];
        if (ok) alive[off + __popcll(m & lanemask_lt())] = h;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wcnt[w];
            carry += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        n_alive[0] = carry;
        n_alive[1] = carry;
        rounds_done[0] = 0;
    }
}

// ---------------------------------------------------------------------------
// preemptive rounds
// ---------------------------------------------------------------------------

struct RoundArgs {
    Frame fr;
    const int32_t *__restrict__ pool;
    const int32_t *__restrict__ pool_size;
    const int32_t *__restrict__ leaves;
    const int32_t *__restrict__ nmodes;
    const Mode *__restrict__ modes;
    int T, L, M, P, B, N;
    uint64_t seed;
    float inl2;
    int refine;
    Hyp *hyp;
    float *energy;
    double *sums;
    int32_t *alive;
    int32_t *n_alive;
    int32_t *rounds_done;
    float4 *draws;
    float *partial;
    uint16_t *inl;
    int32_t *tr_alive;
    float *tr_energy;
    int32_t *tr_n_alive;
};

// round r runs when r == 0 and at least one hypothesis is live, or r > 0 and
// more than one is
__global__ void k_draw(RoundArgs A, int r)
{
    int na = A.n_alive[0];
    if (r == 0 ? na < 1 : na <= 1) return;
    if (A.rounds_done[0] != r) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int np = *A.pool_size;
    if (i < A.B) {
        U4 u = philox((uint64_t)r, (uint64_t)i, 0, 0, A.seed, TAG_PIX);
        int p = A.pool[uniform_int(u.x[0], (uint64_t)np)];
        float c[3];
        cam_point(A.fr, p % A.fr.W, p / A.fr.W, A.fr.depth[p], c);
        A.draws[i] = make_float4(c[0], c[1], c[2], __int_as_float(p));
    }
}

__global__ void k_round_mark(RoundArgs A, int r)
{
    int na = A.n_alive[0];
    if (r == 0 ? na < 1 : na <= 1) return;
    if (A.rounds_done[0] == r) A.rounds_done[0] = r + 1;
}

__global__ void __launch_bounds__(64) k_score(RoundArgs A, int r)
{
    if (A.rounds_done[0] != r + 1) return;
    const int na = A.n_alive[0];
    const int a0 = blockIdx.x * 64;
    if (a0 >= na) return;
    const int a = a0 + __lane_id();
    const bool act = a < na;
    const int h = act ? A.alive[a] : A.alive[a0];
    const Hyp &hy = A.hyp[h];
    float R0 = hy.R32[0], R1 = hy.R32[1], R2 = hy.R32[2], R3 = hy.R32[3], R4 = hy.R32[4], R5 = hy.R32[5],
          R6 = hy.R32[6], R7 = hy.R32[7], R8 = hy.R32[8];
    float t0 = hy.t32[0], t1 = hy.t32[1], t2 = hy.t32[2];
    const int g = blockIdx.y;
    const int i0 = g * GROUP, i1 = min(i0 + GROUP, A.B);
    float gsum = 0.0f;
    for (int i = i0; i < i1; ++i) {
        const float4 dr = A.draws[i];
        const int p = __float_as_int(dr.w);
        const float y0 = fmaf(R0, dr.x, fmaf(R1, dr.y, fmaf(R2, dr.z, t0)));
        const float y1 = fmaf(R3, dr.x, fmaf(R4, dr.y, fmaf(R5, dr.z, t1)));
        const float y2 = fmaf(R6, dr.x, fmaf(R7, dr.y, fmaf(R8, dr.z, t2)));
        float best = INFINITY, b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
        int bid = 0xFFFF;
        for (int tt = 0; tt < A.T; ++tt) {
            const int li = tt * A.L + A.leaves[(int64_t)tt * A.P + p];
            const int nm = A.nmodes[li];
            const Mode *mb = A.modes + (int64_t)li * A.M;
            for (int m = 0; m < nm; ++m) {
                float d0, d1, d2;
                float term = mode_term(mb[m], y0, y1, y2, d0, d1, d2);
                if (term < best) {
                    best = term;
                    bid = tt * A.M + m;
                    b0 = d0;
                    b1 = d1;
                    b2 = d2;
                }
            }
        }
        float e = best < 0.0f ? best : 0.0f;
        gsum = gsum + e;
        bool in = bid != 0xFFFF && (b0 * b0 + b1 * b1) + b2 * b2 <= A.inl2;
        if (act) A.inl[(int64_t)h * A.B + i] = in ? (uint16_t)bid : (uint16_t)0xFFFF;
    }
    if (act) A.partial[(int64_t)g * A.N + a] = gsum;
}

constexpr int CULL_THREADS = 1024;

__global__ void __launch_bounds__(CULL_THREADS) k_cull(RoundArgs A, int r)
{
    if (A.rounds_done[0] != r + 1) return;
    __shared__ unsigned long long keys[MAX_HYP];
    const int na = A.n_alive[0];
    const int G = (A.B + GROUP - 1) / GROUP;
    int n2 = 1;
    while (n2 < na) n2 <<= 1;
    for (int a = threadIdx.x; a < n2; a += CULL_THREADS) {
        if (a < na) {
            int h = A.alive[a];
            float S = 0.0f;
            for (int g = 0; g < G; ++g) S = S + A.partial[(int64_t)g * A.N + a];
            float E = A.energy[h] + S;
            A.energy[h] = E;
            keys[a] = ((unsigned long long)float_key(E) << 32) | (unsigned)h;
            if (r < MAX_ROUNDS) {
                A.tr_alive[r * MAX_HYP + a] = h;
                A.tr_energy[r * MAX_HYP + a] = E;
            }
        } else {
            keys[a] = ~0ull;
        }
    }
    __syncthreads();
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n2; i += CULL_THREADS) {
                int ixj = i ^ j;
                if (ixj > i) {
                    unsigned long long x = keys[i], y = keys[ixj];
                    bool asc = (i & k) == 0;
                    if ((x > y) == asc) {
                        keys[i] = y;
                        keys[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int keep = (na + 1) / 2;
    for (int a = threadIdx.x; a < keep; a += CULL_THREADS) A.alive[a] = (int32_t)(keys[a] & 0xFFFFFFFFull);
    if (threadIdx.x == 0) {
        if (r < MAX_ROUNDS) A.tr_n_alive[r] = na;
        A.n_alive[0] = keep;
    }
}

// wave per survivor: this round's inliers (lane-strided sums in draw order,
// xor butterfly), running sums, Kabsch refinement
__global__ void __launch_bounds__(64) k_refine(RoundArgs A, int r)
{
    if (A.rounds_done[0] != r + 1) return;
    const int na = A.n_alive[0];
    const int a = blockIdx.x;
    if (a >= na) return;
    const int h = A.alive[a];
    const int lane = __lane_id();
    double s[NSUM];
#pragma unroll
    for (int k = 0; k < NSUM; ++k) s[k] = 0.0;
    for (int i = lane; i < A.B; i += 64) {
        uint16_t id = A.inl[(int64_t)h * A.B + i];
        if (id == 0xFFFF) continue;
        float4 dr = A.draws[i];
        int p = __float_as_int(dr.w);
        int tt = id / A.M, m = id % A.M;
        int li = tt * A.L + A.leaves[(int64_t)tt * A.P + p];
        const Mode &md = A.modes[(int64_t)li * A.M + m];
        float c[3] = {dr.x, dr.y, dr.z};
        float w[3] = {md.mu[0], md.mu[1], md.mu[2]};
        sums_add_point(s, c, w);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
        for (int k = 0; k < NSUM; ++k) s[k] = s[k] + __shfl_xor(s[k], o, 64);
    if (lane == 0) {
        double *run = A.sums + (int64_t)h * NSUM;
        double tot[NSUM];
#pragma unroll
        for (int k = 0; k < NSUM; ++k) {
            tot[k] = run[k] + s[k];
            run[k] = tot[k];
        }
        double R[9], t[3];
        if (A.refine && pose_from_sums(tot, R, t)) {
            Hyp &hy = A.hyp[h];
            for (int k = 0; k < 9; ++k) {
                hy.R[k] = R[k];
                hy.R32[k] = (float)R[k];
            }
            for (int k = 0; k < 3; ++k) {
                hy.t[k] = t[k];
                hy.t32[k] = (float)t[k];
            }
        }
    }
}

__global__ void k_finish(RoundArgs A, const unsigned long long *__restrict__ total_samples,
                         Result *__restrict__ res)
{
    if (threadIdx.x != 0) return;
    Result o;
    for (int k = 0; k < 16; ++k) o.pose[k] = (k % 5 == 0) ? 1.0 : 0.0;
    o.score = 0.0f;
    o.pad[0] = o.pad[1] = 0;
    o.pool_size = *A.pool_size;
    o.n_valid = A.n_alive[1];
    o.n_rounds = A.rounds_done[0];
    o.final_hyp = -1;
    if (o.pool_size == 0) {
        o.status = RELOC_FAIL_NO_VALID_PIXELS;
    } else if (o.n_valid == 0) {
        o.status = *total_samples == 0ull ? RELOC_FAIL_NO_MODES : RELOC_FAIL_NO_HYPOTHESIS;
    } else {
        int h = A.alive[0];
        const Hyp &hy = A.hyp[h];
        for (int rr = 0; rr < 3; ++rr) {
            for (int c = 0; c < 3; ++c) o.pose[rr * 4 + c] = hy.R[rr * 3 + c];
            o.pose[rr * 4 + 3] = hy.t[rr];
        }
        o.score = (float)(A.sums[(int64_t)h * NSUM] / ((double)o.n_rounds * (double)A.B));
        o.status = RELOC_OK;
        o.final_hyp = h;
    }
    *res = o;
}

static int rounds_for(int N)
{
    int r = 0;
    while ((1 << r) < N) ++r;
    return r < 1 ? 1 : r;
}

// Queues one attempt on `s` (no host synchronisation); the result lands in
// f->result.
int relocalise_async(Forest *f, const Frame &fr, uint64_t seed, int N, hipStream_t s)
{
    int rc = update_modes(f, s);
    if (rc) return rc;
    rc = traverse_frame(f, fr, s);
    if (rc) return rc;
    int64_t P = (int64_t)fr.W * fr.H;
    int nb = (int)((P + POOL_BLOCK - 1) / POOL_BLOCK);
    RL_LAUNCH("k_pool_count", k_pool_count, dim3(nb), dim3(POOL_BLOCK), 0, s, fr, f->blockcnt);
    RL_LAUNCH("k_pool_scan", k_pool_scan, dim3(1), dim3(1024), 0, s, f->blockcnt, nb, f->pool_size);
    RL_LAUNCH("k_pool_write", k_pool_write, dim3(nb), dim3(POOL_BLOCK), 0, s, fr, f->blockcnt, f->pool);

    HypArgs H;
    H.fr = fr; H.pool = f->pool; H.pool_size = f->pool_size; H.leaves = f->leaves; H.nmodes = f->nmodes;
    H.modes = f->modes; H.T = f->T; H.L = f->L; H.M = f->M; H.P = (int)P;
    H.max_tries = f->p.max_tries; H.rgb_tol = f->p.rgb_tol;
    H.ratio2 = f->p.rigid_ratio2; H.min_pair2 = f->p.min_pair2_m2; H.min_area2 = f->p.min_area2_m4;
    H.resid2 = (double)f->p.resid_m * (double)f->p.resid_m;
    H.seed = seed; H.hyp = f->hyp; H.hyp_init = f->hyp_init; H.hyp_try = f->hyp_try; H.energy = f->energy;
    H.sums = f->sums;
    RL_LAUNCH("k_hypgen", k_hypgen, dim3(N), dim3(64), 0, s, H);
    RL_LAUNCH("k_alive_init", k_alive_init, dim3(1), dim3(1024), 0, s, f->hyp_try, N, f->alive, f->n_alive,
                       f->rounds_done);

    RoundArgs A;
    A.fr = fr; A.pool = f->pool; A.pool_size = f->pool_size; A.leaves = f->leaves; A.nmodes = f->nmodes;
    A.modes = f->modes; A.T = f->T; A.L = f->L; A.M = f->M; A.P = (int)P; A.B = f->p.batch_pixels; A.N = N;
    A.seed = seed; A.inl2 = f->p.inlier_m * f->p.inlier_m; A.refine = f->p.refine;
    A.hyp = f->hyp; A.energy = f->energy; A.sums = f->sums; A.alive = f->alive; A.n_alive = f->n_alive;
    A.rounds_done = f->rounds_done; A.draws = f->draws; A.partial = f->partial; A.inl = f->inl;
    A.tr_alive = f->tr_alive; A.tr_energy = f->tr_energy; A.tr_n_alive = f->tr_n_alive;
    const int rounds = rounds_for(N);
    const int G = (A.B + GROUP - 1) / GROUP;
    int bound = N;   // live hypotheses at the start of round r are at most ceil(N / 2^r)
    for (int r = 0; r < rounds; ++r) {
        RL_LAUNCH("k_draw", k_draw, dim3((A.B + 255) / 256), dim3(256), 0, s, A, r);
        RL_LAUNCH("k_round_mark", k_round_mark, dim3(1), dim3(1), 0, s, A, r);
        RL_LAUNCH("k_score", k_score, dim3((bound + 63) / 64, G), dim3(64), 0, s, A, r);
        RL_LAUNCH("k_cull", k_cull, dim3(1), dim3(CULL_THREADS), 0, s, A, r);
        bound = (bound + 1) / 2;
        RL_LAUNCH("k_refine", k_refine, dim3(bound), dim3(64), 0, s, A, r);
    }
    RL_LAUNCH("k_finish", k_finish, dim3(1), dim3(64), 0, s, A, f->total_samples, f->result);
    RL_HIP(hipGetLastError());
    f->last_N = N;
    return RELOC_OK;
}

}  // namespace rl

using namespace rl;

extern "C" int reloc_relocalise(reloc_forest *f, const uint16_t *depth_dev, const uint8_t *rgb_dev,
                                const reloc_intrinsics *K, uint64_t attempt_seed, int32_t n_hypotheses,
                                const uint32_t *pixel_weights_dev, double pose_c2w_out[16], float *score_out,
                                void *stream)
{
    if (!f || !pose_c2w_out || !score_out) return RELOC_E_ARG;
    if (pixel_weights_dev) return RELOC_E_ARG;   // weighted picks: see the learned-proposal entry points
    Frame fr;
    int rc = frame_from(f, depth_dev, rgb_dev, K, fr);
    if (rc) return rc;
    int N = n_hypotheses > 0 ? n_hypotheses : f->p.n_hypotheses;
    if (N > MAX_HYP) return RELOC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    rc = relocalise_async(f, fr, attempt_seed, N, s);
    if (rc) return rc;
    RL_HIP(hipMemcpyAsync(f->result_host, f->result, sizeof(Result), hipMemcpyDeviceToHost, s));
    RL_HIP(hipStreamSynchronize(s));
    const Result &o = *f->result_host;
    memcpy(pose_c2w_out, o.pose, sizeof(o.pose));
    *score_out = o.score;
    return o.status;
}

extern "C" int reloc_debug_trace(const reloc_forest *f, reloc_trace *tr)
{
    if (!f || !tr) return RELOC_E_ARG;
    RL_HIP(hipDeviceSynchronize());
    const Result &o = *f->result_host;
    int N = f->last_N;
    if (tr->pool_size) *tr->pool_size = o.pool_size;
    if (tr->final_hyp) *tr->final_hyp = o.final_hyp;
    if (tr->n_rounds) *tr->n_rounds = o.n_rounds;
    int nh = std::min(N, tr->cap_hyp);
    if (tr->hyp_try) RL_HIP(hipMemcpy(tr->hyp_try, f->hyp_try, (size_t)nh * 4, hipMemcpyDeviceToHost));
    if (tr->hyp_pose) RL_HIP(hipMemcpy(tr->hyp_pose, f->hyp_init, (size_t)nh * 12 * 8, hipMemcpyDeviceToHost));
    int nr = std::min(std::min(o.n_rounds, tr->cap_rounds), MAX_ROUNDS);
    if (tr->n_alive) RL_HIP(hipMemcpy(tr->n_alive, f->tr_n_alive, (size_t)nr * 4, hipMemcpyDeviceToHost));
    for (int r = 0; r < nr; ++r) {
        if (tr->alive)
            RL_HIP(hipMemcpy(tr->alive + (size_t)r * tr->cap_hyp, f->tr_alive + (size_t)r * MAX_HYP, (size_t)nh * 4,
                             hipMemcpyDeviceToHost));
        if (tr->energy)
            RL_HIP(hipMemcpy(tr->energy + (size_t)r * tr->cap_hyp, f->tr_energy + (size_t)r * MAX_HYP,
                             (size_t)nh * 4, hipMemcpyDeviceToHost));
    }
    return RELOC_OK;
}
