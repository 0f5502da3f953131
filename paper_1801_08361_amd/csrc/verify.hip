// Depth-difference verification of a proposed relocalisation (Sec. 3.3.1,
// Eqs. 3-4): with D_a the target sub-scene's depth rendered at the proposed
// pose and D_b the relocalised frame's depth, count the pixels valid in D_a
// (depth > 0), and sum |D_a - D_b| over the pixels valid in both.
//
// The three sums are exact integers. Each workgroup reduces its share of the
// image (16-byte loads, eight pixels per load, when both images are 16-byte
// aligned) and writes one partial triple of its own; a one-workgroup kernel
// adds the partials. No atomics, so nothing has to be cleared before a call.
#include <math.h>

#include <mutex>

#include "common.h"

namespace rl {

constexpr int VERIFY_THREADS = 256;
constexpr int VERIFY_MAX_PARTS = 2048;   // workgroups of the partial pass (grid cap)

__device__ __forceinline__ void verify_px(uint32_t a, uint32_t b, uint32_t &na, uint32_t &nab, uint32_t &sum)
{
    const bool va = a != 0u, vb = b != 0u;
    na += va ? 1u : 0u;
    const bool both = va && vb;
    nab += both ? 1u : 0u;
    sum += both ? (a > b ? a - b : b - a) : 0u;
}

// workgroup reduction of one thread triple into parts[3 * blockIdx.x + k]
__device__ __forceinline__ void verify_store(uint32_t na, uint32_t nab, uint32_t sum,
                                             unsigned long long *__restrict__ parts)
{
    __shared__ unsigned long long red[VERIFY_THREADS / 64][3];
    unsigned long long x0 = na, x1 = nab, x2 = sum;
    for (int o = 32; o >= 1; o >>= 1) {
        x0 += __shfl_xor(x0, o, 64);
        x1 += __shfl_xor(x1, o, 64);
        x2 += __shfl_xor(x2, o, 64);
    }
    const int wave = (int)(threadIdx.x >> 6);
    if (__lane_id() == 0) {
        red[wave][0] = x0;
        red[wave][1] = x1;
        red[wave][2] = x2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long s = 0ull;
        for (int w = 0; w < VERIFY_THREADS / 64; ++w) s += red[w][threadIdx.x];
        parts[3 * blockIdx.x + threadIdx.x] = s;
    }
}

// both images 16-byte aligned: pixel groups of 8 by uint4 loads, then the
// P % 8 tail pixels one by one (by workgroup 0)
__global__ void __launch_bounds__(VERIFY_THREADS) k_verify_vec(const uint16_t *__restrict__ da,
                                                               const uint16_t *__restrict__ db, int P,
                                                               unsigned long long *__restrict__ parts)
{
    const int nvec = P >> 3;
    const uint4 *a4 = (const uint4 *)da;
    const uint4 *b4 = (const uint4 *)db;
    uint32_t na = 0u, nab = 0u, sum = 0u;
    for (int v = blockIdx.x * VERIFY_THREADS + (int)threadIdx.x; v < nvec; v += gridDim.x * VERIFY_THREADS) {
        const uint4 x = a4[v], y = b4[v];
        const uint32_t xa[4] = {x.x, x.y, x.z, x.w}, yb[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            verify_px(xa[k] & 0xFFFFu, yb[k] & 0xFFFFu, na, nab, sum);
            verify_px(xa[k] >> 16, yb[k] >> 16, na, nab, sum);
        }
    }
    if (blockIdx.x == 0) {
        const int p = (nvec << 3) + (int)threadIdx.x;
        if (p < P) verify_px(da[p], db[p], na, nab, sum);
    }
    verify_store(na, nab, sum, parts);
}

// any alignment: one pixel at a time
__global__ void __launch_bounds__(VERIFY_THREADS) k_verify_px(const uint16_t *__restrict__ da,
                                                              const uint16_t *__restrict__ db, int P,
                                                              unsigned long long *__restrict__ parts)
{
    uint32_t na = 0u, nab = 0u, sum = 0u;
    for (int p = blockIdx.x * VERIFY_THREADS + (int)threadIdx.x; p < P; p += gridDim.x * VERIFY_THREADS)
        verify_px(da[p], db[p], na, nab, sum);
    verify_store(na, nab, sum, parts);
}

// one workgroup: totals[k] = sum over the g partials of parts[3 i + k]
__global__ void __launch_bounds__(VERIFY_THREADS) k_verify_total(const unsigned long long *__restrict__ parts, int g,
                                                                 unsigned long long *__restrict__ totals)
{
    unsigned long long s0 = 0ull, s1 = 0ull, s2 = 0ull;
    for (int i = (int)threadIdx.x; i < g; i += VERIFY_THREADS) {
        s0 += parts[3 * i + 0];
        s1 += parts[3 * i + 1];
        s2 += parts[3 * i + 2];
    }
    __shared__ unsigned long long red[VERIFY_THREADS / 64][3];
    for (int o = 32; o >= 1; o >>= 1) {
        s0 += __shfl_xor(s0, o, 64);
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
    }
    const int wave = (int)(threadIdx.x >> 6);
    if (__lane_id() == 0) {
        red[wave][0] = s0;
        red[wave][1] = s1;
        red[wave][2] = s2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long s = 0ull;
        for (int w = 0; w < VERIFY_THREADS / 64; ++w) s += red[w][threadIdx.x];
        totals[threadIdx.x] = s;
    }
}

// workgroups of the partial pass for P pixels
static int verify_grid(int P, bool vec)
{
    const int units = vec ? (P >> 3) : P;
    int g = (units + VERIFY_THREADS - 1) / VERIFY_THREADS;
    if (g < 1) g = 1;
    return g < VERIFY_MAX_PARTS ? g : VERIFY_MAX_PARTS;
}

// Runs the two passes on `s` with `work` (3 * VERIFY_MAX_PARTS + 3 device
// u64: partials, then the totals), copies the totals to the host and derives
// the outputs. Synchronous on `s`.
static int verify_run(const uint16_t *da, const uint16_t *db, int32_t W, int32_t H, unsigned long long *work,
                      double *valid_frac, double *mu_m, int32_t *accept, hipStream_t s)
{
    const int P = W * H;
    const bool vec = (((uintptr_t)da | (uintptr_t)db) & 15u) == 0u;
    const int g = verify_grid(P, vec);
    unsigned long long *totals = work + 3 * VERIFY_MAX_PARTS;
    if (vec)
        RL_LAUNCH("k_verify", k_verify_vec, dim3(g), dim3(VERIFY_THREADS), 0, s, da, db, P, work);
    else
        RL_LAUNCH("k_verify", k_verify_px, dim3(g), dim3(VERIFY_THREADS), 0, s, da, db, P, work);
    RL_LAUNCH("k_verify_total", k_verify_total, dim3(1), dim3(VERIFY_THREADS), 0, s, work, g, totals);
    RL_HIP(hipGetLastError());
    unsigned long long h[3] = {0ull, 0ull, 0ull};
    RL_HIP(hipMemcpyAsync(h, totals, sizeof(h), hipMemcpyDeviceToHost, s));
    RL_HIP(hipStreamSynchronize(s));
    *valid_frac = (double)h[0] / (double)P;
    *mu_m = h[1] ? ((double)h[2] / (double)h[1]) / 1000.0 : INFINITY;
    *accept = (*valid_frac > 0.5 && *mu_m < 0.05) ? 1 : 0;
    return RELOC_OK;
}

static bool verify_args_ok(const uint16_t *da, const uint16_t *db, int32_t W, int32_t H, const double *vf,
                           const double *mu, const int32_t *acc)
{
    return da && db && W >= 1 && H >= 1 && W <= 8191 && H <= 8191 && vf && mu && acc;
}

}  // namespace rl

using namespace rl;

extern "C" int reloc_verify(const uint16_t *da_dev, const uint16_t *db_dev, int32_t W, int32_t H, double *valid_frac,
                            double *mu_m, int32_t *accept, void *stream)
{
    if (!verify_args_ok(da_dev, db_dev, W, H, valid_frac, mu_m, accept)) return RELOC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *work = nullptr;
    RL_HIP(hipMallocAsync((void **)&work, (3 * VERIFY_MAX_PARTS + 3) * sizeof(unsigned long long), s));
    const int rc = verify_run(da_dev, db_dev, W, H, work, valid_frac, mu_m, accept, s);
    const hipError_t e = hipFreeAsync(work, s);
    if (rc) return rc;
    return e == hipSuccess ? RELOC_OK : RELOC_E_HIP;
}

// ---- the allocation-free variant ---------------------------------------------
//
// For callers that cannot allocate device memory (graph capture, tight
// serving loops): the partials and totals live in a file-scope device array,
// one copy per GPU, held until the process ends. Its device address is looked
// up once per device, with that device current, and kept; the host never
// passes the array's name itself to a kernel or a copy.

namespace {

constexpr int NOALLOC_WORDS = 3 * VERIFY_MAX_PARTS + 3;   // 49 176 bytes
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned long long scratch[NOALLOC_WORDS];

std::mutex scratch_mu;
unsigned long long *scratch_ptr[MAX_DEVICES] = {};

int scratch_of_current_device(unsigned long long **out)
{
    int dev = -1;
    RL_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return RELOC_E_STATE;
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RELOC_E_HIP;
        scratch_ptr[dev] = (unsigned long long *)p;
    }
    *out = scratch_ptr[dev];
    return RELOC_OK;
}

}  // namespace

extern "C" int reloc_verify_noalloc(const uint16_t *da_dev, const uint16_t *db_dev, int32_t W, int32_t H,
                                    double *valid_frac, double *mu_m, int32_t *accept, void *stream)
{
    if (!verify_args_ok(da_dev, db_dev, W, H, valid_frac, mu_m, accept)) return RELOC_E_ARG;
    unsigned long long *work = nullptr;
    const int rc = scratch_of_current_device(&work);
    if (rc) return rc;
    return verify_run(da_dev, db_dev, W, H, work, valid_frac, mu_m, accept, (hipStream_t)stream);
}
