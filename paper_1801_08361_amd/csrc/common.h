// Internal definitions shared by the HIP translation units of libreloc.
//
// Everything here is gfx950 device code or host glue for it. Floating-point
// code is compiled with -ffp-contract=off: each operation is the IEEE
// operation written, and fused multiply-adds appear only where the method
// defines one (fmaf). Integer parts (features, traversal, reservoir ranks and
// slots, cluster membership) are exact by construction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "reloc.h"

namespace rl {

// ---------------------------------------------------------------------------
// status helpers
// ---------------------------------------------------------------------------

#define RL_HIP(expr)                                      \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return RELOC_E_HIP;         \
    } while (0)

// optional per-kernel event timing (prof.hip)
bool prof_on();
void *prof_begin(const char *name, hipStream_t s);
void prof_end(const char *name, void *tok, hipStream_t s);
// queues a wait of a fixed wall-clock time for a timed pass of `launches`
// launches (so that the host can queue them all before the first one runs)
void prof_delay(hipStream_t s, int launches);

#define RL_LAUNCH(name, kern, grid, block, smem, stream, ...)                  \
    do {                                                                      \
        void *tok_ = prof_on() ? prof_begin(name, stream) : nullptr;          \
        hipLaunchKernelGGL(kern, grid, block, smem, stream, __VA_ARGS__);     \
        prof_end(name, tok_, stream);                                         \
    } while (0)

// ---------------------------------------------------------------------------
// device data layouts
// ---------------------------------------------------------------------------

// one reservoir sample: world position in integer mm and the pixel colour
struct Entry {
    int32_t x, y, z;
    uint32_t rgb;     // r | g << 8 | b << 16
};
static_assert(sizeof(Entry) == 16, "entry layout");

// one leaf mode: mean (m), inverse covariance (m^-2: xx xy xz yy yz zz),
// kappa = -log(pi) + 0.5 (3 log 2 pi + log det Sigma), cluster size, colour
struct Mode {
    float mu[3];
    float sinv[6];
    float kappa;
    int32_t n;
    uint32_t rgb;
};
static_assert(sizeof(Mode) == 48, "mode layout");

// one pose hypothesis: FP64 pose and its FP32 rounding used for scoring
struct Hyp {
    double R[9], t[3];
    float R32[9], t32[3];
};

// correspondence sums: n, sum c (3), sum w (3), sum c w^T (9, row a col b),
// sum c c^T (xx xy xz yy yz zz)
constexpr int NSUM = 22;

// result of one attempt: the public reloc_result
using Result = reloc_result;

constexpr uint64_t TAG_FOREST = 1, TAG_RESERVOIR = 2, TAG_HYP = 3, TAG_PIX = 4, TAG_TRAIN = 8;

constexpr int GROUP = 8;        // energy partial sums run over 8 consecutive draws
constexpr int CHUNK = 4096;     // pixels per reservoir-rank chunk
constexpr int MAX_HYP = 4096;
constexpr int MAX_B = 2048;
constexpr int MAX_R = 1024;
constexpr int MAX_M = 64;       // modes per leaf
constexpr int MAX_TM = 512;     // modes over all trees of one pixel (T * M)
constexpr int MAX_ROUNDS = 13;  // ceil(log2(MAX_HYP)) + 1

// mode colour rows: M colours padded to a multiple of 4 (16-byte rows for
// vector loads); slots without a mode hold RGB_NONE (a real colour has a zero
// top byte)
constexpr uint32_t RGB_NONE = 0xFFFFFFFFu;
__host__ __device__ __forceinline__ int rgb_stride(int M) { return (M + 3) & ~3; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC 2011) and the integer range map
// ---------------------------------------------------------------------------

struct U4 { uint64_t x[4]; };

__device__ __forceinline__ U4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                     uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        uint64_t lo0 = m0 * c0, hi0 = __umul64hi(m0, c0);
        uint64_t lo1 = m1 * c2, hi1 = __umul64hi(m1, c2);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    U4 o;
    o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
    return o;
}

// floor(u * n / 2^64)
__device__ __forceinline__ uint64_t uniform_int(uint64_t u, uint64_t n) { return __umul64hi(u, n); }

// ---------------------------------------------------------------------------
// packed split node (8 bytes): kind 2 bits | dx 21 | dy 21 | thr 20 (signed)
// ---------------------------------------------------------------------------

constexpr int32_t NODE_OFF_MAX = (1 << 20) - 1;
constexpr int32_t NODE_THR_MAX = (1 << 19) - 1;

__host__ __device__ __forceinline__ uint64_t pack_node(int32_t kind, int32_t dx, int32_t dy, int32_t thr)
{
    return (uint64_t)(uint32_t)(kind & 3) | ((uint64_t)((uint32_t)dx & 0x1FFFFFu) << 2) |
           ((uint64_t)((uint32_t)dy & 0x1FFFFFu) << 23) | ((uint64_t)((uint32_t)thr & 0xFFFFFu) << 44);
}

__host__ __device__ __forceinline__ void unpack_node(uint64_t w, int32_t &kind, int32_t &dx, int32_t &dy,
                                                     int32_t &thr)
{
    kind = (int32_t)(w & 3u);
    dx = (int32_t)((int64_t)(w << 41) >> 43);
    dy = (int32_t)((int64_t)(w << 20) >> 43);
    thr = (int32_t)((int64_t)w >> 44);
}

// A split from four generator words: kind from u0 (0-2 depth, 3-5 colour
// channel 1-3), offsets dx, dy uniform in [-O, O] from u1, u2, threshold
// uniform in [-T, T] from u3, with T the depth or the colour threshold range
__device__ __forceinline__ uint64_t split_from_draw(const U4 &u, int32_t O, int32_t thr_d, int32_t thr_c)
{
    const int32_t k = (int32_t)uniform_int(u.x[0], 6);
    const int32_t kind = k < 3 ? 0 : k - 2;
    const int64_t Ow = 2 * (int64_t)O + 1;
    const int32_t dx = (int32_t)((int64_t)uniform_int(u.x[1], (uint64_t)Ow) - O);
    const int32_t dy = (int32_t)((int64_t)uniform_int(u.x[2], (uint64_t)Ow) - O);
    const int32_t Tk = kind == 0 ? thr_d : thr_c;
    const int32_t thr = (int32_t)((int64_t)uniform_int(u.x[3], (uint64_t)(2 * (int64_t)Tk + 1)) - Tk);
    return pack_node(kind, dx, dy, thr);
}

// ---------------------------------------------------------------------------
// frames
// ---------------------------------------------------------------------------

// Pointers that device code reads out of device memory (the batch's attempt
// descriptors) are generic unless declared global: the compiler then issues
// flat loads, which also count against the LDS/scalar wait counter, so that
// every wait for an LDS or scalar result waits for them too. In the device
// pass these members are global-address-space pointers; the host pass sees
// plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define RL_GLOBAL __attribute__((address_space(1)))
#else
#define RL_GLOBAL
#endif

struct Frame {
    const uint16_t RL_GLOBAL *__restrict__ depth;
    const uint8_t RL_GLOBAL *__restrict__ rgb;
    int32_t W, H;
    float fx, fy, cx, cy;
    int32_t Fx, Fy;       // focal lengths in 1/16 px, rounded half up
    int32_t dmin, dmax, Fref;
};

__device__ __forceinline__ bool valid_depth(const Frame &fr, uint32_t d)
{
    return (int32_t)d >= fr.dmin && (int32_t)d <= fr.dmax;
}

// camera-frame point, one IEEE float operation at a time in this order
__device__ __forceinline__ void cam_point(const Frame &fr, int u, int v, uint32_t d, float c[3])
{
    float z = (float)d * 0.001f;
    c[0] = ((float)u - fr.cx) * z / fr.fx;
    c[1] = ((float)v - fr.cy) * z / fr.fy;
    c[2] = z;
}

// The divisor of a pixel's probe offsets, D = d * F_ref, turned into a
// multiplier for exact truncating division by multiplication (Granlund and
// Montgomery, 1994): with l = ceil(log2 D) and m = ceil(2^(31 + l) / D), which
// is below 2^32, every 0 <= a < 2^31 has floor(a / D) = floor(2a m / 2^(32 + l)):
// the high word of the 32 x 32-bit product (2a) m, shifted right by l.
// (Write m = (2^(31 + l) + e) / D with 0 <= e < D; then a m / 2^(31 + l)
// exceeds a / D by less than 2^-l <= 1 / D, which cannot reach the next
// integer.)
struct PixelDen {
    uint32_t magic;
    uint32_t shift;
};

__host__ __device__ __forceinline__ PixelDen pixel_den_of(uint32_t D)
{
    PixelDen p;
    const uint32_t l = D > 1u ? 32u - (uint32_t)__builtin_clz(D - 1u) : 0u;
    p.shift = l;
    p.magic = (uint32_t)(((1ull << (31u + l)) + (uint64_t)D - 1ull) / (uint64_t)D);
    return p;
}

__device__ __forceinline__ PixelDen pixel_den(const Frame &fr, int32_t d)
{
    return pixel_den_of((uint32_t)(d * fr.Fref));
}

// floor(a / D) for a2 = 2a, a < 2^31
__host__ __device__ __forceinline__ uint32_t div_mag2(uint32_t a2, const PixelDen &p)
{
    return (uint32_t)(((uint64_t)a2 * (uint64_t)p.magic) >> 32) >> p.shift;
}

// trunc(n / D) for |n| < 2^31
__host__ __device__ __forceinline__ int32_t div_trunc(int32_t n, const PixelDen &p)
{
    const uint32_t an = (uint32_t)(n < 0 ? -n : n);
    const uint32_t q = div_mag2(an << 1, p);
    return n < 0 ? -(int32_t)q : (int32_t)q;
}

// Response of a packed node at pixel (u, v) with valid depth d (mm). The probe
// offset is trunc(delta * F / (d * F_ref)); all products fit in 32 bits (the
// host checks |delta| * F < 2^31). Depth probes outside the image or on an
// invalid depth read 65535; colour probes clamp to the border.
__device__ __forceinline__ int32_t node_response_d(const Frame &fr, uint64_t w, int u, int v, int32_t d,
                                                   const PixelDen &pd, int32_t &thr)
{
    int32_t kind, dx, dy;
    unpack_node(w, kind, dx, dy, thr);
    int32_t qx = u + div_trunc(dx * fr.Fx, pd);
    int32_t qy = v + div_trunc(dy * fr.Fy, pd);
    if (kind == 0) {
        int32_t dq = 65535;
        if (qx >= 0 && qx < fr.W && qy >= 0 && qy < fr.H) {
            uint32_t z = fr.depth[qy * fr.W + qx];
            if (valid_depth(fr, z)) dq = (int32_t)z;
        }
        return dq - d;
    }
    int c = kind - 1;
    qx = qx < 0 ? 0 : (qx > fr.W - 1 ? fr.W - 1 : qx);
    qy = qy < 0 ? 0 : (qy > fr.H - 1 ? fr.H - 1 : qy);
    return (int32_t)fr.rgb[(qy * fr.W + qx) * 3 + c] - (int32_t)fr.rgb[(v * fr.W + u) * 3 + c];
}

// implicit heap: children of node i are 2i+1 (left) and 2i+2 (right); go
// right iff response >= threshold; leaf = i - (L - 1)
__device__ __forceinline__ int32_t traverse_d(const uint64_t *__restrict__ tree, int32_t L, const Frame &fr, int u,
                                              int v, int32_t d, const PixelDen &pd)
{
    int32_t i = 0;
    while (i < L - 1) {
        int32_t thr;
        int32_t r = node_response_d(fr, tree[i], u, v, d, pd, thr);
        i = 2 * i + 1 + (r >= thr ? 1 : 0);
    }
    return i - (L - 1);
}

__device__ __forceinline__ int32_t traverse(const uint64_t *__restrict__ tree, int32_t L, const Frame &fr, int u,
                                            int v, int32_t d)
{
    return traverse_d(tree, L, fr, u, v, d, pixel_den(fr, d));
}

// ---------------------------------------------------------------------------
// whole-frame traversal: the workgroup keeps the top levels of its tree in
// LDS, unpacked and with the offsets already multiplied by the frame's focal
// lengths; each pixel's divisor and own colour are set up once
// ---------------------------------------------------------------------------

constexpr int TOP_NODES = 1023;   // levels 0..9, 32 KB prepared

// One pixel of a frame packed for probing: four 16-bit fields, each holding
// the complement of its value, so that every probe's response is the pixel's
// own field minus the probed one and a zero field reads as "no depth". Bits
// 0-15 hold 65535 - z, where z is the depth, or 65535 outside the valid
// range (the host keeps the range below 65535), so an invalid pixel's field
// is 0; bits 16-31, 32-47 and 48-63 hold 255 - r, 255 - g and 255 - b.
__device__ __forceinline__ uint64_t pack_pixel(const Frame &fr, int64_t p)
{
    const uint32_t d = fr.depth[p];
    const uint64_t z = valid_depth(fr, d) ? (uint64_t)(65535u - d) : 0ull;
    return z | ((uint64_t)(255u - fr.rgb[p * 3]) << 16) | ((uint64_t)(255u - fr.rgb[p * 3 + 1]) << 32) |
           ((uint64_t)(255u - fr.rgb[p * 3 + 2]) << 48);
}

__device__ __forceinline__ bool packed_valid(uint64_t w) { return (w & 0xFFFFull) != 0ull; }

// the depth of a packed pixel (65535 where it is invalid)
__device__ __forceinline__ uint32_t packed_depth(uint64_t w) { return 65535u - (uint32_t)(w & 0xFFFFull); }

// colour channel c (0 r, 1 g, 2 b) of a packed pixel
__device__ __forceinline__ uint32_t packed_colour(uint64_t w, int c)
{
    return 255u - ((uint32_t)(w >> (16 + 16 * c)) & 0xFFFFu);
}

// A split node prepared for one frame: its offsets multiplied by the focal
// lengths, as the doubled magnitudes that div_mag2 takes and their signs, the
// threshold, and where its channel sits in a packed pixel word.
struct ProbeNode {
    uint32_t ax, ay;   // 2 |dx Fx|, 2 |dy Fy|
    uint32_t sxy;      // signs of dx Fx (bits 0-15) and dy Fy (bits 16-31) as 16-bit +1 or -1
    uint32_t spare;
    int32_t thr;
    uint32_t sh;       // bits 0-5: 16 kind, the field's bit position in the word (bits 0-4: in its
                       // 32-bit half); higher bits are not read
    uint32_t half;     // byte offset of the field's 32-bit half in the word (0 or 4)
    uint32_t wout;     // width the field is read with when the probe leaves the image: 0 for a depth
                       // probe (no depth), 16 for a colour probe (the clamped pixel's colour)
};

__device__ __forceinline__ ProbeNode probe_node(uint64_t w, const Frame &fr)
{
    int32_t kind, dx, dy, thr;
    unpack_node(w, kind, dx, dy, thr);
    const int32_t nx = dx * fr.Fx, ny = dy * fr.Fy;
    ProbeNode n;
    n.ax = (uint32_t)(nx < 0 ? -nx : nx) << 1;
    n.ay = (uint32_t)(ny < 0 ? -ny : ny) << 1;
    n.sxy = (nx < 0 ? 0xFFFFu : 1u) | ((ny < 0 ? 0xFFFFu : 1u) << 16);
    n.spare = 0u;
    n.thr = thr;
    n.sh = 16u * (uint32_t)kind;
    n.half = 2u * (uint32_t)(kind & 2);
    n.wout = kind ? 16u : 0u;
    return n;
}

// A split node as the deep levels of the traversal read it, 16 bytes that do
// not depend on the frame: x and y hold 2 |dx| and 2 |dy| in bits 0-21 and
// the offset's sign in bit 31; meta holds 16 kind in bits 0-5, the byte
// offset of the field's 32-bit half (0 or 4) in bits 6-8 and the width the
// field is read with outside the image (0 or 16) in bits 9-13.
struct DeepNode {
    uint32_t x, y;
    int32_t thr;
    uint32_t meta;
};

__host__ __device__ __forceinline__ DeepNode deep_node(uint64_t w)
{
    int32_t kind, dx, dy, thr;
    unpack_node(w, kind, dx, dy, thr);
    DeepNode d;
    d.x = ((uint32_t)(dx < 0 ? -dx : dx) << 1) | (dx < 0 ? 0x80000000u : 0u);
    d.y = ((uint32_t)(dy < 0 ? -dy : dy) << 1) | (dy < 0 ? 0x80000000u : 0u);
    d.thr = thr;
    d.meta = 16u * (uint32_t)kind | ((kind & 2) ? 4u : 0u) << 6 | (kind ? 16u : 0u) << 9;
    return d;
}

// probe_node of a DeepNode: the focal lengths (below 2^24, checked by the
// host) scale 2 |dx| and 2 |dy| with 24-bit multiplies; the signs of dx Fx,
// dy Fy are those of dx, dy. sh keeps the meta word: only its low 6 bits are
// read.
__device__ __forceinline__ ProbeNode probe_node_deep(const DeepNode &d, const Frame &fr)
{
    ProbeNode n;
    n.ax = __umul24(d.x, (uint32_t)fr.Fx);
    n.ay = __umul24(d.y, (uint32_t)fr.Fy);
    n.sxy = ((uint32_t)(((int32_t)d.x >> 31) | 1) & 0xFFFFu) | ((uint32_t)(((int32_t)d.y >> 31) | 1) << 16);
    n.spare = 0u;
    n.thr = d.thr;
    n.sh = d.meta;
    n.half = __builtin_amdgcn_ubfe(d.meta, 6, 3);
    n.wout = __builtin_amdgcn_ubfe(d.meta, 9, 5);
    return n;
}

__device__ __forceinline__ void stage_top(ProbeNode *__restrict__ top, const uint64_t *__restrict__ tree, int ntop,
                                          const Frame &fr, int tid, int nthreads)
{
    for (int k = tid; k < ntop; k += nthreads) top[k] = probe_node(tree[k], fr);
}

// A buffer resource over a packed frame of P words (P < 2^26: the host keeps
// width and height at most 8191): probe loads take a 32-bit byte offset from
// it, and the hardware range-checks them against the P * 8 bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t packed_rsrc(const uint64_t *packed, int P)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)packed, (short)0, P * 8, 0x00020000);
}

typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));

// node_response_d of a prepared node, from the packed frame: `own` is the
// pixel's own packed word. Branch-free: the probe position is clamped into
// the image and the field's 32-bit half is loaded; a depth probe whose
// position was clamped reads its field with width 0, that is as "no depth".
// Both coordinates are placed, clamped and turned into the byte offset
// together as 16-bit lanes (x low, y high): the host keeps W and H below 8192
// and every probe offset below 2^14, so u + o, v + o and 8 W fit the lanes.
__device__ __forceinline__ int32_t probe_response(__amdgpu_buffer_rsrc_t packed, int W, int H, int u, int v,
                                                  uint64_t own, const PixelDen &pd, const ProbeNode &n)
{
    const uint32_t ox = div_mag2(n.ax, pd), oy = div_mag2(n.ay, pd);
    const i16x2 o = __builtin_bit_cast(i16x2, ox | (oy << 16));
    const i16x2 uv = __builtin_bit_cast(i16x2, (uint32_t)u | ((uint32_t)v << 16));
    const i16x2 q = o * __builtin_bit_cast(i16x2, n.sxy) + uv;
    const i16x2 zero = {0, 0};
    const i16x2 hi = __builtin_bit_cast(i16x2, (uint32_t)(W - 1) | ((uint32_t)(H - 1) << 16));
    const i16x2 c = __builtin_elementwise_min(__builtin_elementwise_max(q, zero), hi);
    // (c.y W + c.x) 8 + half
    const u16x2_t rowb = __builtin_bit_cast(u16x2_t, 8u | ((uint32_t)(8 * W) << 16));
    const uint32_t at = __builtin_amdgcn_udot2(__builtin_bit_cast(u16x2_t, c), rowb, n.half, false);
    const uint32_t word = __builtin_bit_cast(uint32_t, __builtin_amdgcn_raw_buffer_load_b32(packed, (int)at, 0, 0));
    const uint32_t width = __builtin_bit_cast(uint32_t, q) != __builtin_bit_cast(uint32_t, c) ? n.wout : 16u;
    const uint32_t probed = __builtin_amdgcn_ubfe(word, n.sh, width);
    const uint32_t mine = (uint32_t)(own >> (n.sh & 63u)) & 0xFFFFu;
    return (int32_t)mine - (int32_t)probed;
}

// Traversal of one tree for K pixels of a packed frame at once (their
// chains of dependent probe loads interleave): every leaf of a complete tree
// lies at the same depth, so the K node indices stay on one level. Pixel k is
// p[k] with packed word own[k]; lanes whose pixel is invalid (ok[k] false)
// walk with the smallest valid depth on a clamped position and get -1. In
// the prepared top levels a node is tracked by its byte offset (32 per node);
// the levels below read the tree's DeepNodes.
template <int K>
__device__ __forceinline__ void traverse_packed_k(const ProbeNode *__restrict__ top, int32_t ntop,
                                                  const DeepNode *__restrict__ tree, int32_t L, const Frame &fr,
                                                  const uint64_t *__restrict__ packed, const int p[K],
                                                  const uint64_t own[K], const bool ok[K], int32_t leaf[K])
{
    static_assert(sizeof(ProbeNode) == 32, "prepared nodes are 32 bytes");
    const __amdgpu_buffer_rsrc_t rs = packed_rsrc(packed, fr.W * fr.H);
    PixelDen pd[K];
    int u[K], v[K];
    uint32_t o[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        u[k] = p[k] % fr.W;
        v[k] = p[k] / fr.W;
        pd[k] = pixel_den(fr, ok[k] ? (int32_t)packed_depth(own[k]) : fr.dmin);
        o[k] = 0;
    }
    const uint32_t otop = (uint32_t)ntop * 32u;
    const char *tb = (const char *)top;
    while (o[0] < otop) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const ProbeNode n = *(const ProbeNode *)__builtin_assume_aligned(tb + o[k], 32);
            const int32_t r = probe_response(rs, fr.W, fr.H, u[k], v[k], own[k], pd[k], n);
            // child 2 i + 1 + (r >= thr) at byte offset 2 o + 32 + 32 (r >= thr)
            o[k] = 2u * o[k] + (r >= n.thr ? 64u : 32u);
        }
    }
    // below: byte offsets into the tree's DeepNodes (16 per node), read
    // through a buffer resource over its (L - 1) 16 bytes (below 2^20)
    const __amdgpu_buffer_rsrc_t ts = __builtin_amdgcn_make_buffer_rsrc((void *)tree, (short)0, (L - 1) * 16,
                                                                        0x00020000);
    const uint32_t oend = (uint32_t)(L - 1) * 16u;
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] >>= 1;
    while (o[0] < oend) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const DeepNode d =
                __builtin_bit_cast(DeepNode, __builtin_amdgcn_raw_buffer_load_b128(ts, (int)o[k], 0, 0));
            const ProbeNode n = probe_node_deep(d, fr);
            const int32_t r = probe_response(rs, fr.W, fr.H, u[k], v[k], own[k], pd[k], n);
            o[k] = 2u * o[k] + (r >= n.thr ? 32u : 16u);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) leaf[k] = ok[k] ? (int32_t)(o[k] >> 4) - (L - 1) : -1;
}


// ---------------------------------------------------------------------------
// FP64 rigid alignment from correspondence sums (Horn's unit-quaternion
// method, 1987: the rotation maximising tr(R H^T) is given by the eigenvector
// of the largest eigenvalue of a symmetric 4x4 matrix built from H)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void sums_add_point(double s[NSUM], const float c[3], const float w[3])
{
    double cd[3] = {c[0], c[1], c[2]}, wd[3] = {w[0], w[1], w[2]};
    s[0] = s[0] + 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[1 + a] = s[1 + a] + cd[a];
        s[4 + a] = s[4 + a] + wd[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) s[7 + a * 3 + b] = s[7 + a * 3 + b] + cd[a] * wd[b];
    s[16] = s[16] + cd[0] * cd[0];
    s[17] = s[17] + cd[0] * cd[1];
    s[18] = s[18] + cd[0] * cd[2];
    s[19] = s[19] + cd[1] * cd[1];
    s[20] = s[20] + cd[1] * cd[2];
    s[21] = s[21] + cd[2] * cd[2];
}

// Reciprocal for the alignment's normalisations, pivots and Newton steps
// (none of which needs a correctly rounded quotient): on the device the
// hardware estimate refined by two Newton-Raphson steps (each squares the
// relative error), within about an ulp; on the host the division. The
// divisors here are finite and non-zero where the reciprocal is used.
__host__ __device__ __forceinline__ double rcp_d(double b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / b;
#endif
}

// Top-eigenspace vector of a symmetric 4x4 matrix by power iteration on
// N + s I with s = sqrt(tr N^2) (which makes every eigenvalue non-negative,
// the largest one largest in magnitude), from (1, 0, 0, 0). Only the
// degenerate inputs that the closed-form step declines come here (N = 0,
// where it returns (1, 0, 0, 0), or an exactly repeated largest eigenvalue,
// where any vector of that eigenspace is a best rotation).
__device__ __forceinline__ void power_top(const double N[16], double q[4])
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s = s + N[k] * N[k];
    s = sqrt(s);
    q[0] = 1.0; q[1] = 0.0; q[2] = 0.0; q[3] = 0.0;
    if (!(s > 0.0)) return;
    for (int it = 0; it < 200; ++it) {
        double y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            y[i] = ((N[i * 4] * q[0] + N[i * 4 + 1] * q[1]) + (N[i * 4 + 2] * q[2] + N[i * 4 + 3] * q[3])) + s * q[i];
        const double n = sqrt(((y[0] * y[0] + y[1] * y[1]) + y[2] * y[2]) + y[3] * y[3]);
        if (!(n > 0.0)) return;
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = y[i] / n;
    }
}

// Horn's symmetric 4x4 matrix of the cross-covariance H (H[a][b] = sum of
// centred c_a w_b): its top eigenvector is the quaternion of the rotation
// that best maps the c onto the w
__host__ __device__ __forceinline__ void horn_matrix(const double H[9], double N[16])
{
    const double Sxx = H[0], Sxy = H[1], Sxz = H[2], Syx = H[3], Syy = H[4], Syz = H[5], Szx = H[6], Szy = H[7],
                 Szz = H[8];
    N[0] = (Sxx + Syy) + Szz; N[1] = Syz - Szy;         N[2] = Szx - Sxz;          N[3] = Sxy - Syx;
    N[4] = Syz - Szy;         N[5] = (Sxx - Syy) - Szz; N[6] = Sxy + Syx;          N[7] = Szx + Sxz;
    N[8] = Szx - Sxz;         N[9] = Sxy + Syx;         N[10] = (-Sxx + Syy) - Szz; N[11] = Syz + Szy;
    N[12] = Sxy - Syx;        N[13] = Szx + Sxz;        N[14] = Syz + Szy;         N[15] = (-Sxx - Syy) + Szz;
}

// determinant of rows r0 < r1 < r2 and columns c0 < c1 < c2 of a row-major 4x4
__host__ __device__ __forceinline__ double det3_of(const double A[16], int r0, int r1, int r2, int c0, int c1, int c2)
{
    return (A[r0 * 4 + c0] * (A[r1 * 4 + c1] * A[r2 * 4 + c2] - A[r1 * 4 + c2] * A[r2 * 4 + c1]) -
            A[r0 * 4 + c1] * (A[r1 * 4 + c0] * A[r2 * 4 + c2] - A[r1 * 4 + c2] * A[r2 * 4 + c0])) +
           A[r0 * 4 + c2] * (A[r1 * 4 + c0] * A[r2 * 4 + c1] - A[r1 * 4 + c1] * A[r2 * 4 + c0]);
}

// the 3x3 minor of a 4x4 without row i and column j (i, j compile-time after unrolling)
__host__ __device__ __forceinline__ double minor4(const double A[16], int i, int j)
{
    const int r0 = i == 0 ? 1 : 0, r1 = i <= 1 ? 2 : 1, r2 = i <= 2 ? 3 : 2;
    const int c0 = j == 0 ? 1 : 0, c1 = j <= 1 ? 2 : 1, c2 = j <= 2 ? 3 : 2;
    return det3_of(A, r0, r1, r2, c0, c1, c2);
}

// Largest-eigenvalue eigenvector of Horn's traceless 4x4 matrix N built from
// the 3x3 cross-covariance H (Horn's quaternion method; the eigenvalue step is
// the quaternion characteristic polynomial method of Theobald). The
// eigenvalue is the largest root of
// det(N - l I) = l^4 + c2 l^2 + c1 l + c0 with c2 = -2 |H|_F^2,
// c1 = -8 det H, c0 = det N, reached by Newton's method from the upper bound
// sqrt(3) |H|_F (every root is real, so the iterates decrease monotonically
// onto it). A column of adj(N - l I) (the one on its largest diagonal entry)
// gives the eigenvector, and one step of inverse iteration with
// (N - l I), by elimination with partial pivoting, brings it to full
// accuracy. Returns false when no such column exists or a value is not
// finite (H = 0, or an exactly repeated largest eigenvalue).
__host__ __device__ __forceinline__ bool top_eigvec_horn(const double N[16], const double H[9], double q[4])
{
    double hf2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) hf2 = hf2 + H[k] * H[k];
    const double c2 = -2.0 * hf2;
    const double detH = (H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6])) +
                        H[2] * (H[3] * H[7] - H[4] * H[6]);
    const double c1 = -8.0 * detH;
    double c0 = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) c0 = c0 + ((j & 1) ? -N[j] : N[j]) * minor4(N, 0, j);
    double lam = sqrt(3.0 * hf2);
    if (!(lam > 0.0)) return false;
    if (fabs(detH) <= 1e-9 * hf2 * lam) {
        // H nearly of rank 2 (three correspondences): the polynomial is
        // nearly l^4 + c2 l^2 + c0, whose largest root is closed-form. After
        // one Newton step from it, a point just above is a tighter start
        // whenever p, p' and p'' are positive there (Budan-Fourier: with the
        // constant p''' and p'''' positive too, no root lies above it);
        // otherwise the bound above stays. Newton from sqrt(3) |H|_F takes
        // about 9 steps here, from this start about 2.
        const double disc = c2 * c2 - 4.0 * c0;
        double x = sqrt(0.5 * (sqrt(disc > 0.0 ? disc : 0.0) - c2));
        const double p0 = ((x * x + c2) * x + c1) * x + c0, d0 = (4.0 * (x * x) + 2.0 * c2) * x + c1;
        if (d0 > 0.0) x = x - p0 * rcp_d(d0);
        x = x * (1.0 + 1e-9);
        const double p1 = ((x * x + c2) * x + c1) * x + c0, d1 = (4.0 * (x * x) + 2.0 * c2) * x + c1;
        if (p1 >= 0.0 && d1 > 0.0 && 12.0 * (x * x) + 2.0 * c2 > 0.0 && x > 0.0 && x < lam) lam = x;
    }
    for (int it = 0; it < 64; ++it) {
        const double l2 = lam * lam;
        const double p = ((l2 + c2) * lam + c1) * lam + c0;
        const double dp = (4.0 * l2 + 2.0 * c2) * lam + c1;
        if (!(dp > 0.0)) break;
        const double st = p * rcp_d(dp);
        if (!(st > 1e-15 * lam)) {
            if (st > 0.0) lam = lam - st;
            break;
        }
        lam = lam - st;
    }
    double A[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) A[k] = (k % 5 == 0) ? N[k] - lam : N[k];
    // adjugate column on the largest diagonal cofactor
    double d[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) d[j] = minor4(A, j, j);
    int jm = 0;
#pragma unroll
    for (int j = 1; j < 4; ++j)
        if (fabs(d[j]) > fabs(d[jm])) jm = j;
    // the columns of A other than jm, in order (the same 3x3 determinants as
    // minor4(A, i, jm), without forming the other columns' minors)
    double Bc[12];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Bc[r * 3 + c] = c < jm ? A[r * 4 + c] : A[r * 4 + c + 1];
    double v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r0 = i == 0 ? 1 : 0, r1 = i <= 1 ? 2 : 1, r2 = i <= 2 ? 3 : 2;
        const double m = (Bc[r0 * 3] * (Bc[r1 * 3 + 1] * Bc[r2 * 3 + 2] - Bc[r1 * 3 + 2] * Bc[r2 * 3 + 1]) -
                          Bc[r0 * 3 + 1] * (Bc[r1 * 3] * Bc[r2 * 3 + 2] - Bc[r1 * 3 + 2] * Bc[r2 * 3])) +
                         Bc[r0 * 3 + 2] * (Bc[r1 * 3] * Bc[r2 * 3 + 1] - Bc[r1 * 3 + 1] * Bc[r2 * 3]);
        v[i] = ((i + jm) & 1) ? -m : m;
    }
    double vn = sqrt(((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]) + v[3] * v[3]);
    if (!(vn > 0.0) || !(vn < INFINITY)) return false;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = v[i] * rcp_d(vn);
    // one step of inverse iteration: solve (N - l I) x = v (reciprocal
    // pivots, reused by the back substitution)
    const double floor_ = 1e-17 * lam;
    double rpiv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int p = k;
        double best = fabs(A[k * 4 + k]);
#pragma unroll
        for (int i = k + 1; i < 4; ++i)
            if (fabs(A[i * 4 + k]) > best) {
                best = fabs(A[i * 4 + k]);
                p = i;
            }
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            const bool sw = p == i;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double a = A[k * 4 + j], b = A[i * 4 + j];
                A[k * 4 + j] = sw ? b : a;
                A[i * 4 + j] = sw ? a : b;
            }
            const double a = v[k], b = v[i];
            v[k] = sw ? b : a;
            v[i] = sw ? a : b;
        }
        double piv = A[k * 4 + k];
        if (fabs(piv) < floor_) piv = piv < 0.0 ? -floor_ : floor_;
        A[k * 4 + k] = piv;
        rpiv[k] = rcp_d(piv);
#pragma unroll
        for (int i = k + 1; i < 4; ++i) {
            const double f = A[i * 4 + k] * rpiv[k];
#pragma unroll
            for (int j = k + 1; j < 4; ++j) A[i * 4 + j] = A[i * 4 + j] - f * A[k * 4 + j];
            v[i] = v[i] - f * v[k];
        }
    }
    double x[4];
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        double r = v[k];
#pragma unroll
        for (int j = k + 1; j < 4; ++j) r = r - A[k * 4 + j] * x[j];
        x[k] = r * rpiv[k];
    }
    double mx = fmax(fmax(fabs(x[0]), fabs(x[1])), fmax(fabs(x[2]), fabs(x[3])));
    if (!(mx > 0.0) || !(mx < INFINITY)) return false;
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = x[k] * rcp_d(mx);
    return true;
}

// Pose from sums. Succeeds when n >= 3 and the camera points are spread in two
// directions: with S their centred scatter, the sum of S's principal 2x2
// minors must reach 1e-4 * n * trace(S).
__device__ __forceinline__ bool pose_from_sums(const double s[NSUM], double R[9], double t[3])
{
    double n = s[0];
    if (n < 3.0) return false;
    const double *c = s + 1, *w = s + 4, *cw = s + 7, *cc = s + 16;
    // one reciprocal per normalisation instead of a division per entry (the
    // solve is a latency chain on one lane)
    const double rn = rcp_d(n);
    double H[9], S[6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) H[a * 3 + b] = cw[a * 3 + b] - (c[a] * w[b]) * rn;
    S[0] = cc[0] - (c[0] * c[0]) * rn;
    S[1] = cc[1] - (c[0] * c[1]) * rn;
    S[2] = cc[2] - (c[0] * c[2]) * rn;
    S[3] = cc[3] - (c[1] * c[1]) * rn;
    S[4] = cc[4] - (c[1] * c[2]) * rn;
    S[5] = cc[5] - (c[2] * c[2]) * rn;
    double I2 = ((S[0] * S[3] - S[1] * S[1]) + (S[0] * S[5] - S[2] * S[2])) + (S[3] * S[5] - S[4] * S[4]);
    double tr = (S[0] + S[3]) + S[5];
    if (!(I2 >= (1e-4 * n) * tr)) return false;
    double N[16];
    horn_matrix(H, N);
    double q[4];
    if (!top_eigvec_horn(N, H, q)) power_top(N, q);
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double rq = rcp_d(qn);
    double q0 = q[0] * rq, qx = q[1] * rq, qy = q[2] * rq, qz = q[3] * rq;
    R[0] = q0 * q0 + qx * qx - qy * qy - qz * qz;
    R[1] = 2.0 * (qx * qy - q0 * qz);
    R[2] = 2.0 * (qx * qz + q0 * qy);
    R[3] = 2.0 * (qy * qx + q0 * qz);
    R[4] = q0 * q0 - qx * qx + qy * qy - qz * qz;
    R[5] = 2.0 * (qy * qz - q0 * qx);
    R[6] = 2.0 * (qz * qx - q0 * qy);
    R[7] = 2.0 * (qz * qy + q0 * qx);
    R[8] = q0 * q0 - qx * qx - qy * qy + qz * qz;
    double cm[3], wm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cm[k] = c[k] * rn;
        wm[k] = w[k] * rn;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        t[k] = wm[k] - ((R[k * 3 + 0] * cm[0] + R[k * 3 + 1] * cm[1]) + R[k * 3 + 2] * cm[2]);
    return true;
}


// ---------------------------------------------------------------------------
// cross-lane moves within a wavefront through the VALU (DPP and gfx950's
// permlane swaps) instead of the LDS crossbar: shorter latency on the serial
// chains of a single wavefront
// ---------------------------------------------------------------------------

// v of lane (lane ^ M), every lane active
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v)
{
    static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16 || M == 32, "xor of one lane bit");
    const int x = (int)v;
    if constexpr (M == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);     // quad_perm [1, 0, 3, 2]
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);     // quad_perm [2, 3, 0, 1]
    } else if constexpr (M == 4) {
        const int up = __builtin_amdgcn_mov_dpp(x, 0x104, 0xF, 0xF, true);     // row_shl:4, lane + 4
        const int dn = __builtin_amdgcn_mov_dpp(x, 0x114, 0xF, 0xF, true);     // row_shr:4, lane - 4
        return (uint32_t)((__lane_id() & 4) ? dn : up);
    } else if constexpr (M == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, true);    // row_ror:8
    } else if constexpr (M == 16) {
        // odd rows of the first operand swap with even rows of the second
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (__lane_id() & 16) ? p[0] : p[1];
    } else {
        // upper half of the first operand swaps with the lower half of the second
        const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (__lane_id() & 32) ? p[0] : p[1];
    }
}

template <int M>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v)
{
    return ((uint64_t)xor_lane<M>((uint32_t)(v >> 32)) << 32) | xor_lane<M>((uint32_t)v);
}

template <int M>
__device__ __forceinline__ double xor_lane_f64(double v)
{
    return __longlong_as_double((long long)xor_lane64<M>((uint64_t)__double_as_longlong(v)));
}

// lane j's value (j wavefront-uniform)
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int j)
{
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), j) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, j);
}

__device__ __forceinline__ double lane_f64(double v, int j)
{
    return __longlong_as_double((long long)lane_u64((uint64_t)__double_as_longlong(v), j));
}

// the value O lanes below within the lane's row of 16 (0 for the row's first
// O lanes), O in {1, 2, 4, 8}
template <int O>
__device__ __forceinline__ int row_up(int v)
{
    static_assert(O == 1 || O == 2 || O == 4 || O == 8, "row shift");
    return __builtin_amdgcn_mov_dpp(v, 0x110 + O, 0xF, 0xF, true);   // row_shr:O
}

// float -> uint32 key that sorts like the float (no NaN, no -0 here)
__device__ __forceinline__ uint32_t float_key(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// its inverse
__device__ __forceinline__ float key_float(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// ---------------------------------------------------------------------------
// the forest handle
// ---------------------------------------------------------------------------

struct Forest {
    reloc_params p;
    int T, D, L, R, M;
    int device;
    // forest state
    uint64_t *nodes = nullptr;     // [T][L-1] then 8 extra
    DeepNode *deep = nullptr;      // [T][L-1] the split nodes as deep traversal levels read them
    uint32_t *counter = nullptr;   // [T][L]
    uint32_t *base = nullptr;      // [T][L]
    Entry *res = nullptr;          // [T][L][R]
    uint32_t *stamp = nullptr;     // [T][L][R]
    Mode *modes = nullptr;         // [T][L][M]
    uint32_t *mode_rgb = nullptr;  // [T][L][rgb_stride(M)] colour of each mode (compact copy for hypothesis picks)
    float4 *leaf_in = nullptr;     // [T][L][4] per-leaf summary for the learned proposal's inputs
    int32_t *nmodes = nullptr;     // [T][L]
    uint32_t *dirty = nullptr;     // [T][L]
    uint32_t *dirty_list = nullptr;
    uint32_t *dirty_count = nullptr;
    unsigned long long *total_samples = nullptr;
    bool maybe_dirty = false;
    bool dropped = false;
    // per-frame adaptation scratch (grows with the frame size)
    int64_t cap_P = 0;
    int32_t *leaves = nullptr;     // [T][P]
    uint64_t *packed = nullptr;    // [P] the frame packed for probing
    uint16_t *rank = nullptr;      // [T][P]
    int32_t *slot = nullptr;       // [T][P]
    uint32_t *kval = nullptr;      // [T][P]
    uint16_t *chunk_cnt = nullptr; // [T][C][L]
    uint32_t *chunk_pref = nullptr;// [T][C][L]
    // the plain relocalisation path: a batch of one attempt
    reloc_batch *plain = nullptr;
    uint64_t bytes = 0;
};

// ---------------------------------------------------------------------------
// one relocalisation attempt as the device sees it (ragged batches)
// ---------------------------------------------------------------------------

struct Attempt {
    Frame fr;
    // the target forest (read-only here)
    const uint64_t RL_GLOBAL *nodes;
    const DeepNode RL_GLOBAL *deep;
    const int32_t RL_GLOBAL *nmodes;
    const Mode RL_GLOBAL *modes;
    const uint32_t RL_GLOBAL *mode_rgb;
    const unsigned long long RL_GLOBAL *total_samples;
    const uint32_t RL_GLOBAL *weights;      // [P] integer pick weights or null
    const float4 RL_GLOBAL *leaf_in;        // [T][L][4] per-leaf summaries (learned inputs)
    const uint16_t RL_GLOBAL *mq;           // learned proposal: bfloat16 weight copies, or null
    const float RL_GLOBAL *mw;              // learned proposal: FP32 parameters
    int32_t T, L, M, R, P, N, B, max_tries, rgb_tol, refine, rounds;
    float ratio2, min_pair2, min_area2, inl2;
    double resid2;
    uint64_t seed;
    // scratch owned by the batch
    int32_t RL_GLOBAL *leaves;              // [T][P] leaf of each pixel in each tree (-1: invalid pixel)
    uint64_t RL_GLOBAL *packed;             // [P] the frame packed for probing
    int32_t RL_GLOBAL *pool;                // [P]
    int32_t RL_GLOBAL *blockcnt;            // [nb]
    unsigned long long RL_GLOBAL *blockw;   // [nb] weight sums per pixel block
    unsigned long long RL_GLOBAL *cdf;      // [P] inclusive weight prefix over the pool
    int32_t RL_GLOBAL *guide;               // [P] weighted picks: first pool entry of each draw bucket
    unsigned long long RL_GLOBAL *gsel;     // [0] total weight [1] bucket multiplier [2] buckets in use
    uint32_t RL_GLOBAL *wbuf;               // [P] learned pick weights (learned proposal only)
    int32_t RL_GLOBAL *misc;                // [0] pool size [2] valid hypotheses
    int32_t RL_GLOBAL *rl;                  // [MAX_ROUNDS + 1] live hypotheses at the start of round r (r = 0: the
                                            // valid ones; 0 once the attempt has finished): round r runs iff
                                            // rl[r] >= 1 (r = 0) or rl[r] > 1; the cull of round r writes rl[r + 1]
    Hyp RL_GLOBAL *hyp;                     // [N]
    double RL_GLOBAL *hyp_init;             // [N][12]
    int32_t RL_GLOBAL *hyp_try;             // [N]
    float RL_GLOBAL *energy;                // [2][N] accumulated energy of the hypothesis at each live position
    double RL_GLOBAL *sums;                 // [N][NSUM] running inlier sums
    int32_t RL_GLOBAL *alive;               // [2][N] the live list scored in round r is buffer r & 1; the cull of round r
                                            // writes buffer (r + 1) & 1, so that it never overwrites what it reads
    int32_t RL_GLOBAL *pos;                 // [N] survivor i's position in the list it was scored in
    float RL_GLOBAL *lpose;                 // [N][12] FP32 pose (R row-major, t) of the hypothesis at each live position
    float4 RL_GLOBAL *draws;                // [rounds][B] camera point, pixel index bits of every draw
    int2 RL_GLOBAL *dtree;                  // [rounds][B][T] per draw and tree: first global mode index (leaf * M), mode count
    float RL_GLOBAL *gs;                    // [ceil(B / GROUP)][N] energy sum of each group of GROUP draws, per live position
    int32_t RL_GLOBAL *inl;                 // [ceil(B/8)][N][8] global index (leaf * M + mode) of an inlier's best mode, -1 otherwise
    unsigned long long RL_GLOBAL *stats;    // [0] mode evaluations [1] pair evaluations [2] round mode count
    int32_t RL_GLOBAL *tr_alive;            // [MAX_ROUNDS][N]
    float RL_GLOBAL *tr_energy;             // [MAX_ROUNDS][N]
    int32_t RL_GLOBAL *tr_n_alive;          // [MAX_ROUNDS]
    Result RL_GLOBAL *result;
};

// The inlier ids are stored in tiles of 8 consecutive draws per live
// position: a survivor's ids for 8 draws share one 32-byte sector (the
// refinement reads them per survivor), and the 8 draws of one scoring group,
// written together by the workgroup's wavefronts, fill whole tiles.
constexpr int INL_TILE = 8;

__device__ __forceinline__ int64_t inl_at(const Attempt &A, int i, int ap)
{
    return ((int64_t)(i / INL_TILE) * A.N + ap) * INL_TILE + (i % INL_TILE);
}

// work-unit layout of one stage over a batch: the units of attempt a are
// [off[a], off[a+1]); off has n + 1 entries
struct Stage {
    const int32_t *off;
    int32_t n;
    int32_t total;
    int32_t xcd;     // 1: units of each XCD's workgroups are contiguous
};

// Units walked by workgroup `b` of a grid of `g` in a persistent loop
//   for (u = start; u < end; u += step)
// Workgroups are dispatched round robin over the 8 XCDs; with xcd set and a
// grid that is a whole multiple of 8, XCD x walks the x-th contiguous eighth
// of the units, so that the units of one attempt share an L2. Any other grid
// walks the units round robin. Either way every unit has exactly one owner and
// step >= 1.
__host__ __device__ __forceinline__ void unit_range_of(int xcd, int total, unsigned b, unsigned g, int &start,
                                                       int &end, int &step)
{
    if (xcd && g >= 8u && (g % 8u) == 0u) {
        const int x = (int)(b % 8u), chunk = (total + 7) / 8;
        start = x * chunk + (int)(b / 8u);
        end = x * chunk + chunk < total ? x * chunk + chunk : total;
        step = (int)(g / 8u);
    } else {
        start = (int)b;
        end = total;
        step = (int)g;
    }
}

__device__ __forceinline__ void unit_range(const Stage &S, int &start, int &end, int &step)
{
    unit_range_of(S.xcd, S.total, blockIdx.x, gridDim.x, start, end, step);
}

__device__ __forceinline__ int attempt_of(const Stage &S, int u)
{
    int lo = 0, hi = S.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (S.off[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace rl

struct reloc_forest : public rl::Forest {};

// the learned proposal's device parameters (mlp.hip)
const uint16_t *rl_mlp_q(const reloc_mlp *m);
const float *rl_mlp_w(const reloc_mlp *m);

// releases a forest's plain-path batch (relocalise.hip)
void rl_free_plain(rl::Forest *f);
