// Inter-agent scheduling and pose optimisation around the relocaliser
// (Sec. 3.3.1 and Sec. 3.3.2). Host code only: the problems are tiny (one
// node per agent, at most one edge per pair of agents).
//
//  - relative transform sample of a verified relocalisation: with P_a the
//    relocalised camera-to-world pose of a frame in sub-scene a and P_b its
//    own pose in sub-scene b, aT_b = P_a P_b^-1 maps b's coordinates to a's
//    (the paper's (fT_a)^-1 fT_b with world-to-camera poses fT_s = P_s^-1);
//  - candidate scheduling: candidates (a, (b, i)) drawn from a counter-based
//    generator, scored by Phi = phi_new - phi_conf - phi_homog (Eqs. 1-2),
//    the best (first on ties) chosen;
//  - incremental clustering of the samples of each pair: a sample joins the
//    first cluster holding a sample within 20 deg and 10 cm of it, else it
//    starts a new cluster (Sec. 4.2.4);
//  - pose graph: G' has an edge for every pair whose largest cluster holds
//    at least N = 2 samples, weighted by the dual-quaternion blend of that
//    cluster (Kavan et al. 2006); G is the connected component of G' that
//    holds the first agent's sub-scene; Levenberg-Marquardt minimises the sum
//    over G's edges of |v(gT_b^-1 gT_a aT_b)|^2, v = (imaginary part of the
//    rotation's unit quaternion, translation) (Eq. 5), with the first agent's
//    global pose fixed at the identity.
//
// Samples of a pair are kept in one orientation: for the pair {a, b} with
// a < b, as aT_b (a sample bT_a is stored as its inverse).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "reloc.h"

namespace {

constexpr int CONFIDENT = 2;               // N: samples that make a relative transform confident
constexpr double CLUSTER_DEG = 20.0, CLUSTER_M = 0.10;
constexpr double HOMOG_DEG = 5.0, HOMOG_M = 0.05;
constexpr float HOMOG_PENALTY = 5.0f;
constexpr uint64_t TAG_SCHEDULE = 7;
constexpr double PI = 3.14159265358979323846;

// ---- rigid transforms: R row-major, t ----------------------------------------

struct Rt {
    double R[9];
    double t[3];
};

Rt identity()
{
    Rt x;
    for (int k = 0; k < 9; ++k) x.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
    x.t[0] = x.t[1] = x.t[2] = 0.0;
    return x;
}

Rt from_mat(const double T[16])
{
    Rt x;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) x.R[r * 3 + c] = T[r * 4 + c];
        x.t[r] = T[r * 4 + 3];
    }
    return x;
}

void to_mat(const Rt &x, double T[16])
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) T[r * 4 + c] = x.R[r * 3 + c];
        T[r * 4 + 3] = x.t[r];
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
}

Rt compose(const Rt &a, const Rt &b)
{
    Rt x;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            x.R[r * 3 + c] = a.R[r * 3 + 0] * b.R[0 * 3 + c] + a.R[r * 3 + 1] * b.R[1 * 3 + c] + a.R[r * 3 + 2] * b.R[2 * 3 + c];
        x.t[r] = a.R[r * 3 + 0] * b.t[0] + a.R[r * 3 + 1] * b.t[1] + a.R[r * 3 + 2] * b.t[2] + a.t[r];
    }
    return x;
}

Rt inverse(const Rt &a)
{
    Rt x;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) x.R[r * 3 + c] = a.R[c * 3 + r];
    for (int r = 0; r < 3; ++r) x.t[r] = -(x.R[r * 3 + 0] * a.t[0] + x.R[r * 3 + 1] * a.t[1] + x.R[r * 3 + 2] * a.t[2]);
    return x;
}

// angle of Ra^T Rb in degrees: atan2(|axis vector| / 2, (trace - 1) / 2)
double angle_deg(const double Ra[9], const double Rb[9])
{
    double Q[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Q[r * 3 + c] = Ra[0 * 3 + r] * Rb[0 * 3 + c] + Ra[1 * 3 + r] * Rb[1 * 3 + c] + Ra[2 * 3 + r] * Rb[2 * 3 + c];
    const double vx = Q[7] - Q[5], vy = Q[2] - Q[6], vz = Q[3] - Q[1];
    return atan2(0.5 * sqrt(vx * vx + vy * vy + vz * vz), 0.5 * (Q[0] + Q[4] + Q[8] - 1.0)) * 180.0 / PI;
}

double dist(const double a[3], const double b[3])
{
    const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

bool close(const Rt &a, const Rt &b, double deg, double m)
{
    return angle_deg(a.R, b.R) <= deg && dist(a.t, b.t) <= m;
}

// unit quaternion (w, x, y, z) of a rotation, w >= 0 (Shepperd: from the
// largest of 1 + trace and the diagonal terms)
void quat_of(const double R[9], double q[4])
{
    const double tr = R[0] + R[4] + R[8];
    if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
        const double s = 2.0 * sqrt(1.0 + tr);
        q[0] = 0.25 * s;
        q[1] = (R[7] - R[5]) / s;
        q[2] = (R[2] - R[6]) / s;
        q[3] = (R[3] - R[1]) / s;
    } else if (R[0] >= R[4] && R[0] >= R[8]) {
        const double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]);
        q[0] = (R[7] - R[5]) / s;
        q[1] = 0.25 * s;
        q[2] = (R[1] + R[3]) / s;
        q[3] = (R[2] + R[6]) / s;
    } else if (R[4] >= R[8]) {
        const double s = 2.0 * sqrt(1.0 + R[4] - R[0] - R[8]);
        q[0] = (R[2] - R[6]) / s;
        q[1] = (R[1] + R[3]) / s;
        q[2] = 0.25 * s;
        q[3] = (R[5] + R[7]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]);
        q[0] = (R[3] - R[1]) / s;
        q[1] = (R[2] + R[6]) / s;
        q[2] = (R[5] + R[7]) / s;
        q[3] = 0.25 * s;
    }
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double sg = q[0] < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < 4; ++k) q[k] = sg * q[k] / n;
}

// rotation of a unit quaternion (w, x, y, z)
void rot_of(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

void qmul(const double a[4], const double b[4], double o[4])
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// Dual-quaternion linear blending with equal weights (Kavan et al. 2006):
// each sample as q_r + eps q_d, q_d = (0, t) q_r / 2, signs aligned with the
// first sample's rotation, summed, divided by the norm of the summed real
// part; the rotation from the real part, the translation 2 (q_d conj(q_r)).
Rt blend(const std::vector<Rt> &xs)
{
    double br[4] = {0, 0, 0, 0}, bd[4] = {0, 0, 0, 0}, q0[4];
    for (size_t i = 0; i < xs.size(); ++i) {
        double qr[4], qd[4];
        quat_of(xs[i].R, qr);
        if (i == 0) memcpy(q0, qr, sizeof(q0));
        const double tq[4] = {0.0, xs[i].t[0], xs[i].t[1], xs[i].t[2]};
        qmul(tq, qr, qd);
        const double sg = (qr[0] * q0[0] + qr[1] * q0[1] + qr[2] * q0[2] + qr[3] * q0[3]) < 0.0 ? -1.0 : 1.0;
        for (int k = 0; k < 4; ++k) {
            br[k] += sg * qr[k];
            bd[k] += sg * 0.5 * qd[k];
        }
    }
    const double n = sqrt(br[0] * br[0] + br[1] * br[1] + br[2] * br[2] + br[3] * br[3]);
    for (int k = 0; k < 4; ++k) {
        br[k] /= n;
        bd[k] /= n;
    }
    Rt x;
    rot_of(br, x.R);
    const double cr[4] = {br[0], -br[1], -br[2], -br[3]};
    double tq[4];
    qmul(bd, cr, tq);
    for (int k = 0; k < 3; ++k) x.t[k] = 2.0 * tq[k + 1];
    return x;
}

// v(T): the imaginary part of T's rotation quaternion (w >= 0) and T's
// translation
void vee(const Rt &x, double v[6])
{
    double q[4];
    quat_of(x.R, q);
    v[0] = q[1]; v[1] = q[2]; v[2] = q[3];
    v[3] = x.t[0]; v[4] = x.t[1]; v[5] = x.t[2];
}

// rotation by the rotation vector w (Rodrigues)
void exp_rot(const double w[3], double R[9])
{
    const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (th < 1e-300) {
        for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    const double half = 0.5 * th, s = sin(half) / th;
    const double q[4] = {cos(half), w[0] * s, w[1] * s, w[2] * s};
    rot_of(q, R);
}

// the node's pose moved by a 6-vector (rotation vector, translation):
// (Exp(w) R, t + d)
Rt perturb(const Rt &x, const double d[6])
{
    double E[9];
    exp_rot(d, E);
    Rt y;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            y.R[r * 3 + c] = E[r * 3 + 0] * x.R[0 * 3 + c] + E[r * 3 + 1] * x.R[1 * 3 + c] + E[r * 3 + 2] * x.R[2 * 3 + c];
        y.t[r] = x.t[r] + d[3 + r];
    }
    return y;
}

// solves the n x n system A x = b in place (Gaussian elimination, partial
// pivoting); false if singular
bool solve(std::vector<double> &A, std::vector<double> &b, int n)
{
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[(size_t)r * n + c]) > fabs(A[(size_t)p * n + c])) p = r;
        if (fabs(A[(size_t)p * n + c]) < 1e-300) return false;
        if (p != c) {
            for (int k = 0; k < n; ++k) std::swap(A[(size_t)p * n + k], A[(size_t)c * n + k]);
            std::swap(b[p], b[c]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[(size_t)r * n + c] / A[(size_t)c * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[(size_t)r * n + k] * b[k];
        b[r] = s / A[(size_t)r * n + r];
    }
    return true;
}

// ---- Philox4x64-10 on the host (Salmon et al., SC 2011) ----------------------

void philox_host(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c[0];
        const unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c[2];
        const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0;
        const uint64_t n2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint64_t)p1;
        c[2] = n2;
        c[3] = (uint64_t)p0;
    }
}

uint64_t uniform_host(uint64_t u, uint64_t n) { return (uint64_t)(((unsigned __int128)u * n) >> 64); }

struct PairState {
    std::vector<std::vector<Rt>> clusters;   // samples as lo_T_hi
};

}  // namespace

struct reloc_collab {
    int n = 0;
    uint64_t seed = 0;
    uint64_t attempts = 0;                        // scheduling rounds so far
    std::vector<std::vector<Rt>> frames;          // per scene: local camera-to-world poses
    std::vector<std::vector<int32_t>> tried;      // per ordered pair a * n + b: frames of b tried against a
    std::vector<PairState> pairs;                 // per unordered pair lo * n + hi
    std::vector<int32_t> in_graph;                // last optimisation: scene in G
    std::vector<Rt> global;                       // last optimisation: gT_s
};

namespace {

int largest(const PairState &ps)
{
    int best = -1;
    size_t bs = 0;
    for (size_t c = 0; c < ps.clusters.size(); ++c)
        if (ps.clusters[c].size() > bs) {
            bs = ps.clusters[c].size();
            best = (int)c;
        }
    return best;
}

float score_candidate(const reloc_collab *c, int a, int b, int i, float parts[3])
{
    const float phi_new = (c->in_graph[a] != 0) != (c->in_graph[b] != 0) ? 1.0f : 0.0f;
    const PairState &ps = c->pairs[(size_t)std::min(a, b) * c->n + std::max(a, b)];
    long conf = 0;
    for (const auto &cl : ps.clusters) conf = std::max(conf, (long)cl.size() - CONFIDENT);
    const float phi_conf = (float)conf;
    float phi_homog = 0.0f;
    const Rt &P = c->frames[b][i];
    for (int32_t j : c->tried[(size_t)a * c->n + b])
        if (close(P, c->frames[b][j], HOMOG_DEG, HOMOG_M)) {
            phi_homog = HOMOG_PENALTY;
            break;
        }
    if (parts) {
        parts[0] = phi_new;
        parts[1] = phi_conf;
        parts[2] = phi_homog;
    }
    return phi_new - phi_conf - phi_homog;
}

bool scene_ok(const reloc_collab *c, int s) { return s >= 0 && s < c->n; }

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" int reloc_relative_transform(const double pose_in_a[16], const double pose_in_b[16], double a_T_b[16])
{
    if (!pose_in_a || !pose_in_b || !a_T_b) return RELOC_E_ARG;
    to_mat(compose(from_mat(pose_in_a), inverse(from_mat(pose_in_b))), a_T_b);
    return RELOC_OK;
}

extern "C" int reloc_collab_create(int32_t n_scenes, uint64_t seed, reloc_collab **out)
{
    if (!out || n_scenes < 2 || n_scenes > 4096) return RELOC_E_ARG;
    reloc_collab *c = new (std::nothrow) reloc_collab();
    if (!c) return RELOC_E_NOMEM;
    c->n = n_scenes;
    c->seed = seed;
    c->frames.resize(n_scenes);
    c->tried.resize((size_t)n_scenes * n_scenes);
    c->pairs.resize((size_t)n_scenes * n_scenes);
    c->in_graph.assign(n_scenes, 0);
    c->global.assign(n_scenes, identity());
    *out = c;
    return RELOC_OK;
}

extern "C" int reloc_collab_destroy(reloc_collab *c)
{
    if (!c) return RELOC_E_ARG;
    delete c;
    return RELOC_OK;
}

extern "C" int reloc_collab_set_frames(reloc_collab *c, int32_t scene, const double *poses, int32_t n)
{
    if (!c || !scene_ok(c, scene) || n < 1 || !poses) return RELOC_E_ARG;
    std::vector<Rt> v((size_t)n);
    for (int32_t i = 0; i < n; ++i) v[i] = from_mat(poses + (size_t)i * 16);
    c->frames[scene] = v;
    return RELOC_OK;
}

extern "C" int reloc_collab_schedule(reloc_collab *c, int32_t n_cand, int32_t *a_out, int32_t *b_out,
                                     int32_t *frame_out, float *cands_out)
{
    if (!c || n_cand < 1 || !a_out || !b_out || !frame_out) return RELOC_E_ARG;
    for (int s = 0; s < c->n; ++s)
        if (c->frames[s].empty()) return RELOC_E_STATE;
    const uint64_t n_pairs = (uint64_t)c->n * (uint64_t)(c->n - 1);
    float best = 0.0f;
    int ba = -1, bb = -1, bi = -1;
    for (int j = 0; j < n_cand; ++j) {
        uint64_t u[4] = {c->attempts, (uint64_t)j, 0, 0};
        philox_host(u, c->seed, TAG_SCHEDULE);
        const uint64_t pr = uniform_host(u[0], n_pairs);
        const int a = (int)(pr / (uint64_t)(c->n - 1));
        const int r = (int)(pr % (uint64_t)(c->n - 1));
        const int b = r < a ? r : r + 1;
        const int i = (int)uniform_host(u[1], (uint64_t)c->frames[b].size());
        float parts[3];
        const float phi = score_candidate(c, a, b, i, parts);
        if (cands_out) {
            float *o = cands_out + (size_t)j * 7;
            o[0] = (float)a; o[1] = (float)b; o[2] = (float)i; o[3] = phi;
            o[4] = parts[0]; o[5] = parts[1]; o[6] = parts[2];
        }
        if (ba < 0 || phi > best) {
            best = phi;
            ba = a;
            bb = b;
            bi = i;
        }
    }
    c->attempts++;
    *a_out = ba;
    *b_out = bb;
    *frame_out = bi;
    return RELOC_OK;
}

extern "C" int reloc_collab_tried(reloc_collab *c, int32_t a, int32_t b, int32_t frame)
{
    if (!c || !scene_ok(c, a) || !scene_ok(c, b) || a == b || frame < 0 || frame >= (int32_t)c->frames[b].size())
        return RELOC_E_ARG;
    c->tried[(size_t)a * c->n + b].push_back(frame);
    return RELOC_OK;
}

extern "C" int reloc_collab_add_sample(reloc_collab *c, int32_t a, int32_t b, const double a_T_b[16],
                                       int32_t *cluster_size)
{
    if (!c || !scene_ok(c, a) || !scene_ok(c, b) || a == b || !a_T_b) return RELOC_E_ARG;
    Rt x = from_mat(a_T_b);
    if (a > b) x = inverse(x);
    PairState &ps = c->pairs[(size_t)std::min(a, b) * c->n + std::max(a, b)];
    int joined = -1;
    for (size_t k = 0; k < ps.clusters.size() && joined < 0; ++k)
        for (const Rt &y : ps.clusters[k])
            if (close(x, y, CLUSTER_DEG, CLUSTER_M)) {
                joined = (int)k;
                break;
            }
    if (joined < 0) {
        ps.clusters.emplace_back();
        joined = (int)ps.clusters.size() - 1;
    }
    ps.clusters[joined].push_back(x);
    if (cluster_size) *cluster_size = (int32_t)ps.clusters[joined].size();
    return RELOC_OK;
}

extern "C" int reloc_collab_clusters(const reloc_collab *c, int32_t a, int32_t b, int32_t *sizes, double *blended,
                                     int32_t cap, int32_t *n_out)
{
    if (!c || !scene_ok(c, a) || !scene_ok(c, b) || a == b || !n_out || cap < 0) return RELOC_E_ARG;
    const PairState &ps = c->pairs[(size_t)std::min(a, b) * c->n + std::max(a, b)];
    *n_out = (int32_t)ps.clusters.size();
    for (int k = 0; k < (int)ps.clusters.size() && k < cap; ++k) {
        if (sizes) sizes[k] = (int32_t)ps.clusters[k].size();
        if (blended) {
            Rt x = blend(ps.clusters[k]);
            if (a > b) x = inverse(x);
            to_mat(x, blended + (size_t)k * 16);
        }
    }
    return RELOC_OK;
}

extern "C" int reloc_collab_optimise(reloc_collab *c, int32_t *in_graph, double *global_poses, double *cost_out)
{
    if (!c) return RELOC_E_ARG;
    const int n = c->n;
    // G': confident pairs and their blended transforms
    struct Edge {
        int a, b;
        Rt T;   // aT_b, a < b
    };
    std::vector<Edge> edges;
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) {
            const PairState &ps = c->pairs[(size_t)a * n + b];
            const int k = largest(ps);
            if (k >= 0 && (int)ps.clusters[k].size() >= CONFIDENT) edges.push_back({a, b, blend(ps.clusters[k])});
        }
    // G: the connected component of scene 0, found breadth first; the first
    // visit of each node sets its initial pose from its parent (gT_b = gT_a aT_b)
    std::vector<int32_t> in(n, 0);
    std::vector<Rt> X(n, identity());
    std::vector<int> queue{0};
    in[0] = 1;
    for (size_t h = 0; h < queue.size(); ++h) {
        const int s = queue[h];
        for (const Edge &e : edges) {
            int o = -1;
            Rt Xo;
            if (e.a == s && !in[e.b]) {
                o = e.b;
                Xo = compose(X[s], e.T);
            } else if (e.b == s && !in[e.a]) {
                o = e.a;
                Xo = compose(X[s], inverse(e.T));
            }
            if (o >= 0) {
                in[o] = 1;
                X[o] = Xo;
                queue.push_back(o);
            }
        }
    }
    std::vector<const Edge *> ge;
    for (const Edge &e : edges)
        if (in[e.a]) ge.push_back(&e);
    // unknowns: 6 per node of G other than scene 0
    std::vector<int> var(n, -1);
    int nv = 0;
    for (int s = 1; s < n; ++s)
        if (in[s]) var[s] = nv++;
    auto residuals = [&](const std::vector<Rt> &Y, std::vector<double> &r) {
        r.assign(ge.size() * 6, 0.0);
        double cost = 0.0;
        for (size_t k = 0; k < ge.size(); ++k) {
            const Edge &e = *ge[k];
            vee(compose(inverse(Y[e.b]), compose(Y[e.a], e.T)), &r[k * 6]);
            for (int j = 0; j < 6; ++j) cost += r[k * 6 + j] * r[k * 6 + j];
        }
        return cost;
    };
    std::vector<double> r;
    double cost = residuals(X, r);
    if (nv > 0 && !ge.empty()) {
        const int m = (int)r.size(), p = 6 * nv;
        double lambda = 1e-4;
        for (int it = 0; it < 200; ++it) {
            // Jacobian by central differences of the 6-vector node moves
            std::vector<double> J((size_t)m * p, 0.0), rp, rm;
            const double h = 1e-7;
            for (int s = 1; s < n; ++s) {
                if (var[s] < 0) continue;
                for (int j = 0; j < 6; ++j) {
                    double d[6] = {0, 0, 0, 0, 0, 0};
                    std::vector<Rt> Y = X;
                    d[j] = h;
                    Y[s] = perturb(X[s], d);
                    residuals(Y, rp);
                    d[j] = -h;
                    Y[s] = perturb(X[s], d);
                    residuals(Y, rm);
                    for (int q = 0; q < m; ++q) J[(size_t)q * p + var[s] * 6 + j] = (rp[q] - rm[q]) / (2.0 * h);
                }
            }
            std::vector<double> JtJ((size_t)p * p, 0.0), g(p, 0.0);
            for (int q = 0; q < m; ++q)
                for (int x = 0; x < p; ++x) {
                    const double jx = J[(size_t)q * p + x];
                    if (jx == 0.0) continue;
                    g[x] += jx * r[q];
                    for (int y = 0; y < p; ++y) JtJ[(size_t)x * p + y] += jx * J[(size_t)q * p + y];
                }
            bool improved = false;
            for (int tries = 0; tries < 20 && !improved; ++tries) {
                std::vector<double> A = JtJ, step(p);
                for (int x = 0; x < p; ++x) {
                    A[(size_t)x * p + x] += lambda * (JtJ[(size_t)x * p + x] > 0.0 ? JtJ[(size_t)x * p + x] : 1.0);
                    step[x] = -g[x];
                }
                if (!solve(A, step, p)) {
                    lambda *= 10.0;
                    continue;
                }
                std::vector<Rt> Y = X;
                for (int s = 1; s < n; ++s)
                    if (var[s] >= 0) Y[s] = perturb(X[s], &step[(size_t)var[s] * 6]);
                std::vector<double> rn;
                const double cn = residuals(Y, rn);
                if (cn < cost) {
                    const double drop = cost - cn;
                    X = Y;
                    r = rn;
                    cost = cn;
                    lambda = std::max(lambda * 0.1, 1e-12);
                    improved = true;
                    double sn = 0.0;
                    for (double v : step) sn += v * v;
                    if (drop <= 1e-15 * (1.0 + cost) || sn < 1e-24) it = 1 << 20;
                } else {
                    lambda *= 10.0;
                }
            }
            if (!improved) break;
        }
    }
    c->in_graph = in;
    c->global = X;
    if (in_graph) memcpy(in_graph, in.data(), sizeof(int32_t) * n);
    if (global_poses)
        for (int s = 0; s < n; ++s) to_mat(X[s], global_poses + (size_t)s * 16);
    if (cost_out) *cost_out = cost;
    return RELOC_OK;
}
