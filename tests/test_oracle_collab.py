"""Pins of the oracle's inter-agent steps (Sec. 3.3.1, 3.3.2, 4.2.3, 4.2.4):
the relative transform against the composition of the sub-scene frames it
should recover; the verifier and clustering statistics against the numbers
Tables 3 and 4 print; dual-quaternion blending against closed forms (screw
motions about one axis, pure translations); the cluster rule, the candidate
scores and the Philox draws on constructed cases; the connected component
against scipy's; and the pose-graph optimum against exact recovery and, for
translation-only graphs, the linear least-squares solution (numpy)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from oracle import collab as oc
from oracle_util import np_philox, np_uniform_int, rand_rotation

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rigid(rng, scale=2.0):
    T = np.eye(4)
    T[:3, :3] = rand_rotation(rng)
    T[:3, 3] = rng.normal(size=3) * scale
    return T


def axis_rotation(axis, theta, through=np.zeros(3)):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    R = np.eye(3) + math.sin(theta) * K + (1 - math.cos(theta)) * K @ K
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = through - R @ through
    return T


def test_relative_transform_recovers_subscene_frames():
    """Frame f seen by agents a and b, whose sub-scenes sit at W_a and W_b in
    the world: aT_b = W_a^-1 W_b, and it maps a point's b-coordinates to its
    a-coordinates."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        Wa, Wb, C = rigid(rng), rigid(rng), rigid(rng)
        Pa = np.linalg.inv(Wa) @ C          # the frame's pose in a
        Pb = np.linalg.inv(Wb) @ C          # and in b
        aTb = oc.relative_transform(Pa, Pb)
        np.testing.assert_allclose(aTb, np.linalg.inv(Wa) @ Wb, atol=1e-12)
        x = np.append(rng.normal(size=3), 1.0)
        np.testing.assert_allclose(aTb @ (np.linalg.inv(Wb) @ x), np.linalg.inv(Wa) @ x, atol=1e-12)


def test_verifier_stats_reproduce_table3():
    g = json.load(open(os.path.join(GOLDEN, "table3_verifier.json")))
    stats = []
    for row in g["rows"]:
        p, r, s = oc.verifier_stats(row["TP"], row["FP"], row["TN"], row["FN"])
        assert round(100 * p, 1) == row["precision"]
        assert round(100 * r, 1) == row["recall"]
        assert round(100 * s, 1) == row["specificity"]
        stats.append((round(100 * p, 1), round(100 * r, 1), round(100 * s, 1)))
    # the printed averages are means of the printed (rounded) per-pair figures
    # (recall: 99.16 from the rounded figures, 99.15 from the exact ones)
    mean = np.mean(stats, axis=0)
    assert [round(v, 1) for v in mean] == [g["average"][k] for k in ("precision", "recall", "specificity")]


def test_cluster_stats_reproduce_table4():
    g = json.load(open(os.path.join(GOLDEN, "table4_clusters.json")))
    for row in g["rows"]:
        c, i, margin = oc.cluster_stats(row["samples"], row["correct"], row["incorrect"])
        assert round(100 * c, 1) == row["correct_pct"] and round(100 * i, 1) == row["incorrect_pct"]
        assert margin == row["margin"]


def test_dq_blend_closed_forms():
    rng = np.random.default_rng(1)
    T = rigid(rng)
    np.testing.assert_allclose(oc.dq_blend([T]), T, atol=1e-12)
    # screw motions about one axis through p: the blend turns about the same
    # axis through the same point, by the angle of the summed half-angle
    # vectors, 2 atan2(sum sin(th / 2), sum cos(th / 2)) (the mean angle for
    # two samples)
    axis, p = rng.normal(size=3), rng.normal(size=3)
    for th in ((0.1, 0.5), (-0.3, 0.9, 0.2), (2.0, 2.6), (0.4, 0.4, 1.3, -0.2)):
        got = oc.dq_blend([axis_rotation(axis, t, p) for t in th])
        want = 2.0 * math.atan2(sum(math.sin(t / 2) for t in th), sum(math.cos(t / 2) for t in th))
        if len(th) == 2:
            assert want == pytest.approx(float(np.mean(th)), abs=1e-15)
        np.testing.assert_allclose(got, axis_rotation(axis, want, p), atol=1e-12)
    # pure translations: the mean translation
    ts = rng.normal(size=(5, 3))
    Ts = []
    for t in ts:
        M = np.eye(4)
        M[:3, 3] = t
        Ts.append(M)
    np.testing.assert_allclose(oc.dq_blend(Ts)[:3, 3], ts.mean(0), atol=1e-12)
    np.testing.assert_allclose(oc.dq_blend(Ts)[:3, :3], np.eye(3), atol=1e-12)


def test_cluster_rule_first_cluster_any_member():
    """A sample joins the first cluster holding any sample within 20 deg and
    10 cm (not the cluster's centre), else starts a new one; both orientations
    of a pair share the clusters."""
    s = oc.Session(3, 0)
    I = np.eye(4)
    A = axis_rotation([0, 0, 1], math.radians(15))            # 15 deg from I: joins
    B = I.copy(); B[:3, 3] = [0.15, 0, 0]                      # 15 cm from I: new cluster
    C = axis_rotation([0, 0, 1], math.radians(30))            # 30 deg from I, 15 from A: joins via A
    D = B.copy(); D[:3, 3] = [0.08, 0, 0]                      # 8 cm from I and 7 cm from B: the first cluster
    assert [s.add_sample(0, 1, T) for T in (I, A, B, C, D)] == [1, 2, 1, 3, 4]
    assert [len(c) for c in s.clusters[(0, 1)]] == [4, 1]
    # a sample of the reverse orientation is inverted before the test: G is
    # 9 cm from B (second cluster) and 16 cm from D; its inverse is far from all
    G = I.copy(); G[:3, 3] = [0.24, 0, 0]
    assert s.add_sample(1, 0, np.linalg.inv(G)) == 2
    assert [len(c) for c in s.clusters[(0, 1)]] == [4, 2]
    # a sample near members of both clusters joins the first (D is 7 cm away)
    assert s.add_sample(0, 1, B) == 5
    assert [len(c) for c in s.clusters[(0, 1)]] == [5, 2]


def test_candidate_scores_constructed():
    s = oc.Session(3, 5)
    frames = [np.eye(4) for _ in range(4)]
    frames[1] = frames[0].copy(); frames[1][:3, 3] = [0.03, 0, 0]   # within 5 cm of frame 0
    frames[2] = frames[0].copy(); frames[2][:3, 3] = [0.30, 0, 0]
    frames[3] = axis_rotation([0, 1, 0], math.radians(4))           # within 5 deg of frame 0
    for k in range(3):
        s.set_frames(k, frames)
    assert s.score(0, 1, 0) == (0.0, 0.0, 0.0, 0.0)
    s.mark_tried(0, 1, 0)
    assert s.score(0, 1, 1)[3] == 5.0 and s.score(0, 1, 3)[3] == 5.0 and s.score(0, 1, 2)[3] == 0.0
    assert s.score(1, 0, 1)[3] == 0.0            # tried against a different scene
    for _ in range(5):
        s.add_sample(0, 1, np.eye(4))
    assert s.score(1, 0, 2) == (-3.0, 0.0, 3.0, 0.0)          # one cluster of 5: phi_conf = 5 - 2
    s.in_graph[0] = True
    assert s.score(0, 2, 2) == (1.0, 1.0, 0.0, 0.0)           # exactly one of the pair has a global pose
    assert s.score(0, 1, 2)[1] == 1.0
    s.in_graph[1] = True
    assert s.score(0, 1, 2)[1] == 0.0


def test_schedule_draws_follow_philox():
    rng = np.random.default_rng(3)
    s = oc.Session(5, 1234)
    n_frames = [7, 3, 11, 5, 2]
    for k in range(5):
        s.set_frames(k, [rigid(rng) for _ in range(n_frames[k])])
    for rnd in range(3):
        best, cands = s.schedule(10)
        for j, (a, b, i, phi, *_) in enumerate(cands):
            u = np_philox((rnd, j, 0, 0), (1234, 7))
            p = np_uniform_int(u[0], 20)
            assert (a, b) == (p // 4, p % 4 if p % 4 < p // 4 else p % 4 + 1)
            assert a != b and i == np_uniform_int(u[1], n_frames[b])
        assert best == cands[0][:3]         # nothing tried or clustered: every score is 0, the first wins


def test_connected_component_matches_scipy():
    rng = np.random.default_rng(4)
    for _ in range(30):
        n = int(rng.integers(2, 12))
        edges = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(int(rng.integers(0, 2 * n)), 2)) if a != b]
        M = np.zeros((n, n))
        for a, b in edges:
            M[a, b] = M[b, a] = 1
        _, lab = connected_components(csr_matrix(M), directed=False)
        assert oc.connected_component(n, edges) == [k for k in range(n) if lab[k] == lab[0]]


def _session_from_truth(W, pairs, rng, noise_t=0.0, noise_deg=0.0, reps=2):
    n = len(W)
    s = oc.Session(n, 0)
    for a, b in pairs:
        for _ in range(reps):
            T = np.linalg.inv(W[a]) @ W[b]
            if noise_t or noise_deg:
                E = axis_rotation(rng.normal(size=3), math.radians(noise_deg) * rng.normal())
                E[:3, 3] = rng.normal(size=3) * noise_t
                T = T @ E
            s.add_sample(a, b, T)
    return s


def test_pose_graph_exact_recovery():
    """Noise-free samples on a graph with a cycle: every scene reachable from
    scene 0 gets gT_s = W_0^-1 W_s and the cost is zero; a scene without a
    confident edge stays out of G."""
    rng = np.random.default_rng(5)
    W = [rigid(rng) for _ in range(6)]
    s = _session_from_truth(W, [(0, 1), (1, 2), (2, 0), (2, 3), (4, 3)], rng)
    s.add_sample(0, 5, np.eye(4))        # a single sample: not confident
    ing, X, cost = s.optimise()
    assert list(np.flatnonzero(ing)) == [0, 1, 2, 3, 4]
    for k in range(5):
        np.testing.assert_allclose(X[k], np.linalg.inv(W[0]) @ W[k], atol=1e-9)
    np.testing.assert_allclose(X[5], np.eye(4))
    assert cost < 1e-20


def test_pose_graph_optimum_is_the_minimum():
    """Noisy samples (1 cm, 1 deg) on a graph with cycles: the Levenberg-
    Marquardt result is the minimum that a different minimiser (scipy's BFGS
    on the scalar cost, with poses as quaternion and translation, started at
    the true poses) finds, and no worse than the chained start."""
    from scipy.optimize import minimize
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(6)
    W = [rigid(rng) for _ in range(5)]
    pairs = [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (1, 3), (0, 2)]
    s = _session_from_truth(W, pairs, rng, noise_t=0.01, noise_deg=1.0, reps=3)
    edges = s.edges()
    assert len(edges) == len(pairs)
    ing, X, cost = s.optimise()
    assert ing.all()

    def cost_of(p):
        Y = [np.eye(4)]
        for k in range(4):
            M = np.eye(4)
            q = p[7 * k:7 * k + 4]
            M[:3, :3] = Rotation.from_quat(q / np.linalg.norm(q)).as_matrix()
            M[:3, 3] = p[7 * k + 4:7 * k + 7]
            Y.append(M)
        return sum(float(np.sum(oc.vee(np.linalg.inv(Y[b]) @ Y[a] @ T) ** 2)) for a, b, T in edges)

    p0 = []
    for k in range(1, 5):
        T = np.linalg.inv(W[0]) @ W[k]
        p0 += list(Rotation.from_matrix(T[:3, :3]).as_quat()) + list(T[:3, 3])
    sol = minimize(cost_of, np.array(p0), method="BFGS", options={"gtol": 1e-12, "maxiter": 10000})
    assert cost == pytest.approx(sol.fun, rel=1e-6, abs=1e-14)
    for k in range(1, 5):
        q = sol.x[7 * (k - 1):7 * (k - 1) + 4]
        R = Rotation.from_quat(q / np.linalg.norm(q)).as_matrix()
        np.testing.assert_allclose(X[k][:3, :3], R, atol=1e-5)
        np.testing.assert_allclose(X[k][:3, 3], sol.x[7 * (k - 1) + 4:7 * (k - 1) + 7], atol=1e-5)
        # and close to the truth
        assert np.linalg.norm(X[k][:3, 3] - (np.linalg.inv(W[0]) @ W[k])[:3, 3]) < 0.05
