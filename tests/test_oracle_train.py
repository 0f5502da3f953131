"""Pins of the oracle's split training (oracle_train_forest).

The brute force below trains the same small forest a different way: it
routes pixels with the oracle's traversal (a one-node forest holding the
candidate split, so the feature arithmetic is the one pinned by the
traversal tests), keeps the samples of every node as explicit index sets,
and scores candidates with exact rational arithmetic. The objective is the
summed squared deviation of the samples' world points (integer mm) from
their child's mean, ties to the lower candidate."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synthroom as sr

TAG_TRAIN = 8


def _draw_split(p, t, i, k):
    """Candidate k of node i of tree t: the random-split recipe on the
    generator keyed by (seed, TRAIN)."""
    u = oracle.philox([t, i, k, 0], [p.seed, TAG_TRAIN])
    kk = oracle.uniform_int(int(u[0]), 6)
    kind = 0 if kk < 3 else kk - 2
    O = p.offset_pxmm
    dx = oracle.uniform_int(int(u[1]), 2 * O + 1) - O
    dy = oracle.uniform_int(int(u[2]), 2 * O + 1) - O
    Tk = p.thr_depth_mm if kind == 0 else p.thr_rgb
    thr = oracle.uniform_int(int(u[3]), 2 * Tk + 1) - Tk
    return kind, dx, dy, thr


def _router(p):
    q = oracle.Params()
    oracle.lib().oracle_params_default(oracle.C.byref(q))
    for f, _ in q._fields_:
        setattr(q, f, getattr(p, f))
    q.n_trees, q.depth = 1, 1
    return oracle.Forest(q)


def _sides(router, split, frames, K):
    """Per frame: 1 where a pixel goes right under `split` (oracle traversal)."""
    kind = np.array([split[0]] + [0] * 8, np.int32)
    dx = np.array([split[1]] + [0] * 8, np.int32)
    dy = np.array([split[2]] + [0] * 8, np.int32)
    thr = np.array([split[3]] + [0] * 8, np.int32)
    router.set_nodes(kind, dx, dy, thr)
    return [router.leaves(d, c, K)[0] for d, c, _ in frames]


def _samples(p, frames, K, stride):
    fx, fy, cx, cy = (np.float32(k) for k in K)
    out = []
    for fi, (d, _, T) in enumerate(frames):
        d = np.asarray(d)
        H, W = d.shape
        R32 = np.asarray(T, np.float64)[:3, :3].astype(np.float32)
        t32 = np.asarray(T, np.float64)[:3, 3].astype(np.float32)
        for v in range(stride // 2, H, stride):
            for u in range(stride // 2, W, stride):
                z0 = int(d[v, u])
                if not (p.depth_min_mm <= z0 <= p.depth_max_mm):
                    continue
                z = np.float32(z0) * np.float32(0.001)
                c = [(np.float32(u) - cx) * z / fx, (np.float32(v) - cy) * z / fy, z]
                w = [((R32[a, 0] * c[0] + R32[a, 1] * c[1]) + R32[a, 2] * c[2]) + t32[a] for a in range(3)]
                q = [int(np.rint(np.float32(x) * np.float32(1000.0))) for x in w]
                out.append((fi, v * W + u, q))
    return out


def _sse(points):
    n = len(points)
    if n == 0:
        return Fraction(0)
    s = [sum(q[a] for q in points) for a in range(3)]
    s2 = sum(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] for q in points)
    return Fraction(s2) - Fraction(s[0] * s[0] + s[1] * s[1] + s[2] * s[2], n)


def brute_train(p, frames, K, stride, n_cand):
    smp = _samples(p, frames, K, stride)
    router = _router(p)
    L = 1 << p.depth
    nodes = []
    for t in range(p.n_trees):
        members = {0: list(range(len(smp)))}
        tree = [None] * (L - 1)
        for i in range(L - 1):
            idx = members.get(i, [])
            best = None
            for k in range(n_cand):
                cand = _draw_split(p, t, i, k)
                sides = _sides(router, cand, frames, K)
                left = [smp[s][2] for s in idx if sides[smp[s][0]][smp[s][1]] == 0]
                right = [smp[s][2] for s in idx if sides[smp[s][0]][smp[s][1]] == 1]
                cost = _sse(left) + _sse(right)
                if best is None or cost < best[0]:
                    best = (cost, cand)
            tree[i] = best[1]
            if 2 * i + 1 < L - 1:
                sides = _sides(router, tree[i], frames, K)
                members[2 * i + 1] = [s for s in idx if sides[smp[s][0]][smp[s][1]] == 0]
                members[2 * i + 2] = [s for s in idx if sides[smp[s][0]][smp[s][1]] == 1]
        nodes.extend(tree)
    return nodes


@pytest.fixture(scope="module")
def small():
    sc = sr.small_scene(71, 64, 48)
    frames = []
    for k in (0, 5):
        d, c = sc.render_adapt(k)
        frames.append((d.numpy(), c.numpy(), sc.adapt_poses[k]))
    return sc, frames


@pytest.mark.parametrize("stride,n_cand", [(3, 6), (2, 3)])
def test_training_equals_brute_force(small, stride, n_cand):
    sc, frames = small
    p = oracle.Params()
    oracle.lib().oracle_params_default(oracle.C.byref(p))
    p.n_trees, p.depth = 2, 3
    f = oracle.Forest(p)
    f.train(frames, sc.K, stride, n_cand)
    kind, dx, dy, thr = f.nodes()
    got = list(zip(kind, dx, dy, thr))[: p.n_trees * ((1 << p.depth) - 1)]
    want = brute_train(p, frames, sc.K, stride, n_cand)
    assert [tuple(int(x) for x in g) for g in got] == [tuple(int(x) for x in w) for w in want]


def test_training_lowers_leaf_variance_and_empties_leaves(small):
    """Trained splits leave a smaller summed squared deviation of the
    training samples within their leaves than random splits of the same
    depth; training empties every leaf (adaptation then fills them)."""
    sc, frames = small
    p = oracle.Params()
    oracle.lib().oracle_params_default(oracle.C.byref(p))
    p.n_trees, p.depth = 1, 4
    rnd = oracle.Forest(p)
    trained = oracle.Forest(p)
    d0, c0, T0 = frames[0]
    trained.adapt(d0, c0, sc.K, T0)
    trained.train(frames, sc.K, 2, 16)
    assert trained.total_samples == 0
    smp = _samples(p, frames, sc.K, 2)

    def leaf_sse(forest):
        leaves = [forest.leaves(d, c, sc.K)[0] for d, c, _ in frames]
        groups = {}
        for fi, px, q in smp:
            groups.setdefault(int(leaves[fi][px]), []).append(q)
        return sum(_sse(g) for g in groups.values())

    assert leaf_sse(trained) < 0.8 * leaf_sse(rnd)
    # arguments
    with pytest.raises(ValueError):
        trained.train(frames, sc.K, 0, 16)
    with pytest.raises(ValueError):
        trained.train(frames, sc.K, 2, 65)
