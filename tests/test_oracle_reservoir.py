"""Pins of the online leaf reservoirs: the first R samples are kept verbatim,
Algorithm R keeps each of n samples with probability R/n and every R-subset
equally often, and the one-pixel-at-a-time oracle equals an independent
rank-and-scatter formulation with numpy's own Philox."""
import numpy as np
import pytest
from scipy import stats

import synthroom as sr
from tests.oracle_util import reservoir_by_ranks, world_mm_f32, cam_points_f32

I32_MAX = (1 << 31) - 1


def line_frame(n, base=1000):
    depth = (base + 7 * np.arange(n)).astype(np.uint16)[None, :]
    rgb = np.zeros((1, n, 3), dtype=np.uint8)
    rgb[0, :, 0] = np.arange(n)
    return depth, rgb


def single_leaf_forest(orc, R, seed):
    p = orc.default_params(n_trees=1, depth=1, reservoir_size=R, seed=seed)
    f = orc.Forest(p)
    kind, dx, dy, thr = f.nodes()
    thr[0] = I32_MAX                 # every pixel goes left: leaf 0
    f.set_nodes(kind, dx, dy, thr)
    return f


def test_first_R_samples_kept_verbatim(orc):
    R = 16
    f = single_leaf_forest(orc, R, 11)
    depth, rgb = line_frame(10)
    K = (277.0, 277.0, 5.0, 0.0)
    pose = np.eye(4)
    f.adapt(depth, rgb, K, pose)
    e, cnt = f.reservoir(0, 0)
    assert cnt == 10
    q = world_mm_f32(cam_points_f32(depth, K), pose)
    assert np.array_equal(np.stack([e["x"], e["y"], e["z"]], 1)[:10], q)
    assert np.array_equal(e["r"][:10], np.arange(10))
    assert np.all(e["x"][10:] == 0)


def test_algorithm_r_distribution(orc):
    n, R, seeds = 5, 2, 3000
    depth, rgb = line_frame(n)
    K = (277.0, 277.0, 2.0, 0.0)
    subsets = {}
    kept = np.zeros(n)
    for s in range(seeds):
        f = single_leaf_forest(orc, R, 1000 + s)
        f.adapt(depth, rgb, K, np.eye(4))
        e, cnt = f.reservoir(0, 0)
        assert cnt == n
        ids = tuple(sorted(int(x) for x in e["r"][:R]))
        assert len(set(ids)) == R
        subsets[ids] = subsets.get(ids, 0) + 1
        for i in ids:
            kept[i] += 1
    assert len(subsets) == 10
    assert stats.chisquare(list(subsets.values())).pvalue > 1e-3
    for i in range(n):
        assert stats.binomtest(int(kept[i]), seeds, R / n).pvalue > 1e-3


def test_rank_and_scatter_equivalence(orc):
    """Several frames of a rendered room into a small forest: the oracle's
    reservoirs and counters equal the per-frame stable-rank formulation."""
    sc = sr.small_scene(3, 64, 48)
    p = orc.default_params(n_trees=2, depth=4, reservoir_size=8, seed=77)
    f = orc.Forest(p)
    frames = []
    for k in range(4):
        d, c = sc.render_adapt(k)
        d, c = d.numpy(), c.numpy()
        frames.append((d, c, sc.adapt_poses[k]))
        f.adapt(d, c, sc.K, sc.adapt_poses[k])
    ent, cnt = reservoir_by_ranks(frames, lambda d, c: f.leaves(d, c, sc.K), sc.K, 77, 2, 16, 8)
    for t in range(2):
        for leaf in range(16):
            e, c = f.reservoir(t, leaf)
            assert c == cnt[t, leaf]
            got = np.stack([e["x"], e["y"], e["z"], e["r"], e["g"], e["b"]], 1)
            assert np.array_equal(got, ent[t, leaf]), (t, leaf)
    # the test must have exercised the replacement branch
    assert cnt.max() > 8 * 4


def test_adapt_rejects_non_rigid_pose(orc):
    f = orc.Forest(orc.default_params(n_trees=1, depth=2))
    depth, rgb = line_frame(4)
    bad = np.eye(4)
    bad[0, 0] = 1.01
    with pytest.raises(ValueError):
        f.adapt(depth, rgb, (277.0, 277.0, 2.0, 0.0), bad)
    refl = np.diag([1.0, 1.0, -1.0, 1.0])
    with pytest.raises(ValueError):
        f.adapt(depth, rgb, (277.0, 277.0, 2.0, 0.0), refl)
    with pytest.raises(ValueError):
        f.adapt(depth, rgb, (0.0, 277.0, 2.0, 0.0), np.eye(4))
