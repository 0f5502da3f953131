"""The library's inter-agent host code (reloc_relative_transform,
reloc_collab_*) against the oracle (no GPU): the same scheduling decisions
and scores over many rounds, the same clusters and blended transforms, the
same pose graph and optimised global poses."""
import math

import numpy as np
import pytest

from oracle import collab as oc
from oracle_util import rand_rotation


def rigid(rng, scale=2.0):
    T = np.eye(4)
    T[:3, :3] = rand_rotation(rng)
    T[:3, 3] = rng.normal(size=3) * scale
    return T


def jitter(rng, T, m, deg):
    E = np.eye(4)
    axis = rng.normal(size=3)
    E[:3, :3] = oc.Rotation.from_rotvec(axis / np.linalg.norm(axis) * math.radians(deg) * rng.normal()).as_matrix()
    E[:3, 3] = rng.normal(size=3) * m
    return T @ E


def test_relative_transform_matches_oracle():
    import paper_1801_08361_amd as rl
    rng = np.random.default_rng(0)
    for _ in range(20):
        Pa, Pb = rigid(rng), rigid(rng)
        np.testing.assert_allclose(rl.relative_transform(Pa, Pb), oc.relative_transform(Pa, Pb), atol=1e-13)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_session_matches_oracle(seed):
    """A simulated session: scheduling rounds whose chosen attempts are marked
    tried, and samples (mostly near the true aT_b, some wrong) added for the
    chosen pairs; every few rounds the pose graph is optimised. Decisions,
    scores, clusters, blends and global poses equal the oracle's."""
    import paper_1801_08361_amd as rl
    rng = np.random.default_rng(seed)
    n = 5
    W = [rigid(rng) for _ in range(n)]
    g = rl.Collab(n, seed=99 + seed)
    o = oc.Session(n, 99 + seed)
    for k in range(n):
        frames = np.stack([rigid(rng, 1.0) for _ in range(int(rng.integers(3, 9)))])
        frames[1] = jitter(rng, frames[0], 0.02, 2.0)          # some frames close to others
        g.set_frames(k, frames)
        o.set_frames(k, frames)
    for rnd in range(40):
        a, b, i, cands = g.schedule(10)
        (ao, bo, io), co = o.schedule(10)
        assert (a, b, i) == (ao, bo, io), rnd
        np.testing.assert_allclose(cands, np.array([c for c in co], dtype=np.float32), atol=0)
        g.tried(a, b, i)
        o.mark_tried(a, b, i)
        if rng.random() < 0.8:
            T = jitter(rng, np.linalg.inv(W[a]) @ W[b], 0.01, 1.0)
        else:
            T = rigid(rng)                                           # a wrong relocalisation
        assert g.add_sample(a, b, T) == o.add_sample(a, b, T)
        if rnd % 8 == 7:
            ing, X, cost = g.optimise()
            ing_o, X_o, cost_o = o.optimise()
            assert np.array_equal(ing, ing_o), rnd
            np.testing.assert_allclose(X, X_o, atol=1e-7)
            assert cost == pytest.approx(cost_o, rel=1e-6, abs=1e-14)
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            sizes, blended = g.clusters(a, b)
            cl = o.clusters.get((min(a, b), max(a, b)), [])
            assert list(sizes) == [len(c) for c in cl]
            for k, c in enumerate(cl):
                want = oc.dq_blend(c) if a < b else np.linalg.inv(oc.dq_blend(c))
                np.testing.assert_allclose(blended[k], want, atol=1e-12)
    assert g.optimise()[0].sum() >= 2


def test_collab_argument_errors():
    import ctypes as C
    import paper_1801_08361_amd as rl
    L = rl.lib()
    out = C.c_void_p()
    assert L.reloc_collab_create(1, 0, C.byref(out)) == rl.E_ARG
    c = rl.Collab(3)
    with pytest.raises(rl.RelocError):           # no frames yet
        c.schedule(10)
    with pytest.raises(rl.RelocError):
        c.add_sample(1, 1, np.eye(4))
    with pytest.raises(rl.RelocError):
        c.tried(0, 1, 0)                          # scene 1 has no frame 0
    assert L.reloc_relative_transform(None, None, None) == rl.E_ARG
