"""Pins of the oracle's checkpoint (the relocaliser keeps training online and
can drop its training data once trained, Sec. 4.3.2): adapting on frames 0-4,
saving, loading and adapting on frames 5-9 gives exactly the forest adapted on
frames 0-9; a checkpoint taken after the reservoirs were dropped relocalises
as before and refuses further adaptation."""
import numpy as np
import pytest

import synthroom as sr


def _adapt(f, sc, frames):
    for k in frames:
        d, c = sc.render_adapt(k)
        f.adapt(d, c, sc.K, sc.adapt_poses[k])


def test_resume_equals_uninterrupted(orc, tmp_path):
    sc = sr.small_scene(31)
    p = orc.default_params(depth=8, reservoir_size=16)      # small reservoirs: replacement draws happen
    a = orc.Forest(p)
    _adapt(a, sc, range(10))
    b = orc.Forest(p)
    _adapt(b, sc, range(5))
    # some leaves' modes built before the save, the rest lazily after
    b.leaf_modes(0, 0)
    path = str(tmp_path / "forest.bin")
    b.save(path)
    c = orc.Forest.load(path, p)
    _adapt(c, sc, range(5, 10))
    assert c.total_samples == a.total_samples
    replaced = 0
    for t in range(a.T):
        for leaf in range(a.L):
            ea, ka = a.reservoir(t, leaf)
            ec, kc = c.reservoir(t, leaf)
            assert ka == kc, (t, leaf)
            assert np.array_equal(ea, ec), (t, leaf)
            replaced += int(ka > a.R)
    assert replaced > 100
    for t, leaf in ((0, 3), (1, 100), (4, 255)):
        assert np.array_equal(a.leaf_modes(t, leaf), c.leaf_modes(t, leaf))
    d, col = sc.render_query(2)
    ra = a.relocalise(d, col, sc.K, seed=9)
    rc_ = c.relocalise(d, col, sc.K, seed=9)
    assert ra[0] == rc_[0] and np.array_equal(ra[1], rc_[1]) and ra[2] == rc_[2]


def test_checkpoint_after_drop(orc, tmp_path):
    sc = sr.small_scene(32)
    p = orc.default_params(depth=8)
    a = orc.Forest(p)
    _adapt(a, sc, range(6))
    d, col = sc.render_query(1)
    before = a.relocalise(d, col, sc.K, seed=4)
    a.drop_reservoirs()
    path = str(tmp_path / "dropped.bin")
    a.save(path)
    c = orc.Forest.load(path, p)
    after = c.relocalise(d, col, sc.K, seed=4)
    assert before[0] == after[0] and np.array_equal(before[1], after[1]) and before[2] == after[2]
    d0, c0 = sc.render_adapt(7)
    with pytest.raises(ValueError):
        c.adapt(d0, c0, sc.K, sc.adapt_poses[7])


def test_checkpoint_rejects_other_files(orc, tmp_path):
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"ORACLEF1" + b"\0" * 10)
    with pytest.raises(ValueError):
        orc.Forest.load(str(bad), orc.default_params())
    with pytest.raises(ValueError):
        orc.Forest.load(str(tmp_path / "none.bin"), orc.default_params())
