"""GPU split training (reloc_forest_train) against the oracle: the trained
split nodes bit for bit (nodes of one evaluation unit and nodes whose samples
span several units, empty nodes, ragged sampling grids), then traversal,
adaptation and relocalisation with the trained structure as with any other."""
import numpy as np
import pytest

import synthroom as sr
from tests.gpu_util import banner, need_gpu, pair, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def _frames(sc, ks, dev, width=None, height=None):
    out_g, out_o = [], []
    for k in ks:
        d, c = sc.render_adapt(k, width=width, height=height)
        dg, cg = to_dev(d, c, dev)
        out_g.append((dg, cg, sc.K if width is None else sr.intrinsics(width, height), sc.adapt_poses[k]))
        out_o.append((d.numpy(), c.numpy(), sc.adapt_poses[k]))
    return out_g, out_o


@pytest.mark.parametrize("cfg", [
    dict(n_trees=3, depth=6, W=160, H=120, stride=4, n_cand=64, frames=(0, 4, 9)),
    dict(n_trees=2, depth=9, W=161, H=97, stride=3, n_cand=7, frames=(1, 6)),
    dict(n_trees=5, depth=10, W=320, H=240, stride=4, n_cand=32, frames=(0, 3, 7, 12)),
])
def test_trained_nodes_match_oracle(dev, cfg):
    import oracle
    import paper_1801_08361_amd as rl
    import torch
    sc = sr.small_scene(81, cfg["W"], cfg["H"])
    pp, po = pair(n_trees=cfg["n_trees"], depth=cfg["depth"], reservoir_size=64, max_modes=10)
    fg, fo = _frames(sc, cfg["frames"], dev)
    banner(f"train {cfg}")
    g = rl.Forest(pp)
    g.train(fg, cfg["stride"], cfg["n_cand"])
    torch.cuda.synchronize()
    o = oracle.Forest(po)
    o.train(fo, sc.K, cfg["stride"], cfg["n_cand"])
    for a, b in zip(g.nodes(), o.nodes()):
        assert np.array_equal(a, b)
    # the extra feature nodes are untouched, the structure differs from the random one
    r = rl.Forest(pp)
    kr = r.nodes()[0]
    kg = g.nodes()[0]
    n_split = cfg["n_trees"] * ((1 << cfg["depth"]) - 1)
    assert np.array_equal(kg[n_split:], kr[n_split:])
    assert g.memory() > 0


def test_trained_forest_adapts_and_relocalises_like_the_oracle(dev):
    """Leaves, reservoirs and a relocalisation with a trained structure (split
    structure from room A, leaves adapted in room B) equal the oracle's."""
    import oracle
    import paper_1801_08361_amd as rl
    import torch
    A = sr.small_scene(90, 160, 120)
    B = sr.small_scene(91, 160, 120)
    pp, po = pair(n_trees=3, depth=8, reservoir_size=64, max_modes=10, n_hypotheses=64, batch_pixels=32)
    fg, fo = _frames(A, (0, 5, 10), dev)
    banner("train room A, adapt room B")
    g = rl.Forest(pp)
    g.train(fg, 4, 16)
    o = oracle.Forest(po)
    o.train(fo, A.K, 4, 16)
    for k in range(6):
        d, c = B.render_adapt(k)
        dg, cg = to_dev(d, c, dev)
        g.adapt_frame(dg, cg, B.K, B.adapt_poses[k])
        o.adapt(d.numpy(), c.numpy(), B.K, B.adapt_poses[k])
    torch.cuda.synchronize()
    d, c = B.render_query(1)
    dg, cg = to_dev(d, c, dev)
    assert np.array_equal(g.leaves(dg, cg, B.K), o.leaves(d.numpy(), c.numpy(), B.K))
    for t in range(3):
        cg_ = g.counters(t)
        for leaf in np.nonzero(cg_)[0][:20]:
            eg, ng = g.reservoir(t, int(leaf))
            eo, no = o.reservoir(t, int(leaf))
            assert int(ng[0]) == no
            n = min(no, pp.reservoir_size)
            assert np.array_equal(eg[0][:n], eo[:n])
    r = g.relocalise_ex(dg, cg, B.K, seed=5)
    rc, pose, score, _ = o.relocalise(d.numpy(), c.numpy(), B.K, 5)
    assert r["status"] == rc
    if rc == 0:
        assert np.abs(r["pose"] - pose).max() < 1e-4


def test_train_argument_errors(dev):
    import paper_1801_08361_amd as rl
    pp, _ = pair(n_trees=1, depth=3, reservoir_size=16)
    g = rl.Forest(pp)
    sc = sr.small_scene(81, 64, 48)
    fg, _ = _frames(sc, (0,), dev)
    with pytest.raises(rl.RelocError):
        g.train(fg, 0, 8)
    with pytest.raises(rl.RelocError):
        g.train(fg, 2, 65)
    bad = [(fg[0][0], fg[0][1], fg[0][2], np.diag([1.0, 1.0, 2.0, 1.0]))]
    with pytest.raises(rl.RelocError):
        g.train(bad, 2, 8)
    g.drop_reservoirs()
    with pytest.raises(rl.RelocError):
        g.train(fg, 2, 8)
