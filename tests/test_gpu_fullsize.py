"""GPU against the oracle at the full-size configuration: a 640x480 room with
1 % depth noise, 5 trees of depth 15 with 1024-entry reservoirs, 1024
hypotheses and 500 draws per round (a partial last group of 8 draws, 63
groups, a 1024-key cull, tiled inlier ids with a partial last tile). The
forests are adapted on 20 of the 200 adaptation frames to bound the oracle's
time. Also: a ragged batch (640x480 and 480x360, 512 and 1024 hypotheses) big
enough to take the 8-pixels-per-thread traversal and the split refinement,
each attempt checked against the oracle; 50 modes per leaf (the paper's
setting, Sec. 4.2.2), which takes 64-bit colour masks and the reduced-wave
scoring path; and checkpoints that resume exactly."""
import numpy as np
import pytest

import synthroom as sr
from tests.gpu_util import FULL, assert_modes_equal, banner, need_gpu, pair, rot_angle_deg, to_dev

pytestmark = pytest.mark.gpu

ADAPT = list(range(0, 200, 10))


@pytest.fixture(scope="module")
def full_pair():
    dev = need_gpu()
    import oracle
    import paper_1801_08361_amd as rl
    pp, po = pair(**FULL)
    g = rl.Forest(pp)
    o = oracle.Forest(po)
    sc = sr.full_scene(0)
    for k in ADAPT:
        d0, c0 = sc.render_adapt(k)
        d, c = to_dev(d0, c0, dev)
        banner(f"full-size adapt frame {k}")
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        o.adapt(d0, c0, sc.K, sc.adapt_poses[k])
    return dev, sc, g, o


def test_fullsize_reservoirs_counters_modes_sample(full_pair):
    """Reservoirs (with the replacement branch: counters above R), counters
    and modes of sampled leaves equal the oracle's bit for bit."""
    dev, sc, g, o = full_pair
    rng = np.random.default_rng(0)
    banner("full-size counters")
    total = 0
    n_replaced = 0
    for t in range(g.T):
        cnt = g.counters(t)
        total += int(cnt.sum())
        busy = np.argsort(-cnt.astype(np.int64))[:12]
        touched = np.flatnonzero(cnt > 0)
        some = rng.choice(touched, size=min(12, len(touched)), replace=False)
        for leaf in np.concatenate([busy, some]):
            leaf = int(leaf)
            eg, kg = g.reservoir(t, leaf, 1)
            eo, ko = o.reservoir(t, leaf)
            assert int(kg[0]) == ko, (t, leaf)
            n = min(ko, g.R)
            assert np.array_equal(eg[0][:n].view(np.uint8), eo[:n].view(np.uint8)), (t, leaf)
            n_replaced += int(ko > g.R)
            mg, ng = g.modes(t, leaf, 1)
            mo = o.leaf_modes(t, leaf)
            assert int(ng[0]) == len(mo), (t, leaf)
            assert_modes_equal(mg[0][: ng[0]], mo)
    assert total == o.total_samples
    assert n_replaced >= 5


def _compare_traces(tg, to, n_hyp):
    assert tg["pool_size"][0] == to["pool_size"][0]
    assert np.array_equal(tg["hyp_try"][:n_hyp], to["hyp_try"][:n_hyp])
    ok = to["hyp_try"][:n_hyp] >= 0
    np.testing.assert_allclose(tg["hyp_pose"][:n_hyp][ok], to["hyp_pose"][:n_hyp][ok], atol=1e-9)
    nr = int(to["n_rounds"][0])
    assert tg["n_rounds"][0] == nr
    for r in range(nr):
        na = int(to["n_alive"][r])
        assert tg["n_alive"][r] == na, r
        assert np.array_equal(tg["alive"][r, :na], to["alive"][r, :na]), r
        np.testing.assert_allclose(tg["energy"][r, :na], to["energy"][r, :na], rtol=1e-4, atol=1e-4)
    assert tg["final_hyp"][0] == to["final_hyp"][0]


@pytest.mark.parametrize("q", [0, 7])
def test_fullsize_relocalise_matches_oracle(full_pair, q):
    dev, sc, g, o = full_pair
    d0, c0 = sc.render_query(q)
    d, c = to_dev(d0, c0, dev)
    seed = 1 + q
    banner(f"full-size relocalise q={q}")
    sg, Tg, scg = g.relocalise(d, c, sc.K, seed=seed)
    tg = g.trace(1024)
    so, To, sco, to = o.relocalise(d0, c0, sc.K, seed=seed, trace=True)
    assert sg == so == 0
    if q == 0:   # more than 512 valid hypotheses: the cull sorts 1024 keys in LDS
        assert int(to["n_alive"][0]) > 512 and int(to["n_rounds"][0]) >= 10
    _compare_traces(tg, to, 1024)
    assert np.linalg.norm(Tg[:3, 3] - To[:3, 3]) < 1e-4
    assert rot_angle_deg(Tg[:3, :3], To[:3, :3]) < 1e-3
    assert abs(scg - sco) < 1e-6


def test_fullsize_ragged_batch_matches_oracle(full_pair):
    """Six attempts in one batch (five 640x480, one 480x360; 1024 and 512
    hypotheses): the batch walks 8 pixels per traversal thread and refines
    its large rounds in two kernels; every attempt equals the oracle."""
    import paper_1801_08361_amd as rl
    dev, sc, g, o = full_pair
    plan = [(1, 640, 480, 1024), (3, 640, 480, 512), (12, 480, 360, 1024), (20, 640, 480, 1024),
            (33, 640, 480, 512), (41, 640, 480, 1024)]
    att, ref = [], []
    for q, W, H, N in plan:
        d0, c0 = sc.render_query(q, width=W, height=H)
        d, c = to_dev(d0, c0, dev)
        K = sr.intrinsics(W, H)
        att.append(dict(forest=g, depth=d, rgb=c, K=K, seed=500 + q, n_hyp=N))
        ref.append((d0, c0, K, 500 + q, N))
    b = rl.Batch(tune=True)
    banner("full-size ragged batch")
    res = b.run(att)
    assert "pix_per_thread=8" in b.schedule()
    rl.profile_reset()
    rl.profile_enable(True)
    banner("full-size ragged batch, kernels one by one")
    res2 = b.run(att)
    rl.profile_enable(False)
    kernels = rl.profile_kernels()
    rl.profile_reset()
    assert "k_b_refine_sums" in kernels and "k_b_refine_solve" in kernels, kernels
    for r, r2 in zip(res, res2):
        assert r["status"] == r2["status"] and np.array_equal(r["pose"], r2["pose"])
    for i, (r, (d0, c0, K, seed, N)) in enumerate(zip(res, ref)):
        banner(f"full-size ragged batch: oracle attempt {i}")
        so, To, sco, to = o.relocalise(d0, c0, K, seed=seed, n_hyp=N, trace=True)
        assert r["status"] == so, i
        assert r["pool_size"] == to["pool_size"][0], i
        if so != 0:
            continue
        assert r["n_valid"] == int((to["hyp_try"][:N] >= 0).sum()), i
        assert r["n_rounds"] == int(to["n_rounds"][0]), i
        assert r["final_hyp"] == int(to["final_hyp"][0]), i
        assert np.linalg.norm(r["pose"][:3, 3] - To[:3, 3]) < 1e-4, i
        assert rot_angle_deg(r["pose"][:3, :3], To[:3, :3]) < 1e-3, i
        assert abs(r["score"] - sco) < 1e-6, i


def test_fifty_modes_per_leaf_matches_oracle():
    """M = 50 (the paper's setting) with T = 5: up to 250 modes per pixel, so
    the scoring workgroup stages them with 4 wavefronts instead of 8, and
    leaves with more than 32 modes pick through 64-bit colour masks."""
    dev = need_gpu()
    import oracle
    import paper_1801_08361_amd as rl
    pp, po = pair(n_trees=5, depth=8, reservoir_size=512, max_modes=50, min_cluster=1, n_hypotheses=256,
                  batch_pixels=64, rgb_tol=40)
    g = rl.Forest(pp)
    o = oracle.Forest(po)
    sc = sr.small_scene(13)
    for k in range(10):
        d0, c0 = sc.render_adapt(k)
        d, c = to_dev(d0, c0, dev)
        banner(f"fifty modes: adapt frame {k}")
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        o.adapt(d0, c0, sc.K, sc.adapt_poses[k])
    g.update_modes()
    _, ng = g.modes(0, 0, g.L)
    assert ng.max() > 32, ng.max()
    busiest = int(np.argmax(ng))
    mg, ngb = g.modes(0, busiest, 1)
    mo = o.leaf_modes(0, busiest)
    assert int(ngb[0]) == len(mo)
    assert_modes_equal(mg[0][: ngb[0]], mo)
    for q in (2, 9):
        d0, c0 = sc.render_query(q)
        d, c = to_dev(d0, c0, dev)
        banner(f"fifty modes: relocalise q={q}")
        sg, Tg, scg = g.relocalise(d, c, sc.K, seed=70 + q)
        tg = g.trace(256)
        so, To, sco, to = o.relocalise(d0, c0, sc.K, seed=70 + q, trace=True)
        assert sg == so
        if sg != 0:
            continue
        _compare_traces(tg, to, 256)
        assert np.linalg.norm(Tg[:3, 3] - To[:3, 3]) < 1e-4
        assert rot_angle_deg(Tg[:3, :3], To[:3, :3]) < 1e-3


def test_checkpoint_resume_equals_uninterrupted(tmp_path):
    """Adapt on frames 0-4, save, load, adapt on 5-9: reservoirs, counters,
    modes and relocalisations equal a forest adapted on 0-9 without a break,
    and the oracle's resumed forest; a checkpoint after dropping the
    reservoirs relocalises as before and refuses adaptation."""
    dev = need_gpu()
    import oracle
    import paper_1801_08361_amd as rl
    pp, po = pair(n_trees=5, depth=8, reservoir_size=16, max_modes=10, n_hypotheses=256, batch_pixels=64)
    sc = sr.small_scene(33)
    frames = [sc.render_adapt(k) for k in range(10)]
    dframes = [to_dev(d0, c0, dev) for d0, c0 in frames]

    def adapt(f, ks):
        for k in ks:
            f.adapt_frame(*dframes[k], sc.K, sc.adapt_poses[k])

    a = rl.Forest(pp)
    banner("checkpoint: uninterrupted forest")
    adapt(a, range(10))
    b = rl.Forest(pp)
    adapt(b, range(5))
    path = str(tmp_path / "gpu_forest.bin")
    banner("checkpoint: save")
    b.save(path)
    banner("checkpoint: load and resume")
    c = rl.Forest.load(path)
    assert c.params.depth == 8 and c.params.reservoir_size == 16
    adapt(c, range(5, 10))
    o = oracle.Forest(po)
    for k in range(5):
        o.adapt(*frames[k], sc.K, sc.adapt_poses[k])
    opath = str(tmp_path / "oracle_forest.bin")
    o.save(opath)
    o2 = oracle.Forest.load(opath, po)
    for k in range(5, 10):
        o2.adapt(*frames[k], sc.K, sc.adapt_poses[k])
    for t in range(a.T):
        ea, ka = a.reservoir(t, 0, a.L)
        ec, kc = c.reservoir(t, 0, c.L)
        assert np.array_equal(ka, kc) and np.array_equal(ea.view(np.uint8), ec.view(np.uint8)), t
        ma, na = a.modes(t, 0, a.L)
        mc, nc = c.modes(t, 0, c.L)
        assert np.array_equal(na, nc), t
        used = np.arange(a.M)[None, :] < na[:, None]      # slots past a leaf's count hold nothing
        assert np.array_equal(ma[used].view(np.uint8), mc[used].view(np.uint8)), t
        for leaf in range(0, a.L, 17):
            eo, ko = o2.reservoir(t, leaf)
            assert ko == int(kc[leaf])
            n = min(ko, c.R)
            assert np.array_equal(ec[leaf][:n].view(np.uint8), eo[:n].view(np.uint8)), (t, leaf)
    d0, c0 = sc.render_query(3)
    d, c_ = to_dev(d0, c0, dev)
    ra = a.relocalise(d, c_, sc.K, seed=8)
    rc = c.relocalise(d, c_, sc.K, seed=8)
    ro = o2.relocalise(d0, c0, sc.K, seed=8)
    assert ra[0] == rc[0] == ro[0] and np.array_equal(ra[1], rc[1]) and ra[2] == rc[2]
    if ro[0] == 0:
        assert np.linalg.norm(rc[1][:3, 3] - ro[1][:3, 3]) < 1e-4
    banner("checkpoint: after drop")
    c.drop_reservoirs()
    dpath = str(tmp_path / "gpu_dropped.bin")
    c.save(dpath)
    e = rl.Forest.load(dpath)
    re_ = e.relocalise(d, c_, sc.K, seed=8)
    assert re_[0] == rc[0] and np.array_equal(re_[1], rc[1]) and re_[2] == rc[2]
    assert e.memory() < a.memory()
    with pytest.raises(rl.RelocError):
        e.adapt_frame(*dframes[0], sc.K, sc.adapt_poses[0])
