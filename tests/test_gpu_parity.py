"""GPU parity: the HIP path against the CPU oracle, stage by stage, through the
C ABI. Integer stages (split nodes, features, leaves, reservoirs, cluster
membership) must match bit for bit; energies within 1e-4 relative; poses
within 1e-4 m and 1e-3 degrees. Sizes span several tiles and ragged tails."""
import numpy as np
import pytest

import synthroom as sr
from tests.gpu_util import FULL, SMALL, banner, need_gpu, pair, rot_angle_deg, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return need_gpu()


def make(pp, po):
    import oracle
    import paper_1801_08361_amd as rl
    return rl.Forest(pp), oracle.Forest(po)


def test_lane_moves(dev):
    """The cross-lane helpers that the cull's sort, the refinement's
    butterfly and the scoring's tree scan use move exactly the lanes they
    name (the butterfly's additions pair the same lanes as the oracle's)."""
    import paper_1801_08361_amd as rl
    banner("lane moves")
    out = rl.lane_probe().astype(np.int64)
    lane = np.arange(64)
    v = 1000 + lane
    for k in range(6):
        assert np.array_equal(out[k], v[lane ^ (1 << k)]), k
    for k, o in enumerate((1, 2, 4, 8)):
        want = np.where(lane % 16 >= o, v[np.maximum(lane - o, 0)], 0)
        assert np.array_equal(out[6 + k], want), o
    assert np.array_equal(out[10], 5000 + (lane ^ (1 << (lane % 6))))
    assert np.all(out[11] == 5037)


@pytest.mark.parametrize("cfg", ["small", "full"])
def test_nodes_match(dev, cfg):
    kw = SMALL if cfg == "small" else FULL
    pp, po = pair(**kw)
    banner(f"nodes {cfg}")
    g, o = make(pp, po)
    for a, b in zip(g.nodes(), o.nodes()):
        assert np.array_equal(a, b)


def test_features8_by_hand(dev):
    from tests.test_oracle_features import image, K_REF
    pp, po = pair(n_trees=1, depth=2, reservoir_size=4)
    g, o = make(pp, po)
    kind, dx, dy, thr = o.nodes()
    base = 3
    spec = [(0, -1300, 0, 0), (0, -5000, 0, 0), (0, 0, 1000, 0), (1, 5000, 0, 0), (3, -1999, -1999, 0),
            (2, 0, 0, 0), (0, 1000, 0, 0), (0, 2600, 0, 0)]
    for j, (k, x, y, t) in enumerate(spec):
        kind[base + j], dx[base + j], dy[base + j], thr[base + j] = k, x, y, t
    o.set_nodes(kind, dx, dy, thr)
    g.set_nodes(kind, dx, dy, thr)
    depth, rgb = image()
    d, c = to_dev(depth, rgb, dev)
    banner("features8 by hand")
    for K in (K_REF, (554.0, 554.0, 4.0, 3.0)):
        assert np.array_equal(g.features8(d, c, K), o.features8(depth, rgb, K))


@pytest.mark.parametrize("size", [(320, 240), (97, 61), (640, 480)])
def test_leaves_and_features_rendered(dev, size):
    W, H = size
    kw = dict(SMALL)
    if W == 640:
        kw = dict(FULL)
    pp, po = pair(**kw)
    g, o = make(pp, po)
    sc = sr.small_scene(7, W, H)
    d0, c0 = sc.render_query(3)
    d, c = to_dev(d0, c0, dev)
    banner(f"leaves {W}x{H}")
    lg = g.leaves(d, c, sc.K)
    lo = o.leaves(d0, c0, sc.K)
    assert np.array_equal(lg, lo)
    assert np.array_equal(g.features8(d, c, sc.K), o.features8(d0, c0, sc.K))
    assert (lg >= 0).any() and (lg < 0).sum() == (lo < 0).sum()


@pytest.mark.parametrize("size", [(97, 61), (161, 97), (640, 480)])
def test_valid_pixels_match_oracle(dev, size):
    """reloc_valid_pixels lists exactly the pixels the oracle gives a leaf
    (valid depth), in raster order, over several 1024-pixel blocks and a
    ragged last one; depths on both ends of the range, out of range and all
    invalid frames included."""
    import paper_1801_08361_amd as rl
    import torch
    W, H = size
    pp, po = pair(**SMALL)
    g, o = make(pp, po)
    sc = sr.small_scene(7, W, H)
    d0, c0 = sc.render_query(3)
    dn = d0.numpy().copy()
    flat = dn.reshape(-1)
    rng = np.random.default_rng(W)
    for val in (0, pp.depth_min_mm - 1, pp.depth_min_mm, pp.depth_max_mm, pp.depth_max_mm + 1, 65535):
        flat[rng.choice(flat.size, max(1, flat.size // 50), replace=False)] = val
    d0 = torch.from_numpy(dn)
    banner(f"valid pixels {W}x{H}")
    for dd in (d0, torch.zeros_like(d0)):
        d, c = to_dev(dd, c0, dev)
        got = rl.valid_pixels(g, d, c, sc.K).cpu().numpy()
        want = np.nonzero(o.leaves(dd.numpy(), c0.numpy(), sc.K)[0].reshape(-1) >= 0)[0]
        assert np.array_equal(got, want)


def test_leaves_special_thresholds(dev):
    pp, po = pair(n_trees=3, depth=6, reservoir_size=8)
    g, o = make(pp, po)
    kind, dx, dy, thr = g.nodes()
    n = 3 * 63
    sc = sr.small_scene(8, 64, 48)
    d0, c0 = sc.render_query(0)
    d, c = to_dev(d0, c0, dev)
    for val, leaf in ((-400000, 63), (400000, 0)):
        thr2 = thr.copy()
        thr2[:n] = val
        g.set_nodes(kind, dx, dy, thr2)
        banner(f"leaves thr={val}")
        lg = g.leaves(d, c, sc.K)
        valid = d0.numpy().reshape(-1) > 0
        assert np.all(lg[:, valid] == leaf) and np.all(lg[:, ~valid] == -1)


@pytest.mark.parametrize("R,frames,size", [(16, 6, (160, 120)), (256, 4, (320, 240)), (64, 3, (333, 201))])
def test_reservoirs_match(dev, R, frames, size):
    W, H = size
    pp, po = pair(n_trees=5, depth=8, reservoir_size=R, seed=1234 + R)
    g, o = make(pp, po)
    sc = sr.small_scene(9, W, H)
    for k in range(frames):
        d0, c0 = sc.render_adapt(k)
        d, c = to_dev(d0, c0, dev)
        banner(f"adapt R={R} frame {k} {W}x{H}")
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        o.adapt(d0, c0, sc.K, sc.adapt_poses[k])
    import torch
    torch.cuda.synchronize()
    for t in range(5):
        eg, cg = g.reservoir(t, 0, g.L)
        co = np.zeros(g.L, np.uint32)
        eo = np.zeros((g.L, R), dtype=eg.dtype)
        for leaf in range(g.L):
            e, cnt = o.reservoir(t, leaf)
            co[leaf] = cnt
            eo[leaf] = e.view(eg.dtype)
        assert np.array_equal(cg, co), t
        n = np.minimum(co, R)
        mask = np.arange(R)[None, :] < n[:, None]
        assert np.array_equal(eg[mask], eo[mask]), t
    assert co.max() > R


def pts(xyz, rgb=None):
    from oracle import ENTRY_DTYPE
    a = np.zeros(len(xyz), dtype=ENTRY_DTYPE)
    a["x"], a["y"], a["z"] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    if rgb is not None:
        a["r"], a["g"], a["b"] = rgb[:, 0], rgb[:, 1], rgb[:, 2]
    return a


def assert_modes_equal(mg, mo):
    assert len(mg) == len(mo)
    if len(mo) == 0:
        return
    assert np.array_equal(mg["n"], mo["n"])
    assert np.array_equal(mg["mu"].view(np.uint32), mo["mu"].view(np.uint32))
    assert np.array_equal(mg["sinv"].view(np.uint32), mo["sinv"].view(np.uint32))
    np.testing.assert_allclose(mg["kappa"], mo["kappa"], rtol=1e-6, atol=1e-6)
    assert np.array_equal(mg["rgb"], mo["rgb"])


@pytest.mark.parametrize("seed", range(8))
def test_modes_from_points_match(dev, seed):
    import oracle
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(0, 1025))
    xyz = rng.integers(0, 14, size=(n, 3)) * 25 + (rng.integers(0, 3, size=(n, 1)) * 1500)
    rgb = rng.integers(0, 256, size=(n, 3))
    pp, po = pair(reservoir_size=1024, max_modes=10, min_cluster=[0, 1, 3, 8][seed % 4])
    g, _ = make(pp, po)
    banner(f"modes_from_points seed={seed} n={n}")
    mg = g.modes_from_points(pts(xyz, rgb))
    mo, _ = oracle.modes_from_points(po, pts(xyz, rgb))
    assert_modes_equal(mg, mo.view(mg.dtype) if len(mo) else mg[:0])


def test_leaf_modes_match(dev):
    pp, po = pair(**SMALL)
    g, o = make(pp, po)
    sc = sr.small_scene(10)
    for k in range(6):
        d0, c0 = sc.render_adapt(k)
        d, c = to_dev(d0, c0, dev)
        banner(f"adapt for modes frame {k}")
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        o.adapt(d0, c0, sc.K, sc.adapt_poses[k])
    banner("modes all leaves")
    for t in range(5):
        mg, ng = g.modes(t, 0, g.L)
        for leaf in range(0, g.L, 1 if t == 0 else 7):
            mo = o.leaf_modes(t, leaf)
            assert ng[leaf] == len(mo), (t, leaf)
            assert_modes_equal(mg[leaf, : ng[leaf]], mo.view(mg.dtype))


@pytest.fixture(scope="module")
def adapted_pair(dev):
    pp, po = pair(**SMALL)
    g, o = make(pp, po)
    sc = sr.small_scene(11)
    for k in range(12):
        d0, c0 = sc.render_adapt(k)
        d, c = to_dev(d0, c0, dev)
        banner(f"adapt pair frame {k}")
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        o.adapt(d0, c0, sc.K, sc.adapt_poses[k])
    return sc, g, o


@pytest.mark.parametrize("q,n_hyp", [(1, 256), (4, 256), (9, 100), (13, 1), (17, 33)])
def test_relocalise_matches_oracle(dev, adapted_pair, q, n_hyp):
    sc, g, o = adapted_pair
    d0, c0 = sc.render_query(q)
    d, c = to_dev(d0, c0, dev)
    seed = 7000 + q
    banner(f"relocalise q={q} N={n_hyp}")
    sg, Tg, scg = g.relocalise(d, c, sc.K, seed=seed, n_hyp=n_hyp)
    tg = g.trace(n_hyp)
    so, To, sco, to = o.relocalise(d0, c0, sc.K, seed=seed, n_hyp=n_hyp, trace=True)
    assert sg == so
    assert tg["pool_size"][0] == to["pool_size"][0]
    assert np.array_equal(tg["hyp_try"], to["hyp_try"])
    ok = tg["hyp_try"] >= 0
    np.testing.assert_allclose(tg["hyp_pose"][ok], to["hyp_pose"][ok], atol=1e-9)
    if sg != 0:
        return
    nr = int(to["n_rounds"][0])
    assert tg["n_rounds"][0] == nr
    for r in range(nr):
        na = int(to["n_alive"][r])
        assert tg["n_alive"][r] == na
        assert np.array_equal(tg["alive"][r, :na], to["alive"][r, :na]), r
        np.testing.assert_allclose(tg["energy"][r, :na], to["energy"][r, :na], rtol=1e-4, atol=1e-4)
    assert tg["final_hyp"][0] == to["final_hyp"][0]
    assert np.linalg.norm(Tg[:3, 3] - To[:3, 3]) < 1e-4
    assert rot_angle_deg(Tg[:3, :3], To[:3, :3]) < 1e-3
    assert abs(scg - sco) < 1e-6


@pytest.mark.parametrize("tol", [0, 40, 300])
def test_relocalise_many_modes_colour_tolerances(dev, tol):
    """Leaves with more than 12 modes (the general colour-mask path) and
    colour tolerances at 0, inside the byte range and beyond it."""
    pp, po = pair(**dict(SMALL, max_modes=20, min_cluster=1, rgb_tol=tol))
    g, o = make(pp, po)
    sc = sr.small_scene(12)
    for k in range(8):
        d0, c0 = sc.render_adapt(k)
        d, c = to_dev(d0, c0, dev)
        banner(f"many modes tol={tol}: adapt frame {k}")
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        o.adapt(d0, c0, sc.K, sc.adapt_poses[k])
    g.update_modes()
    _, ng = g.modes(0, 0, g.L)
    assert ng.max() > 12, ng.max()
    for q in (3, 6):
        d0, c0 = sc.render_query(q)
        d, c = to_dev(d0, c0, dev)
        banner(f"many modes tol={tol}: relocalise q={q}")
        sg, Tg, _ = g.relocalise(d, c, sc.K, seed=900 + q, n_hyp=128)
        tg = g.trace(128)
        so, To, _, to = o.relocalise(d0, c0, sc.K, seed=900 + q, n_hyp=128, trace=True)
        assert sg == so
        assert np.array_equal(tg["hyp_try"], to["hyp_try"]), q
        if sg == 0:
            assert np.linalg.norm(Tg[:3, 3] - To[:3, 3]) < 1e-4
            assert rot_angle_deg(Tg[:3, :3], To[:3, :3]) < 1e-3


def test_negative_colour_tolerance_rejected():
    import paper_1801_08361_amd as rl
    with pytest.raises(rl.RelocError):
        rl.Forest(rl.params_default(rgb_tol=-1))


def test_relocalise_failures(dev, adapted_pair):
    import paper_1801_08361_amd as rl
    sc, g, o = adapted_pair
    d0, c0 = sc.render_query(2)
    d, c = to_dev(d0, c0, dev)
    banner("failure: zero depth")
    import torch
    assert g.relocalise(torch.zeros_like(d), c, sc.K, seed=1)[0] == rl.FAIL_NO_VALID_PIXELS
    banner("failure: empty forest")
    e = rl.Forest(rl.params_default())
    assert e.relocalise(d, c, sc.K, seed=1)[0] == rl.FAIL_NO_MODES
    banner("failure: strict rigidity")
    s = rl.Forest(rl.params_default(rigid_ratio2=0.0))
    s.adapt_frame(d, c, sc.K, sc.query_poses[2])
    assert s.relocalise(d, c, sc.K, seed=1)[0] == rl.FAIL_NO_HYPOTHESIS
    banner("failure: bad args")
    with pytest.raises(rl.RelocError):
        g.relocalise(d, c, (0.0, 277.0, 160.0, 120.0), seed=1)
    bad = np.eye(4)
    bad[0, 0] = 1.1
    with pytest.raises(rl.RelocError):
        g.adapt_frame(d, c, sc.K, bad)
    with pytest.raises(rl.RelocError):
        rl.Forest(rl.params_default(depth=17))
    with pytest.raises(rl.RelocError):
        rl.Forest(rl.params_default(offset_pxmm=2_000_000))
    banner("failure: focal length beyond the 24-bit probe placement")
    with pytest.raises(rl.RelocError):
        g.relocalise(d, c, (2.0e6, 277.0, 160.0, 120.0), seed=1)
    banner("failure: probe offsets of 2^14 px or more")
    far = rl.Forest(rl.params_default(depth_min_mm=1, f_ref_px16=1))
    with pytest.raises(rl.RelocError):
        far.adapt_frame(d, c, sc.K, sc.query_poses[2])


def test_drop_reservoirs_keeps_results(dev):
    import paper_1801_08361_amd as rl
    pp, _ = pair(**SMALL)
    g = rl.Forest(pp)
    sc = sr.small_scene(12)
    for k in range(5):
        d, c = to_dev(*sc.render_adapt(k), dev)
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
    d, c = to_dev(*sc.render_query(2), dev)
    banner("drop reservoirs")
    a = g.relocalise(d, c, sc.K, seed=5)
    before = g.memory()
    g.drop_reservoirs()
    assert g.memory() < before
    b = g.relocalise(d, c, sc.K, seed=5)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2] == b[2]
    with pytest.raises(rl.RelocError):
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[0])


def test_success_small_rooms_gpu(dev):
    """The GPU path alone on rendered rooms: >= 95 % within 5 cm / 5 deg."""
    import oracle
    import paper_1801_08361_amd as rl
    ok = tot = 0
    for room in range(300, 306):
        sc = sr.small_scene(room)
        g = rl.Forest(rl.params_default(**SMALL))
        for k in range(len(sc.adapt_poses)):
            d, c = to_dev(*sc.render_adapt(k, device=dev), dev)
            g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        banner(f"success room {room}")
        for q in range(len(sc.query_poses)):
            d, c = to_dev(*sc.render_query(q, device=dev), dev)
            st, T, _ = g.relocalise(d, c, sc.K, seed=q + 1)
            ok += int(st == 0 and oracle.pose_success(T, sc.query_poses[q])[0])
            tot += 1
    assert ok / tot >= 0.95, (ok, tot)
