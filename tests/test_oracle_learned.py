"""Pins of the oracle's verifier (Eqs. 3-4), bfloat16 rounding, MLP
initialisation, forward and gradient, per-pixel features and inlier labels:
closed forms, torch's own bfloat16 conversion and autograd, numpy's Philox,
and re-derivations from the oracle's already-pinned primitives."""
import math

import numpy as np
import pytest
import torch

import synthroom as sr
from tests.oracle_util import cam_points_f32, np_philox

torch.set_num_threads(4)


def test_verify_closed_forms(orc):
    rng = np.random.default_rng(0)
    db = rng.integers(500, 4000, size=(48, 64)).astype(np.uint16)
    vf, mu, acc = orc.verify(db, db)
    assert vf == 1.0 and mu == 0.0 and acc
    da = db + 30
    vf, mu, acc = orc.verify(da, db)
    assert mu == pytest.approx(0.030, abs=1e-12) and acc
    da = db + 60
    assert not orc.verify(da, db)[2]
    # half the rendered pixels invalid: fraction 0.5 is not enough (strictly greater)
    da = db.copy()
    da[:24] = 0
    vf, mu, acc = orc.verify(da, db)
    assert vf == 0.5 and mu == 0.0 and not acc
    da[23] = db[23]
    assert orc.verify(da, db)[2]
    # invalid query pixels are masked out of the mean
    da = db.copy()
    dbm = db.copy()
    dbm[:, :32] = 0
    da[:, :32] = 4000
    vf, mu, acc = orc.verify(da, dbm)
    assert mu == 0.0 and acc


def test_verify_valid_fraction_is_the_renders(orc):
    """|Omega_a| / |Omega| is taken over D_a, the render at the estimated pose:
    a pose that looks mostly past the modelled scene (render 30 % valid,
    matching the query where valid) is rejected although the query frame is
    fully valid; taking the fraction over the query would accept it."""
    rng = np.random.default_rng(4)
    query = rng.integers(800, 4000, size=(60, 80)).astype(np.uint16)
    render = query.copy()
    render[:, 24:] = 0                       # 24 of 80 columns valid: 30 %
    vf, mu, acc = orc.verify(render, query)
    assert vf == pytest.approx(0.3) and mu == 0.0 and not acc
    vf_q, _, acc_q = orc.verify(query, render)
    assert vf_q == 1.0 and acc_q


def test_bf16_matches_torch(orc):
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.normal(size=3000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, size=3000),
                         np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 3.4e38, 1e-40], np.float32)])
    ref = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([orc.bf16(float(x)) for x in xs], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_mlp_init_from_philox(orc):
    w = orc.mlp_init(42)
    assert w.shape == (5825,)
    fi, fo, off, cnt = [24, 64, 64], [64, 64, 1], [0, 24 * 64 + 64, 24 * 64 + 64 + 64 * 64 + 64], [1536, 4096, 64]
    for l in range(3):
        a = np.float32(math.sqrt(6.0 / (fi[l] + fo[l])))
        for k in (0, 1, cnt[l] - 1):
            u = np_philox((off[l] + k, 0, 0, 0), (42, 5))[0]
            r = np.float32(u >> 40) / np.float32(16777216.0)
            assert w[off[l] + k] == (np.float32(2.0) * r - np.float32(1.0)) * a
        assert np.all(np.abs(w[off[l]:off[l] + cnt[l]]) <= a)
    assert np.all(w[1536:1600] == 0) and w[-1] == 0


def torch_forward(w, x):
    """float64 torch forward with the oracle's roundings as straight-through
    estimators, so autograd gives the gradient the oracle defines."""
    def st(t):
        r = t.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64)
        return t + (r - t).detach()
    W1 = st(w[:1536].reshape(64, 24)); b1 = w[1536:1600]
    W2 = st(w[1600:5696].reshape(64, 64)); b2 = w[5696:5760]
    w3 = st(w[5760:5824]); b3 = w[5824]
    xb = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64)
    h1 = torch.relu(xb @ W1.T + b1)
    h1 = st(h1)
    h2 = torch.relu(h1 @ W2.T + b2)
    h2 = st(h2)
    return h2 @ w3 + b3


def test_mlp_forward_and_grad_match_torch(orc):
    rng = np.random.default_rng(2)
    w = orc.mlp_init(7)
    w[1536:1600] = rng.normal(scale=0.1, size=64)
    w[5696:5760] = rng.normal(scale=0.1, size=64)
    w[-1] = 0.3
    x = rng.normal(size=(200, 24)).astype(np.float32)
    # labels 0..255 are the targets y / 255 (hard 0 and 1 included)
    y = np.where(rng.random(200) < 0.3, 255, rng.integers(0, 256, 200) * (rng.random(200) < 0.5)).astype(np.uint8)
    z = orc.mlp_forward(w, x)
    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    zt = torch_forward(wt, x)
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-9, atol=1e-9)
    g, loss = orc.mlp_grad(w, x, y)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(zt, torch.tensor(y / 255.0, dtype=torch.float64))
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, wt.grad.numpy(), rtol=1e-9, atol=1e-12)


@pytest.fixture(scope="module")
def small_forest():
    import oracle
    sc = sr.small_scene(230, 160, 120)
    f = oracle.Forest(oracle.default_params(n_trees=3, depth=7, reservoir_size=64))
    for k in range(6):
        d, c = sc.render_adapt(k)
        f.adapt(d, c, sc.K, sc.adapt_poses[k])
    return sc, f


def test_features24_rederived(orc, small_forest):
    sc, f = small_forest
    d, c = sc.render_query(2)
    d, c = d.numpy(), c.numpy()
    H, W = d.shape
    valid = np.flatnonzero((d.reshape(-1) >= 500) & (d.reshape(-1) <= 5000))
    rng = np.random.default_rng(3)
    pix = rng.choice(valid, 60, replace=False)
    x = f.features24(d, c, sc.K, pix)
    f8 = f.features8(d, c, sc.K)
    kind = f.nodes()[0][-8:]
    leaves = f.leaves(d, c, sc.K)
    for i, p in enumerate(pix):
        dd = np.float32(d.reshape(-1)[p])
        assert x[i, 0] == dd / np.float32(5000.0)
        for j in range(8):
            r = f8[p, j]
            ref = np.float32(np.clip(r, -5000, 5000)) / np.float32(1000.0) if kind[j] == 0 else np.float32(r) / np.float32(255.0)
            assert x[i, 1 + j] == ref
        cand = []
        fill = 0
        for t in range(f.T):
            lf = int(leaves[t, p])
            _, cnt = f.reservoir(t, lf)
            cap = min(cnt, f.R)
            fill += cap
            for m in f.leaf_modes(t, lf):
                cand.append((np.float32(m["n"]) / np.float32(cap), m))
        top = sorted(range(len(cand)), key=lambda k: (-cand[k][0], k))[:3]
        for s, k in enumerate(top):
            pi, m = cand[k]
            assert x[i, 9 + 4 * s] == pi
            for a, si in enumerate((0, 3, 5)):
                assert x[i, 10 + 4 * s + a] == pytest.approx(-math.log(float(m["sinv"][si])) / 10.0, rel=1e-6)
        for s in range(len(top), 3):
            assert np.all(x[i, 9 + 4 * s:13 + 4 * s] == 0)
        assert x[i, 21] == np.float32(fill) / np.float32(f.T * f.R)
        assert x[i, 22] == np.float32(p % W) / np.float32(W)
        assert x[i, 23] == np.float32(p // W) / np.float32(H)


def test_labels_rederived(orc, small_forest):
    """A label is round(255 good / candidates): candidates are the modes of
    the pixel's leaves within rgb_tol of its colour in every channel (the
    pick's candidate set), good those within 5 cm of its world point,
    recomputed here in float64."""
    sc, f = small_forest
    d, c = sc.render_query(4)
    d, c = d.numpy(), c.numpy()
    valid = np.flatnonzero(d.reshape(-1) > 0)
    pix = np.random.default_rng(4).choice(valid, 300, replace=False)
    T = sc.query_poses[4]
    lab = f.label(d, c, sc.K, T, pix)
    cam = cam_points_f32(d, sc.K).astype(np.float64)
    leaves = f.leaves(d, c, sc.K)
    R32 = T[:3, :3].astype(np.float32).astype(np.float64)
    t32 = T[:3, 3].astype(np.float32).astype(np.float64)
    tol = f.params.rgb_tol
    rgb = c.reshape(-1, 3).astype(np.int64)
    checked = fractional = 0
    for i, p in enumerate(pix):
        y = R32 @ cam[p] + t32
        cand = [m for t in range(f.T) for m in f.leaf_modes(t, int(leaves[t, p]))
                if np.all(np.abs(m["rgb"].astype(np.int64) - rgb[p]) <= tol)]
        if not cand:
            assert lab[i] == 0
            continue
        dist2 = [float(np.sum((y - m["mu"].astype(np.float64)) ** 2)) for m in cand]
        if any(abs(x - 0.0025) <= 1e-6 for x in dist2):
            continue
        good = sum(1 for x in dist2 if x <= 0.0025)
        assert lab[i] == (255 * good + len(cand) // 2) // len(cand), (p, good, len(cand))
        checked += 1
        fractional += int(0 < lab[i] < 255)
    assert checked > 250 and fractional > 10 and 0 < lab.mean() < 255
