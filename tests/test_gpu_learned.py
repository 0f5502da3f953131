"""GPU: the learned proposal and the verifier. The matrix-core lane layout is
checked against numpy; initialisation, per-pixel inputs, labels and the
verifier against the oracle (exact where both sides do the same integer or
FP32 steps); the MLP forward and gradient against the oracle's FP64 network
(which applies the same bfloat16 roundings); training must lower the loss
and the trained network must rank inliers above outliers on held-out
frames."""
import numpy as np
import pytest

import synthroom as sr
from tests.gpu_util import SMALL, banner, need_gpu, pair, to_dev

pytestmark = pytest.mark.gpu

SMALL_L = dict(n_trees=3, depth=8, reservoir_size=64, max_modes=10, n_hypotheses=64, batch_pixels=64)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16).view(torch.int16) \
        .numpy().view(np.uint16)


def bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32)


def rows32(x24: np.ndarray) -> np.ndarray:
    out = np.zeros((len(x24), 32), dtype=np.uint16)
    out[:, :24] = bf16_bits(x24)
    return out


def test_mfma_lane_layout():
    need_gpu()
    import paper_1801_08361_amd as rl
    rng = np.random.default_rng(0)
    for trial in range(3):
        banner(f"mfma probe {trial}")
        a = bf16_bits(rng.normal(size=(16, 32)))
        bt = bf16_bits(rng.normal(size=(16, 32)))
        if trial == 2:   # single nonzero entries locate every lane's rows and columns
            a = bf16_bits(np.eye(16, 32) * np.arange(1, 17)[:, None])
        c = rl.mfma_probe(a, bt)
        ref = bits_to_f32(a).astype(np.float64) @ bits_to_f32(bt).astype(np.float64).T
        bound = np.abs(bits_to_f32(a)).astype(np.float64) @ np.abs(bits_to_f32(bt)).astype(np.float64).T
        assert np.all(np.abs(c - ref) <= 1e-6 * bound + 1e-30), trial


def test_bf16_conversion_rounds_to_nearest_even():
    """The conversion instruction used for the network's inputs and hidden
    layers against round-to-nearest-even on the float's bit pattern: ties
    either way, values next to ties, denormals, overflow to infinity."""
    need_gpu()
    import paper_1801_08361_amd as rl
    rng = np.random.default_rng(11)
    hi = rng.integers(0, 1 << 16, 20000, dtype=np.uint64)
    lows = np.array([0x0000, 0x0001, 0x7FFF, 0x8000, 0x8001, 0xFFFF], dtype=np.uint64)
    bits = ((hi[:, None] << 16) | lows[None, :]).reshape(-1)
    bits = np.concatenate([bits, rng.integers(0, 1 << 32, 50000, dtype=np.uint64),
                           np.array([0x00000001, 0x00008000, 0x007FFFFF, 0x80008000, 0x7F7FFFFF, 0x7F7F8000,
                                     0x7F800000, 0xFF800000, 0x00000000, 0x80000000], dtype=np.uint64)])
    x = bits.astype(np.uint32).view(np.float32)
    finite = np.isfinite(x) | np.isinf(x)
    x = x[finite]
    b = x.view(np.uint32).astype(np.uint64)
    want = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)
    want[np.isinf(x)] = (b[np.isinf(x)] >> 16).astype(np.uint16)
    got = rl.bf16_round(x)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, [(hex(int(b[i])), hex(int(got[i])), hex(int(want[i]))) for i in bad[:5]]


def test_verify_matches_oracle():
    dev = need_gpu()
    import torch
    import oracle
    import paper_1801_08361_amd as rl
    rng = np.random.default_rng(1)
    cases = []
    db = rng.integers(500, 4000, size=(61, 97)).astype(np.uint16)
    cases.append((db + 30, db))
    da = db.copy(); da[:30] = 0
    cases.append((da, db))
    cases.append((db, np.zeros_like(db)))                       # nothing rendered: mu = inf
    cases.append((np.zeros_like(db), db))
    big = rng.integers(0, 65535, size=(480, 640)).astype(np.uint16)
    big2 = np.where(rng.random((480, 640)) < 0.2, 0, big + rng.integers(-40, 40, size=(480, 640))).astype(np.uint16)
    cases.append((big, big2))
    cases.append((np.full((1, 1), 1000, np.uint16), np.full((1, 1), 1049, np.uint16)))
    for i, (a, b) in enumerate(cases):
        banner(f"verify case {i} {a.shape}")
        got = rl.verify(torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev))
        ref = oracle.verify(a, b)
        assert got[0] == ref[0] and got[2] == ref[2], (i, got, ref)
        assert (got[1] == ref[1]) or (np.isinf(got[1]) and np.isinf(ref[1])), (i, got, ref)


def test_mlp_init_matches_oracle():
    need_gpu()
    import oracle
    import paper_1801_08361_amd as rl
    for seed in (0, 42, 12345678901):
        banner(f"mlp init seed {seed}")
        m = rl.Mlp(seed)
        assert np.array_equal(m.weights().view(np.uint32), oracle.mlp_init(seed).view(np.uint32))
        w = m.weights()
        w[1536:1600] = np.linspace(-1, 1, 64)
        m.set_weights(w)
        assert np.array_equal(m.weights(), w)


@pytest.fixture(scope="module")
def adapted():
    """The same small forest on the GPU and in the oracle, and its scene."""
    dev = need_gpu()
    import oracle
    import paper_1801_08361_amd as rl
    pp, po = pair(**SMALL_L)
    sc = sr.small_scene(610, 160, 120)
    g = rl.Forest(pp)
    o = oracle.Forest(po)
    for k in range(len(sc.adapt_poses)):
        d, c = sc.render_adapt(k)
        banner(f"learned forest adapt {k}")
        g.adapt_frame(*to_dev(d, c, dev), sc.K, sc.adapt_poses[k])
        o.adapt(d, c, sc.K, sc.adapt_poses[k])
    return dev, sc, g, o


def query_pixels(d: np.ndarray, n: int, seed: int) -> np.ndarray:
    """valid pixels, invalid pixels and both image corners"""
    rng = np.random.default_rng(seed)
    flat = d.reshape(-1)
    valid = np.flatnonzero((flat >= 500) & (flat <= 5000))
    invalid = np.flatnonzero((flat < 500) | (flat > 5000))
    pix = list(rng.choice(valid, min(n, len(valid)), replace=False))
    pix += list(invalid[:5]) + [0, len(flat) - 1]
    return np.array(pix, dtype=np.int32)


def test_pixel_features_match_oracle(adapted):
    import torch
    import paper_1801_08361_amd as rl
    dev, sc, g, o = adapted
    for q in (0, 3):
        d, c = sc.render_query(q)
        if q == 3:      # a hole of invalid depth
            d = d.clone(); d[40:60, 50:90] = 0
        pix = query_pixels(d.numpy(), 500, q)
        banner(f"pixel features query {q} n={len(pix)}")
        x, xf = rl.pixel_features(g, *to_dev(d, c, dev), sc.K, torch.from_numpy(pix).to(dev), with_fp32=True)
        xf = xf.cpu().numpy()
        ref = o.features24(d.numpy(), c.numpy(), sc.K, pix)
        exact = [k for k in range(24) if k not in (10, 11, 12, 14, 15, 16, 18, 19, 20)]
        assert np.array_equal(xf[:, exact], ref[:, exact]), q
        # -log(Sigma^-1_ii) / 10: logf of the two sides may differ in the last ulp
        np.testing.assert_allclose(xf, ref, rtol=2e-6, atol=1e-7)
        xb = x.cpu().numpy().view(np.uint16)
        assert np.array_equal(xb, rows32(xf)), q
        assert np.all(xb[:, 24:] == 0)
    # no pixels: nothing to do, no error
    rl.pixel_features(g, *to_dev(d, c, dev), sc.K, torch.zeros(0, dtype=torch.int32, device=dev))


def test_labels_match_oracle(adapted):
    import torch
    import paper_1801_08361_amd as rl
    dev, sc, g, o = adapted
    for q in (1, 2, 5):
        d, c = sc.render_query(q)
        pix = query_pixels(d.numpy(), 2000, 10 + q)
        for which, pose in (("true", sc.query_poses[q]), ("other", sc.adapt_poses[0])):
            banner(f"labels query {q} pose {which}")
            y = rl.label_pixels(g, *to_dev(d, c, dev), sc.K, pose, torch.from_numpy(pix).to(dev)).cpu().numpy()
            ref = o.label(d.numpy(), c.numpy(), sc.K, pose, pix)
            assert np.array_equal(y, ref), (q, which, int((y != ref).sum()))
            rate = {} if which == "true" else rate
            rate[which] = y.mean()
        # the true pose explains many pixels, a wrong one few
        assert rate["true"] > 0.1 and rate["other"] < 0.5 * rate["true"], (q, rate)


def random_weights(seed: int) -> np.ndarray:
    import oracle
    rng = np.random.default_rng(seed)
    w = oracle.mlp_init(seed)
    w[1536:1600] = rng.normal(scale=0.2, size=64)
    w[5696:5760] = rng.normal(scale=0.2, size=64)
    w[5824] = -0.4
    return w


def test_mlp_forward_matches_oracle():
    dev = need_gpu()
    import torch
    import oracle
    import paper_1801_08361_amd as rl
    rng = np.random.default_rng(3)
    m = rl.Mlp(5)
    for n in (1, 63, 64, 1000):
        w = random_weights(n)
        m.set_weights(w)
        x = rng.normal(size=(n, 24)).astype(np.float32)
        x = bits_to_f32(bf16_bits(x))              # inputs the GPU receives exactly
        banner(f"mlp forward n={n}")
        z = m.logits(torch.from_numpy(rows32(x).view(np.int16)).to(dev)).cpu().numpy()
        ref = oracle.mlp_forward(w, x)
        err = np.abs(z - ref)
        # FP32 accumulation vs FP64: a hidden value may round to the other
        # neighbouring bfloat16 (one unit in 2^8); the bulk agrees to ~1e-6
        assert np.all(err <= 5e-3 * (1.0 + np.abs(ref))), (n, err.max())
        assert np.median(err) <= 1e-5 * (1.0 + np.median(np.abs(ref))), n


def test_mlp_gradient_matches_oracle():
    dev = need_gpu()
    import torch
    import oracle
    import paper_1801_08361_amd as rl
    rng = np.random.default_rng(4)
    m = rl.Mlp(6)
    for n in (1, 64, 777, 4096):
        w = random_weights(100 + n)
        m.set_weights(w)
        x = bits_to_f32(bf16_bits(rng.normal(size=(n, 24)).astype(np.float32)))
        y = np.where(rng.random(n) < 0.4, 255, rng.integers(0, 256, n) * (rng.random(n) < 0.5)).astype(np.uint8)
        banner(f"mlp gradient n={n}")
        g, loss = m.gradient(torch.from_numpy(rows32(x).view(np.int16)).to(dev), torch.from_numpy(y).to(dev))
        gr, lr = oracle.mlp_grad(w, x, y)
        assert loss == pytest.approx(lr, rel=1e-4, abs=1e-6), n
        cos = float(g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr)))
        assert cos >= 0.9999, (n, cos)
        assert np.max(np.abs(g - gr)) <= 1e-2 * np.max(np.abs(gr)), n
        # every block of the gradient, separately
        for lo, hi in ((0, 1536), (1536, 1600), (1600, 5696), (5696, 5760), (5760, 5824), (5824, 5825)):
            if np.any(gr[lo:hi] != 0):
                assert np.max(np.abs(g[lo:hi] - gr[lo:hi])) <= 2e-2 * np.max(np.abs(gr[lo:hi])) + 1e-7, (n, lo)


def test_training_lowers_loss_and_ranks_inliers(adapted):
    import torch
    import paper_1801_08361_amd as rl
    from paper_1801_08361_amd import learned
    dev, sc, g, o = adapted
    frames = []
    for q in range(0, 14):
        d, c = to_dev(*sc.render_query(q), dev)
        frames.append((d, c, sc.K, sc.query_poses[q]))
    banner("training rows")
    # train on the even queries of the adapted stretch of the path, hold out the odd ones
    x, y = learned.training_rows(g, frames[0::2])
    assert x.shape[0] == y.shape[0] > 50000
    base = float(y.float().mean()) / 255.0
    assert 0.02 < base < 0.95
    m = rl.Mlp(9)
    g0, l0 = m.gradient(x, y)
    banner("training")
    losses = m.train(x, y, epochs=6, batch_rows=2048, lr=2e-3, seed=3)
    g1, l1 = m.gradient(x, y)
    # better than the untrained network and than the best constant guess
    h = -(base * np.log(base) + (1 - base) * np.log(1 - base))
    assert l1 < min(l0, h) - 0.01, (l0, l1, h, losses)
    # held-out frames: pixels whose pick can be correct rank above those
    # whose pick cannot (area under the ROC curve)
    xh, yh = learned.training_rows(g, frames[1::2])
    z = m.logits(xh).cpu().numpy().astype(np.float64)
    yh = yh.cpu().numpy() > 0
    ranks = np.empty(len(z))
    ranks[np.argsort(z, kind="stable")] = np.arange(1, len(z) + 1)
    npos, nneg = int(yh.sum()), int((~yh).sum())
    auc = (ranks[yh].sum() - npos * (npos + 1) / 2) / (npos * nneg)
    assert auc > 0.6, auc
    # pick weights of whole frames are floor(sigma 65536) + 1 of the same network
    d, c, K, _ = frames[12]
    banner("pixel weights")
    wts, prob = m.pixel_weights(g, d, c, K, with_prob=True)
    wts = wts.cpu().numpy().view(np.uint32)
    prob = prob.cpu().numpy()
    flat = d.reshape(-1).cpu().numpy()
    ok = (flat >= 500) & (flat <= 5000)
    assert np.all(wts[~ok] == 0) and np.all(prob[~ok] == 0)
    assert np.array_equal(wts[ok], np.floor(prob[ok] * np.float32(65536.0)).astype(np.uint32) + 1)
    pix = torch.from_numpy(np.flatnonzero(ok).astype(np.int32)).to(dev)
    z = m.logits(rl.pixel_features(g, d, c, K, pix)).cpu().numpy()
    np.testing.assert_allclose(prob[ok], 1.0 / (1.0 + np.exp(-z.astype(np.float64))), rtol=1e-6, atol=1e-7)


def test_learned_weights_drive_the_relocaliser(adapted):
    """The trained network's weights, passed to the relocaliser, give the
    oracle's result for the same weights (the picks follow the integer CDF)."""
    import oracle
    import paper_1801_08361_amd as rl
    from paper_1801_08361_amd import learned
    dev, sc, g, o = adapted
    frames = [(*to_dev(*sc.render_query(q), dev), sc.K, sc.query_poses[q]) for q in range(8)]
    x, y = learned.training_rows(g, frames)
    m, _ = learned.train(x, y, seed=2, epochs=3, batch_rows=2048)
    for q in (8, 9):
        d, c = sc.render_query(q)
        dd, cc = to_dev(d, c, dev)
        wts = m.pixel_weights(g, dd, cc, sc.K)
        banner(f"learned relocalise query {q}")
        res = g.relocalise_ex(dd, cc, sc.K, seed=77 + q, n_hyp=64, weights=wts)
        rc, pose, score = o.relocalise(d.numpy(), c.numpy(), sc.K, seed=77 + q, n_hyp=64,
                                       weights=wts.cpu().numpy().view(np.uint32))[:3]
        assert res["status"] == rc
        if rc == 0:
            assert np.max(np.abs(res["pose"] - pose)) < 1e-4
            assert res["score"] == pytest.approx(score, rel=1e-4)


def test_learned_in_graph_equals_given_weights(adapted):
    """The proposal computed inside the relocalisation graph (from the
    attempt's own leaves) gives the same result as passing the stand-alone
    kernel's weights; and a batch of such attempts equals the plain calls."""
    import paper_1801_08361_amd as rl
    dev, sc, g, o = adapted
    m = rl.Mlp(21)
    w = random_weights(21)
    m.set_weights(w)
    atts = []
    for q in (3, 6, 11):
        d, c = to_dev(*sc.render_query(q), dev)
        banner(f"learned in graph query {q}")
        wts = m.pixel_weights(g, d, c, sc.K)
        r1 = g.relocalise_ex(d, c, sc.K, seed=500 + q, n_hyp=64, weights=wts)
        r2 = g.relocalise_learned(m, d, c, sc.K, seed=500 + q, n_hyp=64)
        for k in ("status", "score", "final_hyp", "n_rounds", "n_valid", "mode_evals", "pair_evals", "pool_size"):
            assert r1[k] == r2[k], (q, k)
        assert np.array_equal(r1["pose"], r2["pose"]), q
        atts.append(dict(forest=g, depth=d, rgb=c, K=sc.K, seed=500 + q, n_hyp=64, proposal=m))
        atts.append(dict(forest=g, depth=d, rgb=c, K=sc.K, seed=700 + q, n_hyp=32))
    banner("learned in a batch")
    res = rl.Batch(tune=True).run(atts)
    for a, r in zip(atts, res):
        if "proposal" in a:
            p = g.relocalise_learned(m, a["depth"], a["rgb"], a["K"], seed=a["seed"], n_hyp=a["n_hyp"])
        else:
            p = g.relocalise_ex(a["depth"], a["rgb"], a["K"], seed=a["seed"], n_hyp=a["n_hyp"])
        assert r["status"] == p["status"] and np.array_equal(r["pose"], p["pose"]) and r["score"] == p["score"]
    import paper_1801_08361_amd as rl2
    with pytest.raises(rl2.RelocError):
        rl.Batch().run([dict(atts[0], weights=m.pixel_weights(g, atts[0]["depth"], atts[0]["rgb"], sc.K))])


def test_learned_proposal_gains_good_hypotheses():
    """What the trained network gains over uniform picks: on held-out queries
    of ten small rooms (one network for all ten, trained on the GPU from
    verified extra frames of the same rooms), hypotheses drawn with learned
    pick weights land within 5 cm / 5 deg of the truth more often, and more
    attempts succeed, at small hypothesis counts where uniform picks still
    miss (measured: 0.28 vs 0.20 good hypotheses per attempt at N = 8, 0.53 vs
    0.40 at N = 16; success 50.5 vs 45.5 % and 69.5 vs 64.0 %)."""
    dev = need_gpu()
    import oracle
    import paper_1801_08361_amd as rl
    from paper_1801_08361_amd import learned
    forests, scenes, items = [], [], []
    for room in range(200, 210):
        sc = sr.small_scene(room)
        g = rl.Forest(rl.params_default(**SMALL))
        for k in range(len(sc.adapt_poses)):
            d, c = sc.render_adapt(k, device=dev)
            g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        g.update_modes()
        forests.append(g)
        scenes.append(sc)
        for j, T in enumerate(sc.extra_poses(4, tag=7)):
            items.append((g, sc, T, 900 + 10 * room + j))
    banner("learned gain: training rows from verified extra frames")
    xs, ys = [], []
    for g, sc, T, tag in items:
        d, c = sc.render_pose(T, noise_tag=tag, device=dev)
        pose, _ = learned.verified_pose(g, d, c, sc.K, seed=tag, model_depth=lambda P: sc.model_depth(P, device=dev))
        if pose is None:
            continue
        x, y = learned.frame_rows(g, d, c, sc.K, pose, max_pixels=60_000, seed=tag)
        xs.append(x)
        ys.append(y)
    import torch
    assert len(xs) >= 5
    x, y = torch.cat(xs).contiguous(), torch.cat(ys).contiguous()
    banner("learned gain: training")
    m, losses = learned.train(x, y, seed=4, epochs=20, batch_rows=4096, lr=2e-3)
    assert losses[-1] < losses[0]

    def evaluate(n_hyp, use):
        good = ok = 0
        for g, sc in zip(forests, scenes):
            for q in range(len(sc.query_poses)):
                d, c = sc.render_query(q, device=dev)
                if use:
                    r = g.relocalise_learned(m, d, c, sc.K, seed=5000 + q, n_hyp=n_hyp)
                else:
                    r = g.relocalise_ex(d, c, sc.K, seed=5000 + q, n_hyp=n_hyp)
                ok += int(r["status"] == 0 and oracle.pose_success(r["pose"], sc.query_poses[q])[0])
                tr = g.trace(n_hyp)
                for h in np.flatnonzero(tr["hyp_try"] >= 0):
                    T = np.eye(4)
                    T[:3, :3] = tr["hyp_pose"][h, :9].reshape(3, 3)
                    T[:3, 3] = tr["hyp_pose"][h, 9:]
                    good += int(oracle.pose_success(T, sc.query_poses[q])[0])
        return good, ok

    for n_hyp in (8, 16):
        banner(f"learned gain: evaluation at N={n_hyp}")
        gl, sl = evaluate(n_hyp, True)
        gu, su = evaluate(n_hyp, False)
        assert gl >= 1.15 * gu, (n_hyp, gl, gu)
        assert sl >= su, (n_hyp, sl, su)
