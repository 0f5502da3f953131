"""Pins of the single steps inside the oracle's relocalisation: the mode
energy term (closed forms on constructed modes, scipy's Gaussian
log-density), the per-round energies, culls and inlier counts (recomputed in
float64 from the traced poses, numpy's Philox draws and the leaf modes), the
hypothesis checks (constructed triples that each fail exactly one check), the
colour test, the degeneracy threshold of the pose solve, and the preemptive
loop's special cases (exact modes give the exact pose, duplicated hypotheses
keep the lower index, one hypothesis is one alignment and one refinement)."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import synthroom as sr
from oracle_util import cam_points_f32, horn_rotation, np_philox, np_uniform_int, rand_rotation

SINV = dict(xx=4.0e4, xy=-1.2e4, xz=0.7e4, yy=2.5e4, yz=-0.3e4, zz=1.8e4)


def _mode(orc, mu, sinv, kappa):
    m = np.zeros(1, dtype=orc.MODE_DTYPE)
    m["mu"] = np.asarray(mu, dtype=np.float32)
    m["sinv"] = np.asarray(sinv, dtype=np.float32)
    m["kappa"] = np.float32(kappa)
    return m[0]


def test_mode_term_closed_forms(orc):
    """q = d^T Sigma^-1 d along each axis and each axis pair picks out one
    stored element: a swapped or misplaced inverse-covariance entry fails."""
    s = SINV
    mu = np.array([1.0, -2.0, 0.5])
    kappa = -3.25
    m = _mode(orc, mu, [s["xx"], s["xy"], s["xz"], s["yy"], s["yz"], s["zz"]], kappa)
    dl = 0.01
    cases = {
        (1, 0, 0): s["xx"], (0, 1, 0): s["yy"], (0, 0, 1): s["zz"],
        (1, 1, 0): s["xx"] + 2 * s["xy"] + s["yy"],
        (1, 0, 1): s["xx"] + 2 * s["xz"] + s["zz"],
        (0, 1, 1): s["yy"] + 2 * s["yz"] + s["zz"],
        (1, -1, 1): s["xx"] + s["yy"] + s["zz"] - 2 * s["xy"] + 2 * s["xz"] - 2 * s["yz"],
    }
    for d, coef in cases.items():
        y = (mu + dl * np.array(d, dtype=np.float64)).astype(np.float32)
        dd = y.astype(np.float64) - mu.astype(np.float32).astype(np.float64)
        want = kappa + 0.5 * coef * float(dd @ dd) / (dl * dl) * dl * dl if d.count(0) == 2 else None
        # exact float64 quadratic form of the rounded offsets
        S = np.array([[s["xx"], s["xy"], s["xz"]], [s["xy"], s["yy"], s["yz"]], [s["xz"], s["yz"], s["zz"]]])
        exact = kappa + 0.5 * float(dd @ S @ dd)
        got = orc.mode_term(m, y)
        assert got == pytest.approx(exact, rel=2e-6, abs=1e-6), (d, got, exact)
        if want is not None:
            assert got == pytest.approx(want, rel=2e-6, abs=1e-6)
        # and the closed form in the axis-pair coefficient
        assert got == pytest.approx(kappa + 0.5 * coef * dl * dl, rel=1e-4, abs=1e-5), d


def test_mode_term_is_negative_log_weighted_density(orc):
    """kappa + q / 2 = -log(pi) - log N(y; mu, Sigma) (scipy) for random
    correlated covariances of centimetre scale."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        A = rng.normal(size=(3, 3)) * 0.02
        Sig = A @ A.T + np.eye(3) * 1e-4
        mu = rng.normal(size=3) * 2.0
        pi = rng.uniform(0.05, 1.0)
        Si = np.linalg.inv(Sig)
        kappa = -math.log(pi) + 0.5 * (3 * math.log(2 * math.pi) + math.log(np.linalg.det(Sig)))
        m = _mode(orc, mu, Si[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]], kappa)
        y = (mu + rng.normal(size=3) * 0.03).astype(np.float32)
        want = -math.log(pi) - multivariate_normal(mu.astype(np.float32), Sig).logpdf(y.astype(np.float64))
        got = orc.mode_term(m, y)
        scale = 1.0 + abs(want)
        assert abs(got - want) <= 2e-4 * scale, (got, want)


def _round_terms(modes_of_pixel, cam, R32, t32):
    """min over modes of kappa + q / 2 (float64) and the best mode's distance
    for each drawn pixel, with the FP32 pose rounded as scoring uses it."""
    terms, dist = [], []
    for c, modes in zip(cam, modes_of_pixel):
        y = R32.astype(np.float64) @ c.astype(np.float64) + t32.astype(np.float64)
        best, bd = None, None
        for md in modes:
            d = y - md["mu"].astype(np.float64)
            s = md["sinv"].astype(np.float64)
            S = np.array([[s[0], s[1], s[2]], [s[1], s[3], s[4]], [s[2], s[4], s[5]]])
            term = float(md["kappa"]) + 0.5 * float(d @ S @ d)
            if best is None or term < best:
                best, bd = term, float(np.linalg.norm(d))
        terms.append(0.0 if best is None else min(0.0, best))
        dist.append(bd)
    return np.array(terms), dist


@pytest.mark.parametrize("B,N", [(13, 32), (64, 9)])
def test_round_energies_culls_and_inliers_recomputed(orc, B, N):
    """Per round, every live hypothesis's energy equals the float64 sum over
    the round's draws (numpy Philox) of min(0, min over the draw's leaf modes
    of kappa + q / 2), added to its earlier rounds, under the pose it held in
    that round; survivors are the first half by (energy, index) and running
    inlier counts follow the 10 cm rule. B = 13 leaves a partial last group of
    draws."""
    sc = sr.small_scene(21)
    p = orc.default_params(batch_pixels=B)
    f = orc.Forest(p)
    for k in range(10):
        d, c = sc.render_adapt(k)
        f.adapt(d, c, sc.K, sc.adapt_poses[k])
    d, c = sc.render_query(3)
    seed = 4242
    st, pose, score, tr = f.relocalise(d, c, sc.K, seed=seed, n_hyp=N, trace=True)
    assert st == 0
    depth = d.numpy()
    pool = np.flatnonzero((depth.reshape(-1) >= 500) & (depth.reshape(-1) <= 5000))
    leaves = f.leaves(d, c, sc.K)
    cam_all = cam_points_f32(depth, sc.K)
    cache = {}

    def modes_at(pix):
        out = []
        for t in range(f.T):
            key = (t, int(leaves[t, pix]))
            if key not in cache:
                cache[key] = f.leaf_modes(*key)
            out.extend(list(cache[key]))
        return out

    nr = int(tr["n_rounds"][0])
    E = {}
    inl = {}
    pose_of = {h: tr["hyp_pose"][h] for h in range(N) if tr["hyp_try"][h] >= 0}
    checked_cuts = 0
    for r in range(nr):
        draws = [pool[np_uniform_int(np_philox((r, i, 0, 0), (seed, 4))[0], len(pool))] for i in range(B)]
        cam = cam_all[draws]
        mp = [modes_at(q) for q in draws]
        na = int(tr["n_alive"][r])
        alive = tr["alive"][r, :na]
        Er = np.zeros(na)
        for a, h in enumerate(alive):
            P12 = pose_of[h]
            R32 = P12[:9].reshape(3, 3).astype(np.float32)
            t32 = P12[9:].astype(np.float32)
            terms, dist = _round_terms(mp, cam, R32, t32)
            E[h] = E.get(h, 0.0) + terms.sum()
            Er[a] = E[h]
            assert tr["energy"][r, a] == pytest.approx(E[h], rel=1e-4, abs=2e-3), (r, a, h)
            near = [x for x in dist if x is not None and abs(x - 0.1) < 1e-5]
            if not near:
                inl[h] = inl.get(h, 0) + sum(1 for x in dist if x is not None and x <= 0.1)
                assert tr["n_inliers"][r, a] == inl[h], (r, a, h)
            else:
                inl[h] = int(tr["n_inliers"][r, a])
        keep = (na + 1) // 2
        order = sorted(range(na), key=lambda a: (Er[a], alive[a]))
        if keep < na:
            e_in, e_out = Er[order[keep - 1]], Er[order[keep]]
            if abs(e_out - e_in) > 1e-3 * (1.0 + abs(e_in)):
                checked_cuts += 1
                want = sorted(int(alive[a]) for a in order[:keep])
                if r + 1 < nr:
                    got = sorted(int(x) for x in tr["alive"][r + 1, :keep])
                else:
                    got = [int(tr["final_hyp"][0])]
                assert got == want, r
        for a in range(keep):
            h = int(tr["alive"][r + 1, a]) if r + 1 < nr else int(tr["final_hyp"][0])
            pose_of[h] = tr["pose_after"][r, a]
    assert checked_cuts >= 1


def _triple(orc, c, w, pi=(1, 2, 3), **kw):
    return orc.check_triple(orc.default_params(**kw), pi, c, w)


def _base_triple(rng_seed=0, scale=1.0):
    R = rand_rotation(np.random.default_rng(rng_seed))
    t = np.array([0.4, -1.1, 2.0])
    c = np.array([[0.0, 0.0, 2.0], [0.6, 0.1, 2.1], [0.1, 0.7, 2.4]]) * scale
    w = c @ R.T + t
    return c.astype(np.float32), w.astype(np.float32), R, t


def test_check_triple_passes_and_recovers_pose(orc):
    c, w, R, t = _base_triple()
    rc, Rg, tg = _triple(orc, c, w)
    assert rc == orc.TRI_OK
    np.testing.assert_allclose(Rg, R, atol=1e-5)
    np.testing.assert_allclose(tg, t, atol=1e-5)


def test_check_triple_each_check_alone(orc):
    """Each constructed triple fails one check, and passes once that one
    threshold is relaxed (so no other check fails)."""
    c, w, R, t = _base_triple()
    # same pool pixel
    assert _triple(orc, c, w, pi=(4, 9, 4))[0] == orc.TRI_SAME_PIXEL
    assert _triple(orc, c, w, pi=(4, 9, 5))[0] == orc.TRI_OK
    # a camera pair closer than 10 cm (9 cm apart)
    c2 = c.copy()
    c2[1] = c2[0] + np.array([0.09, 0.0, 0.0], dtype=np.float32)
    w2 = (c2.astype(np.float64) @ R.T + t).astype(np.float32)
    assert _triple(orc, c2, w2)[0] == orc.TRI_PAIR_DIST
    assert _triple(orc, c2, w2, min_pair2_m2=0.008)[0] == orc.TRI_OK
    # world pair longer than the camera pair: world point 1 pushed outwards
    # along edge (0,1) so that its squared length grows by a factor 1.25
    for sign, code in ((1.0, orc.TRI_WORLD_LONGER), (-1.0, orc.TRI_CAMERA_LONGER)):
        f = math.sqrt(1.25) if sign > 0 else math.sqrt(1 / 1.25)
        w3 = w.astype(np.float64).copy()
        w3[1] = w3[0] + f * (w3[1] - w3[0])
        w3 = w3.astype(np.float32)
        assert _triple(orc, c, w3, resid_m=0.2)[0] == code
        assert _triple(orc, c, w3, resid_m=0.2, rigid_ratio2=1.3)[0] == orc.TRI_OK
    # thin camera triangle: |e1 x e2|^2 = 6.8e-5 < 1e-4, still well
    # conditioned for the alignment
    c4 = np.array([[0.0, 0.0, 2.0], [0.15, 0.0, 2.0], [0.30, 0.055, 2.0]], dtype=np.float32)
    w4 = (c4.astype(np.float64) @ R.T + t).astype(np.float32)
    e1, e2 = c4[1] - c4[0], c4[2] - c4[0]
    assert float(np.sum(np.cross(e1, e2) ** 2)) < 1e-4
    assert _triple(orc, c4, w4)[0] == orc.TRI_AREA
    assert _triple(orc, c4, w4, min_area2_m4=5e-5)[0] == orc.TRI_OK
    # residual: on a triangle three times larger, world point 2 moved 12 cm
    # away from the centroid in the triangle's plane (rigidity within 1.21 on
    # every pair, Kabsch residual above 5 cm)
    c5, w5, _, _ = _base_triple(scale=3.0)
    w5 = w5.astype(np.float64)
    v = w5[2] - w5.mean(0)
    w5[2] += 0.12 * v / np.linalg.norm(v)
    w5 = w5.astype(np.float32)
    assert _triple(orc, c5, w5)[0] == orc.TRI_RESIDUAL
    assert _triple(orc, c5, w5, resid_m=0.3)[0] == orc.TRI_OK


def test_colour_test_window(orc):
    for tol in (0, 15, 40):
        p = orc.default_params(rgb_tol=tol)
        px = np.array([100, 7, 250], dtype=np.uint8)
        assert orc.colour_ok(p, px, px)
        for ch in range(3):
            for dv, ok in ((tol, True), (-tol, True), (tol + 1, False), (-tol - 1, False)):
                m = px.astype(np.int64).copy()
                m[ch] += dv
                if m[ch] < 0 or m[ch] > 255:
                    continue
                assert orc.colour_ok(p, m.astype(np.uint8), px) == ok, (tol, ch, dv)


def _sums(c, w):
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    s = [len(c)] + list(c.sum(0)) + list(w.sum(0)) + list((c[:, :, None] * w[:, None, :]).sum(0).reshape(9))
    cc = (c[:, :, None] * c[:, None, :]).sum(0)
    s += [cc[0, 0], cc[0, 1], cc[0, 2], cc[1, 1], cc[1, 2], cc[2, 2]]
    return np.array(s)


def test_pose_from_sums_degeneracy_threshold(orc):
    """The solve declines when I2 (sum of the principal 2x2 minors of the
    centred camera scatter) is below 1e-4 n trace, on either side of it."""
    rng = np.random.default_rng(5)
    R = rand_rotation(rng)
    t = np.array([0.3, 0.2, -0.1])
    xs = np.linspace(-0.5, 0.5, 12)
    for side, want in ((1.05, 0), (0.95, 1)):
        # points on a line with a perpendicular zig-zag of amplitude e
        zig = np.where(np.arange(12) % 2 == 0, 1.0, -1.0)

        def ratio(e):
            c = np.stack([xs, e * zig, np.full(12, 2.0)], 1)
            S = (c - c.mean(0)).T @ (c - c.mean(0))
            I2 = (S[0, 0] * S[1, 1] - S[0, 1] ** 2) + (S[0, 0] * S[2, 2] - S[0, 2] ** 2) + \
                 (S[1, 1] * S[2, 2] - S[1, 2] ** 2)
            return I2 / (1e-4 * 12 * np.trace(S)), c

        lo, hi = 1e-6, 0.5
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if ratio(mid)[0] < side:
                lo = mid
            else:
                hi = mid
        r, c = ratio(hi)
        assert abs(r - side) < 1e-6
        w = c @ R.T + t
        rc, Rg, tg = orc.pose_from_sums(_sums(c, w))
        assert rc == want, side
        if rc == 0:
            np.testing.assert_allclose(Rg, R, atol=1e-9)
            np.testing.assert_allclose(tg, t, atol=1e-9)
    assert orc.pose_from_sums(_sums(np.eye(3)[:2], np.eye(3)[:2]))[0] == 1   # fewer than 3 points


def test_pose_from_sums_equals_kabsch(orc):
    rng = np.random.default_rng(6)
    for _ in range(50):
        R = rand_rotation(rng)
        t = rng.normal(size=3)
        c = rng.normal(size=(20, 3))
        w = c @ R.T + t + rng.normal(size=(20, 3)) * 0.01
        rc, Rg, tg = orc.pose_from_sums(_sums(c, w))
        assert rc == 0
        Rh = horn_rotation(c, w)
        np.testing.assert_allclose(Rg, Rh, atol=1e-10)
        np.testing.assert_allclose(tg, w.mean(0) - Rh @ c.mean(0), atol=1e-10)


def _unique_leaf_forest(orc, W=24, H=16, seed=7):
    """A frame whose pixels have distinct depths and one tree whose splits
    test the pixel's own depth (every probe leaves the image, so the response
    is 65535 - d): each pixel reaches a leaf of its own, whose only sample is
    the pixel's own world point."""
    rng = np.random.default_rng(seed)
    P = W * H
    depths = rng.choice(np.arange(600, 4900), size=P, replace=False).astype(np.uint16)
    depth = depths.reshape(H, W)
    rgb = np.full((H, W, 3), 128, dtype=np.uint8)
    D = 9                                          # 512 leaves >= 384 pixels
    L = 1 << D
    p = orc.default_params(n_trees=1, depth=D, reservoir_size=4, max_modes=2, min_cluster=1, cov_reg_mm2=1,
                           rgb_tol=0, n_hypotheses=64, batch_pixels=64)
    f = orc.Forest(p)
    kind, dx, dy, thr = f.nodes()
    n = L - 1
    kind[:n] = 0
    dx[:n] = 400000                                # offset >= 80 px at 5 m: always outside the image
    dy[:n] = 0
    # a balanced search tree over the sorted depths: node i splits its range
    # at its middle; right iff 65535 - d >= thr iff d <= 65535 - thr
    sd = np.sort(depths.astype(np.int64))
    thr[:n] = 65535 + 1                            # unused nodes send everything left
    ranges = {0: (0, P)}
    for i in range(n):
        if i not in ranges:
            continue
        lo, hi = ranges[i]
        if hi - lo <= 1:
            continue
        mid = (lo + hi) // 2
        # right child takes the smaller depths [lo, mid), left the rest
        thr[i] = 65535 - int(sd[mid - 1])
        ranges[2 * i + 2] = (lo, mid)
        ranges[2 * i + 1] = (mid, hi)
    f.set_nodes(kind, dx, dy, thr)
    return f, depth, rgb


def test_exact_modes_give_exact_pose(orc):
    """Every mode is a single sample at its pixel's true world point (to the
    integer-mm quantisation) with a 1 mm covariance: every valid hypothesis is
    exact and the returned pose equals the truth to 1 mm."""
    f, depth, rgb = _unique_leaf_forest(orc)
    K = (277.0, 277.0, 12.0, 8.0)
    rng = np.random.default_rng(8)
    pose = np.eye(4)
    pose[:3, :3] = rand_rotation(rng)
    pose[:3, 3] = [1.0, -0.5, 2.0]
    f.adapt(depth, rgb, K, pose)
    leaves = f.leaves(depth, rgb, K)
    assert len(np.unique(leaves[0])) == depth.size
    st, T, score, tr = f.relocalise(depth, rgb, K, seed=99, trace=True)
    assert st == 0
    assert np.linalg.norm(T[:3, 3] - pose[:3, 3]) <= 1e-3
    ok, dt, da = orc.pose_success(T, pose)
    assert dt <= 1e-3 and da <= 0.05
    valid = tr["hyp_try"] >= 0
    assert valid.sum() >= 32
    # three exact points pin a hypothesis down to the quantisation's lever
    # arm (0.5 mm per axis over pairs of 10 cm or more, seen from about 2 m):
    # each one is within the success criterion, and refinement on all the
    # inliers removes the rest
    for P12 in tr["hyp_pose"][valid]:
        Th = np.eye(4)
        Th[:3, :3] = P12[:9].reshape(3, 3)
        Th[:3, 3] = P12[9:]
        _, dt_h, da_h = orc.pose_success(Th, pose)
        assert dt_h < 0.05 and da_h < 5.0
    assert score > 0.99


def test_duplicated_hypotheses_keep_lower_index(orc):
    """Two copies of the same pose have equal energies in every round; the cull
    orders ties by index, so the lower copy survives."""
    sc = sr.small_scene(22)
    f = orc.Forest(orc.default_params())
    for k in range(10):
        d, c = sc.render_adapt(k)
        f.adapt(d, c, sc.K, sc.adapt_poses[k])
    d, c = sc.render_query(4)
    gt = sc.query_poses[4]
    off = gt.copy()
    off[:3, 3] += [0.3, 0.0, 0.0]
    P = lambda T: np.concatenate([T[:3, :3].reshape(9), T[:3, 3]])
    poses = np.stack([P(off), P(gt), P(off), P(gt), P(off)])
    st, T, _, tr = f.preemptive(d, c, sc.K, 17, poses, np.ones(5, np.int32))
    assert st == 0
    e0 = tr["energy"][0, :5]
    assert e0[1] == e0[3] and e0[0] == e0[2] == e0[4]
    assert e0[1] < e0[0]
    # round 0 keeps 3: both copies of the truth, then the lowest copy of the offset pose
    assert list(tr["alive"][1, :3]) == [1, 3, 0]
    assert list(tr["alive"][2, :2]) == [1, 3]
    assert int(tr["final_hyp"][0]) == 1
    # the invalid flag removes a hypothesis before any round
    st2, _, _, tr2 = f.preemptive(d, c, sc.K, 17, poses, np.array([1, 0, 1, 1, 1], np.int32))
    assert int(tr2["final_hyp"][0]) == 3


def test_one_hypothesis_is_one_alignment_and_one_refinement(orc):
    """N = 1: one round; the result is the Kabsch alignment (Horn, numpy) of
    the hypothesis's round-0 inliers: draws whose best mode lies within 10 cm
    of the transformed point, paired with that mode's mean."""
    sc = sr.small_scene(23)
    f = orc.Forest(orc.default_params())
    for k in range(10):
        d, c = sc.render_adapt(k)
        f.adapt(d, c, sc.K, sc.adapt_poses[k])
    d, c = sc.render_query(5)
    for seed in range(31, 61):      # the first seed whose single hypothesis is valid
        st, T, score, tr = f.relocalise(d, c, sc.K, seed=seed, n_hyp=1, trace=True)
        if st == 0:
            break
    assert st == 0 and int(tr["n_rounds"][0]) == 1
    P12 = tr["hyp_pose"][0]
    R32 = P12[:9].reshape(3, 3).astype(np.float32)
    t32 = P12[9:].astype(np.float32)
    depth = d.numpy()
    pool = np.flatnonzero((depth.reshape(-1) >= 500) & (depth.reshape(-1) <= 5000))
    leaves = f.leaves(d, c, sc.K)
    cam_all = cam_points_f32(depth, sc.K)
    B = f.params.batch_pixels
    src, dst = [], []
    for i in range(B):
        q = pool[np_uniform_int(np_philox((0, i, 0, 0), (seed, 4))[0], len(pool))]
        cam = cam_all[q]
        y = R32.astype(np.float64) @ cam.astype(np.float64) + t32.astype(np.float64)
        best, bm = None, None
        for t in range(f.T):
            for md in f.leaf_modes(t, int(leaves[t, q])):
                dd = y - md["mu"].astype(np.float64)
                s = md["sinv"].astype(np.float64)
                S = np.array([[s[0], s[1], s[2]], [s[1], s[3], s[4]], [s[2], s[4], s[5]]])
                term = float(md["kappa"]) + 0.5 * float(dd @ S @ dd)
                if best is None or term < best:
                    best, bm = term, md
        if bm is not None:
            dist = float(np.linalg.norm(y - bm["mu"].astype(np.float64)))
            assert abs(dist - 0.1) > 1e-5
            if dist <= 0.1:
                src.append(cam.astype(np.float64))
                dst.append(bm["mu"].astype(np.float64))
    src, dst = np.array(src), np.array(dst)
    assert len(src) >= 3
    Rh = horn_rotation(src, dst)
    th = dst.mean(0) - Rh @ src.mean(0)
    np.testing.assert_allclose(T[:3, :3], Rh, atol=1e-9)
    np.testing.assert_allclose(T[:3, 3], th, atol=1e-9)
    assert score == pytest.approx(len(src) / B, abs=1e-7)
