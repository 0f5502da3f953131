"""Pins of the leaf-mode finder and the Gaussian energy: separated blobs give
one mode each with the exact mean and covariance; the pruned search equals the
plain double loop; the density tie rule is the documented one; and kappa +
q / 2 equals -log(pi) minus scipy's Gaussian log-density."""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import ENTRY_DTYPE


def pts_from(xyz, rgb=None):
    a = np.zeros(len(xyz), dtype=ENTRY_DTYPE)
    a["x"], a["y"], a["z"] = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    if rgb is not None:
        a["r"], a["g"], a["b"] = rgb[:, 0], rgb[:, 1], rgb[:, 2]
    return a


def blobs(rng, centres, sizes, spread=20):
    xyz, lab = [], []
    for i, (c, n) in enumerate(zip(centres, sizes)):
        xyz.append(np.asarray(c) + rng.integers(-spread, spread + 1, size=(n, 3)))
        lab += [i] * n
    return np.concatenate(xyz).astype(np.int64), np.array(lab)


def expected_stats(xyz, n_total, reg=100):
    n = len(xyz)
    mu = xyz.mean(0) / 1000.0
    C = np.cov(xyz.T.astype(np.float64), bias=True) + reg * np.eye(3)
    S = C * 1e-6
    kappa = -np.log(n / n_total) + 0.5 * (3 * np.log(2 * np.pi) + np.log(np.linalg.det(S)))
    return mu, S, kappa


def test_blobs_give_exact_modes(orc):
    rng = np.random.default_rng(1)
    centres = [(1000, 2000, 500), (3000, 500, 1500), (-2000, 0, 800), (0, 0, 0)]
    sizes = [40, 25, 60, 2]                 # the 2-point blob is below the minimum size
    xyz, lab = blobs(rng, centres, sizes)
    perm = rng.permutation(len(xyz))
    xyz, lab = xyz[perm], lab[perm]
    rgb = rng.integers(0, 256, size=(len(xyz), 3))
    p = orc.default_params(reservoir_size=256, max_modes=10)
    modes, labels = orc.modes_from_points(p, pts_from(xyz, rgb))
    assert len(modes) == 3
    order = [2, 0, 1]                       # by size: 60, 40, 25
    for m, b in enumerate(order):
        sel = lab == b
        assert modes[m]["n"] == sizes[b]
        assert np.all(labels[sel] == m)
        mu, S, kappa = expected_stats(xyz[sel], len(xyz))
        np.testing.assert_allclose(modes[m]["mu"], mu, rtol=0, atol=1e-6)
        np.testing.assert_allclose(modes[m]["sinv"][[0, 1, 2, 3, 4, 5]],
                                   np.linalg.inv(S)[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]], rtol=2e-6)
        assert modes[m]["kappa"] == pytest.approx(kappa, rel=1e-6, abs=1e-5)
        assert np.array_equal(modes[m]["rgb"], rgb[sel].sum(0) // sizes[b])
    assert np.all(labels[lab == 3] == -1)


def test_max_modes_and_min_size(orc):
    rng = np.random.default_rng(2)
    centres = [(i * 1000, 0, 0) for i in range(6)]
    sizes = [10, 12, 14, 16, 18, 3]
    xyz, lab = blobs(rng, centres, sizes, spread=10)
    p = orc.default_params(reservoir_size=256, max_modes=3)
    modes, labels = orc.modes_from_points(p, pts_from(xyz))
    assert [int(m["n"]) for m in modes] == [18, 16, 14]
    p = orc.default_params(reservoir_size=256, max_modes=10, min_cluster=13)
    modes, _ = orc.modes_from_points(p, pts_from(xyz))
    assert [int(m["n"]) for m in modes] == [18, 16, 14]
    # default minimum is max(3, R / 64): R = 1024 -> 16
    p = orc.default_params(reservoir_size=1024, max_modes=10)
    modes, _ = orc.modes_from_points(p, pts_from(xyz))
    assert [int(m["n"]) for m in modes] == [18, 16]


def test_density_tie_rule(orc):
    """Two points 80 mm apart: each has density 1 (radius 50), they are within
    the 100 mm link radius, and on equal density the lower index is denser, so
    point 1 links to point 0 and point 0 is the root."""
    xyz = np.array([[0, 0, 0], [80, 0, 0], [5000, 0, 0]])
    p = orc.default_params(min_cluster=1, max_modes=10)
    modes, labels = orc.modes_from_points(p, pts_from(xyz))
    assert list(labels) == [0, 0, 1]
    assert [int(m["n"]) for m in modes] == [2, 1]
    # same size clusters order by root index
    xyz = np.array([[5000, 0, 0], [0, 0, 0]])
    modes, labels = orc.modes_from_points(p, pts_from(xyz))
    assert list(labels) == [0, 1]
    assert modes[0]["mu"][0] == pytest.approx(5.0)


@pytest.mark.parametrize("seed", range(6))
def test_pruned_search_equals_bruteforce(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 400))
    # a coarse grid makes exact distance and density ties common
    xyz = rng.integers(0, 12, size=(n, 3)) * 25
    if seed % 2:
        xyz[: n // 2] += 2000
    p = orc.default_params(reservoir_size=256, max_modes=8, min_cluster=1 + seed % 4)
    a, la = orc.modes_from_points(p, pts_from(xyz))
    b, lb = orc.modes_from_points(p, pts_from(xyz), brute=True)
    assert np.array_equal(la, lb)
    assert a.tobytes() == b.tobytes()


def test_energy_is_gaussian_negative_log_likelihood(orc):
    rng = np.random.default_rng(4)
    xyz, lab = blobs(rng, [(1500, -700, 900), (4000, 4000, 100)], [50, 30], spread=35)
    p = orc.default_params(reservoir_size=256)
    modes, labels = orc.modes_from_points(p, pts_from(xyz))
    for mi, m in enumerate(modes):
        sel = labels == mi
        mu, S, _ = expected_stats(xyz[sel], len(xyz))
        pi = m["n"] / len(xyz)
        Sinv = np.zeros((3, 3))
        iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
        for k, (a, b) in enumerate(iu):
            Sinv[a, b] = Sinv[b, a] = m["sinv"][k]
        for _ in range(20):
            y = m["mu"].astype(np.float64) + rng.normal(scale=0.03, size=3)
            d = y - m["mu"].astype(np.float64)
            ours = float(m["kappa"]) + 0.5 * d @ Sinv @ d
            ref = -np.log(pi) - multivariate_normal.logpdf(y, mean=mu, cov=S)
            assert ours == pytest.approx(ref, rel=1e-5, abs=1e-4)


def test_empty_and_tiny_inputs(orc):
    p = orc.default_params()
    modes, labels = orc.modes_from_points(p, pts_from(np.zeros((0, 3), dtype=np.int64)))
    assert len(modes) == 0
    modes, labels = orc.modes_from_points(p, pts_from(np.array([[1, 2, 3], [1, 2, 3]])))
    assert len(modes) == 0 and list(labels) == [-1, -1]
    # three coincident points (minimum size max(3, 64 / 64) = 3): one mode whose
    # covariance is the regulariser alone
    p = orc.default_params(reservoir_size=64)
    modes, labels = orc.modes_from_points(p, pts_from(np.array([[1, 2, 3]] * 3)))
    assert len(modes) == 1
    np.testing.assert_allclose(modes[0]["sinv"], [1e4, 0, 0, 1e4, 0, 1e4], rtol=1e-6)
