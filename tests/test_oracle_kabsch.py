"""Pins of the FP64 rigid alignment: exact recovery of random rigid motions
from noise-free correspondences, agreement with Horn's quaternion method and
scipy's Rotation.align_vectors, SE(3) invariants, the reflection case, and the
3x3 SVD against numpy's LAPACK SVD."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from tests.oracle_util import horn_rotation, rand_rotation


@pytest.mark.parametrize("n", [3, 4, 10, 200])
def test_noise_free_recovery(orc, n):
    rng = np.random.default_rng(n)
    for _ in range(50):
        R = rand_rotation(rng)
        t = rng.normal(scale=3.0, size=3)
        src = rng.normal(scale=1.5, size=(n, 3))
        dst = src @ R.T + t
        rc, Re, te = orc.kabsch(src, dst)
        assert rc == 0
        assert np.abs(Re - R).max() < 1e-12
        assert np.abs(te - t).max() < 1e-12
        assert np.linalg.det(Re) == pytest.approx(1.0, abs=1e-12)
        assert np.abs(Re.T @ Re - np.eye(3)).max() < 1e-12


def test_matches_horn_and_scipy_with_noise(orc):
    rng = np.random.default_rng(9)
    for _ in range(100):
        n = int(rng.integers(3, 40))
        R = rand_rotation(rng)
        src = rng.normal(size=(n, 3))
        dst = src @ R.T + rng.normal(scale=0.05, size=(n, 3)) + rng.normal(size=3)
        rc, Re, te = orc.kabsch(src, dst)
        assert rc == 0
        Rh = horn_rotation(src, dst)
        assert np.abs(Re - Rh).max() < 1e-9
        rot, _ = Rotation.align_vectors(dst - dst.mean(0), src - src.mean(0))
        assert np.abs(Re - rot.as_matrix()).max() < 1e-9
        np.testing.assert_allclose(te, dst.mean(0) - Re @ src.mean(0), atol=1e-12)


def test_reflection_case(orc):
    """Noisy, nearly coplanar sets: the unconstrained orthogonal Procrustes
    solution is often a reflection; Kabsch must still return det = +1 and agree
    with Horn's method (which only ever returns rotations)."""
    rng = np.random.default_rng(11)
    seen_reflection = 0
    for _ in range(200):
        n = 6
        src = np.c_[rng.normal(size=(n, 2)), 1e-4 * rng.normal(size=n)]
        R = rand_rotation(rng)
        dst = src @ R.T + rng.normal(scale=0.3, size=(n, 3))
        a, b = src - src.mean(0), dst - dst.mean(0)
        U, S, Vt = np.linalg.svd(a.T @ b)
        if np.linalg.det(Vt.T @ U.T) < 0:
            seen_reflection += 1
        rc, Re, _ = orc.kabsch(src, dst)
        assert rc == 0
        assert np.linalg.det(Re) == pytest.approx(1.0, abs=1e-10)
        assert np.abs(Re - horn_rotation(src, dst)).max() < 1e-7
    assert seen_reflection > 10


def test_three_points_rank_two(orc):
    """Three centred points span a plane, so the cross-covariance has rank 2;
    the rotation is still unique and exact."""
    rng = np.random.default_rng(12)
    for _ in range(100):
        R = rand_rotation(rng)
        src = rng.normal(size=(3, 3))
        dst = src @ R.T + rng.normal(size=3)
        rc, Re, _ = orc.kabsch(src, dst)
        assert rc == 0 and np.abs(Re - R).max() < 1e-10


def test_degenerate_collinear_rejected(orc):
    src = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [3, 0, 0]])
    rc, _, _ = orc.kabsch(src, src + 1.0)
    assert rc == 1


def test_svd3_against_lapack(orc):
    rng = np.random.default_rng(13)
    for _ in range(200):
        A = rng.normal(size=(3, 3))
        if _ % 3 == 0:
            A[:, 2] = A[:, 0] * 0.5 - A[:, 1]          # rank 2
        rc, U, S, V = orc.svd3(A)
        assert rc == 0
        np.testing.assert_allclose(S, np.linalg.svd(A, compute_uv=False), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(U @ np.diag(S) @ V.T, A, atol=1e-12)
        np.testing.assert_allclose(U.T @ U, np.eye(3), atol=1e-10)
        np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-12)
