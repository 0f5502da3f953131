"""Helpers for the GPU parity tests: parameter mirroring between the product's
reloc_params and the oracle's params, device frames, and a case banner that
is printed and flushed before every GPU step so a failing run names its case."""
from __future__ import annotations

import sys

import numpy as np
import pytest

FIELDS = ["n_trees", "depth", "reservoir_size", "max_modes", "seed", "depth_min_mm", "depth_max_mm",
          "offset_pxmm", "f_ref_px16", "thr_depth_mm", "thr_rgb", "dens_radius_mm", "link_radius_mm",
          "min_cluster", "cov_reg_mm2", "n_hypotheses", "batch_pixels", "max_tries", "refine", "rgb_tol",
          "rigid_ratio2", "min_pair2_m2", "min_area2_m4", "resid_m", "inlier_m"]

SMALL = dict(n_trees=5, depth=10, reservoir_size=256, max_modes=10, n_hypotheses=256, batch_pixels=64)
FULL = dict(n_trees=5, depth=15, reservoir_size=1024, max_modes=10, n_hypotheses=1024, batch_pixels=500)


def banner(msg: str) -> None:
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def pair(**kw):
    """(product params, oracle params) with identical values."""
    import oracle
    import paper_1801_08361_amd as rl
    pp = rl.params_default(**kw)
    po = oracle.default_params()
    for f in FIELDS:
        setattr(po, f, getattr(pp, f))
    return pp, po


def to_dev(depth, rgb, dev):
    import torch
    d = depth if isinstance(depth, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(depth))
    c = rgb if isinstance(rgb, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(rgb))
    return d.to(dev).contiguous(), c.to(dev).contiguous()


def rot_angle_deg(Ra: np.ndarray, Rb: np.ndarray) -> float:
    Q = Ra.T @ Rb
    v = np.array([Q[2, 1] - Q[1, 2], Q[0, 2] - Q[2, 0], Q[1, 0] - Q[0, 1]])
    return float(np.degrees(np.arctan2(0.5 * np.linalg.norm(v), 0.5 * (np.trace(Q) - 1.0))))


def assert_modes_equal(mg, mo):
    """GPU modes against the oracle's: counts, means, inverse covariances and
    colours bit for bit; kappa (a logarithm) to 1e-6."""
    assert len(mg) == len(mo)
    if len(mo) == 0:
        return
    assert np.array_equal(mg["n"], mo["n"])
    assert np.array_equal(mg["mu"].view(np.uint32), mo["mu"].view(np.uint32))
    assert np.array_equal(mg["sinv"].view(np.uint32), mo["sinv"].view(np.uint32))
    np.testing.assert_allclose(mg["kappa"], mo["kappa"], rtol=1e-6, atol=1e-6)
    assert np.array_equal(mg["rgb"], mo["rgb"])
