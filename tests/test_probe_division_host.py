"""The kernels' probe-offset division (a multiply-high by a per-pixel
multiplier instead of a divide) against exact integer truncation, on the host
build of the same functions. The offset of a split's depth-adaptive feature
(this library's definition; the paper leaves the features to the relocaliser
it adopts) is trunc(delta F / (d F_ref)); numerators stay below 2^31 in magnitude and the
divisor d F_ref is at least 1."""
import numpy as np
import pytest

import paper_1801_08361_amd as rl


def trunc_div(n, d):
    q = abs(n) // d
    return -q if n < 0 else q


def check(ns, ds):
    ns = np.asarray(ns, dtype=np.int64)
    ds = np.asarray(ds, dtype=np.int64)
    q = rl.probe_div(ns.astype(np.int32), ds.astype(np.int32))
    want = np.array([trunc_div(int(a), int(b)) for a, b in zip(ns, ds)], dtype=np.int64)
    bad = np.nonzero(q.astype(np.int64) != want)[0]
    assert bad.size == 0, [(int(ns[i]), int(ds[i]), int(q[i]), int(want[i])) for i in bad[:5]]


def edge_divisors():
    ds = {1, 2, 3, 5, 7, 500 * 4432, 5000 * 4432, 2 ** 31 - 1, 2 ** 31 - 2, 2 ** 30 + 1}
    for k in range(31):
        for e in (-1, 0, 1):
            v = 2 ** k + e
            if 1 <= v < 2 ** 31:
                ds.add(v)
    return sorted(ds)


def test_edges_of_every_divisor():
    top = 2 ** 31 - 1
    ns, ds = [], []
    for d in edge_divisors():
        cand = {0, 1, top, d - 1, d, d + 1, 2 * d - 1, 2 * d, top - top % d, top - top % d - 1}
        for q in (3, 1000, top // d):
            cand.update({q * d - 1, q * d, q * d + 1})
        for n in cand:
            if 0 <= n <= top:
                ns += [n, -n]
                ds += [d, d]
    check(ns, ds)


def test_random_numerators_and_divisors():
    rng = np.random.default_rng(7)
    # divisors of the shape d F_ref (valid depth in mm times a focal length in 1/16 px) and arbitrary ones
    d1 = rng.integers(500, 5001, 20000) * rng.integers(1, 20000, 20000)
    d1 = np.minimum(d1, 2 ** 31 - 1)
    d2 = np.exp(rng.uniform(0, np.log(2 ** 31 - 1), 20000)).astype(np.int64).clip(1, 2 ** 31 - 1)
    ds = np.concatenate([d1, d2])
    ns = rng.integers(-(2 ** 31 - 1), 2 ** 31, ds.size)
    # numerators next to multiples of the divisor, where a rounding slip shows
    near = (rng.integers(0, 2 ** 31 - 1, ds.size) // ds) * ds + rng.integers(-1, 2, ds.size)
    near = np.clip(near, -(2 ** 31 - 1), 2 ** 31 - 1) * np.where(rng.random(ds.size) < 0.5, -1, 1)
    check(np.concatenate([ns, near]), np.concatenate([ds, ds]))


def test_small_range_exhaustive():
    n = np.arange(-3000, 3001)
    for d in range(1, 130):
        check(n, np.full(n.shape, d))


def test_rejects_out_of_range():
    with pytest.raises(rl.RelocError):
        rl.probe_div(np.array([5], np.int32), np.array([0], np.int32))
    with pytest.raises(rl.RelocError):
        rl.probe_div(np.array([-2 ** 31], np.int32), np.array([3], np.int32))
