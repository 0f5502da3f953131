"""GPU: the depth-difference check (Sec. 3.3.1, Eqs. 3-4) against the oracle
on images that take each path of the kernel: 16-byte aligned images (eight
pixels per load) with and without a tail of fewer than eight pixels,
misaligned images (one pixel at a time), and an image large enough that the
partial pass is capped at its maximum grid and loops."""
import numpy as np
import pytest

from tests.gpu_util import banner, need_gpu

pytestmark = pytest.mark.gpu


def _pair(rng, H, W, invalid=0.2, noise=40):
    a = rng.integers(0, 65535, size=(H, W)).astype(np.uint16)
    b = np.where(rng.random((H, W)) < invalid, 0, a.astype(np.int64) + rng.integers(-noise, noise, size=(H, W)))
    return a, np.clip(b, 0, 65535).astype(np.uint16)


def _check(dev, a, b, offset=0):
    import torch
    import oracle
    import paper_1801_08361_amd as rl
    H, W = a.shape
    if offset:
        # views that start `offset` elements into a larger buffer (not 16-byte aligned)
        ba = torch.zeros(H * W + offset, dtype=torch.uint16, device=dev)
        bb = torch.zeros(H * W + offset, dtype=torch.uint16, device=dev)
        ba[offset:] = torch.from_numpy(a.reshape(-1)).to(dev)
        bb[offset:] = torch.from_numpy(b.reshape(-1)).to(dev)
        ta, tb = ba[offset:].view(H, W), bb[offset:].view(H, W)
        assert ta.data_ptr() % 16 != 0
    else:
        ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    got = rl.verify(ta, tb)
    ref = oracle.verify(a, b)
    assert got[0] == ref[0] and got[2] == ref[2], (got, ref)
    assert got[1] == ref[1] or (np.isinf(got[1]) and np.isinf(ref[1])), (got, ref)


@pytest.mark.parametrize("H,W,offset", [(480, 640, 0), (61, 97, 0), (61, 97, 1), (480, 640, 3), (1, 7, 0),
                                        (2304, 2048, 0), (2304, 2047, 5)])
def test_verify_paths_match_oracle(H, W, offset):
    dev = need_gpu()
    rng = np.random.default_rng(H * 7 + W + offset)
    a, b = _pair(rng, H, W)
    banner(f"verify {H}x{W} offset {offset}")
    _check(dev, a, b, offset)


def test_verify_degenerate_images():
    dev = need_gpu()
    z = np.zeros((48, 64), np.uint16)
    o = np.full((48, 64), 1234, np.uint16)
    banner("verify degenerate images")
    _check(dev, z, z)        # nothing valid: fraction 0, mean +inf
    _check(dev, o, z)        # query empty: mean +inf
    _check(dev, z, o)
    _check(dev, o, o)        # identical: mean 0, accepted
