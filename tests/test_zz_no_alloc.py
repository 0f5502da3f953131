"""GPU: the allocation-free verifier (reloc_verify_noalloc) called through the
C ABI returns what reloc_verify returns, on two calls in a row, the second on
a smaller frame, so that the second call reads partials of its own and never
the larger first call's leftovers."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_util import banner, need_gpu

pytestmark = pytest.mark.gpu


def _call(fn, a, b):
    import torch
    H, W = a.shape
    vf, mu, acc = C.c_double(0), C.c_double(0), C.c_int32(0)
    rc = fn(a.data_ptr(), b.data_ptr(), W, H, C.byref(vf), C.byref(mu), C.byref(acc),
            torch.cuda.current_stream().cuda_stream)
    assert rc == 0, rc
    return vf.value, mu.value, acc.value


@pytest.mark.parametrize("offset", [0, 3])
def test_noalloc_verify_equals_verify(offset):
    dev = need_gpu()
    import torch
    import paper_1801_08361_amd as rl
    L = rl.lib()
    rng = np.random.default_rng(11 + offset)
    for step, (H, W) in enumerate(((1200, 1600), (240, 321))):   # large first, then smaller
        a = rng.integers(0, 6000, size=(H, W)).astype(np.uint16)
        b = np.where(rng.random((H, W)) < 0.3, 0, a.astype(np.int64) + rng.integers(-30, 30, size=(H, W)))
        b = np.clip(b, 0, 65535).astype(np.uint16)
        ta = torch.zeros(H * W + offset, dtype=torch.uint16, device=dev)
        tb = torch.zeros(H * W + offset, dtype=torch.uint16, device=dev)
        ta[offset:] = torch.from_numpy(a.reshape(-1)).to(dev)
        tb[offset:] = torch.from_numpy(b.reshape(-1)).to(dev)
        va, vb = ta[offset:].view(H, W), tb[offset:].view(H, W)
        banner(f"noalloc verify step {step} {H}x{W} offset {offset}")
        want = _call(L.reloc_verify, va, vb)
        got = _call(L.reloc_verify_noalloc, va, vb)
        assert got == want, (step, got, want)
        assert 0.0 < got[0] <= 1.0 and np.isfinite(got[1])


def test_noalloc_verify_argument_errors():
    need_gpu()
    import paper_1801_08361_amd as rl
    L = rl.lib()
    assert L.reloc_verify_noalloc(None, None, 4, 4, None, None, None, None) == rl.E_ARG
    x = C.c_double(0)
    acc = C.c_int32(0)
    assert L.reloc_verify_noalloc(1, 1, 8192, 4, C.byref(x), C.byref(x), C.byref(acc), None) == rl.E_ARG
