"""CPU checks of the C ABI boundary: the built library loads, exports every
function include/reloc.h declares, its structs have the layout the header
implies, and argument errors come back as status codes (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "reloc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(reloc_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    import paper_1801_08361_amd as rl
    L = rl.lib()
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding wraps each of them
    assert set(names) <= set(rl._SIGS), set(names) - set(rl._SIGS)


def test_struct_layouts():
    import paper_1801_08361_amd as rl
    assert C.sizeof(rl.reloc_intrinsics) == 24
    assert C.sizeof(rl.reloc_result) == 168
    assert C.sizeof(rl.reloc_attempt) == 80
    assert C.sizeof(rl.reloc_params) == 4 * 4 + 8 + 4 * 15 + 4 * 5
    assert rl.ENTRY_DTYPE.itemsize == 16 and rl.MODE_DTYPE.itemsize == 48


def test_defaults_match_the_oracle():
    import oracle
    import paper_1801_08361_amd as rl
    from tests.gpu_util import FIELDS
    a = rl.params_default()
    b = oracle.default_params()
    for f in FIELDS:
        assert getattr(a, f) == getattr(b, f), f


def test_argument_errors_without_gpu():
    import paper_1801_08361_amd as rl
    L = rl.lib()
    assert L.reloc_params_default(None) == rl.E_ARG
    out = C.c_void_p()
    assert L.reloc_forest_create(None, None, C.byref(out)) == rl.E_ARG
    p = rl.params_default(depth=0)
    assert L.reloc_forest_create(C.byref(p), None, C.byref(out)) == rl.E_ARG
    p = rl.params_default(offset_pxmm=1 << 21)
    assert L.reloc_forest_create(C.byref(p), None, C.byref(out)) == rl.E_RANGE
    p = rl.params_default(cov_reg_mm2=0)
    assert L.reloc_forest_create(C.byref(p), None, C.byref(out)) == rl.E_ARG
    assert L.reloc_forest_destroy(None) == rl.E_ARG
    assert L.reloc_relocalise(None, None, None, None, 0, 0, None, None, None, None) == rl.E_ARG
    assert L.reloc_relocalise_batch(None, None, 0, None, None) == rl.E_ARG
    assert L.reloc_batch_destroy(None) == rl.E_ARG
    assert L.reloc_verify(None, None, 4, 4, None, None, None, None) == rl.E_ARG
    p = rl.params_default(max_modes=65)
    assert L.reloc_forest_create(C.byref(p), None, C.byref(out)) == rl.E_ARG
    p = rl.params_default(n_trees=16, max_modes=40)          # 640 modes per pixel > 512
    assert L.reloc_forest_create(C.byref(p), None, C.byref(out)) == rl.E_ARG
    assert L.reloc_forest_save(None, b"/tmp/x", None) == rl.E_ARG
    assert L.reloc_forest_load(None, None, C.byref(out)) == rl.E_ARG
    assert L.reloc_forest_params(None, None) == rl.E_ARG
    assert L.reloc_forest_train(None, None, 1, 1, 1, None) == rl.E_ARG
    assert L.reloc_mlp_create(0, None, None) == rl.E_ARG
    assert L.reloc_mlp_destroy(None) == rl.E_ARG
    assert L.reloc_mlp_gradient(None, None, None, 1, None, None, None) == rl.E_ARG
    assert L.reloc_mlp_train(None, None, None, 1, 1, 1, C.c_float(1e-3), 0, None, None) == rl.E_ARG
    assert L.reloc_mlp_logits(None, None, 1, None, None) == rl.E_ARG
    assert L.reloc_mlp_pixel_weights(None, None, None, None, None, None, None, None) == rl.E_ARG
    assert L.reloc_pixel_features(None, None, None, None, None, 0, None, None, None) == rl.E_ARG
    assert L.reloc_pixel_features(None, None, None, None, None, -1, None, None, None) == rl.E_ARG
    assert L.reloc_label_pixels(None, None, None, None, None, None, 0, None, None) == rl.E_ARG
    assert L.reloc_debug_mfma_probe(None, None, None) == rl.E_ARG
    assert L.reloc_debug_lane_probe(None) == rl.E_ARG
    assert L.reloc_valid_pixels(None, None, None, None, None, None, None) == rl.E_ARG
    assert L.reloc_relocalise_learned(None, None, None, None, None, 0, 0, None, None) == rl.E_ARG
    for code in (0, 1, 2, 3, -1, -2, -3, -4, -5, 99):
        assert isinstance(rl.status_string(code), str)
    with pytest.raises(rl.RelocError):
        rl._check(-1, "x")


@pytest.mark.parametrize("xcd", [0, 1])
def test_every_work_unit_has_exactly_one_owner(xcd):
    """The persistent kernels' unit ownership (run here on the host): every
    unit is processed by exactly one workgroup for any grid, including grids
    that are not a multiple of 8 under the XCD-contiguous order (a grid of 14
    once gave two owners to some units)."""
    import paper_1801_08361_amd as rl
    for total in (0, 1, 5, 7, 8, 9, 14, 63, 64, 65, 1000, 4097):
        for grid in (1, 2, 3, 7, 8, 9, 14, 16, 24, 64, 256, 1000, 2048, 4096, 5000):
            own = rl.unit_owners(xcd, total, grid)
            assert np.all(own == 1), (xcd, total, grid, own)


def test_no_cpu_fallback_when_library_missing(tmp_path, monkeypatch):
    import paper_1801_08361_amd as rl
    monkeypatch.setattr(rl, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(rl, "_lib", None)
    with pytest.raises(RuntimeError):
        rl.lib()


def test_checkpoint_file_errors_without_gpu(tmp_path):
    """Files that are missing, empty, truncated or not checkpoints are
    rejected with RELOC_E_IO before any device work."""
    import paper_1801_08361_amd as rl
    L = rl.lib()
    out = C.c_void_p()
    assert L.reloc_forest_load(str(tmp_path / "missing.bin").encode(), None, C.byref(out)) == rl.E_IO
    empty = tmp_path / "empty.bin"
    empty.write_bytes(b"")
    assert L.reloc_forest_load(str(empty).encode(), None, C.byref(out)) == rl.E_IO
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"NOTAFORESTFILE" * 64)
    assert L.reloc_forest_load(str(junk).encode(), None, C.byref(out)) == rl.E_IO
    assert out.value is None
