"""Pins of back-projection, the depth-adaptive features and traversal:
hand-computed responses on a tiny 8x6 image, and traversal special cases whose
leaves are known in closed form."""
import numpy as np
import pytest

from tests.oracle_util import cam_points_f32

I32_MIN = -(1 << 31)
I32_MAX = (1 << 31) - 1
W, H = 8, 6
K_REF = (277.0, 277.0, 4.0, 3.0)       # F = round(277 * 16) = F_ref: offset = trunc(delta / d)


def tiny_forest(orc, depth=2, T=1):
    p = orc.default_params(n_trees=T, depth=depth, reservoir_size=4)
    return orc.Forest(p)


def set_extra(f, nodes):
    """nodes: list of up to 8 (kind, dx, dy, thr) for the 8 extra feature nodes"""
    kind, dx, dy, thr = f.nodes()
    base = f.T * (f.L - 1)
    for j, (k, x, y, t) in enumerate(nodes):
        kind[base + j], dx[base + j], dy[base + j], thr[base + j] = k, x, y, t
    f.set_nodes(kind, dx, dy, thr)


def image():
    depth = np.full((H, W), 1000, dtype=np.uint16)
    depth[2, 3] = 2000
    depth[2, 2] = 0          # invalid
    depth[0, 7] = 6000       # beyond the 5 m limit: invalid
    rgb = np.zeros((H, W, 3), dtype=np.uint8)
    for v in range(H):
        for u in range(W):
            rgb[v, u] = (10 * u + v, 5 * v + 2 * u, (u * v) % 251)
    return depth, rgb


def test_feature_values_by_hand(orc):
    f = tiny_forest(orc)
    depth, rgb = image()
    set_extra(f, [
        (0, -1300, 0, 0),      # 0: offset trunc(-1.3) = -1 (toward zero, not -2)
        (0, -5000, 0, 0),      # 1: 5 px left
        (0, 0, 1000, 0),       # 2: 1 px down
        (1, 5000, 0, 0),       # 3: red, 5 px right (clamped at the border)
        (3, -1999, -1999, 0),  # 4: blue, trunc(-1.999) = -1 in x and y
        (2, 0, 0, 0),          # 5: green, no offset -> 0
        (0, 1000, 0, 0),       # 6: 1 px right
        (0, 2600, 0, 0),       # 7: trunc(2.6) = 2 px right
    ])
    F = f.features8(depth, rgb, K_REF).reshape(H, W, 8)
    # node 0 at (4, 2), d = 1000: probe (3, 2) has depth 2000
    assert F[2, 4, 0] == 2000 - 1000
    # node 0 at (3, 2), d = 2000: offset trunc(-1300 / 2000) = 0 -> probe itself
    assert F[2, 3, 0] == 0
    # node 0 at (3, 3), d = 1000: probe (2, 3) valid 1000 -> 0
    assert F[3, 3, 0] == 0
    # node 0 at (3, 2) already checked; at (0, 0): probe (-1, 0) is outside -> 65535 sentinel
    assert F[0, 0, 0] == 65535 - 1000
    # node 1 at (4, 0): probe (-1, 0) outside -> sentinel; at (6, 4): probe (1, 4) -> 0
    assert F[0, 4, 1] == 65535 - 1000
    assert F[4, 6, 1] == 0
    # node 2 at (2, 1): probe (2, 2) is invalid depth -> sentinel
    assert F[1, 2, 2] == 65535 - 1000
    # node 2 at (2, 5): probe (2, 6) outside -> sentinel
    assert F[5, 2, 2] == 65535 - 1000
    # node 6 at (6, 0): probe (7, 0) holds 6000 mm, outside the valid range -> sentinel
    assert F[0, 6, 6] == 65535 - 1000
    # node 3 (red channel) at (5, 1): probe (10, 1) clamps to (7, 1)
    assert F[1, 5, 3] == int(rgb[1, 7, 0]) - int(rgb[1, 5, 0])
    # node 4 (blue) at (4, 4): probe (3, 3)
    assert F[4, 4, 4] == int(rgb[3, 3, 2]) - int(rgb[4, 4, 2])
    # node 4 at (0, 0): probe (-1, -1) clamps to (0, 0) -> 0
    assert F[0, 0, 4] == 0
    assert np.all(F[:, :, 5][depth > 0] == 0)
    # node 7 at (1, 4): trunc(2.6) = 2 -> probe (3, 4) valid 1000
    assert F[4, 1, 7] == 0
    # invalid pixels report 0 for every feature
    assert np.all(F[2, 2] == 0) and np.all(F[0, 7] == 0)


def test_focal_scaling(orc):
    """At twice the reference focal length the same metric offset spans twice
    the pixels: trunc(delta * F / (d * F_ref))."""
    f = tiny_forest(orc)
    depth, rgb = image()
    set_extra(f, [(1, 1300, 0, 0), (1, -1300, 0, 0)] + [(0, 0, 0, 0)] * 6)
    K2 = (554.0, 554.0, 4.0, 3.0)
    F = f.features8(depth, rgb, K2).reshape(H, W, 8)
    # trunc(1300 * 8864 / (1000 * 4432)) = trunc(2.6) = 2
    assert F[1, 1, 0] == int(rgb[1, 3, 0]) - int(rgb[1, 1, 0])
    assert F[1, 4, 1] == int(rgb[1, 2, 0]) - int(rgb[1, 4, 0])


def test_traversal_special_cases(orc):
    depth, rgb = image()
    for D in (1, 3, 5):
        f = tiny_forest(orc, depth=D, T=2)
        kind, dx, dy, thr = f.nodes()
        n = f.T * (f.L - 1)
        thr[:n] = I32_MIN
        f.set_nodes(kind, dx, dy, thr)
        lv = f.leaves(depth, rgb, K_REF)
        valid = ((depth >= 500) & (depth <= 5000)).reshape(-1)
        assert np.all(lv[:, valid] == f.L - 1) and np.all(lv[:, ~valid] == -1)
        thr[:n] = I32_MAX
        f.set_nodes(kind, dx, dy, thr)
        lv = f.leaves(depth, rgb, K_REF)
        assert np.all(lv[:, valid] == 0)


def test_constant_image_follows_threshold_bits(orc):
    """With zero offsets every response is 0, so the path is the bit string of
    (0 >= thr) decisions from the root."""
    D = 6
    f = tiny_forest(orc, depth=D, T=3)
    kind, dx, dy, thr = f.nodes()
    n = f.T * (f.L - 1)
    dx[:n] = 0
    dy[:n] = 0
    f.set_nodes(kind, dx, dy, thr)
    depth = np.full((H, W), 1500, dtype=np.uint16)
    rgb = np.full((H, W, 3), 77, dtype=np.uint8)
    lv = f.leaves(depth, rgb, K_REF)
    for t in range(f.T):
        i = 0
        while i < f.L - 1:
            i = 2 * i + 1 + (1 if 0 >= thr[t * (f.L - 1) + i] else 0)
        assert np.all(lv[t] == i - (f.L - 1))


def test_camera_point_matches_float32(orc):
    rng = np.random.default_rng(5)
    depth = rng.integers(300, 5200, size=(24, 32)).astype(np.uint16)
    K = (277.0, 281.5, 16.0, 12.0)
    ref = cam_points_f32(depth, K)
    p = orc.default_params()
    out = np.zeros(3, dtype=np.float32)
    import ctypes as C
    Kf = np.asarray(K, dtype=np.float32)
    for v in range(24):
        for u in range(32):
            rc = orc.lib().oracle_camera_point(depth.ctypes.data, 32, 24, Kf.ctypes.data, u, v, C.byref(p),
                                               out.ctypes.data)
            d = int(depth[v, u])
            if 500 <= d <= 5000:
                assert rc == 0
                assert np.array_equal(out.view(np.uint32), ref[v * 32 + u].view(np.uint32))
            else:
                assert rc == 1


def test_generated_nodes_ranges(orc):
    f = tiny_forest(orc, depth=8, T=4)
    kind, dx, dy, thr = f.nodes()
    p = f.params
    assert set(np.unique(kind)) <= {0, 1, 2, 3}
    assert np.all(np.abs(dx) <= p.offset_pxmm) and np.all(np.abs(dy) <= p.offset_pxmm)
    assert np.all(np.abs(thr[kind == 0]) <= p.thr_depth_mm)
    assert np.all(np.abs(thr[kind > 0]) <= p.thr_rgb)
    # half the nodes are depth tests (kind draw uniform over 6, 3 of them depth)
    assert 0.4 < np.mean(kind == 0) < 0.6
    # same seed -> same forest; another seed -> another forest
    g = tiny_forest(orc, depth=8, T=4)
    assert all(np.array_equal(a, b) for a, b in zip(f.nodes(), g.nodes()))
    h = orc.Forest(orc.default_params(n_trees=4, depth=8, reservoir_size=4, seed=5))
    assert not np.array_equal(f.nodes()[1], h.nodes()[1])
