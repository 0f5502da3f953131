"""ctypes binding of the plain CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to say what the GPU path must compute. The product
package never imports it. See oracle.h for what the paper fixes and what the
oracle defines.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(verbose: bool = False) -> str:
    """Compiles liboracle.so with gcc (no FMA contraction, no fast-math)."""
    cmd = ["gcc", *CFLAGS, _SRC, "-o", _LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd, cwd=_HERE)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("n_trees", C.c_int32), ("depth", C.c_int32), ("reservoir_size", C.c_int32), ("max_modes", C.c_int32),
        ("seed", C.c_uint64),
        ("depth_min_mm", C.c_int32), ("depth_max_mm", C.c_int32), ("offset_pxmm", C.c_int32),
        ("f_ref_px16", C.c_int32), ("thr_depth_mm", C.c_int32), ("thr_rgb", C.c_int32),
        ("dens_radius_mm", C.c_int32), ("link_radius_mm", C.c_int32), ("min_cluster", C.c_int32),
        ("cov_reg_mm2", C.c_int32),
        ("n_hypotheses", C.c_int32), ("batch_pixels", C.c_int32), ("max_tries", C.c_int32), ("refine", C.c_int32),
        ("rgb_tol", C.c_int32),
        ("rigid_ratio2", C.c_float), ("min_pair2_m2", C.c_float), ("min_area2_m4", C.c_float),
        ("resid_m", C.c_float), ("inlier_m", C.c_float),
    ]


MODE_DTYPE = np.dtype([("mu", "<f4", 3), ("sinv", "<f4", 6), ("kappa", "<f4"), ("n", "<i4"),
                       ("rgb", "u1", 3), ("pad", "u1")])
ENTRY_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("z", "<i4"), ("r", "u1"), ("g", "u1"), ("b", "u1"),
                        ("pad", "u1")])
assert MODE_DTYPE.itemsize == 48 and ENTRY_DTYPE.itemsize == 16


class Trace(C.Structure):
    _fields_ = [
        ("cap_hyp", C.c_int32), ("cap_rounds", C.c_int32),
        ("pool_size", C.c_void_p), ("hyp_try", C.c_void_p), ("hyp_pose", C.c_void_p),
        ("n_rounds", C.c_void_p), ("n_alive", C.c_void_p), ("alive", C.c_void_p), ("energy", C.c_void_p),
        ("n_inliers", C.c_void_p), ("pose_after", C.c_void_p), ("final_hyp", C.c_void_p),
    ]


OK = 0
FAIL_NO_VALID_PIXELS = 1
FAIL_NO_MODES = 2
FAIL_NO_HYPOTHESIS = 3

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        vp, i32, u64 = C.c_void_p, C.c_int32, C.c_uint64
        L.oracle_philox.argtypes = [vp, vp, vp]
        L.oracle_uniform_int.argtypes = [u64, u64]
        L.oracle_uniform_int.restype = u64
        L.oracle_params_default.argtypes = [vp]
        L.oracle_forest_create.argtypes = [vp, vp]
        L.oracle_forest_destroy.argtypes = [vp]
        L.oracle_forest_destroy.restype = None
        L.oracle_forest_nodes.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_set_nodes.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_camera_point.argtypes = [vp, i32, i32, vp, i32, i32, vp, vp]
        L.oracle_leaves.argtypes = [vp, vp, vp, i32, i32, vp, vp]
        L.oracle_features8.argtypes = [vp, vp, vp, i32, i32, vp, vp]
        L.oracle_adapt_frame.argtypes = [vp, vp, vp, i32, i32, vp, vp]
        L.oracle_train_forest.argtypes = [vp, i32, vp, vp, i32, i32, vp, vp, i32, i32]
        L.oracle_reservoir.argtypes = [vp, i32, i32, vp, vp]
        L.oracle_leaf_modes.argtypes = [vp, i32, i32, vp, vp]
        L.oracle_modes_from_points.argtypes = [vp, vp, i32, vp, vp, vp]
        L.oracle_modes_bruteforce.argtypes = [vp, vp, i32, vp, vp, vp]
        L.oracle_build_all_modes.argtypes = [vp]
        L.oracle_drop_reservoirs.argtypes = [vp]
        L.oracle_total_samples.argtypes = [vp]
        L.oracle_total_samples.restype = u64
        L.oracle_kabsch.argtypes = [vp, vp, i32, vp, vp]
        L.oracle_svd3.argtypes = [vp, vp, vp, vp]
        L.oracle_relocalise.argtypes = [vp, vp, vp, i32, i32, vp, u64, i32, vp, vp, vp, vp]
        L.oracle_pose_success.argtypes = [vp, vp, vp, vp]
        L.oracle_verify.argtypes = [vp, vp, i32, i32, vp, vp, vp]
        L.oracle_bf16.argtypes = [C.c_float]
        L.oracle_bf16.restype = C.c_float
        L.oracle_features24.argtypes = [vp, vp, vp, i32, i32, vp, vp, i32, vp]
        L.oracle_label.argtypes = [vp, vp, vp, i32, i32, vp, vp, vp, i32, vp]
        L.oracle_mlp_init.argtypes = [u64, vp]
        L.oracle_mlp_init.restype = None
        L.oracle_mlp_forward.argtypes = [vp, vp, i32, vp]
        L.oracle_mlp_grad.argtypes = [vp, vp, vp, i32, vp, vp]
        L.oracle_forest_save.argtypes = [vp, C.c_char_p]
        L.oracle_forest_load.argtypes = [C.c_char_p, vp]
        L.oracle_check_triple.argtypes = [vp, vp, vp, vp, vp, vp]
        L.oracle_colour_ok.argtypes = [vp, vp, vp]
        L.oracle_mode_term.argtypes = [vp, vp]
        L.oracle_mode_term.restype = C.c_float
        L.oracle_pose_from_sums.argtypes = [vp, vp, vp]
        L.oracle_preemptive.argtypes = [vp, vp, vp, i32, i32, vp, u64, i32, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def default_params(**kw) -> Params:
    p = Params()
    lib().oracle_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox(_p(c), _p(k), _p(out))
    return out


def uniform_int(u: int, n: int) -> int:
    return int(lib().oracle_uniform_int(C.c_uint64(u), C.c_uint64(n)))


def svd3(A: np.ndarray):
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    U = np.zeros(9); S = np.zeros(3); V = np.zeros(9)
    rc = lib().oracle_svd3(_p(A), _p(U), _p(S), _p(V))
    return rc, U.reshape(3, 3), S, V.reshape(3, 3)


def kabsch(src: np.ndarray, dst: np.ndarray):
    s = np.ascontiguousarray(src, dtype=np.float64)
    d = np.ascontiguousarray(dst, dtype=np.float64)
    R = np.zeros(9); t = np.zeros(3)
    rc = lib().oracle_kabsch(_p(s), _p(d), len(s), _p(R), _p(t))
    return rc, R.reshape(3, 3), t


def modes_from_points(params: Params, pts: np.ndarray, brute: bool = False):
    pts = np.ascontiguousarray(pts, dtype=ENTRY_DTYPE)
    modes = np.zeros(params.max_modes, dtype=MODE_DTYPE)
    nm = C.c_int32(0)
    labels = np.zeros(max(len(pts), 1), dtype=np.int32)
    fn = lib().oracle_modes_bruteforce if brute else lib().oracle_modes_from_points
    rc = fn(C.byref(params), _p(pts), len(pts), _p(modes), C.byref(nm), _p(labels))
    assert rc == 0, rc
    return modes[: nm.value].copy(), labels[: len(pts)].copy()


def pose_success(est: np.ndarray, gt: np.ndarray) -> Tuple[bool, float, float]:
    e = np.ascontiguousarray(est, dtype=np.float64).reshape(16)
    g = np.ascontiguousarray(gt, dtype=np.float64).reshape(16)
    dt = C.c_double(0); da = C.c_double(0)
    ok = lib().oracle_pose_success(_p(e), _p(g), C.byref(dt), C.byref(da))
    return bool(ok == 1), dt.value, da.value


def _np(x) -> np.ndarray:
    try:
        import torch
        if isinstance(x, torch.Tensor):
            x = x.detach().cpu().numpy()
    except ImportError:  # pragma: no cover
        pass
    return np.ascontiguousarray(x)


def _K(K) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(K, dtype=np.float32).reshape(4))


class Forest:
    """One relocalisation forest held by the oracle."""

    def __init__(self, params: Params, _handle=None):
        self.params = params
        self._h = C.c_void_p()
        if _handle is not None:
            self._h = _handle
        else:
            rc = lib().oracle_forest_create(C.byref(params), C.byref(self._h))
            if rc != 0:
                raise ValueError(f"oracle_forest_create failed: {rc}")
        self.T = params.n_trees
        self.L = 1 << params.depth
        self.R = params.reservoir_size
        self.M = params.max_modes

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.oracle_forest_destroy(h)
            self._h = C.c_void_p()

    def nodes(self):
        n = self.T * (self.L - 1) + 8
        kind, dx, dy, thr = (np.zeros(n, dtype=np.int32) for _ in range(4))
        lib().oracle_forest_nodes(self._h, _p(kind), _p(dx), _p(dy), _p(thr))
        return kind, dx, dy, thr

    def set_nodes(self, kind, dx, dy, thr):
        arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (kind, dx, dy, thr)]
        assert rc_ok(lib().oracle_set_nodes(self._h, *[_p(a) for a in arrs]))

    def leaves(self, depth, rgb, K) -> np.ndarray:
        d = _np(depth).astype(np.uint16, copy=False)
        c = _np(rgb).astype(np.uint8, copy=False)
        H, W = d.shape
        out = np.zeros((self.T, H * W), dtype=np.int32)
        rc = lib().oracle_leaves(self._h, _p(d), _p(c), W, H, _p(_K(K)), _p(out))
        if rc != 0:
            raise ValueError(rc)
        return out

    def features8(self, depth, rgb, K) -> np.ndarray:
        d = _np(depth).astype(np.uint16, copy=False)
        c = _np(rgb).astype(np.uint8, copy=False)
        H, W = d.shape
        out = np.zeros((H * W, 8), dtype=np.int32)
        rc = lib().oracle_features8(self._h, _p(d), _p(c), W, H, _p(_K(K)), _p(out))
        if rc != 0:
            raise ValueError(rc)
        return out

    def adapt(self, depth, rgb, K, pose) -> None:
        d = _np(depth).astype(np.uint16, copy=False)
        c = _np(rgb).astype(np.uint8, copy=False)
        H, W = d.shape
        T = np.ascontiguousarray(pose, dtype=np.float64).reshape(16)
        rc = lib().oracle_adapt_frame(self._h, _p(d), _p(c), W, H, _p(_K(K)), _p(T))
        if rc != 0:
            raise ValueError(rc)

    def train(self, frames, K, stride: int, n_cand: int) -> None:
        """Split training (oracle_train_forest) on [(depth, rgb, pose)] of one
        size and intrinsics; empties every leaf."""
        ds = [np.ascontiguousarray(_np(d), dtype=np.uint16) for d, _, _ in frames]
        cs = [np.ascontiguousarray(_np(c), dtype=np.uint8) for _, c, _ in frames]
        H, W = ds[0].shape
        dp = (C.c_void_p * len(ds))(*[a.ctypes.data for a in ds])
        cp = (C.c_void_p * len(cs))(*[a.ctypes.data for a in cs])
        P = np.ascontiguousarray(np.stack([np.asarray(T, dtype=np.float64).reshape(16) for _, _, T in frames]))
        rc = lib().oracle_train_forest(self._h, len(ds), dp, cp, W, H, _p(_K(K)), _p(P), int(stride), int(n_cand))
        if rc != 0:
            raise ValueError(rc)

    def reservoir(self, t: int, leaf: int):
        e = np.zeros(self.R, dtype=ENTRY_DTYPE)
        cnt = C.c_uint32(0)
        rc = lib().oracle_reservoir(self._h, t, leaf, _p(e), C.byref(cnt))
        if rc != 0:
            raise ValueError(rc)
        return e, cnt.value

    def leaf_modes(self, t: int, leaf: int) -> np.ndarray:
        m = np.zeros(self.M, dtype=MODE_DTYPE)
        nm = C.c_int32(0)
        rc = lib().oracle_leaf_modes(self._h, t, leaf, _p(m), C.byref(nm))
        if rc != 0:
            raise ValueError(rc)
        return m[: nm.value].copy()

    def save(self, path: str) -> None:
        rc = lib().oracle_forest_save(self._h, os.fsencode(path))
        if rc != 0:
            raise ValueError(f"oracle_forest_save failed: {rc}")

    @classmethod
    def load(cls, path: str, params: Params) -> "Forest":
        """A forest from a checkpoint file; `params` must be those it was
        saved with (the file carries them too, and the load checks nothing
        against these)."""
        h = C.c_void_p()
        rc = lib().oracle_forest_load(os.fsencode(path), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_forest_load failed: {rc}")
        return cls(params, _handle=h)

    def build_all_modes(self) -> None:
        assert lib().oracle_build_all_modes(self._h) == 0

    def drop_reservoirs(self) -> None:
        assert lib().oracle_drop_reservoirs(self._h) == 0

    @property
    def total_samples(self) -> int:
        return int(lib().oracle_total_samples(self._h))

    @staticmethod
    def _trace(N: int):
        RND = 40
        bufs = dict(pool_size=np.zeros(1, np.int32), hyp_try=np.full(N, -2, np.int32),
                    hyp_pose=np.zeros((N, 12)), n_rounds=np.zeros(1, np.int32),
                    n_alive=np.zeros(RND, np.int32), alive=np.full((RND, N), -1, np.int32),
                    energy=np.zeros((RND, N), np.float32), n_inliers=np.zeros((RND, N), np.int32),
                    pose_after=np.zeros((RND, N, 12)), final_hyp=np.full(1, -1, np.int32))
        return bufs, Trace(cap_hyp=N, cap_rounds=RND, **{k: v.ctypes.data for k, v in bufs.items()})

    def relocalise(self, depth, rgb, K, seed: int, n_hyp: int = 0, weights=None, trace: bool = False):
        d = _np(depth).astype(np.uint16, copy=False)
        c = _np(rgb).astype(np.uint8, copy=False)
        H, W = d.shape
        pose = np.zeros(16)
        score = C.c_float(0)
        w = None if weights is None else np.ascontiguousarray(_np(weights), dtype=np.uint32).reshape(-1)
        tr = None
        bufs = {}
        if trace:
            bufs, tr = self._trace(n_hyp if n_hyp > 0 else self.params.n_hypotheses)
        rc = lib().oracle_relocalise(self._h, _p(d), _p(c), W, H, _p(_K(K)), C.c_uint64(seed), n_hyp, _p(w),
                                     _p(pose), C.byref(score), C.byref(tr) if tr is not None else None)
        if rc < 0:
            raise ValueError(rc)
        return rc, pose.reshape(4, 4), score.value, bufs

    def preemptive(self, depth, rgb, K, seed: int, poses, valid):
        """The preemptive rounds over given hypotheses: poses [n, 12] (R
        row-major then t), valid [n]. Returns (status, pose, score, trace)."""
        d = _np(depth).astype(np.uint16, copy=False)
        c = _np(rgb).astype(np.uint8, copy=False)
        H, W = d.shape
        P = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 12)
        v = np.ascontiguousarray(valid, dtype=np.int32).reshape(-1)
        assert len(P) == len(v)
        pose = np.zeros(16)
        score = C.c_float(0)
        bufs, tr = self._trace(len(P))
        rc = lib().oracle_preemptive(self._h, _p(d), _p(c), W, H, _p(_K(K)), C.c_uint64(seed), len(P), _p(P), _p(v),
                                     _p(pose), C.byref(score), C.byref(tr))
        if rc < 0:
            raise ValueError(rc)
        return rc, pose.reshape(4, 4), score.value, bufs


TRI_OK, TRI_SAME_PIXEL, TRI_PAIR_DIST, TRI_WORLD_LONGER, TRI_CAMERA_LONGER, TRI_AREA, TRI_DEGENERATE, \
    TRI_RESIDUAL = range(8)


def check_triple(params: Params, pi, c, w):
    """(check code, R, t) of one hypothesis triple: pool indices pi [3],
    camera points c [3, 3] and mode means w [3, 3] (FP32)."""
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.float32).reshape(9)
    w = np.ascontiguousarray(w, dtype=np.float32).reshape(9)
    R = np.zeros(9); t = np.zeros(3)
    rc = lib().oracle_check_triple(C.byref(params), _p(pi), _p(c), _p(w), _p(R), _p(t))
    return rc, R.reshape(3, 3), t


def colour_ok(params: Params, mode_rgb, px) -> bool:
    a = np.ascontiguousarray(mode_rgb, dtype=np.uint8)
    b = np.ascontiguousarray(px, dtype=np.uint8)
    return lib().oracle_colour_ok(C.byref(params), _p(a), _p(b)) == 1


def mode_term(mode: np.ndarray, y) -> float:
    """The FP32 energy term of one mode (a MODE_DTYPE record) at y."""
    m = np.ascontiguousarray(np.asarray(mode, dtype=MODE_DTYPE).reshape(1))
    yy = np.ascontiguousarray(y, dtype=np.float32).reshape(3)
    return float(lib().oracle_mode_term(_p(m), _p(yy)))


def pose_from_sums(sums):
    s = np.ascontiguousarray(sums, dtype=np.float64).reshape(22)
    R = np.zeros(9); t = np.zeros(3)
    rc = lib().oracle_pose_from_sums(_p(s), _p(R), _p(t))
    return rc, R.reshape(3, 3), t


MLP_NPARAM = 5825


def verify(da, db):
    """(valid fraction of da, mean |da - db| in m over pixels valid in both, accept)"""
    a = np.ascontiguousarray(_np(da), dtype=np.uint16)
    b = np.ascontiguousarray(_np(db), dtype=np.uint16)
    H, W = a.shape
    vf = C.c_double(0); mu = C.c_double(0); acc = C.c_int(0)
    rc = lib().oracle_verify(_p(a), _p(b), W, H, C.byref(vf), C.byref(mu), C.byref(acc))
    if rc != 0:
        raise ValueError(rc)
    return vf.value, mu.value, bool(acc.value)


def bf16(x: float) -> float:
    return float(lib().oracle_bf16(C.c_float(x)))


def mlp_init(seed: int) -> np.ndarray:
    w = np.zeros(MLP_NPARAM, dtype=np.float32)
    lib().oracle_mlp_init(C.c_uint64(seed), _p(w))
    return w


def mlp_forward(w: np.ndarray, x: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 24)
    z = np.zeros(len(x))
    assert lib().oracle_mlp_forward(_p(w), _p(x), len(x), _p(z)) == 0
    return z


def mlp_grad(w: np.ndarray, x: np.ndarray, y: np.ndarray):
    w = np.ascontiguousarray(w, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 24)
    y = np.ascontiguousarray(y, dtype=np.uint8)
    g = np.zeros(MLP_NPARAM)
    loss = C.c_double(0)
    assert lib().oracle_mlp_grad(_p(w), _p(x), _p(y), len(x), _p(g), C.byref(loss)) == 0
    return g, loss.value


def _forest_features24(self, depth, rgb, K, pix) -> np.ndarray:
    d = _np(depth).astype(np.uint16, copy=False)
    c = _np(rgb).astype(np.uint8, copy=False)
    H, W = d.shape
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    out = np.zeros((len(pix), 24), dtype=np.float32)
    rc = lib().oracle_features24(self._h, _p(d), _p(c), W, H, _p(_K(K)), _p(pix), len(pix), _p(out))
    if rc != 0:
        raise ValueError(rc)
    return out


def _forest_label(self, depth, rgb, K, pose, pix) -> np.ndarray:
    d = _np(depth).astype(np.uint16, copy=False)
    c = _np(rgb).astype(np.uint8, copy=False)
    H, W = d.shape
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    T = np.ascontiguousarray(pose, dtype=np.float64).reshape(16)
    out = np.zeros(len(pix), dtype=np.uint8)
    rc = lib().oracle_label(self._h, _p(d), _p(c), W, H, _p(_K(K)), _p(T), _p(pix), len(pix), _p(out))
    if rc != 0:
        raise ValueError(rc)
    return out


Forest.features24 = _forest_features24
Forest.label = _forest_label


def rc_ok(rc: int) -> bool:
    return rc == 0
