"""Python binding of libreloc (the gfx950 forest relocaliser behind include/reloc.h).

Argument marshalling only: every step of adaptation and relocalisation runs
in the HIP kernels of libreloc.so. Frames are torch tensors on the GPU
(depth uint16 [H, W] in mm, rgb uint8 [H, W, 3]); torch supplies device
memory and the current stream. There is no CPU fallback: if the library is
not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libreloc.so")

OK = 0
FAIL_NO_VALID_PIXELS = 1
FAIL_NO_MODES = 2
FAIL_NO_HYPOTHESIS = 3
E_ARG = -1
E_NOMEM = -2
E_HIP = -3
E_STATE = -4
E_RANGE = -5
E_IO = -6


class RelocError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


class reloc_params(C.Structure):
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


class reloc_intrinsics(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class reloc_trace(C.Structure):
    _fields_ = [("cap_hyp", C.c_int32), ("cap_rounds", C.c_int32),
                ("pool_size", C.c_void_p), ("hyp_try", C.c_void_p), ("hyp_pose", C.c_void_p),
                ("n_rounds", C.c_void_p), ("n_alive", C.c_void_p), ("alive", C.c_void_p),
                ("energy", C.c_void_p), ("n_inliers", C.c_void_p), ("final_hyp", C.c_void_p)]


class reloc_result(C.Structure):
    _fields_ = [("pose_c2w", C.c_double * 16), ("score", C.c_float), ("status", C.c_int32),
                ("n_rounds", C.c_int32), ("final_hyp", C.c_int32), ("pool_size", C.c_int32),
                ("n_valid", C.c_int32), ("mode_evals", C.c_uint64), ("pair_evals", C.c_uint64)]

    def as_dict(self) -> dict:
        return dict(pose=np.array(self.pose_c2w[:], dtype=np.float64).reshape(4, 4), score=self.score,
                    status=self.status, n_rounds=self.n_rounds, final_hyp=self.final_hyp,
                    pool_size=self.pool_size, n_valid=self.n_valid, mode_evals=self.mode_evals,
                    pair_evals=self.pair_evals)


class reloc_train_frame(C.Structure):
    _fields_ = [("depth_dev", C.c_void_p), ("rgb_dev", C.c_void_p), ("K", reloc_intrinsics),
                ("pose_c2w", C.c_double * 16)]


class reloc_attempt(C.Structure):
    _fields_ = [("forest", C.c_void_p), ("depth_dev", C.c_void_p), ("rgb_dev", C.c_void_p),
                ("K", reloc_intrinsics), ("seed", C.c_uint64), ("n_hypotheses", C.c_int32),
                ("pixel_weights_dev", C.c_void_p), ("proposal", C.c_void_p)]


ENTRY_DTYPE = np.dtype([("x", "<i4"), ("y", "<i4"), ("z", "<i4"), ("r", "u1"), ("g", "u1"), ("b", "u1"),
                        ("pad", "u1")])
MODE_DTYPE = np.dtype([("mu", "<f4", 3), ("sinv", "<f4", 6), ("kappa", "<f4"), ("n", "<i4"),
                       ("rgb", "u1", 3), ("pad", "u1")])

_lib = None

_SIGS = {
    "reloc_params_default": [C.c_void_p],
    "reloc_forest_create": [C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_forest_destroy": [C.c_void_p],
    "reloc_adapt_frame": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_update_modes": [C.c_void_p, C.c_void_p],
    "reloc_relocalise": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p,
                         C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_forest_drop_reservoirs": [C.c_void_p, C.c_void_p],
    "reloc_forest_save": [C.c_void_p, C.c_char_p, C.c_void_p],
    "reloc_forest_load": [C.c_char_p, C.c_void_p, C.c_void_p],
    "reloc_forest_params": [C.c_void_p, C.c_void_p],
    "reloc_forest_train": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p],
    "reloc_forest_memory": [C.c_void_p, C.c_void_p],
    "reloc_status_string": [C.c_int],
    "reloc_debug_nodes": [C.c_void_p] * 5,
    "reloc_debug_set_nodes": [C.c_void_p] * 5,
    "reloc_debug_leaves": [C.c_void_p] * 6,
    "reloc_debug_features8": [C.c_void_p] * 6,
    "reloc_debug_reservoir": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p],
    "reloc_debug_modes": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p],
    "reloc_debug_modes_from_points": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p],
    "reloc_debug_trace": [C.c_void_p, C.c_void_p],
    "reloc_profile_enable": [C.c_int],
    "reloc_profile_reset": [],
    "reloc_profile_read": [C.c_char_p, C.c_void_p, C.c_void_p],
    "reloc_profile_read_raw": [C.c_char_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_profile_kernels": [C.c_char_p, C.c_int32],
    "reloc_relocalise_ex": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32, C.c_void_p,
                            C.c_void_p, C.c_void_p],
    "reloc_batch_create": [C.c_void_p],
    "reloc_batch_destroy": [C.c_void_p],
    "reloc_relocalise_batch": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p],
    "reloc_batch_set_tuning": [C.c_void_p, C.c_int32],
    "reloc_batch_schedule": [C.c_void_p, C.c_char_p, C.c_int32],
    "reloc_batch_memory": [C.c_void_p, C.c_void_p],
    "reloc_debug_unit_owners": [C.c_int32, C.c_int32, C.c_int32, C.c_void_p],
    "reloc_verify": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                     C.c_void_p],
    "reloc_verify_noalloc": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p],
    "reloc_relative_transform": [C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_collab_create": [C.c_int32, C.c_uint64, C.c_void_p],
    "reloc_collab_destroy": [C.c_void_p],
    "reloc_collab_set_frames": [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32],
    "reloc_collab_schedule": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_collab_tried": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32],
    "reloc_collab_add_sample": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p],
    "reloc_collab_clusters": [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "reloc_collab_optimise": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_mlp_create": [C.c_uint64, C.c_void_p, C.c_void_p],
    "reloc_mlp_destroy": [C.c_void_p],
    "reloc_mlp_get_weights": [C.c_void_p, C.c_void_p],
    "reloc_mlp_set_weights": [C.c_void_p, C.c_void_p],
    "reloc_mlp_gradient": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_mlp_train": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_uint64,
                        C.c_void_p, C.c_void_p],
    "reloc_mlp_logits": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p],
    "reloc_mlp_pixel_weights": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p],
    "reloc_pixel_features": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                             C.c_void_p, C.c_void_p],
    "reloc_label_pixels": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                           C.c_void_p, C.c_void_p],
    "reloc_debug_mfma_probe": [C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_debug_lane_probe": [C.c_void_p],
    "reloc_valid_pixels": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "reloc_debug_horn": [C.c_void_p, C.c_int32, C.c_void_p],
    "reloc_debug_div": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "reloc_debug_bf16": [C.c_void_p, C.c_int32, C.c_void_p],
    "reloc_relocalise_learned": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32,
                                 C.c_void_p, C.c_void_p],
}

MLP_NPARAM = 5825


def unit_owners(xcd: int, total: int, grid: int) -> np.ndarray:
    """Host run of the persistent kernels' work-unit ownership rule."""
    out = np.zeros(max(total, 1), dtype=np.int32)
    _check(lib().reloc_debug_unit_owners(int(xcd), int(total), int(grid), out.ctypes.data), "reloc_debug_unit_owners")
    return out[:total]


def horn_quaternions(H: np.ndarray) -> np.ndarray:
    """Host run of the pose solver's eigenvector step on cross-covariances
    H [n, 3, 3]; NaN rows where the device falls back to power iteration."""
    H = np.ascontiguousarray(H, dtype=np.float64).reshape(-1, 9)
    q = np.zeros((len(H), 4))
    _check(lib().reloc_debug_horn(H.ctypes.data if len(H) else None, len(H), q.ctypes.data), "reloc_debug_horn")
    return q


def probe_div(n: np.ndarray, den: np.ndarray) -> np.ndarray:
    """Host run of the kernels' probe-offset division: trunc(n / den)."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    den = np.ascontiguousarray(den, dtype=np.int32)
    if n.shape != den.shape:
        raise ValueError("n and den differ in shape")
    q = np.zeros(n.shape, dtype=np.int32)
    _check(lib().reloc_debug_div(n.ctypes.data if n.size else None, den.ctypes.data if n.size else None, n.size,
                                 q.ctypes.data if n.size else None), "reloc_debug_div")
    return q


def lib() -> C.CDLL:
    """Loads libreloc.so (built by build.py); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libreloc.so is not built ({LIB_PATH}); run paper_1801_08361_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.reloc_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().reloc_status_string(int(code)).decode()


def _check(code: int, what: str) -> int:
    if code < 0:
        raise RelocError(code, what)
    return code


def profile_enable(on: bool = True) -> None:
    _check(lib().reloc_profile_enable(1 if on else 0), "reloc_profile_enable")


def profile_reset() -> None:
    _check(lib().reloc_profile_reset(), "reloc_profile_reset")


def profile_read(kernel: str) -> Tuple[float, int]:
    """(total milliseconds, launches) of one kernel since the last reset."""
    ms = C.c_double(0)
    n = C.c_int64(0)
    _check(lib().reloc_profile_read(kernel.encode(), C.byref(ms), C.byref(n)), "reloc_profile_read")
    return ms.value, n.value


def profile_kernels() -> list:
    buf = C.create_string_buffer(8192)
    _check(lib().reloc_profile_kernels(buf, 8192), "reloc_profile_kernels")
    return [k for k in buf.value.decode().split(",") if k]


def params_default(**kw) -> reloc_params:
    p = reloc_params()
    _check(lib().reloc_params_default(C.byref(p)), "reloc_params_default")
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


def _frame(depth, rgb, K) -> Tuple[int, int, reloc_intrinsics]:
    import torch
    if not (isinstance(depth, torch.Tensor) and isinstance(rgb, torch.Tensor)):
        raise TypeError("depth and rgb must be torch tensors on the GPU")
    if depth.dtype != torch.uint16 or rgb.dtype != torch.uint8 or not depth.is_cuda or not rgb.is_cuda:
        raise TypeError("depth must be uint16 and rgb uint8, both on the GPU")
    if not depth.is_contiguous() or not rgb.is_contiguous():
        raise ValueError("frames must be contiguous")
    H, W = depth.shape
    if tuple(rgb.shape) != (H, W, 3):
        raise ValueError("rgb must be [H, W, 3] matching depth [H, W]")
    fx, fy, cx, cy = (float(k) for k in K)
    return depth.data_ptr(), rgb.data_ptr(), reloc_intrinsics(W, H, fx, fy, cx, cy)


def _pose(T) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(16))


class Forest:
    """One sub-scene relocaliser held on the GPU (reloc_forest)."""

    def __init__(self, params: Optional[reloc_params] = None, stream=None, _handle=None, **kw):
        self._h = C.c_void_p()
        if _handle is not None:
            self._h = _handle
            self.params = params
        else:
            self.params = params if params is not None else params_default(**kw)
            _check(lib().reloc_forest_create(C.byref(self.params), _stream(stream), C.byref(self._h)),
                   "reloc_forest_create")
        self.T = self.params.n_trees
        self.L = 1 << self.params.depth
        self.R = self.params.reservoir_size
        self.M = self.params.max_modes

    def save(self, path: str, stream=None) -> None:
        """Checkpoint to a file (reloc_forest_save)."""
        _check(lib().reloc_forest_save(self._h, os.fsencode(path), _stream(stream)), "reloc_forest_save")

    @classmethod
    def load(cls, path: str, stream=None) -> "Forest":
        """A new forest from a checkpoint file (reloc_forest_load)."""
        h = C.c_void_p()
        _check(lib().reloc_forest_load(os.fsencode(path), _stream(stream), C.byref(h)), "reloc_forest_load")
        p = reloc_params()
        rc = lib().reloc_forest_params(h, C.byref(p))
        if rc < 0:
            lib().reloc_forest_destroy(h)
            raise RelocError(rc, "reloc_forest_params")
        return cls(p, _handle=h)

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def close(self) -> None:
        if self._h is not None and self._h.value and _lib is not None:
            _lib.reloc_forest_destroy(self._h)
        self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the method --------------------------------------------------------

    def adapt_frame(self, depth, rgb, K, pose, stream=None) -> None:
        d, c, k = _frame(depth, rgb, K)
        T = _pose(pose)
        _check(lib().reloc_adapt_frame(self._h, d, c, C.byref(k), T.ctypes.data, _stream(stream)),
               "reloc_adapt_frame")

    def train(self, frames, stride: int, n_candidates: int, stream=None) -> None:
        """Split training (reloc_forest_train) on [(depth, rgb, K, pose)]
        device frames of one scene; empties every leaf."""
        arr = (reloc_train_frame * len(frames))()
        keep = []
        for x, (depth, rgb, K, pose) in zip(arr, frames):
            d, c, k = _frame(depth, rgb, K)
            x.depth_dev, x.rgb_dev, x.K = d, c, k
            x.pose_c2w[:] = [float(v) for v in _pose(pose)]
            keep.append((depth, rgb))
        _check(lib().reloc_forest_train(self._h, arr, len(frames), int(stride), int(n_candidates), _stream(stream)),
               "reloc_forest_train")

    def update_modes(self, stream=None) -> None:
        _check(lib().reloc_update_modes(self._h, _stream(stream)), "reloc_update_modes")

    def relocalise(self, depth, rgb, K, seed: int, n_hyp: int = 0, weights=None, stream=None):
        """Returns (status, pose 4x4 float64, score)."""
        d, c, k = _frame(depth, rgb, K)
        pose = np.zeros(16)
        score = C.c_float(0)
        w = None
        if weights is not None:
            w = weights.data_ptr()
        rc = lib().reloc_relocalise(self._h, d, c, C.byref(k), C.c_uint64(seed), int(n_hyp), w,
                                    pose.ctypes.data, C.byref(score), _stream(stream))
        _check(rc, "reloc_relocalise")
        return rc, pose.reshape(4, 4), score.value

    def relocalise_ex(self, depth, rgb, K, seed: int, n_hyp: int = 0, weights=None, stream=None) -> dict:
        """Full result of one plain attempt (reloc_relocalise_ex) as a dict."""
        d, c, k = _frame(depth, rgb, K)
        res = reloc_result()
        w = weights.data_ptr() if weights is not None else None
        rc = lib().reloc_relocalise_ex(self._h, d, c, C.byref(k), C.c_uint64(seed), int(n_hyp), w, C.byref(res),
                                       _stream(stream))
        _check(rc, "reloc_relocalise_ex")
        return res.as_dict()

    def relocalise_learned(self, mlp: "Mlp", depth, rgb, K, seed: int, n_hyp: int = 0, stream=None) -> dict:
        """One attempt with the learned proposal computed inside the graph
        (reloc_relocalise_learned)."""
        d, c, k = _frame(depth, rgb, K)
        res = reloc_result()
        rc = lib().reloc_relocalise_learned(self._h, mlp.handle, d, c, C.byref(k), C.c_uint64(seed), int(n_hyp),
                                            C.byref(res), _stream(stream))
        _check(rc, "reloc_relocalise_learned")
        return res.as_dict()

    def drop_reservoirs(self, stream=None) -> None:
        _check(lib().reloc_forest_drop_reservoirs(self._h, _stream(stream)), "reloc_forest_drop_reservoirs")

    def memory(self) -> int:
        b = C.c_uint64(0)
        _check(lib().reloc_forest_memory(self._h, C.byref(b)), "reloc_forest_memory")
        return b.value

    # -- parity and debug exports -------------------------------------------

    def nodes(self):
        n = self.T * (self.L - 1) + 8
        arrs = [np.zeros(n, dtype=np.int32) for _ in range(4)]
        _check(lib().reloc_debug_nodes(self._h, *[a.ctypes.data for a in arrs]), "reloc_debug_nodes")
        return tuple(arrs)

    def set_nodes(self, kind, dx, dy, thr) -> None:
        arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (kind, dx, dy, thr)]
        _check(lib().reloc_debug_set_nodes(self._h, *[a.ctypes.data for a in arrs]), "reloc_debug_set_nodes")

    def leaves(self, depth, rgb, K, stream=None) -> np.ndarray:
        d, c, k = _frame(depth, rgb, K)
        out = np.zeros((self.T, k.width * k.height), dtype=np.int32)
        _check(lib().reloc_debug_leaves(self._h, d, c, C.byref(k), out.ctypes.data, _stream(stream)),
               "reloc_debug_leaves")
        return out

    def features8(self, depth, rgb, K, stream=None) -> np.ndarray:
        d, c, k = _frame(depth, rgb, K)
        out = np.zeros((k.width * k.height, 8), dtype=np.int32)
        _check(lib().reloc_debug_features8(self._h, d, c, C.byref(k), out.ctypes.data, _stream(stream)),
               "reloc_debug_features8")
        return out

    def reservoir(self, t: int, leaf0: int = 0, n: int = 1):
        e = np.zeros((n, self.R), dtype=ENTRY_DTYPE)
        cnt = np.zeros(n, dtype=np.uint32)
        _check(lib().reloc_debug_reservoir(self._h, t, leaf0, n, e.ctypes.data, cnt.ctypes.data),
               "reloc_debug_reservoir")
        return e, cnt

    def counters(self, t: int, leaf0: int = 0, n: Optional[int] = None) -> np.ndarray:
        n = self.L - leaf0 if n is None else n
        cnt = np.zeros(n, dtype=np.uint32)
        _check(lib().reloc_debug_reservoir(self._h, t, leaf0, n, None, cnt.ctypes.data), "reloc_debug_reservoir")
        return cnt

    def modes(self, t: int, leaf0: int = 0, n: int = 1):
        m = np.zeros((n, self.M), dtype=MODE_DTYPE)
        nm = np.zeros(n, dtype=np.int32)
        _check(lib().reloc_debug_modes(self._h, t, leaf0, n, m.ctypes.data, nm.ctypes.data), "reloc_debug_modes")
        return m, nm

    def modes_from_points(self, pts: np.ndarray):
        pts = np.ascontiguousarray(pts, dtype=ENTRY_DTYPE)
        m = np.zeros(self.M, dtype=MODE_DTYPE)
        nm = C.c_int32(0)
        _check(lib().reloc_debug_modes_from_points(self._h, pts.ctypes.data if len(pts) else None, len(pts),
                                                   m.ctypes.data, C.byref(nm)), "reloc_debug_modes_from_points")
        return m[: nm.value].copy()

    def trace(self, n_hyp: int, rounds: int = 16):
        b = dict(pool_size=np.zeros(1, np.int32), hyp_try=np.full(n_hyp, -2, np.int32),
                 hyp_pose=np.zeros((n_hyp, 12)), n_rounds=np.zeros(1, np.int32),
                 n_alive=np.zeros(rounds, np.int32), alive=np.full((rounds, n_hyp), -1, np.int32),
                 energy=np.zeros((rounds, n_hyp), np.float32), final_hyp=np.full(1, -1, np.int32))
        tr = reloc_trace(cap_hyp=n_hyp, cap_rounds=rounds, n_inliers=None,
                         **{k: v.ctypes.data for k, v in b.items()})
        _check(lib().reloc_debug_trace(self._h, C.byref(tr)), "reloc_debug_trace")
        return b


class Batch:
    """A reloc_batch handle: many attempts (any forests, frame sizes and
    hypothesis counts) per call, run as one captured graph launch."""

    def __init__(self, tune: bool = True):
        self._h = C.c_void_p()
        _check(lib().reloc_batch_create(C.byref(self._h)), "reloc_batch_create")
        self.set_tuning(tune)

    def close(self) -> None:
        if self._h is not None and self._h.value and _lib is not None:
            _lib.reloc_batch_destroy(self._h)
        self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, on: bool) -> None:
        _check(lib().reloc_batch_set_tuning(self._h, 1 if on else 0), "reloc_batch_set_tuning")

    def schedule(self) -> str:
        buf = C.create_string_buffer(512)
        _check(lib().reloc_batch_schedule(self._h, buf, 512), "reloc_batch_schedule")
        return buf.value.decode()

    def memory(self) -> int:
        b = C.c_uint64(0)
        _check(lib().reloc_batch_memory(self._h, C.byref(b)), "reloc_batch_memory")
        return b.value

    def run(self, attempts: Sequence[dict], stream=None) -> list:
        """attempts: dicts with forest, depth, rgb, K, seed, and optionally
        n_hyp, weights (a device weight tensor) or proposal (an Mlp whose
        weights are computed inside the batch). Returns one result dict per
        attempt."""
        n = len(attempts)
        arr = (reloc_attempt * n)()
        for i, a in enumerate(attempts):
            d, c, k = _frame(a["depth"], a["rgb"], a["K"])
            w = a.get("weights")
            m = a.get("proposal")
            arr[i] = reloc_attempt(a["forest"].handle, d, c, k, int(a["seed"]), int(a.get("n_hyp", 0)),
                                   w.data_ptr() if w is not None else None, m.handle if m is not None else None)
        res = (reloc_result * n)()
        _check(lib().reloc_relocalise_batch(self._h, arr, n, res, _stream(stream)), "reloc_relocalise_batch")
        return [r.as_dict() for r in res]


# -- verification and the learned proposal -------------------------------------


def verify(da, db, noalloc: bool = False) -> Tuple[float, float, bool]:
    """Depth-difference verification of a proposed pose (reloc_verify, or
    reloc_verify_noalloc): da is the target scene rendered at the pose, db the
    relocalised frame; returns (valid fraction of da, mean |da - db| in
    metres, accepted)."""
    import torch
    for t in (da, db):
        if not (isinstance(t, torch.Tensor) and t.dtype == torch.uint16 and t.is_cuda and t.is_contiguous()):
            raise TypeError("depth images must be contiguous uint16 tensors on the GPU")
    if da.shape != db.shape or da.dim() != 2:
        raise ValueError("depth images must both be [H, W]")
    H, W = da.shape
    vf, mu, acc = C.c_double(0), C.c_double(0), C.c_int32(0)
    fn = lib().reloc_verify_noalloc if noalloc else lib().reloc_verify
    _check(fn(da.data_ptr(), db.data_ptr(), W, H, C.byref(vf), C.byref(mu), C.byref(acc), _stream(None)),
           "reloc_verify_noalloc" if noalloc else "reloc_verify")
    return vf.value, mu.value, bool(acc.value)


def _dev_tensor(t, dtype, shape=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.dtype == dtype and t.is_cuda and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} tensor on the GPU")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def valid_pixels(forest: "Forest", depth, rgb, K, stream=None):
    """int32 GPU tensor of the indices v W + u of the frame's valid pixels
    (depth in the forest's range), raster order (reloc_valid_pixels)."""
    import torch
    d, c, k = _frame(depth, rgb, K)
    pix = torch.empty(int(depth.numel()), dtype=torch.int32, device=depth.device)
    n = C.c_int32(0)
    _check(lib().reloc_valid_pixels(forest.handle, d, c, C.byref(k), pix.data_ptr(), C.byref(n), _stream(stream)),
           "reloc_valid_pixels")
    return pix[:n.value]


def pixel_features(forest: "Forest", depth, rgb, K, pix, with_fp32: bool = False, stream=None):
    """MLP inputs of the pixels `pix` (int32 GPU tensor of v W + u): bfloat16
    rows [n, 32] as int16 bit patterns and, optionally, FP32 values [n, 24]."""
    import torch
    d, c, k = _frame(depth, rgb, K)
    n = int(pix.numel())
    _dev_tensor(pix, torch.int32)
    x = torch.empty((n, 32), dtype=torch.int16, device=depth.device)
    xf = torch.empty((n, 24), dtype=torch.float32, device=depth.device) if with_fp32 else None
    _check(lib().reloc_pixel_features(forest.handle, d, c, C.byref(k), pix.data_ptr(), n, x.data_ptr(),
                                      xf.data_ptr() if xf is not None else None, _stream(stream)),
           "reloc_pixel_features")
    return (x, xf) if with_fp32 else x


def label_pixels(forest: "Forest", depth, rgb, K, pose, pix, stream=None):
    """Inlier labels (uint8 GPU tensor) of the pixels `pix` under `pose`."""
    import torch
    d, c, k = _frame(depth, rgb, K)
    n = int(pix.numel())
    _dev_tensor(pix, torch.int32)
    T = _pose(pose)
    y = torch.empty(n, dtype=torch.uint8, device=depth.device)
    _check(lib().reloc_label_pixels(forest.handle, d, c, C.byref(k), T.ctypes.data, pix.data_ptr(), n,
                                    y.data_ptr(), _stream(stream)), "reloc_label_pixels")
    return y


def lane_probe() -> np.ndarray:
    """The kernels' cross-lane helpers on one wavefront ([12, 64] uint32,
    reloc_debug_lane_probe)."""
    out = np.zeros((12, 64), dtype=np.uint32)
    _check(lib().reloc_debug_lane_probe(out.ctypes.data), "reloc_debug_lane_probe")
    return out


def mfma_probe(a: np.ndarray, bt: np.ndarray) -> np.ndarray:
    """C = A B of bfloat16 bit patterns a [16, 32] and bt = B^T [16, 32] on the
    matrix cores (reloc_debug_mfma_probe)."""
    a = np.ascontiguousarray(a, dtype=np.uint16)
    bt = np.ascontiguousarray(bt, dtype=np.uint16)
    assert a.shape == (16, 32) and bt.shape == (16, 32)
    c = np.zeros((16, 16), dtype=np.float32)
    _check(lib().reloc_debug_mfma_probe(a.ctypes.data, bt.ctypes.data, c.ctypes.data), "reloc_debug_mfma_probe")
    return c


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Bit patterns of x rounded to bfloat16 by the inference kernels'
    conversion on the GPU (reloc_debug_bf16)."""
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    y = np.zeros(x.shape, dtype=np.uint16)
    _check(lib().reloc_debug_bf16(x.ctypes.data if x.size else None, x.size, y.ctypes.data if x.size else None),
           "reloc_debug_bf16")
    return y


class Mlp:
    """The learned proposal network on the GPU (reloc_mlp)."""

    def __init__(self, seed: int, stream=None):
        self._h = C.c_void_p()
        _check(lib().reloc_mlp_create(C.c_uint64(seed), _stream(stream), C.byref(self._h)), "reloc_mlp_create")

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def close(self) -> None:
        if self._h is not None and self._h.value and _lib is not None:
            _lib.reloc_mlp_destroy(self._h)
        self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self) -> np.ndarray:
        w = np.zeros(MLP_NPARAM, dtype=np.float32)
        _check(lib().reloc_mlp_get_weights(self._h, w.ctypes.data), "reloc_mlp_get_weights")
        return w

    def set_weights(self, w: np.ndarray) -> None:
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.shape == (MLP_NPARAM,)
        _check(lib().reloc_mlp_set_weights(self._h, w.ctypes.data), "reloc_mlp_set_weights")

    def gradient(self, x, y, stream=None) -> Tuple[np.ndarray, float]:
        import torch
        n = int(y.numel())
        _dev_tensor(x, torch.int16, (n, 32))
        _dev_tensor(y, torch.uint8)
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        loss = C.c_float(0)
        _check(lib().reloc_mlp_gradient(self._h, x.data_ptr(), y.data_ptr(), n, g.ctypes.data, C.byref(loss),
                                        _stream(stream)), "reloc_mlp_gradient")
        return g, loss.value

    def train(self, x, y, epochs: int, batch_rows: int = 4096, lr: float = 1e-3, seed: int = 0,
              stream=None) -> np.ndarray:
        import torch
        n = int(y.numel())
        _dev_tensor(x, torch.int16, (n, 32))
        _dev_tensor(y, torch.uint8)
        losses = np.zeros(max(epochs, 1), dtype=np.float32)
        _check(lib().reloc_mlp_train(self._h, x.data_ptr(), y.data_ptr(), n, int(epochs), int(batch_rows),
                                     C.c_float(lr), C.c_uint64(seed), losses.ctypes.data, _stream(stream)),
               "reloc_mlp_train")
        return losses[:epochs]

    def logits(self, x, stream=None):
        import torch
        n = int(x.shape[0])
        _dev_tensor(x, torch.int16, (n, 32))
        z = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(lib().reloc_mlp_logits(self._h, x.data_ptr(), n, z.data_ptr(), _stream(stream)), "reloc_mlp_logits")
        return z

    def pixel_weights(self, forest: "Forest", depth, rgb, K, with_prob: bool = False, stream=None):
        """Pick weights (int32 GPU tensor [H*W], uint32 values) of every pixel
        of a query frame, and optionally the sigmoid outputs."""
        import torch
        d, c, k = _frame(depth, rgb, K)
        P = k.width * k.height
        w = torch.empty(P, dtype=torch.int32, device=depth.device)
        pr = torch.empty(P, dtype=torch.float32, device=depth.device) if with_prob else None
        _check(lib().reloc_mlp_pixel_weights(self._h, forest.handle, d, c, C.byref(k), w.data_ptr(),
                                             pr.data_ptr() if pr is not None else None, _stream(stream)),
               "reloc_mlp_pixel_weights")
        return (w, pr) if with_prob else w


# -- inter-agent scheduling and pose optimisation (host code in the library) ----


def relative_transform(pose_in_a, pose_in_b) -> np.ndarray:
    """a_T_b = pose_in_a pose_in_b^-1 (reloc_relative_transform)."""
    A, B = _pose(pose_in_a), _pose(pose_in_b)
    out = np.zeros(16)
    _check(lib().reloc_relative_transform(A.ctypes.data, B.ctypes.data, out.ctypes.data), "reloc_relative_transform")
    return out.reshape(4, 4)


class Collab:
    """Scheduling, clustering and pose-graph state of a collaborative session
    (reloc_collab)."""

    def __init__(self, n_scenes: int, seed: int = 0):
        self.n = int(n_scenes)
        self._h = C.c_void_p()
        _check(lib().reloc_collab_create(self.n, C.c_uint64(seed), C.byref(self._h)), "reloc_collab_create")

    def close(self) -> None:
        if self._h is not None and self._h.value and _lib is not None:
            _lib.reloc_collab_destroy(self._h)
        self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_frames(self, scene: int, poses) -> None:
        P = np.ascontiguousarray(np.asarray(poses, dtype=np.float64).reshape(-1, 16))
        _check(lib().reloc_collab_set_frames(self._h, int(scene), P.ctypes.data, len(P)), "reloc_collab_set_frames")

    def schedule(self, n_cand: int = 10):
        """(a, b, frame, candidates [n_cand, 7]: a, b, i, Phi, phi_new, phi_conf, phi_homog)."""
        a, b, i = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        cands = np.zeros((n_cand, 7), dtype=np.float32)
        _check(lib().reloc_collab_schedule(self._h, int(n_cand), C.byref(a), C.byref(b), C.byref(i),
                                           cands.ctypes.data), "reloc_collab_schedule")
        return a.value, b.value, i.value, cands

    def tried(self, a: int, b: int, frame: int) -> None:
        _check(lib().reloc_collab_tried(self._h, int(a), int(b), int(frame)), "reloc_collab_tried")

    def add_sample(self, a: int, b: int, a_T_b) -> int:
        T = _pose(a_T_b)
        size = C.c_int32(0)
        _check(lib().reloc_collab_add_sample(self._h, int(a), int(b), T.ctypes.data, C.byref(size)),
               "reloc_collab_add_sample")
        return size.value

    def clusters(self, a: int, b: int, cap: int = 256):
        """(sizes [k], blended a_T_b [k, 4, 4]) of the pair's clusters."""
        sizes = np.zeros(cap, dtype=np.int32)
        blended = np.zeros((cap, 16))
        n = C.c_int32(0)
        _check(lib().reloc_collab_clusters(self._h, int(a), int(b), sizes.ctypes.data, blended.ctypes.data, cap,
                                           C.byref(n)), "reloc_collab_clusters")
        k = min(n.value, cap)
        return sizes[:k].copy(), blended[:k].reshape(k, 4, 4).copy()

    def optimise(self):
        """(in_graph [n] bool, global poses [n, 4, 4], final cost)."""
        ing = np.zeros(self.n, dtype=np.int32)
        X = np.zeros((self.n, 16))
        cost = C.c_double(0)
        _check(lib().reloc_collab_optimise(self._h, ing.ctypes.data, X.ctypes.data, C.byref(cost)),
               "reloc_collab_optimise")
        return ing.astype(bool), X.reshape(self.n, 4, 4), cost.value
