"""Independent re-statements used to pin the oracle in the CPU tests.

Nothing here is called by the oracle or by the GPU path. Each helper restates
one step of the method by other means (numpy's own Philox, numpy float32
arithmetic, a rank-and-scatter formulation of the reservoir update), so that
a mistake in the oracle's C code shows up as a disagreement.
"""
from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1


def np_philox(ctr, key):
    """Philox4x64-10 block for counter `ctr` via numpy.random.Philox.

    numpy advances its 256-bit counter before producing a block, so the block
    for counter c is the first output of a generator started at c - 1."""
    c = [int(x) & M64 for x in ctr]
    # subtract one with borrow across the four words
    i = 0
    while i < 4:
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = M64
        i += 1
    bg = np.random.Philox(key=np.array([int(k) & M64 for k in key], dtype=np.uint64),
                          counter=np.array(c, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def np_uniform_int(u: int, n: int) -> int:
    return (int(u) * int(n)) >> 64


def cam_points_f32(depth: np.ndarray, K) -> np.ndarray:
    """Camera points in float32, one IEEE op at a time in the defined order."""
    H, W = depth.shape
    fx, fy, cx, cy = (np.float32(k) for k in K)
    v, u = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    z = depth.astype(np.float32) * np.float32(0.001)
    x = ((u.astype(np.float32) - cx) * z) / fx
    y = ((v.astype(np.float32) - cy) * z) / fy
    return np.stack([x, y, z], axis=-1).reshape(-1, 3)


def world_mm_f32(cam: np.ndarray, pose: np.ndarray) -> np.ndarray:
    R = pose[:3, :3].astype(np.float32)
    t = pose[:3, 3].astype(np.float32)
    out = np.zeros((len(cam), 3), dtype=np.int32)
    for k in range(3):
        w = ((R[k, 0] * cam[:, 0] + R[k, 1] * cam[:, 1]) + R[k, 2] * cam[:, 2]) + t[k]
        out[:, k] = np.rint(w * np.float32(1000.0)).astype(np.int32)
    return out


def reservoir_by_ranks(frames, leaves_fn, K, seed, T, L, R, dmin=500, dmax=5000):
    """Reservoir contents after a sequence of posed frames, computed per frame
    by stable per-leaf ranks and a 'largest k wins each slot' scatter instead
    of one pixel at a time. Returns (entries [T][L][R] x (x, y, z, r, g, b),
    counters [T][L])."""
    ent = np.zeros((T, L, R, 6), dtype=np.int64)
    cnt = np.zeros((T, L), dtype=np.int64)
    for depth, rgb, pose in frames:
        leaves = leaves_fn(depth, rgb)                   # [T][P]
        d = depth.reshape(-1).astype(np.int64)
        valid = (d >= dmin) & (d <= dmax)
        q = world_mm_f32(cam_points_f32(depth, K), pose)
        col = rgb.reshape(-1, 3).astype(np.int64)
        pix = np.flatnonzero(valid)
        for t in range(T):
            lf = leaves[t, pix]
            order = np.argsort(lf, kind="stable")
            sl = lf[order]
            start = np.searchsorted(sl, sl, side="left")
            rank = np.empty(len(pix), dtype=np.int64)
            rank[order] = np.arange(len(pix)) - start
            k = cnt[t, lf] + rank
            best = {}
            for i in range(len(pix)):
                kk = int(k[i])
                if kk < R:
                    slot = kk
                else:
                    u = np_philox((t, int(lf[i]), kk, 0), (seed, 2))[0]
                    j = np_uniform_int(u, kk + 1)
                    if j >= R:
                        continue
                    slot = j
                key = (int(lf[i]), slot)
                if key not in best or best[key][0] < kk:
                    best[key] = (kk, int(pix[i]))
            for (leaf, slot), (_, p) in best.items():
                ent[t, leaf, slot, :3] = q[p]
                ent[t, leaf, slot, 3:] = col[p]
            np.add.at(cnt[t], lf, 1)
    return ent, cnt


def rand_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def horn_rotation(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """Horn's closed-form quaternion solution (1987): the optimal rotation is
    the eigenvector of the largest eigenvalue of a symmetric 4x4 matrix."""
    a = src - src.mean(0)
    b = dst - dst.mean(0)
    S = a.T @ b
    Sxx, Sxy, Sxz = S[0]
    Syx, Syy, Syz = S[1]
    Szx, Szy, Szz = S[2]
    N = np.array([
        [Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx],
        [Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz],
        [Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy],
        [Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz],
    ])
    w, V = np.linalg.eigh(N)
    q = V[:, np.argmax(w)]
    q0, qx, qy, qz = q
    return np.array([
        [q0 * q0 + qx * qx - qy * qy - qz * qz, 2 * (qx * qy - q0 * qz), 2 * (qx * qz + q0 * qy)],
        [2 * (qy * qx + q0 * qz), q0 * q0 - qx * qx + qy * qy - qz * qz, 2 * (qy * qz - q0 * qx)],
        [2 * (qz * qx - q0 * qy), 2 * (qz * qy + q0 * qx), q0 * q0 - qx * qx - qy * qy + qz * qz],
    ])
