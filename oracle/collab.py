"""Plain oracle of the inter-agent steps around the relocaliser (Sec. 3.3.1,
Sec. 3.3.2, Sec. 4.2.3-4.2.4): relative transform samples, candidate scoring,
incremental clustering, dual-quaternion blending, the pose graph and its
Levenberg-Marquardt optimisation.

TEST INFRASTRUCTURE ONLY: used by the tests to say what the library's host
code must compute; the product never imports it. Written with numpy and
scipy (Rotation for quaternions, least_squares for the optimisation) in
float64, one step per function, in the paper's order. Conventions are the
library's: poses are 4x4 camera-to-world matrices of a frame in one
sub-scene; aT_b maps sub-scene b's coordinates to a's; gT_s maps sub-scene
s's coordinates to the global (scene 0's) frame.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np
from scipy.optimize import least_squares
from scipy.spatial.transform import Rotation

N_CONFIDENT = 2          # Eq. 2: samples before a pair's relative transform is confident
HOMOG_PENALTY = 5.0      # phi_homog for a frame too close to one already tried
TAG_SCHEDULE = 7


def relative_transform(pose_in_a: np.ndarray, pose_in_b: np.ndarray) -> np.ndarray:
    """aT_b of a frame relocalised in a with pose pose_in_a and known pose
    pose_in_b in b: the paper's (fT_a)^-1 fT_b with fT_s = pose_in_s^-1."""
    return np.linalg.inv(np.linalg.inv(pose_in_a)) @ np.linalg.inv(pose_in_b)


def angle_deg(Ra: np.ndarray, Rb: np.ndarray) -> float:
    return float(np.degrees(Rotation.from_matrix(Ra.T @ Rb).magnitude()))


def close(Ta: np.ndarray, Tb: np.ndarray, deg: float, m: float) -> bool:
    return angle_deg(Ta[:3, :3], Tb[:3, :3]) <= deg and float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3])) <= m


def vee(T: np.ndarray) -> np.ndarray:
    """v(T): imaginary part of T's rotation quaternion (real part >= 0), then
    T's translation (Eq. 5)."""
    x, y, z, w = Rotation.from_matrix(T[:3, :3]).as_quat()
    if w < 0:
        x, y, z = -x, -y, -z
    return np.array([x, y, z, *T[:3, 3]])


def dq_blend(Ts: Sequence[np.ndarray]) -> np.ndarray:
    """Equal-weight dual-quaternion linear blending (Kavan et al. 2006): unit
    dual quaternions q_r + eps q_d with q_d = (0, t) q_r / 2, signs aligned
    to the first, averaged, divided by the norm of the real part; rotation
    from the real part, translation from 2 q_d conj(q_r)."""

    def qmul(a, b):   # (w, x, y, z)
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])

    reals, duals = [], []
    for T in Ts:
        x, y, z, w = Rotation.from_matrix(T[:3, :3]).as_quat()
        qr = np.array([w, x, y, z])
        qd = 0.5 * qmul(np.array([0.0, *T[:3, 3]]), qr)
        if reals and float(qr @ reals[0]) < 0:
            qr, qd = -qr, -qd
        reals.append(qr)
        duals.append(qd)
    br = np.mean(reals, axis=0)
    bd = np.mean(duals, axis=0)
    n = np.linalg.norm(br)
    br, bd = br / n, bd / n
    out = np.eye(4)
    out[:3, :3] = Rotation.from_quat([br[1], br[2], br[3], br[0]]).as_matrix()
    conj = np.array([br[0], -br[1], -br[2], -br[3]])
    out[:3, 3] = 2.0 * qmul(bd, conj)[1:]
    return out


def connected_component(n: int, edges: Sequence[Tuple[int, int]], root: int = 0) -> List[int]:
    """Nodes reachable from `root` (breadth first)."""
    seen = {root}
    frontier = [root]
    while frontier:
        nxt = []
        for s in frontier:
            for a, b in edges:
                for u, v in ((a, b), (b, a)):
                    if u == s and v not in seen:
                        seen.add(v)
                        nxt.append(v)
        frontier = nxt
    return sorted(seen)


def verifier_stats(tp: int, fp: int, tn: int, fn: int) -> Tuple[float, float, float]:
    """Precision, recall and specificity of the depth-difference check
    (Table 3's columns)."""
    return tp / (tp + fp), tp / (tp + fn), tn / (tn + fp)


def cluster_stats(samples: int, correct: int, incorrect: int) -> Tuple[float, float, int]:
    """Shares of the correct cluster and the largest incorrect one among the
    samples added, and the safety margin (Table 4's columns)."""
    return correct / samples, incorrect / samples, correct - incorrect


class Session:
    """The state the library's reloc_collab keeps, in plain Python."""

    def __init__(self, n_scenes: int, seed: int):
        self.n = n_scenes
        self.seed = seed
        self.rounds = 0
        self.frames: Dict[int, np.ndarray] = {}
        self.tried: Dict[Tuple[int, int], List[int]] = {}
        self.clusters: Dict[Tuple[int, int], List[List[np.ndarray]]] = {}
        self.in_graph = np.zeros(n_scenes, dtype=bool)

    def set_frames(self, scene: int, poses) -> None:
        self.frames[scene] = np.asarray(poses, dtype=np.float64).reshape(-1, 4, 4).copy()

    def _pair(self, a: int, b: int):
        return self.clusters.setdefault((min(a, b), max(a, b)), [])

    def score(self, a: int, b: int, i: int) -> Tuple[float, float, float, float]:
        """Phi = phi_new - phi_conf - phi_homog (Eqs. 1-2)."""
        phi_new = 1.0 if bool(self.in_graph[a]) != bool(self.in_graph[b]) else 0.0
        phi_conf = float(max([0] + [len(c) - N_CONFIDENT for c in self._pair(a, b)]))
        P = self.frames[b][i]
        phi_homog = HOMOG_PENALTY if any(close(P, self.frames[b][j], 5.0, 0.05)
                                         for j in self.tried.get((a, b), [])) else 0.0
        return phi_new - phi_conf - phi_homog, phi_new, phi_conf, phi_homog

    def schedule(self, n_cand: int):
        """Candidates (a, (b, i)): a pair of scenes uniformly, then a frame of
        b uniformly, from Philox (seed, 7) at counter (round, j, 0, 0); the
        best-scoring (first on ties) is returned with all candidates."""
        import oracle
        cands = []
        for j in range(n_cand):
            u = oracle.philox([self.rounds, j, 0, 0], [self.seed, TAG_SCHEDULE])
            p = oracle.uniform_int(int(u[0]), self.n * (self.n - 1))
            a, r = divmod(p, self.n - 1)
            b = r if r < a else r + 1
            i = oracle.uniform_int(int(u[1]), len(self.frames[b]))
            cands.append((a, b, i, *self.score(a, b, i)))
        self.rounds += 1
        best = max(range(n_cand), key=lambda j: (cands[j][3], -j))
        return cands[best][:3], cands

    def mark_tried(self, a: int, b: int, i: int) -> None:
        self.tried.setdefault((a, b), []).append(i)

    def add_sample(self, a: int, b: int, aTb: np.ndarray) -> int:
        """Incremental clustering (Sec. 4.2.4): the first cluster holding a
        sample within 20 deg and 10 cm, else a new cluster; samples of the
        pair kept as loT_hi."""
        x = aTb if a < b else np.linalg.inv(aTb)
        cl = self._pair(a, b)
        for c in cl:
            if any(close(x, y, 20.0, 0.10) for y in c):
                c.append(x)
                return len(c)
        cl.append([x])
        return 1

    def edges(self):
        """G': (a, b, blended aT_b) for pairs whose largest (earliest on ties)
        cluster holds at least N samples."""
        out = []
        for (a, b), cl in sorted(self.clusters.items()):
            if not cl:
                continue
            big = max(range(len(cl)), key=lambda k: (len(cl[k]), -k))
            if len(cl[big]) >= N_CONFIDENT:
                out.append((a, b, dq_blend(cl[big])))
        return out

    def optimise(self):
        """G = the component of G' holding scene 0; minimise the sum over its
        edges of |v(gT_b^-1 gT_a aT_b)|^2 with gT_0 = I (Eq. 5; Levenberg-
        Marquardt through scipy's least_squares), each other node's pose
        parameterised by its rotation vector and translation."""
        edges = self.edges()
        nodes = connected_component(self.n, [(a, b) for a, b, _ in edges])
        ge = [(a, b, T) for a, b, T in edges if a in nodes]
        X = {0: np.eye(4)}
        frontier = [0]
        while frontier:   # initial poses chained from scene 0
            nxt = []
            for s in frontier:
                for a, b, T in ge:
                    if a == s and b not in X:
                        X[b] = X[a] @ T
                        nxt.append(b)
                    elif b == s and a not in X:
                        X[a] = X[b] @ np.linalg.inv(T)
                        nxt.append(a)
            frontier = nxt
        free = [s for s in nodes if s != 0]

        def unpack(p):
            Y = {0: np.eye(4)}
            for k, s in enumerate(free):
                M = np.eye(4)
                M[:3, :3] = Rotation.from_rotvec(p[6 * k:6 * k + 3]).as_matrix()
                M[:3, 3] = p[6 * k + 3:6 * k + 6]
                Y[s] = M
            return Y

        def res(p):
            Y = unpack(p)
            return np.concatenate([vee(np.linalg.inv(Y[b]) @ Y[a] @ T) for a, b, T in ge]) if ge else np.zeros(0)

        p0 = np.concatenate([np.concatenate([Rotation.from_matrix(X[s][:3, :3]).as_rotvec(), X[s][:3, 3]])
                             for s in free]) if free else np.zeros(0)
        if free and len(res(p0)) >= len(p0):
            sol = least_squares(res, p0, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=20000)
            p0 = sol.x
        Y = unpack(p0)
        self.in_graph = np.zeros(self.n, dtype=bool)
        self.in_graph[nodes] = True
        poses = np.stack([Y.get(s, np.eye(4)) for s in range(self.n)])
        r = res(p0)
        return self.in_graph.copy(), poses, float(r @ r)
