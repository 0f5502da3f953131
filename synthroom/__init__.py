"""Seeded synthetic RGB-D rooms: the input generator shared by the CPU oracle
tests and the GPU path.

This module holds none of the relocaliser's arithmetic. It draws box rooms
with a procedural texture, smooth camera trajectories, and renders depth
(uint16 millimetres along the optical axis) and RGB8 frames for them. It
stands in for the 7-Scenes and ZenFone sequences the paper measures on
(Table 2, Sec. 4.2.2; dataset appendix), neither of which is available.

Conventions
-----------
* World frame: x, y horizontal, z up. A room is the box [0, Lx] x [0, Ly] x
  [0, Lz] seen from inside; furniture is axis-aligned boxes standing on the
  floor.
* Camera frame (OpenCV): x right, y down, z forward. A pose is a row-major
  float64 4x4 camera-to-world matrix; its translation column is the camera
  centre.
* Depth is the hit point's camera-frame z, rounded to the nearest mm; values
  outside [500, 5000] mm are written as 0 (invalid).
* Intrinsics at width W: fx = fy = 277 W / 320, cx = W / 2, cy = H / 2.

Rendering runs in float64 with torch, on whatever device the caller asks for
(CPU in the oracle tests, the GPU in the benchmark, where rendering 200
640x480 frames on the host would dominate the run). Results on the two
devices agree to the millimetre except for rare rounding ties.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

BASE_SEED = 180108361

DEPTH_MIN_MM = 500
DEPTH_MAX_MM = 5000


# ---------------------------------------------------------------------------
# seeds
# ---------------------------------------------------------------------------

def sub_seed(*tags: int) -> int:
    """Derives a 63-bit seed from the base seed and integer tags."""
    ss = np.random.SeedSequence([BASE_SEED, *[int(t) & 0xFFFFFFFF for t in tags]])
    return int(ss.generate_state(2, dtype=np.uint64)[0] >> np.uint64(1))


def rng(*tags: int) -> np.random.Generator:
    return np.random.default_rng(sub_seed(*tags))


# ---------------------------------------------------------------------------
# room description
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Room:
    size: np.ndarray            # (3,) metres
    boxes: np.ndarray           # (n, 2, 3): [min corner, max corner]
    face_rgb: np.ndarray        # (6 + 6n, 3) float base colour 0..255
    face_period: np.ndarray     # (6 + 6n,) stripe period (metres)
    face_seed: np.ndarray       # (6 + 6n,) int hash seed
    portals: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 2, 3)))

    @property
    def n_faces(self) -> int:
        return 6 + 6 * len(self.boxes)


def make_room(seed: int, size: Sequence[float] = (5.0, 4.0, 2.7), n_boxes: int = 6,
              side: Tuple[float, float] = (0.3, 1.2)) -> Room:
    """A box room with `n_boxes` axis-aligned boxes standing on the floor."""
    g = np.random.default_rng(seed)
    size = np.asarray(size, dtype=np.float64)
    boxes = np.zeros((n_boxes, 2, 3))
    for b in range(n_boxes):
        s = g.uniform(side[0], side[1], size=3)
        s[2] = g.uniform(side[0], min(side[1], 1.2))
        lo = np.array([g.uniform(0.0, size[0] - s[0]), g.uniform(0.0, size[1] - s[1]), 0.0])
        boxes[b, 0] = lo
        boxes[b, 1] = lo + s
    nf = 6 + 6 * n_boxes
    face_rgb = g.uniform(40.0, 215.0, size=(nf, 3))
    face_period = g.uniform(0.25, 0.9, size=nf)
    face_seed = g.integers(1, 1 << 30, size=nf)
    return Room(size=size, boxes=boxes, face_rgb=face_rgb, face_period=face_period,
                face_seed=face_seed)


def intrinsics(width: int, height: int) -> Tuple[float, float, float, float]:
    f = 277.0 * width / 320.0
    return (f, f, width / 2.0, height / 2.0)


# ---------------------------------------------------------------------------
# trajectories
# ---------------------------------------------------------------------------

def _catmull_rom(p: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Uniform Catmull-Rom through control points p (n, 3) at parameters s in
    [1, n - 2]."""
    i = np.clip(np.floor(s).astype(int), 1, len(p) - 3)
    u = (s - i)[:, None]
    p0, p1, p2, p3 = p[i - 1], p[i], p[i + 1], p[i + 2]
    return 0.5 * ((2 * p1) + (-p0 + p2) * u + (2 * p0 - 5 * p1 + 4 * p2 - p3) * u ** 2
                  + (-p0 + 3 * p1 - 3 * p2 + p3) * u ** 3)


def look_at(pos: np.ndarray, target: np.ndarray) -> np.ndarray:
    """Camera-to-world pose at `pos` looking at `target`, world z up."""
    z = target - pos
    z = z / np.linalg.norm(z)
    up = np.array([0.0, 0.0, 1.0])
    x = np.cross(z, up)
    x = x / np.linalg.norm(x)
    y = np.cross(z, x)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = x, y, z, pos
    return T


def _walk(g: np.random.Generator, n: int, lo: np.ndarray, hi: np.ndarray, step: float) -> np.ndarray:
    pts = np.zeros((n, 3))
    pts[0] = g.uniform(lo, hi)
    for k in range(1, n):
        for _ in range(64):
            d = g.normal(size=3)
            d[2] *= 0.3
            cand = pts[k - 1] + step * d / np.linalg.norm(d)
            if np.all(cand >= lo) and np.all(cand <= hi):
                break
        else:
            cand = np.clip(cand, lo, hi)
        pts[k] = cand
    return pts


def make_trajectory(room: Room, n_poses: int, seed: int, poses_per_segment: int = 5,
                    cam_step: float = 0.8, height: Tuple[float, float] = (1.3, 1.8),
                    region: Optional[Tuple[np.ndarray, np.ndarray]] = None) -> np.ndarray:
    """A smooth camera path of `n_poses` poses (n, 4, 4) with look-at targets.

    Camera centres follow a Catmull-Rom spline through a random walk of
    control points at `height` above the floor and at least 0.6 m from the
    walls (boxes are at most 1.2 m tall, so the camera never starts inside
    one); look-at targets follow a second spline through points inside the
    room, kept at least 1.2 m from the camera.
    """
    g = np.random.default_rng(seed)
    n_ctrl = int(math.ceil((n_poses - 1) / poses_per_segment)) + 3
    if region is None:
        lo = np.array([0.6, 0.6, height[0]])
        hi = np.array([room.size[0] - 0.6, room.size[1] - 0.6, height[1]])
    else:
        lo = np.array([region[0][0], region[0][1], height[0]])
        hi = np.array([region[1][0], region[1][1], height[1]])
    cams = _walk(g, n_ctrl, lo, hi, cam_step)
    tlo = np.array([0.2, 0.2, 0.2])
    thi = np.array([room.size[0] - 0.2, room.size[1] - 0.2, 1.4])
    tgts = _walk(g, n_ctrl, tlo, thi, 1.0)
    s = 1.0 + np.arange(n_poses) * (n_ctrl - 3) / max(n_poses - 1, 1)
    pos = _catmull_rom(cams, s)
    tgt = _catmull_rom(tgts, s)
    poses = np.zeros((n_poses, 4, 4))
    for k in range(n_poses):
        d = tgt[k] - pos[k]
        n = np.linalg.norm(d)
        if n < 1.2:
            # push the target away along the current direction (or +x)
            d = d / n if n > 1e-6 else np.array([1.0, 0.0, 0.0])
            tgt[k] = pos[k] + 1.2 * d
        if abs((tgt[k] - pos[k])[2]) > 0.95 * np.linalg.norm(tgt[k] - pos[k]):
            tgt[k][0] += 0.5
        poses[k] = look_at(pos[k], tgt[k])
    return poses


# ---------------------------------------------------------------------------
# texture
# ---------------------------------------------------------------------------

_M = 0xFFFFFFFF


def _hash3(a: torch.Tensor, b: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    """32-bit integer hash of int64 lattice coordinates, returned in [0, 1)."""
    h = ((a & _M) * 0x2545F491) & _M
    h = h ^ (((b & _M) * 0x6A09E667) & _M)
    h = h ^ (((s & _M) * 0x3C6EF372) & _M)
    h = h ^ (h >> 15)
    h = (h * 0x2C1B3C6D) & _M
    h = h ^ (h >> 12)
    h = (h * 0x297A2D39) & _M
    h = h ^ (h >> 15)
    return (h & 0xFFFFFF).to(torch.float64) / float(1 << 24)


def _value_noise(a: torch.Tensor, b: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    fa = torch.floor(a)
    fb = torch.floor(b)
    ia = fa.to(torch.int64)
    ib = fb.to(torch.int64)
    ta = a - fa
    tb = b - fb
    ta = ta * ta * (3 - 2 * ta)
    tb = tb * tb * (3 - 2 * tb)
    v00 = _hash3(ia, ib, s)
    v10 = _hash3(ia + 1, ib, s)
    v01 = _hash3(ia, ib + 1, s)
    v11 = _hash3(ia + 1, ib + 1, s)
    return (v00 * (1 - ta) + v10 * ta) * (1 - tb) + (v01 * (1 - ta) + v11 * ta) * tb


# ---------------------------------------------------------------------------
# renderer
# ---------------------------------------------------------------------------

_BIG = 1e30


def render(room: Room, pose: np.ndarray, width: int, height: int,
           device: str | torch.device = "cpu", noise_rel: float = 0.0,
           noise_seed: int = 0, K: Optional[Tuple[float, float, float, float]] = None
           ) -> Tuple[torch.Tensor, torch.Tensor]:
    """Ray-casts the room from `pose`.

    Returns (depth uint16 [H, W] in mm, rgb uint8 [H, W, 3]) on `device`.
    With noise_rel > 0 the camera-frame depth z is perturbed by
    N(0, (noise_rel * z)^2) before rounding (the 1 % Kinect-class model of
    the full-size workload).
    """
    dev = torch.device(device)
    f64 = torch.float64
    fx, fy, cx, cy = K if K is not None else intrinsics(width, height)
    v, u = torch.meshgrid(torch.arange(height, device=dev, dtype=f64),
                          torch.arange(width, device=dev, dtype=f64), indexing="ij")
    dc = torch.stack([(u - cx) / fx, (v - cy) / fy, torch.ones_like(u)], dim=-1).reshape(-1, 3)
    Rw = torch.as_tensor(pose[:3, :3], dtype=f64, device=dev)
    o = torch.as_tensor(pose[:3, 3], dtype=f64, device=dev)
    d = dc @ Rw.T                                       # (P, 3) world directions, t == camera z
    P = d.shape[0]
    inv = torch.where(d.abs() > 1e-15, 1.0 / d, torch.full_like(d, _BIG))

    # room interior: exit distance
    size = torch.as_tensor(room.size, dtype=f64, device=dev)
    bound = torch.where(d > 0, size.expand_as(d), torch.zeros_like(d))
    tk = torch.where(d.abs() > 1e-15, (bound - o) * inv, torch.full_like(d, _BIG))
    t_best, ax = tk.min(dim=1)
    face = 2 * ax + (d.gather(1, ax[:, None])[:, 0] > 0).to(torch.int64)

    for b in range(len(room.boxes)):
        bmin = torch.as_tensor(room.boxes[b, 0], dtype=f64, device=dev)
        bmax = torch.as_tensor(room.boxes[b, 1], dtype=f64, device=dev)
        t1 = (bmin - o) * inv
        t2 = (bmax - o) * inv
        tmin = torch.minimum(t1, t2)
        tmax = torch.maximum(t1, t2)
        tnear, axn = tmin.max(dim=1)
        tfar = tmax.min(dim=1).values
        hit = (tnear <= tfar) & (tnear > 1e-6) & (tnear < t_best)
        entered = 2 * axn + (d.gather(1, axn[:, None])[:, 0] < 0).to(torch.int64)
        t_best = torch.where(hit, tnear, t_best)
        face = torch.where(hit, 6 + 6 * b + entered, face)

    z = t_best
    if noise_rel > 0.0:
        gen = torch.Generator(device="cpu")
        gen.manual_seed(int(noise_seed) & ((1 << 63) - 1))
        n = torch.randn(P, generator=gen, dtype=f64).to(dev)
        z = z + noise_rel * z * n
    dmm = torch.round(z * 1000.0)
    valid = (dmm >= DEPTH_MIN_MM) & (dmm <= DEPTH_MAX_MM)
    depth = torch.where(valid, dmm, torch.zeros_like(dmm)).to(torch.int32).to(torch.uint16)

    # texture on the true (noise-free) hit point
    p = o + t_best[:, None] * d
    axis = face // 2
    a_idx = torch.where(axis == 0, 1, 0)
    b_idx = torch.where(axis == 2, 1, 2)
    pa = p.gather(1, a_idx[:, None])[:, 0]
    pb = p.gather(1, b_idx[:, None])[:, 0]
    fseed = torch.as_tensor(room.face_seed, dtype=torch.int64, device=dev)[face]
    fper = torch.as_tensor(room.face_period, dtype=f64, device=dev)[face]
    frgb = torch.as_tensor(room.face_rgb, dtype=f64, device=dev)[face]
    n1 = _value_noise(pa / 0.05, pb / 0.05, fseed)
    n2 = _value_noise(pa / 0.2, pb / 0.2, fseed + 7)
    stripe = 0.5 + 0.5 * torch.sin(2 * math.pi * (pa + 0.37 * pb) / fper)
    shade = 0.30 + 0.35 * n2 + 0.25 * n1 + 0.25 * stripe
    rgb = torch.clamp(torch.round(frgb * shade[:, None] * torch.stack(
        [0.9 + 0.2 * n1, 1.0 - 0.1 * n2, 0.85 + 0.3 * n2], dim=1)), 0, 255).to(torch.uint8)
    return depth.reshape(height, width), rgb.reshape(height, width, 3)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Scene:
    """One room with its trajectory split into adaptation and query poses."""
    room: Room
    adapt_poses: np.ndarray
    query_poses: np.ndarray
    width: int
    height: int
    noise_rel: float
    seed: int

    @property
    def K(self) -> Tuple[float, float, float, float]:
        return intrinsics(self.width, self.height)

    def render_adapt(self, k: int, device="cpu", width=None, height=None):
        w = width or self.width
        h = height or self.height
        return render(self.room, self.adapt_poses[k], w, h, device, self.noise_rel,
                      sub_seed(self.seed, 1, k))

    def render_query(self, k: int, device="cpu", width=None, height=None):
        w = width or self.width
        h = height or self.height
        return render(self.room, self.query_poses[k], w, h, device, self.noise_rel,
                      sub_seed(self.seed, 2, k))

    def render_query_synthetic(self, k: int, device="cpu", width=None, height=None):
        """A noise-free raycast of the room from query pose k: the synthetic
        RGB-D image of an agent's reconstructed scene that inter-agent
        relocalisation relocalises (Sec. 3.3.1, Fig. 4) instead of a sensor
        frame."""
        w = width or self.width
        h = height or self.height
        return render(self.room, self.query_poses[k], w, h, device, 0.0, 0)

    def extra_poses(self, n: int, tag: int = 0) -> np.ndarray:
        """A second camera path of n poses in the same room (for frames that
        neither adapt the forest nor serve as held-out queries)."""
        return make_trajectory(self.room, n, sub_seed(self.seed, 13, tag))

    def render_pose(self, pose: np.ndarray, noise_tag: int, device="cpu", width=None, height=None):
        """A sensor frame (with the scene's depth noise) from an arbitrary pose."""
        w = width or self.width
        h = height or self.height
        return render(self.room, pose, w, h, device, self.noise_rel, sub_seed(self.seed, 3, noise_tag))

    def model_depth(self, pose: np.ndarray, device="cpu", width=None, height=None):
        """Noise-free depth of the room model from `pose` (the rendering a
        proposed pose is verified against)."""
        w = width or self.width
        h = height or self.height
        return render(self.room, pose, w, h, device, 0.0, 0)[0]


def small_scene(index: int, width: int = 320, height: int = 240) -> Scene:
    """Single-relocalisation workload: a 5 x 4 x 2.7 m room with 6 boxes, a
    40-pose path; even poses adapt the forest (20 frames), odd poses are
    held-out queries (20)."""
    seed = sub_seed(1, index)
    room = make_room(sub_seed(seed, 10), (5.0, 4.0, 2.7), 6)
    traj = make_trajectory(room, 40, sub_seed(seed, 11))
    return Scene(room, traj[0::2].copy(), traj[1::2].copy(), width, height, 0.0, seed)


def full_scene(index: int = 0) -> Scene:
    """Full-size workload: a 6 x 8 x 3 m room with 30 boxes at 640 x 480,
    f = 554, depth noise sigma = 1 % of z; a 250-pose path of which every
    fifth pose (offset 2) is a held-out query: 200 adaptation frames and 50
    queries."""
    seed = sub_seed(2, index)
    room = make_room(sub_seed(seed, 10), (6.0, 8.0, 3.0), 30)
    traj = make_trajectory(room, 250, sub_seed(seed, 11))
    q = np.arange(250) % 5 == 2
    return Scene(room, traj[~q].copy(), traj[q].copy(), 640, 480, 0.01, seed)


def batched_attempts(n_attempts: int = 64, n_forests: int = 8, seed_tag: int = 3):
    """Mixed-size attempt list for the batched workload: each attempt picks a
    forest (scene) uniformly, a frame size from {320x240, 480x360, 640x480}
    and a hypothesis count from {256, 512, 1024}, and one of that scene's
    held-out query poses."""
    g = rng(seed_tag, n_attempts, n_forests)
    sizes = [(320, 240), (480, 360), (640, 480)]
    hyps = [256, 512, 1024]
    out = []
    for a in range(n_attempts):
        f = int(g.integers(0, n_forests))
        s = sizes[int(g.integers(0, 3))]
        n = hyps[int(g.integers(0, 3))]
        q = int(g.integers(0, 20))
        out.append(dict(forest=f, width=s[0], height=s[1], n_hyp=n, query=q,
                        seed=int(g.integers(1, 1 << 62))))
    return out


def queue_attempts(n_attempts: int, n_forests: int, n_queries: int, overlap: float = 0.3, seed_tag: int = 5):
    """Cross-agent attempt queue: each attempt targets a forest uniformly; with
    probability `overlap` its frame comes from the target's own room (a held-out
    query pose of that room, so a correct relocalisation exists), otherwise
    from another room (the correct outcome is a rejection). Frame sizes are
    uniform over {320x240, 480x360, 640x480}."""
    g = rng(seed_tag, n_attempts, n_forests)
    sizes = [(320, 240), (480, 360), (640, 480)]
    out = []
    for a in range(n_attempts):
        f = int(g.integers(0, n_forests))
        same = bool(g.random() < overlap)
        src = f if same else int((f + 1 + g.integers(0, n_forests - 1)) % n_forests)
        s = sizes[int(g.integers(0, 3))]
        out.append(dict(forest=f, source=src, overlap=same, width=s[0], height=s[1],
                        query=int(g.integers(0, n_queries)), seed=int(g.integers(1, 1 << 62))))
    return out


def collaborative_session(n_agents: int = 3, index: int = 0, n_poses: int = 40, width: int = 320, height: int = 240):
    """Several agents reconstructing one room, each in its own sub-scene
    coordinate frame: the room of small_scene(index) and one camera path
    through it, of which agent k walks poses [k n_poses / 2, k n_poses / 2 +
    n_poses) (consecutive agents share half of their paths, as agents whose
    sub-scenes overlap), and per agent a random rigid transform W that maps
    its sub-scene coordinates to the room's. An agent's local poses are W^-1
    times its world poses. Returns (scene, world poses [n_agents][n_poses],
    W [n_agents])."""
    sc = small_scene(index, width, height)
    g = rng(17, index, n_agents)
    half = n_poses // 2
    path = make_trajectory(sc.room, half * (n_agents - 1) + n_poses, sub_seed(sc.seed, 21))
    world, frames = [], []
    for k in range(n_agents):
        world.append(path[k * half:k * half + n_poses].copy())
        q = g.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        W = np.eye(4)
        W[:3, :3] = [[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]]
        W[:3, 3] = g.uniform(-3.0, 3.0, size=3)
        frames.append(W)
    return sc, world, frames
