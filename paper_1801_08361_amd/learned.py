"""Host side of the learned proposal: gathering labelled training rows from
posed frames and turning a trained network into pick weights. Every per-pixel
computation (inputs, labels, training, inference, verification) runs in the
library's kernels; this module only chooses frames and pixels and
concatenates device buffers.

Supervision: a frame whose pose is known (an agent's own tracked frame, or a
relocalisation accepted by the depth-difference check of Sec. 3.3.1,
Eqs. 3-4) labels each of its valid pixels with the probability that the
pixel's hypothesis pick is correct: the fraction of the colour-consistent
modes of its leaves that lie within 5 cm of the pixel's world point (uint8,
times 255)."""
from __future__ import annotations

from typing import Callable, Iterable, Optional, Tuple

import numpy as np

from . import Forest, Mlp, label_pixels, pixel_features, valid_pixels, verify


def frame_rows(forest: Forest, depth, rgb, K, pose, max_pixels: Optional[int] = None,
               seed: int = 0) -> Tuple["object", "object"]:
    """(inputs [n, 32] bfloat16 bits, labels [n] uint8) of the valid pixels of
    one posed frame, or of max_pixels of them drawn without replacement by a
    seeded numpy generator."""
    import torch
    pix = valid_pixels(forest, depth, rgb, K)
    if max_pixels is not None and pix.numel() > max_pixels:
        sel = np.sort(np.random.default_rng(seed).choice(pix.numel(), max_pixels, replace=False))
        pix = pix[torch.from_numpy(sel).to(pix.device)].contiguous()
    x = pixel_features(forest, depth, rgb, K, pix)
    y = label_pixels(forest, depth, rgb, K, pose, pix)
    return x, y


def training_rows(forest: Forest, frames: Iterable[tuple], max_pixels: Optional[int] = None, seed: int = 0):
    """Concatenated rows of frames given as (depth, rgb, K, pose) tuples."""
    import torch
    xs, ys = [], []
    for i, (d, c, K, pose) in enumerate(frames):
        x, y = frame_rows(forest, d, c, K, pose, max_pixels, seed + i)
        xs.append(x)
        ys.append(y)
    if not xs:
        raise ValueError("no frames")
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def verified_pose(forest: Forest, depth, rgb, K, seed: int, model_depth: Callable, n_hyp: int = 0):
    """Relocalises a frame and checks the result as the paper does before
    trusting it (Sec. 3.3.1, Eqs. 3-4): the scene model's depth rendered at
    the proposed pose (`model_depth(pose)` returns a device uint16 image of the
    same size) is the first image, whose valid fraction says whether the pose
    points at the modelled scene, and the frame's own depth the second.
    Returns (pose or None, result)."""
    r = forest.relocalise_ex(depth, rgb, K, seed=seed, n_hyp=n_hyp)
    if r["status"] != 0:
        return None, r
    vf, mu, ok = verify(model_depth(r["pose"]), depth)
    r["verify"] = (vf, mu, ok)
    return (r["pose"] if ok else None), r


def train(x, y, seed: int = 1, epochs: int = 8, batch_rows: int = 4096, lr: float = 2e-3) -> Tuple[Mlp, np.ndarray]:
    """A new network trained on the rows; returns it and the per-epoch loss."""
    m = Mlp(seed)
    losses = m.train(x, y, epochs=epochs, batch_rows=batch_rows, lr=lr, seed=seed)
    return m, losses
