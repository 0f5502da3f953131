"""Throughput of forest relocalisation on one MI355X.

Workload (the full-size configuration): a 6 x 8 x 3 m synthetic room with 30
boxes rendered at 640 x 480 (f = 554, depth noise 1 % of z), a forest of 5
trees of depth 15 with 1024-entry reservoirs adapted on 200 posed frames,
relocalised with 1024 hypotheses and 500 pixels per cull round. Frames are
resident in HBM and the forest is adapted and its modes built before the
timed region. A step relocalises the 50 held-out query frames (one plain
call each); `value` is relocalisations per second over the timed steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 78.6     # non-packed FP32 FMA rate: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def full_workload(dev):
    import torch
    import synthroom as sr
    sc = sr.full_scene(0)
    adapt = [sc.render_adapt(k, device=dev) for k in range(len(sc.adapt_poses))]
    queries = [sc.render_query(k, device=dev) for k in range(len(sc.query_poses))]
    torch.cuda.synchronize()
    return sc, adapt, queries


def gpu_params():
    import paper_1801_08361_amd as rl
    return rl.params_default(n_trees=5, depth=15, reservoir_size=1024, max_modes=10, n_hypotheses=1024,
                             batch_pixels=500)


def cpu_baseline(sc, budget_s: float = 25.0):
    """The CPU oracle (single thread) on a bounded sample of the same workload:
    a forest with the same parameters adapted on every 10th adaptation frame
    (20 frames), then relocalisation of held-out queries. Lazily built leaf
    modes are computed by an untimed first call per query; the timed call
    repeats it with the modes cached (the GPU times relocalisation with its
    modes built, too)."""
    import oracle
    import synthroom as sr
    po = oracle.default_params()
    gp = gpu_params()
    for f in ("n_trees", "depth", "reservoir_size", "max_modes", "n_hypotheses", "batch_pixels"):
        setattr(po, f, getattr(gp, f))
    o = oracle.Forest(po)
    t0 = time.time()
    frames = list(range(0, len(sc.adapt_poses), 10))
    for k in frames:
        d, c = sc.render_adapt(k)
        o.adapt(d, c, sc.K, sc.adapt_poses[k])
    log(f"oracle adapted {len(frames)} frames in {time.time() - t0:.1f}s")
    n = 0
    timed = 0.0
    ok = 0
    for q in range(0, len(sc.query_poses), 5):
        d, c = sc.render_query(q)
        o.relocalise(d, c, sc.K, seed=1 + q)
        t = time.perf_counter()
        st, T, _, _ = o.relocalise(d, c, sc.K, seed=1 + q)
        timed += time.perf_counter() - t
        n += 1
        ok += int(st == 0 and oracle.pose_success(T, sc.query_poses[q])[0])
        if timed > budget_s or time.time() - t0 > 3 * budget_s:
            break
    return {"value": n / timed, "unit": "relocalisations/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} held-out 640x480 queries relocalised (N=1024, B=500) against a forest adapted on "
                      f"{len(frames)} of the 200 frames; modes cached by an untimed first call; "
                      f"{ok}/{n} within 5 cm/5 deg"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (every box here has one GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1801_08361_amd as rl
    import synthroom as sr

    dev = torch.device("cuda:0")
    t0 = time.time()
    sc, adapt, queries = full_workload(dev)
    log(f"rendered {len(adapt)} + {len(queries)} frames in {time.time() - t0:.1f}s")
    g = rl.Forest(gpu_params())
    t0 = time.time()
    for k, (d, c) in enumerate(adapt):
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
    torch.cuda.synchronize()
    t_adapt = time.time() - t0
    t0 = time.time()
    g.update_modes()
    torch.cuda.synchronize()
    t_modes = time.time() - t0
    log(f"adapted {len(adapt)} frames in {t_adapt:.2f}s, modes in {t_modes:.2f}s")

    def step(seed0):
        res = []
        for q, (d, c) in enumerate(queries):
            st, T, score = g.relocalise(d, c, sc.K, seed=seed0 + q)
            res.append((st, T))
        return res

    for w in range(args.warmup):
        step(1000 * (w + 1))
        log(f"warmup {w} done")
    torch.cuda.synchronize()
    rl.profile_reset()
    rl.profile_enable(True)
    ok = tot = 0
    t0 = time.perf_counter()
    for s in range(args.steps):
        res = step(1)
        for q, (st, T) in enumerate(res):
            import oracle as _  # noqa: F401  (not used: success is checked against ground truth below)
        for q, (st, T) in enumerate(res):
            dt = np.linalg.norm(T[:3, 3] - sc.query_poses[q][:3, 3])
            Q = T[:3, :3].T @ sc.query_poses[q][:3, :3]
            ang = np.degrees(np.arccos(np.clip((np.trace(Q) - 1) / 2, -1, 1)))
            ok += int(st == 0 and dt <= 0.05 and ang <= 5.0)
            tot += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rl.profile_enable(False)
    n_att = args.steps * len(queries)
    kernels = {}
    for k in rl.profile_kernels():
        ms, n = rl.profile_read(k)
        kernels[k] = (ms, n)
    log("kernel totals over the timed region: " +
        ", ".join(f"{k}={v[0]:.2f}ms/{v[1]}" for k, v in sorted(kernels.items(), key=lambda kv: -kv[1][0])))
    dom = max(kernels.items(), key=lambda kv: kv[1][0])
    out = {
        "metric": "relocalisations/sec at >=95% success (<=5cm/5deg), plain vs batched+learned",
        "value": n_att / wall,
        "unit": "relocalisations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "full-size plain: 640x480 room 6x8x3 m, 30 boxes, 1% depth noise; 5 trees depth 15, "
                               "R=1024, 200 adaptation frames; N=1024 hypotheses, B=500 pixels per round; "
                               "step = 50 held-out queries, one plain call each"},
        "success_rate": ok / max(tot, 1),
        "dominant_kernel": {"name": dom[0], "ms_total": dom[1][0], "launches": dom[1][1]},
        "kernels_ms": {k: round(v[0], 4) for k, v in kernels.items()},
        "adapt_frames_per_s": len(adapt) / t_adapt,
    }
    out["roofline"] = None
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
