"""Throughput of forest relocalisation on one MI355X.

Headline workload (the full-size configuration): a 6 x 8 x 3 m synthetic
room with 30 boxes rendered at 640 x 480 (f = 554, depth noise 1 % of z), a
forest of 5 trees of depth 15 with 1024-entry reservoirs adapted on 200 posed
frames, relocalised with 1024 hypotheses and 500 pixels per cull round.
Frames are resident in HBM and the forest is adapted and its modes built
before the timed region. A step relocalises the 50 held-out query frames
(one plain call each); `value` is relocalisations per second over the timed
steps.

Also reported (same JSON line, `forms`): the batched form on the mixed
workload (64 attempts against 8 small-room forests, frame sizes drawn from
320x240 / 480x360 / 640x480 and hypothesis counts from 256 / 512 / 1024), as
one batched call versus 64 sequential plain calls.

Per-kernel times come from a separate profiled pass over the same steps
(HIP events around each launch on its stream; kernels are then launched one
by one instead of as a graph). The roofline line is for the scoring kernel:
its algorithmic FLOPs (25 per (hypothesis, draw, mode) energy term, 18 per
(hypothesis, draw) transform, counted by the kernels themselves) over its
average duration.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batched]
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

FP32_PEAK_TFLOPS = 157.3          # MI355X vector FP32 (published; packed FP32)
FLOP_PER_MODE_TERM = 25           # d: 3 sub; Sigma^-1 d: 3 mul + 6 fma; q: 1 mul + 2 fma; term: 1 fma
FLOP_PER_PAIR = 18                # y = R c + t: 9 fma


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def full_params():
    import paper_1801_08361_amd as rl
    return rl.params_default(n_trees=5, depth=15, reservoir_size=1024, max_modes=10, n_hypotheses=1024,
                             batch_pixels=500)


def small_params():
    import paper_1801_08361_amd as rl
    return rl.params_default(n_trees=5, depth=10, reservoir_size=256, max_modes=10, n_hypotheses=256,
                             batch_pixels=64)


def success(T, gt) -> bool:
    import numpy as np
    dt = float(np.linalg.norm(T[:3, 3] - gt[:3, 3]))
    Q = T[:3, :3].T @ gt[:3, :3]
    v = np.array([Q[2, 1] - Q[1, 2], Q[0, 2] - Q[2, 0], Q[1, 0] - Q[0, 1]])
    ang = float(np.degrees(np.arctan2(0.5 * np.linalg.norm(v), 0.5 * (np.trace(Q) - 1.0))))
    return dt <= 0.05 and ang <= 5.0


def cpu_baseline(sc, budget_s: float = 25.0):
    """The CPU oracle (single thread) on a bounded sample of the same workload:
    a forest with the same parameters adapted on every 10th adaptation frame
    (20 frames), then relocalisation of held-out queries. Lazily built leaf
    modes are computed by an untimed first call per query; the timed call
    repeats it with the modes cached (the GPU is timed with its modes built)."""
    import oracle
    po = oracle.default_params()
    gp = full_params()
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
        ok += int(st == 0 and success(T, sc.query_poses[q]))
        if timed > budget_s or time.time() - t0 > 3 * budget_s:
            break
    return {"value": n / timed, "unit": "relocalisations/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} held-out 640x480 queries relocalised (N=1024, B=500) against a forest adapted on "
                      f"{len(frames)} of the 200 frames; modes cached by an untimed first call; "
                      f"{ok}/{n} within 5 cm/5 deg"}


def plain_full(args, dev):
    import torch
    import paper_1801_08361_amd as rl
    import synthroom as sr
    t0 = time.time()
    sc = sr.full_scene(0)
    adapt = [sc.render_adapt(k, device=dev) for k in range(len(sc.adapt_poses))]
    queries = [sc.render_query(k, device=dev) for k in range(len(sc.query_poses))]
    torch.cuda.synchronize()
    log(f"rendered {len(adapt)} + {len(queries)} frames in {time.time() - t0:.1f}s")
    g = rl.Forest(full_params())
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

    def step():
        return [g.relocalise_ex(d, c, sc.K, seed=1 + q) for q, (d, c) in enumerate(queries)]

    for w in range(args.warmup):
        step()
        log(f"warmup {w} done")
    torch.cuda.synchronize()
    ok = tot = 0
    t0 = time.perf_counter()
    for s in range(args.steps):
        res = step()
        for q, r in enumerate(res):
            ok += int(r["status"] == 0 and success(r["pose"], sc.query_poses[q]))
            tot += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"plain full: {tot / wall:.1f} relocalisations/s, success {ok}/{tot}")

    # profiled pass: the same step with per-kernel events
    rl.profile_reset()
    rl.profile_enable(True)
    res = step()
    torch.cuda.synchronize()
    rl.profile_enable(False)
    kernels = {k: rl.profile_read(k) for k in rl.profile_kernels()}
    rl.profile_reset()
    flops = sum(r["mode_evals"] * FLOP_PER_MODE_TERM + r["pair_evals"] * FLOP_PER_PAIR for r in res)
    sc_ms, sc_n = kernels.get("k_b_score", (0.0, 0))
    log("kernel totals over one profiled step: " +
        ", ".join(f"{k}={v[0]:.2f}ms/{v[1]}" for k, v in sorted(kernels.items(), key=lambda kv: -kv[1][0])))
    roof = None
    if sc_n:
        avg_s = sc_ms / sc_n * 1e-3
        achieved = flops / sc_n / avg_s / 1e12
        roof = {"kernel": "k_b_score", "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                "avg_launch_us": avg_s * 1e6, "flops_per_launch": flops / sc_n}
    return dict(sc=sc, value=tot / wall, wall=wall, success=ok / max(tot, 1), n=tot, kernels=kernels, roof=roof,
                adapt_fps=len(adapt) / t_adapt, modes_s=t_modes, mem=g.memory())


def batched_mixed(args, dev):
    import torch
    import paper_1801_08361_amd as rl
    import synthroom as sr
    t0 = time.time()
    n_forests = 8
    scenes = [sr.small_scene(500 + k) for k in range(n_forests)]
    forests = []
    for sc in scenes:
        g = rl.Forest(small_params())
        for k in range(len(sc.adapt_poses)):
            d, c = sc.render_adapt(k, device=dev)
            g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        g.update_modes()
        forests.append(g)
    plan = sr.batched_attempts(64, n_forests)
    att, gts = [], []
    for a in plan:
        sc = scenes[a["forest"]]
        d, c = sc.render_query(a["query"], device=dev, width=a["width"], height=a["height"])
        att.append(dict(forest=forests[a["forest"]], depth=d.contiguous(), rgb=c.contiguous(),
                        K=sr.intrinsics(a["width"], a["height"]), seed=a["seed"], n_hyp=a["n_hyp"]))
        gts.append(sc.query_poses[a["query"]])
    torch.cuda.synchronize()
    log(f"batched workload ready in {time.time() - t0:.1f}s")
    b = rl.Batch(tune=True)
    for w in range(max(1, args.warmup)):
        b.run(att)
    log(f"batched schedule: {b.schedule()}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        res = b.run(att)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0

    def seq():
        return [a["forest"].relocalise_ex(a["depth"], a["rgb"], a["K"], seed=a["seed"], n_hyp=a["n_hyp"])
                for a in att]

    seq()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        res_p = seq()
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t0
    import numpy as np
    identical = all(r["status"] == p["status"] and np.array_equal(r["pose"], p["pose"]) and r["score"] == p["score"]
                    for r, p in zip(res, res_p))
    ok = sum(int(r["status"] == 0 and success(r["pose"], gt)) for r, gt in zip(res, gts))
    n = len(att) * args.steps
    log(f"batched: {n / wall_b:.1f}/s vs sequential plain {n / wall_p:.1f}/s; identical={identical}; "
        f"success {ok}/{len(att)}")
    return {"batched": {"value": n / wall_b, "unit": "relocalisations/s", "schedule": b.schedule()},
            "sequential_plain": {"value": n / wall_p, "unit": "relocalisations/s"},
            "speedup": wall_p / wall_b, "identical_to_plain": identical, "success_rate": ok / len(att),
            "workload": "64 attempts, 8 forests (320x240 rooms, 5 trees depth 10, R=256, 20 frames each); "
                        "frames 320x240/480x360/640x480, N in {256, 512, 1024}, B=64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (every box here has one GPU)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    dev = torch.device("cuda:0")
    full = plain_full(args, dev)
    out = {
        "metric": "relocalisations/sec at >=95% success (<=5cm/5deg), plain vs batched+learned",
        "value": full["value"],
        "unit": "relocalisations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * full["wall"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "full-size plain: 640x480 room 6x8x3 m, 30 boxes, 1% depth noise; 5 trees depth 15, "
                               "R=1024, 200 adaptation frames; N=1024 hypotheses, B=500 pixels per round; "
                               "step = 50 held-out queries, one plain call each"},
        "success_rate": full["success"],
        "roofline": full["roof"],
        "kernels_ms_per_step": {k: round(v[0], 4) for k, v in full["kernels"].items()},
        "adapt_frames_per_s": full["adapt_fps"],
        "forest_bytes": full["mem"],
    }
    forms = {"plain_full": {"value": full["value"], "unit": "relocalisations/s", "success_rate": full["success"]}}
    if not args.no_batched:
        forms["mixed"] = batched_mixed(args, dev)
    out["forms"] = forms
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(full["sc"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
