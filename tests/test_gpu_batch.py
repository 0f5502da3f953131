"""GPU: the batched form. A ragged batch (several forests, mixed frame sizes
and hypothesis counts) must return, for every attempt, exactly the result of
the plain call on the same arguments, whatever schedule the autotuner picks;
weighted pixel picks (the learned proposal's entry point) must match the
oracle."""
import numpy as np
import pytest

import synthroom as sr
from tests.gpu_util import SMALL, banner, need_gpu, pair, rot_angle_deg, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def forests():
    dev = need_gpu()
    import paper_1801_08361_amd as rl
    out = []
    for room in (400, 401, 402):
        sc = sr.small_scene(room)
        g = rl.Forest(rl.params_default(**SMALL))
        for k in range(8):
            d, c = to_dev(*sc.render_adapt(k), dev)
            banner(f"batch forest {room} adapt {k}")
            g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        out.append((sc, g))
    return dev, out


def attempts(dev, forests, n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(320, 240), (480, 360), (97, 61), (640, 480)]
    hyps = [64, 256, 100, 1, 512]
    att = []
    for i in range(n):
        sc, g = forests[int(rng.integers(0, len(forests)))]
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        q = int(rng.integers(0, len(sc.query_poses)))
        d, c = sc.render_query(q, device=dev, width=W, height=H)
        att.append(dict(forest=g, depth=d.contiguous(), rgb=c.contiguous(), K=sr.intrinsics(W, H),
                        seed=int(rng.integers(1, 1 << 40)), n_hyp=hyps[int(rng.integers(0, len(hyps)))],
                        gt=sc.query_poses[q]))
    return att


def same(a, b):
    return (a["status"] == b["status"] and np.array_equal(a["pose"], b["pose"]) and a["score"] == b["score"]
            and a["final_hyp"] == b["final_hyp"] and a["n_rounds"] == b["n_rounds"]
            and a["n_valid"] == b["n_valid"] and a["mode_evals"] == b["mode_evals"]
            and a["pair_evals"] == b["pair_evals"] and a["pool_size"] == b["pool_size"])


def test_tuned_batches_of_tiny_attempts(forests):
    """The autotuner's per-launch timings of launches with nothing to do (the
    late rounds of attempts with a handful of hypotheses) can come out below
    the events' own cost; they count as zero, never as an error. Fresh tuned
    batches of such attempts equal the plain calls."""
    import paper_1801_08361_amd as rl
    dev, fs = forests
    for rep in range(4):
        att = attempts(dev, fs, 6, seed=40 + rep)
        for k, a in enumerate(att):
            a["n_hyp"] = (2, 3, 5, 1, 8, 4)[k]
        banner(f"tiny tuned batch {rep}")
        res = rl.Batch(tune=True).run(att)
        for a, r in zip(att, res):
            p = a["forest"].relocalise_ex(a["depth"], a["rgb"], a["K"], seed=a["seed"], n_hyp=a["n_hyp"])
            assert same(r, p)


@pytest.mark.parametrize("tune", [False, True])
def test_batch_equals_plain(forests, tune):
    import paper_1801_08361_amd as rl
    dev, fs = forests
    att = attempts(dev, fs, 14, seed=5 + int(tune))
    b = rl.Batch(tune=tune)
    banner(f"batch of {len(att)} tune={tune}")
    res = b.run(att)
    banner(f"schedule: {b.schedule()}")
    res2 = b.run(att)                     # graph replay of the cached shape
    for i, a in enumerate(att):
        banner(f"plain attempt {i}")
        p = a["forest"].relocalise_ex(a["depth"], a["rgb"], a["K"], seed=a["seed"], n_hyp=a["n_hyp"])
        assert same(res[i], p), (i, res[i], p)
        assert same(res2[i], p), i
    ok = [r["status"] == 0 for r in res]
    assert sum(ok) >= len(att) // 2


def test_batch_eight_pixels_per_thread_equals_plain(forests):
    """Six 640x480 attempts (about 9.2M pixel-tree walks) take the traversal
    with 8 pixels per thread; every result equals the plain call's."""
    import paper_1801_08361_amd as rl
    dev, fs = forests
    att = []
    for i in range(6):
        sc, g = fs[i % len(fs)]
        d, c = sc.render_query(i % len(sc.query_poses), device=dev, width=640, height=480)
        att.append(dict(forest=g, depth=d.contiguous(), rgb=c.contiguous(), K=sr.intrinsics(640, 480),
                        seed=900 + i, n_hyp=64))
    b = rl.Batch(tune=False)
    banner("batch of six 640x480 attempts")
    res = b.run(att)
    assert "pix_per_thread=8" in b.schedule()
    for i, a in enumerate(att):
        p = a["forest"].relocalise_ex(a["depth"], a["rgb"], a["K"], seed=a["seed"], n_hyp=a["n_hyp"])
        assert same(res[i], p), (i, res[i], p)


def test_batch_single_and_failures(forests):
    import torch
    import paper_1801_08361_amd as rl
    dev, fs = forests
    sc, g = fs[0]
    d, c = to_dev(*sc.render_query(1), dev)
    empty = rl.Forest(rl.params_default(**SMALL))
    att = [dict(forest=g, depth=d, rgb=c, K=sc.K, seed=3),
           dict(forest=g, depth=torch.zeros_like(d), rgb=c, K=sc.K, seed=3),
           dict(forest=empty, depth=d, rgb=c, K=sc.K, seed=3)]
    banner("batch with failures")
    res = rl.Batch(tune=False).run(att)
    assert res[0]["status"] == 0
    assert res[1]["status"] == rl.FAIL_NO_VALID_PIXELS
    assert res[2]["status"] == rl.FAIL_NO_MODES
    with pytest.raises(rl.RelocError):
        rl.Batch().run([dict(forest=g, depth=d, rgb=c, K=(0.0, 1.0, 1.0, 1.0), seed=1)])


def test_weighted_picks_match_oracle():
    """Integer pick weights (the learned proposal's output) through the CDF
    path: hypotheses, culls and pose equal the oracle's."""
    dev = need_gpu()
    import torch
    import oracle
    import paper_1801_08361_amd as rl
    pp, po = pair(**SMALL)
    g, o = rl.Forest(pp), oracle.Forest(po)
    sc = sr.small_scene(403)
    for k in range(8):
        d0, c0 = sc.render_adapt(k)
        d, c = to_dev(d0, c0, dev)
        banner(f"weights adapt {k}")
        g.adapt_frame(d, c, sc.K, sc.adapt_poses[k])
        o.adapt(d0, c0, sc.K, sc.adapt_poses[k])
    rng = np.random.default_rng(9)
    # weight patterns: the proposal's range (half of them 1); mostly zero with
    # a few near 2^32 (one entry spans many draw buckets); a few 1s among
    # zeros (fewer weight units than pool entries); all zero (uniform picks)
    cases = [(0, "proposal"), (5, "proposal"), (2, "sparse_huge"), (3, "few_ones"), (4, "zero")]
    for q, kind in cases:
        d0, c0 = sc.render_query(q)
        n = d0.numel()
        if kind == "proposal":
            w = rng.integers(1, 65537, size=n).astype(np.uint32)
            w[rng.random(n) < 0.5] = 1
        elif kind == "sparse_huge":
            w = rng.integers(1, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
            w[rng.random(n) < 0.9] = 0
        elif kind == "few_ones":
            w = (rng.random(n) < 0.01).astype(np.uint32)
        else:
            w = np.zeros(n, np.uint32)
        d, c = to_dev(d0, c0, dev)
        wd = torch.from_numpy(w.view(np.int32)).to(dev)
        banner(f"weights relocalise q={q} {kind}")
        rg = g.relocalise_ex(d, c, sc.K, seed=77 + q, weights=wd)
        tg = g.trace(pp.n_hypotheses)
        so, To, sco, to = o.relocalise(d0, c0, sc.K, seed=77 + q, weights=w, trace=True)
        assert rg["status"] == so
        assert np.array_equal(tg["hyp_try"], to["hyp_try"])
        if so == 0:
            assert np.linalg.norm(rg["pose"][:3, 3] - To[:3, 3]) < 1e-4
            assert rot_angle_deg(rg["pose"][:3, :3], To[:3, :3]) < 1e-3
            assert abs(rg["score"] - sco) < 1e-6
