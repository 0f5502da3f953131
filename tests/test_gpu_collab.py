"""GPU end to end: collaborative relocalisation and pose optimisation
(Sec. 3.3.1, 3.3.2). Three agents map one room, each in its own sub-scene
frame; each agent's forest adapts on its own frames with its local poses.
Attempts are scheduled by candidate scores, the chosen frame of agent b is
rendered as a synthetic RGB-D image and relocalised with agent a's forest on
the GPU, the pose is checked by the depth-difference test against a's model
rendered at that pose, accepted relative transforms are clustered, and the
pose graph is optimised. The optimised global poses must recover each
agent's frame relative to the first agent's within 5 cm and 5 degrees."""
import numpy as np
import pytest

import synthroom as sr
from tests.gpu_util import SMALL, banner, need_gpu

pytestmark = pytest.mark.gpu


def test_collaborative_session_recovers_subscene_frames():
    dev = need_gpu()
    import oracle
    import paper_1801_08361_amd as rl
    n = 3
    sc, world, W = sr.collaborative_session(n, index=41)
    local = [np.stack([np.linalg.inv(W[s]) @ P for P in world[s]]) for s in range(n)]
    forests = []
    for s in range(n):
        g = rl.Forest(rl.params_default(**SMALL))
        for k in range(0, len(world[s]), 2):           # every second frame trains the forest
            d, c = sr.render(sc.room, world[s][k], sc.width, sc.height, dev)
            g.adapt_frame(d, c, sc.K, local[s][k])
        g.update_modes()
        forests.append(g)
    col = rl.Collab(n, seed=7)
    for s in range(n):
        col.set_frames(s, local[s])
    accepted = 0
    for attempt in range(36):
        a, b, i, cands = col.schedule(10)
        col.tried(a, b, i)
        banner(f"collab attempt {attempt}: frame {i} of agent {b} in agent {a}")
        d, c = sr.render(sc.room, world[b][i], sc.width, sc.height, dev)
        st, pose, _ = forests[a].relocalise(d, c, sc.K, seed=1000 + attempt)
        if st != 0:
            continue
        model = sr.render(sc.room, W[a] @ pose, sc.width, sc.height, dev)[0]
        if not rl.verify(model, d)[2]:
            continue
        accepted += 1
        size = col.add_sample(a, b, rl.relative_transform(pose, local[b][i]))
        if size >= 2:
            col.optimise()
    ing, X, cost = col.optimise()
    assert accepted >= 6
    assert ing.all(), ing
    for s in range(1, n):
        want = np.linalg.inv(W[0]) @ W[s]
        ok, dt, da = oracle.pose_success(X[s], want)
        assert ok, (s, dt, da)
