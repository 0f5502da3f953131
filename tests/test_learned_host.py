"""Host logic of the learned proposal's supervision (no GPU): a relocalised
pose is accepted only through the depth-difference check with the render at
that pose as the first image (Sec. 3.3.1, Eqs. 3-4)."""
import numpy as np

import oracle


class _FakeForest:
    def __init__(self, status, pose):
        self.status, self.pose = status, pose

    def relocalise_ex(self, depth, rgb, K, seed, n_hyp=0):
        return {"status": self.status, "pose": self.pose}


def test_verified_pose_renders_first(monkeypatch):
    from paper_1801_08361_amd import learned as L
    calls = []

    def fake_verify(da, db):
        calls.append((da, db))
        return oracle.verify(da, db)

    monkeypatch.setattr(L, "verify", fake_verify)
    rng = np.random.default_rng(0)
    query = rng.integers(800, 4000, size=(30, 40)).astype(np.uint16)
    render = query.copy()
    render[:, 12:] = 0                       # the pose looks mostly past the scene
    pose = np.eye(4)
    got, r = L.verified_pose(_FakeForest(0, pose), query, None, None, seed=1, model_depth=lambda T: render)
    assert calls and calls[0][0] is render and calls[0][1] is query
    assert got is None and r["verify"][2] is False
    # a render that matches the query is accepted
    got, r = L.verified_pose(_FakeForest(0, pose), query, None, None, seed=1, model_depth=lambda T: query.copy())
    assert got is pose
    # a failed relocalisation is never verified
    calls.clear()
    got, r = L.verified_pose(_FakeForest(3, pose), query, None, None, seed=1, model_depth=lambda T: query)
    assert got is None and not calls
