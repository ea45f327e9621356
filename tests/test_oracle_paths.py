"""Pins of the oracle's sequential path inflation with the containment skip
(Sec. V-A): hand-worked paths with box-shaped stand-in sets, the statuses
whose sets do not count, and the real disc-scene inflation."""
import numpy as np

import oracle


def box_around(v1, v2, m=0.5):
    """Axis-aligned box [min - m, max + m] around the segment, as rows A x <= b."""
    lo, hi = np.minimum(v1, v2) - m, np.maximum(v1, v2) + m
    d = len(v1)
    return np.concatenate([np.eye(d), -np.eye(d)]), np.concatenate([hi, -lo])


def test_skip_pattern_with_box_sets():
    calls = []

    def inflate(k, v1, v2):
        calls.append(k)
        A, b = box_around(v1, v2)
        return dict(status=oracle.CERTIFIED, A=A, b=b)

    V = np.array([[0.0, 0.0], [0.3, 0.0], [0.6, 0.0], [2.0, 0.0], [2.2, 0.1], [5.0, 5.0], [0.0, 0.2]])
    out = oracle.inflate_path(inflate, V)
    # edge 0's box is [-0.5, 0.8] x [-0.5, 0.5]: it holds edge 1 (0.3 -> 0.6);
    # edge 2 (0.6 -> 2.0) leaves it; edge 2's box [0.1, 2.5] x [-0.5, 0.5]
    # holds edge 3 (2.0 -> (2.2, 0.1)); edge 4 leaves every box; edge 5 ends
    # at (0, 0.2), outside edge 4's box [1.7, 5.5] x [-0.4, 5.5] but the
    # start (5, 5) is outside boxes 0 and 2: inflated
    assert [o["covered_by"] for o in out] == [-1, 0, -1, 2, -1, -1]
    assert calls == [0, 2, 4, 5]
    assert [o["status"] for o in out] == [0, oracle.CONTAINED, 0, oracle.CONTAINED, 0, 0]
    assert all(len(o["b"]) == 0 for o in out if o["covered_by"] >= 0)


def test_first_containing_set_is_recorded():
    def inflate(k, v1, v2):
        A, b = box_around(v1, v2, m=0.3)
        return dict(status=oracle.CERTIFIED, A=A, b=b)

    # box 0 = [-0.3, 0.8] x [-0.3, 0.3]; edge 1 climbs to (0.5, 2): box 1 =
    # [0.2, 0.8] x [-0.3, 2.3]; edge 2 comes back to (-0.2, 0), in neither:
    # box 2 = [-0.5, 0.8] x [-0.3, 2.3]; edge 3 ((-0.2, 0) -> (0.6, 0.1)) lies
    # in boxes 0 and 2, not 1: the first, 0, is recorded
    V = np.array([[0.0, 0.0], [0.5, 0.0], [0.5, 2.0], [-0.2, 0.0], [0.6, 0.1]])
    out = oracle.inflate_path(inflate, V)
    assert [o["covered_by"] for o in out] == [-1, -1, -1, 0]


def test_sets_of_failed_or_contained_edges_do_not_count():
    def inflate(k, v1, v2):
        A, b = box_around(v1, v2)
        return dict(status=oracle.IN_COLLISION if k == 0 else oracle.MAX_ITERS, A=A, b=b)

    V = np.array([[0.0, 0.0], [0.3, 0.0], [0.1, 0.0], [0.2, 0.0]])
    out = oracle.inflate_path(inflate, V)
    # edge 0 ends IN_COLLISION: edge 1 is inflated (MAX_ITERS); edge 2 lies in
    # edge 1's box and in edge 0's, but only edge 1's counts
    assert [o["covered_by"] for o in out] == [-1, -1, 1]
    assert [o["status"] for o in out] == [oracle.IN_COLLISION, oracle.MAX_ITERS, oracle.CONTAINED]
    # a set with no rows contains nothing
    assert oracle.covering_set([np.zeros((0, 2))], [np.zeros(0)], [0, 0], [1, 1]) == -1


def test_disc_scene_path_inflation():
    """Real inflations (point robot, discs): every inflated edge's set holds
    its segment and equals the inflation of that edge alone; every skipped
    edge lies in the recorded set and in no earlier set that counts."""
    centres = np.array([[0.0, 1.0], [1.5, -0.5], [-1.2, -1.0]])
    radii = np.array([0.4, 0.3, 0.35])
    A_D = np.concatenate([np.eye(2), -np.eye(2)])
    b_D = np.full(4, 3.0)
    V = np.array([[-1.0, 0.2], [-0.2, 0.3], [-0.6, 0.25], [0.8, 0.4], [0.9, -0.1], [0.85, 0.2]])

    def prm(k):
        return oracle.make_params(eps=0.1, delta=0.05, n_p=300, n_mix=20, max_iters=20, seed=7, edge_id=k)

    def inflate(k, v1, v2):
        return oracle.eizo_balls(centres, radii, A_D, b_D, v1, v2, prm(k))

    out = oracle.inflate_path(inflate, V)
    skipped = [k for k, o in enumerate(out) if o["covered_by"] >= 0]
    assert 1 in skipped                     # edge 1 runs back along edge 0
    for k, o in enumerate(out):
        seg = V[k:k + 2]
        if o["covered_by"] < 0:
            assert np.all(seg @ o["A"].T <= o["b"] + 1e-12)
            alone = inflate(k, V[k], V[k + 1])
            assert alone["status"] == o["status"] and np.array_equal(alone["A"], o["A"])
            for j in range(k):
                oj = out[j]
                if oj["covered_by"] < 0 and oj["status"] in (oracle.CERTIFIED, oracle.MAX_ITERS):
                    assert not np.all(seg @ oj["A"].T <= oj["b"])
        else:
            h = o["covered_by"]
            assert h < k and out[h]["covered_by"] == -1
            assert np.all(seg @ out[h]["A"].T <= out[h]["b"])
            for j in range(h):
                oj = out[j]
                if oj["covered_by"] < 0 and oj["status"] in (oracle.CERTIFIED, oracle.MAX_ITERS):
                    assert not np.all(seg @ oj["A"].T <= oj["b"])
