"""Pins of the oracle's recovery functions (Sec. V-B): path discretisation,
polytope membership, segment containment and the set update, against closed
forms and hand-worked cases."""
import numpy as np
import pytest

import oracle


def test_discretisation_counts_spacing_and_vertices():
    rng = np.random.default_rng(0)
    for trial in range(50):
        K, d = rng.integers(1, 7), rng.integers(1, 8)
        w = rng.uniform(-1, 1, size=(K, d))
        if K > 2:
            w[1] = w[0]                                   # a zero-length segment
        step = rng.uniform(0.01, 0.5)
        p = oracle.discretize_path(w, step)
        m = [max(1, int(np.ceil(np.max(np.abs(w[i + 1] - w[i])) / step))) for i in range(K - 1)]
        assert len(p) == 1 + sum(m)
        # every waypoint is a point, at the cumulative index
        idx = np.concatenate([[0], np.cumsum(m)]).astype(int)
        assert np.allclose(p[idx], w, atol=1e-12)
        # consecutive points at most `step` apart in every coordinate, on the segment
        if len(p) > 1:
            assert np.max(np.abs(np.diff(p, axis=0))) <= step + 1e-12
        for i in range(K - 1):
            seg = p[idx[i]:idx[i + 1] + 1]
            dlt = w[i + 1] - w[i]
            t = np.linspace(0.0, 1.0, m[i] + 1)
            assert np.allclose(seg, w[i] + t[:, None] * dlt, atol=1e-12)


def test_membership_and_containment_closed_forms():
    # unit cube as 6 rows
    A = np.concatenate([np.eye(3), -np.eye(3)])
    b = np.concatenate([np.ones(3), np.zeros(3)])
    X = np.array([[0.5, 0.5, 0.5], [1.0, 1.0, 1.0], [1.0001, 0.5, 0.5], [-1e-9, 0.2, 0.2], [0.0, 0.0, 0.0]])
    assert list(oracle.points_in_polytope(A, b, X)) == [True, True, False, False, True]
    # a second set: the cube shifted by (0.8, 0, 0)
    A2, b2 = A.copy(), b + np.array([0.8, 0, 0, -0.8, 0, 0])
    sets = ([A, A2], [b, b2])
    assert oracle.covering_set(*sets, [0.1, 0.1, 0.1], [0.9, 0.9, 0.9]) == 0
    assert oracle.covering_set(*sets, [0.9, 0.1, 0.1], [1.7, 0.9, 0.9]) == 1
    assert oracle.covering_set(*sets, [0.1, 0.1, 0.1], [1.7, 0.9, 0.9]) == -1
    assert oracle.covering_set(*sets, [0.1, 0.1, 0.1], [1.7, 0.9, 0.9], tol=1.0) == 0


def test_set_update_for_a_disc_obstacle_closed_form():
    """Point robot in the plane, one disc: the found collision at the disc's
    centre yields one plane through the disc's near boundary point, stepped
    back by Delta_max, with L untouched."""
    centre, r = np.array([[0.0, 0.5]]), np.array([0.3])
    bis = lambda v1, v2, c, n_b: oracle.bisect_balls(centre, r, v1, v2, c, n_b)
    v1, v2 = np.array([-1.0, -1.0]), np.array([1.0, -1.0])
    A = np.concatenate([np.eye(2), -np.eye(2)])
    b = np.full(4, 2.0)
    pts = np.array([[0.0, 0.5], [5.0, 5.0]])              # the second point lies outside P
    A2, b2, st, res, idx = oracle.recover_set(bis, v1, v2, A, b, pts, 11, 10, 0.01, 1e-4)
    assert st == oracle.CERTIFIED and list(idx) == [0] and len(b2) == 5
    assert np.allclose(A2[4], [0.0, 1.0])
    # c* on the bisection bracket around the crossing y = 0.2: |c - c_proj| = 1.5
    assert abs(res[0]["c_star"][1] - 0.2) <= 1.5 * 2.0 ** -11 + 1e-12
    assert abs(b2[4] - (res[0]["c_star"][1] - 0.01)) < 1e-12
    assert np.all(np.stack([v1, v2]) @ A2.T <= b2 + 1e-12)          # L stays inside
    assert not oracle.points_in_polytope(A2, b2, pts[:1])[0]        # the collision is excluded


def test_set_update_with_no_collision_inside_leaves_the_set():
    centre, r = np.array([[0.0, 0.5]]), np.array([0.3])
    bis = lambda v1, v2, c, n_b: oracle.bisect_balls(centre, r, v1, v2, c, n_b)
    A = np.concatenate([np.eye(2), -np.eye(2)])
    b = np.full(4, 1.0)
    A2, b2, st, res, idx = oracle.recover_set(bis, np.array([-0.5, -0.9]), np.array([0.5, -0.9]), A, b,
                                              np.array([[3.0, 0.0]]), 11, 10, 0.01, 1e-4)
    assert st == oracle.CERTIFIED and len(idx) == 0 and np.array_equal(A2, A) and np.array_equal(b2, b)


def test_set_update_fails_fast_when_a_projection_collides():
    """A disc that covers part of L: the projection of the found point onto L
    collides, so the edge is reported in collision (fail-fast check)."""
    centre, r = np.array([[0.0, -0.9]]), np.array([0.3])
    bis = lambda v1, v2, c, n_b: oracle.bisect_balls(centre, r, v1, v2, c, n_b)
    A = np.concatenate([np.eye(2), -np.eye(2)])
    b = np.full(4, 2.0)
    _, _, st, res, idx = oracle.recover_set(bis, np.array([-1.0, -1.0]), np.array([1.0, -1.0]), A, b,
                                            np.array([[0.0, -0.7]]), 11, 10, 0.01, 1e-4)
    assert st == oracle.IN_COLLISION and res[0]["proj_collides"]
