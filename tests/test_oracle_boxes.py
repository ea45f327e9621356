"""Pins of the oracle's box geometry (the box collision geometry of
Sec. IV-D): sphere-box signed distance and the separating-axis value of two
boxes against closed forms, an exact LP intersection test, sampled surface
distances and rigid-motion invariance; a one-link box arm in closed form."""
import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle

I3 = np.eye(3)


def test_sphere_box_closed_forms():
    h = np.array([1.0, 2.0, 3.0])
    c = np.zeros(3)
    r = 0.25
    assert oracle.sd_sphere_box([3, 0, 0], r, c, I3, h) == pytest.approx(2.0 - r)      # face
    assert oracle.sd_sphere_box([2, 3, 0], r, c, I3, h) == pytest.approx(np.sqrt(2) - r)  # edge
    assert oracle.sd_sphere_box([2, 3, 4], r, c, I3, h) == pytest.approx(np.sqrt(3) - r)  # corner
    assert oracle.sd_sphere_box([0.5, 0, 0], r, c, I3, h) == pytest.approx(-0.5 - r)   # inside, nearest face x
    assert oracle.sd_sphere_box([0, 0, 2.9], r, c, I3, h) == pytest.approx(-0.1 - r)   # inside, nearest face z


def test_sphere_box_rigid_invariance_and_sampled_surface():
    rng = np.random.default_rng(1)
    for _ in range(40):
        h = rng.uniform(0.1, 1.0, 3)
        x = rng.uniform(-2, 2, 3)
        r = rng.uniform(0.0, 0.3)
        base = oracle.sd_sphere_box(x, r, np.zeros(3), I3, h)
        R = Rotation.random(random_state=rng).as_matrix()
        t = rng.uniform(-1, 1, 3)
        moved = oracle.sd_sphere_box(R @ x + t, r, t, R, h)
        assert moved == pytest.approx(base, abs=1e-12)
        # outside: distance to a dense sample of the surface is an upper bound within the sample spacing
        if base > 0:
            g = np.linspace(-1, 1, 41)
            pts = []
            for ax in range(3):
                for sgn in (-1, 1):
                    u, v = np.meshgrid(g, g)
                    p = np.zeros((u.size, 3))
                    o1, o2 = [k for k in range(3) if k != ax]
                    p[:, ax] = sgn * h[ax]
                    p[:, o1] = u.ravel() * h[o1]
                    p[:, o2] = v.ravel() * h[o2]
                    pts.append(p)
            d = np.min(np.linalg.norm(np.concatenate(pts) - x, axis=1)) - r
            assert base <= d + 1e-12 and d - base <= np.max(h) * 2 / 40 * np.sqrt(2)


def test_sat_axis_aligned_closed_forms():
    hA, hB = np.array([1.0, 1.0, 1.0]), np.array([0.5, 2.0, 0.25])
    v, fr = oracle.sat_boxes(np.zeros(3), I3, hA, [2.0, 0.3, 0.1], I3, hB)
    assert v == pytest.approx(0.5) and fr == 0                   # face-face gap along x
    v, _ = oracle.sat_boxes(np.zeros(3), I3, hA, [1.2, 0.5, 1.1], I3, hB)
    assert v == pytest.approx(-0.15)                              # overlaps 0.3, 2.5, 0.15 -> -min
    v, _ = oracle.sat_boxes(np.zeros(3), I3, hA, [1.5, 0.0, 0.0], I3, hB)
    assert v == pytest.approx(0.0)                                # touching: not a collision (sd < 0 collides)


def boxes_intersect_lp(cA, RA, hA, cB, RB, hB):
    """Exact feasibility of a common point: |R^T (x - c)| <= h for both boxes."""
    rows, rhs = [], []
    for c, R, h in ((cA, RA, hA), (cB, RB, hB)):
        for k in range(3):
            a = R[:, k]
            rows += [a, -a]
            rhs += [h[k] + a @ c, h[k] - a @ c]
    res = linprog(np.zeros(3), A_ub=np.array(rows), b_ub=np.array(rhs), bounds=[(None, None)] * 3,
                  method="highs")
    return res.status == 0


def test_sat_sign_matches_exact_intersection_and_bounds_distance():
    rng = np.random.default_rng(2)
    n_apart = n_overlap = 0
    for _ in range(300):
        hA, hB = rng.uniform(0.1, 0.6, 3), rng.uniform(0.1, 0.6, 3)
        RA, RB = Rotation.random(2, random_state=rng).as_matrix()
        cA, cB = np.zeros(3), rng.uniform(-1.2, 1.2, 3)
        v, _ = oracle.sat_boxes(cA, RA, hA, cB, RB, hB)
        if abs(v) < 1e-6:
            continue
        inter = boxes_intersect_lp(cA, RA, hA, cB, RB, hB)
        assert inter == (v < 0)
        # rigid motion of the pair leaves the value unchanged
        Q = Rotation.random(random_state=rng).as_matrix()
        t = rng.uniform(-1, 1, 3)
        v2, _ = oracle.sat_boxes(Q @ cA + t, Q @ RA, hA, Q @ cB + t, Q @ RB, hB)
        assert v2 == pytest.approx(v, abs=1e-12)
        if v > 0:
            n_apart += 1
            # a lower bound of the distance: below the distance between sampled points of the two boxes
            g = rng.uniform(-1, 1, (4000, 3))
            pa = cA + (g * hA) @ RA.T
            pb = cB + (rng.uniform(-1, 1, (4000, 3)) * hB) @ RB.T
            dist, _ = cKDTree(pb).query(pa)
            assert v <= dist.min() + 1e-12
        else:
            n_overlap += 1
    assert n_apart > 50 and n_overlap > 50


def test_sat_penetration_depth_axis_aligned():
    # B pushed into A along y by 0.2 with large overlaps elsewhere: depth 0.2
    hA, hB = np.array([1.0, 1.0, 1.0]), np.array([1.0, 0.5, 1.0])
    v, _ = oracle.sat_boxes(np.zeros(3), I3, hA, [0.0, 1.3, 0.0], I3, hB)
    assert v == pytest.approx(-0.2)


def one_link_box_robot(L, w):
    """1-DOF arm (a = L, d = 0, alpha = 0) with one box along the link:
    centre (-L/2, 0, 0) in the link frame, half extents (L/2, w, w)."""
    pose = np.concatenate([[-L / 2, 0.0, 0.0], np.eye(3).ravel()])
    return dict(dof=1, a=np.array([L]), alpha=np.array([0.0]), d=np.array([0.0]),
                q_lo=np.array([-np.pi]), q_hi=np.array([np.pi]),
                sphere_link=np.zeros(0, np.int32), sphere_xyz=np.zeros((0, 3)), sphere_r=np.zeros(0),
                box_link=np.array([0], np.int32), box_pose=pose[None], box_half=np.array([[L / 2, w, w]]))


def test_box_arm_against_obstacle_sphere_and_box_closed_form():
    L, w = 1.0, 0.1
    rob = oracle.Robot(one_link_box_robot(L, w))
    # obstacle sphere on the circle of radius 0.5 at angle 0.7 rad, 0.3 m above the plane
    th, r_o = 0.7, 0.05
    obs = np.array([[0.5 * np.cos(th), 0.5 * np.sin(th), 0.3, r_o]])
    for q in np.linspace(-np.pi, np.pi, 37):
        f, sd, se, ss = oracle.check(rob, obs, [[q]])
        # in the box frame the sphere sits at (0.5 cos(th-q) - L/2, 0.5 sin(th-q), 0.3)
        p = np.array([0.5 * np.cos(th - q) - L / 2, 0.5 * np.sin(th - q), 0.3])
        out = np.maximum(np.abs(p) - [L / 2, w, w], 0)
        assert se[0] == pytest.approx(np.linalg.norm(out) - r_o, abs=1e-12)
        assert ss[0] == np.inf and f[0] == (se[0] < 0)
    # an obstacle box (a slab under the arm): axis-aligned, top face at z = -0.15
    slab = np.concatenate([[0.0, 0.0, -0.65], np.eye(3).ravel(), [2.0, 2.0, 0.5]])
    for q in (0.0, 1.0, -2.5):
        _, _, se, _ = oracle.check(rob, np.zeros((0, 4)), [[q]], env_boxes=slab[None])
        assert se[0] == pytest.approx(0.15 - w, abs=1e-12)        # gap between the faces
    slab_hi = slab.copy()
    slab_hi[2] = -0.55                                             # top face at z = -0.05: overlap 0.05
    f, _, se, _ = oracle.check(rob, np.zeros((0, 4)), [[0.3]], env_boxes=slab_hi[None])
    assert se[0] == pytest.approx(-0.05, abs=1e-12) and f[0] == 1


def test_box_self_pairs_two_link_fold():
    """2-link planar arm (a = 1, 1), a box on each link along it; the pair
    collides once the elbow folds back far enough."""
    L, w = 1.0, 0.05
    desc = one_link_box_robot(L, w)
    desc.update(dof=2, a=np.array([L, L]), alpha=np.zeros(2), d=np.zeros(2), q_lo=np.full(2, -np.pi),
                q_hi=np.full(2, np.pi), box_link=np.array([0, 1], np.int32),
                box_pose=np.repeat(desc["box_pose"], 2, axis=0), box_half=np.repeat(desc["box_half"], 2, axis=0),
                box_pairs=np.array([[0, 1]], np.int32))
    rob = oracle.Robot(desc)
    # straight arm: box 0 spans x in [0, 1], box 1 [1, 2]; they touch end to
    # end (value 0), which is not a collision
    f0, sd0, _, ss0 = oracle.check(rob, np.zeros((0, 4)), [[0.0, 0.0]])
    assert f0[0] == 0 and ss0[0] == pytest.approx(0.0, abs=1e-12)
    # boxes shortened by 0.1 at both ends: [0.1, 0.9] and [1.1, 1.9], a face
    # gap of 0.2 when straight; folded back (q2 = 3 rad) the pair collides
    desc["box_half"] = desc["box_half"].copy()
    desc["box_half"][:, 0] = L / 2 - 0.1
    rob = oracle.Robot(desc)
    f, _, _, ss = oracle.check(rob, np.zeros((0, 4)), [[0.0, 0.0], [0.0, 3.0]])
    assert list(f) == [0, 1]
    assert ss[0] == pytest.approx(0.2, abs=1e-12)
