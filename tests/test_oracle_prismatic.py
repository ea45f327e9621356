"""Pins of prismatic joints and the Forest scene (Sec. VI-A): the point
robot on two prismatic joints against the disc scene's own distance code,
a one-prismatic-joint arm in closed form, and whole EI-ZO runs of the point
robot against the same runs on the disc scene."""
import numpy as np
import pytest

import oracle
import workloads


def test_point_robot_matches_disc_distances():
    data = workloads.load("forest")
    rob = oracle.Robot(workloads.robot(data))
    discs = data["discs"].astype(np.float64)
    q = np.random.default_rng(0).uniform(0, 10, (2000, 2))
    f, sd, se, ss = oracle.check(rob, data["obstacles"].astype(np.float64), q)
    # closed form in configuration coordinates: min |q - c| - r
    ref = np.min(np.linalg.norm(q[:, None, :] - discs[None, :, :2], axis=2) - discs[None, :, 2], axis=1)
    assert np.abs(sd - ref).max() < 1e-6          # alpha_1 = -pi/2 is rounded to FP32
    assert np.array_equal(f.astype(bool), ref < 0) and np.all(np.isinf(ss))


def test_prismatic_joint_closed_form():
    """Revolute joint about z, then a prismatic joint: the sphere at the
    second frame's origin sits at (a1 cos q1, a1 sin q1, d2 + q2)."""
    desc = dict(dof=2, a=np.array([0.5, 0.0]), alpha=np.zeros(2), d=np.array([0.0, 0.2]),
                q_lo=np.array([-np.pi, 0.0]), q_hi=np.array([np.pi, 1.0]), sphere_link=np.array([1], np.int32),
                sphere_xyz=np.zeros((1, 3)), sphere_r=np.array([0.0]), joint_type=np.array([0, 1], np.int32))
    rob = oracle.Robot(desc)
    for q1, q2 in ((0.3, 0.1), (-2.0, 0.7), (1.5, 0.0)):
        c = oracle.sphere_centres(rob, [q1, q2])[0]
        assert np.allclose(c, [0.5 * np.cos(q1), 0.5 * np.sin(q1), 0.2 + q2], atol=1e-15)


def test_forest_inflation_equals_disc_scene_inflation():
    data = workloads.load("forest")
    rob = oracle.Robot(workloads.robot(data))
    discs = data["discs"].astype(np.float64)
    A_D, b_D = rob.box()
    for e in range(len(data["edges"])):
        v1, v2 = data["edges"][e].astype(np.float64)
        prm = oracle.make_params(**workloads.PARAMS["forest"], seed=3, edge_id=e)
        a = oracle.eizo_arm(rob, data["obstacles"].astype(np.float64), v1, v2, prm)
        b = oracle.eizo_balls(discs[:, :2], discs[:, 2], A_D, b_D, v1, v2, prm)
        assert a["status"] == b["status"] == oracle.CERTIFIED
        assert a["A"].shape == b["A"].shape and np.abs(a["A"] - b["A"]).max() < 1e-5
        assert np.abs(a["b"] - b["b"]).max() < 1e-5
        for v in (v1, v2):
            assert np.all(a["A"] @ v <= a["b"] + 1e-12)
