"""Whole-algorithm checks of the oracle's EI-ZO (Alg. 1).

The output polytope has no closed form (the method is randomised and many
outputs are correct), so these tests pin what the paper guarantees:
L is contained in P, P lies in D (Alg. 1 Output), every placed plane separates
its candidate from L with the relaxed step back (Sec. IV-C), the status paths
(Sec. IV-C: t_col error, maximum iterations), and the (eps, delta) guarantee
(eq:prob_polytope_cfree) measured by exact rejection sampling from D.
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def forest_scene(seed=0, n=15):
    """Forest scene of Sec. VI-A: 15 discs of radius 0.35 scattered in the
    central 7x7 part of a 10x10 square, point robot."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(1.5, 8.5, size=(n, 2))
    return c, np.full(n, 0.35)


def free_segment(centres, radii, rng, length=1.5):
    while True:
        v1 = rng.uniform(0.5, 9.5, 2)
        ang = rng.uniform(0, 2 * np.pi)
        v2 = v1 + length * np.array([np.cos(ang), np.sin(ang)])
        if np.any(v2 < 0.01) or np.any(v2 > 9.99):
            continue
        w = np.linspace(0, 1, 400)[:, None]
        P = (1 - w) * v1 + w * v2
        d = np.linalg.norm(P[:, None] - centres[None], axis=2) - radii
        if d.min() > 0.05:
            return v1, v2


def check_polytope_invariants(out, A_D, b_D, v1, v2, t_col=1e-4):
    A, b = out["A"], out["b"]
    nD = len(b_D)
    np.testing.assert_array_equal(A[:nD], A_D)          # P starts from D: P is inside D
    np.testing.assert_array_equal(b[:nD], b_D)
    assert np.all(A @ v1 <= b + 1e-12) and np.all(A @ v2 <= b + 1e-12)   # L inside P
    if len(b) > nD:
        np.testing.assert_allclose(np.linalg.norm(A[nD:], axis=1), 1.0, atol=1e-12)


def test_forest_point_robot_certifies_and_contains_segment(orc):
    centres, radii = forest_scene(0)
    rng = np.random.default_rng(1)
    A_D = np.concatenate([np.eye(2), -np.eye(2)])
    b_D = np.array([10.0, 10.0, 0.0, 0.0])
    for trial in range(5):
        v1, v2 = free_segment(centres, radii, rng)
        prm = orc.make_params(eps=0.01, delta=0.05, n_p=1000, n_f=10, n_b=11, n_mix=30, seed=trial)
        out = orc.eizo_balls(centres, radii, A_D, b_D, v1, v2, prm)
        assert out["status"] == oracle.CERTIFIED
        check_polytope_invariants(out, A_D, b_D, v1, v2)
        st = out["stats"]
        assert st["planes"] == len(out["b"]) - 4
        assert st["planes"] <= 10 * st["iterations"]
        M, T = orc.test_constants(0.01, 0.05, 0.5, st["iterations"])
        assert st["final_m"] == M and st["test_collisions"] <= T


def collision_fraction_balls(A, b, centres, radii, rng, n=200_000):
    x = rng.uniform(0, 10, size=(n, 2))
    x = x[np.all(x @ A.T <= b, axis=1)]
    d = np.min(np.linalg.norm(x[:, None] - centres[None], axis=2) - radii, axis=1)
    return float(np.mean(d < 0)), len(x)


def test_forest_polytopes_mostly_collision_free(orc):
    centres, radii = forest_scene(3)
    rng = np.random.default_rng(2)
    A_D = np.concatenate([np.eye(2), -np.eye(2)])
    b_D = np.array([10.0, 10.0, 0.0, 0.0])
    eps = 0.05
    bad = 0
    for trial in range(20):
        v1, v2 = free_segment(centres, radii, rng)
        prm = orc.make_params(eps=eps, delta=0.05, n_p=1000, n_mix=30, seed=100 + trial)
        out = orc.eizo_balls(centres, radii, A_D, b_D, v1, v2, prm)
        assert out["status"] == oracle.CERTIFIED
        frac, n_in = collision_fraction_balls(out["A"], out["b"], centres, radii, rng)
        assert n_in > 1000
        bad += frac > eps
    assert bad <= 3       # P(Bin(20, 0.05) > 3) ~ 1.6 %


def tiny_setup():
    data = workloads.load("tiny")
    rob = oracle.Robot(workloads.robot(data))
    prm = oracle.make_params(**workloads.PARAMS["tiny"], seed=0)
    return data, rob, prm


def test_tiny_arm_certifies_with_invariants(orc):
    data, rob, prm = tiny_setup()
    v1, v2 = data["edges"][0].astype(np.float64)
    out = orc.eizo_arm(rob, data["obstacles"], v1, v2, prm)
    assert out["status"] == oracle.CERTIFIED
    A_D, b_D = rob.box()
    check_polytope_invariants(out, A_D, b_D, v1, v2)
    # the segment itself is collision free
    w = np.linspace(0, 1, 200)[:, None]
    f, *_ = orc.check(rob, data["obstacles"], (1 - w) * v1 + w * v2)
    assert not f.any()


def test_status_in_collision_for_colliding_segment(orc):
    data, rob, prm = tiny_setup()
    # a segment through a configuration in collision
    qs = np.random.default_rng(3).uniform(-np.pi, np.pi, size=(2000, 3))
    f, sd, *_ = orc.check(rob, data["obstacles"], qs)
    q_bad = qs[np.argmin(sd)]
    assert f[np.argmin(sd)]
    v1 = np.clip(q_bad - 0.2, -np.pi, np.pi)
    v2 = np.clip(q_bad + 0.2, -np.pi, np.pi)
    out = orc.eizo_arm(rob, data["obstacles"], v1, v2, prm)
    assert out["status"] == oracle.IN_COLLISION


def test_status_max_iters_and_invalid(orc):
    data, rob, prm = tiny_setup()
    v1, v2 = data["edges"][0].astype(np.float64)
    prm.max_iters = 1
    out = orc.eizo_arm(rob, data["obstacles"], v1, v2, prm)
    assert out["status"] == oracle.MAX_ITERS
    assert out["stats"]["iterations"] == 1
    A_D, b_D = rob.box()
    check_polytope_invariants(out, A_D, b_D, v1, v2)
    prm.max_iters = 50
    bad = v2.copy()
    bad[0] = 4.0
    out = orc.eizo_arm(rob, data["obstacles"], v1, bad, prm)
    assert out["status"] == oracle.INVALID and len(out["b"]) == 6
    bad[0] = np.nan
    assert orc.eizo_arm(rob, data["obstacles"], v1, bad, prm)["status"] == oracle.INVALID


def test_checks_accounting(orc):
    data, rob, prm = tiny_setup()
    v1, v2 = data["edges"][0].astype(np.float64)
    out = orc.eizo_arm(rob, data["obstacles"], v1, v2, prm)
    st = out["stats"]
    assert st["samples"] == prm.n_p * st["iterations"]        # |S| = max(N_p, M_k) = N_p here
    extra = st["checks"] - st["samples"]
    assert extra % (1 + prm.n_b) == 0                         # projection + N_b midpoints each


@pytest.mark.slow
def test_guarantee_eps_delta_tiny_arm(orc):
    """eq:prob_polytope_cfree on the tiny workload: over R independent seeds,
    the number of certified polytopes whose collision fraction exceeds eps
    must not exceed the 99.9 % quantile of Bin(R, delta).  Fractions are
    estimated by exact rejection sampling from D (uniform in the box, kept if
    inside P), so the estimate does not inherit the sampler's mixing bias."""
    from scipy.stats import binom
    data, rob, prm = tiny_setup()
    v1, v2 = data["edges"][0].astype(np.float64)
    R, n_mc = 60, 40_000
    rng = np.random.default_rng(11)
    bad, certified = 0, 0
    for r in range(R):
        prm.seed = 1000 + r
        out = orc.eizo_arm(rob, data["obstacles"], v1, v2, prm)
        if out["status"] != oracle.CERTIFIED:
            continue
        certified += 1
        A, b = out["A"], out["b"]
        inside = []
        while sum(len(x) for x in inside) < n_mc:
            x = rng.uniform(-np.pi, np.pi, size=(200_000, 3))
            inside.append(x[np.all(x @ A.T <= b, axis=1)])
        x = np.concatenate(inside)[:n_mc]
        f, *_ = orc.check(rob, data["obstacles"], x)
        # one-sided margin for the Monte-Carlo error of the estimate
        frac = f.mean()
        bad += frac > prm.eps + 3 * math.sqrt(prm.eps * (1 - prm.eps) / n_mc)
    assert certified >= R - 2
    assert bad <= binom.ppf(0.999, certified, prm.delta)


def test_stored_workloads_are_valid(orc):
    """Stored segments lie in D, are free of self-collision and obstacles
    along their whole length (checked here on a 1e-3 rad grid)."""
    for name in ("tiny", "dof7", "batched"):
        data = workloads.load(name)
        rob = oracle.Robot(workloads.robot(data))
        obs = data["obstacles"]
        lo, hi = data["q_lo"], data["q_hi"]
        for e in data["edges"]:
            v1, v2 = e.astype(np.float64)
            assert np.all(e >= lo) and np.all(e <= hi)
            n = int(np.ceil(np.max(np.abs(v2 - v1)) / 1e-3)) + 1
            w = np.linspace(0, 1, n)[:, None]
            f, sd, *_ = orc.check(rob, obs, (1 - w) * v1 + w * v2)
            assert not f.any() and sd.min() > 1e-3
    b = workloads.load("batched")
    assert b["edges"].shape == (96, 2, 7)
    counts = np.bincount(b["path_id"])
    assert tuple(counts) == (2, 5, 8, 11, 14, 17, 19, 20)
    # consecutive segments of a path share their vertex
    for i in range(95):
        if b["path_id"][i] == b["path_id"][i + 1]:
            np.testing.assert_array_equal(b["edges"][i, 1], b["edges"][i + 1, 0])


def test_first_test_count_does_not_depend_on_n_p(orc):
    """Sec. IV-B: |S| = max(N_p, M_k) and the unadaptive test counts the
    collisions among the first M_k samples only.  At k = 1 the polytope is
    the joint box whatever N_p is, and sample i is drawn from the same
    counter-based stream, so the test's count (and M_1) is the same for N_p
    below, near and far above M_1 = 280 -- what lets a tuner pick N_p
    without touching the certificate; the planes placed from the larger
    candidate sets may differ."""
    data = workloads.load("tiny")
    rob = orc.Robot(workloads.robot(data))
    v1, v2 = data["edges"][0].astype(np.float64)
    outs = []
    for n_p in (100, 300, 1000, 5000):
        prm = orc.make_params(**dict(workloads.PARAMS["tiny"], n_p=n_p, max_iters=1), seed=3)
        o = orc.eizo_arm(rob, data["obstacles"], v1, v2, prm)
        assert o["stats"]["samples"] == max(n_p, 280) and o["stats"]["final_m"] == 280
        outs.append(o["stats"]["test_collisions"])
    assert len(set(outs)) == 1 and outs[0] > 14           # the same count; above T_1 = 14 (not yet certified)
