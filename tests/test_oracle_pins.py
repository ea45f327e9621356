"""Pins of the FP64 oracle against facts fixed outside the oracle itself:
published test vectors, closed forms, invariants of the geometry the paper
states (Sec. IV-A), brute force on tiny inputs, and special cases.

Each test names the passage it pins.  None of these tests touch a GPU.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from workloads import draw

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox4x32-10 (random stream used by the hit-and-run sampler)
# --------------------------------------------------------------------------

def test_philox_known_answer_vectors(orc):
    rows = 0
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            out = orc.philox(w[0:4], w[4:6])
            assert [int(x) for x in out] == w[6:10]
            rows += 1
    assert rows == 3


def test_u01_map_exact_and_open_interval(orc):
    assert orc.u01(0) == 2.0 ** -24
    assert orc.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for x in (0, 255, 256, 0x12345678, 0xFFFFFFFF):
        u = orc.u01(x)
        assert float(np.float32(u)) == u          # exactly representable in FP32
        assert 0.0 < u < 1.0


# --------------------------------------------------------------------------
# Forward kinematics (standard DH)
# --------------------------------------------------------------------------

def dh_closed_form(th, d, a, al):
    """Textbook standard-DH homogeneous matrix Rz(th) Tz(d) Tx(a) Rx(al),
    written out as one matrix."""
    ct, st, ca, sa = math.cos(th), math.sin(th), math.cos(al), math.sin(al)
    return np.array([[ct, -st * ca, st * sa, a * ct],
                     [st, ct * ca, -ct * sa, a * st],
                     [0.0, sa, ca, d],
                     [0.0, 0.0, 0.0, 1.0]])


def planar_robot(lengths, per_link=1, radii=0.05):
    dof = len(lengths)
    link, xyz, r = [], [], []
    for i, l in enumerate(lengths):
        for j in range(per_link):
            link.append(i)
            xyz.append([-(1.0 - (j + 1) / per_link) * l, 0.0, 0.0])
            r.append(radii)
    return dict(dof=dof, a=np.array(lengths, float), alpha=np.zeros(dof), d=np.zeros(dof),
                q_lo=-np.pi * np.ones(dof), q_hi=np.pi * np.ones(dof),
                sphere_link=np.array(link, np.int32), sphere_xyz=np.array(xyz, float),
                sphere_r=np.array(r, float))


def planar_centres(lengths, per_link, q):
    """Closed-form planar chain: o_i = sum_{j<=i} l_j (cos th_j, sin th_j),
    th_j = q_1 + ... + q_j; a sphere at local x on link i sits at
    o_i + x (cos th_i, sin th_i)."""
    th = np.cumsum(q)
    o = np.cumsum(np.stack([np.array(lengths) * np.cos(th), np.array(lengths) * np.sin(th)], 1), 0)
    out = []
    for i, l in enumerate(lengths):
        for j in range(per_link):
            x = -(1.0 - (j + 1) / per_link) * l
            out.append([o[i, 0] + x * math.cos(th[i]), o[i, 1] + x * math.sin(th[i]), 0.0])
    return np.array(out)


def test_fk_two_link_planar_closed_form(orc):
    l1, l2 = 0.7, 0.45
    rob = orc.Robot(planar_robot([l1, l2], per_link=1))
    rng = np.random.default_rng(0)
    for q in rng.uniform(-np.pi, np.pi, size=(50, 2)):
        c = orc.sphere_centres(rob, q)
        x = l1 * math.cos(q[0]) + l2 * math.cos(q[0] + q[1])
        y = l1 * math.sin(q[0]) + l2 * math.sin(q[0] + q[1])
        assert abs(c[1, 0] - x) < 1e-12 and abs(c[1, 1] - y) < 1e-12 and abs(c[1, 2]) < 1e-15
        assert abs(c[0, 0] - l1 * math.cos(q[0])) < 1e-12


def test_fk_three_link_planar_with_interior_spheres(orc):
    L = [0.5, 0.35, 0.6]
    rob = orc.Robot(planar_robot(L, per_link=4))
    rng = np.random.default_rng(1)
    for q in rng.uniform(-np.pi, np.pi, size=(50, 3)):
        np.testing.assert_allclose(orc.sphere_centres(rob, q), planar_centres(L, 4, q), atol=1e-12)


def test_fk_matches_textbook_dh_matrix_7dof(orc):
    data = workloads.load("dof7")
    rob = orc.Robot(workloads.robot(data))
    rng = np.random.default_rng(2)
    for q in rng.uniform(-np.pi, np.pi, size=(20, 7)):
        T = np.eye(4)
        frames = orc.link_frames(rob, q)
        for i in range(7):
            T = T @ dh_closed_form(q[i], rob.d[i], rob.a[i], rob.alpha[i])
            np.testing.assert_allclose(frames[i], T, atol=1e-12)


def test_fk_rigid_body_invariants(orc):
    data = workloads.load("dof7")
    rob = orc.Robot(workloads.robot(data))
    rng = np.random.default_rng(3)
    c0 = orc.sphere_centres(rob, np.zeros(7))
    for q in rng.uniform(-np.pi, np.pi, size=(20, 7)):
        F = orc.link_frames(rob, q)
        for i in range(7):
            R = F[i, :3, :3]
            np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
            assert abs(np.linalg.det(R) - 1.0) < 1e-12
        c = orc.sphere_centres(rob, q)
        for i in range(7):
            idx = np.where(rob.sphere_link == i)[0]
            D0 = np.linalg.norm(c0[idx, None] - c0[None, idx], axis=2)
            D = np.linalg.norm(c[idx, None] - c[None, idx], axis=2)
            np.testing.assert_allclose(D, D0, atol=1e-12)


def test_fk_q_zero_straight_chain(orc):
    """All twists zero and q = 0: every x axis is aligned, so frame i's origin
    is (sum a_j, 0, sum d_j), j <= i."""
    a = np.array([0.3, 0.2, 0.1])
    d = np.array([0.05, 0.1, 0.2])
    desc = dict(dof=3, a=a, alpha=np.zeros(3), d=d, q_lo=-np.ones(3), q_hi=np.ones(3),
                sphere_link=np.arange(3, dtype=np.int32), sphere_xyz=np.zeros((3, 3)),
                sphere_r=np.full(3, 0.01))
    c = orc.sphere_centres(orc.Robot(desc), np.zeros(3))
    np.testing.assert_allclose(c, np.stack([np.cumsum(a), np.zeros(3), np.cumsum(d)], 1), atol=1e-15)


# --------------------------------------------------------------------------
# Collision checker (plain definition) vs brute force
# --------------------------------------------------------------------------

def brute_force_min_sd(centres, r, obs, pairs):
    env = np.inf
    for s in range(len(r)):
        for o in range(len(obs)):
            env = min(env, float(np.linalg.norm(centres[s] - obs[o, :3])) - r[s] - obs[o, 3])
    slf = np.inf
    for s, t in pairs:
        slf = min(slf, float(np.linalg.norm(centres[s] - centres[t])) - r[s] - r[t])
    return env, slf


@pytest.mark.parametrize("L,per_link,grid", [([0.6, 0.5], 2, 64), ([0.5, 0.4, 0.45], 2, 32)])
def test_checker_matches_brute_force_on_grid(orc, L, per_link, grid):
    desc = planar_robot(L, per_link, radii=0.04)
    dof = len(L)
    desc["sphere_r"] = np.linspace(0.03, 0.06, dof * per_link)
    sp = draw.self_pair_candidates(desc["sphere_link"], 2) if dof >= 3 else np.zeros((0, 2), np.int32)
    rob = orc.Robot(desc, sp)
    rng = np.random.default_rng(4)
    obs = np.concatenate([rng.uniform(-1.2, 1.2, (6, 2)), np.zeros((6, 1)), rng.uniform(0.05, 0.2, (6, 1))], 1)
    axes = [np.linspace(-np.pi, np.pi, grid, endpoint=False)] * dof
    Q = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, dof)
    if len(Q) > 4096:
        Q = Q[rng.choice(len(Q), 4096, replace=False)]
    flags, sd, se, ss = orc.check(rob, obs, Q)
    for i, q in enumerate(Q):
        e, s = brute_force_min_sd(planar_centres(L, per_link, q), desc["sphere_r"], obs, sp)
        assert abs(se[i] - e) < 1e-12
        if len(sp):
            assert abs(ss[i] - s) < 1e-12
        else:
            assert np.isinf(ss[i])
        m = min(e, s)
        assert abs(sd[i] - m) < 1e-12
        if abs(m) > 1e-12:
            assert flags[i] == (m < 0)
    assert 0 < flags.mean() < 1          # both outcomes occur on the grid


def test_checker_single_pair_closed_form(orc):
    """One sphere of radius r at the tip of a 1-link arm (length l) and one
    obstacle at distance D from the base on the x axis: at q = 0 the signed
    distance is |D - l| - r - r_o."""
    desc = dict(dof=1, a=np.array([1.0]), alpha=np.zeros(1), d=np.zeros(1), q_lo=-np.ones(1),
                q_hi=np.ones(1), sphere_link=np.zeros(1, np.int32), sphere_xyz=np.zeros((1, 3)),
                sphere_r=np.array([0.1]))
    rob = orc.Robot(desc)
    for D, ro in ((1.5, 0.2), (1.25, 0.2), (0.9, 0.05)):
        f, sd, se, ss = orc.check(rob, np.array([[D, 0, 0, ro]]), np.zeros((1, 1)))
        assert abs(sd[0] - (abs(D - 1.0) - 0.1 - ro)) < 1e-15
        assert f[0] == (abs(D - 1.0) - 0.1 - ro < 0)
        assert np.isinf(ss[0])


def test_checker_obstacle_permutation_invariance(orc):
    data = workloads.load("dof7")
    rob = orc.Robot(workloads.robot(data))
    obs = data["obstacles"][:64]
    q = draw.uniform_q(7, 256, data["q_lo"], data["q_hi"])
    a = orc.check(rob, obs, q)
    perm = np.random.default_rng(5).permutation(len(obs))
    b = orc.check(rob, obs[perm], q)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# --------------------------------------------------------------------------
# Unadaptive test constants (Sec. IV-B)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("eps,delta,tau", [(0.1, 0.05, 0.5), (0.05, 0.05, 0.5), (0.005, 0.005, 0.5),
                                           (0.01, 0.05, 0.5), (0.05, 0.01, 0.3)])
def test_test_constants_chernoff_minimality_and_binomial_tail(orc, eps, delta, tau):
    from scipy.stats import binom
    for k in (1, 2, 3, 7, 20, 50):
        M, T = orc.test_constants(eps, delta, tau, k)
        dk = 6 * delta / (math.pi ** 2 * k * k)
        # M is the smallest integer with exp(-tau^2 eps M / 2) <= delta_k.
        assert math.exp(-tau * tau * eps * M / 2) <= dk * (1 + 1e-12)
        assert math.exp(-tau * tau * eps * (M - 1) / 2) > dk
        # The threshold is the largest integer count <= M (1 - tau) eps.
        assert T <= M * (1 - tau) * eps + 1e-9 < T + 1
        # A polytope whose collision fraction is exactly eps passes with
        # probability at most delta_k (exact binomial tail).
        assert binom.cdf(T, M, eps) <= dk


def test_test_constants_paper_workload_values(orc):
    # integer tie: 280 * 0.5 * 0.1 = 14 collisions are still accepted
    assert orc.test_constants(0.1, 0.05, 0.5, 1) == (280, 14)
    assert orc.test_constants(0.05, 0.05, 0.5, 1) == (559, 13)


def test_delta_schedule_sums_to_delta():
    # sum_k 6 delta / (pi^2 k^2) = delta (Basel problem)
    k = np.arange(1, 2_000_001, dtype=np.float64)
    s = np.sum(6 * 0.05 / (np.pi ** 2 * k ** 2))
    assert abs(s - 0.05) < 0.05 * 1e-6


# --------------------------------------------------------------------------
# Hit-and-run sampler
# --------------------------------------------------------------------------

def box_rows(lo, hi):
    d = len(lo)
    return np.concatenate([np.eye(d), -np.eye(d)]), np.concatenate([hi, -np.asarray(lo)])


def test_hit_and_run_start_on_segment(orc):
    A, b = box_rows(-np.ones(3), np.ones(3))
    v1, v2 = np.array([-0.5, 0.1, 0.2]), np.array([0.5, -0.3, 0.4])
    S = orc.hit_and_run(A, b, v1, v2, 0, 11, 0, 1, 4000)
    w = (S - v1) @ (v2 - v1) / np.dot(v2 - v1, v2 - v1)
    np.testing.assert_allclose(S, v1 + w[:, None] * (v2 - v1), atol=1e-14)
    from scipy.stats import kstest
    assert kstest(w, "uniform").pvalue > 1e-3


def test_hit_and_run_box_marginals_uniform(orc):
    from scipy.stats import kstest
    lo, hi = np.array([-1.0, -2.0, 0.0]), np.array([1.0, 0.5, 3.0])
    A, b = box_rows(lo, hi)
    S = orc.hit_and_run(A, b, np.array([0, 0, 1.0]), np.array([0.5, 0, 1.0]), 60, 3, 0, 1, 20000)
    assert np.all(S <= hi + 1e-12) and np.all(S >= lo - 1e-12)
    for j in range(3):
        assert kstest((S[:, j] - lo[j]) / (hi[j] - lo[j]), "uniform").pvalue > 1e-3


def test_hit_and_run_triangle_area_fractions(orc):
    """Uniform law in the triangle x >= 0, y >= 0, x + y <= 1: the fraction
    below the line x + y = s is s^2."""
    A = np.array([[-1.0, 0.0], [0.0, -1.0], [1.0, 1.0]])
    b = np.array([0.0, 0.0, 1.0])
    S = orc.hit_and_run(A, b, np.array([0.1, 0.1]), np.array([0.3, 0.2]), 60, 5, 2, 3, 40000)
    assert np.all(S @ A.T <= b + 1e-12)
    for s in (0.3, 0.5, 0.8):
        frac = np.mean(S.sum(1) <= s)
        assert abs(frac - s * s) < 4 * math.sqrt(s * s * (1 - s * s) / len(S)) + 0.01


def test_hit_and_run_streams_are_independent_of_batch(orc):
    A, b = box_rows(-np.ones(2), np.ones(2))
    v1, v2 = np.zeros(2), np.array([0.5, 0.5])
    S1 = orc.hit_and_run(A, b, v1, v2, 10, 99, 4, 2, 100)
    S2 = orc.hit_and_run(A, b, v1, v2, 10, 99, 4, 2, 37)
    np.testing.assert_array_equal(S1[:37], S2)
    S3 = orc.hit_and_run(A, b, v1, v2, 10, 99, 5, 2, 37)
    assert not np.allclose(S3, S2)


def test_hit_and_run_step_one_dimension_closed_form(orc):
    """In one dimension P = [lo, hi] and u = +-1, so the chord is [lo, hi]
    whatever the current point is: step s lands at lo + w (hi - lo) (u = +1)
    or hi - w (hi - lo) (u = -1), w the chord word (word 2 of the step's
    Philox call, counter (i, e, k, 16 s)).  Both chord ends are bounded by a
    row with |a^T u| = 1."""
    lo, hi = -0.7, 1.9
    A, b = box_rows(np.array([lo]), np.array([hi]))
    rng = np.random.default_rng(4)
    n, seed, e, k, s = 500, 12345, 3, 2, 7
    X = rng.uniform(lo, hi, size=(n, 1))
    Y, den = orc.hit_and_run_step(A, b, X, seed, e, k, s, first=40)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
    for i in range(n):
        w = orc.u01(int(orc.philox([40 + i, e, k, 16 * s], key)[2]))
        y = Y[i, 0]
        assert min(abs(y - (lo + w * (hi - lo))), abs(y - (hi - w * (hi - lo)))) <= 1e-12
    np.testing.assert_array_equal(np.abs(den), 1.0)
    assert np.all(den[:, 0] < 0) and np.all(den[:, 1] > 0)


def test_hit_and_run_step_chord_ends_on_boundary(orc):
    """A step moves along a line through x and stays in P; the two rows it
    reports as binding are the rows where that line leaves P on either side
    of x (brute force over the rows along the line's direction)."""
    A = np.array([[-1.0, 0.0], [0.0, -1.0], [1.0, 1.0], [1.0, -2.0]])
    b = np.array([0.0, 0.0, 1.0, 0.5])
    X = np.tile([[0.2, 0.2]], (300, 1))
    Y, den = orc.hit_and_run_step(A, b, X, 9, 0, 1, 1)
    assert np.all(Y @ A.T <= b + 1e-12)
    for x, y, dd in zip(X, Y, den):
        u = (y - x) / np.linalg.norm(y - x)
        au = A @ u
        t = (b - A @ x) / au
        fwd = np.where(au > 0, t, np.inf).argmin()
        bwd = np.where(au < 0, t, -np.inf).argmax()
        want = sorted([abs(au[fwd]), abs(au[bwd])])
        np.testing.assert_allclose(sorted(np.abs(dd)), want, atol=1e-9)
        assert dd[0] < 0 < dd[1]


def test_hit_and_run_steps_reproduce_the_walk(orc):
    A = np.array([[-1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 1.0, 1.0]])
    b = np.array([0.0, 0.0, 0.0, 1.0])
    v1, v2 = np.array([0.1, 0.1, 0.1]), np.array([0.3, 0.2, 0.1])
    X = orc.hit_and_run(A, b, v1, v2, 0, 21, 2, 5, 64)
    for s in range(1, 13):
        X, _ = orc.hit_and_run_step(A, b, X, 21, 2, 5, s)
    np.testing.assert_array_equal(X, orc.hit_and_run(A, b, v1, v2, 12, 21, 2, 5, 64))


# --------------------------------------------------------------------------
# Projection, gradient, tangent plane (Sec. IV-A), bisection (Sec. IV-B)
# --------------------------------------------------------------------------

def test_projection_invariants_and_brute_force(orc):
    rng = np.random.default_rng(6)
    for _ in range(300):
        d = rng.integers(2, 8)
        v1, v2, c = rng.normal(size=d), rng.normal(size=d), rng.normal(size=d) * 2
        cp, al = orc.project(v1, v2, c)
        # brute force over a fine grid of L
        w = np.linspace(0, 1, 20001)[:, None]
        P = (1 - w) * v1 + w * v2
        dist = np.linalg.norm(P - c, axis=1)
        assert np.linalg.norm(c - cp) <= dist.min() + 1e-12
        assert np.linalg.norm(c - cp) >= dist.min() - 1e-4 * np.linalg.norm(v2 - v1)
        # I1: (c - c_proj)^T (x - c_proj) <= 0 for x in L
        for x in P[::1000]:
            assert np.dot(c - cp, x - cp) <= 1e-12
        # I2: the plane through c with normal a = grad dist supports B_L(t)
        t = np.linalg.norm(c - cp)
        a = (c - cp) / t
        assert max(a @ v1, a @ v2) <= a @ c - t + 1e-12
        # I3: the projection is constant along the ray c_proj + s (c - c_proj)
        for s in (0.01, 0.3, 1.0, 3.0):
            cp2, _ = orc.project(v1, v2, cp + s * (c - cp))
            np.testing.assert_allclose(cp2, cp, atol=1e-12)


def test_projection_degenerate_segment(orc):
    v = np.array([0.3, -0.2, 0.1])
    cp, al = orc.project(v, v, np.array([1.0, 1.0, 1.0]))
    np.testing.assert_array_equal(cp, v)
    assert al == 0.0


def test_bisection_point_robot_ray_circle(orc):
    """Point robot among discs (identity kinematics, the Forest geometry):
    the boundary crossing on the ray from c_proj to c is a closed-form
    ray-circle intersection and c* lies within 2^-N_b |c - c_proj| of it,
    on the colliding side."""
    rng = np.random.default_rng(7)
    v1, v2 = np.array([-1.0, -1.0]), np.array([1.0, -1.0])
    n_ok = 0
    for _ in range(200):
        centre = rng.uniform([-1.5, 0.0], [1.5, 1.5])
        r = rng.uniform(0.2, 0.6)
        if centre[1] - r < -0.9:
            continue
        ang = rng.uniform(0, 2 * np.pi)
        c = centre + rng.uniform(0, r) * np.array([np.cos(ang), np.sin(ang)])
        out = orc.bisect_balls(centre[None], np.array([r]), v1, v2, c, 11)
        assert not out["proj_collides"]
        cp = out["c_proj"]
        u = (c - cp) / np.linalg.norm(c - cp)
        # |cp + s u - centre| = r, smallest s > 0 (cp is outside the disc)
        f = cp - centre
        bq, cq = 2 * f @ u, f @ f - r * r
        s = (-bq - math.sqrt(bq * bq - 4 * cq)) / 2
        cross = cp + s * u
        assert np.linalg.norm(out["c_star"] - cross) <= 2.0 ** -11 * np.linalg.norm(c - cp) + 1e-12
        assert np.linalg.norm(out["c_star"] - centre) < r          # still colliding
        np.testing.assert_allclose(out["a"], u, atol=1e-12)
        assert abs(out["t_star"] - np.linalg.norm(out["c_star"] - cp)) < 1e-15
        n_ok += 1
    assert n_ok > 50


def test_bisection_reports_colliding_projection(orc):
    out = orc.bisect_balls(np.array([[0.0, 0.0]]), np.array([0.5]), np.array([-0.2, 0.0]),
                           np.array([0.2, 0.0]), np.array([0.0, 0.3]), 5)
    assert out["proj_collides"]


# --------------------------------------------------------------------------
# Ordering and placing hyperplanes with step back (Sec. IV-B, IV-C)
# --------------------------------------------------------------------------

def test_place_hand_worked_step_back():
    """L from (0,0) to (1,0); one candidate at (0.5, 0.005): a = (0, 1),
    b = 0.005, r = max(0, 0) - 0.005 + 0.01 = 0.005 > 0, so Delta = 0.005
    and the row is y <= 0 (the plane touches L instead of cutting it)."""
    A, b, st, idx = oracle.place([0, 0], [1, 0], [[0.5, 0.005]], [[0, 1]], [0.005], 10, 0.01, 1e-4,
                                 np.zeros((0, 2)), np.zeros(0))
    assert st == oracle.CERTIFIED
    np.testing.assert_allclose(A, [[0.0, 1.0]])
    np.testing.assert_allclose(b, [0.0], atol=1e-15)
    # far candidate: full step back
    A, b, st, idx = oracle.place([0, 0], [1, 0], [[0.5, 0.5]], [[0, 1]], [0.5], 10, 0.01, 1e-4,
                                 np.zeros((0, 2)), np.zeros(0))
    np.testing.assert_allclose(b, [0.49])


def test_place_t_col_error():
    A, b, st, idx = oracle.place([0, 0], [1, 0], [[0.5, 5e-5]], [[0, 1]], [5e-5], 10, 0.01, 1e-4,
                                 np.zeros((0, 2)), np.zeros(0))
    assert st == oracle.IN_COLLISION and len(b) == 0


def test_place_invariants_random(orc):
    """I4 and the greedy semantics: planes come in increasing t*; every
    placed candidate lay inside all earlier planes; L stays inside every
    plane; each placed candidate is cut off by its own plane; the step back
    obeys min(t*, Delta_max) <= Delta <= Delta_max; every unplaced candidate
    is cut off by some plane unless N_f planes were placed."""
    rng = np.random.default_rng(8)
    for trial in range(100):
        d = int(rng.integers(2, 8))
        v1, v2 = rng.normal(size=d) * 0.3, rng.normal(size=d) * 0.3
        n = int(rng.integers(1, 200))
        c = rng.normal(size=(n, d))
        cs, ad, ts = [], [], []
        for x in c:
            cp, _ = orc.project(v1, v2, x)
            a = (x - cp) / np.linalg.norm(x - cp)
            s = rng.uniform(0.001, 1.0)
            cs.append(cp + s * (x - cp))
            ad.append(a)
            ts.append(np.linalg.norm(cs[-1] - cp))
        cs, ad, ts = np.array(cs), np.array(ad), np.array(ts)
        n_f = int(rng.integers(1, 12))
        dmax = float(rng.choice([0.01, 0.1]))
        A, b, st, idx = orc.place(v1, v2, cs, ad, ts, n_f, dmax, 1e-6, np.zeros((0, d)), np.zeros(0))
        assert st == oracle.CERTIFIED
        assert len(idx) == len(b) <= n_f
        assert np.all(np.diff(ts[idx]) >= 0)
        for r, j in enumerate(idx):
            np.testing.assert_allclose(A[r], ad[j])
            assert np.all(A[:r] @ cs[j] <= b[:r])                      # alive when taken
            assert A[r] @ v1 <= b[r] + 1e-12 and A[r] @ v2 <= b[r] + 1e-12
            assert A[r] @ cs[j] > b[r]
            delta = A[r] @ cs[j] - b[r]
            assert min(ts[j], dmax) - 1e-12 <= delta <= dmax + 1e-12
        if len(idx) < n_f:
            assert np.all(np.any(cs @ A.T > b, axis=1))
