"""What every GPU-produced polytope must satisfy, checked on the library's
own outputs against the oracle:

* every hyperplane row the fused inflation places excludes the collision
  point c* it was placed for (Sec. IV-C: the row is a^T x <= a^T c* - Delta
  with Delta > 0), and that c* truly collides (the oracle's exact check,
  outside the FP32 signed-distance band) -- the collision points a set was
  built from lie outside it;
* the probabilistic guarantee of Alg. 1's output (eq:prob_polytope_cfree):
  over R independent random streams, at most the 99.9 % quantile of
  Bin(R_certified, delta) certified sets may have a collision fraction above
  eps.  Fractions are estimated by exact rejection sampling (uniform in a
  box around P, kept if inside P) with the oracle's checker, so neither the
  hit-and-run sampler's mixing nor the GPU checker enters the estimate.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

from gpu_common import BAND, f32_up, load, print_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ezo():
    import paper_2504_10783_amd as ezo
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return ezo


@pytest.fixture(scope="module")
def ctx(ezo):
    return ezo.Context(0)


def inflate_with_points(ezo, ctx, data, desc, edges, prm):
    rob = ezo.Robot(ctx, desc)
    E, dof, cap = len(edges), desc["dof"], prm.face_capacity
    pts = torch.full((E, cap, dof), float("nan"), dtype=torch.float32, device="cuda")
    r = ezo.inflate_edges(ctx, rob, torch.from_numpy(data["obstacles"]).cuda(),
                          torch.from_numpy(np.ascontiguousarray(edges, np.float32)).cuda(), prm, row_points=pts)
    torch.cuda.synchronize()
    return (r.A.cpu().numpy().astype(np.float64), r.b.cpu().numpy().astype(np.float64), r.n_faces.cpu().numpy(),
            r.status.cpu().numpy(), pts.cpu().numpy().astype(np.float64), r.stats)


@pytest.mark.parametrize("name,n_edges,seed", [("tiny", 1, 3), ("dof7", 1, 0), ("batched", 96, 1)])
def test_placed_rows_exclude_their_collision_points(ezo, ctx, name, n_edges, seed):
    data, desc = load(name)
    dof = desc["dof"]
    edges = data["edges"][:n_edges]
    p = dict(workloads.PARAMS[name])
    if name == "batched":
        p["n_p"] = 1000
    prm = ezo.make_params(dof=dof, seed=seed, **p)
    print_case("row points", name, n_edges, seed)
    A, b, nf, st, pts, stats = inflate_with_points(ezo, ctx, data, desc, edges, prm)
    orob = oracle.Robot(desc)
    obs = f32_up(data["obstacles"])
    margins, cs = [], []
    for e in range(len(edges)):
        F = int(nf[e])
        assert np.all(np.isnan(pts[e, :2 * dof]))            # box rows carry no point
        assert np.all(np.isnan(pts[e, F:]))                   # nothing past the last row
        if F == 2 * dof:
            continue
        Ae, be, ce = A[e, 2 * dof:F], b[e, 2 * dof:F], pts[e, 2 * dof:F]
        assert np.all(np.isfinite(ce))
        m = np.einsum("fd,fd->f", Ae, ce) - be                # a^T c* - b_row = Delta
        margins.append(m)
        # c* is outside its own row, hence outside the returned set
        assert np.all(m > 0)
        assert np.all(np.max(ce @ A[e, :F].T - b[e, :F], axis=1) > 0)
        cs.append(ce)
    m, c = np.concatenate(margins), np.concatenate(cs)
    f, sd, *_ = oracle.check(orob, obs, c)
    out = np.abs(sd) >= BAND
    print(f"{name}: {len(c)} placed rows; a^T c* - b from {m.min():.2e} to {m.max():.2e}; "
          f"colliding (oracle) {f[out].mean():.4f} of {out.sum()} outside the band, {np.sum(~out)} in it")
    assert np.all(f[out] == 1)                                # every c* collides
    # Delta >= min(t*, Delta_max) > t_col for every row (Sec. IV-C)
    assert m.min() > prm.t_col * 0.5


def bounding_box(A, b, lo, hi):
    """Tightest axis box around {x : A x <= b} (linear programs)."""
    from scipy.optimize import linprog
    d = A.shape[1]
    blo, bhi = np.array(lo, float), np.array(hi, float)
    for j in range(d):
        c = np.zeros(d)
        c[j] = 1.0
        r1 = linprog(c, A_ub=A, b_ub=b, bounds=list(zip(lo, hi)), method="highs")
        r2 = linprog(-c, A_ub=A, b_ub=b, bounds=list(zip(lo, hi)), method="highs")
        assert r1.status == 0 and r2.status == 0
        blo[j], bhi[j] = max(lo[j], r1.x[j] - 1e-9), min(hi[j], r2.x[j] + 1e-9)
    return blo, bhi


def test_gpu_sets_meet_the_eps_delta_guarantee(ezo, ctx):
    """eq:prob_polytope_cfree on the tiny workload for the GPU's own sets: R =
    200 inflations of the tiny edge in one batched call (edge e draws the
    random stream of edge id e, so the runs are independent)."""
    from scipy.stats import binom
    data, desc = load("tiny")
    dof = desc["dof"]
    R, n_mc = 200, 20_000
    edges = np.repeat(data["edges"][:1], R, axis=0)
    prm = ezo.make_params(dof=dof, seed=77, **workloads.PARAMS["tiny"])
    print_case("guarantee", R)
    A, b, nf, st, pts, stats = inflate_with_points(ezo, ctx, data, desc, edges, prm)
    orob = oracle.Robot(desc)
    obs = f32_up(data["obstacles"])
    lo, hi = data["q_lo"].astype(np.float64), data["q_hi"].astype(np.float64)
    rng = np.random.default_rng(2024)
    eps, delta = prm.eps, prm.delta
    certified = np.nonzero(st == ezo.CERTIFIED)[0]
    fracs = []
    for e in certified:
        F = int(nf[e])
        Ae, be = A[e, :F], b[e, :F]
        blo, bhi = bounding_box(Ae, be, lo, hi)
        inside = []
        while sum(len(x) for x in inside) < n_mc:
            x = rng.uniform(blo, bhi, size=(4 * n_mc, dof))
            inside.append(x[np.all(x @ Ae.T <= be, axis=1)])
        x = np.concatenate(inside)[:n_mc]
        f, *_ = oracle.check(orob, obs, x)
        fracs.append(f.mean())
    fracs = np.array(fracs)
    thr = eps + 3 * math.sqrt(eps * (1 - eps) / n_mc)       # one-sided Monte-Carlo margin
    bad = int(np.sum(fracs > thr))
    allowed = binom.ppf(0.999, len(certified), delta)
    print(f"{len(certified)}/{R} certified; collision fraction mean {fracs.mean():.4f}, max {fracs.max():.4f}; "
          f"{bad} above eps (allowed {allowed:.0f}); iterations mean "
          f"{np.mean([stats[e]['iterations'] for e in certified]):.2f}")
    assert len(certified) >= R - 4
    assert bad <= allowed
