"""GPU parity of the individual EI-ZO steps (Alg. 1) against the oracle, on
the same inputs:

* UniformSample   -- hit-and-run walks (same Philox stream) inside the same P;
* UnadaptiveTest + candidate selection -- bit-exact against numpy;
* ProjectPoints + UpdatePointsViaBisection -- per candidate, wherever no
  evaluated point lies within the 1e-5 m signed-distance band;
* OrderAndPlaceHyperplanes -- same rows in the same order.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import draw

from gpu_common import BAND, bisection_agreement, f32_up, load, print_case, sampler_step_replay

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


def oracle_polytope(name, iters):
    """A realistic P: the oracle's own polytope after `iters` iterations,
    rounded to FP32 (both sides then read the same rows)."""
    data, desc = load(name)
    orob = oracle.Robot(desc)
    v1, v2 = f32_up(data["edges"][0])
    prm = oracle.make_params(**dict(workloads.PARAMS[name], max_iters=iters), seed=1)
    out = oracle.eizo_arm(orob, f32_up(data["obstacles"]), v1, v2, prm)
    return data, desc, out["A"].astype(np.float32), out["b"].astype(np.float32)


@pytest.mark.parametrize("name,iters,n_mix", [("tiny", 0, 0), ("tiny", 0, 30), ("tiny", 2, 30), ("dof7", 2, 60),
                                              ("dof7", 4, 60)])
def test_sampler_step_replay(ezo, ctx, name, iters, n_mix):
    """Hit-and-run (Sec. IV-B) replayed step by step against the oracle on
    4099 walks (a ragged count) inside the joint box or the oracle's own
    polytope after `iters` iterations."""
    print_case("sampler step replay", name, iters, n_mix)
    if iters == 0:
        data, desc = load(name)
        A, b = oracle.Robot(desc).box()
        A, b = A.astype(np.float32), b.astype(np.float32)
    else:
        data, desc, A, b = oracle_polytope(name, iters)
    dof = desc["dof"]
    F, cap = len(b), len(b) + 8
    At = torch.zeros((1, cap, dof), dtype=torch.float32, device="cuda")
    bt = torch.zeros((1, cap), dtype=torch.float32, device="cuda")
    At[0, :F] = torch.from_numpy(A).cuda()
    bt[0, :F] = torch.from_numpy(b).cuda()
    nf = torch.tensor([F], dtype=torch.int32, device="cuda")
    edges = torch.from_numpy(data["edges"][:1]).cuda()
    sampler_step_replay(ezo, ctx, dof, At, bt, nf, edges, 4099, n_mix, seed=7, k=3, eid=5,
                        label=f"{name} k={iters}")


def test_sampler_marginals_match_oracle(ezo, ctx):
    """Whole walks (dof7, P after two iterations): the GPU's final samples and
    the oracle's FP64 walks from the same stream have indistinguishable
    coordinate marginals (two-sample KS)."""
    from scipy.stats import ks_2samp
    data, desc, A, b = oracle_polytope("dof7", 2)
    dof = desc["dof"]
    n, seed, k, eid = 4099, 7, 3, 5
    print_case("sampler marginals", n)
    F, cap = len(b), len(b) + 8
    At = torch.zeros((1, cap, dof), dtype=torch.float32, device="cuda")
    bt = torch.zeros((1, cap), dtype=torch.float32, device="cuda")
    At[0, :F] = torch.from_numpy(A).cuda()
    bt[0, :F] = torch.from_numpy(b).cuda()
    S = torch.empty((1, dof, 4160), dtype=torch.float32, device="cuda")
    ezo.sample_polytopes(ctx, dof, At, bt, torch.tensor([F], dtype=torch.int32, device="cuda"),
                         torch.from_numpy(data["edges"][:1]).cuda(), n, 60, seed=seed, iteration=k, samples=S,
                         edge_id_base=eid)
    torch.cuda.synchronize()
    got = S[0, :, :n].cpu().numpy().T.astype(np.float64)
    v1, v2 = f32_up(data["edges"][0])
    ref = oracle.hit_and_run(f32_up(A), f32_up(b), v1, v2, 60, seed, eid, k, n)
    for j in range(dof):
        assert ks_2samp(got[:, j], ref[:, j]).pvalue > 1e-3


def test_test_and_select_bit_exact(ezo, ctx):
    rng = np.random.default_rng(0)
    E, stride, n = 5, 10048, 10000
    flags = (rng.random((E, stride)) < np.array([0.0, 0.01, 0.3, 0.9, 1.0])[:, None]).astype(np.uint8)
    for (M, T, n_p) in ((559, 13, 10000), (1810, 45, 100), (10000, 5000, 3000), (280, 14, 1)):
        print_case("test_and_select", M, T, n_p)
        ft = torch.from_numpy(flags).cuda()
        ci = torch.full((E, 10000), -1, dtype=torch.int32, device="cuda")
        nc = torch.empty(E, dtype=torch.int32, device="cuda")
        acc = torch.empty(E, dtype=torch.uint8, device="cuda")
        cnt = torch.empty(E, dtype=torch.int32, device="cuda")
        ezo.test_and_select(ctx, ft, n, M, T, n_p, ci, nc, acc, cnt)
        torch.cuda.synchronize()
        for e in range(E):
            c = int(flags[e, :M].sum())
            assert cnt[e].item() == c
            assert acc[e].item() == (c <= T)
            if c <= T:
                assert nc[e].item() == 0
            else:
                idx = np.nonzero(flags[e, :n])[0][:n_p]
                assert nc[e].item() == len(idx)
                assert np.array_equal(ci[e, :len(idx)].cpu().numpy(), idx)


def colliding_candidates(ezo, ctx, name, n_want, seed):
    """Samples of the oracle's polytope after one iteration that collide."""
    data, desc, A, b = oracle_polytope(name, 1)
    v1, v2 = f32_up(data["edges"][0])
    S = oracle.hit_and_run(f32_up(A), f32_up(b), v1, v2, 10, seed, 0, 2, 4 * n_want).astype(np.float32)
    fo, sdo, *_ = oracle.check(oracle.Robot(desc), f32_up(data["obstacles"]), f32_up(S))
    cand = S[fo.astype(bool)][:n_want]
    return data, desc, cand


@pytest.mark.parametrize("name,n", [("tiny", 300), ("dof7", 700)])
def test_project_bisect_parity(ezo, ctx, name, n):
    print_case("project_bisect", name, n)
    data, desc, cand = colliding_candidates(ezo, ctx, name, n, seed=3)
    n = len(cand)
    dof = desc["dof"]
    rob = ezo.Robot(ctx, desc)
    stride = n + 5
    S = torch.zeros((1, dof, stride), dtype=torch.float32, device="cuda")
    S[0, :, :n] = torch.from_numpy(np.ascontiguousarray(cand.T)).cuda()
    cap = n + 3                                            # ragged tail
    ci = torch.zeros((1, cap), dtype=torch.int32, device="cuda")
    ci[0, :n] = torch.arange(n, dtype=torch.int32, device="cuda")
    nc = torch.tensor([n], dtype=torch.int32, device="cuda")
    cs = torch.empty((1, dof, cap), dtype=torch.float32, device="cuda")
    ad = torch.empty((1, dof, cap), dtype=torch.float32, device="cuda")
    ts = torch.empty((1, cap), dtype=torch.float32, device="cuda")
    pc = torch.empty((1, cap), dtype=torch.uint8, device="cuda")
    edges = torch.from_numpy(data["edges"][:1]).cuda()
    obs = torch.from_numpy(data["obstacles"]).cuda()
    ezo.project_bisect(ctx, rob, obs, edges, S, ci, nc, 11, cs, ad, ts, pc)
    torch.cuda.synchronize()
    cs, ad, ts, pc = (x.cpu().numpy() for x in (cs, ad, ts, pc))
    orob = oracle.Robot(desc)
    v1, v2 = f32_up(data["edges"][0])
    steps = []
    for j in range(n):
        o = oracle.bisect_arm(orob, f32_up(data["obstacles"]), v1, v2, f32_up(cand[j]), 11)
        assert np.abs(ad[0, :, j] - o["a"]).max() <= 1e-5
        steps.append(bisection_agreement(cs[0, :, j], ts[0, j], pc[0, j], o, f32_up(cand[j])))
    steps = np.array(steps)
    print(f"bisection steps decided outside the band: mean {steps.mean():.2f} of 11; "
          f"all 11 for {np.mean(steps == 11):.2f} of candidates")
    assert np.mean(steps >= 8) >= 0.9


def synthetic_candidates(rng, dof, n):
    v1, v2 = rng.normal(size=dof) * 0.3, rng.normal(size=dof) * 0.3
    c = rng.normal(size=(n, dof))
    cs, ad, ts = [], [], []
    for x in c:
        cp, _ = oracle.project(v1, v2, x)
        a = (x - cp) / np.linalg.norm(x - cp)
        s = rng.uniform(0.001, 1.0)
        cs.append(cp + s * (x - cp))
        ad.append(a)
        ts.append(np.linalg.norm(cs[-1] - cp))
    f = np.float32
    return (v1.astype(f), v2.astype(f), np.array(cs, f), np.array(ad, f), np.array(ts, f))


def sphere_candidates(rng, dof, n):
    """Collision points on the unit sphere around a short segment, all at
    nearly the same distance t*: each placed row separates only a small cap
    of them, so many rows are placed."""
    v1, v2 = np.zeros(dof), np.zeros(dof)
    v2[0] = 1e-3
    cs, ad, ts = [], [], []
    for _ in range(n):
        u = rng.normal(size=dof)
        x = 0.5 * (v1 + v2) + u / np.linalg.norm(u)
        cp, _ = oracle.project(v1, v2, x)
        cs.append(cp + rng.uniform(0.9, 1.0) * (x - cp))
        ad.append((x - cp) / np.linalg.norm(x - cp))
        ts.append(np.linalg.norm(cs[-1] - cp))
    f = np.float32
    return (v1.astype(f), v2.astype(f), np.array(cs, f), np.array(ad, f), np.array(ts, f))


def place_parity(ezo, ctx, dof, n_f, v1, v2, cs, ad, ts):
    n = len(ts)
    E, capc, capf = 1, n + 7, 2 * dof + n_f
    edges = torch.from_numpy(np.stack([v1, v2])[None]).cuda()
    cst = torch.zeros((E, dof, capc), dtype=torch.float32, device="cuda")
    adt = torch.zeros((E, dof, capc), dtype=torch.float32, device="cuda")
    tst = torch.zeros((E, capc), dtype=torch.float32, device="cuda")
    cst[0, :, :n] = torch.from_numpy(np.ascontiguousarray(cs.T)).cuda()
    adt[0, :, :n] = torch.from_numpy(np.ascontiguousarray(ad.T)).cuda()
    tst[0, :n] = torch.from_numpy(ts).cuda()
    nc = torch.tensor([n], dtype=torch.int32, device="cuda")
    A = torch.zeros((E, capf, dof), dtype=torch.float32, device="cuda")
    b = torch.zeros((E, capf), dtype=torch.float32, device="cuda")
    nf = torch.tensor([2 * dof], dtype=torch.int32, device="cuda")
    status = torch.tensor([-1], dtype=torch.int32, device="cuda")
    placed = torch.full((E, n_f), -1, dtype=torch.int32, device="cuda")
    npl = torch.zeros(E, dtype=torch.int32, device="cuda")
    ezo.place_hyperplanes(ctx, dof, edges, cst, adt, tst, nc, n_f, 0.01, 1e-4, A, b, nf, status, placed, npl)
    torch.cuda.synchronize()
    Ao, bo, st, idx = oracle.place(f32_up(v1), f32_up(v2), f32_up(cs), f32_up(ad), f32_up(ts), n_f, 0.01, 1e-4,
                                   np.zeros((0, dof)), np.zeros(0))
    assert status.item() == -1 and st == oracle.CERTIFIED
    k = npl.item()
    assert k == len(idx) and nf.item() == 2 * dof + k
    assert np.array_equal(placed[0, :k].cpu().numpy(), idx)
    assert np.abs(A[0, 2 * dof:2 * dof + k].cpu().numpy() - Ao).max() <= 1e-6
    assert np.abs(b[0, 2 * dof:2 * dof + k].cpu().numpy() - bo).max() <= 1e-5
    return k


@pytest.mark.parametrize("dof,n,n_f", [(3, 50, 10), (7, 2000, 10), (7, 6000, 10), (7, 10000, 20), (2, 1, 10)])
def test_place_parity(ezo, ctx, dof, n, n_f):
    """Up to 4096 candidates are held with their directions in registers, up
    to 8192 without them, the rest re-read from memory every round."""
    print_case("place", dof, n, n_f)
    rng = np.random.default_rng(dof * 1000 + n)
    place_parity(ezo, ctx, dof, n_f, *synthetic_candidates(rng, dof, n))


@pytest.mark.parametrize("dof,n,n_f", [(3, 5000, 100), (4, 6000, 100)])
def test_place_many_rows_parity(ezo, ctx, dof, n, n_f):
    """More rows in one call than the kernel keeps in LDS until its end (64):
    the later rows are written as they are placed."""
    print_case("place many rows", dof, n, n_f)
    rng = np.random.default_rng(dof * 77 + n)
    assert place_parity(ezo, ctx, dof, n_f, *sphere_candidates(rng, dof, n)) > 64


def test_place_t_col_aborts_edge(ezo, ctx):
    dof = 2
    edges = torch.tensor([[[0.0, 0.0], [1.0, 0.0]]], dtype=torch.float32, device="cuda")
    cs = torch.tensor([[[0.5], [5e-5]]], dtype=torch.float32, device="cuda")
    ad = torch.tensor([[[0.0], [1.0]]], dtype=torch.float32, device="cuda")
    ts = torch.tensor([[5e-5]], dtype=torch.float32, device="cuda")
    nc = torch.tensor([1], dtype=torch.int32, device="cuda")
    A = torch.zeros((1, 8, 2), dtype=torch.float32, device="cuda")
    b = torch.zeros((1, 8), dtype=torch.float32, device="cuda")
    nf = torch.tensor([4], dtype=torch.int32, device="cuda")
    status = torch.tensor([-1], dtype=torch.int32, device="cuda")
    ezo.place_hyperplanes(ctx, dof, edges, cs, ad, ts, nc, 4, 0.01, 1e-4, A, b, nf, status)
    torch.cuda.synchronize()
    assert status.item() == ezo.IN_COLLISION and nf.item() == 4
