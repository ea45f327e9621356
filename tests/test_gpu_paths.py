"""GPU tests of the sequential path inflation with the containment skip
(Sec. V-A):

* every inflated edge's set is bit-identical to the independent inflation of
  that edge (same parameters, edge id = global edge index), every skipped
  edge is CONTAINED with no rows;
* the skip decisions follow their definition, re-evaluated in FP64 on the
  sets wherever no endpoint lies within 1e-5 of a face;
* on the 3-DOF arm, end to end against the oracle's own path inflation
  (statuses and skip pattern equal for most seeds, like the single-edge
  runs);
* containment over all sets ignores the skipped edges' empty sets.
"""
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


def batched_paths(data, n_paths, copies=1):
    """The first n_paths paths of the batched workload as vertex lists, each
    with one extra vertex back at the middle of its last edge (that edge's
    segment lies on L and must be skipped); the list repeated `copies` times
    (the copies' edges draw other random streams)."""
    verts, counts = [], []
    for p in list(range(n_paths)) * copies:
        idx = np.nonzero(data["path_id"] == p)[0]
        e = data["edges"][idx]
        v = np.concatenate([e[:, 0], e[-1:, 1], 0.5 * (e[-1:, 0] + e[-1:, 1])])
        verts.append(v)
        counts.append(len(v))
    return np.concatenate(verts).astype(np.float32), counts


def expected_skips(A, b, nf, status, counts, verts):
    """The skip definition in FP64 on the given sets, path by path; a path is
    followed only while every containment test it needs is decided outside
    the band.  Returns {edge: expected covered_by} for the decided edges."""
    exp, g, v0 = {}, 0, 0
    for nv in counts:
        K = nv - 1
        mine = {}
        for k in range(K):
            seg = f32_up(verts[v0 + k:v0 + k + 2])
            cov, ambiguous = -1, False
            for h in range(g, g + k):
                if mine[h] != -1 or status[h] not in (0, 1):
                    continue
                F = int(nf[h])
                s = np.max(seg @ f32_up(A[h, :F]).T - f32_up(b[h, :F]))
                if abs(s) < BAND:
                    ambiguous = True
                    break
                if s < 0:
                    cov = h
                    break
            if ambiguous:
                break
            mine[g + k] = cov
            exp[g + k] = cov
        g += K
        v0 += nv
    return exp


@pytest.mark.parametrize("n_paths,copies", [(4, 1), (4, 16)])
def test_paths_equal_independent_inflation(ezo, ctx, n_paths, copies):
    """4 paths: one round holds every edge (window = the longest path); 64
    paths: windows of 2 edges, so later rounds skip edges inside sets of
    earlier rounds before inflating them."""
    data, desc = load("batched")
    rob = ezo.Robot(ctx, desc)
    dof = desc["dof"]
    verts, counts = batched_paths(data, n_paths, copies)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    prm = ezo.make_params(dof=dof, seed=3, **workloads.PARAMS["batched"])
    print_case("paths vs independent", counts)
    res = ezo.inflate_paths(ctx, rob, obs, torch.from_numpy(verts).cuda(), counts, prm)
    torch.cuda.synchronize()
    E = sum(counts) - len(counts)
    edges = np.concatenate([np.stack([verts[v0 + k:v0 + k + 2] for k in range(nv - 1)])
                            for v0, nv in zip(np.cumsum([0] + counts[:-1]), counts)]).astype(np.float32)
    assert edges.shape == (E, 2, dof)
    ind = ezo.inflate_edges(ctx, rob, obs, torch.from_numpy(edges).cuda(), prm)
    torch.cuda.synchronize()
    cov = res.covered_by.cpu().numpy()
    st, nf = res.status.cpu().numpy(), res.n_faces.cpu().numpy()
    ist, inf_ = ind.status.cpu().numpy(), ind.n_faces.cpu().numpy()
    print("covered_by", cov.tolist()[:40])
    print("status", st.tolist()[:40])
    n_inf = 0
    for g in range(E):
        if cov[g] < 0:
            n_inf += 1
            assert st[g] == ist[g] and nf[g] == inf_[g]
            F = int(nf[g])
            assert torch.equal(res.A[g, :F], ind.A[g, :F]) and torch.equal(res.b[g, :F], ind.b[g, :F])
            assert res.stats[g]["iterations"] == ind.stats[g]["iterations"]
        else:
            assert st[g] == ezo.CONTAINED and nf[g] == 0 and cov[g] < g
            assert res.stats[g]["iterations"] == 0 and res.stats[g]["exact_checks"] == 0
    # the extra vertex of every path lies on the previous edge's segment, so
    # the set holding that edge contains it -- decidedly so unless a relaxed
    # step-back plane (through an end of L, Sec. IV-C) runs along the segment
    # within rounding: required wherever it lies inside by at least BAND
    ends = np.cumsum([nv - 1 for nv in counts]) - 1
    vstart = np.cumsum([0] + counts[:-1])
    IA, Ib = ind.A.cpu().numpy(), ind.b.cpu().numpy()
    n_req = 0
    for pi, g in enumerate(ends):
        h = cov[g - 1] if cov[g - 1] >= 0 else g - 1
        if cov[g - 1] < 0 and st[g - 1] not in (ezo.CERTIFIED, ezo.MAX_ITERS):
            continue
        F = int(inf_[h])
        seg = f32_up(verts[vstart[pi] + counts[pi] - 2:vstart[pi] + counts[pi]])
        slack = np.max(seg @ f32_up(IA[h, :F]).T - f32_up(Ib[h, :F]))
        if cov[g] < 0:
            print(f"end edge {g} not skipped: slack {slack:.2e} in the set of edge {h}")
        if slack <= -BAND:
            n_req += 1
            assert cov[g] >= 0
    print(f"{n_req} of {len(ends)} backtracking end edges decidedly inside the previous set")
    exp = expected_skips(ind.A.cpu().numpy(), ind.b.cpu().numpy(), inf_, ist, counts, verts)
    print(f"{n_inf} of {E} edges inflated; {len(exp)} skip decisions checked")
    assert len(exp) >= 0.8 * E
    for g, c in exp.items():
        assert cov[g] == c, (g, cov[g], c)


def free_path_tiny(data, desc, n_extra, seed):
    """The 3-DOF edge, a vertex back at its middle, then n_extra vertices each
    joined to the previous one by a segment whose points (every 0.01 rad) are
    at least 1 cm clear of obstacles and self-collision (oracle check)."""
    rng = np.random.default_rng(seed)
    orob = oracle.Robot(desc)
    obs = f32_up(data["obstacles"])
    e = data["edges"][0].astype(np.float32)
    V = [e[0], e[1], (0.5 * (e[0] + e[1])).astype(np.float32)]
    lo, hi = np.asarray(data["q_lo"]), np.asarray(data["q_hi"])
    for _ in range(10000):
        if len(V) == 3 + n_extra:
            break
        w = np.clip(V[-1] + rng.uniform(-1.5, 1.5, size=V[-1].shape), lo + 0.05, hi - 0.05).astype(np.float32)
        pts = oracle.discretize_path(f32_up(np.stack([V[-1], w])), 0.01)
        _, sd, *_ = oracle.check(orob, obs, pts)
        if np.min(sd) > 0.01:                        # collision <=> signed distance < 0
            V.append(w)
    assert len(V) == 3 + n_extra
    return np.stack(V).astype(np.float32)


def test_paths_against_oracle_tiny(ezo, ctx):
    data, desc = load("tiny")
    rob = ezo.Robot(ctx, desc)
    orob = oracle.Robot(desc)
    dof = desc["dof"]
    obs_np = f32_up(data["obstacles"])
    obs = torch.from_numpy(data["obstacles"]).cuda()
    V = free_path_tiny(data, desc, 5, seed=5)
    print_case("paths vs oracle tiny", V.shape)
    same, n = 0, 8
    for seed in range(n):
        prm = ezo.make_params(dof=dof, seed=seed, **workloads.PARAMS["tiny"])
        res = ezo.inflate_paths(ctx, rob, obs, torch.from_numpy(V).cuda(), [len(V)], prm)
        torch.cuda.synchronize()

        def inflate(k, v1, v2):
            return oracle.eizo_arm(orob, obs_np, v1, v2,
                                   oracle.make_params(**workloads.PARAMS["tiny"], seed=seed, edge_id=k))

        o = oracle.inflate_path(inflate, f32_up(V))
        cov = res.covered_by.cpu().numpy().tolist()
        st = res.status.cpu().numpy().tolist()
        ocov = [x["covered_by"] for x in o]
        ost = [x["status"] for x in o]
        print(seed, cov, st, ocov, ost)
        assert cov[1] == ocov[1] == 0                 # back along edge 0: always contained
        same += cov == ocov and st == ost
    assert same >= 0.75 * n


def test_containment_ignores_skipped_edges(ezo, ctx):
    data, desc = load("batched")
    rob = ezo.Robot(ctx, desc)
    verts, counts = batched_paths(data, 3)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    prm = ezo.make_params(dof=desc["dof"], seed=5, **workloads.PARAMS["batched"])
    res = ezo.inflate_paths(ctx, rob, obs, torch.from_numpy(verts).cuda(), counts, prm)
    segs = []
    v0 = 0
    for nv in counts:
        segs += [verts[v0 + k:v0 + k + 2] for k in range(nv - 1)]
        v0 += nv
    segs = torch.from_numpy(np.stack(segs).astype(np.float32)).cuda()
    c = ezo.segments_contained(ctx, res.A, res.b, res.n_faces, segs)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    cov = res.covered_by.cpu().numpy()
    st = res.status.cpu().numpy()
    skipped = np.nonzero(cov >= 0)[0]
    print_case("containment", len(skipped), "skipped")
    assert len(skipped) >= len(counts)
    assert not np.isin(c, skipped).any()                  # an empty set contains nothing
    own = np.where(cov >= 0, cov, np.arange(len(cov)))
    ok = (st[own] == 0) | (st[own] == 1)
    assert np.all(c[ok] >= 0) and np.all(c[ok] <= own[ok])


def test_paths_reject_bad_input(ezo, ctx):
    data, desc = load("tiny")
    rob = ezo.Robot(ctx, desc)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    prm = ezo.make_params(dof=desc["dof"], seed=0, **workloads.PARAMS["tiny"])
    V = torch.from_numpy(data["edges"][0].astype(np.float32)).cuda()
    with pytest.raises(ezo.EzoError) as ei:
        ezo.inflate_paths(ctx, rob, obs, torch.cat([V, V[:1]]), [2, 1], prm)
    assert ei.value.code == ezo.EZO_E_INVALID
