"""GPU parity of the recovery calls (Sec. V-B) against the oracle:

* ezo_check_path: the same discretisation (point count exact, points within
  FP32 rounding) and collision flags identical outside the 1e-5 m band;
* ezo_update_polytopes: on found collisions whose bisection is decided outside
  the band, the same candidates, the same placed rows in the same order
  (a, b within 1e-5) and the same status, with L kept inside every set;
* ezo_segments_contained: exact against the plain definition.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import draw

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


def match_rows(got, ref):
    """Index into ref of each row of got: rows of got come in path order, so
    each matches (within 1e-5) the first row of ref after the previous match
    (a zero-length segment repeats a point)."""
    idx, j0 = [], 0
    for g in got:
        d = np.max(np.abs(ref[j0:] - g), axis=1)
        hits = np.nonzero(d <= 1e-5)[0]
        assert len(hits) > 0, d.min()
        idx.append(j0 + int(hits[0]))
        j0 = idx[-1] + 1
    return np.array(idx, int)


@pytest.mark.parametrize("name,step,K", [("tiny", 0.02, 7), ("dof7", 0.05, 6)])
def test_check_path_parity(ezo, ctx, name, step, K):
    data, desc = load(name)
    rob = ezo.Robot(ctx, desc)
    dof = desc["dof"]
    w = draw.uniform_q(71, K, data["q_lo"], data["q_hi"])
    w[2] = w[1]                                               # a zero-length segment
    print_case("check_path", name, K, step)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    pts, n_col, n_pts = ezo.check_path(ctx, rob, obs, torch.from_numpy(w).cuda(), step, point_capacity=100000)
    torch.cuda.synchronize()
    ref_pts = oracle.discretize_path(f32_up(w), step)
    fo, sdo, *_ = oracle.check(oracle.Robot(desc), f32_up(data["obstacles"]), ref_pts)
    print(f"{n_pts} points, {n_col} colliding (oracle {int(fo.sum())})")
    assert n_pts == len(ref_pts)
    assert len(pts) == n_col
    got = pts.cpu().numpy().astype(np.float64)
    idx = match_rows(got, ref_pts)
    gflag = np.zeros(len(ref_pts), bool)
    gflag[idx] = True
    decided = np.abs(sdo) >= BAND
    assert np.array_equal(gflag[decided], fo.astype(bool)[decided])
    assert 0 < n_col < n_pts
    # a smaller capacity returns the first colliding points and the full count
    cap = max(1, n_col // 3)
    pts2, n_col2, _ = ezo.check_path(ctx, rob, obs, torch.from_numpy(w).cuda(), step, point_capacity=cap)
    torch.cuda.synchronize()
    assert n_col2 == n_col and len(pts2) == cap
    assert torch.equal(pts2, pts[:cap])


def decided_collisions(desc, data, A, b, v1, v2, n, seed, n_b=11):
    """Colliding configurations inside P (hit-and-run samples of P) whose
    membership, projection check and every bisection decision lie outside the
    band (so FP32 and FP64 agree)."""
    orob = oracle.Robot(desc)
    obs = f32_up(data["obstacles"])
    q = oracle.hit_and_run(A, b, v1, v2, 30, seed, 0, 1, 4000).astype(np.float32)
    qd = f32_up(q)
    f, sd, *_ = oracle.check(orob, obs, qd)
    slack = qd @ A.T - b
    keep = (f.astype(bool)) & (sd <= -BAND) & np.all(slack <= -1e-4, axis=1)
    out = []
    for x in q[keep]:
        r = oracle.bisect_arm(orob, obs, v1, v2, f32_up(x), n_b)
        if np.all(np.abs(r["sd_trace"]) >= BAND) and not r["proj_collides"]:
            out.append(x)
        if len(out) == n:
            break
    return np.array(out, np.float32)


def oracle_set(desc, data, name, v1, v2, seed):
    """An early, loose set of the edge from the oracle's own FP64 inflation
    (one iteration), rounded to FP32 as the GPU holds it."""
    p = dict(workloads.PARAMS[name], max_iters=1)
    if name == "dof7":
        p["n_p"] = 2000                                   # keeps the FP64 run short
    o = oracle.eizo_arm(oracle.Robot(desc), f32_up(data["obstacles"]), v1, v2,
                        oracle.make_params(**p, seed=seed, edge_id=0))
    return o["A"].astype(np.float32), o["b"].astype(np.float32), o["status"]


@pytest.mark.parametrize("name,n", [("tiny", 40), ("dof7", 120)])
def test_update_polytopes_parity(ezo, ctx, name, n):
    data, desc = load(name)
    rob = ezo.Robot(ctx, desc)
    dof = desc["dof"]
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"][:1]).cuda()
    v1, v2 = f32_up(data["edges"][0])
    A0f, b0f, st0 = oracle_set(desc, data, name, v1, v2, seed=2)
    F0 = len(b0f)
    cap = F0 + 40                                         # room for the new rows
    res = ezo.InflateResult(torch.zeros((1, cap, dof), dtype=torch.float32, device="cuda"),
                            torch.zeros((1, cap), dtype=torch.float32, device="cuda"),
                            torch.tensor([F0], dtype=torch.int32, device="cuda"),
                            torch.tensor([st0], dtype=torch.int32, device="cuda"), [])
    res.A[0, :F0] = torch.from_numpy(A0f).cuda()
    res.b[0, :F0] = torch.from_numpy(b0f).cuda()
    A0, b0 = f32_up(A0f), f32_up(b0f)
    pts = decided_collisions(desc, data, A0, b0, v1, v2, n, seed=81)
    print_case("update_polytopes", name, len(pts), "rows", F0, "status", st0)
    assert len(pts) >= 5
    # plus points outside the set, which must be ignored
    far = np.tile(np.asarray(data["q_hi"], np.float32) * 2.0, (3, 1))
    allp = np.concatenate([pts, far]).astype(np.float32)
    added = ezo.update_polytopes(ctx, rob, obs, edges, torch.from_numpy(allp).cuda(), res, n_b=11, n_f=10,
                                 step_back_max=workloads.PARAMS[name]["step_back_max"],
                                 t_col=workloads.PARAMS[name]["t_col"])
    torch.cuda.synchronize()
    F1 = int(res.n_faces[0].item())
    assert F1 == F0 + int(added[0].item()) and F1 > F0
    assert np.array_equal(res.A[0, :F0].cpu().numpy(), A0f)            # existing rows untouched
    bis = lambda a, b_, c, nb: oracle.bisect_arm(oracle.Robot(desc), f32_up(data["obstacles"]), a, b_, c, nb)
    A2, b2, st, _, idx = oracle.recover_set(bis, v1, v2, A0, b0, f32_up(allp), 11, 10,
                                            workloads.PARAMS[name]["step_back_max"], workloads.PARAMS[name]["t_col"])
    assert len(idx) == len(pts)
    assert int(res.status[0].item()) == (ezo.IN_COLLISION if st == oracle.IN_COLLISION else st0)
    assert F1 == len(b2)
    gA = res.A[0, F0:F1].cpu().numpy().astype(np.float64)
    gb = res.b[0, F0:F1].cpu().numpy().astype(np.float64)
    assert np.abs(gA - A2[F0:]).max() <= 1e-5 and np.abs(gb - b2[F0:]).max() <= 1e-5
    A1 = res.A[0, :F1].cpu().numpy().astype(np.float64)
    b1 = res.b[0, :F1].cpu().numpy().astype(np.float64)
    for v in (v1, v2):
        assert np.all(A1 @ v <= b1 + 1e-5)                            # L stays inside


def test_segments_contained_exact(ezo, ctx):
    rng = np.random.default_rng(5)
    dof, n_sets, cap, K = 4, 9, 12, 300
    A = np.zeros((n_sets, cap, dof), np.float32)
    b = np.zeros((n_sets, cap), np.float32)
    nf = np.zeros(n_sets, np.int32)
    for e in range(n_sets):
        F = int(rng.integers(2 * dof, cap + 1))
        a = rng.normal(size=(F, dof))
        a /= np.linalg.norm(a, axis=1, keepdims=True)
        A[e, :F] = a
        b[e, :F] = rng.uniform(0.3, 1.0, size=F)
        nf[e] = F
    seg = (rng.normal(size=(K, 2, dof)) * 0.35).astype(np.float32)
    print_case("segments_contained", K)
    cov = ezo.segments_contained(ctx, torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda(),
                                 torch.from_numpy(nf).cuda(), torch.from_numpy(seg).cuda())
    torch.cuda.synchronize()
    cov = cov.cpu().numpy()
    ref = np.array([oracle.covering_set([f32_up(A[e, :nf[e]]) for e in range(n_sets)],
                                        [f32_up(b[e, :nf[e]]) for e in range(n_sets)],
                                        f32_up(seg[k, 0]), f32_up(seg[k, 1])) for k in range(K)])
    # exact wherever no endpoint lies within 1e-5 of a face of a set
    near = np.zeros(K, bool)
    for e in range(n_sets):
        s = np.abs(f32_up(seg).reshape(-1, dof) @ f32_up(A[e, :nf[e]]).T - f32_up(b[e, :nf[e]])).reshape(K, 2, -1)
        near |= (s < 1e-5).any(axis=(1, 2))
    print(f"covered {np.mean(ref >= 0):.2f} of segments; {near.sum()} near a face")
    assert np.array_equal(cov[~near], ref[~near])
    assert 0.1 < np.mean(ref >= 0) < 0.95


def test_recovery_round_trip(ezo, ctx):
    """Inflate, route a trajectory through collisions inside the set, find
    them by the path check, edit the set: the found points leave the set, L
    stays inside and the segment is still covered.  GPU calls only; the
    properties are checked with plain numpy."""
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    dof = desc["dof"]
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"][:1]).cuda()
    p = dict(workloads.PARAMS["dof7"], max_iters=1)            # an early, loose set
    res = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=dof, seed=3, face_capacity=400, **p))
    # colliding configurations inside the set: hit-and-run samples, checked
    S = torch.empty((1, dof, 4096), dtype=torch.float32, device="cuda")
    ezo.sample_polytopes(ctx, dof, res.A, res.b, res.n_faces, edges, 4096, 60, 91, 0, S)
    q = S[0].t().contiguous()
    flags = torch.empty(4096, dtype=torch.uint8, device="cuda")
    ezo.check_collisions(ctx, rob, obs, q, flags)
    torch.cuda.synchronize()
    cols = q[flags.bool()][:2].cpu().numpy()
    assert len(cols) == 2
    v1, v2 = data["edges"][0].astype(np.float64)
    way = np.stack([data["edges"][0][0], cols[0], cols[1], data["edges"][0][1]]).astype(np.float32)
    print_case("recovery round trip")
    found, n_col, n_pts = ezo.check_path(ctx, rob, obs, torch.from_numpy(way).cuda(), 0.05, point_capacity=4096)
    assert n_col > 0
    added = ezo.update_polytopes(ctx, rob, obs, edges, found, res, n_b=11, n_f=200)
    torch.cuda.synchronize()
    assert int(added[0].item()) > 0
    F1 = int(res.n_faces[0].item())
    A1 = res.A[0, :F1].cpu().numpy().astype(np.float64)
    b1 = res.b[0, :F1].cpu().numpy().astype(np.float64)
    for v in (v1, v2):
        assert np.all(A1 @ v <= b1 + 1e-5)
    P = found.cpu().numpy().astype(np.float64)
    inside = np.all(P @ A1.T <= b1, axis=1)
    print(f"{n_col} found collisions, {int(added[0].item())} planes, {int(inside.sum())} still inside")
    assert inside.mean() <= 0.5
    cov = ezo.segments_contained(ctx, res.A, res.b, res.n_faces, edges)
    torch.cuda.synchronize()
    assert int(cov[0].item()) == 0


def test_recovery_reinflates_segments_the_edit_uncovered(ezo, ctx):
    """The last step of Sec. V-B: after the sets are edited, every segment of
    the path must still lie in some set; a segment that does not is inflated
    anew.  The path is inflated with the containment skip (Sec. V-A), so some
    segments hold no set of their own and are covered by an earlier edge's
    set; a found collision placed just off the middle of such a segment
    (inside the covering set, 0.004 rad from the segment, less than
    Delta_max) makes the edit cut that segment out of the set while the set's
    own segment stays inside.  The segment containment check finds it,
    ezo_inflate_edges inflates it, and then every segment of the path is
    covered again."""
    data, desc = load("batched")
    rob = ezo.Robot(ctx, desc)
    dof = desc["dof"]
    obs = torch.from_numpy(data["obstacles"]).cuda()
    pid = data["path_id"]
    p = dict(workloads.PARAMS["batched"], n_p=2000)
    prm = ezo.make_params(dof=dof, seed=4, **p)
    cap = prm.face_capacity
    # the longest path
    q = int(np.argmax(np.bincount(pid)))
    idx = np.nonzero(pid == q)[0]
    segs = data["edges"][idx]
    verts = np.concatenate([segs[:, 0], segs[-1:, 1]]).astype(np.float32)
    print_case("recovery re-inflation", len(segs), "segments")
    res = ezo.inflate_paths(ctx, rob, obs, torch.from_numpy(verts).cuda(), [len(verts)], prm)
    torch.cuda.synchronize()
    cov = res.covered_by.cpu().numpy()
    st = res.status.cpu().numpy()
    A = res.A.cpu().numpy().astype(np.float64)
    b = res.b.cpu().numpy().astype(np.float64)
    nf = res.n_faces.cpu().numpy()
    # a contained segment g (covered by h) and a point 0.004 rad off its middle
    # on the side away from h's segment, well inside h's set
    pick = None
    for g in np.nonzero(cov >= 0)[0]:
        h = int(cov[g])
        v1, v2 = segs[h].astype(np.float64)
        m = 0.5 * (segs[g, 0] + segs[g, 1]).astype(np.float64)
        cp, _ = oracle.project(v1, v2, m)
        if np.linalg.norm(m - cp) < 0.05:
            continue
        x = m + 0.004 * (m - cp) / np.linalg.norm(m - cp)
        Ah, bh = A[h, :nf[h]], b[h, :nf[h]]
        if np.all(Ah @ x <= bh - 0.02) and np.all(Ah @ m <= bh - 0.02):
            pick = (int(g), h, x)
            break
    assert pick is not None, "no contained segment with room around its middle"
    g, h, x = pick
    seeds = torch.from_numpy(np.ascontiguousarray(segs, np.float32)).cuda()
    added = ezo.update_polytopes(ctx, rob, obs, seeds, torch.from_numpy(x[None].astype(np.float32)).cuda(), res,
                                 n_b=11, n_f=10)
    torch.cuda.synchronize()
    assert int(added[h].item()) >= 1
    Fh = int(res.n_faces[h].item())
    Ah = res.A[h, :Fh].cpu().numpy().astype(np.float64)
    bh = res.b[h, :Fh].cpu().numpy().astype(np.float64)
    assert np.any(Ah @ x > bh)                                      # the found point is excluded
    for v in segs[h].astype(np.float64):
        assert np.all(Ah @ v <= bh + 1e-5)                          # the set's own segment stays
    # every path segment against every set: g is no longer covered
    covered = ezo.segments_contained(ctx, res.A, res.b, res.n_faces, seeds).cpu().numpy()
    missing = np.nonzero(covered < 0)[0]
    print(f"segment {g} covered by {h}; after the edit uncovered: {missing.tolist()}")
    assert g in missing
    # inflate the missing segments, append their sets, check again
    new = ezo.inflate_edges(ctx, rob, obs, seeds[missing].contiguous(),
                            ezo.make_params(dof=dof, seed=5, edge_id_base=1000, **p))
    torch.cuda.synchronize()
    assert np.all(new.status.cpu().numpy() == ezo.CERTIFIED)
    A2 = torch.cat([res.A, new.A])
    b2 = torch.cat([res.b, new.b])
    n2 = torch.cat([res.n_faces, new.n_faces])
    covered2 = ezo.segments_contained(ctx, A2, b2, n2, seeds).cpu().numpy()
    assert np.all(covered2 >= 0)
    assert covered2[g] >= len(segs)                                 # g now lies in its own new set
