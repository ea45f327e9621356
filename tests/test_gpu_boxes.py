"""GPU parity of the box collision geometry (Sec. IV-D: box and sphere
geometries) against the oracle:

* raw check of the 11-box arm among voxel spheres and a table box, flags and
  signed distances, with and without the table;
* a sphere arm against an obstacle box;
* projection + bisection of the box arm's colliding samples;
* the obstacle-box call's errors, removal, and the inflation graph following
  a change of the obstacle boxes.

Box-box values: the kernel evaluates every separating axis from products
of the components of A_i x B_j, so its own arithmetic keeps full relative
precision on nearly parallel edges; what remains is the conditioning of the
problem itself.  The FP32 forward kinematics rotates each box by about 1e-7
rad away from the FP64 pose, which turns a cross axis of |A_i x B_j| by
about 1e-7 / |A_i x B_j| and moves its value by that times the centre
distance (about 1 m): <= 1e-5 m for |A_i x B_j| >= WEAK_AXIS = 0.01.  The
oracle marks configurations whose value (fragile bit 0) or sign (bit 1)
rests on a weaker cross axis, and their fractions are printed; measured, the
errors on them stay as small as elsewhere (a few 1e-7 m), so no
configuration is excluded: flags must agree wherever the oracle's minimum
lies outside +-1e-5 m (the band of the sphere checker), and signed distances
agree to 1e-5 m everywhere.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import draw

from gpu_common import bisection_agreement, f32_up, load, print_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BOX_BAND = 1e-5
WEAK_AXIS = 0.01


@pytest.fixture(scope="module", autouse=True)
def fragility_thresholds():
    oracle.set_fragility(WEAK_AXIS, BOX_BAND)
    yield
    oracle.set_fragility()


@pytest.fixture(scope="module")
def ezo():
    import paper_2504_10783_amd as ezo
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return ezo


@pytest.fixture(scope="module")
def ctx(ezo):
    return ezo.Context(0)


def compare(ezo, ctx, desc, obs_np, ebox, q, label):
    rob = ezo.Robot(ctx, desc)
    ctx.set_obstacle_boxes(ebox)
    try:
        obs = torch.from_numpy(np.ascontiguousarray(obs_np, np.float32)).cuda()
        qt = torch.from_numpy(q).cuda()
        n = len(q)
        flags = torch.empty(n, dtype=torch.uint8, device="cuda")
        flags_sd = torch.empty(n, dtype=torch.uint8, device="cuda")
        msd = torch.empty(n, dtype=torch.float32, device="cuda")
        mss = torch.empty(n, dtype=torch.float32, device="cuda")
        ezo.check_collisions(ctx, rob, obs, qt, flags)
        ezo.check_collisions(ctx, rob, obs, qt, flags_sd, msd, mss)
        torch.cuda.synchronize()
    finally:
        ctx.set_obstacle_boxes(None)
    f, sd, se, ss, fr = oracle.check(oracle.Robot(desc), f32_up(obs_np), f32_up(q),
                                     env_boxes=None if ebox is None else f32_up(ebox), fragile=True)
    g, gs, gsd, gss = (x.cpu().numpy() for x in (flags, flags_sd, msd, mss))
    ok = np.abs(sd) >= BOX_BAND
    weak = (fr & 1) != 0
    print(f"{label}: {n} configs, collision {f.mean():.3f}, in band {np.mean(np.abs(sd) < BOX_BAND):.4f}, "
          f"fragile value {np.mean(weak):.4f} sign {np.mean((fr & 2) > 0):.4f}, "
          f"max |sd err| {np.abs(gsd - sd).max():.2e} (on fragile ones "
          f"{np.abs(gsd - sd)[weak].max() if weak.any() else 0.0:.2e}), "
          f"flags differing outside the band {int(np.sum((g != f) & ok))}")
    assert np.array_equal(g[ok], f[ok]) and np.array_equal(gs[ok], f[ok])
    assert np.abs(gsd - sd).max() <= BOX_BAND
    fin = np.isfinite(ss)
    assert np.abs(gss[fin] - ss[fin]).max() <= BOX_BAND
    assert np.all(np.isinf(gss[~fin]))
    return f


@pytest.mark.parametrize("table", [True, False])
def test_box_arm_check_parity(ezo, ctx, table):
    data, desc = load("boxes")
    q = draw.uniform_q(21, 20001, data["q_lo"], data["q_hi"])          # ragged tail
    print_case("box check", "table" if table else "no table", len(q))
    f = compare(ezo, ctx, desc, data["obstacles"], data["env_boxes"] if table else None, q, "boxes")
    assert 0.2 < f.mean() < 0.95


def test_sphere_arm_against_obstacle_box(ezo, ctx):
    data, desc = load("dof7")
    box = load("boxes")[0]["env_boxes"]
    q = draw.uniform_q(22, 8000, data["q_lo"], data["q_hi"])
    print_case("sphere arm vs box", len(q))
    f = compare(ezo, ctx, desc, data["obstacles"], box, q, "spheres+table")
    assert f.mean() > 0.3


def test_box_arm_bisection_parity(ezo, ctx):
    data, desc = load("boxes")
    dof = desc["dof"]
    rob = ezo.Robot(ctx, desc)
    orob = oracle.Robot(desc)
    obs_np, eb = f32_up(data["obstacles"]), f32_up(data["env_boxes"])
    v1, v2 = f32_up(data["edges"][0])
    A, b = orob.box()
    S = oracle.hit_and_run(A, b, v1, v2, 10, 5, 0, 1, 800).astype(np.float32)
    fo, *_ = oracle.check(orob, obs_np, f32_up(S), env_boxes=eb)
    cand = S[fo.astype(bool)][:150]
    n = len(cand)
    print_case("box bisection", n)
    St = torch.zeros((1, dof, n + 5), dtype=torch.float32, device="cuda")
    St[0, :, :n] = torch.from_numpy(np.ascontiguousarray(cand.T)).cuda()
    ci = torch.arange(n, dtype=torch.int32, device="cuda")[None]
    nc = torch.tensor([n], dtype=torch.int32, device="cuda")
    cs = torch.empty((1, dof, n), dtype=torch.float32, device="cuda")
    ad = torch.empty((1, dof, n), dtype=torch.float32, device="cuda")
    ts = torch.empty((1, n), dtype=torch.float32, device="cuda")
    pc = torch.empty((1, n), dtype=torch.uint8, device="cuda")
    ctx.set_obstacle_boxes(data["env_boxes"])
    try:
        ezo.project_bisect(ctx, rob, torch.from_numpy(data["obstacles"]).cuda(),
                           torch.from_numpy(data["edges"][:1]).cuda(), St, ci, nc, 11, cs, ad, ts, pc)
        torch.cuda.synchronize()
    finally:
        ctx.set_obstacle_boxes(None)
    cs, ad, ts, pc = (x.cpu().numpy() for x in (cs, ad, ts, pc))
    steps, skipped = [], 0
    t = np.arange(2049) / 2048.0
    for j in range(n):
        o = oracle.bisect_arm(orob, obs_np, v1, v2, f32_up(cand[j]), 11, env_boxes=eb)
        assert np.abs(ad[0, :, j] - o["a"]).max() <= 1e-5
        # every midpoint lies at a dyadic fraction of [c_proj, c]; skip the
        # candidate if the flag of any of them may change (fragile sign)
        pts = o["c_proj"][None] + t[:, None] * (f32_up(cand[j]) - o["c_proj"])[None]
        *_, fr = oracle.check(orob, obs_np, pts, env_boxes=eb, fragile=True)
        if (fr & 2).any():
            skipped += 1
            continue
        steps.append(bisection_agreement(cs[0, :, j], ts[0, j], pc[0, j], o, f32_up(cand[j]), band=BOX_BAND))
    steps = np.array(steps)
    print(f"{len(steps)} candidates compared ({skipped} with a fragile midpoint skipped); "
          f"decided steps mean {steps.mean():.2f} of 11")
    assert skipped <= 0.2 * n and np.mean(steps >= 8) >= 0.9


def test_obstacle_box_errors_and_removal(ezo, ctx):
    data, desc = load("boxes")
    bad = np.array(data["env_boxes"], np.float32)
    with pytest.raises(ezo.EzoError) as ei:
        ctx.set_obstacle_boxes(np.repeat(bad, 65, axis=0))
    assert ei.value.code == ezo.EZO_E_UNSUPPORTED
    nan = bad.copy()
    nan[0, 4] = np.nan
    with pytest.raises(ezo.EzoError) as ei:
        ctx.set_obstacle_boxes(nan)
    assert ei.value.code == ezo.EZO_E_INVALID
    neg = bad.copy()
    neg[0, 13] = -0.1
    with pytest.raises(ezo.EzoError):
        ctx.set_obstacle_boxes(neg)
    # set, then remove: flags equal those of a context that never had boxes
    rob = ezo.Robot(ctx, desc)
    q = torch.from_numpy(draw.uniform_q(23, 4096, data["q_lo"], data["q_hi"])).cuda()
    obs = torch.from_numpy(data["obstacles"]).cuda()
    f1 = torch.empty(4096, dtype=torch.uint8, device="cuda")
    f2 = torch.empty_like(f1)
    f3 = torch.empty_like(f1)
    ezo.check_collisions(ctx, rob, obs, q, f1)
    ctx.set_obstacle_boxes(bad)
    ezo.check_collisions(ctx, rob, obs, q, f2)
    ctx.set_obstacle_boxes(None)
    ezo.check_collisions(ctx, rob, obs, q, f3)
    torch.cuda.synchronize()
    assert torch.equal(f1, f3) and int(f2.sum()) > int(f1.sum())
    assert bool(((f2 == 1) | (f1 == 0)).all())                 # the table only adds collisions


def test_box_arm_inflation_and_graph_follows_box_change(ezo, ctx):
    """The box arm's edge inflates (L in P in D, certified); an inflation
    on a context whose obstacle boxes were changed between calls equals one
    on a fresh context."""
    data, desc = load("boxes")
    dof = desc["dof"]
    rob = ezo.Robot(ctx, desc)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"]).cuda()
    prm = ezo.make_params(dof=dof, seed=4, **workloads.PARAMS["boxes"])
    print_case("box inflation")
    ctx.set_obstacle_boxes(data["env_boxes"])
    r1 = ezo.inflate_edges(ctx, rob, obs, edges, prm)
    ctx.set_obstacle_boxes(None)
    r2 = ezo.inflate_edges(ctx, rob, obs, edges, prm)
    torch.cuda.synchronize()
    st = int(r1.status[0].item())
    F = int(r1.n_faces[0].item())
    print("status", st, "faces", F, "iterations", r1.stats[0]["iterations"], "without table", int(r2.n_faces[0].item()))
    assert st == ezo.CERTIFIED
    A = r1.A[0, :F].cpu().numpy().astype(np.float64)
    b = r1.b[0, :F].cpu().numpy().astype(np.float64)
    for v in data["edges"][0].astype(np.float64):
        assert np.all(A @ v <= b + 1e-5)
    for with_table, r in ((True, r1), (False, r2)):
        c2 = ezo.Context(0)
        if with_table:
            c2.set_obstacle_boxes(data["env_boxes"])
        ref = ezo.inflate_edges(c2, ezo.Robot(c2, desc), obs.clone(), edges.clone(), prm)
        torch.cuda.synchronize()
        assert torch.equal(ref.status, r.status) and torch.equal(ref.n_faces, r.n_faces)
        Fr = int(ref.n_faces[0].item())
        assert torch.equal(ref.A[0, :Fr], r.A[0, :Fr]) and torch.equal(ref.b[0, :Fr], r.b[0, :Fr])


def test_box_arm_full_runs_agree_with_oracle(ezo, ctx):
    """Whole inflations of the box arm's edge (reduced N_p) against the
    oracle's own: statuses equal, iterations and face counts equal on most
    seeds, as for the single-edge sphere runs."""
    data, desc = load("boxes")
    dof = desc["dof"]
    rob = ezo.Robot(ctx, desc)
    orob = oracle.Robot(desc)
    p = dict(workloads.PARAMS["boxes"], n_p=1000, eps=0.1)
    v1, v2 = f32_up(data["edges"][0])
    ctx.set_obstacle_boxes(data["env_boxes"])
    same_it = same_f = 0
    n = 4
    try:
        for seed in range(n):
            r = ezo.inflate_edges(ctx, rob, torch.from_numpy(data["obstacles"]).cuda(),
                                  torch.from_numpy(data["edges"]).cuda(), ezo.make_params(dof=dof, seed=seed, **p))
            torch.cuda.synchronize()
            o = oracle.eizo_arm(orob, f32_up(data["obstacles"]), v1, v2, oracle.make_params(**p, seed=seed),
                                env_boxes=f32_up(data["env_boxes"]))
            st = int(r.status[0].item())
            print(seed, st, o["status"], r.stats[0]["iterations"], o["stats"]["iterations"],
                  int(r.n_faces[0].item()), len(o["b"]))
            assert st == o["status"]
            same_it += r.stats[0]["iterations"] == o["stats"]["iterations"]
            same_f += int(r.n_faces[0].item()) == len(o["b"])
    finally:
        ctx.set_obstacle_boxes(None)
    assert same_it >= n // 2 and same_f >= n // 2


def max_robot(seed=77):
    """The largest robot the library takes (include/ezo.h limits): 8 joints,
    1024 spheres (128 per link, radii halved), 64 link boxes (8 per link,
    small cuboids along each link); 6 000 sphere self pairs drawn from the
    pairs of links at least two apart that are 2 cm clear at q = 0 (spread
    over the link pairs) and every box pair of links at least three apart;
    obstacle spheres and the 64 obstacle boxes beside the arm."""
    rng = draw.rng_for(seed)
    desc = draw.arm_dh(rng, dof=8, spheres_per_link=128)
    desc["sphere_r"] = (desc["sphere_r"] * 0.5).astype(np.float32)
    cand = draw.self_pair_candidates(desc["sphere_link"], 2)
    x0 = oracle.sphere_centres(oracle.Robot(dict(desc, self_pairs=np.zeros((0, 2), np.int32))), np.zeros(8))
    r = desc["sphere_r"].astype(np.float64)
    gap = np.linalg.norm(x0[cand[:, 0]] - x0[cand[:, 1]], axis=1) - r[cand[:, 0]] - r[cand[:, 1]]
    cand = cand[gap > 0.02]
    desc["self_pairs"] = cand[np.sort(rng.choice(len(cand), 6000, replace=False))]
    a, d, al = (np.asarray(desc[k], np.float64) for k in ("a", "d", "alpha"))
    prev = np.stack([-a, -d * np.sin(al), -d * np.cos(al)], axis=1)
    link, pose, half = [], [], []
    for i in range(8):
        for j in range(8):
            c = (1.0 - (j + 0.5) / 8) * prev[i]
            link.append(i)
            pose.append(np.concatenate([c, np.eye(3).ravel()]))
            half.append([0.02, 0.03, 0.025])
    bl = np.asarray(link, np.int32)
    i, j = np.triu_indices(64, k=1)
    keep = np.abs(bl[i] - bl[j]) >= 3
    desc.update(box_link=bl, box_pose=np.asarray(pose, np.float32), box_half=np.asarray(half, np.float32),
                box_pairs=np.stack([i[keep], j[keep]], axis=1).astype(np.int32))
    obs = draw.obstacle_candidates(rng, 64, [0.6, -1.0, 0.0], [1.6, 1.0, 1.2], 0.02, 0.06)
    ebox = np.zeros((64, 15), np.float32)
    ebox[:, :3] = rng.uniform([-1.6, -1.0, 0.0], [-0.6, 1.0, 1.2], size=(64, 3))
    ebox[:, 3:12] = np.eye(3).ravel()
    ebox[:, 12:] = 0.04
    return desc, obs, ebox


def test_max_size_robot_check_and_bisection(ezo, ctx):
    """Every size at its maximum at once (dof, spheres, link boxes, obstacle
    boxes): the checker in flags and signed-distance mode on a ragged batch,
    and the projection + bisection, whose tile then only just fits the
    workgroup's LDS, against the oracle."""
    desc, obs_np, ebox = max_robot()
    assert len(desc["sphere_r"]) == 1024 and len(desc["box_link"]) == 64 and desc["dof"] == 8
    q = draw.uniform_q(23, 333, desc["q_lo"], desc["q_hi"])
    print_case("max robot check", len(q))
    f = compare(ezo, ctx, desc, obs_np, ebox, q, "max robot")
    assert 0.05 < f.mean() < 0.99
    # projection + bisection of a few colliding configurations toward an edge
    orob = oracle.Robot(desc)
    ob64, eb64 = f32_up(obs_np), f32_up(ebox)
    v1, v2 = f32_up(np.zeros(8, np.float32)), f32_up(np.full(8, 0.3, np.float32))
    cand = q[f.astype(bool)][:8]
    n = len(cand)
    print_case("max robot bisection", n)
    rob = ezo.Robot(ctx, desc)
    St = torch.zeros((1, 8, n + 3), dtype=torch.float32, device="cuda")
    St[0, :, :n] = torch.from_numpy(np.ascontiguousarray(cand.T)).cuda()
    ci = torch.arange(n, dtype=torch.int32, device="cuda")[None]
    nc = torch.tensor([n], dtype=torch.int32, device="cuda")
    cs = torch.empty((1, 8, n), dtype=torch.float32, device="cuda")
    ad = torch.empty((1, 8, n), dtype=torch.float32, device="cuda")
    ts = torch.empty((1, n), dtype=torch.float32, device="cuda")
    pc = torch.empty((1, n), dtype=torch.uint8, device="cuda")
    edge = torch.from_numpy(np.stack([v1, v2]).astype(np.float32)[None]).cuda()
    ctx.set_obstacle_boxes(ebox)
    try:
        ezo.project_bisect(ctx, rob, torch.from_numpy(obs_np).cuda(), edge, St, ci, nc, 11, cs, ad, ts, pc)
        torch.cuda.synchronize()
    finally:
        ctx.set_obstacle_boxes(None)
    cs, ad, ts, pc = (x.cpu().numpy() for x in (cs, ad, ts, pc))
    t = np.arange(2049) / 2048.0
    steps, skipped = [], 0
    for j in range(n):
        o = oracle.bisect_arm(orob, ob64, v1, v2, f32_up(cand[j]), 11, env_boxes=eb64)
        assert np.abs(ad[0, :, j] - o["a"]).max() <= 1e-5
        pts = o["c_proj"][None] + t[:, None] * (f32_up(cand[j]) - o["c_proj"])[None]
        *_, fr = oracle.check(orob, ob64, pts, env_boxes=eb64, fragile=True)
        if (fr & 2).any():
            skipped += 1
            continue
        steps.append(bisection_agreement(cs[0, :, j], ts[0, j], pc[0, j], o, f32_up(cand[j]), band=BOX_BAND))
    print(f"max robot bisection: {len(steps)} compared, {skipped} with a fragile midpoint skipped, steps {steps}")
    # every compared candidate's end point lies in the oracle's bracket (checked
    # above); a midpoint inside the band may end the decided steps early
    assert len(steps) >= n // 2 and np.mean(np.array(steps) >= 8) >= 0.5
