"""GPU checks of the launch-shape autotuner.

A tile kernel's launch shape (configurations per workgroup T, waves W,
obstacle records staged in LDS or not) must never change a result.  Each
shape is forced through the tuning cache and the outputs are compared bit
for bit with those of the size heuristic: collision flags, signed distances,
projection + bisection results, and a whole fused inflation with tuning on
versus off.
"""
import json

import numpy as np
import pytest

from workloads import draw

from gpu_common import load, print_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SHAPES = [(T, W, st) for T in (4, 8, 16, 32) for W in (1, 2, 4, 8) for st in (0, 1)]


@pytest.fixture(scope="module")
def ezo():
    import paper_2504_10783_amd as ezo
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return ezo


@pytest.fixture(scope="module")
def ctx(ezo):
    return ezo.Context(0)


def arch():
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def entry(kernel, desc, n_obs, items, T, W, stage, depth=1):
    return json.dumps({"arch": arch(), "kernel": kernel, "dof": int(desc["dof"]),
                       "spheres": int(len(desc["sphere_r"])), "self_pairs": int(len(desc["self_pairs"])),
                       "obstacles": int(n_obs), "log2_items": int(items).bit_length() - 1,
                       "T": T, "W": W, "stage": stage, "depth": depth, "us": 0.0}, separators=(",", ":"))


def run_check(ezo, ctx, rob, obs, q, sd):
    n = q.shape[0]
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    msd = torch.empty(n, dtype=torch.float32, device="cuda") if sd else None
    mss = torch.empty(n, dtype=torch.float32, device="cuda") if sd else None
    ezo.check_collisions(ctx, rob, obs, q, flags, msd, mss)
    torch.cuda.synchronize()
    return [x for x in (flags, msd, mss) if x is not None]


def test_check_shapes_give_identical_results(ezo, ctx):
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    n = 20_011                                               # ragged tail for every T
    print_case("check shapes", n)
    q = torch.from_numpy(draw.uniform_q(51, n, data["q_lo"], data["q_hi"])).cuda()
    ctx.set_autotune(False)
    try:
        ezo.tune_cache_clear()
        ref_f = run_check(ezo, ctx, rob, obs, q, False)
        ref_s = run_check(ezo, ctx, rob, obs, q, True)
        assert 0.05 < ref_f[0].float().mean().item() < 0.95
        for T, W, st in SHAPES:
            ezo.tune_cache_clear()
            ezo.tune_cache_import(entry("check_flags", desc, len(obs), n, T, W, st) + "\n" +
                                  entry("check_sd", desc, len(obs), n, T, W, 0))
            got_f = run_check(ezo, ctx, rob, obs, q, False)
            got_s = run_check(ezo, ctx, rob, obs, q, True)
            assert torch.equal(got_f[0], ref_f[0]), (T, W, st)
            for a, b in zip(got_s, ref_s):
                assert torch.equal(a, b), (T, W)
    finally:
        ezo.tune_cache_clear()
        ctx.set_autotune(True)


def test_bisect_shapes_give_identical_results(ezo, ctx):
    """Candidates per workgroup, waves, staging and bisection levels per
    round (the same midpoints and decisions in fewer dependent rounds) must
    not change any output."""
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    dof = 7
    obs = torch.from_numpy(data["obstacles"]).cuda()
    pool = torch.from_numpy(draw.uniform_q(52, 8000, data["q_lo"], data["q_hi"])).cuda()
    flags = run_check(ezo, ctx, rob, obs, pool, False)[0]
    cand = pool[flags.bool()][:1500]
    n = cand.shape[0]
    print_case("bisect shapes", n)
    stride = n + 7
    S = torch.zeros((1, dof, stride), dtype=torch.float32, device="cuda")
    S[0, :, :n] = cand.t()
    cap = n + 3
    ci = torch.zeros((1, cap), dtype=torch.int32, device="cuda")
    ci[0, :n] = torch.arange(n, dtype=torch.int32, device="cuda")
    nc = torch.tensor([n], dtype=torch.int32, device="cuda")
    edges = torch.from_numpy(data["edges"][:1]).cuda()

    def run():
        out = (torch.full((1, dof, cap), -7.0, device="cuda"), torch.full((1, dof, cap), -7.0, device="cuda"),
               torch.full((1, cap), -7.0, device="cuda"), torch.full((1, cap), 9, dtype=torch.uint8, device="cuda"))
        ezo.project_bisect(ctx, rob, obs, edges, S, ci, nc, 11, *out)
        torch.cuda.synchronize()
        return out

    ctx.set_autotune(False)
    try:
        ezo.tune_cache_clear()
        ref = run()
        for dp, Ts in ((1, (2, 4, 8, 16, 32)), (2, (1, 2, 4, 8, 16)), (3, (1, 2, 4, 8))):
            for T, W, st in ((T, W, st) for T in Ts for W in (1, 2, 4, 8) for st in (0, 1)):
                ezo.tune_cache_clear()
                ezo.tune_cache_import(entry("bisect", desc, len(obs), cap, T, W, st, dp))
                got = run()
                for a, b in zip(got, ref):
                    assert torch.equal(a, b), (T, W, st, dp)
    finally:
        ezo.tune_cache_clear()
        ctx.set_autotune(True)


@pytest.mark.parametrize("name,n_mix", [("tiny", 30), ("dof7", 60)])
def test_sampler_lane_counts_give_identical_samples(ezo, ctx, name, n_mix):
    """Lanes per walk split the rows; the chord ends are exact min/max."""
    import oracle
    data, desc = load(name)
    dof = int(desc["dof"])
    A, b = oracle.Robot(desc).box()
    rng = np.random.default_rng(4)
    extra = rng.normal(size=(20, dof))                     # 20 more faces, all outside the edge
    v = data["edges"][0].astype(np.float64)
    bx = np.max(extra @ v.T, axis=1) + rng.uniform(0.05, 0.5, size=20)
    A = np.vstack([A, extra]).astype(np.float32)
    b = np.concatenate([b, bx]).astype(np.float32)
    F, cap = len(b), len(b) + 5
    At = torch.zeros((1, cap, dof), dtype=torch.float32, device="cuda")
    bt = torch.zeros((1, cap), dtype=torch.float32, device="cuda")
    At[0, :F] = torch.from_numpy(A).cuda()
    bt[0, :F] = torch.from_numpy(b).cuda()
    nf = torch.tensor([F], dtype=torch.int32, device="cuda")
    edges = torch.from_numpy(data["edges"][:1]).cuda()
    n = 3001
    print_case("sampler lanes", name, n)
    out = {}
    ctx.set_autotune(False)
    try:
        for L in (1, 2, 4, 8, 16):
            ezo.tune_cache_clear()
            ezo.tune_cache_import(json.dumps({"arch": arch(), "kernel": "sample", "dof": dof, "spheres": 0,
                                              "self_pairs": 0, "obstacles": 0,
                                              "log2_items": n.bit_length() - 1, "T": L, "W": 4, "stage": 0,
                                              "us": 0.0}, separators=(",", ":")))
            S = torch.full((1, dof, n + 3), -9.0, dtype=torch.float32, device="cuda")
            ezo.sample_polytopes(ctx, dof, At, bt, nf, edges, n, n_mix, seed=11, iteration=2, samples=S)
            torch.cuda.synchronize()
            out[L] = S
        for L in (1, 2, 4, 16):
            assert torch.equal(out[L], out[8]), L
        x = out[8][0, :, :n].cpu().numpy().T.astype(np.float64)
        assert np.all(x @ A.T.astype(np.float64) <= b + 1e-4)
    finally:
        ezo.tune_cache_clear()
        ctx.set_autotune(True)


def test_raw_check_tuning_fills_cache(ezo, ctx):
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    n = 1 << 16
    q = torch.from_numpy(draw.uniform_q(53, n, data["q_lo"], data["q_hi"])).cuda()
    ctx.set_autotune(False)
    ezo.tune_cache_clear()
    ref = run_check(ezo, ctx, rob, obs, q, False) + run_check(ezo, ctx, rob, obs, q, True)
    ctx.set_autotune(True)
    got = run_check(ezo, ctx, rob, obs, q, False) + run_check(ezo, ctx, rob, obs, q, True)
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    ents = ezo.tune_cache_entries()
    print("tuned:", ents)
    kinds = {(e["kernel"], e["log2_items"], e["obstacles"]) for e in ents}
    assert ("check_flags", 16, len(obs)) in kinds and ("check_sd", 16, len(obs)) in kinds
    for e in ents:
        assert e["us"] > 0 and e["arch"] == arch()


@pytest.mark.parametrize("name,max_iters", [("dof7", 50), ("batched", 3)])
def test_autotuned_inflation_equals_heuristic(ezo, ctx, name, max_iters):
    import workloads
    data, desc = load(name)
    rob = ezo.Robot(ctx, desc)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"]).cuda()
    p = dict(workloads.PARAMS[name], max_iters=max_iters)
    print_case("autotuned inflation", name, edges.shape[0])
    ctx.set_autotune(False)
    ezo.tune_cache_clear()
    r0 = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=5, **p))
    torch.cuda.synchronize()
    ctx.set_autotune(True)
    r1 = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=5, **p))
    torch.cuda.synchronize()
    assert torch.equal(r0.status, r1.status) and torch.equal(r0.n_faces, r1.n_faces)
    for e, F in enumerate(r0.n_faces.tolist()):           # rows past n_faces are not written
        assert torch.equal(r0.A[e, :F], r1.A[e, :F]) and torch.equal(r0.b[e, :F], r1.b[e, :F])
    assert r0.stats == r1.stats
    kinds = {e["kernel"] for e in ezo.tune_cache_entries() if e["obstacles"] == len(obs)}
    assert {"check_flags", "bisect"} <= kinds
    st = r1.status.cpu().numpy()
    assert np.all(st == ezo.CERTIFIED) or max_iters < 50


def test_sample_count_tuning(ezo, ctx):
    """n_p = 0: the first call times whole inflations with each candidate
    N_p and caches one ("samples" entry: the largest within 5 % of the
    fastest, a timing-dependent pick); the timed inflations drew from their
    own Philox key (seed ^ 0x9E3779B97F4A7C15, recorded in the entry), never
    from the call's, so the pick cannot favour a run whose own draws ended it
    early (Alg. 1 Output: the delta bound holds for the returned sets); the
    call's result equals an explicit call with that N_p on the call's seed bit
    for bit; a second call reuses the entry; with tuning off and no entry
    N_p = 10000."""
    import workloads
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"]).cuda()
    p = dict(workloads.PARAMS["dof7"], n_p=0)
    print_case("sample-count tuning")
    ezo.tune_cache_clear()
    ctx.set_autotune(True)
    try:
        r = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=6, **p))
        torch.cuda.synchronize()
        ent = [e for e in ezo.tune_cache_entries() if e["kernel"] == "samples"]
        print("samples entries", ent)
        assert len(ent) == 1 and ent[0]["T"] in (1000, 2000, 5000, 10000) and ent[0]["log2_items"] == 0
        assert ent[0]["tune_seed"] == 6 ^ 0x9E3779B97F4A7C15 and ent[0]["tune_seed"] != 6
        chosen = ent[0]["T"]
        assert int(r.status[0].item()) == ezo.CERTIFIED
        ref = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=6, **dict(p, n_p=chosen)))
        again = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=6, **p))
        torch.cuda.synchronize()
        F = int(r.n_faces[0].item())
        for x in (ref, again):
            assert torch.equal(x.status, r.status) and torch.equal(x.n_faces, r.n_faces)
            assert torch.equal(x.A[0, :F], r.A[0, :F]) and torch.equal(x.b[0, :F], r.b[0, :F])
        assert len([e for e in ezo.tune_cache_entries() if e["kernel"] == "samples"]) == 1
        # tuning off, no entry: the default count
        ezo.tune_cache_clear()
        ctx.set_autotune(False)
        d = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=6, **p))
        dref = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=6, **dict(p, n_p=10000)))
        torch.cuda.synchronize()
        assert torch.equal(d.n_faces, dref.n_faces) and torch.equal(d.status, dref.status)
        assert not [e for e in ezo.tune_cache_entries() if e["kernel"] == "samples"]
    finally:
        ctx.set_autotune(True)
