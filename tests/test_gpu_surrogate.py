"""GPU checks of the learned self-collision screen.

* forward pass and loss gradient of the library's own BF16-MFMA kernels vs
  the FP64 oracle evaluated on the same BF16-rounded weights and the same
  inputs (BF16 activations bound the agreement to a few 1e-3 relative);
* training on exact-checker labels lowers the loss, and the calibrated
  margin keeps the miss rate on held-out data near the target;
* screened inflation never screens the unadaptive test's samples or the
  fail-fast projections (it screens the other samples and the bisection
  midpoints), gives the same polytope as the exact method when the margin
  screens nothing, and keeps every invariant when it does; the planes of a
  screened run are placed at points that truly collide;
* what a trained screen gains: the same certified inflation with fewer
  exact pair tests per checked configuration (times printed).
"""
import time

import numpy as np
import pytest

import oracle
import workloads
from workloads import draw

from gpu_common import f32_up, load, print_case

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


def bf16_round(x):
    """Round FP32 values to BF16 (nearest even) and back, in FP64."""
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def oracle_view(params, D, H):
    """GPU parameters as the oracle sees them: W2, W3 rounded to BF16 (the
    MFMA layers' operands), everything else FP32."""
    p = np.asarray(params, np.float64).copy()
    o2 = H * D + H
    o3 = o2 + H * H + H
    p[o2:o2 + H * H] = bf16_round(params[o2:o2 + H * H])
    p[o3:o3 + H * H] = bf16_round(params[o3:o3 + H * H])
    return p


def self_labels(ezo, ctx, rob, q):
    n = q.shape[0]
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    msd = torch.empty(n, dtype=torch.float32, device="cuda")
    mss = torch.empty(n, dtype=torch.float32, device="cuda")
    ezo.check_collisions(ctx, rob, torch.zeros((0, 4), dtype=torch.float32, device="cuda"), q, flags, msd, mss)
    return mss


def test_forward_and_gradient_match_oracle(ezo, ctx):
    data, desc = load("dof7")
    D, H, n = 7, 256, 256
    print_case("mlp grad parity", n)
    s = ezo.Surrogate(ctx, D, H, seed=3)
    q = torch.from_numpy(draw.uniform_q(31, n, data["q_lo"], data["q_hi"])).cuda()
    rob = ezo.Robot(ctx, desc)
    t = self_labels(ezo, ctx, rob, q)
    tp = ezo.make_train_params()
    loss, g = s.loss_grad(q, t, tp)
    params = s.get_params()
    pv = oracle_view(params, D, H)
    x = f32_up(q.cpu().numpy()) / np.pi
    x = f32_up(x)                                   # the GPU multiplies by 1/pi in FP32
    lo, go = oracle.mlp_loss_grad(D, H, pv, x, f32_up(t.cpu().numpy()))
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    print(f"loss gpu {loss:.6f} oracle {lo:.6f}; grad rel err {rel:.3e}")
    assert abs(loss - lo) <= 2e-2 * abs(lo)
    assert rel <= 2e-2
    pred = torch.empty(n, dtype=torch.float32, device="cuda")
    s.predict(q, pred)
    torch.cuda.synchronize()
    yo = oracle.mlp_forward(D, H, pv, x)
    err = np.abs(pred.cpu().numpy() - yo).max()
    print(f"forward max abs err {err:.3e} (|y| max {np.abs(yo).max():.3f})")
    assert err <= 2e-2 * max(1.0, np.abs(yo).max())


def test_set_get_params_roundtrip(ezo, ctx):
    s = ezo.Surrogate(ctx, 7, 64, seed=1)
    p = np.random.default_rng(0).normal(size=s.n_params).astype(np.float32)
    s.set_params(p)
    assert np.array_equal(s.get_params(), p)


def test_training_lowers_loss_and_calibration_controls_misses(ezo, ctx):
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    n_train, n_cal, n_test = 200_704, 32_768, 32_768
    print_case("mlp training", n_train)
    q = torch.from_numpy(draw.uniform_q(41, n_train + n_cal + n_test, data["q_lo"], data["q_hi"])).cuda()
    t = self_labels(ezo, ctx, rob, q)
    qa, ta = q[:n_train], t[:n_train]
    qc, tc = q[n_train:n_train + n_cal], t[n_train:n_train + n_cal]
    qt, tt = q[n_train + n_cal:], t[n_train + n_cal:]
    s = ezo.Surrogate(ctx, 7, 256, seed=7)
    tp = ezo.make_train_params(epochs=3, batch=4096, lr=1e-3, seed=1)
    l0, _ = s.loss_grad(qt[:4096], tt[:4096], tp)
    losses = s.train(qa, ta, tp)
    l1, _ = s.loss_grad(qt[:4096], tt[:4096], tp)
    print(f"held-out loss {l0:.5f} -> {l1:.5f}; epoch losses {losses}")
    assert l1 < 0.5 * l0
    m = s.calibrate(qc, tc, 0.01)
    miss, frac = s.miss_rate(qt, tt)
    n_col = int((tt < 0).sum().item())
    print(f"margin {m:.4f}; held-out miss rate {miss:.4f} over {n_col} colliding; screened fraction {frac:.3f}")
    assert np.isfinite(m)
    assert miss <= 0.01 + 4 * np.sqrt(0.01 / max(n_col, 1)) + 2.0 / max(n_col, 1)
    assert frac > 0.05           # the screen clears a useful share of configurations


def test_screened_inflation_safety(ezo, ctx):
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    s = ezo.Surrogate(ctx, 7, 256, seed=9)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"]).cuda()
    p = dict(workloads.PARAMS["dof7"])
    base = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=3, **p))
    torch.cuda.synchronize()
    # margin +inf: the screen runs but clears nothing -> identical result
    s.set_margin(float("inf"))
    r0 = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=3, surrogate=s, **p))
    torch.cuda.synchronize()
    F = int(base.n_faces[0].item())
    assert int(r0.n_faces[0].item()) == F and int(r0.status[0].item()) == int(base.status[0].item())
    assert torch.equal(r0.A[0, :F], base.A[0, :F]) and torch.equal(r0.b[0, :F], base.b[0, :F])
    assert r0.stats[0]["screened_checks"] == 0
    # margin -inf: every optimizer sample's and every bisection midpoint's
    # self pairs are skipped; test samples and projections never
    s.set_margin(float("-inf"))
    r1 = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=3, surrogate=s, **p))
    torch.cuda.synchronize()
    st = r1.stats[0]
    M_total = sum(ezo.test_constants(p["eps"], p["delta"], p["tau"], k)[0] for k in range(1, st["iterations"] + 1))
    n_b = p["n_b"]
    bis = st["exact_checks"] - st["samples"]                  # (1 + N_b) per candidate
    print("screened stats", st, "test samples", M_total)
    assert bis % (1 + n_b) == 0
    assert st["screened_checks"] == (st["samples"] - M_total) + bis // (1 + n_b) * n_b
    # scope: the samples only, then the midpoints only
    s.set_scope(samples=True, midpoints=False)
    r2 = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=3, surrogate=s, **p))
    torch.cuda.synchronize()
    st2 = r2.stats[0]
    M2 = sum(ezo.test_constants(p["eps"], p["delta"], p["tau"], k)[0] for k in range(1, st2["iterations"] + 1))
    assert st2["screened_checks"] == st2["samples"] - M2
    s.set_scope(samples=False, midpoints=True)
    r3 = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=7, seed=3, surrogate=s, **p))
    torch.cuda.synchronize()
    st3 = r3.stats[0]
    assert st3["screened_checks"] == (st3["exact_checks"] - st3["samples"]) // (1 + n_b) * n_b
    s.set_scope()
    assert int(r1.status[0].item()) in (ezo.CERTIFIED, ezo.MAX_ITERS)
    F1 = int(r1.n_faces[0].item())
    A1 = r1.A[0, :F1].cpu().numpy().astype(np.float64)
    b1 = r1.b[0, :F1].cpu().numpy().astype(np.float64)
    for v in data["edges"][0].astype(np.float64):
        assert np.all(A1 @ v <= b1 + 1e-5)


def test_screened_inflation_in_fresh_context(ezo):
    """The first call on a new context is a screened 96-edge inflation: every
    workspace buffer (the screen's included) must exist before the iteration
    is captured into a graph."""
    c2 = ezo.Context(0)
    data, desc = load("batched")
    rob = ezo.Robot(c2, desc)
    s = ezo.Surrogate(c2, 7, 256, seed=2)
    s.set_margin(0.0)
    p = dict(workloads.PARAMS["batched"], max_iters=2)
    r = ezo.inflate_edges(c2, rob, torch.from_numpy(data["obstacles"]).cuda(),
                          torch.from_numpy(data["edges"]).cuda(), ezo.make_params(dof=7, seed=1, surrogate=s, **p))
    torch.cuda.synchronize()
    st = r.status.cpu().numpy()
    assert np.all((st == ezo.CERTIFIED) | (st == ezo.MAX_ITERS))
    assert sum(x["screened_checks"] for x in r.stats) > 0


def test_trained_screen_gain(ezo, ctx):
    """What the trained network gains over the method without it, on the
    dof7 edge at identical eps / delta / tau / seed: both runs certify; the
    screened run skips the exact self pairs of the optimizer samples the
    network clears, so its check phase performs fewer exact pair tests per
    checked configuration.  Both wall times are printed (the exact self pairs
    cost ~100 pair tests per configuration after the broad phase, fewer flops
    than the network, so the time gain can be negative)."""
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    n_train, n_cal = 200_704, 32_768
    print_case("screen gain", n_train)
    q = torch.from_numpy(draw.uniform_q(43, n_train + n_cal, data["q_lo"], data["q_hi"])).cuda()
    t = self_labels(ezo, ctx, rob, q)
    s = ezo.Surrogate(ctx, 7, 256, seed=11)
    s.train(q[:n_train], t[:n_train], ezo.make_train_params(epochs=3, batch=4096, lr=1e-3, seed=2))
    margin = s.calibrate(q[n_train:], t[n_train:], 1e-3)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"]).cuda()
    p = dict(workloads.PARAMS["dof7"])
    res = {}
    cap = ezo.make_params(dof=7, seed=5, **p).face_capacity
    pts = torch.full((1, cap, 7), float("nan"), dtype=torch.float32, device="cuda")
    for mode in ("exact", "screened"):
        prm = ezo.make_params(dof=7, seed=5, surrogate=s if mode == "screened" else None, **p)
        r = ezo.inflate_edges(ctx, rob, obs, edges, prm, row_points=pts if mode == "screened" else None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            r = ezo.inflate_edges(ctx, rob, obs, edges, prm)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / 3 * 1e3
        ctx.set_phase_timing(True)
        rt = ezo.inflate_edges(ctx, rob, obs, edges, prm)
        _, _, tests = ctx.phase_timing(with_tests=True)
        ctx.set_phase_timing(False)
        st = rt.stats[0]
        assert torch.equal(rt.n_faces, r.n_faces) and torch.equal(rt.status, r.status)
        res[mode] = {"ms": ms, "status": int(r.status[0].item()), "samples": st["samples"],
                     "screened": st["screened_checks"], "tests_per_sample": tests["check"] / st["samples"]}
    print(f"margin {margin:.4f}; exact {res['exact']}; screened {res['screened']}; "
          f"time ratio exact/screened {res['exact']['ms'] / res['screened']['ms']:.3f}")
    assert res["exact"]["status"] == ezo.CERTIFIED and res["screened"]["status"] == ezo.CERTIFIED
    assert res["exact"]["screened"] == 0 and res["screened"]["screened"] > 0
    assert res["screened"]["tests_per_sample"] < res["exact"]["tests_per_sample"]
    # the screened bisection (midpoints screened one-sidedly) still places
    # every plane at a point that truly collides (oracle, outside the band)
    F = int(r.n_faces[0].item())
    c = pts[0, 14:F].cpu().numpy().astype(np.float64)
    assert F > 14 and np.all(np.isfinite(c))
    f, sd, *_ = oracle.check(oracle.Robot(desc), f32_up(data["obstacles"]), c)
    out = np.abs(sd) >= 1e-5
    print(f"screened run: {F - 14} planes, every c* colliding: {bool(np.all(f[out] == 1))}")
    assert np.all(f[out] == 1)
