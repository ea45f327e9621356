"""Shared helpers of the GPU parity tests (imported by tests/test_gpu_*.py)."""
import numpy as np

import oracle
import workloads

# Flags may differ only where the exact signed distance is inside this band
# (metres); signed distances must agree to the same amount.
BAND = 1e-5
SD_TOL = 1e-5
CENTRE_TOL = 1e-5


def load(name):
    data = workloads.load(name)
    return data, workloads.robot(data)


def f32_up(x):
    """FP32 values as FP64 (what the oracle reads when it mirrors GPU inputs)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# Hit-and-run replayed one step at a time.  A chord end t = (b_f - a_f^T x) /
# (a_f^T u) rounds in FP32 with an absolute error of about 2^-24 (|b_f| +
# sum_j |a_fj x_j|) <= 1e-6 (|x| <= pi sqrt(7), unit rows), which the division
# by the binding row's a_f^T u amplifies.  Steps whose two binding rows both
# have |a_f^T u| >= KAPPA are held to STEP_TOL; the others (a row nearly
# parallel to the direction) to that rounding estimate, STEP_TOL + 1e-6 /
# min |a_f^T u|, and their fraction is reported.
KAPPA = 0.05
STEP_TOL = 1e-5


def sampler_step_replay(ezo, ctx, dof, At, bt, nf, edges, n, n_mix, seed, k, eid, label=""):
    """Runs the GPU sampler with n_mix = 0, 1, ..., n_mix (step s of a walk does
    not depend on the walk's length, so these are the walks' points after
    each step); from the GPU's FP32 point after step s - 1 the oracle takes
    step s of the same walk (same Philox words, FP64), which must land on the
    GPU's point after step s to the bar above.  Step 0 (the start on L) must
    equal the oracle's.  At, bt, nf, edges: the device inputs of the call
    (edge 0 is replayed).  Returns (fraction of ill-conditioned steps, largest
    error of the conditioned ones)."""
    import torch
    F = int(nf[0].item())
    Af = At[0, :F].cpu().numpy().astype(np.float64)
    bf = bt[0, :F].cpu().numpy().astype(np.float64)
    v1, v2 = (x.astype(np.float64) for x in edges[0].cpu().numpy())
    stride = (n + 63) // 64 * 64
    S = torch.empty((1, dof, stride), dtype=torch.float32, device=At.device)
    prev, errs, conds = None, [], []
    for s in range(n_mix + 1):
        ezo.sample_polytopes(ctx, dof, At, bt, nf, edges[:1], n, s, seed=seed, iteration=k, samples=S,
                             edge_id_base=eid)
        torch.cuda.synchronize()
        X = S[0, :, :n].cpu().numpy().T.astype(np.float64)
        assert np.all(X @ Af.T <= bf + 1e-4)             # every point inside P
        if s == 0:
            assert np.abs(X - oracle.hit_and_run(Af, bf, v1, v2, 0, seed, eid, k, n)).max() <= 1e-6
        else:
            Y, den = oracle.hit_and_run_step(Af, bf, prev, seed, eid, k, s)
            errs.append(np.abs(X - Y).max(axis=1))
            conds.append(np.abs(den).min(axis=1))
        prev = X
    if n_mix == 0:
        return 0.0, 0.0
    err, cond = np.concatenate(errs), np.concatenate(conds)
    good = cond >= KAPPA
    frac = float(np.mean(~good))
    emax = float(err[good].max()) if good.any() else 0.0
    print(f"sampler step replay {label}: {err.size} steps, binding |a^T u| < {KAPPA} on {frac:.4f}; max error "
          f"{emax:.2e} (conditioned), {err[~good].max() if (~good).any() else 0.0:.2e} (others)", flush=True)
    assert emax <= STEP_TOL
    assert np.all(err[~good] <= STEP_TOL + 1e-6 / np.maximum(cond[~good], 1e-30))
    assert frac < 0.05
    return frac, emax


def bisection_agreement(c_star_gpu, t_star_gpu, proj_gpu, o, c, band=BAND):
    """Until the first evaluated point whose exact signed distance lies in the
    band, FP32 and FP64 take the same bisection decisions; the bisection is
    meant to converge onto the boundary, so later midpoints often do lie in
    the band.  Both end points then lie inside the oracle's bracket at that
    step, whose length is |c - c_proj| 2^-(s) for a first band midpoint at
    step s.  Returns the number of decided steps."""
    tr = o["sd_trace"]
    if abs(tr[0]) >= band:
        assert bool(proj_gpu) == o["proj_collides"]
    n_b = len(tr) - 1
    first = next((i for i in range(1, n_b + 1) if abs(tr[i]) < band), n_b + 1)
    steps_equal = first - 1                  # decisions 0 .. first-2 are certain
    L = float(np.linalg.norm(c - o["c_proj"]))
    tol = L * 2.0 ** (-steps_equal) + 1e-5 if first <= n_b else 1e-5
    assert np.abs(c_star_gpu - o["c_star"]).max() <= tol
    assert abs(t_star_gpu - o["t_star"]) <= tol
    return steps_equal


def print_case(*parts):
    print("[case]", *parts, flush=True)


def oracle_robot(desc):
    return oracle.Robot(desc)
