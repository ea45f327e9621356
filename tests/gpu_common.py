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


def sampler_agreement(got, ref, A, b, label=""):
    """Hit-and-run in FP32 and FP64 from the same Philox stream follow the
    same walk until a chord endpoint is decided by a row that is nearly
    parallel to the direction; there the rounding difference is amplified.
    Bar: every sample inside P, >= 95 % of walks within 1e-4, >= 99 % within
    1e-3, median within 1e-5, and the coordinate marginals of the two sample
    sets indistinguishable (two-sample KS, p > 1e-3)."""
    from scipy.stats import ks_2samp
    err = np.abs(got - ref).max(axis=1)
    q = np.quantile(err, [0.5, 0.9, 0.95, 0.99, 1.0])
    print(f"sampler {label} error quantiles 50/90/95/99/100%: " + " ".join(f"{x:.1e}" for x in q), flush=True)
    assert np.all(got @ A.T <= b + 1e-4)
    assert np.mean(err <= 1e-4) >= 0.95
    assert np.mean(err <= 1e-3) >= 0.99
    assert q[0] <= 1e-5
    for j in range(got.shape[1]):
        assert ks_2samp(got[:, j], ref[:, j]).pvalue > 1e-3
    return q


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
