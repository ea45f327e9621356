"""GPU parity of forward kinematics and the collision checker against the
FP64 oracle (plain definition of Sec. IV-D: all pairs, minimum signed
distance, flag = minimum < 0).

Bar: sphere centres within 1e-5 m; flags identical wherever the oracle's
signed distance is outside +-1e-5 m; signed distances within 1e-5 m."""
import numpy as np
import pytest

import oracle
from workloads import draw

from gpu_common import BAND, CENTRE_TOL, SD_TOL, f32_up, load, print_case

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


def gpu_check(ezo, ctx, rob, obs, q, sd=True):
    qt = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
    ot = torch.from_numpy(np.ascontiguousarray(obs, np.float32).reshape(-1, 4)).cuda()
    n = len(q)
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    msd = torch.empty(n, dtype=torch.float32, device="cuda") if sd else None
    mss = torch.empty(n, dtype=torch.float32, device="cuda") if sd else None
    ezo.check_collisions(ctx, rob, ot, qt, flags, msd, mss)
    torch.cuda.synchronize()
    return (flags.cpu().numpy(), msd.cpu().numpy() if sd else None, mss.cpu().numpy() if sd else None)


@pytest.mark.parametrize("name", ["tiny", "dof7"])
def test_fk_sphere_centres(ezo, ctx, name):
    data, desc = load(name)
    print_case("fk", name)
    rob = ezo.Robot(ctx, desc)
    orob = oracle.Robot(desc)
    q = draw.uniform_q(21, 4099, data["q_lo"], data["q_hi"])
    q[0] = 0.0
    q[1] = data["q_lo"]
    q[2] = data["q_hi"]
    out = torch.empty((len(q), rob.n_spheres, 3), dtype=torch.float32, device="cuda")
    ezo.sphere_centres(ctx, rob, torch.from_numpy(q).cuda(), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = np.stack([oracle.sphere_centres(orob, f32_up(x)) for x in q])
    err = np.abs(got - ref).max()
    print(f"max centre error {err:.3e} m")
    assert err <= CENTRE_TOL


CASES = [("tiny", "obstacles", 4099), ("dof7", "obstacles", 8191), ("sweep", "obstacles_256", 4099),
         ("sweep", "obstacles_1024", 4099), ("sweep", "obstacles_4096", 2053)]


@pytest.mark.parametrize("name,key,n", CASES)
def test_checker_parity(ezo, ctx, name, key, n):
    data, desc = load(name)
    obs = data[key]
    print_case("checker", name, key, n)
    rob = ezo.Robot(ctx, desc)
    orob = oracle.Robot(desc)
    q = draw.uniform_q(100 + n, n, data["q_lo"], data["q_hi"])
    f_sd, msd, mss = gpu_check(ezo, ctx, rob, obs, q, sd=True)
    f_fl, _, _ = gpu_check(ezo, ctx, rob, obs, q, sd=False)
    fo, sdo, seo, sso = oracle.check(orob, f32_up(obs), f32_up(q))
    out = np.abs(sdo) >= BAND
    print(f"band cases {np.sum(~out)} of {n}; collision fraction {fo.mean():.3f}")
    assert 0.02 < fo.mean() < 0.98
    assert np.array_equal(f_sd[out], fo[out])
    assert np.array_equal(f_fl[out], fo[out])
    assert np.abs(msd - sdo).max() <= SD_TOL
    finite = np.isfinite(sso)
    assert np.array_equal(np.isfinite(mss), finite)
    if finite.any():
        assert np.abs(mss[finite] - sso[finite]).max() <= SD_TOL


def test_checker_strided_layout_matches(ezo, ctx):
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    q = draw.uniform_q(5, 3001, data["q_lo"], data["q_hi"])
    obs = torch.from_numpy(data["obstacles"]).cuda()
    a = gpu_check(ezo, ctx, rob, data["obstacles"], q)
    qs = torch.from_numpy(np.ascontiguousarray(q.T)).cuda()      # [dof][n]
    flags = torch.empty(len(q), dtype=torch.uint8, device="cuda")
    msd = torch.empty(len(q), dtype=torch.float32, device="cuda")
    ezo.check_collisions(ctx, rob, obs, qs, flags, msd, None, stride_n=1, stride_d=len(q))
    torch.cuda.synchronize()
    assert np.array_equal(flags.cpu().numpy(), a[0])
    assert np.array_equal(msd.cpu().numpy(), a[1])


def test_checker_edge_cases(ezo, ctx):
    data, desc = load("tiny")
    rob = ezo.Robot(ctx, desc)
    orob = oracle.Robot(desc)
    # n = 0 is a no-op
    flags = torch.zeros(1, dtype=torch.uint8, device="cuda")
    ezo.check_collisions(ctx, rob, torch.from_numpy(data["obstacles"]).cuda(),
                         torch.zeros((0, 3), dtype=torch.float32, device="cuda"), flags)
    torch.cuda.synchronize()
    # n = 1, and no obstacles: the overall minimum is the self minimum
    q = draw.uniform_q(9, 257, data["q_lo"], data["q_hi"])
    f, msd, mss = gpu_check(ezo, ctx, rob, np.zeros((0, 4), np.float32), q)
    fo, sdo, seo, sso = oracle.check(orob, np.zeros((0, 4)), f32_up(q))
    assert np.isinf(seo).all()
    assert np.abs(msd - sso).max() <= SD_TOL
    out = np.abs(sdo) >= BAND
    assert np.array_equal(f[out], fo[out])
    f1, m1, _ = gpu_check(ezo, ctx, rob, data["obstacles"], q[:1])
    fo1, so1, *_ = oracle.check(orob, f32_up(data["obstacles"]), f32_up(q[:1]))
    assert abs(m1[0] - so1[0]) <= SD_TOL
    # robot without self pairs: the self minimum is +inf
    desc2 = dict(desc, self_pairs=np.zeros((0, 2), np.int32))
    rob2 = ezo.Robot(ctx, desc2)
    f2, m2, s2 = gpu_check(ezo, ctx, rob2, data["obstacles"], q)
    assert np.isinf(s2).all()
    fo2, so2, *_ = oracle.check(oracle.Robot(desc2), f32_up(data["obstacles"]), f32_up(q))
    assert np.abs(m2 - so2).max() <= SD_TOL


def test_checker_full_size_sweep_sampled(ezo, ctx):
    """Largest raw-sweep point, 16M configurations x 4096 obstacles, in the
    launch configuration used for throughput runs; 1024 sampled outputs are
    recomputed by the oracle one by one."""
    data, desc = load("sweep")
    obs = data["obstacles_4096"]
    n = 16 * 1024 * 1024
    print_case("checker full size", n, "x 4096")
    rob = ezo.Robot(ctx, desc)
    q = draw.uniform_q_fast(303, n, data["q_lo"], data["q_hi"])
    f, msd, _ = gpu_check(ezo, ctx, rob, obs, q)
    idx = np.random.default_rng(0).choice(n, 1024, replace=False)
    fo, sdo, *_ = oracle.check(oracle.Robot(desc), f32_up(obs), f32_up(q[idx]))
    out = np.abs(sdo) >= BAND
    assert np.array_equal(f[idx][out], fo[out])
    assert np.abs(msd[idx] - sdo).max() <= SD_TOL
    ff, _, _ = gpu_check(ezo, ctx, rob, obs, q, sd=False)
    assert np.array_equal(ff[idx][out], fo[out])


def broad_phase_scenes():
    rng = np.random.default_rng(77)
    def cloud(n, lo, hi, rlo, rhi):
        c = rng.uniform(lo, hi, size=(n, 3))
        return np.concatenate([c, rng.uniform(rlo, rhi, size=(n, 1))], 1).astype(np.float32)
    return {
        # 4096 obstacles packed in a 0.25 m cube: most grid cells overflow their lists
        "overflow": cloud(4096, [0.4, -0.1, 0.3], [0.65, 0.15, 0.55], 0.01, 0.03),
        # a cloud far from the arm: every sphere falls outside the grid
        "far": cloud(1000, [20.0, 20.0, 20.0], [21.0, 21.0, 21.0], 0.02, 0.08),
        # grid-size thresholds and large obstacles
        "n31": cloud(31, [-1.0, -1.0, -0.5], [1.0, 1.0, 1.0], 0.05, 0.5),
        "n32": cloud(32, [-1.0, -1.0, -0.5], [1.0, 1.0, 1.0], 0.05, 0.5),
        "n255": cloud(255, [-1.0, -1.0, -0.5], [1.0, 1.0, 1.0], 0.02, 0.2),
        "n256": cloud(256, [-1.0, -1.0, -0.5], [1.0, 1.0, 1.0], 0.02, 0.2),
        "single": cloud(1, [0.5, 0.0, 0.5], [0.5, 0.0, 0.5], 0.3, 0.3),
    }


@pytest.mark.parametrize("scene", ["overflow", "far", "n31", "n32", "n255", "n256", "single"])
def test_broad_phase_flags_equal_all_pairs(ezo, ctx, scene):
    """Flags-only checks use the grid broad phase and link-bound culling of
    self pairs; flags must equal the plain definition's (oracle) outside the
    band, and the signed-distance mode's flags (all pairs) everywhere the two
    modes' own arithmetic agrees."""
    data, desc = load("dof7")
    obs = broad_phase_scenes()[scene]
    print_case("broad phase", scene, len(obs))
    rob = ezo.Robot(ctx, desc)
    q = draw.uniform_q(500, 3001, data["q_lo"], data["q_hi"])
    f_fl, _, _ = gpu_check(ezo, ctx, rob, obs, q, sd=False)
    f_sd, msd, _ = gpu_check(ezo, ctx, rob, obs, q, sd=True)
    fo, sdo, seo, sso = oracle.check(oracle.Robot(desc), f32_up(obs), f32_up(q))
    out = np.abs(sdo) >= BAND
    print(f"collision fraction {fo.mean():.3f} (env {np.mean(seo < 0):.3f}), band {np.sum(~out)}")
    assert np.array_equal(f_fl[out], fo[out])
    assert np.array_equal(f_sd[out], fo[out])
    if scene == "far":
        assert np.all(seo > 10.0)
    if scene == "overflow":
        assert np.mean(seo < 0) > 0.05
