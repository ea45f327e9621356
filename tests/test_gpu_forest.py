"""GPU parity on the Forest scene (Sec. VI-A): a point robot on two prismatic
joints among 15 discs.  Checks: flags identical outside +-1e-5 m and signed
distances within 1e-5 m on uniform configurations of the whole domain;
whole inflations of the scene's 4-edge path against the oracle's own runs
(statuses equal on every seed, face and iteration counts on most)."""
import numpy as np
import pytest

import oracle
import workloads
from workloads import draw

from gpu_common import BAND, SD_TOL, f32_up, load, print_case

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


def test_forest_check_parity(ezo, ctx):
    data, desc = load("forest")
    rob = ezo.Robot(ctx, desc)
    q = draw.uniform_q(41, 200_003, data["q_lo"], data["q_hi"])
    print_case("forest check", len(q))
    qt = torch.from_numpy(q).cuda()
    obs = torch.from_numpy(data["obstacles"]).cuda()
    n = len(q)
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    flags2 = torch.empty(n, dtype=torch.uint8, device="cuda")
    msd = torch.empty(n, dtype=torch.float32, device="cuda")
    ezo.check_collisions(ctx, rob, obs, qt, flags)
    ezo.check_collisions(ctx, rob, obs, qt, flags2, msd)
    torch.cuda.synchronize()
    f, sd, *_ = oracle.check(oracle.Robot(desc), f32_up(data["obstacles"]), f32_up(q))
    ok = np.abs(sd) >= BAND
    g, g2, gs = flags.cpu().numpy(), flags2.cpu().numpy(), msd.cpu().numpy()
    print(f"collision fraction {f.mean():.4f}, max |sd err| {np.abs(gs - sd).max():.2e}")
    assert np.array_equal(g[ok], f[ok]) and np.array_equal(g2[ok], f[ok])
    assert np.abs(gs - sd).max() <= SD_TOL
    assert 0.02 < f.mean() < 0.2


def test_forest_path_inflation_against_oracle(ezo, ctx):
    data, desc = load("forest")
    rob = ezo.Robot(ctx, desc)
    orob = oracle.Robot(desc)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    edges = torch.from_numpy(data["edges"]).cuda()
    E = len(data["edges"])
    same_f = same_it = total = 0
    for seed in range(4):
        prm = ezo.make_params(dof=2, seed=seed, **workloads.PARAMS["forest"])
        r = ezo.inflate_edges(ctx, rob, obs, edges, prm)
        torch.cuda.synchronize()
        st, nf = r.status.cpu().numpy(), r.n_faces.cpu().numpy()
        for e in range(E):
            v1, v2 = f32_up(data["edges"][e])
            o = oracle.eizo_arm(orob, f32_up(data["obstacles"]), v1, v2,
                                oracle.make_params(**workloads.PARAMS["forest"], seed=seed, edge_id=e))
            assert st[e] == o["status"] == ezo.CERTIFIED
            F = int(nf[e])
            A = r.A[e, :F].cpu().numpy().astype(np.float64)
            b = r.b[e, :F].cpu().numpy().astype(np.float64)
            for v in (v1, v2):
                assert np.all(A @ v <= b + 1e-5)
            total += 1
            same_it += r.stats[e]["iterations"] == o["stats"]["iterations"]
            if F == len(o["b"]):
                same_f += 1
                assert np.abs(A - o["A"]).max() < 1e-3
    print(f"same iterations {same_it}/{total}, same faces {same_f}/{total}")
    assert same_it >= 0.75 * total and same_f >= 0.75 * total
