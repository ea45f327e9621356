"""ezo_check_collisions_noalloc (the checker for callers that cannot
allocate device memory) against ezo_check_collisions on the same inputs:
flags and signed distances bit for bit, on two calls in a row, the second
with fewer configurations and fewer obstacles (a smaller broad-phase grid),
so that what the first call left in the shared fixed scratch must not leak
into the second; the obstacle limit; no device allocation by the call."""
import numpy as np
import pytest

import workloads
from workloads import draw

from gpu_common import load, print_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ezo():
    import paper_2504_10783_amd as ezo
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return ezo


def run(ezo, ctx, rob, obs, q, noalloc, sd):
    n = q.shape[0]
    flags = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    msd = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda") if sd else None
    mss = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda") if sd else None
    ezo.check_collisions(ctx, rob, obs, q, flags, msd, mss, noalloc=noalloc)
    torch.cuda.synchronize()
    return flags.cpu().numpy(), (msd.cpu().numpy() if sd else None), (mss.cpu().numpy() if sd else None)


@pytest.mark.parametrize("sd", [False, True])
def test_noalloc_equals_check_collisions_on_two_calls(ezo, sd):
    ctx = ezo.Context(0)
    data = workloads.load("sweep")
    desc = workloads.robot(data)
    rob = ezo.Robot(ctx, desc)
    calls = [(4096, 30011, 41), (300, 1001, 42)]            # second call: smaller input, smaller grid
    for n_obs, n, seed in calls:
        print_case("noalloc", "sd" if sd else "flags", n_obs, n)
        obs = torch.from_numpy(np.ascontiguousarray(data["obstacles_4096"][:n_obs])).cuda()
        q = torch.from_numpy(draw.uniform_q(seed, n, data["q_lo"], data["q_hi"])).cuda()
        f0, s0, e0 = run(ezo, ctx, rob, obs, q, False, sd)
        f1, s1, e1 = run(ezo, ctx, rob, obs, q, True, sd)
        assert np.array_equal(f0, f1)
        assert set(np.unique(f1)) <= {0, 1}
        if sd:
            assert np.array_equal(s0, s1) and np.array_equal(e0, e1)
        print(f"  collision fraction {f1.mean():.3f}")


def test_noalloc_limit_and_no_allocation(ezo):
    ctx = ezo.Context(0)
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    q = torch.from_numpy(draw.uniform_q(5, 777, data["q_lo"], data["q_hi"])).cuda()
    flags = torch.empty(777, dtype=torch.uint8, device="cuda")
    big = torch.zeros((ezo.NOALLOC_MAX_OBSTACLES + 1, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(ezo.EzoError) as ei:
        ezo.check_collisions(ctx, rob, big, q, flags, noalloc=True)
    assert ei.value.code == ezo.EZO_E_CAPACITY
    # after a first call (which has the code object, and with it the fixed
    # scratch, loaded), further calls must leave the device's free memory
    # unchanged (torch's allocator is not involved: the driver's figure is
    # compared)
    obs = torch.from_numpy(data["obstacles"]).cuda()
    ezo.check_collisions(ctx, rob, obs, q, flags, noalloc=True)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        ezo.check_collisions(ctx, rob, obs, q, flags, noalloc=True)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print_case("noalloc free memory before / after", free0, free1)
    assert free1 == free0
    f_ref = torch.empty_like(flags)
    ezo.check_collisions(ctx, rob, obs, q, f_ref)
    torch.cuda.synchronize()
    assert torch.equal(f_ref, flags)
