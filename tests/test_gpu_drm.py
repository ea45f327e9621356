"""GPU parity of the DRM collision map (appendix, DRM construction) against
the oracle's plain definition: every (voxel, node) bit equal wherever the
oracle's signed distance lies outside +-1e-5 m (the map tests robot spheres
and boxes against voxel spheres: exact distances, no box-box axes), on the whole grid for the 3-DOF arm and on a dense block plus
random voxels for the 7-DOF sphere and box arms; id lists equal the bitset
rows; ragged node counts, padded rows and empty inputs."""
import numpy as np
import pytest

import oracle
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


def unpack(cmap, n):
    """bool [V][n] from the int32 bitset rows."""
    w = cmap.cpu().numpy().view(np.uint32)
    bits = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")
    return bits[:, :n].astype(bool), bits[:, n:]


def check_rows(got, voxels, desc, q, lo, side, dims, band, label):
    hits, sd = oracle.collision_map(oracle.Robot(desc), f32_up(q), f32_up(lo), float(np.float32(side)), dims, voxels)
    ok = np.abs(sd) >= band
    print(f"{label}: {len(voxels)} voxels x {len(q)} nodes, hit fraction {hits.mean():.4f}, "
          f"in band {1 - ok.mean():.2e}")
    assert np.array_equal(got[voxels][ok], hits[ok])
    return hits


def test_map_whole_grid_tiny(ezo, ctx):
    data, desc = load("tiny")
    rob = ezo.Robot(ctx, desc)
    q = draw.uniform_q(31, 301, data["q_lo"], data["q_hi"])            # ragged: 9 full words + 13 bits
    lo, side, dims = np.array([-1.6, -1.6, -0.15], np.float32), 0.1, (32, 32, 3)
    print_case("map tiny", len(q), dims)
    cmap = ezo.collision_map(ctx, rob, torch.from_numpy(q).cuda(), lo, side, dims)
    torch.cuda.synchronize()
    got, pad = unpack(cmap, len(q))
    assert not pad.any()                                             # no bit past the last node
    hits = check_rows(got, np.arange(np.prod(dims)), desc, q, lo, side, dims, BAND, "tiny")
    assert 0.001 < hits.mean() < 0.5


@pytest.mark.parametrize("name,band", [("dof7", BAND), ("boxes", BAND)])
def test_map_block_and_random_voxels(ezo, ctx, name, band):
    data, desc = load(name)
    rob = ezo.Robot(ctx, desc)
    q = draw.uniform_q(32, 2001, data["q_lo"], data["q_hi"])
    lo, side, dims = np.array([-1.3, -1.3, -0.6], np.float32), 0.1, (26, 26, 20)
    print_case("map", name, len(q), dims)
    cmap = ezo.collision_map(ctx, rob, torch.from_numpy(q).cuda(), lo, side, dims)
    torch.cuda.synchronize()
    got, pad = unpack(cmap, len(q))
    assert not pad.any()
    i, j, k = np.meshgrid(np.arange(7, 19), np.arange(7, 19), np.arange(4, 14), indexing="ij")
    block = ((k * dims[1] + j) * dims[0] + i).ravel()
    rnd = np.random.default_rng(6).choice(np.prod(dims), 400, replace=False)
    hits = check_rows(got, np.unique(np.concatenate([block, rnd])), desc, q, lo, side, dims, band, name)
    assert hits.mean() > 0.01


def test_map_lists_padding_and_empty(ezo, ctx):
    data, desc = load("dof7")
    rob = ezo.Robot(ctx, desc)
    q = torch.from_numpy(draw.uniform_q(33, 333, data["q_lo"], data["q_hi"])).cuda()
    lo, side, dims = np.array([-1.0, -1.0, -0.5], np.float32), 0.125, (16, 16, 12)
    V = int(np.prod(dims))
    # a padded row stride gives the same bits
    wide = torch.full((V, 16), -1, dtype=torch.int32, device="cuda")       # stale contents: cleared by the call
    m1 = ezo.collision_map(ctx, rob, q, lo, side, dims)
    m2 = ezo.collision_map(ctx, rob, q, lo, side, dims, out=wide)
    torch.cuda.synchronize()
    assert torch.equal(m2[:, :m1.shape[1]], m1) and not bool(m2[:, m1.shape[1]:].any())
    offsets, ids = ezo.collision_map_lists(ctx, m1, 333)
    torch.cuda.synchronize()
    got, _ = unpack(m1, 333)
    off = offsets.cpu().numpy()
    idn = ids.cpu().numpy()
    assert off[0] == 0 and off[-1] == len(idn) == got.sum()
    for v in np.random.default_rng(7).choice(V, 300, replace=False):
        assert np.array_equal(idn[off[v]:off[v + 1]], np.nonzero(got[v])[0])
    # no nodes: the map is cleared, the lists are empty
    m3 = ezo.collision_map(ctx, rob, q[:0], lo, side, dims, out=wide)
    torch.cuda.synchronize()
    assert not bool(m3.any())
    offsets, ids = ezo.collision_map_lists(ctx, m1[:, :0], 0)
    torch.cuda.synchronize()
    assert len(ids) == 0 and not bool(offsets.any())
