"""Pins of the oracle's DRM collision map (appendix, DRM construction):
voxel sets of a single robot sphere and an axis-aligned robot box in closed
form, and a whole-voxel shift of the arm's base shifting the map."""
import numpy as np

import oracle


def point_arm(r_sphere, box_half=None):
    """1-DOF arm, a = 0, d = 0: its one sphere (or box) sits at the base
    origin whatever q is."""
    desc = dict(dof=1, a=np.zeros(1), alpha=np.zeros(1), d=np.zeros(1), q_lo=np.array([-np.pi]),
                q_hi=np.array([np.pi]), sphere_link=np.zeros(1, np.int32), sphere_xyz=np.zeros((1, 3)),
                sphere_r=np.array([r_sphere]))
    if box_half is not None:
        desc.update(sphere_link=np.zeros(0, np.int32), sphere_xyz=np.zeros((0, 3)), sphere_r=np.zeros(0),
                    box_link=np.zeros(1, np.int32), box_pose=np.concatenate([np.zeros(3), np.eye(3).ravel()])[None],
                    box_half=np.asarray(box_half, float)[None])
    return oracle.Robot(desc)


def ijk(v, dims):
    return v % dims[0], (v // dims[0]) % dims[1], v // (dims[0] * dims[1])


def test_single_sphere_voxel_sets():
    s, dims = 0.1, (9, 9, 9)
    lo = -4.5 * s * np.ones(3)             # the origin is the centre of voxel (4, 4, 4)
    for r_s, expect in ((0.01, 1), (0.2 * s, 7), (0.6 * s, 19), (0.9 * s, 27)):
        # distance to a face / edge / corner neighbour's centre: s, sqrt2 s, sqrt3 s;
        # they touch iff that distance < r_s + sqrt(3)/2 s
        hits, sd = oracle.collision_map(point_arm(r_s), [[0.3]], lo, s, dims)
        got = np.nonzero(hits[:, 0])[0]
        assert len(got) == expect, (r_s, len(got))
        for v in got:
            d = np.abs(np.array(ijk(v, dims)) - 4)
            assert d.max() <= 1
        assert np.isclose(sd[4 + 9 * 4 + 81 * 4, 0], -r_s - np.sqrt(3) / 2 * s)


def test_axis_aligned_box_voxel_set():
    s, dims = 0.1, (12, 12, 12)
    lo = -6 * s * np.ones(3)               # voxel boundaries at multiples of s
    half = np.array([0.25, 0.05, 0.05])    # box [-0.25, 0.25] x [-0.05, 0.05]^2
    hits, sd = oracle.collision_map(point_arm(0.0, half), [[0.0]], lo, s, dims)   # q = 0: link frame = world
    rv = np.sqrt(3) / 2 * s
    ref = []
    for v in range(int(np.prod(dims))):
        i, j, k = ijk(v, dims)
        x = lo + s * (np.array([i, j, k]) + 0.5)
        out = np.maximum(np.abs(x) - half, 0.0)            # the box is axis-aligned: closed form
        inside = np.all(np.abs(x) <= half)
        d = (np.max(np.abs(x) - half) if inside else np.linalg.norm(out)) - rv
        ref.append(d)
    ref = np.array(ref)
    assert np.array_equal(hits[:, 0], ref < 0) and np.allclose(sd[:, 0], ref)
    # voxel centres sit at +-0.05, +-0.15, +-0.25, +-0.35 ...: six of them
    # within the box's x extent, two within its y and z extents; one more
    # step out on any axis is 0.1 > sqrt(3)/2 s = 0.0866 away
    assert hits[:, 0].sum() == 6 * 2 * 2


def test_map_shifts_with_the_robot():
    rng = np.random.default_rng(4)
    a, d = rng.uniform(0, 0.3, 3), rng.uniform(0, 0.3, 3)
    desc = dict(dof=3, a=a, alpha=np.array([0.0, np.pi / 2, 0.0]), d=d, q_lo=-np.pi * np.ones(3),
                q_hi=np.pi * np.ones(3), sphere_link=np.repeat(np.arange(3), 3).astype(np.int32),
                sphere_xyz=rng.uniform(-0.1, 0.1, (9, 3)), sphere_r=rng.uniform(0.02, 0.06, 9))
    rob = oracle.Robot(desc)
    q = rng.uniform(-np.pi, np.pi, (20, 3))
    s, dims = 0.05, (30, 30, 30)
    lo = np.array([-0.75, -0.75, -0.75])
    h1, _ = oracle.collision_map(rob, q, lo, s, dims)
    # moving the grid by -s in x moves every voxel index by +1 in x
    h2, _ = oracle.collision_map(rob, q, lo - np.array([s, 0, 0]), s, dims)
    H1 = h1.reshape(dims[2], dims[1], dims[0], -1)
    H2 = h2.reshape(dims[2], dims[1], dims[0], -1)
    assert np.array_equal(H1[:, :, :-1], H2[:, :, 1:])
    assert h1.any(axis=0).all()            # every node touches some voxel
