"""Seeded raw draws for the synthetic workloads.

This module only draws numbers: arm geometry parameters, candidate obstacle
spheres, candidate segment end points and uniform configuration batches.  It
holds none of the inflation method's arithmetic (no kinematics, no distances,
no collision tests); rejection of draws that touch the arm is done by the
workload maker that owns a collision predicate.  Every value is rounded to
float32 here, so the GPU path (FP32) and the FP64 reference read bit-identical
inputs.

Geometry readings (stand-ins for the paper's Franka / iiwa models, which are
not available; Sec. VI-A "Environments" and Sec. VI-B describe what they are
standing in for):

* planar arm: standard DH with alpha = d = 0, link lengths U[0.3, 0.6] m,
  4 spheres per link evenly spaced on the link, radii U[0.03, 0.06] m;
* 7-DOF arm: standard DH, a_i, d_i ~ U[0, 0.4] m, alpha_i uniform on
  {0, +pi/2, -pi/2}, 10 spheres per link evenly spaced on the segment from
  the previous frame origin to the link's own origin, radii U[0.03, 0.06] m;
* joint limits [-pi, pi] on every joint;
* box arm (the iiwa's 11-box model): the 7-DOF arm's links, each covered by
  a box aligned with the segment from the previous frame origin to the link's
  own origin (x axis along it), the four longest segments split in two boxes;
  half widths U[0.04, 0.07] m, lengths covering the segment plus the width at
  each end; a link whose segment has zero length gets a cube of half width
  0.05 m at its origin;
* perceived obstacles: voxels of side 0.08 m filling a few random boxes,
  each voxel represented by its circumscribing sphere (radius sqrt(3)/2 s),
  as in the paper's perception pipeline; a table as one box.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
PI = np.pi


def rng_for(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([0x455A4F, int(seed)]))


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(F32)


def arm_planar(rng: np.random.Generator, dof: int = 3, spheres_per_link: int = 4):
    """Planar serial arm: DH with alpha = d = 0; spheres on the x axis of
    each link frame at x = ((j + 1/2)/n - 1) * l, i.e. spread along the link
    from the previous joint to the link's end."""
    a = _f32(rng.uniform(0.3, 0.6, size=dof))
    alpha = np.zeros(dof, F32)
    d = np.zeros(dof, F32)
    link, xyz, r = [], [], []
    for i in range(dof):
        for j in range(spheres_per_link):
            t = (j + 0.5) / spheres_per_link
            link.append(i)
            xyz.append([(t - 1.0) * float(a[i]), 0.0, 0.0])
            r.append(rng.uniform(0.03, 0.06))
    return dict(
        dof=dof, a=a, alpha=alpha, d=d,
        q_lo=_f32(np.full(dof, -PI)), q_hi=_f32(np.full(dof, PI)),
        sphere_link=np.asarray(link, np.int32),
        sphere_xyz=_f32(xyz).reshape(-1, 3), sphere_r=_f32(r),
    )


def arm_dh(rng: np.random.Generator, dof: int = 7, spheres_per_link: int = 10):
    """Serial arm with seeded standard-DH parameters.  In frame i the
    previous origin o_{i-1} sits at (-a_i, -d_i sin(alpha_i), -d_i cos(alpha_i));
    spheres are placed at (1 - t_j) * o_{i-1}, t_j = (j + 1/2)/n."""
    a = _f32(rng.uniform(0.0, 0.4, size=dof))
    d = _f32(rng.uniform(0.0, 0.4, size=dof))
    choice = rng.integers(0, 3, size=dof)
    sa = np.array([0.0, 1.0, -1.0])[choice]
    ca = np.array([1.0, 0.0, 0.0])[choice]
    alpha = _f32(np.array([0.0, PI / 2, -PI / 2])[choice])
    link, xyz, r = [], [], []
    for i in range(dof):
        prev = np.array([-float(a[i]), -float(d[i]) * sa[i], -float(d[i]) * ca[i]])
        for j in range(spheres_per_link):
            t = (j + 0.5) / spheres_per_link
            link.append(i)
            xyz.append((1.0 - t) * prev)
            r.append(rng.uniform(0.03, 0.06))
    return dict(
        dof=dof, a=a, alpha=alpha, d=d,
        q_lo=_f32(np.full(dof, -PI)), q_hi=_f32(np.full(dof, PI)),
        sphere_link=np.asarray(link, np.int32),
        sphere_xyz=_f32(xyz).reshape(-1, 3), sphere_r=_f32(r),
    )


def self_pair_candidates(sphere_link: np.ndarray, min_link_gap: int = 2) -> np.ndarray:
    """All sphere pairs (s, t), s < t, whose links are at least
    `min_link_gap` apart in the chain."""
    S = len(sphere_link)
    s, t = np.triu_indices(S, k=1)
    keep = np.abs(sphere_link[s] - sphere_link[t]) >= min_link_gap
    return np.stack([s[keep], t[keep]], axis=1).astype(np.int32)


def obstacle_candidates(rng, n, lo, hi, r_lo, r_hi, planar=False):
    """n candidate obstacle spheres [n][4] = (x, y, z, r), centres uniform in
    the box [lo, hi] (z = 0 for planar scenes), radii uniform in [r_lo, r_hi]."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = rng.uniform(lo, hi, size=(n, len(lo)))
    if planar:
        c = np.concatenate([c[:, :2], np.zeros((n, 1))], axis=1)
    r = rng.uniform(r_lo, r_hi, size=(n, 1))
    return _f32(np.concatenate([c, r], axis=1))


def unit_direction(rng, dof):
    g = rng.standard_normal(dof)
    return g / np.linalg.norm(g)


def segment_candidate(rng, q_lo, q_hi, length, start=None):
    """Candidate segment (v1, v2): v1 uniform in the limits (or `start`),
    v2 = v1 + length * u with u uniform on the unit sphere.  Returns None if
    v2 leaves the limits (the caller draws again)."""
    q_lo = np.asarray(q_lo, np.float64)
    q_hi = np.asarray(q_hi, np.float64)
    v1 = rng.uniform(q_lo, q_hi) if start is None else np.asarray(start, np.float64)
    v2 = v1 + length * unit_direction(rng, len(q_lo))
    v1f, v2f = _f32(v1), _f32(v2)
    if np.any(v2f < q_lo.astype(F32)) or np.any(v2f > q_hi.astype(F32)):
        return None
    if np.any(v1f < q_lo.astype(F32)) or np.any(v1f > q_hi.astype(F32)):
        return None
    return np.stack([v1f, v2f])


def uniform_q(seed: int, n: int, q_lo, q_hi) -> np.ndarray:
    """n configurations uniform in the joint limits, [n][dof] float32."""
    rng = rng_for(seed)
    q_lo = np.asarray(q_lo, np.float64)
    q_hi = np.asarray(q_hi, np.float64)
    out = np.empty((n, len(q_lo)), F32)
    step = 1 << 22
    for s in range(0, n, step):
        m = min(step, n - s)
        out[s:s + m] = rng.uniform(q_lo, q_hi, size=(m, len(q_lo))).astype(F32)
    return out


def uniform_q_fast(seed: int, n: int, q_lo, q_hi) -> np.ndarray:
    """Same law as `uniform_q`, drawn as float32 directly (for the large
    throughput sweeps where 16M x 7 doubles would be wasteful)."""
    rng = rng_for(seed)
    q_lo = np.asarray(q_lo, F32)
    q_hi = np.asarray(q_hi, F32)
    u = rng.random((n, len(q_lo)), dtype=F32)
    return (q_lo + u * (q_hi - q_lo)).astype(F32)


PATH_SEGMENTS = (2, 5, 8, 11, 14, 17, 19, 20)


def arm_boxes(rng: np.random.Generator, desc: dict, n_boxes: int = 11):
    """Boxes on the links of a DH arm (see the module docstring): returns
    box_link [B], box_pose [B][12] (centre, rotation row-major with the box
    axes as columns, link frame), box_half [B][3]."""
    dof = int(desc["dof"])
    a, d, al = (np.asarray(desc[k], np.float64) for k in ("a", "d", "alpha"))
    prev = np.stack([-a, -d * np.sin(al), -d * np.cos(al)], axis=1)      # previous origin in frame i
    length = np.linalg.norm(prev, axis=1)
    split = set(np.argsort(-length)[:max(0, n_boxes - dof)].tolist())
    link, pose, half = [], [], []
    for i in range(dof):
        w = rng.uniform(0.04, 0.07)
        if length[i] < 1e-9:
            link.append(i)
            pose.append(np.concatenate([np.zeros(3), np.eye(3).ravel()]))
            half.append([0.05, 0.05, 0.05])
            continue
        u = -prev[i] / length[i]                      # from the previous origin towards this one
        t = np.array([0.0, 0.0, 1.0]) if abs(u[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
        y = np.cross(t, u)
        y /= np.linalg.norm(y)
        z = np.cross(u, y)
        R = np.stack([u, y, z], axis=1)               # columns = box axes
        parts = 2 if i in split else 1
        for k in range(parts):
            c = prev[i] + (k + 0.5) / parts * (-prev[i])
            link.append(i)
            pose.append(np.concatenate([c, R.ravel()]))
            half.append([length[i] / (2 * parts) + w, w, w])
    return (np.asarray(link, np.int32), _f32(pose).reshape(-1, 12), _f32(half).reshape(-1, 3))


def voxel_obstacles(rng: np.random.Generator, lo, hi, side: float = 0.08, n_shapes: int = 6,
                    size_lo: float = 0.1, size_hi: float = 0.4):
    """Voxel spheres [n][4] (centre, r = sqrt(3)/2 side) of the voxels of a
    side-`side` grid over [lo, hi] whose centres fall in one of n_shapes
    random axis-aligned boxes (sizes U[size_lo, size_hi] per axis)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n = np.floor((hi - lo) / side).astype(int)
    g = [lo[k] + side * (np.arange(n[k]) + 0.5) for k in range(3)]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    cen = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    keep = np.zeros(len(cen), bool)
    for _ in range(n_shapes):
        sz = rng.uniform(size_lo, size_hi, 3)
        c0 = rng.uniform(lo + sz / 2, hi - sz / 2)
        keep |= np.all(np.abs(cen - c0) <= sz / 2, axis=1)
    v = cen[keep]
    return _f32(np.concatenate([v, np.full((len(v), 1), np.sqrt(3) / 2 * side)], axis=1))


def point_robot_plane(extent: float = 10.0):
    """A point robot in a plane as a 2-DOF arm of two prismatic joints
    (theta = 0, offset d + q): joint 1 slides along world z, alpha_1 = -pi/2
    turns the next axis onto world y, joint 2 slides along it; the point
    (one sphere of radius 0 on link 2) sits at world (0, q_2, q_1).  Limits
    [0, extent] on both joints."""
    return dict(
        dof=2, a=np.zeros(2, F32), alpha=_f32([-PI / 2, 0.0]), d=np.zeros(2, F32),
        q_lo=np.zeros(2, F32), q_hi=_f32([extent, extent]),
        sphere_link=np.array([1], np.int32), sphere_xyz=np.zeros((1, 3), F32), sphere_r=np.zeros(1, F32),
        joint_type=np.array([1, 1], np.int32),
    )


def forest_discs(rng: np.random.Generator, n: int = 15, lo: float = 1.5, hi: float = 8.5, r: float = 0.35):
    """The Forest scene's discs in configuration coordinates (q_1, q_2, r):
    centres uniform in the central [lo, hi]^2 of the domain, radius r."""
    c = rng.uniform(lo, hi, size=(n, 2))
    return _f32(np.concatenate([c, np.full((n, 1), r)], axis=1))
