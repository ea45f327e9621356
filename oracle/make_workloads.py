"""Writes the stored synthetic workloads `workloads/*.npz`.

Test infrastructure: it draws raw values with `workloads.draw` and uses the
FP64 oracle only to reject draws (self-colliding arms, segments that
self-collide, obstacles that touch the arm anywhere along a segment).  The
GPU path never contributes to any stored value.

Recipe (stand-ins for the paper's Forest / Franka / iiwa scenes, whose models
and data are not public in this form):

  tiny     seed 0: 3-DOF planar arm, 3 links x 4 spheres; self pairs = link 1
           x link 3; one self-free segment of length 0.5 rad; 20 obstacle
           discs (z = 0) with centres U[-1.5, 1.5]^2, r U[0.05, 0.15],
           each redrawn while it comes within `MARGIN` of the arm anywhere
           along the segment.
  dof7     seed 1: 7-DOF DH arm (7 x 10 spheres); self pairs = links at
           least two apart, minus pairs already touching at q = 0; arm
           redrawn while more than half of 10^4 uniform configurations
           self-collide; one self-free segment of length U[0.3, 1.0] rad;
           512 obstacles in [0.3,1.3]x[-0.5,0.5]x[0,1] m, r U[0.02, 0.08],
           rejected as for tiny.
  batched  seed 2: arm of dof7; 8 piecewise-linear paths with
           2,5,8,11,14,17,19,20 segments (96 edges) of length U[0.3, 1.0]
           rad each, self-free, inside the limits; then 2048 obstacles in
           the same box rejected against all 96 swept segments.
  sweep    seed 3: arm of dof7; 256 / 1024 / 4096 obstacles in the box, no
           rejection (configurations are drawn at run time, uniform).
  boxes    seed 4: the dof7 arm's links covered by 11 boxes (no spheres);
           box self pairs = links at least two apart, minus pairs touching at
           q = 0; voxel obstacles (side 0.08 m, circumscribing spheres)
           filling 6 random boxes in the obstacle box, plus a table box whose
           top is 20 cm below the base; one segment of length U[0.3, 1.0] rad
           free of self-collision, voxels and table along its length.
  forest   seed 5: the Forest scene: a point robot in [0, 10]^2 (two
           prismatic joints), 15 discs of radius 0.35 with centres uniform in
           the central [1.5, 8.5]^2; a piecewise-linear path from (0.5, 0.5)
           to (9.5, 9.5) found by breadth-first search on a 0.1 grid keeping
           0.1 clearance, thinned to straight pieces that stay free.

"Along the segment" is checked on a discretisation fine enough that no
sphere moves more than MARGIN/2 between neighbouring points, so keeping a
signed distance >= MARGIN at every point keeps the whole segment free.

Usage:  python -m oracle.make_workloads [--only NAME]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
from scipy.spatial import cKDTree

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from workloads import draw  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads")
MARGIN = 2e-3
OBS_BOX = ([0.3, -0.5, 0.0], [1.3, 0.5, 1.0])


def robot_reach_sum(desc) -> float:
    """Upper bound of sum_i (max distance of any sphere from joint axis i)."""
    L = np.abs(desc["a"]).astype(np.float64) + np.abs(desc["d"]).astype(np.float64)
    tail = np.cumsum(L[::-1])[::-1]            # length of the chain from joint i outward
    return float(np.sum(tail + float(np.max(desc["sphere_r"]))))


def discretise(v1, v2, reach_sum):
    """Points on [v1, v2] spaced so that every sphere moves <= MARGIN/2."""
    v1 = v1.astype(np.float64)
    v2 = v2.astype(np.float64)
    h = MARGIN / max(reach_sum, 1e-9)           # max joint step (inf-norm)
    n = int(np.ceil(np.max(np.abs(v2 - v1)) / h)) + 1
    w = np.linspace(0.0, 1.0, n)[:, None]
    return (1 - w) * v1 + w * v2


def self_free(rob: oracle.Robot, qs) -> bool:
    _, _, _, ss = oracle.check(rob, np.zeros((0, 4)), qs)
    return bool(np.all(ss >= MARGIN))


def swept_centres(rob: oracle.Robot, qs):
    pts = np.empty((len(qs), rob.n_spheres, 3))
    for i, q in enumerate(qs):
        pts[i] = oracle.sphere_centres(rob, q)
    return pts.reshape(-1, 3), np.tile(rob.sphere_r, len(qs))


def reject_obstacles(rng, n, box_lo, box_hi, r_lo, r_hi, pts, prad, planar=False, batch=4096):
    tree = cKDTree(pts)
    rmax = float(np.max(prad))
    kept, drawn = [], 0
    while len(kept) < n:
        cand = draw.obstacle_candidates(rng, batch, box_lo, box_hi, r_lo, r_hi, planar)
        for o in cand:
            drawn += 1
            oc = o[:3].astype(np.float64)
            ro = float(o[3])
            idx = tree.query_ball_point(oc, ro + rmax + MARGIN)
            if idx:
                sd = np.linalg.norm(pts[idx] - oc, axis=1) - prad[idx] - ro
                if np.min(sd) < MARGIN:
                    continue
            kept.append(o)
            if len(kept) == n:
                break
    return np.asarray(kept, np.float32), len(kept) / drawn


def robot_arrays(desc, self_pairs):
    return dict(dof=np.int32(desc["dof"]), a=desc["a"], alpha=desc["alpha"], d=desc["d"],
                q_lo=desc["q_lo"], q_hi=desc["q_hi"], sphere_link=desc["sphere_link"],
                sphere_xyz=desc["sphere_xyz"], sphere_r=desc["sphere_r"],
                self_pairs=np.asarray(self_pairs, np.int32).reshape(-1, 2))


def make_tiny():
    rng = draw.rng_for(0)
    desc = draw.arm_planar(rng)
    sp = draw.self_pair_candidates(desc["sphere_link"], 2)
    rob = oracle.Robot(desc, sp)
    reach = robot_reach_sum(desc)
    while True:
        e = draw.segment_candidate(rng, desc["q_lo"], desc["q_hi"], 0.5)
        if e is None:
            continue
        qs = discretise(e[0], e[1], reach)
        if self_free(rob, qs):
            break
    pts, prad = swept_centres(rob, qs)
    obs, acc = reject_obstacles(rng, 20, [-1.5, -1.5], [1.5, 1.5], 0.05, 0.15, pts, prad, planar=True,
                                batch=64)
    return dict(robot_arrays(desc, sp), obstacles=obs, edges=e[None], path_id=np.zeros(1, np.int32),
                obstacle_acceptance=np.float64(acc))


def make_arm7():
    rng = draw.rng_for(1)
    while True:
        desc = draw.arm_dh(rng)
        cand = draw.self_pair_candidates(desc["sphere_link"], 2)
        rob0 = oracle.Robot(desc, cand)
        q0 = np.zeros(desc["dof"])
        c = oracle.sphere_centres(rob0, q0)
        r = rob0.sphere_r
        sd0 = np.linalg.norm(c[cand[:, 0]] - c[cand[:, 1]], axis=1) - r[cand[:, 0]] - r[cand[:, 1]]
        sp = cand[sd0 >= 0.0]
        rob = oracle.Robot(desc, sp)
        qs = draw.uniform_q(12345, 10_000, desc["q_lo"], desc["q_hi"])
        _, _, _, ss = oracle.check(rob, np.zeros((0, 4)), qs)
        frac = float(np.mean(ss < 0))
        if frac <= 0.5:
            return rng, desc, sp, rob, frac


def make_dof7():
    rng, desc, sp, rob, frac = make_arm7()
    reach = robot_reach_sum(desc)
    while True:
        e = draw.segment_candidate(rng, desc["q_lo"], desc["q_hi"], rng.uniform(0.3, 1.0))
        if e is None:
            continue
        qs = discretise(e[0], e[1], reach)
        if self_free(rob, qs):
            break
    pts, prad = swept_centres(rob, qs)
    lo, hi = OBS_BOX
    obs, acc = reject_obstacles(rng, 512, lo, hi, 0.02, 0.08, pts, prad)
    return dict(robot_arrays(desc, sp), obstacles=obs, edges=e[None], path_id=np.zeros(1, np.int32),
                obstacle_acceptance=np.float64(acc), self_collision_fraction=np.float64(frac))


def make_batched():
    _, desc, sp, rob, frac = make_arm7()
    rng = draw.rng_for(2)
    reach = robot_reach_sum(desc)
    edges, pid, qs_all = [], [], []
    for p, nseg in enumerate(draw.PATH_SEGMENTS):
        while True:      # draw a whole path; restart the path if it gets stuck
            start = rng.uniform(desc["q_lo"], desc["q_hi"])
            segs, ok = [], True
            for _ in range(nseg):
                for _attempt in range(200):
                    e = draw.segment_candidate(rng, desc["q_lo"], desc["q_hi"], rng.uniform(0.3, 1.0),
                                               start=start if not segs else segs[-1][1])
                    if e is None:
                        continue
                    qs = discretise(e[0], e[1], reach)
                    if self_free(rob, qs):
                        segs.append(e)
                        break
                else:
                    ok = False
                    break
            if ok:
                break
        for e in segs:
            edges.append(e)
            pid.append(p)
            qs_all.append(discretise(e[0], e[1], reach))
    qs = np.concatenate(qs_all)
    pts, prad = swept_centres(rob, qs)
    lo, hi = OBS_BOX
    obs, acc = reject_obstacles(rng, 2048, lo, hi, 0.02, 0.08, pts, prad)
    return dict(robot_arrays(desc, sp), obstacles=obs, edges=np.asarray(edges, np.float32),
                path_id=np.asarray(pid, np.int32), obstacle_acceptance=np.float64(acc),
                self_collision_fraction=np.float64(frac))


def make_sweep():
    _, desc, sp, rob, frac = make_arm7()
    rng = draw.rng_for(3)
    lo, hi = OBS_BOX
    out = robot_arrays(desc, sp)
    for n in (256, 1024, 4096):
        out[f"obstacles_{n}"] = draw.obstacle_candidates(rng, n, lo, hi, 0.02, 0.08)
    return out


TABLE = np.concatenate([[0.4, 0.0, -0.45], np.eye(3).ravel(), [1.2, 1.2, 0.25]])   # top at z = -0.2


def box_reach_sum(desc, half) -> float:
    """As robot_reach_sum, with the largest box half-diagonal as the radius."""
    L = np.abs(desc["a"]).astype(np.float64) + np.abs(desc["d"]).astype(np.float64)
    tail = np.cumsum(L[::-1])[::-1]
    return float(np.sum(tail + float(np.max(np.linalg.norm(half, axis=1)))))


def make_boxes():
    _, arm, _, _, _ = make_arm7()
    rng = draw.rng_for(4)
    bl, bp, bh = draw.arm_boxes(rng, arm)
    desc = dict(arm, sphere_link=np.zeros(0, np.int32), sphere_xyz=np.zeros((0, 3), np.float32),
                sphere_r=np.zeros(0, np.float32), box_link=bl, box_pose=bp, box_half=bh)
    i, j = np.triu_indices(len(bl), 1)
    cand = np.stack([i, j], axis=1)[np.abs(bl[i] - bl[j]) >= 2].astype(np.int32)
    keep = []
    for pr in cand:
        _, _, _, ss = oracle.check(oracle.Robot(dict(desc, box_pairs=pr[None])), np.zeros((0, 4)),
                                   np.zeros((1, arm["dof"])))
        keep.append(ss[0] >= 0.0)
    bpairs = cand[np.array(keep, bool)]
    desc["box_pairs"] = bpairs
    rob = oracle.Robot(desc, np.zeros((0, 2), np.int32))
    qs = draw.uniform_q(12346, 10_000, arm["q_lo"], arm["q_hi"])
    _, _, _, ss = oracle.check(rob, np.zeros((0, 4)), qs)
    frac = float(np.mean(ss < 0))
    lo, hi = OBS_BOX
    vox = draw.voxel_obstacles(rng, lo, hi)
    table = draw._f32(TABLE)[None]
    reach = box_reach_sum(arm, bh)
    for _ in range(100_000):
        e = draw.segment_candidate(rng, arm["q_lo"], arm["q_hi"], rng.uniform(0.3, 1.0))
        if e is None:
            continue
        qd = discretise(e[0], e[1], reach)
        _, sd, _, _ = oracle.check(rob, vox, qd, env_boxes=table)
        if np.all(sd >= MARGIN):
            break
    else:
        raise RuntimeError("no free segment found")
    out = dict(robot_arrays(desc, np.zeros((0, 2), np.int32)), box_link=bl, box_pose=bp, box_half=bh,
               box_pairs=bpairs, obstacles=vox, env_boxes=table, edges=e[None], path_id=np.zeros(1, np.int32),
               self_collision_fraction=np.float64(frac))
    return out


def make_forest():
    from collections import deque
    rng = draw.rng_for(5)
    desc = draw.point_robot_plane(10.0)
    discs = draw.forest_discs(rng)
    # world spheres: the point sits at (0, q_2, q_1)
    obs = draw._f32(np.stack([np.zeros(len(discs)), discs[:, 1], discs[:, 0], discs[:, 2]], axis=1))
    rob = oracle.Robot(desc)
    h = 0.1
    g = np.arange(0.05, 10.0, h)
    X, Y = np.meshgrid(g, g, indexing="ij")
    clear = np.min(np.hypot(X[..., None] - discs[:, 0], Y[..., None] - discs[:, 1]) - discs[:, 2], axis=2)
    free = clear >= 0.1
    start, goal = (4, 4), (94, 94)
    prev = {start: None}
    dq = deque([start])
    while dq:
        c = dq.popleft()
        if c == goal:
            break
        for di, dj in ((1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)):
            n = (c[0] + di, c[1] + dj)
            if 0 <= n[0] < len(g) and 0 <= n[1] < len(g) and free[n] and n not in prev:
                prev[n] = c
                dq.append(n)
    cells = [goal]
    while prev[cells[-1]] is not None:
        cells.append(prev[cells[-1]])
    pts = np.array([[g[i], g[j]] for i, j in cells[::-1]])

    def seg_free(a, b):
        n = int(np.ceil(np.max(np.abs(b - a)) / 1e-3)) + 1
        w = np.linspace(0.0, 1.0, n)[:, None]
        _, sd, _, _ = oracle.check(rob, obs, (1 - w) * a + w * b)
        return bool(np.all(sd >= MARGIN))

    verts, i = [pts[0]], 0
    while i < len(pts) - 1:                 # greedy: the farthest grid point reachable in a straight free line
        j = len(pts) - 1
        while j > i + 1 and not seg_free(pts[i], pts[j]):
            j -= 1
        verts.append(pts[j])
        i = j
    V = draw._f32(verts)
    edges = np.stack([V[:-1], V[1:]], axis=1)
    return dict(robot_arrays(desc, np.zeros((0, 2), np.int32)), joint_type=desc["joint_type"], obstacles=obs,
                discs=discs, edges=edges, path_id=np.zeros(len(edges), np.int32))


MAKERS = dict(tiny=make_tiny, dof7=make_dof7, batched=make_batched, sweep=make_sweep, boxes=make_boxes,
              forest=make_forest)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    args = ap.parse_args()
    oracle.build(force=False)
    for name, fn in MAKERS.items():
        if args.only and name != args.only:
            continue
        t0 = time.time()
        data = fn()
        np.savez(os.path.join(OUT, f"{name}.npz"), **data)
        extra = {k: float(v) for k, v in data.items() if k in ("obstacle_acceptance", "self_collision_fraction")}
        print(f"{name}: {time.time() - t0:.1f}s {extra}", flush=True)


if __name__ == "__main__":
    main()
