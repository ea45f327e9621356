"""Stored synthetic workloads and their inflation parameters.

`load(name)` reads `workloads/<name>.npz` (numpy, allow_pickle=False).  The
files are written by `oracle/make_workloads.py`; `draw.py` holds the seeded
raw draws.  Parameter presets follow the paper's EI-ZO tables (Appendix,
"Supplementary Information on Experimental Evaluation") where they give a
value, with eps/confidence taken from the workload definitions:

  step back Delta_max = 0.01, N_f = 10 faces per iteration,
  N_mix = 30 (2-D/planar table) or 60 (7-DOF table),
  tau = 0.5 (Sec. IV-B footnote), delta = 1 - confidence = 0.05,
  N_b = 11 = ceil(log2(diam(D)/Delta_max)) (Sec. IV-C rule of thumb),
  t_col = 1e-4, N_it = 50.
"""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

ROBOT_KEYS = ("dof", "a", "alpha", "d", "q_lo", "q_hi", "sphere_link", "sphere_xyz",
              "sphere_r", "self_pairs")

PARAMS = {
    "tiny": dict(eps=0.1, delta=0.05, tau=0.5, step_back_max=0.01, t_col=1e-4, n_p=1000,
                 n_f=10, n_b=11, n_mix=30, max_iters=50),
    "dof7": dict(eps=0.05, delta=0.05, tau=0.5, step_back_max=0.01, t_col=1e-4, n_p=10000,
                 n_f=10, n_b=11, n_mix=60, max_iters=50),
    "batched": dict(eps=0.05, delta=0.05, tau=0.5, step_back_max=0.01, t_col=1e-4, n_p=10000,
                    n_f=10, n_b=11, n_mix=60, max_iters=50),
    "boxes": dict(eps=0.05, delta=0.05, tau=0.5, step_back_max=0.01, t_col=1e-4, n_p=10000,
                  n_f=20, n_b=11, n_mix=60, max_iters=50),
    # the paper's Forest table: delta 0.05, eps 0.01, N_p 1000, N_f 10, N_ms 30, Delta 0.01
    "forest": dict(eps=0.01, delta=0.05, tau=0.5, step_back_max=0.01, t_col=1e-4, n_p=1000,
                   n_f=10, n_b=11, n_mix=30, max_iters=50),
}


def load(name: str) -> dict:
    with np.load(os.path.join(HERE, f"{name}.npz"), allow_pickle=False) as z:
        data = {k: z[k] for k in z.files}
    data["dof"] = int(data["dof"])
    return data


BOX_KEYS = ("box_link", "box_pose", "box_half", "box_pairs", "joint_type")


def robot(data: dict) -> dict:
    out = {k: data[k] for k in ROBOT_KEYS}
    out.update({k: data[k] for k in BOX_KEYS if k in data})
    return out
