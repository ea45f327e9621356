#!/usr/bin/env python
"""Throughput of the EI-ZO hot path on one MI355X.

A step is one pass of the whole hot path -- ezo_inflate_edges on the
workload's edges (hit-and-run sampling, FK + collision checks, unadaptive
test, projection + bisection, hyperplane placement, every iteration until
every edge is certified) -- with all inputs resident in HBM.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dof7|batched|tiny]

Prints one JSON line.  `value` = collision-checked configurations per second
(exact checks counted by the library, summed over the step, divided by the
step time); `edges_per_s` is the same run's edges inflated per second.
`roofline` reports the dominant kernel phase timed live with hipEvents on the
stream it runs on; `cpu_baseline` times the FP64 reference on one full
inflation of the same workload (rank 0 only).

The default run (the 7-DOF edge) also carries the metric's other
configurations as sub-objects of the same line (`--no-extras` leaves them
out): `batched` (the 96 edges of 8 uneven paths in one call, the plain
one-call-per-edge form at identical certification, its own roofline and CPU
baseline), `sweep` (the raw checker at 16 M configurations x 256 / 1024 /
4096 obstacles, flags and signed distances) and `screen` (the learned
self-collision screen against the exact form on the batched workload).
Progress lines go to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X FP32 vector peak
FK_FLOP = 1800                # forward kinematics per configuration (7 links)
PAIR_FLOP = 13                # one sphere-sphere signed-distance test

WORKLOADS = {
    "dof7": "7-DOF DH arm (7x10 spheres, 1500 self pairs), 512 obstacle spheres, one edge; "
            "N_p=10000, eps=0.05, delta=0.05, tau=0.5, N_f=10, N_b=11, N_mix=60",
    "batched": "7-DOF DH arm, 2048 obstacle spheres, 96 edges of 8 uneven paths in one call; "
               "eps=0.05, delta=0.05, N_mix=60 (N_p in config.n_p)",
    "tiny": "3-DOF planar arm (12 spheres), 20 obstacle discs, one edge; N_p=1000, eps=0.1, delta=0.05",
    "forest": "Forest scene: point robot in [0,10]^2 (two prismatic joints), 15 discs r=0.35, a 4-edge path; "
              "N_p=1000, eps=0.01, delta=0.05, N_f=10, N_b=11, N_mix=30",
    "boxes": "7-DOF DH arm as 11 link boxes (36 box self pairs), 194 voxel spheres (8 cm voxels) and a table "
             "box, one edge; N_p=10000, eps=0.05, delta=0.05, N_f=20, N_b=11, N_mix=60",
}


KERNEL_SOURCES = ("paper_2504_10783_amd/csrc/ezo_device.hpp", "paper_2504_10783_amd/csrc/ezo_kernels.hpp",
                  "paper_2504_10783_amd/csrc/ezo_screen.hpp")


def kernel_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel_instance, n_p):
    """HBM bytes per launch of `kernel_instance` (that template instance,
    i.e. that launch shape) from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload (each counter scaled by its reading
    for a plain 1 GiB copy), or None when there is no summary, the instance
    was not measured, the kernel sources changed since the counters were
    taken, or the counters were taken at another N_p (samples per
    iteration)."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic__{workload}_inflate.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            if rec.get("source_sha256") != kernel_source_sha256() or rec.get("n_p") != n_p:
                return None
            return rec.get("bytes_per_launch_by_instance", {}).get(kernel_instance)
    return None


def measured_valu(workload, kernel_instance, n_p):
    """Counted FP32 VALU flop per launch (64 lanes x (ADD + MUL + TRANS +
    2 FMA) wave instructions, rocprofv3 SQ_INSTS_VALU_*_F32) of
    `kernel_instance` from the committed summary of this workload, or None
    (no summary, instance not measured, kernel sources changed since, or
    another N_p)."""
    path = os.path.join(ROOT, "profiles", f"valu_fp32__{workload}_inflate.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("valu-json: "):
            rec = json.loads(line[len("valu-json: "):])
            if rec.get("source_sha256") != kernel_source_sha256() or rec.get("n_p") != n_p:
                return None
            return rec.get("fp32_flop_per_launch_by_instance", {}).get(kernel_instance)
    return None


def flop_per_check(n_spheres, n_obs, n_self):
    return PAIR_FLOP * (n_spheres * n_obs + n_self) + FK_FLOP


def samples_arg(v):
    if v in ("paper", "tuned"):
        return v
    if not v.isdigit() or int(v) < 1:
        raise argparse.ArgumentTypeError("--samples takes 'paper', 'tuned' or a positive count")
    return int(v)


def sample_mode(args, name):
    """N_p source: the batched workload's configuration leaves the sample
    count to the tuner; the single-edge workloads use the paper's table."""
    return args.samples or ("tuned" if name == "batched" else "paper")


def sample_params(args, name):
    """Workload parameters with N_p set as --samples asks (n_p = 0: tuned)."""
    import workloads
    wp = dict(workloads.PARAMS[name])
    m = sample_mode(args, name)
    if m == "tuned":
        wp["n_p"] = 0
    elif m != "paper":
        wp["n_p"] = m
    return wp


def tuned_sample_count(ezo, rob, n_obs):
    """N_p the sample-count tuner picked for this robot and obstacle count."""
    hits = [x["T"] for x in ezo.tune_cache_entries()
            if x["kernel"] == "samples" and x["dof"] == rob.dof and x["spheres"] == rob.n_spheres
            and x["obstacles"] == n_obs]
    if len(set(hits)) != 1:
        raise RuntimeError(f"expected one tuned sample count for this workload, cache holds {hits}")
    return hits[0]


def timed_shapes(ezo, rob, n_obs, prm, n_p, E):
    """The cached launch shapes the inflation of E edges with N_p = n_p used:
    the entries whose key matches the call's work sizes (the check on
    max_k max(N_p, M_k) samples per edge, the bisection on N_p candidate
    slots per edge; bucket = floor(log2(items)))."""
    s_cap = max(max(n_p, ezo.test_constants(prm.eps, prm.delta, prm.tau, k)[0]) for k in range(1, prm.max_iters + 1))
    want = {"check_flags": (s_cap * E).bit_length() - 1, "bisect": (n_p * E).bit_length() - 1}
    out = {}
    for e in ezo.tune_cache_entries():
        if (e["kernel"] in want and e["log2_items"] == want[e["kernel"]] and e["obstacles"] == n_obs
                and e["dof"] == rob.dof and e["spheres"] == rob.n_spheres):
            out[e["kernel"]] = e
    return out


def cpu_model():
    """The host CPU's model name (lscpu's "Model name", from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.lower().startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(name, data, desc, seed, edges_idx, n_p=None):
    import numpy as np
    import oracle
    import workloads
    orob = oracle.Robot(desc)
    obs = data["obstacles"].astype(np.float64)
    checks = 0
    t0 = time.perf_counter()
    for e in edges_idx:
        v1, v2 = data["edges"][e].astype(np.float64)
        wp = dict(workloads.PARAMS[name], **({"n_p": n_p} if n_p else {}))
        prm = oracle.make_params(**wp, seed=seed, edge_id=int(e))
        out = oracle.eizo_arm(orob, obs, v1, v2, prm, env_boxes=data.get("env_boxes"))
        checks += out["stats"]["checks"]
    dt = time.perf_counter() - t0
    # the same reference on one host thread, first edge of the sample only
    e = edges_idx[0]
    v1, v2 = data["edges"][e].astype(np.float64)
    wp = dict(workloads.PARAMS[name], **({"n_p": n_p} if n_p else {}))
    cores = oracle.max_threads()
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        out = oracle.eizo_arm(orob, obs, v1, v2, oracle.make_params(**wp, seed=seed, edge_id=int(e)),
                              env_boxes=data.get("env_boxes"))
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {"value": checks / dt, "unit": "configs/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"FP64 reference EI-ZO on {len(edges_idx)} edge(s) of the '{name}' workload "
                      f"(seed {seed}, N_p {n_p or workloads.PARAMS[name]['n_p']}): {checks} exact checks "
                      f"in {dt:.2f} s; one thread: edge {e}, {out['stats']['checks']} checks in {dt1:.2f} s",
            "edges_per_s": len(edges_idx) / dt,
            "value_1thread": out["stats"]["checks"] / dt1}


def sweep_measure(args, sizes, reps_cap=None):
    """Raw checker throughput: N uniform configurations x n_obs obstacles,
    flags + minimum signed distance (all pairs) and flags only (broad phase).
    Inputs resident in HBM; wall timing around synchronised repetitions (the
    checker runs on torch's current stream).  Returns (points, cpu baseline
    or None, the tuner's cache entries)."""
    import numpy as np
    import torch

    import paper_2504_10783_amd as ezo
    import workloads
    from workloads import draw

    data = workloads.load("sweep")
    desc = workloads.robot(data)
    ctx = ezo.Context(0)
    rob = ezo.Robot(ctx, desc)
    dev = torch.device("cuda", 0)
    points = []
    qmax = torch.from_numpy(draw.uniform_q_fast(303, max(sizes), data["q_lo"], data["q_hi"])).to(dev)
    for n_obs in (256, 1024, 4096):
        obs = torch.from_numpy(data[f"obstacles_{n_obs}"]).to(dev)
        for n in sizes:
            q = qmax[:n]
            flags = torch.empty(n, dtype=torch.uint8, device=dev)
            msd = torch.empty(n, dtype=torch.float32, device=dev)
            row = {"n": n, "n_obs": n_obs}
            for mode in ("sd", "flags"):
                def run():
                    ezo.check_collisions(ctx, rob, obs, q, flags, msd if mode == "sd" else None)
                run()
                torch.cuda.synchronize()
                reps = max(1, min(args.steps, int(2e8 // n)))
                if reps_cap:
                    reps = min(reps, reps_cap)
                t0 = time.perf_counter()
                for _ in range(reps):
                    run()
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                row[f"{mode}_configs_per_s"] = n / dt
                row[f"{mode}_ms"] = dt * 1e3
                if mode == "sd":
                    fpc = flop_per_check(rob.n_spheres, n_obs, rob.n_self)
                    row["sd_tflops"] = fpc * n / dt / 1e12
                    row["sd_frac"] = row["sd_tflops"] / PEAK_FP32_TFLOPS
                    row["collision_fraction"] = float(flags.float().mean().item())
            points.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orob = oracle.Robot(desc)
        qc = qmax[:1 << 16].cpu().numpy().astype(np.float64)
        cpu = {}
        for n_obs in (256, 1024, 4096):
            ob = data[f"obstacles_{n_obs}"].astype(np.float64)
            t0 = time.perf_counter()
            oracle.check(orob, ob, qc)
            cpu[n_obs] = len(qc) / (time.perf_counter() - t0)
        cores = oracle.max_threads()
        oracle.set_threads(1)
        try:
            t0 = time.perf_counter()
            oracle.check(orob, data["obstacles_4096"].astype(np.float64), qc[:1 << 12])
            one = (1 << 12) / (time.perf_counter() - t0)
        finally:
            oracle.set_threads(cores)
        cpu = {"value": cpu[4096], "unit": "configs/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": "FP64 reference checker (flags and signed distances, all pairs) on the first 65 536 "
                         "configurations at 256 / 1024 / 4096 obstacles; one thread: 4 096 configurations at 4096",
               "configs_per_s_by_obstacles": cpu, "value_1thread": one}
    return points, cpu, ezo.tune_cache_entries()


SWEEP_CONFIG = ("sweep: 7-DOF arm (70 spheres, 1500 self pairs), N uniform configurations in the joint limits, "
                "obstacles in [0.3,1.3]x[-0.5,0.5]x[0,1] m, r U[0.02,0.08]; flags (exact broad phase) and "
                "flags + minimum signed distance (all pairs)")


def sweep(args):
    sizes = [int(x) for x in args.sweep_sizes.split(",")]
    points, cpu, shapes = sweep_measure(args, sizes)
    best = max(points, key=lambda r: r["n"] * (r["n_obs"] == 4096))
    line = {"metric": "collision-checked configs/sec (raw checker sweep, 7-DOF, 70 spheres, 1500 self pairs)",
            "value": best["sd_configs_per_s"], "unit": "configs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic", "config": {"workload": SWEEP_CONFIG}, "points": points, "launch_shapes": shapes}
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def copy_calibration(args):
    """A plain device-to-device copy of 1 GiB (read 1 GiB, write 1 GiB) per
    step: the reference dispatch that scales rocprofv3's FETCH_SIZE and
    WRITE_SIZE counters to bytes."""
    import torch
    n = 1 << 28                                   # float32 elements = 1 GiB
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(max(args.steps, 1)):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": 4 * n, "dispatches": max(args.steps, 1)}), flush=True)


def screen_measure(args, name, epochs):
    """Learned screen: exact self-collision labels of 4 M uniform
    configurations, training, calibration at alpha = 1e-3, then the inflation
    of `name` timed with and without the screen at identical
    eps/delta/tau/seed/N_p.  Returns a dict."""
    import numpy as np
    import torch

    import paper_2504_10783_amd as ezo
    import workloads
    from workloads import draw

    data = workloads.load(name)
    desc = workloads.robot(data)
    if args.tune_import:
        ezo.tune_cache_import(open(args.tune_import).read())
    ctx = ezo.Context(0)
    ctx.set_autotune(not args.no_autotune)
    rob = ezo.Robot(ctx, desc)
    dev = torch.device("cuda", 0)
    n_tr, n_cal, n_te = 3_600_000 // 4096 * 4096, 200_000, 200_000
    alpha = 1e-3
    t0 = time.perf_counter()
    q = torch.from_numpy(draw.uniform_q_fast(404, n_tr + n_cal + n_te, data["q_lo"], data["q_hi"])).to(dev)
    n = q.shape[0]
    flags = torch.empty(n, dtype=torch.uint8, device=dev)
    msd = torch.empty(n, dtype=torch.float32, device=dev)
    lab = torch.empty(n, dtype=torch.float32, device=dev)
    ezo.check_collisions(ctx, rob, torch.zeros((0, 4), dtype=torch.float32, device=dev), q, flags, msd, lab)
    torch.cuda.synchronize()
    t_lab = time.perf_counter() - t0
    sur = ezo.Surrogate(ctx, rob.dof, 256, seed=args.seed)
    tp = ezo.make_train_params(epochs=epochs, batch=4096, lr=1e-3, seed=args.seed)
    t0 = time.perf_counter()
    losses = sur.train(q[:n_tr], lab[:n_tr], tp)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    margin = sur.calibrate(q[n_tr:n_tr + n_cal], lab[n_tr:n_tr + n_cal], alpha)
    miss, frac = sur.miss_rate(q[n_tr + n_cal:], lab[n_tr + n_cal:])
    print(json.dumps({"screen_trained": {"train_s": t_train, "margin": margin, "miss_rate": miss}}),
          file=sys.stderr, flush=True)
    obs = torch.from_numpy(data["obstacles"]).to(dev)
    edges = torch.from_numpy(data["edges"]).to(dev)
    E = edges.shape[0]
    wp = sample_params(args, name)
    if wp["n_p"] == 0:
        # both forms run with the N_p the tuner picks for the exact form
        ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=rob.dof, seed=args.seed, **wp))
        wp["n_p"] = tuned_sample_count(ezo, rob, int(obs.shape[0]))
    res = {}
    for mode in ("exact", "screened", "screened_samples_only"):
        # "screened": the samples after M_k and the bisection midpoints (the
        # default scope); "screened_samples_only": the samples after M_k
        sur.set_scope(samples=True, midpoints=(mode == "screened"))
        prm = ezo.make_params(dof=rob.dof, seed=args.seed, surrogate=None if mode == "exact" else sur, **wp)
        for _ in range(max(args.warmup, 1)):
            ezo.inflate_edges(ctx, rob, obs, edges, prm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        checks = screened = 0
        for _ in range(args.steps):
            r = ezo.inflate_edges(ctx, rob, obs, edges, prm)
            checks += int(r.stats.array["exact_checks"].sum())
            screened += int(r.stats.array["screened_checks"].sum())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        st = r.status.cpu().numpy()
        res[mode] = {"ms_per_step": dt * 1e3, "edges_per_s": E / dt, "configs_per_s": checks / args.steps / dt,
                     "screened_fraction_of_checks": screened / max(checks, 1),
                     "certified": int(np.sum(st == 0)),
                     "iterations_mean": float(np.mean([x["iterations"] for x in r.stats])),
                     "planes_mean": float(np.mean([x["planes"] for x in r.stats]))}
    return {"workload": f"{name}: {WORKLOADS[name]}", "edges": E, "labels": n, "train": n_tr, "calibration": n_cal,
            "test": n_te, "alpha": alpha, "epochs": epochs, "n_p": wp["n_p"],
            "eps": wp["eps"], "delta": wp["delta"], "tau": wp["tau"],
            "speedup_vs_exact": res["screened"]["edges_per_s"] / res["exact"]["edges_per_s"],
            "speedup_vs_exact_samples_only": res["screened_samples_only"]["edges_per_s"] / res["exact"]["edges_per_s"],
            "miss_rate_test": miss, "screened_fraction_test": frac, "margin": margin,
            "label_seconds": t_lab, "train_seconds": t_train,
            "train_samples_per_s": n_tr * epochs / t_train, "epoch_losses": losses, **res}


def screen_compare(args):
    r = screen_measure(args, args.workload, args.screen_epochs)
    if args.tune_export:
        import paper_2504_10783_amd as ezo
        with open(args.tune_export, "w") as f:
            f.write(ezo.tune_cache_export())
    line = {"metric": "edges inflated/sec, learned self-collision screen vs exact (7-DOF)",
            "value": r["screened"]["edges_per_s"], "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 checks, bf16 MFMA screen", "data": "synthetic",
            "config": {"workload": r["workload"], "labels": r["labels"], "train": r["train"],
                       "calibration": r["calibration"], "test": r["test"], "alpha": r["alpha"],
                       "epochs": r["epochs"], "n_p": r["n_p"]}, **r}
    print(json.dumps(line), flush=True)


def recovery(args):
    """Recovery from collisions found on a trajectory (Sec. V-B) on the
    batched workload: the 96 edges inflated for two iterations (loose sets
    that still hold collisions), a trajectory through 8 hit-and-run samples
    of each set in path order, then the three recovery calls timed apart:
    the fine path check (0.01 rad per coordinate), the set update from the
    found collisions, and the containment of the trajectory's segments."""
    import numpy as np
    import torch

    import paper_2504_10783_amd as ezo
    import workloads

    name = "batched"
    data = workloads.load(name)
    desc = workloads.robot(data)
    ctx = ezo.Context(0)
    rob = ezo.Robot(ctx, desc)
    dev = torch.device("cuda", 0)
    obs = torch.from_numpy(data["obstacles"]).to(dev)
    edges = torch.from_numpy(data["edges"]).to(dev)
    E, dof = edges.shape[0], rob.dof
    p = dict(workloads.PARAMS[name], max_iters=2)
    n_f_rec, n_b, per_edge, step = 10, 11, 8, 0.01
    cap = 2 * dof + p["n_f"] * p["max_iters"] + 256
    res0 = ezo.inflate_edges(ctx, rob, obs, edges, ezo.make_params(dof=dof, seed=args.seed, face_capacity=cap, **p))
    smp = torch.empty((E, dof, per_edge), dtype=torch.float32, device=dev)
    ezo.sample_polytopes(ctx, dof, res0.A, res0.b, res0.n_faces, edges, per_edge, p["n_mix"], args.seed + 7, 0, smp)
    way = torch.cat([edges[:, :1, :], smp.transpose(1, 2), edges[:, 1:, :]], dim=1).reshape(-1, dof).contiguous()
    segs = torch.stack([way[:-1], way[1:]], dim=1).contiguous()
    keep = torch.ones(segs.shape[0], dtype=torch.bool, device=dev)
    keep[per_edge + 1::per_edge + 2] = False          # the jumps from one edge's v2 to the next edge's v1
    segs = segs[keep].contiguous()
    work = ezo.InflateResult(res0.A.clone(), res0.b.clone(), res0.n_faces.clone(), res0.status.clone(), [])
    torch.cuda.synchronize()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    found = {}

    def run_check():
        found["pts"], found["n_col"], found["n_pts"] = ezo.check_path(ctx, rob, obs, way, step,
                                                                      point_capacity=64512)

    dt_check = timed(run_check, args.steps)
    pts = found["pts"]

    def restore():
        work.A.copy_(res0.A)
        work.b.copy_(res0.b)
        work.n_faces.copy_(res0.n_faces)
        work.status.copy_(res0.status)

    # the update edits the sets in place: restore them before every call and
    # time the update alone with events on the stream it runs on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    upd_ms = []
    for r in range(args.steps + 1):
        restore()
        ev[0].record()
        added = ezo.update_polytopes(ctx, rob, obs, edges, pts, work, n_b=n_b, n_f=n_f_rec,
                                     step_back_max=p["step_back_max"], t_col=p["t_col"])
        ev[1].record()
        torch.cuda.synchronize()
        if r:
            upd_ms.append(ev[0].elapsed_time(ev[1]))
    cov_before = ezo.segments_contained(ctx, res0.A, res0.b, res0.n_faces, segs)
    dt_cont = timed(lambda: ezo.segments_contained(ctx, work.A, work.b, work.n_faces, segs), args.steps)
    cov_after = ezo.segments_contained(ctx, work.A, work.b, work.n_faces, segs)
    # found collisions still inside some edited set (should be few: the new
    # rows exclude each found point from the set that held it)
    n_keep = pts.shape[0]
    inside = 0
    if n_keep:
        A, b, nf = work.A.cpu().numpy(), work.b.cpu().numpy(), work.n_faces.cpu().numpy()
        P = pts.cpu().numpy()
        for e in range(E):
            s_ = P @ A[e, :nf[e]].T - b[e, :nf[e]]
            inside += int(np.sum(np.all(s_ <= 0.0, axis=1)))
    st = work.status.cpu().numpy()
    line = {"metric": "recovery (Sec. V-B): trajectory configurations checked/sec",
            "value": found["n_pts"] / dt_check, "unit": "configs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"recovery on {name}: {E} sets after {p['max_iters']} iterations, trajectory "
                                   f"through {per_edge} hit-and-run samples per set, step {step} rad; "
                                   f"update N_b={n_b}, N_f={n_f_rec}", "waypoints": int(way.shape[0]),
                       "segments": int(segs.shape[0]), "n_obstacles": int(obs.shape[0]), "n_p": p["n_p"]},
            "path_points": found["n_pts"], "path_check_ms": dt_check * 1e3, "found_collisions": found["n_col"],
            "update_ms": float(np.mean(upd_ms)), "update_ms_min": float(np.min(upd_ms)),
            "planes_added": int(added.sum().item()),
            "edges_edited": int((added > 0).sum().item()),
            "edges_in_collision_after": int(np.sum(st == 2)),
            "found_still_inside_a_set": inside,
            "containment_ms": dt_cont * 1e3, "segments_per_s": segs.shape[0] / dt_cont,
            "segments_covered_before": int((cov_before >= 0).sum().item()),
            "segments_covered_after": int((cov_after >= 0).sum().item())}
    print(json.dumps(line), flush=True)


def paths_compare(args):
    """Sequential path inflation with the containment skip (Sec. V-A) against
    the independent batched form, on the batched workload's 8 paths (96
    edges): time per call and the number of sets built."""
    import numpy as np
    import torch

    import paper_2504_10783_amd as ezo
    import workloads

    name = "batched"
    data = workloads.load(name)
    desc = workloads.robot(data)
    ctx = ezo.Context(0)
    rob = ezo.Robot(ctx, desc)
    dev = torch.device("cuda", 0)
    obs = torch.from_numpy(data["obstacles"]).to(dev)
    e = data["edges"]
    pid = data["path_id"]
    verts, counts = [], []
    for p_ in np.unique(pid):
        ep = e[pid == p_]
        verts.append(np.concatenate([ep[:, 0], ep[-1:, 1]]))
        counts.append(len(ep) + 1)
    V = torch.from_numpy(np.concatenate(verts).astype(np.float32)).to(dev)
    edges = torch.from_numpy(e).to(dev)
    prm = ezo.make_params(dof=desc["dof"], seed=args.seed, **workloads.PARAMS[name])
    res = {}
    for mode in ("independent", "sequential"):
        def run():
            if mode == "sequential":
                return ezo.inflate_paths(ctx, rob, obs, V, counts, prm)
            return ezo.inflate_edges(ctx, rob, obs, edges, prm)
        for _ in range(max(args.warmup, 1)):
            r = run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = r.status.cpu().numpy()
        sets = int(np.sum((st == 0) | (st == 1)))
        res[mode] = {"ms_per_call": dt * 1e3, "sets": sets,
                     "certified": int(np.sum(st == 0)), "contained": int(np.sum(st == 4)),
                     "exact_checks": int(sum(x["exact_checks"] for x in r.stats)),
                     "rows_total": int(r.n_faces.sum().item())}
    line = {"metric": "path inflation (Sec. V-A): sequential with containment skip vs independent, edges/s",
            "value": len(e) / (res["sequential"]["ms_per_call"] * 1e-3), "unit": "edges/s", "n_gpus": 1,
            "steps": args.steps, "warmup": max(args.warmup, 1), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{name}: {WORKLOADS[name]}", "paths": len(counts),
                       "edges_per_path": [c - 1 for c in counts], "n_p": prm.n_p},
            "longest_path_edges": max(counts) - 1,
            "speedup_vs_independent": res["independent"]["ms_per_call"] / res["sequential"]["ms_per_call"],
            **res}
    print(json.dumps(line), flush=True)


def box_sweep(args):
    """Raw checker throughput of the box arm (11 link boxes, 36 box self
    pairs) among 194 voxel spheres and a table box: N uniform configurations,
    flags only and flags + minimum signed distance.  The paper quotes about
    6.9 M configurations/s for its 11-box arm at a batch of 2 M on its own
    GPU (Sec. VI-B, hardware); that scene is not available, so the figure is
    context, not a baseline."""
    import torch

    import paper_2504_10783_amd as ezo
    import workloads
    from workloads import draw

    data = workloads.load("boxes")
    desc = workloads.robot(data)
    ctx = ezo.Context(0)
    rob = ezo.Robot(ctx, desc)
    ctx.set_obstacle_boxes(data["env_boxes"])
    dev = torch.device("cuda", 0)
    obs = torch.from_numpy(data["obstacles"]).to(dev)
    sizes = [int(x) for x in args.sweep_sizes.split(",")]
    qmax = torch.from_numpy(draw.uniform_q_fast(304, max(sizes), data["q_lo"], data["q_hi"])).to(dev)
    points = []
    for n in sizes:
        q = qmax[:n]
        flags = torch.empty(n, dtype=torch.uint8, device=dev)
        msd = torch.empty(n, dtype=torch.float32, device=dev)
        row = {"n": n}
        for mode in ("flags", "sd"):
            def run():
                ezo.check_collisions(ctx, rob, obs, q, flags, msd if mode == "sd" else None)
            run()
            torch.cuda.synchronize()
            reps = max(1, min(args.steps, int(4e8 // n)))
            t0 = time.perf_counter()
            for _ in range(reps):
                run()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            row[f"{mode}_configs_per_s"] = n / dt
            row[f"{mode}_ms"] = dt * 1e3
        row["collision_fraction"] = float(flags.float().mean().item())
        points.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    at2m = min(points, key=lambda r: abs(r["n"] - 2_000_000))
    line = {"metric": "collision-checked configs/sec, box arm (11 boxes) among voxel spheres and a table box",
            "value": at2m["flags_configs_per_s"], "unit": "configs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"boxes raw check: uniform q in joint limits, batch {at2m['n']}; "
                                   f"{WORKLOADS['boxes']}"},
            "paper_context": {"configs_per_s": 6.9e6, "batch": 2_000_000,
                              "hardware": "GeForce RTX 2080 Ti (paper, Sec. VI-B), its own 11-box arm and scene"},
            "points": points,
            "launch_shapes": [e for e in ezo.tune_cache_entries() if e.get("boxes", 0) > 0]}
    print(json.dumps(line), flush=True)


def drm_map(args):
    """DRM collision map (appendix, DRM construction): every voxel of side
    8 cm in [-1.5, 1.5]^2 x [-0.5, 1.5] m (the paper's perception voxels)
    against every node of a 35 000-node roadmap (the paper's hardware
    roadmap size), nodes = self-collision-free uniform configurations of the
    7-DOF sphere arm and of the box arm.  Times the bitset map and its id
    lists."""
    import numpy as np
    import torch

    import paper_2504_10783_amd as ezo
    import workloads
    from workloads import draw

    ctx = ezo.Context(0)
    dev = torch.device("cuda", 0)
    side, lo = 0.08, np.array([-1.5, -1.5, -0.5], np.float32)
    dims = (38, 38, 25)
    V = int(np.prod(dims))
    res = {}
    for name in ("dof7", "boxes"):
        data = workloads.load(name)
        desc = workloads.robot(data)
        rob = ezo.Robot(ctx, desc)
        # nodes: uniform configurations free of self-collision (checked by the
        # library itself before the timed region)
        cand = torch.from_numpy(draw.uniform_q_fast(505, 100_000, data["q_lo"], data["q_hi"])).to(dev)
        flags = torch.empty(cand.shape[0], dtype=torch.uint8, device=dev)
        ezo.check_collisions(ctx, rob, torch.zeros((0, 4), dtype=torch.float32, device=dev), cand, flags)
        q = cand[flags == 0][:35_000].contiguous()
        N = q.shape[0]
        out = torch.empty((V, (N + 31) // 32), dtype=torch.int32, device=dev)
        for _ in range(max(args.warmup, 1)):
            ezo.collision_map(ctx, rob, q, lo, side, dims, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ezo.collision_map(ctx, rob, q, lo, side, dims, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        t1 = time.perf_counter()
        offsets, ids = ezo.collision_map_lists(ctx, out, N)
        torch.cuda.synchronize()
        dl = time.perf_counter() - t1
        res[name] = {"nodes": N, "voxels": V, "map_ms": dt * 1e3, "nodes_per_s": N / dt,
                     "voxel_node_pairs_per_s": V * N / dt, "map_bytes": V * out.shape[1] * 4,
                     "colliding_pairs": int(ids.numel()), "lists_ms": dl * 1e3}
        print(json.dumps({name: res[name]}), file=sys.stderr, flush=True)
    line = {"metric": "DRM collision map: roadmap nodes checked against every voxel per second",
            "value": res["dof7"]["nodes_per_s"], "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
            "warmup": max(args.warmup, 1), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"DRM map: {V} voxels of 8 cm ({dims[0]}x{dims[1]}x{dims[2]}) x 35 000 "
                                   "self-free uniform nodes; 7-DOF sphere arm (70 spheres) and 11-box arm"},
            **res}
    print(json.dumps(line), flush=True)


def forest(args):
    """Forest scene (Sec. VI-A): raw checker throughput at the paper's batch
    of 2 M configurations (the paper quotes about 19.9 M configurations/s on
    its own GPU, appendix), and the inflation of the scene's 4-edge path."""
    import numpy as np
    import torch

    import paper_2504_10783_amd as ezo
    import workloads
    from workloads import draw

    data = workloads.load("forest")
    desc = workloads.robot(data)
    ctx = ezo.Context(0)
    rob = ezo.Robot(ctx, desc)
    dev = torch.device("cuda", 0)
    obs = torch.from_numpy(data["obstacles"]).to(dev)
    n = 2_000_000
    q = torch.from_numpy(draw.uniform_q_fast(606, n, data["q_lo"], data["q_hi"])).to(dev)
    flags = torch.empty(n, dtype=torch.uint8, device=dev)
    msd = torch.empty(n, dtype=torch.float32, device=dev)
    out = {}
    for mode in ("flags", "sd"):
        def run():
            ezo.check_collisions(ctx, rob, obs, q, flags, msd if mode == "sd" else None)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(args.steps, 1)):
            run()
        torch.cuda.synchronize()
        out[f"check_{mode}_configs_per_s"] = n * max(args.steps, 1) / (time.perf_counter() - t0)
    edges = torch.from_numpy(data["edges"]).to(dev)
    E = edges.shape[0]
    prm = ezo.make_params(dof=2, seed=args.seed, **workloads.PARAMS["forest"])
    for _ in range(max(args.warmup, 1)):
        r = ezo.inflate_edges(ctx, rob, obs, edges, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    checks = 0
    for _ in range(args.steps):
        r = ezo.inflate_edges(ctx, rob, obs, edges, prm)
        checks += int(r.stats.array["exact_checks"].sum())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = r.status.cpu().numpy()
    line = {"metric": "Forest scene: collision-checked configs/sec at a batch of 2 M (raw checker, flags)",
            "value": out["check_flags_configs_per_s"], "unit": "configs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": max(args.warmup, 1), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic", "config": {"workload": f"forest: {WORKLOADS['forest']}"},
            "paper_context": {"configs_per_s": 19.9e6, "batch": 2_000_000,
                              "hardware": "GeForce RTX 3090 (paper, appendix), its own Forest instances"},
            **out, "inflate_ms_per_path": dt * 1e3, "edges_per_s": E / dt,
            "inflate_configs_per_s": checks / args.steps / dt,
            "certified": int(np.sum(st == 0)), "edges": E,
            "iterations": [x["iterations"] for x in r.stats], "faces": r.n_faces.cpu().tolist()}
    print(json.dumps(line), flush=True)


def inflation_measure(args, name, plain=True, cpu=True):
    """One workload's inflation measured as bench.py's main line: the timed
    steps (graph replay), a phase pass with dispatch events for the roofline,
    optionally the plain one-call-per-edge form and the paper's N_p (E > 1),
    and the oracle's CPU baseline.  Returns the line as a dict."""
    import numpy as np
    import torch

    import paper_2504_10783_amd as ezo
    import workloads

    data = workloads.load(name)
    desc = workloads.robot(data)
    ctx = ezo.Context(0)
    rob = ezo.Robot(ctx, desc)
    if "env_boxes" in data:
        ctx.set_obstacle_boxes(data["env_boxes"])
    dev = torch.device("cuda", 0)
    obs = torch.from_numpy(data["obstacles"]).to(dev)
    edges = torch.from_numpy(data["edges"]).to(dev)
    E = edges.shape[0]
    samples_mode = sample_mode(args, name)
    wp = sample_params(args, name)
    if args.tune_import:
        ezo.tune_cache_import(open(args.tune_import).read())
    ctx.set_autotune(not args.no_autotune)
    prm = ezo.make_params(dof=desc["dof"], seed=args.seed, **wp)
    out = ezo.InflateResult(torch.empty((E, prm.face_capacity, rob.dof), dtype=torch.float32, device=dev),
                            torch.empty((E, prm.face_capacity), dtype=torch.float32, device=dev),
                            torch.empty(E, dtype=torch.int32, device=dev),
                            torch.empty(E, dtype=torch.int32, device=dev), [])

    def step():
        ezo.inflate_edges(ctx, rob, obs, edges, prm, out=out)
        return out.stats

    # the first call times launch shapes (and, for n_p = 0, the sample count)
    # for this workload when they are not cached yet; it is part of the
    # warm-up, never of the timed steps
    t_first = time.perf_counter()
    for _ in range(max(args.warmup, 1)):
        step()
        torch.cuda.synchronize()
        if t_first is not None:
            first_call_ms = (time.perf_counter() - t_first) * 1e3
            t_first = None
    # timed region: the product path (one replayed hipGraph per iteration)
    checks = samples = 0
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts_ = time.perf_counter()
        st = step().array                 # returns once the call's stream is done
        step_ms.append((time.perf_counter() - ts_) * 1e3)
        checks += int(st["exact_checks"].sum())
        samples += int(st["samples"].sum())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    status = out.status.cpu().numpy()
    n_p_used = wp["n_p"] or tuned_sample_count(ezo, rob, int(obs.shape[0]))
    planes_mean = float(np.mean([s["planes"] for s in out.stats]))
    # phase pass: the same steps with hipEvents between the kernel phases on
    # the library's stream (identical results; kernels launched directly)
    ctx.set_phase_timing(True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt_phase = time.perf_counter() - t1
    phase_ms, iters, tests = ctx.phase_timing(with_tests=True)
    ctx.set_phase_timing(False)

    # Dominant kernel phase.  Algorithmic work = 13 flop per sphere-sphere test
    # the kernel performed (the broad phase skips pairs it proves separated)
    # + FK per configuration checked.
    n_checks = {"check": samples, "bisect": checks - samples}
    dom = max(("check", "bisect"), key=lambda p: phase_ms[p])
    dom_ms = phase_ms[dom]
    work = PAIR_FLOP * tests[dom] + FK_FLOP * n_checks[dom]      # both summed over the K steps
    achieved = work / (dom_ms * 1e-3) / 1e12 if dom_ms > 0 else 0.0
    all_pairs = flop_per_check(rob.n_spheres, obs.shape[0], rob.n_self) * n_checks[dom]
    shapes = timed_shapes(ezo, rob, int(obs.shape[0]), prm, n_p_used, E)
    box = "true" if (rob.n_boxes > 0 or "env_boxes" in data) else "false"
    if dom == "bisect":
        sb = shapes.get("bisect")
        instance = f"ezo::k_project_bisect<{sb['T']}, {sb['depth']}, {box}, false>" if sb else None
    else:
        sc = shapes.get("check_flags")
        instance = f"ezo::k_check<{sc['T']}, false, {box}>" if sc else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": measured_traffic(name, instance, n_p_used) if instance else None,
                "traffic_unit": "bytes per launch (HBM, FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": "k_project_bisect" if dom == "bisect" else "k_check", "kernel_instance": instance,
                "avg_launch_ms": dom_ms / max(iters, 1), "launches": iters,
                "pair_tests_per_check": tests[dom] / max(n_checks[dom], 1),
                "all_pairs_per_check": rob.n_spheres * int(obs.shape[0]) + rob.n_self,
                "box_pair_tests_counted": False if rob.n_boxes > 0 or "env_boxes" in data else None,
                "all_pairs_equivalent_tflops": all_pairs / (dom_ms * 1e-3) / 1e12 if dom_ms > 0 else 0.0}
    if roofline["traffic"] is not None and roofline["avg_launch_ms"] > 0:
        roofline["traffic_gbps"] = roofline["traffic"] / (roofline["avg_launch_ms"] * 1e-3) / 1e9
    counted = measured_valu(name, instance, n_p_used) if instance else None
    if counted is not None and dom_ms > 0:
        # the second form of the FP32 fraction: counted FP32 VALU flop of a
        # launch (committed rocprofv3 summary) over the live average launch time
        ct = counted / (roofline["avg_launch_ms"] * 1e-3) / 1e12
        roofline["counted_fp32"] = {"flop_per_launch": counted, "tflops": ct, "frac": ct / PEAK_FP32_TFLOPS,
                                    "source": f"profiles/valu_fp32__{name}_inflate.md"}

    line = {
        "metric": "collision-checked configs/sec and edges inflated/sec (7-DOF), % FP32 VALU peak",
        "value": checks / dt,
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: {WORKLOADS[name]}", "edges": E, "n_obstacles": int(obs.shape[0]),
                   "robot_spheres": rob.n_spheres, "self_pairs": rob.n_self, "n_p": n_p_used},
        "edges_per_s": E * args.steps / dt,
        "step_ms_p10_p50_p90": [float(np.percentile(step_ms, x)) for x in (10, 50, 90)],
        "checks_per_step": checks // args.steps,
        "iterations_per_step": iters / args.steps,
        "edge_status": {k: int(np.sum(status == v)) for k, v in
                        (("certified", 0), ("max_iters", 1), ("in_collision", 2), ("invalid", 3))},
        "phase_ms_per_step": {k: v / args.steps for k, v in phase_ms.items()},
        "ms_per_step_phase_pass": dt_phase / args.steps * 1e3,
        "roofline": roofline,
        "autotune": not args.no_autotune,
        "n_p": n_p_used,
        "n_p_source": {"tuned": "sample-count tuner (n_p = 0)", "paper": "paper table"}.get(samples_mode, "--samples"),
        "planes_mean": planes_mean,
        "first_call_ms": first_call_ms,
        "launch_shapes": [{k: e[k] for k in ("kernel", "log2_items", "T", "W", "stage", "depth", "us")}
                          for e in shapes.values()],
    }
    if E > 1 and plain:
        # the plain GPU form: the same edges, one call per edge (edge e draws
        # the stream of edge id e in both forms, so the sets are identical),
        # after the timed region
        # the plain form uses the N_p the batched call used (the tuner's pick
        # for n_p = 0), so that both forms compute the same sets
        prm1 = [ezo.make_params(dof=desc["dof"], seed=args.seed, edge_id_base=e, **dict(wp, n_p=n_p_used))
                for e in range(E)]
        outs = [ezo.inflate_edges(ctx, rob, obs, edges[e:e + 1], prm1[e]) for e in range(E)]   # warm-up
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 3))
        t2 = time.perf_counter()
        checks1 = 0
        for _ in range(reps):
            for e in range(E):
                outs[e] = ezo.inflate_edges(ctx, rob, obs, edges[e:e + 1], prm1[e])
                checks1 += outs[e].stats[0]["exact_checks"]
        torch.cuda.synchronize()
        dt1 = (time.perf_counter() - t2) / reps
        same = all(torch.equal(outs[e].n_faces[0], out.n_faces[e]) and torch.equal(outs[e].status[0], out.status[e])
                   and torch.equal(outs[e].A[0, :int(out.n_faces[e])], out.A[e, :int(out.n_faces[e])])
                   for e in range(E))
        line["plain"] = {"ms_per_step": dt1 * 1e3, "edges_per_s": E / dt1, "configs_per_s": checks1 / reps / dt1,
                         "calls_per_step": E, "equal_to_batched": bool(same)}
        line["batched_speedup_vs_plain"] = (E / (dt / args.steps)) / (E / dt1)
    if samples_mode == "tuned" and n_p_used != workloads.PARAMS[name]["n_p"] and plain:
        # the same batched call with the paper's N_p (same eps, delta, tau):
        # what the tuned sample count gains; the sets differ, the certificate
        # does not
        prm_p = ezo.make_params(dof=desc["dof"], seed=args.seed, **workloads.PARAMS[name])
        r = ezo.inflate_edges(ctx, rob, obs, edges, prm_p)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(args.steps):
            r = ezo.inflate_edges(ctx, rob, obs, edges, prm_p)
        torch.cuda.synchronize()
        dt3 = (time.perf_counter() - t3) / args.steps
        st3 = r.status.cpu().numpy()
        line["paper_n_p"] = {"n_p": workloads.PARAMS[name]["n_p"], "ms_per_step": dt3 * 1e3, "edges_per_s": E / dt3,
                             "certified": int(np.sum(st3 == 0)),
                             "iterations_mean": float(np.mean([x["iterations"] for x in r.stats])),
                             "planes_mean": float(np.mean([x["planes"] for x in r.stats]))}
        line["tuned_speedup_vs_paper_n_p"] = dt3 / (dt / args.steps)
    if cpu:
        idx = [0] if E == 1 else sorted({int(np.nonzero(data["path_id"] == p)[0][0]) for p in np.unique(data["path_id"])})
        line["cpu_baseline"] = cpu_baseline(name, data, desc, args.seed, idx, n_p_used)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dof7", choices=sorted(WORKLOADS) + ["sweep"])
    ap.add_argument("--sweep-sizes", default="1048576,4194304,16777216")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the comparison runs after the timed region (one call per edge; the paper's N_p)")
    ap.add_argument("--samples", type=samples_arg, default=None,
                    help="N_p of the inflation: 'paper' (the paper's table value), 'tuned' (chosen by the "
                         "sample-count tuner, n_p = 0) or a count; default tuned for the batched workload, "
                         "paper otherwise")
    ap.add_argument("--screen", action="store_true", help="learned screen vs exact comparison")
    ap.add_argument("--screen-epochs", type=int, default=10)
    ap.add_argument("--recovery", action="store_true", help="trajectory check + set update + containment timings")
    ap.add_argument("--paths", action="store_true", help="sequential path inflation vs independent edges")
    ap.add_argument("--box-sweep", action="store_true", help="raw checker throughput of the box arm")
    ap.add_argument("--drm-map", action="store_true", help="DRM collision map of a 35 000-node roadmap")
    ap.add_argument("--forest", action="store_true", help="Forest scene: raw checker and path inflation")
    ap.add_argument("--no-autotune", action="store_true", help="size-heuristic launch shapes (no tuning)")
    ap.add_argument("--tune-import", default=None,
                    help="JSON-lines tuning cache to load before the run (profiled runs replay the shapes and "
                         "sample count an unprofiled run picked; timing under a profiler distorts the tuner)")
    ap.add_argument("--tune-export", default=None, help="write the tuning cache after the run")
    ap.add_argument("--no-extras", action="store_true",
                    help="dof7: only the main line (no batched / sweep / screen sub-objects)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the EI-ZO path of this library runs on a single MI355X "
              "(edges shard across GPUs with no exchange; multi-GPU runs are not part of this build)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.workload == "sweep":
        sweep(args)
        return
    if args.screen:
        screen_compare(args)
        return
    if args.recovery:
        recovery(args)
        return
    if args.paths:
        paths_compare(args)
        return
    if args.box_sweep:
        box_sweep(args)
        return
    if args.drm_map:
        drm_map(args)
        return
    if args.forest:
        forest(args)
        return

    name = args.workload
    line = inflation_measure(args, name, plain=not args.no_plain, cpu=not args.no_cpu_baseline)
    if name == "dof7" and not args.no_extras:
        # the other configurations the metric is quoted on, as sub-objects of
        # the same line: the batched workload (with the plain form and its own
        # roofline), the raw checker sweep at 16 M configurations, and the
        # learned screen against the exact form
        print(json.dumps({"progress": "dof7 done", "ms_per_step": line["ms_per_step"]}), file=sys.stderr, flush=True)
        line["batched"] = inflation_measure(args, "batched", plain=True, cpu=not args.no_cpu_baseline)
        for k in ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data", "dtype"):
            line["batched"].pop(k, None)
        print(json.dumps({"progress": "batched done", "edges_per_s": line["batched"]["edges_per_s"]}),
              file=sys.stderr, flush=True)
        points, cpu, _ = sweep_measure(args, [1 << 24], reps_cap=3)
        line["sweep"] = {"config": SWEEP_CONFIG, "points": points}
        if cpu is not None:
            line["sweep"]["cpu_baseline"] = cpu
        print(json.dumps({"progress": "sweep done"}), file=sys.stderr, flush=True)
        line["screen"] = screen_measure(args, "batched", args.screen_epochs)
    if args.tune_export:
        with open(args.tune_export, "w") as f:
            f.write(__import__("paper_2504_10783_amd").tune_cache_export())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
