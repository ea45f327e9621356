"""CPU checks of bench.py's measurement plumbing: the N_p options, the
choice of the tuning entries a timed call used (the check keyed on
max_k max(N_p, M_k) samples per edge, the bisection on N_p candidate slots
per edge), and the rule that a committed HBM / VALU summary is used only
for the same kernel sources, N_p and kernel instance."""
import argparse
import json
import os
import re
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.fixture(scope="module")
def ezo():
    import paper_2504_10783_amd as ezo
    if not os.path.exists(ezo.LIB_PATH):
        from paper_2504_10783_amd import build
        build.build()
    ezo.lib()
    return ezo


def test_samples_option():
    assert bench.samples_arg("paper") == "paper" and bench.samples_arg("tuned") == "tuned"
    assert bench.samples_arg("2000") == 2000
    for bad in ("0", "-5", "many"):
        with pytest.raises(argparse.ArgumentTypeError):
            bench.samples_arg(bad)
    args = SimpleNamespace(samples=None)
    assert bench.sample_mode(args, "batched") == "tuned" and bench.sample_mode(args, "dof7") == "paper"
    assert bench.sample_params(args, "batched")["n_p"] == 0
    assert bench.sample_params(args, "dof7")["n_p"] == 10000
    assert bench.sample_params(SimpleNamespace(samples=1234), "dof7")["n_p"] == 1234


def line(kernel, log2_items, T, obstacles=2048, spheres=70):
    return json.dumps({"arch": "gfx950", "kernel": kernel, "dof": 7, "spheres": spheres, "self_pairs": 1500,
                       "obstacles": obstacles, "log2_items": log2_items, "T": T, "W": 4, "stage": 0, "depth": 1,
                       "us": 1.0})


def test_timed_shapes_pick_the_call_keys(ezo):
    """E = 96 edges at N_p = 1000 (eps 0.05, delta 0.05, 50 iterations):
    the check holds max_k M_k = M_50 samples per edge (M_k > N_p from the
    fourth iteration on), the bisection N_p candidate slots per edge."""
    prm = ezo.make_params(dof=7, seed=0, eps=0.05, delta=0.05, tau=0.5, n_p=1000, max_iters=50)
    m50 = ezo.test_constants(0.05, 0.05, 0.5, 50)[0]
    assert m50 > 1000
    want_check = (m50 * 96).bit_length() - 1
    want_bisect = (1000 * 96).bit_length() - 1
    ezo.tune_cache_clear()
    try:
        text = "\n".join([line("check_flags", want_check, 8), line("check_flags", want_check - 1, 16),
                          line("bisect", want_bisect, 16), line("bisect", want_bisect + 3, 32),
                          line("bisect", want_bisect, 64, obstacles=512), line("bisect", want_bisect, 2, spheres=12)])
        assert ezo.tune_cache_import(text) == 6
        rob = SimpleNamespace(dof=7, n_spheres=70)
        got = bench.timed_shapes(ezo, rob, 2048, prm, 1000, 96)
        assert got["check_flags"]["T"] == 8 and got["check_flags"]["log2_items"] == want_check
        assert got["bisect"]["T"] == 16 and got["bisect"]["log2_items"] == want_bisect
        assert bench.timed_shapes(ezo, rob, 4096, prm, 1000, 96) == {}
    finally:
        ezo.tune_cache_clear()


def test_tuned_sample_count_needs_one_entry(ezo):
    rob = SimpleNamespace(dof=7, n_spheres=70)
    ezo.tune_cache_clear()
    try:
        with pytest.raises(RuntimeError):
            bench.tuned_sample_count(ezo, rob, 2048)
        assert ezo.tune_cache_import(line("samples", 6, 2000).replace('"W": 4', '"W": 1')) == 1
        assert bench.tuned_sample_count(ezo, rob, 2048) == 2000
    finally:
        ezo.tune_cache_clear()


def test_committed_summaries_match_only_their_own_run():
    """Each committed HBM / VALU summary names the instances it measured and
    the N_p of its run; any other instance or N_p gets no figure."""
    for w in ("dof7", "batched"):
        text = open(os.path.join(ROOT, "profiles", f"hbm_traffic__{w}_inflate.md")).read()
        rec = json.loads(next(l for l in text.splitlines() if l.startswith("traffic-json: "))[len("traffic-json: "):])
        inst = next(k for k in rec["bytes_per_launch_by_instance"] if "k_project_bisect" in k)
        if rec["source_sha256"] == bench.kernel_source_sha256():
            assert bench.measured_traffic(w, inst, rec["n_p"]) == rec["bytes_per_launch_by_instance"][inst]
            assert bench.measured_valu(w, inst, rec["n_p"]) is not None
        assert bench.measured_traffic(w, inst, rec["n_p"] + 1) is None
        assert bench.measured_traffic(w, "ezo::k_project_bisect<3, 9, false>", rec["n_p"]) is None
        assert bench.measured_valu(w, inst, rec["n_p"] + 1) is None


def test_committed_summaries_have_per_launch_rows():
    """Every per-launch summary of the two inflation workloads lists the
    bisection among its rows, and the trace splits its dispatches into the
    bench's calls (one warm-up, then as many timed as phase-timed)."""
    for w in ("dof7", "batched"):
        for kind in ("hbm_traffic", "valu_fp32", "stall", "kernel_trace"):
            text = open(os.path.join(ROOT, "profiles", f"{kind}__{w}_inflate.md")).read()
            rows = [l for l in text.splitlines() if l.startswith("| ") and "k_project_bisect" in l]
            assert rows, (kind, w)
        text = open(os.path.join(ROOT, "profiles", f"kernel_trace__{w}_inflate.md")).read()
        m = re.search(r"\((\d+) inflation calls: 1 warm-up, (\d+) timed graph replays, (\d+) phase-timed\)", text)
        assert m and int(m.group(2)) > 0 and int(m.group(2)) == int(m.group(3)) and int(m.group(1)) == 1 + 2 * int(m.group(2))
