"""CPU-only checks of the C ABI: the library loads, exports every entry point
declared in include/ezo.h, and its host-side helpers agree with the oracle.
No compute call is made here (no GPU in this environment)."""
import os
import re
import subprocess

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ezo.h")


@pytest.fixture(scope="module")
def ezo():
    import paper_2504_10783_amd as ezo
    if not os.path.exists(ezo.LIB_PATH):
        from paper_2504_10783_amd import build
        build.build()
    ezo.lib()
    return ezo


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ezo_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("ezo_check_collisions", "ezo_inflate_edges", "ezo_ctx_create", "ezo_robot_create",
              "ezo_sample_polytopes", "ezo_project_bisect", "ezo_place_hyperplanes", "ezo_test_and_select"):
        assert n in names


def test_every_declared_symbol_is_exported(ezo):
    out = subprocess.check_output(["nm", "-D", "--defined-only", ezo.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    assert set(ezo.EXPORTS) <= set(declared_functions())


def test_library_carries_gfx950_code_object(ezo):
    blob = open(ezo.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_test_constants_match_oracle(ezo):
    for eps, delta, tau in ((0.1, 0.05, 0.5), (0.05, 0.05, 0.5), (0.005, 0.005, 0.5), (0.01, 0.05, 0.3)):
        for k in range(1, 60):
            assert ezo.test_constants(eps, delta, tau, k) == oracle.test_constants(eps, delta, tau, k)


def test_test_constants_reject_bad_arguments(ezo):
    with pytest.raises(ezo.EzoError):
        ezo.test_constants(0.0, 0.05, 0.5, 1)
    with pytest.raises(ezo.EzoError):
        ezo.test_constants(0.1, 0.05, 0.5, 0)


TUNE_LINE = ('{"arch":"gfx950","kernel":"bisect","dof":7,"spheres":70,"self_pairs":1500,"obstacles":512,'
             '"log2_items":13,"T":16,"W":4,"stage":1,"us":93.5}')


def test_tuning_cache_roundtrip_on_host(ezo):
    """The launch-shape cache is host state: import, export, clear."""
    ezo.tune_cache_clear()
    assert ezo.tune_cache_export() == ""
    extra = TUNE_LINE.replace('"bisect"', '"check_sd"').replace('"T":16', '"T":64')
    assert ezo.tune_cache_import(TUNE_LINE + "\n" + extra + "\n") == 2
    ents = ezo.tune_cache_entries()
    assert len(ents) == 2
    by_kernel = {e["kernel"]: e for e in ents}
    assert by_kernel["bisect"]["T"] == 16 and by_kernel["bisect"]["stage"] == 1
    assert by_kernel["check_sd"]["T"] == 64 and by_kernel["bisect"]["obstacles"] == 512
    assert by_kernel["bisect"]["depth"] == 1                # optional on import, default 1
    assert ezo.tune_cache_import(TUNE_LINE.replace('"us"', '"depth":2,"us"')) == 1
    assert {e["kernel"]: e for e in ezo.tune_cache_entries()}["bisect"]["depth"] == 2
    # re-import of an exported text is the identity
    text = ezo.tune_cache_export()
    ezo.tune_cache_clear()
    assert ezo.tune_cache_import(text) == 2 and ezo.tune_cache_export() == text
    # a sample-count entry keeps any count as T; a box robot's key its boxes
    cnt = TUNE_LINE.replace('"bisect"', '"samples"').replace('"T":16', '"T":5000').replace('"W":4', '"W":1')
    box = TUNE_LINE.replace('"self_pairs":1500,', '"self_pairs":0,"boxes":11,')
    assert ezo.tune_cache_import(cnt + "\n" + box) == 2
    ents = ezo.tune_cache_entries()
    assert any(e["kernel"] == "samples" and e["T"] == 5000 for e in ents)
    assert any(e.get("boxes") == 11 for e in ents) and len(ents) == 4
    ezo.tune_cache_clear()
    assert ezo.tune_cache_entries() == []


@pytest.mark.parametrize("bad", [
    TUNE_LINE.replace('"T":16', '"T":12'),              # tile size not a power of two
    TUNE_LINE.replace('"W":4', '"W":17'),               # more than 16 waves
    TUNE_LINE.replace('"bisect"', '"gemm"'),            # unknown kernel
    TUNE_LINE.replace('"stage":1,', ''),                # missing key
    TUNE_LINE.replace('"us"', '"depth":0,"us"'),        # depth below 1
    TUNE_LINE.replace('"us"', '"depth":4,"us"'),        # depth beyond 3
    TUNE_LINE.replace('"bisect"', '"samples"').replace('"T":16', '"T":0'),   # no samples
])
def test_tuning_cache_rejects_malformed_lines(ezo, bad):
    ezo.tune_cache_clear()
    with pytest.raises(ezo.EzoError):
        ezo.tune_cache_import(TUNE_LINE + "\n" + bad)
    assert ezo.tune_cache_entries() == []               # nothing imported from a rejected text


def test_edge_stats_view_reads_the_c_array(ezo):
    """The per-edge statistics of a call are a view of the C array the
    library filled: dicts on access (indices, negative indices, slices),
    equality with a list of dicts, and a zero-copy numpy view with the C
    struct's layout."""
    import ctypes as C
    arr = (ezo.EdgeStats * 3)()
    arr[0].iterations, arr[0].exact_checks = 2, 10
    arr[2].planes, arr[2].exact_checks, arr[2].screened_checks = 7, 30, 4
    v = ezo.EdgeStatsView(arr, 3)
    assert len(v) == 3 and v[0]["iterations"] == 2 and v[-1]["planes"] == 7
    assert [d["exact_checks"] for d in v] == [10, 0, 30]
    assert v[1:] == [v[1], v[2]] and v == list(v)
    with pytest.raises(IndexError):
        v[3]
    a = v.array
    assert a.dtype.itemsize == C.sizeof(ezo.EdgeStats)
    assert int(a["exact_checks"].sum()) == 40 and int(a["screened_checks"][2]) == 4
    arr[1].samples = 5                                   # a view, not a copy
    assert int(a["samples"][1]) == 5
    assert len(ezo.EdgeStatsView(arr, 0).array) == 0
