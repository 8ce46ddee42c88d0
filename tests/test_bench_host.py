"""Host-side logic of bench.py (no GPU): the profile summaries it reads, the
one-GPU refusal and its arithmetic helpers."""
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_profile_fields_keep_colons_inside_keys(tmp_path):
    p = tmp_path / "p.md"
    p.write_text("# title\n- kernel source sha256[:16]: `0123456789abcdef`\n"
                 "- hbm bytes per launch (scaled): `42`\n- note without value\n")
    vals = bench.read_profile_fields(str(p))
    assert vals["kernel source sha256[:16]"] == "0123456789abcdef"
    assert vals["hbm bytes per launch (scaled)"] == "42"
    assert len(vals) == 2


def test_committed_traffic_profile_is_read_only_for_its_source():
    path = os.path.join(ROOT, "profiles", "k_bu_traffic_scale26.md")
    vals = bench.read_profile_fields(path)
    sha = vals["kernel source sha256[:16]"]
    assert re.fullmatch(r"[0-9a-f]{16}", sha)
    hbm = float(vals["hbm bytes per launch (scaled)"])
    assert hbm > float(vals["algorithmic bytes per launch"]) > 0
    numbering = vals["split core numbering"]
    assert numbering.startswith("hubs first") or numbering == "caller order"
    got = bench.read_traffic_profile(26, numbering)
    if sha == bench.kernel_source_sha():
        assert got == hbm
    else:
        assert got is None
    assert bench.read_traffic_profile(26, numbering + " (another)") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_harmonic_mean_and_byte_models():
    assert abs(bench.hmean([1.0, 2.0, 4.0]) - 3.0 / (1 + 0.5 + 0.25)) < 1e-12
    # bottom-up: 16 B per bitmap word, e + 8 per tested vertex, e + 1/8 per
    # examined entry, 8 per discovery (SPLIT entries: e = 8)
    assert bench.bu_bytes(10, 3, 5, 2, 8) == 16 * 10 + 16 * 3 + 8.125 * 5 + 8 * 2
    # fused pull: 24 B per vertex (32 when the step also pushed), hint, entries, level bytes
    assert bench.ms_pull_bytes(100, 7, 9, False, 8, 8) == 24 * 100 + 8 * 100 + 16 * 7 + 9
    assert bench.ms_pull_bytes(100, 7, 9, True, 8, 8) == 32 * 100 + 8 * 100 + 16 * 7 + 9
    assert np.isfinite(bench.HBM_PEAK_GBS) and bench.HBM_PEAK_GBS == 8000.0


def test_core_numbering_and_tree_table():
    class A:
        hubs_first = True
        hub_share = 2
    assert bench.core_numbering(A) == "hubs first (at most n_core / 2^2)"
    A.hubs_first = False
    assert bench.core_numbering(A) == "caller order"
    info = {"n_edge_trees": 4, "edge_tree_vertices": 10, "edge_tree_max": 5, "edge_tree_min": 1}
    assert bench.tree_table(info) == {"trees": 4, "average": 2.5, "max": 5, "min": 1, "total": 10}
    info = {"n_edge_trees": 0, "edge_tree_vertices": 0, "edge_tree_max": 0, "edge_tree_min": 0}
    assert bench.tree_table(info)["average"] == 0
