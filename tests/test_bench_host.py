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
    # traversal byte model of a bottom-up level over n vertices: both
    # bitmaps, 8 B of row offsets per tested vertex, the 4-byte entry and its
    # bit probe per examined entry, level and parent per discovery
    assert bench.bu_model_bytes(640, 3, 5, 2) == 2 * 640 / 8 + 8 * 3 + 4.125 * 5 + 8 * 2
    # the layout: 16 B per bitmap word, hint + degree per tested vertex,
    # entry + probe, pair + parent caller id per discovery
    assert bench.bu_layout_bytes(10, 3, 5, 2) == 16 * 10 + 8 * 3 + 4.125 * 5 + 12 * 2
    # fused pull: 24 B per vertex (32 when the step also pushed), 4-byte hint,
    # 4-byte entry + 8-byte mask per examined entry, level bytes
    assert bench.ms_pull_bytes(100, 7, 9, False) == 24 * 100 + 4 * 100 + 12 * 7 + 9
    assert bench.ms_pull_bytes(100, 7, 9, True) == 32 * 100 + 4 * 100 + 12 * 7 + 9
    assert np.isfinite(bench.HBM_PEAK_GBS) and bench.HBM_PEAK_GBS == 8000.0


def test_core_numbering_and_tree_table():
    assert bench.core_numbering(True, 2) == "hubs first (at most n_core / 2^2)"
    assert bench.core_numbering(False, 2) == "caller order"
    info = {"n_edge_trees": 4, "edge_tree_vertices": 10, "edge_tree_max": 5, "edge_tree_min": 1}
    assert bench.tree_table(info) == {"trees": 4, "average": 2.5, "max": 5, "min": 1, "total": 10}
    info = {"n_edge_trees": 0, "edge_tree_vertices": 0, "edge_tree_max": 0, "edge_tree_min": 0}
    assert bench.tree_table(info)["average"] == 0


def test_oracle_summary_and_cpu_info():
    res = {"seconds": [1.0, 2.0], "edges": [2e9, 2e9], "build_s": 3.0, "roots": [5, 6]}
    out = bench.oracle_summary(res, 26, "2 roots")
    assert abs(out["value"] - bench.hmean([2.0, 1.0])) < 1e-4
    assert out["cores"] == 1 and out["kind"] == "oracle" and out["roots"] == 2
    assert out["nproc"] >= 1 and out["usable_cpus"] >= 1 and isinstance(out["cpu_model"], str)


def test_oracle_worker_times_roots_and_keeps_levels():
    import graphgen
    import oracle
    n = 1 << 10
    src, dst = graphgen.kronecker_edges(10, 16, seed=3)
    roots = graphgen.sample_roots(n, src, dst, 3, seed=4)
    w = bench.OracleWorker()
    w.start()
    w.add("t", n, src, dst, roots)
    w.finish()
    w.join(60)
    res = w.results["t"]
    g = oracle.build_csr(n, src, dst)
    for r, lv, m in zip(roots, res["levels"], res["edges"]):
        np.testing.assert_array_equal(lv, oracle.bfs(g, int(r))[1])
        assert m == oracle.reached_edges(g, lv)
    assert len(res["seconds"]) == 3 and all(t > 0 for t in res["seconds"])


def test_kernel_hash_ignores_comments_only():
    src = "int a = 1; // why\n/* a block\n   comment */\nint b = 2;\n\n"
    assert bench.code_text(src) == "int a = 1;\nint b = 2;"
    assert bench.code_text(src.replace("why", "because")) == bench.code_text(src)
    assert bench.code_text(src.replace("2", "3")) != bench.code_text(src)


def test_single_root_hub_share_fits_the_lds_hub_frontier():
    # n_core / 2^k hubs: 1/4 at scale 22, 1/64 at scale 26 (the hub class of
    # a Kronecker core at edgefactor 16 then holds under 512 K hubs, which is
    # what one workgroup's 64 KB of LDS holds as bits); --hub-share wins
    class A:
        hub_share = None
    for scale, k in ((16, 2), (22, 2), (24, 4), (26, 6)):
        A.scale = scale
        assert bench.hub_share_for(A) == k
    A.hub_share = 3
    assert bench.hub_share_for(A) == 3
    assert bench.GT_LOOP_NAMES == {1: "host", 2: "graph", 3: "device"}
