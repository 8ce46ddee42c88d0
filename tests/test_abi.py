"""The C ABI without a GPU: libgt.so loads, exports every function that
include/gt.h declares, and the binding's ctypes structs have the C layout.

No call here touches the device: only gt_version (a constant string),
gt_last_error (thread-local text) and gt_build_graph with arguments it
rejects before any device work are called.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)          # drop comments
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_]\w*\s*\**\s+\**\s*(gt_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2009_07463_amd as gt
    return gt.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gt_build_graph", "gt_bfs", "gt_bfs_batch", "gt_graph_destroy", "gt_last_error"):
        assert must in names
    assert len(names) >= 17


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, "declared in gt.h but not exported: %s" % missing


def test_version_and_error_without_device(lib):
    assert b"gfx950" in lib.gt_version()
    assert isinstance(lib.gt_last_error(), bytes)


def test_build_rejects_bad_flags_before_device_work(lib):
    import paper_2009_07463_amd as gt
    h = ctypes.c_void_p()
    for flags in (gt.GT_BUILD_KEEP_LEAVES, 4, 1 << 31, 1 << 20, gt.GT_BUILD_SPLIT | gt.GT_BUILD_HUB_SHARE(3),
                  gt.GT_BUILD_KEEP_ZERO, gt.GT_BUILD_SPLIT | gt.GT_BUILD_KEEP_ZERO,
                  gt.GT_BUILD_RELABELLED | gt.GT_BUILD_MH(1)):
        assert lib.gt_build_graph(None, None, 0, 4, flags, None, ctypes.byref(h)) == gt.GT_E_INVALID
        assert not h.value
        msg = lib.gt_last_error()
        assert b"flags" in msg or b"GT_BUILD_" in msg, msg


def test_struct_layouts_match_the_header():
    import paper_2009_07463_amd as gt
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "gt.h"
#define S(t) printf(#t " %zu\n", sizeof(t))
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f))
int main(void) {
    S(gt_graph_info); O(gt_graph_info, build_ms); O(gt_graph_info, flags);
    S(gt_level_stats); O(gt_level_stats, frontier); O(gt_level_stats, ms); O(gt_level_stats, ms_main);
    O(gt_level_stats, examined_long); O(gt_level_stats, found_long);
    S(gt_run_stats); O(gt_run_stats, ms_total); O(gt_run_stats, level);
    S(gt_tuning); O(gt_tuning, timing); O(gt_tuning, bu_hint); O(gt_tuning, loop); O(gt_tuning, td_hub_deg);
    O(gt_tuning, ms_alpha); O(gt_tuning, bu_gamma); O(gt_tuning, ms_loop); O(gt_tuning, bu_lds); O(gt_tuning, bu_form); O(gt_graph_info, tree_height); O(gt_graph_info, n_core_edge);
    O(gt_graph_info, n_edge_trees); O(gt_graph_info, edge_tree_min);
    S(gt_tune_report); O(gt_tune_report, from_cache); O(gt_tune_report, ms_start); O(gt_tune_report, ms_batch_best);
    S(gt_device_props); O(gt_device_props, compute_units); O(gt_device_props, l2_bytes);
    O(gt_device_props, peak_hbm_gbs);
    return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    c_layout = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    py = {"gt_graph_info": gt.GraphInfo, "gt_level_stats": gt.LevelStats, "gt_run_stats": gt.RunStats,
          "gt_tuning": gt.Tuning, "gt_tune_report": gt.TuneReport, "gt_device_props": gt.DeviceProps}
    for key, val in c_layout.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(py[t], f).offset == int(val), key
        else:
            assert ctypes.sizeof(py[key]) == int(val), key
