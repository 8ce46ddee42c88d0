"""Benchmark: low-degree-split BFS vs plain direction-optimizing BFS on one MI355X.

Default workload: Kronecker graph, scale 26, edgefactor 16 (Graph500
initiator A=.57, B=C=.19, D=.05; 67,108,864 vertices, 1,073,741,824 generated
edges), 64 seeded roots of degree >= 1 run one at a time, as in Section 6.1
of the paper. One step = the 64 roots through gt_bfs on the SPLIT handle.
The metric is Graph500-style: per root, m_r = half the degree sum of the
reached vertices (the traversed undirected edges), t_r = wall time of the
gt_bfs call (output init, root handling, core BFS, leaf pass, id translation);
the headline value is the harmonic mean of m_r / t_r over all timed roots.
The PLAIN handle (same kernels on the whole graph) is timed the same way.

Also printed in the same JSON line:
  roofline      bottom-up kernel, algorithmic bytes per launch / event-timed
                launch duration, against 8 TB/s HBM;
  cpu_baseline  the CPU oracle (single thread) on one root of the same graph,
                timed on this host; its levels are also compared with the GPU's.
Other modes: --mode batch (64-root batched BFS vs 64 single runs, scale 24)
and --mode serve (continuous-batching server over scales 18-24).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
METRIC = "harmonic-mean GTEPS at scale 26 (split vs plain BFS); p50/p99 query latency"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def hmean(x):
    x = np.asarray(x, dtype=np.float64)
    return float(len(x) / np.sum(1.0 / x))


# Algorithmic bytes of one bottom-up launch (one BFS level on n vertices):
# visited word read + next word written per 64 vertices (16 B / word); per
# tested (unvisited) vertex its highest-degree-neighbour entry (e B) and row
# offsets (8 B; consecutive lanes share one boundary); per adjacency entry
# examined, the entry (e B) and its bitmap probe (1/8 B); per discovered
# vertex its level and parent (8 B). e = 4 B (PLAIN: caller id) or 8 B
# (SPLIT: core id + caller id).
def bu_bytes(words, scanned, examined, found, e):
    return 16.0 * words + (e + 8.0) * scanned + (e + 0.125) * examined + 8.0 * found


def kernel_source_sha():
    """Hash of the sources of the bottom-up kernel (its body and the
    host-driven loop that launches it)."""
    h = hashlib.sha256()
    for name in ("bfs_kernels.h", "bfs.hip"):
        with open(os.path.join(ROOT, "paper_2009_07463_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_profile_fields(path):
    """The `- key: value` lines of a profile summary (keys may hold colons,
    as in `sha256[:16]`; the separator is colon-space)."""
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    return vals


def core_numbering(args):
    """How the split handles number their core (recorded with each result)."""
    if not args.hubs_first:
        return "caller order"
    return "hubs first (at most n_core / 2^%d)" % args.hub_share


def read_traffic_profile(scale, numbering):
    """HBM bytes per bottom-up launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and on a split
    handle of the same core numbering (the traffic depends on both)."""
    path = os.path.join(ROOT, "profiles", "k_bu_traffic_scale%d.md" % scale)
    if not os.path.exists(path):
        return None
    vals = read_profile_fields(path)
    if vals.get("kernel source sha256[:16]") != kernel_source_sha():
        return None
    if vals.get("split core numbering") != numbering:
        return None
    try:
        return float(vals["hbm bytes per launch (scaled)"])
    except (KeyError, ValueError):
        return None


class OracleBaseline(threading.Thread):
    """CPU oracle on one root of the same graph, in the background: builds its
    own CSR (untimed), then times one FIFO BFS (single thread)."""

    def __init__(self, n, src, dst, root):
        super().__init__(daemon=True)
        self.n, self.src, self.dst, self.root = n, src, dst, int(root)
        self.result = None
        self.levels = None
        self.error = None

    def run(self):
        try:
            import oracle
            t0 = time.perf_counter()
            g = oracle.build_csr(self.n, self.src, self.dst)
            t_build = time.perf_counter() - t0
            t0 = time.perf_counter()
            _, lvl = oracle.bfs(g, self.root)
            t = time.perf_counter() - t0
            m = oracle.reached_edges(g, lvl)
            self.levels = lvl
            self.result = dict(value=m / t / 1e9, unit="GTEPS", cores=1, kind="oracle",
                               sample="1 of the 64 roots (root %d) on the same scale-%d graph; "
                                      "single-thread FIFO BFS, its own CSR build (%.0f s) untimed"
                                      % (self.root, int(np.log2(self.n)), t_build),
                               seconds=t, traversed_edges=m)
            del g
        except Exception as e:  # reported, never fatal to the GPU numbers
            self.error = repr(e)


def make_graph(scale, edgefactor, seed):
    import graphgen
    n = 1 << scale
    t0 = time.perf_counter()
    src, dst = graphgen.kronecker_edges(scale, edgefactor, seed=seed)
    log("generated %d edges in %.1f s" % (src.size, time.perf_counter() - t0))
    return n, src, dst


def run_single(args):
    import torch
    import graphgen
    import paper_2009_07463_amd as gt

    gt.load_library(build_if_missing=True)
    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        # a plain elementwise kernel of known traffic (reads and writes
        # copy_calibration_mib MiB each) for scaling hardware byte counters
        a = torch.ones(args.copy_calibration_mib << 18, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
    n, src, dst = make_graph(args.scale, args.edgefactor, args.seed)
    roots = graphgen.sample_roots(n, src, dst, args.roots, seed=args.root_seed)
    log("roots sampled")
    base = None
    if args.cpu_baseline:
        base = OracleBaseline(n, src, dst, roots[0])
        base.start()
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    torch.cuda.synchronize()
    handles = {}
    infos = {}
    variants = [("split", True, False, 0), ("plain", False, False, 0)]
    if args.rmzero:
        variants.append(("rmzero", True, True, 0))  # ablation: only isolated vertices removed
    for mh in args.mh:
        variants.append(("mh%d" % mh, True, False, mh))  # edge trees of height <= mh (Algorithm 8)
    names = [v[0] for v in variants]
    for name, split, rmzero, mh in variants:
        # every handle of the split machinery numbers its hubs first (the
        # plain handle has no relabelling)
        g = gt.Graph(s, d, n, split=split, rmzero=rmzero, mh=mh, hubs_first=split and args.hubs_first,
                     hub_share=args.hub_share)
        handles[name] = g
        infos[name] = g.info()
        log("%s build %.0f ms, %.2f GB" % (name, infos[name]["build_ms"], infos[name]["device_bytes"] / 1e9))
    del s, d
    torch.cuda.empty_cache()
    deg = handles["plain"].degrees()
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    level = torch.empty(n, dtype=torch.int32, device="cuda")

    # traversed edges per root (untimed; identical for both variants)
    m_r = []
    root0_split_levels = None
    for i, r in enumerate(roots):
        handles["split"].bfs(int(r), parent, level)
        m_r.append(int(deg[level >= 0].to(torch.int64).sum().item()) // 2)
        if i == 0:
            root0_split_levels = level.cpu().numpy()
    m_r = np.asarray(m_r, dtype=np.float64)

    loop = {"auto": 0, "host": gt.GT_LOOP_HOST, "graph": gt.GT_LOOP_GRAPH, "device": gt.GT_LOOP_DEVICE}[args.loop]
    # knobs: autotuned on a separate sample of roots (not the timed ones)
    tune_roots = graphgen.sample_roots(n, src, dst, 64, seed=args.root_seed + 100)
    tuned = {}
    for name in names:
        if loop == 0:
            t0 = time.perf_counter()
            tun, rep = handles[name].autotune(tune_roots, cache_path=args.tune_cache)
            rep["seconds"] = round(time.perf_counter() - t0, 2)
            tuned[name] = {"knobs": {k: tun[k] for k in ("loop", "graph_levels", "alpha", "beta", "bu_blocks",
                                                            "bu_lane_edges", "bu_hub_deg", "bu_hub_blocks",
                                                            "td_small_edges", "td_blocks", "td_hub_deg", "bu_hint")},
                           "report": rep}
            log("%s autotuned in %.1f s: %s" % (name, rep["seconds"], tuned[name]["knobs"]))
        else:
            handles[name].set_tuning(loop=loop)
    results = {}
    for name in names:
        g = handles[name]
        # timed pass: the chosen level loop, no per-level events
        g.set_tuning(timing=0)
        for _ in range(args.warmup):
            for r in roots:
                g.bfs(int(r), parent, level)
        torch.cuda.synchronize()
        times = []
        t_all = time.perf_counter()
        for step in range(args.steps):
            for r in roots:
                t0 = time.perf_counter()
                g.bfs(int(r), parent, level)
                times.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_all
        # instrumented pass (untimed): host-driven loop with HIP events around
        # every level and around the bottom-up kernel, for the phase split and
        # the bottom-up kernel's bandwidth
        timed_loop = g.tuning().loop
        g.set_tuning(loop=gt.GT_LOOP_HOST, timing=1)
        bu_b, bu_t, bu_n = 0.0, 0.0, 0
        ph = dict(init=0.0, td=0.0, bu=0.0, output=0.0)
        words = (infos[name]["n_core"] + 63) // 64
        for r in roots:
            g.bfs(int(r), parent, level)
            st = g.last_stats()
            ph["init"] += st.ms_init
            ph["output"] += st.ms_output
            for lv in st.levels():
                if lv["dir"] == "BU":
                    if lv["kernel"] == "bu_words":  # the roofline kernel k_bu; list levels run k_bu_list
                        bu_b += bu_bytes(words, lv["scanned"], lv["examined"], lv["found"],
                                         4 if name == "plain" else 8)
                        bu_t += lv["ms_main"]
                        bu_n += 1
                    ph["bu"] += lv["ms"]
                else:
                    ph["td"] += lv["ms"]
        g.set_tuning(loop=timed_loop)
        times = np.asarray(times)
        per_root_gteps = np.tile(m_r, args.steps) / times / 1e9
        nroot = len(roots)
        results[name] = dict(
            hmean_gteps=hmean(per_root_gteps), mean_gteps=float(per_root_gteps.mean()),
            ms_per_step=wall * 1e3 / args.steps,
            p50_ms=float(np.percentile(times, 50) * 1e3), p99_ms=float(np.percentile(times, 99) * 1e3),
            phase_ms_per_root={k: v / nroot for k, v in ph.items()},
            bu_launches=bu_n, bu_bytes_per_launch=bu_b / max(bu_n, 1),
            bu_ms_per_launch=bu_t / max(bu_n, 1),
            bu_gbs=(bu_b / 1e9) / (bu_t / 1e3) if bu_t > 0 else 0.0)
        log("%s: hmean %.2f GTEPS, p50 %.3f ms, BU %.0f GB/s" % (
            name, results[name]["hmean_gteps"], results[name]["p50_ms"], results[name]["bu_gbs"]))

    sp = results["split"]
    degree_aware = degree_aware_ablation(handles["split"], roots, m_r, parent, level) if args.hint_ablation else None
    traffic = read_traffic_profile(args.scale, core_numbering(args))
    out = {
        "metric": METRIC,
        "value": round(sp["hmean_gteps"], 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sp["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "Kronecker scale %d, edgefactor %d, %d seeded roots one at a time, "
                               "low-degree-split BFS" % (args.scale, args.edgefactor, len(roots)),
                   "scale": args.scale, "edgefactor": args.edgefactor, "roots": int(len(roots)),
                   "graph_seed": args.seed, "root_seed": args.root_seed, "level_loop": args.loop,
                   "split_core_numbering": core_numbering(args)},
        "tuning": tuned or None,
        "plain_hmean_gteps": round(results["plain"]["hmean_gteps"], 4),
        "split_over_plain": round(sp["hmean_gteps"] / results["plain"]["hmean_gteps"], 4),
        "mean_gteps": {k: round(v["mean_gteps"], 4) for k, v in results.items()},
        "edge_trees": edge_tree_report(args, infos, results),
        "degree_aware": degree_aware,
        "ablation": None if "rmzero" not in results else {
            "rmzero_hmean_gteps": round(results["rmzero"]["hmean_gteps"], 4),
            "rmzero_over_plain": round(results["rmzero"]["hmean_gteps"] / results["plain"]["hmean_gteps"], 4),
            "split_over_rmzero": round(sp["hmean_gteps"] / results["rmzero"]["hmean_gteps"], 4),
            "rmzero_core": infos["rmzero"]["n_core"], "rmzero_core_entries": infos["rmzero"]["n_core_entries"]},
        "latency_ms": {k: {"p50": round(v["p50_ms"], 4), "p99": round(v["p99_ms"], 4)} for k, v in results.items()},
        "phase_ms_per_root": {k: {p: round(t, 4) for p, t in v["phase_ms_per_root"].items()} for k, v in results.items()},
        "graph": {"n": n, "entries": infos["plain"]["n_entries"], "core": infos["split"]["n_core"],
                  "leaf": infos["split"]["n_leaf"], "zero": infos["split"]["n_zero"],
                  "core_entries": infos["split"]["n_core_entries"],
                  "pruned_fraction": round((infos["split"]["n_leaf"] + infos["split"]["n_zero"]) / n, 4),
                  "build_ms": {k: round(v["build_ms"], 1) for k, v in infos.items()}},
        "roofline": {"kernel": "k_bu (split)", "bound": "hbm",
                     "achieved": round(sp["bu_gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(sp["bu_gbs"] / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": round(sp["bu_bytes_per_launch"]),
                     "ms_per_launch": round(sp["bu_ms_per_launch"], 5),
                     "launches": sp["bu_launches"],
                     "traffic": traffic,
                     "plain_achieved": round(results["plain"]["bu_gbs"], 2)},
        "cpu_baseline": None,
    }
    if base is not None:
        log("waiting for the CPU oracle baseline")
        base.join()
        if base.result is not None:
            out["cpu_baseline"] = base.result
            out["cpu_baseline"]["levels_equal_gpu"] = bool(np.array_equal(base.levels, root0_split_levels))
        else:
            out["cpu_baseline"] = {"error": base.error}
    for g in handles.values():
        g.close()
    print(json.dumps(out), flush=True)


def degree_aware_ablation(g, roots, m_r, parent, level):
    """The degree-aware bottom-up probe (Section 2.3: each vertex first tests
    its highest-degree neighbour) on and off, on the split handle with its
    tuned knobs otherwise: harmonic-mean GTEPS over the roots and the
    bottom-up counters (vertices tested, adjacency entries read) per root."""
    import torch
    out = {}
    knobs = g.tuning()
    for name, hint in (("hint_on", 1), ("hint_off", 2)):
        g.set_tuning(bu_hint=hint, timing=0)
        for r in roots[:8]:
            g.bfs(int(r), parent, level)
        torch.cuda.synchronize()
        times = []
        for r in roots:
            t0 = time.perf_counter()
            g.bfs(int(r), parent, level)
            times.append(time.perf_counter() - t0)
        g.set_tuning(loop=1, timing=1)
        tested = examined = 0
        for r in roots:
            g.bfs(int(r), parent, level)
            for lv in g.last_stats().levels():
                if lv["dir"] == "BU":
                    tested += lv["scanned"]
                    examined += lv["examined"]
        g.set_tuning(loop=knobs.loop, timing=0)
        out[name] = {"hmean_gteps": round(hmean(m_r / np.asarray(times) / 1e9), 4),
                     "bu_tested_per_root": round(tested / len(roots)),
                     "bu_examined_per_root": round(examined / len(roots))}
    g.set_tuning(bu_hint=knobs.bu_hint)
    return out


def tree_table(i):
    """Edge trees grouped by their core-edge vertex (the paper's Table 3
    columns) from a handle's info."""
    n = i["n_edge_trees"]
    return {"trees": n, "average": round(i["edge_tree_vertices"] / n, 3) if n else 0,
            "max": i["edge_tree_max"], "min": i["edge_tree_min"], "total": i["edge_tree_vertices"]}


def edge_tree_report(args, infos, results):
    """Class counts and traversal rate of the MH > 0 handles, beside the
    paper's Table 2 rows for the same graph size (scale 26, edgefactor 16)."""
    if not args.mh:
        return None
    out = {}
    for mh in args.mh:
        i = infos["mh%d" % mh]
        r = results["mh%d" % mh]
        ti = i["n_tree_internal"]
        out["mh%d" % mh] = {
            "classes": {"CI": i["n_core"] - i["n_core_edge"], "CE": i["n_core_edge"], "TI": ti,
                        "TL": i["n_leaf"] - ti, "VZ": i["n_zero"]},
            "tree_height": i["tree_height"], "core_entries": i["n_core_entries"],
            "edge_trees": tree_table(i),
            "hmean_gteps": round(r["hmean_gteps"], 4), "p50_ms": round(r["p50_ms"], 4)}
    out["mh0_edge_trees"] = tree_table(infos["split"])
    if args.scale == 26 and args.edgefactor == 16:
        rows = {}
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                               "table2_scale26.txt")) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    v = [int(x) for x in line.split()]
                    rows["mh%d" % v[0]] = dict(zip(("CI", "CE", "TI", "TL", "VZ"), v[1:]))
        out["paper_table2"] = rows
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                               "table3_scale26.txt")) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    v = [int(x) for x in line.split()]
                    out["paper_table3"] = {"mh%d" % v[0]: dict(zip(("trees", "average", "max", "min", "total"),
                                                                   v[1:]))}
    return out


# Algorithmic bytes of one pull step of the batched BFS on n vertices (the
# pull and the step's finalize are one kernel): per vertex the seen mask read
# (8 B), the next-frontier mask written (8 B), the previous frontier buffer
# cleared (8 B) and, when the step also pushed, the next mask read for the
# push's bits (8 B); the hint entry per vertex still missing a slot (h B,
# counted for all n: an upper bound); per adjacency entry examined the entry
# (e B) plus the neighbour's frontier mask (8 B); per (vertex, slot) pair
# found its level byte (1 B).
def ms_pull_bytes(n, examined, found_pairs, pushed, h, e):
    return (32.0 if pushed else 24.0) * n + h * n + (e + 8.0) * examined + 1.0 * found_pairs


def run_batch(args):
    """64 roots in one batched launch vs 64 single-root runs (scale 24)."""
    import torch
    import graphgen
    import paper_2009_07463_amd as gt

    gt.load_library(build_if_missing=True)
    torch.cuda.set_device(0)
    n, src, dst = make_graph(args.scale, args.edgefactor, args.seed)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, args.roots, seed=args.root_seed)]
    base = OracleBaseline(n, src, dst, roots[0]) if args.cpu_baseline else None
    if base is not None:
        base.start()
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    # both modes on the hubs-first core numbering (the faster for each), on
    # separate handles so that each keeps its own tuned knobs
    g = gt.Graph(s, d, n, split=True, hubs_first=args.hubs_first, hub_share=args.hub_share)
    gs = gt.Graph(s, d, n, split=True, hubs_first=args.hubs_first, hub_share=args.hub_share)
    info = g.info()
    del s, d
    torch.cuda.empty_cache()
    k = len(roots)
    levels = torch.empty((k, n), dtype=torch.uint8, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    level32 = torch.empty(n, dtype=torch.int32, device="cuda")
    tuned = None
    if args.loop == "auto":
        # knobs (single-root and batched) tuned on a separate sample of roots
        tune_roots = graphgen.sample_roots(n, src, dst, 64, seed=args.root_seed + 100)
        t0 = time.perf_counter()
        tun, rep = g.autotune(tune_roots, cache_path=args.tune_cache, batch=True)
        rep["seconds"] = round(time.perf_counter() - t0, 2)
        tun_s, rep_s = gs.autotune(tune_roots, cache_path=args.tune_cache)
        tuned = {"knobs": tun, "report": rep, "single_root_handle": {"knobs": tun_s, "report": rep_s}}
        log("batch handle autotuned in %.1f s" % rep["seconds"])
    g.set_tuning(timing=0)
    gs.set_tuning(timing=0)
    for _ in range(args.warmup):
        g.bfs_batch(roots, levels)
        for r in roots:
            gs.bfs(r, parent, level32)
    torch.cuda.synchronize()
    t_batch = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        g.bfs_batch(roots, levels)
        t_batch.append(time.perf_counter() - t0)
    # instrumented run (untimed): HIP events around every step and around the
    # pull kernel, for the roofline of k_ms_pull and the extraction time
    g.set_tuning(timing=1)
    g.bfs_batch(roots, levels)
    st = g.last_stats()
    g.set_tuning(timing=0)
    pull_b, pull_t, pull_n = 0.0, 0.0, 0
    h = 8 if g.split else 4
    ex_ms = st.ms_output
    for lv in st.levels():
        if lv["dir"] == "BU" and lv["ms_main"] > 0:
            pull_b += ms_pull_bytes(info["n_core"], lv["examined"], lv["found"], lv["frontier"] > 0, h, h)
            pull_t += lv["ms_main"]
            pull_n += 1
    seq_done = []
    seq_service = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        for r in roots:
            t1 = time.perf_counter()
            gs.bfs(r, parent, level32)
            seq_service.append(time.perf_counter() - t1)
            seq_done.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    # parents for 8 sampled slots (device time of the call; the copy to the
    # host for validation is outside it)
    sample = list(range(0, k, max(1, k // 8)))[:8]
    parents = {}
    par_dev = torch.empty(n, dtype=torch.int32, device="cuda")
    t_par = 0.0
    for i in sample:
        lv_i = levels[i].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.reconstruct_parent(roots[i], lv_i, par_dev)
        torch.cuda.synchronize()
        t_par += time.perf_counter() - t0
        parents[i] = par_dev.cpu().numpy()
    t_par /= len(sample)
    tb = float(np.median(t_batch))
    seq_total = float(np.sum(seq_service) / args.steps)
    out = {
        "metric": "queries/s, %d-root batched BFS (scale %d)" % (k, args.scale),
        "value": round(k / tb, 2), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(tb * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "Kronecker scale %d, edgefactor %d, %d roots in one batched run vs "
                               "%d single-root runs" % (args.scale, args.edgefactor, k, k),
                   "scale": args.scale, "edgefactor": args.edgefactor, "roots": k,
                   "batch_core_numbering": core_numbering(args),
                   "single_root_core_numbering": core_numbering(args)},
        "tuning": tuned,
        "batched": {"queries_per_s": round(k / tb, 2), "batch_ms": round(tb * 1e3, 3),
                    "latency_ms_p50": round(tb * 1e3, 3), "latency_ms_p99": round(tb * 1e3, 3),
                    "extract_ms": round(ex_ms, 3)},
        "sequential": {"queries_per_s": round(k / seq_total, 2), "total_ms": round(seq_total * 1e3, 3),
                       "latency_ms_p50": round(float(np.percentile(seq_done, 50)) * 1e3, 3),
                       "latency_ms_p99": round(float(np.percentile(seq_done, 99)) * 1e3, 3),
                       "service_ms_p50": round(float(np.percentile(seq_service, 50)) * 1e3, 3)},
        "batched_over_sequential": round(seq_total / tb, 3),
        "reconstruct_parent_ms": round(t_par * 1e3, 3),
        "roofline": {"kernel": "k_ms_pull (split)", "bound": "hbm",
                     "achieved": round((pull_b / 1e9) / (pull_t / 1e3), 2) if pull_t > 0 else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round((pull_b / 1e9) / (pull_t / 1e3) / HBM_PEAK_GBS, 4) if pull_t > 0 else None,
                     "bytes_per_launch": round(pull_b / max(pull_n, 1)),
                     "ms_per_launch": round(pull_t / max(pull_n, 1), 5), "launches": pull_n,
                     "traffic": None},
        "graph": {"n": n, "core": info["n_core"], "leaf": info["n_leaf"], "zero": info["n_zero"]},
        "cpu_baseline": None,
    }
    if base is not None:
        base.join()
        if base.result is not None:
            import oracle
            out["cpu_baseline"] = base.result
            ref = base.levels
            got = levels[0].cpu().numpy().astype(np.int32)
            got[got == 255] = -1
            out["cpu_baseline"]["levels_equal_gpu"] = bool(np.array_equal(ref, got))
        else:
            out["cpu_baseline"] = {"error": base.error}
    g.close()
    gs.close()
    print(json.dumps(out), flush=True)


def run_serve(args):
    """Continuous batching vs one query at a time over 4 resident graphs."""
    import torch
    import graphgen
    import paper_2009_07463_amd as gt
    from paper_2009_07463_amd import serve

    gt.load_library(build_if_missing=True)
    torch.cuda.set_device(0)
    scales = [int(x) for x in args.serve_scales.split(",")]
    graphs, pools, sizes = {}, {}, {}
    for sc in scales:
        n, src, dst = make_graph(sc, args.edgefactor, args.seed + sc)
        name = "s%d" % sc
        pools[name] = graphgen.sample_roots(n, src, dst, 4096, seed=args.root_seed + sc)
        s = torch.from_numpy(src).cuda()
        d = torch.from_numpy(dst).cuda()
        graphs[name] = gt.Graph(s, d, n, split=True, hubs_first=args.hubs_first, hub_share=args.hub_share)
        sizes[name] = n
        del s, d
    torch.cuda.empty_cache()
    names = sorted(graphs)
    budget = int(args.serve_budget_mb) << 20

    def run(sequential, rate, count, seed):
        srv = serve.Server(hbm_budget_bytes=budget, slots=64, sequential=sequential,
                           solo_max=args.serve_solo_max)
        for nm in names:
            srv.add_graph(nm, graphs[nm], sizes[nm])
        if rate is None:   # saturation: everything scheduled at t = 0
            sched = [(0.0, g_, r_) for (_, g_, r_) in serve.poisson_arrivals(1.0, count, names, pools, seed)]
        else:
            sched = serve.poisson_arrivals(rate, count, names, pools, seed)
        qs, t0 = serve.run_open_loop(srv, sched)
        srv.join()
        summ = serve.latency_summary(qs, t0)
        summ["steps"] = srv.steps()
        if not sequential:
            summ["solo"] = srv.solo_counts()
        return summ

    # warm up both servers
    run(False, None, 128, 7)
    run(True, None, 64, 7)
    cap_cb = run(False, None, args.serve_count, 11)
    cap_seq = run(True, None, args.serve_count, 11)
    log("capacity: continuous batching %.0f q/s, one at a time %.0f q/s" % (cap_cb["qps"], cap_seq["qps"]))
    sweep = []
    for frac in [float(x) for x in args.serve_loads.split(",")]:
        rate = frac * cap_cb["qps"]
        count = max(200, min(args.serve_count, int(rate * args.serve_seconds)))
        cb = run(False, rate, count, 100 + int(frac * 100))
        sq = run(True, rate, count, 100 + int(frac * 100))
        row = {"load": frac, "offered_qps": round(rate, 1), "queries": count,
               "continuous_batching": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in cb.items()},
               "one_at_a_time": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in sq.items()}}
        sweep.append(row)
        log("load %.2f: cb %.0f q/s p50 %.2f p99 %.2f ms | seq %.0f q/s p50 %.2f p99 %.2f ms" % (
            frac, cb["qps"], cb["p50_ms"], cb["p99_ms"], sq["qps"], sq["p50_ms"], sq["p99_ms"]))
    # a result is the same alone and in the mix: replay a mixed burst and compare
    same = check_alone_vs_mix(graphs, names, pools, sizes, budget)
    out = {
        "metric": "queries/s and p50/p99 latency, continuous-batching BFS server (scales %s)" % args.serve_scales,
        "value": round(cap_cb["qps"], 2), "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "4 resident Kronecker graphs (scales %s, edgefactor %d), Poisson arrivals, "
                               "uniform graph, uniform roots of degree >= 1" % (args.serve_scales, args.edgefactor),
                   "hbm_budget_mb": args.serve_budget_mb, "slots": 64, "solo_max": args.serve_solo_max},
        "capacity": {"continuous_batching": cap_cb, "one_at_a_time": cap_seq},
        "sweep": sweep,
        "alone_vs_mix_equal": same,
    }
    for h in graphs.values():
        h.close()
    print(json.dumps(out), flush=True)


def check_alone_vs_mix(graphs, names, pools, sizes, budget):
    """Run a burst through the server, keep results, and compare each with the
    same query run alone (gt_bfs_batch with one root). Exact equality."""
    import torch
    from paper_2009_07463_amd import serve

    kept = {}

    def on_result(q):
        # synchronous copy: the buffer is recycled as soon as on_result returns
        kept[q.qid] = (q.graph, q.root, q.result.cpu())

    on_result.keeps_buffer = True
    srv = serve.Server(hbm_budget_bytes=budget, slots=64, on_result=on_result)
    for nm in names:
        srv.add_graph(nm, graphs[nm], sizes[nm])
    sched = serve.poisson_arrivals(20000.0, 192, names, pools, 99)
    serve.run_open_loop(srv, sched)
    srv.join()
    ok = True
    for qid, (gname, root, res) in kept.items():
        alone = graphs[gname].bfs_batch([root])[0].cpu()
        ok = ok and bool(torch.equal(alone, res))
    return ok and len(kept) == 192


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["single", "batch", "serve"], default="single")
    ap.add_argument("--scale", type=int, default=26)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--root-seed", type=int, default=2)
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--loop", choices=["auto", "host", "graph", "device"], default="auto",
                    help="level loop of the timed single-source pass (auto: autotune every knob)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (default: none, always tune)")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--mh", type=lambda x: [int(v) for v in x.split(",") if v], default=[1, 2],
                    help="also build and time edge-tree handles of these maximum heights ('' for none)")
    ap.add_argument("--no-hubs-first", dest="hubs_first", action="store_false",
                    help="number the core of the split handles in caller order instead of hubs first")
    ap.add_argument("--hub-share", type=int, default=None,
                    help="hubs-first handles: at most n_core / 2^k hubs (default 2 for one root at a "
                         "time, where it moves time from the bottom-up to the top-down phase; 5 for the "
                         "batch and serve modes, whose pull reads the hubs' masks most)")
    ap.add_argument("--no-hint-ablation", dest="hint_ablation", action="store_false",
                    help="skip timing the split handle with the degree-aware probe off")
    ap.add_argument("--no-rmzero", dest="rmzero", action="store_false",
                    help="skip the RmZero ablation handle (only isolated vertices removed)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0)
    ap.add_argument("--serve-scales", default="18,20,22,24")
    ap.add_argument("--serve-loads", default="0.1,0.25,0.5,0.75,1.0,1.25,1.5")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    ap.add_argument("--serve-budget-mb", type=int, default=1024)
    ap.add_argument("--serve-solo-max", type=int, default=8,
                    help="a query meeting an idle session with at most this many waiting runs single-root")
    args = ap.parse_args()
    if args.mode == "batch" and args.scale == 26 and "--scale" not in sys.argv:
        args.scale = 24
    if args.hub_share is None:
        args.hub_share = 2 if args.mode == "single" else 5
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported "
              "(multi-GPU sharding is described, not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.mode == "single":
        run_single(args)
    elif args.mode == "batch":
        run_batch(args)
    else:
        run_serve(args)


if __name__ == "__main__":
    main()
