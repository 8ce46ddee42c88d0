"""Benchmark: low-degree-split BFS vs plain direction-optimizing BFS on one MI355X.

The default run (--mode all) measures the four workloads of the paper's
evaluation (Section 6.1: Graph500 Kronecker graphs, initiator A=.57,
B=C=.19, D=.05, edgefactor 16, 64 random roots) on this GPU:

  scale 26   64 seeded roots one at a time through gt_bfs on the split
             handle (the headline), beside the plain handle and the
             ablations: caller-order split, plain on the hubs-first
             numbering, RmZero, edge trees of height 1 and 2, the
             degree-aware probe off;
  scale 22   split vs plain, 64 roots;
  scale 24   64 roots in one batched launch vs 64 single-root runs;
  serving    four resident graphs (scales 18-24), Poisson arrivals at
             three loads, continuous batching vs one query at a time.

One step = the 64 scale-26 roots through gt_bfs on the split handle. The
metric is Graph500-style: per root, m_r = half the degree sum of the reached
vertices (the traversed undirected edges), t_r = wall time of the gt_bfs call
(output init, root handling, core BFS, leaf pass, id translation); the
headline value is the harmonic mean of m_r / t_r over all timed roots. Every
timed root's result is validated (Graph500 rules over the raw edge list,
tests/level_check.py), and the CPU oracle's levels are compared for the roots
it times.

Also in the same JSON line:
  roofline      the bottom-up word kernel k_bu: algorithmic bytes per launch
                by the traversal byte model (2n/8 + 8S + 4.125Y + 8N' per
                bottom-up level over n traversed vertices, S tested, Y
                adjacency entries examined, N' discovered) over its
                event-timed launch duration, against 8 TB/s; beside it the
                measured streaming-copy ceiling and the hipDeviceProp peak;
  cpu_baseline  the CPU oracle (single thread) timed on 8 of the scale-26
                roots, sequentially, on this host (CPU model and core count
                recorded).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import queue
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s (published)
GT_LOOP_NAMES = {1: "host", 2: "graph", 3: "device"}   # GT_LOOP_HOST / _GRAPH / _DEVICE
METRIC = "harmonic-mean GTEPS at scale 26 (split vs plain BFS); p50/p99 query latency"
TUNE_KEYS = ("loop", "graph_levels", "alpha", "beta", "bu_blocks", "bu_lane_edges", "bu_hub_deg", "bu_hub_blocks",
             "td_small_edges", "td_blocks", "td_hub_deg", "bu_hint", "bu_lds", "bu_form", "bu_gamma", "td_flat", "bu_list_div")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def hmean(x):
    x = np.asarray(x, dtype=np.float64)
    return float(len(x) / np.sum(1.0 / x))


# Algorithmic bytes of one bottom-up level over n traversed vertices, by the
# traversal byte model: the visited bitmap read and the next one written
# (2 n/8), sequential row offsets per tested (unvisited) vertex (8 S), per
# adjacency entry examined the 4-byte entry and its bitmap probe (4.125 Y; a
# probe of the dense highest-degree-neighbour copy counts as one entry), and
# a discovery's level and parent (8 N').
def bu_model_bytes(n, scanned, examined, found):
    return 2.0 * n / 8.0 + 8.0 * scanned + 4.125 * examined + 8.0 * found


# What the kernel's layout touches instead (no cache effects): 16 B per
# 64-vertex bitmap word (read, write), per tested vertex its hint entry and
# degree (8 B), per examined entry 4 B + 1/8, per discovery its (level,
# parent) pair and the parent's caller id (12 B); row offsets of the vertices
# the hint misses are not counted (no counter separates them).
def bu_layout_bytes(words, scanned, examined, found):
    return 16.0 * words + 8.0 * scanned + 4.125 * examined + 12.0 * found


def code_text(text):
    """C++ source without its comments, blank lines and trailing blanks (the
    sources hold no string literal with a comment marker in it)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_sha(root=None):
    """Hash of the code of the bottom-up kernel (its body and the host-driven
    loop that launches it), comments left out, so that rewording a comment
    keeps a profile taken on the same code valid."""
    h = hashlib.sha256()
    for name in ("bfs_kernels.h", "bfs.hip"):
        with open(os.path.join(root or ROOT, "paper_2009_07463_amd", "csrc", name)) as f:
            h.update(code_text(f.read()).encode())
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


def core_numbering(hubs_first, hub_share):
    """How a split handle numbers its core (recorded with each result)."""
    if not hubs_first:
        return "caller order"
    return "hubs first (at most n_core / 2^%d)" % hub_share


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


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


class OracleWorker(threading.Thread):
    """The CPU oracle in the background (one thread, single-threaded C): for
    each job, its own CSR build (untimed), then one FIFO BFS per root, timed
    one after another. Levels are kept for comparison with the GPU's."""

    def __init__(self):
        super().__init__(daemon=True)
        self.jobs = queue.Queue()
        self.results = {}
        self.errors = {}

    def add(self, name, n, src, dst, roots, heights=()):
        """Time BFS from each root; also classify the vertices by
        Algorithm 8 for each maximum tree height in `heights`."""
        self.jobs.put((name, n, src, dst, [int(r) for r in roots], tuple(heights)))

    def finish(self):
        self.jobs.put(None)

    def run(self):
        import oracle
        while True:
            job = self.jobs.get()
            if job is None:
                return
            name, n, src, dst, roots, heights = job
            try:
                t0 = time.perf_counter()
                g = oracle.build_csr(n, src, dst)
                t_build = time.perf_counter() - t0
                secs, edges, levels = [], [], []
                for r in roots:
                    t0 = time.perf_counter()
                    _, lvl = oracle.bfs(g, r)
                    secs.append(time.perf_counter() - t0)
                    edges.append(oracle.reached_edges(g, lvl))
                    levels.append(lvl)
                classes = {}
                for h in heights:
                    cnt = np.bincount(oracle.etvca(g, h), minlength=5)
                    classes[h] = dict(zip(("CI", "CE", "TI", "TL", "VZ"), (int(x) for x in cnt[:5])))
                self.results[name] = dict(seconds=secs, edges=edges, levels=levels, build_s=t_build, roots=roots,
                                          classes=classes)
                del g
            except Exception as e:  # reported, never fatal to the GPU numbers
                self.errors[name] = repr(e)


def oracle_summary(res, scale, what):
    g = np.asarray(res["edges"], np.float64) / np.asarray(res["seconds"]) / 1e9
    out = dict(value=round(hmean(g), 5), unit="GTEPS", cores=1, kind="oracle",
               sample="%s at scale %d, each timed on its own, one after another; single-thread FIFO BFS over the "
                      "whole graph; its own CSR build (%.0f s) untimed" % (what, scale, res["build_s"]),
               mean_gteps=round(float(g.mean()), 5), roots=len(res["roots"]),
               seconds_per_root=round(float(np.mean(res["seconds"])), 3))
    out.update(cpu_info())
    return out


def make_graph(scale, edgefactor, seed):
    import graphgen
    n = 1 << scale
    t0 = time.perf_counter()
    src, dst = graphgen.kronecker_edges(scale, edgefactor, seed=seed)
    log("scale %d: generated %d edges in %.1f s" % (scale, src.size, time.perf_counter() - t0))
    return n, src, dst


def tune_handle(h, tune_roots, cache, batch=False):
    t0 = time.perf_counter()
    tun, rep = h.autotune(tune_roots, cache_path=cache, batch=batch)
    rep["seconds"] = round(time.perf_counter() - t0, 2)
    return {"knobs": {k: tun[k] for k in TUNE_KEYS + (("ms_blocks", "ms_alpha", "ms_loop") if batch else ())},
            "report": rep}


def time_roots(g, roots, steps, warmup, parent, level):
    """Wall time of each gt_bfs call (it returns with the outputs complete)
    over `steps` passes of the roots, after `warmup` passes."""
    import torch
    g.set_tuning(timing=0)
    for _ in range(warmup):
        for r in roots:
            g.bfs(int(r), parent, level)
    torch.cuda.synchronize()
    times = []
    t_all = time.perf_counter()
    for _ in range(steps):
        for r in roots:
            t0 = time.perf_counter()
            g.bfs(int(r), parent, level)
            times.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    return np.asarray(times), time.perf_counter() - t_all


def instrumented_pass(g, roots, n_traversed, parent, level):
    """Host-driven loop with HIP events around every level and around the
    bottom-up word kernel (untimed): phase split per root and the bottom-up
    kernel's bytes (model and layout) and time."""
    import paper_2009_07463_amd as gt
    timed_loop = g.tuning().loop
    g.set_tuning(loop=gt.GT_LOOP_HOST, timing=1)
    words = (n_traversed + 63) // 64
    acc = dict(model=0.0, layout=0.0, ms=0.0, launches=0, S=0, Y=0, N=0)
    ph = dict(init=0.0, td=0.0, bu=0.0, output=0.0)
    td_levels = []
    for r in roots:
        g.bfs(int(r), parent, level)
        st = g.last_stats()
        ph["init"] += st.ms_init
        ph["output"] += st.ms_output
        for lv in st.levels():
            if lv["dir"] == "BU":
                if lv["kernel"] == "bu_words":  # the roofline kernel k_bu; list levels run k_bu_list
                    S = lv["scanned"]
                    Y = lv["examined"] - lv["examined_long"]
                    N = lv["found"] - lv["found_long"]
                    acc["model"] += bu_model_bytes(n_traversed, S, Y, N)
                    acc["layout"] += bu_layout_bytes(words, S, Y, N)
                    acc["ms"] += lv["ms_main"]
                    acc["launches"] += 1
                    acc["S"] += S
                    acc["Y"] += Y
                    acc["N"] += N
                ph["bu"] += lv["ms"]
            else:
                ph["td"] += lv["ms"]
                td_levels.append((lv["examined"], lv["found"], lv["ms"]))
    g.set_tuning(loop=timed_loop, timing=0)
    k = max(acc["launches"], 1)
    bu = dict(launches=acc["launches"], model_bytes_per_launch=acc["model"] / k,
              layout_bytes_per_launch=acc["layout"] / k, ms_per_launch=acc["ms"] / k,
              gbs=(acc["model"] / 1e9) / (acc["ms"] / 1e3) if acc["ms"] > 0 else 0.0,
              sums={"launches": acc["launches"], "S": acc["S"], "Y": acc["Y"], "N": acc["N"],
                    "ms": round(acc["ms"], 4)})
    td_x = sum(x for x, _, _ in td_levels)
    td_n = sum(f for _, f, _ in td_levels)
    return {k: v / len(roots) for k, v in ph.items()}, bu, {"examined_per_root": td_x / len(roots),
                                                             "found_per_root": td_n / len(roots)}


def copy_ceiling(gib=4, reps=10):
    """Achievable HBM bandwidth: the library's streaming copy over `gib` GiB
    (read + written bytes per second), best of `reps`, HIP events."""
    import torch
    import paper_2009_07463_amd as gt
    n = (gib << 30) // 16
    a = torch.empty(n * 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    gt.stream_copy(a, b)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gt.stream_copy(a, b)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    ok = bool(torch.equal(a[:1 << 20], b[:1 << 20]))
    del a, b
    torch.cuda.empty_cache()
    return {"gbs": round(2.0 * (gib << 30) / (best / 1e3) / 1e9, 1), "bytes_copied": gib << 30, "ms": round(best, 4),
            "copy_ok": ok, "kernel": "k_stream_copy (gt_stream_copy)"}


def validate_all(s, d, n, roots, g, parent, level, ref_levels=None, full=True):
    """Every root through g, checked by the Graph500 rules over the raw edge
    list (full) or, with ref_levels, levels equal to those (exact)."""
    import torch
    from tests.level_check import LevelCheckError, check_levels
    ok = 0
    fails = []
    for i, r in enumerate(roots):
        g.bfs(int(r), parent, level)
        torch.cuda.synchronize()
        try:
            if ref_levels is not None and not torch.equal(level, ref_levels[i]):
                raise LevelCheckError("levels differ from the reference handle's")
            if full:
                check_levels(s, d, n, int(r), level, parent)
            ok += 1
        except LevelCheckError as e:
            fails.append({"root": int(r), "error": str(e)})
    return ok, fails


# ----------------------------------------------------------- one-root legs --

def run_scale(args, scale, variants, oracle_worker, oracle_roots, full_checks, hint_ablation):
    """One graph, several handles, 64 roots one at a time. variants: list of
    (name, Graph kwargs). Returns the leg's result dict."""
    import torch
    import graphgen
    import paper_2009_07463_amd as gt

    n, src, dst = make_graph(scale, args.edgefactor, args.seed)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, args.roots, seed=args.root_seed)]
    tune_roots = graphgen.sample_roots(n, src, dst, 64, seed=args.root_seed + 100)
    if oracle_worker is not None and oracle_roots:
        heights = [mh for mh in args.mh] if any(v[0].startswith("mh") for v in variants) else []
        oracle_worker.add("scale%d" % scale, n, src, dst, roots[:oracle_roots], heights)
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    torch.cuda.synchronize()
    handles, infos = {}, {}
    for name, kw in variants:
        handles[name] = gt.Graph(s, d, n, **kw)
        infos[name] = handles[name].info()
        log("scale %d %s: build %.0f ms, %.2f GB" % (scale, name, infos[name]["build_ms"],
                                                    infos[name]["device_bytes"] / 1e9))
    torch.cuda.empty_cache()
    names = [v[0] for v in variants]
    first = names[0]
    deg = handles[first].degrees()
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    level = torch.empty(n, dtype=torch.int32, device="cuda")

    # untimed: traversed edges per root (the same for every handle), the
    # reference levels (first handle), and every root validated
    m_r, ref_levels, host_levels = [], [], []
    for i, r in enumerate(roots):
        handles[first].bfs(r, parent, level)
        m_r.append(int(deg[level >= 0].to(torch.int64).sum().item()) // 2)
        ref_levels.append(level.clone())
        if i < oracle_roots:
            host_levels.append(level.cpu().numpy())
    m_r = np.asarray(m_r, dtype=np.float64)
    validation = {}
    for name in names:
        t0 = time.perf_counter()
        ok, fails = validate_all(s, d, n, roots, handles[name], parent, level,
                                 ref_levels=None if name == first else ref_levels, full=name in full_checks)
        validation[name] = {"validated_roots": ok, "roots": len(roots),
                            "checks": "Graph500 rules V1-V4 over the edge list" + (
                                "" if name == first else " and levels equal to %s" % first)
                            if name in full_checks else "levels equal to %s" % first}
        if fails:
            validation[name]["failures"] = fails[:4]
        log("scale %d %s: %d/%d roots valid (%.1f s)" % (scale, name, ok, len(roots), time.perf_counter() - t0))
    del ref_levels
    torch.cuda.empty_cache()

    tuned = {}
    for name in names:
        if args.loop == "auto":
            tuned[name] = tune_handle(handles[name], tune_roots, args.tune_cache)
            log("scale %d %s autotuned in %.1f s" % (scale, name, tuned[name]["report"]["seconds"]))
        else:
            handles[name].set_tuning(loop={"host": gt.GT_LOOP_HOST, "graph": gt.GT_LOOP_GRAPH,
                                           "device": gt.GT_LOOP_DEVICE}[args.loop])
    results = {}
    for name in names:
        g = handles[name]
        times, wall = time_roots(g, roots, args.steps, args.warmup, parent, level)
        phases, bu, td = instrumented_pass(g, roots, infos[name]["n_core"], parent, level)
        per_root = np.tile(m_r, args.steps) / times / 1e9
        results[name] = dict(hmean_gteps=hmean(per_root), mean_gteps=float(per_root.mean()),
                             ms_per_step=wall * 1e3 / args.steps,
                             p50_ms=float(np.percentile(times, 50) * 1e3),
                             p99_ms=float(np.percentile(times, 99) * 1e3),
                             phase_ms_per_root=phases, bu=bu, td=td)
        log("scale %d %s: hmean %.2f GTEPS, p50 %.3f ms, k_bu %.0f GB/s (model bytes)" % (
            scale, name, results[name]["hmean_gteps"], results[name]["p50_ms"], bu["gbs"]))
    degree_aware = degree_aware_ablation(handles[first], roots, m_r, parent, level) if hint_ablation else None
    bu_forms = (bottom_up_form_ablation(handles[first], roots[:args.form_roots], m_r[:args.form_roots],
                                        parent, level) if hint_ablation and args.form_roots > 0 else None)
    for h in handles.values():
        h.close()
    del s, d, deg, parent, level
    torch.cuda.empty_cache()
    return dict(n=n, roots=roots, m_r=m_r, infos=infos, results=results, tuned=tuned, validation=validation,
                degree_aware=degree_aware, bu_forms=bu_forms, host_levels=host_levels)


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


def bottom_up_form_ablation(g, roots, m_r, parent, level):
    """The bottom-up kernel's form (knob bu_form) on the split handle with
    its tuned knobs otherwise, all with the host-driven loop (the only one
    that has forms 2 and 3): a wave per 64-vertex word (1, the library's),
    Algorithm 5 as written with a thread per word (2), a thread per vertex
    (3). Per form: harmonic-mean GTEPS over the given roots, device time of
    the bottom-up kernels and bottom-up counters per root."""
    import torch
    out = {}
    knobs = g.tuning()
    for name, form in (("wave_per_word", 1), ("thread_per_word_alg5", 2), ("thread_per_vertex", 3)):
        g.set_tuning(bu_form=form, loop=1, timing=0)
        for r in roots[:2]:
            g.bfs(int(r), parent, level)
        torch.cuda.synchronize()
        times = []
        for r in roots:
            t0 = time.perf_counter()
            g.bfs(int(r), parent, level)
            times.append(time.perf_counter() - t0)
        g.set_tuning(timing=1)
        tested = examined = 0
        bu_ms = 0.0
        for r in roots:
            g.bfs(int(r), parent, level)
            for lv in g.last_stats().levels():
                if lv["dir"] == "BU":
                    tested += lv["scanned"]
                    examined += lv["examined"]
                    bu_ms += lv["ms_main"]
        g.set_tuning(timing=0)
        out[name] = {"bu_form": form, "hmean_gteps": round(hmean(m_r / np.asarray(times) / 1e9), 4),
                     "bu_kernel_ms_per_root": round(bu_ms / len(roots), 4),
                     "bu_tested_per_root": round(tested / len(roots)),
                     "bu_examined_per_root": round(examined / len(roots))}
    g.set_tuning(bu_form=knobs.bu_form, loop=knobs.loop, timing=0)
    out["roots"] = len(roots)
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
        if "mh%d" % mh not in infos:
            continue
        i = infos["mh%d" % mh]
        r = results["mh%d" % mh]
        ti = i["n_tree_internal"]
        out["mh%d" % mh] = {
            "classes": {"CI": i["n_core"] - i["n_core_edge"], "CE": i["n_core_edge"], "TI": ti,
                        "TL": i["n_leaf"] - ti, "VZ": i["n_zero"]},
            "tree_height": i["tree_height"], "core_entries": i["n_core_entries"],
            "edge_trees": tree_table(i),
            "hmean_gteps": round(r["hmean_gteps"], 4), "p50_ms": round(r["p50_ms"], 4)}
    if "split" in infos:
        out["mh0_edge_trees"] = tree_table(infos["split"])
    if args.scale == 26 and args.edgefactor == 16:
        rows = {}
        with open(os.path.join(ROOT, "tests", "golden", "table2_scale26.txt")) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    v = [int(x) for x in line.split()]
                    rows["mh%d" % v[0]] = dict(zip(("CI", "CE", "TI", "TL", "VZ"), v[1:]))
        out["paper_table2"] = rows
        with open(os.path.join(ROOT, "tests", "golden", "table3_scale26.txt")) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    v = [int(x) for x in line.split()]
                    out["paper_table3"] = {"mh%d" % v[0]: dict(zip(("trees", "average", "max", "min", "total"),
                                                                   v[1:]))}
    return out


def hub_share_for(args):
    """Hub share k of the one-root-at-a-time hubs-first handles (at most
    n_core / 2^k hubs): --hub-share, else the k that makes the hub class fit
    the 64 KB LDS bitmap of the bottom-up kernel (n_core / 2^k <= 512 K at
    edgefactor 16: k = scale - 20, at least 2)."""
    return args.hub_share if args.hub_share is not None else max(2, args.scale - 20)


def scale_variants(args, headline):
    """Handles of a one-root-at-a-time leg: the first is the reference."""
    hs = hub_share_for(args)
    v = [("split", dict(split=True, hubs_first=args.hubs_first, hub_share=hs)),
         ("plain", dict(split=False))]
    if headline:
        v += [("split_caller", dict(split=True)),
              ("plain_hubs", dict(split=True, keep_all=True, hubs_first=True, hub_share=hs))]
        if args.rmzero:
            v.append(("rmzero", dict(split=True, rmzero=True, hubs_first=args.hubs_first, hub_share=hs)))
        for mh in args.mh:
            v.append(("mh%d" % mh, dict(split=True, mh=mh, hubs_first=args.hubs_first, hub_share=hs)))
    if args.handles:
        v = [x for x in v if x[0] in args.handles]
    return v


def ratio(r, a, b):
    """hmean GTEPS of handle a over handle b (None if either was not run)."""
    if a not in r or b not in r:
        return None
    return round(r[a]["hmean_gteps"] / r[b]["hmean_gteps"], 4)


def hm(r, a):
    return round(r[a]["hmean_gteps"], 4) if a in r else None


def leg_summary(leg, scale):
    r = leg["results"]
    i = leg["infos"]
    sk = "split" if "split" in i else next(iter(i))
    out = {"scale": scale, "roots": len(leg["roots"]),
           "hmean_gteps": {k: round(v["hmean_gteps"], 4) for k, v in r.items()},
           "mean_gteps": {k: round(v["mean_gteps"], 4) for k, v in r.items()},
           "latency_ms": {k: {"p50": round(v["p50_ms"], 4), "p99": round(v["p99_ms"], 4)} for k, v in r.items()},
           "split_over_plain": ratio(r, "split", "plain"),
           "graph": {"n": leg["n"], "entries": i[next(iter(i))]["n_entries"], "core": i[sk]["n_core"],
                     "leaf": i[sk]["n_leaf"], "zero": i[sk]["n_zero"],
                     "core_entries": i[sk]["n_core_entries"],
                     "pruned_fraction": round((i[sk]["n_leaf"] + i[sk]["n_zero"]) / leg["n"], 4),
                     "build_ms": {k: round(v["build_ms"], 1) for k, v in i.items()}},
           "validated_roots": {k: v["validated_roots"] for k, v in leg["validation"].items()},
           "phase_ms_per_root": {k: {p: round(t, 4) for p, t in v["phase_ms_per_root"].items()}
                                 for k, v in r.items()}}
    return out


# ----------------------------------------------------------- batched leg --

# Algorithmic bytes of one pull step of the batched BFS on n vertices (the
# pull and the step's finalize are one kernel): per vertex the seen mask read
# (8 B), the next-frontier mask written (8 B), the previous frontier buffer
# cleared (8 B) and, when the step also pushed, the next mask read for the
# push's bits (8 B); the 4-byte hint entry per vertex (counted for all n: an
# upper bound); per adjacency entry examined the 4-byte entry plus the
# neighbour's frontier mask (8 B); per (vertex, slot) pair found its level
# byte (1 B).
def ms_pull_bytes(n, examined, found_pairs, pushed):
    return (32.0 if pushed else 24.0) * n + 4.0 * n + 12.0 * examined + 1.0 * found_pairs


def run_batch_leg(args, scale, roots_k, steps, warmup):
    """64 roots in one batched launch vs 64 single-root runs; parents
    reconstructed for 8 sampled roots; every slot validated."""
    import torch
    import graphgen
    import paper_2009_07463_amd as gt
    from tests.level_check import LevelCheckError, check_levels, u8_to_i32

    n, src, dst = make_graph(scale, args.edgefactor, args.seed)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, roots_k, seed=args.root_seed)]
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    hs = args.batch_hub_share
    # both modes on the hubs-first core numbering, on separate handles so
    # that each keeps its own tuned knobs
    g = gt.Graph(s, d, n, split=True, hubs_first=args.hubs_first, hub_share=hs)
    gs = gt.Graph(s, d, n, split=True, hubs_first=args.hubs_first, hub_share=hs)
    info = g.info()
    k = len(roots)
    levels = torch.empty((k, n), dtype=torch.uint8, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    level32 = torch.empty(n, dtype=torch.int32, device="cuda")
    tuned = None
    if args.loop == "auto":
        tune_roots = graphgen.sample_roots(n, src, dst, 64, seed=args.root_seed + 100)
        tuned = {"batch_handle": tune_handle(g, tune_roots, args.tune_cache, batch=True),
                 "single_root_handle": tune_handle(gs, tune_roots, args.tune_cache)}
    g.set_tuning(timing=0)
    gs.set_tuning(timing=0)
    for _ in range(warmup):
        g.bfs_batch(roots, levels)
        for r in roots:
            gs.bfs(r, parent, level32)
    torch.cuda.synchronize()
    t_batch = []
    for _ in range(steps):
        t0 = time.perf_counter()
        g.bfs_batch(roots, levels)
        t_batch.append(time.perf_counter() - t0)
    # the same batch under each step loop (same knobs otherwise), median of
    # `steps` runs each
    timed_ms_loop = g.tuning().ms_loop
    by_loop = {}
    for name, lp in (("host", gt.GT_LOOP_HOST), ("graph", gt.GT_LOOP_GRAPH), ("device", gt.GT_LOOP_DEVICE)):
        g.set_tuning(ms_loop=lp)
        g.bfs_batch(roots, levels)
        torch.cuda.synchronize()
        tl = []
        for _ in range(steps):
            t0 = time.perf_counter()
            g.bfs_batch(roots, levels)
            tl.append(time.perf_counter() - t0)
        by_loop[name] = round(float(np.median(tl)) * 1e3, 3)
    g.set_tuning(ms_loop=timed_ms_loop)
    # instrumented run (untimed): HIP events around every step and the pull,
    # with the host-driven step loop (the graph-captured loop records no
    # per-step times); the same kernels and steps as the timed loop
    g.set_tuning(timing=1, ms_loop=gt.GT_LOOP_HOST)
    g.bfs_batch(roots, levels)
    st = g.last_stats()
    g.set_tuning(timing=0, ms_loop=timed_ms_loop)
    pull_b, pull_t, pull_n = 0.0, 0.0, 0
    for lv in st.levels():
        if lv["dir"] == "BU" and lv["ms_main"] > 0:
            pull_b += ms_pull_bytes(info["n_core"], lv["examined"], lv["found"], lv["frontier"] > 0)
            pull_t += lv["ms_main"]
            pull_n += 1
    seq_done, seq_service = [], []
    for _ in range(steps):
        t0 = time.perf_counter()
        for r in roots:
            t1 = time.perf_counter()
            gs.bfs(r, parent, level32)
            seq_service.append(time.perf_counter() - t1)
            seq_done.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    # validation: every slot by the Graph500 rules, slots 0 and 37 against the
    # single-root handle, parents for 8 sampled slots (device time of the
    # reconstruction timed on its own)
    valid, fails = 0, []
    for i, r in enumerate(roots):
        try:
            check_levels(s, d, n, r, u8_to_i32(levels[i]))
            valid += 1
        except LevelCheckError as e:
            fails.append({"slot": i, "root": r, "error": str(e)})
    same_as_single = True
    for i in (0, min(37, k - 1)):
        gs.bfs(roots[i], parent, level32)
        same_as_single &= bool(torch.equal(u8_to_i32(levels[i]), level32))
    sample = list(range(0, k, max(1, k // 8)))[:8]
    par_dev = torch.empty(n, dtype=torch.int32, device="cuda")
    t_par, par_ok = 0.0, 0
    for i in sample:
        lv_i = levels[i].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.reconstruct_parent(roots[i], lv_i, par_dev)
        torch.cuda.synchronize()
        t_par += time.perf_counter() - t0
        try:
            check_levels(s, d, n, roots[i], u8_to_i32(lv_i), par_dev)
            par_ok += 1
        except LevelCheckError as e:
            fails.append({"slot": i, "root": roots[i], "error": "parents: " + str(e)})
    t_par /= len(sample)
    tb = float(np.median(t_batch))
    seq_total = float(np.sum(seq_service) / steps)
    out = {
        "workload": "Kronecker scale %d, edgefactor %d, %d roots in one batched run vs %d single-root runs"
                    % (scale, args.edgefactor, k, k),
        "scale": scale, "roots": k, "core_numbering": core_numbering(args.hubs_first, hs),
        "tuning": tuned,
        "batched": {"queries_per_s": round(k / tb, 2), "batch_ms": round(tb * 1e3, 3),
                    "latency_ms_p50": round(tb * 1e3, 3), "latency_ms_p99": round(float(np.percentile(t_batch, 99)) * 1e3, 3),
                    "extract_ms": round(st.ms_output, 3), "steps": st.n_levels,
                    "step_loop": GT_LOOP_NAMES.get(timed_ms_loop, str(timed_ms_loop)),
                    "batch_ms_by_step_loop": by_loop},
        "sequential": {"queries_per_s": round(k / seq_total, 2), "total_ms": round(seq_total * 1e3, 3),
                       "latency_ms_p50": round(float(np.percentile(seq_done, 50)) * 1e3, 3),
                       "latency_ms_p99": round(float(np.percentile(seq_done, 99)) * 1e3, 3),
                       "service_ms_p50": round(float(np.percentile(seq_service, 50)) * 1e3, 3)},
        "batched_over_sequential": round(seq_total / tb, 3),
        "reconstruct_parent_ms": round(t_par * 1e3, 3),
        "validated_slots": valid, "parents_validated": par_ok, "parent_sample": len(sample),
        "slots_equal_single_root": same_as_single,
        "pull_roofline": {"kernel": "k_ms_pull (split)", "bound": "hbm",
                          "achieved": round((pull_b / 1e9) / (pull_t / 1e3), 2) if pull_t > 0 else None,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round((pull_b / 1e9) / (pull_t / 1e3) / HBM_PEAK_GBS, 4) if pull_t > 0 else None,
                          "bytes_per_launch": round(pull_b / max(pull_n, 1)),
                          "ms_per_launch": round(pull_t / max(pull_n, 1), 5), "launches": pull_n},
        "graph": {"n": n, "core": info["n_core"], "leaf": info["n_leaf"], "zero": info["n_zero"]},
    }
    if fails:
        out["failures"] = fails[:4]
    g.close()
    gs.close()
    del s, d, levels, parent, level32, par_dev
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------ serving leg --

def run_serve_leg(args):
    """Continuous batching vs one query at a time over 4 resident graphs."""
    import torch
    import graphgen
    import paper_2009_07463_amd as gt
    from paper_2009_07463_amd import serve

    scales = [int(x) for x in args.serve_scales.split(",")]
    graphs, pools, sizes = {}, {}, {}
    for sc in scales:
        n, src, dst = make_graph(sc, args.edgefactor, args.seed + sc)
        name = "s%d" % sc
        pools[name] = graphgen.sample_roots(n, src, dst, 4096, seed=args.root_seed + sc)
        s = torch.from_numpy(src).cuda()
        d = torch.from_numpy(dst).cuda()
        graphs[name] = gt.Graph(s, d, n, split=True, hubs_first=args.hubs_first, hub_share=args.batch_hub_share)
        sizes[name] = n
        del s, d
    torch.cuda.empty_cache()
    names = sorted(graphs)
    cap = None if args.serve_budget_mb is None else int(args.serve_budget_mb) << 20
    budget_bytes = {}

    def run(sequential, rate, count, seed):
        srv = serve.Server(hbm_budget_bytes=cap, slots=64, sequential=sequential, solo_max=args.serve_solo_max)
        budget_bytes["admission"] = srv.budget.budget
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
        return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}

    run(False, None, 128, 7)   # warm up both servers
    run(True, None, 64, 7)
    cap_cb = run(False, None, args.serve_count, 11)
    cap_seq = run(True, None, args.serve_count, 11)
    log("serve capacity: continuous batching %.0f q/s, one at a time %.0f q/s" % (cap_cb["qps"], cap_seq["qps"]))
    sweep = []
    for frac in [float(x) for x in args.serve_loads.split(",")]:
        rate = frac * cap_cb["qps"]
        count = max(200, min(args.serve_count, int(rate * args.serve_seconds)))
        cb = run(False, rate, count, 100 + int(frac * 100))
        sq = run(True, rate, count, 100 + int(frac * 100))
        sweep.append({"load": frac, "offered_qps": round(rate, 1), "queries": count,
                      "continuous_batching": cb, "one_at_a_time": sq})
        log("load %.2f: cb %.0f q/s p50 %.2f p99 %.2f ms | seq %.0f q/s p50 %.2f p99 %.2f ms" % (
            frac, cb["qps"], cb["p50_ms"], cb["p99_ms"], sq["qps"], sq["p50_ms"], sq["p99_ms"]))
    same = check_alone_vs_mix(graphs, names, pools, sizes, cap)
    out = {"workload": "4 resident Kronecker graphs (scales %s, edgefactor %d), Poisson arrivals, uniform graph, "
                       "uniform roots of degree >= 1" % (args.serve_scales, args.edgefactor),
           "slots": 64, "solo_max": args.serve_solo_max,
           "admission_budget_bytes": budget_bytes.get("admission"),
           "admission_rule": "free device memory at start minus a 4 GiB reserve" +
                             ("" if cap is None else ", capped at %d MiB" % args.serve_budget_mb),
           "capacity": {"continuous_batching": cap_cb, "one_at_a_time": cap_seq},
           "sweep": sweep, "alone_vs_mix_equal": same}
    for h in graphs.values():
        h.close()
    torch.cuda.empty_cache()
    return out


def check_alone_vs_mix(graphs, names, pools, sizes, cap):
    """Run a burst through the server, keep results, and compare each with the
    same query run alone (gt_bfs_batch with one root). Exact equality."""
    import torch
    from paper_2009_07463_amd import serve

    kept = {}

    def on_result(q):
        # synchronous copy: the buffer is recycled as soon as on_result returns
        kept[q.qid] = (q.graph, q.root, q.result.cpu())

    on_result.keeps_buffer = True
    srv = serve.Server(hbm_budget_bytes=cap, slots=64, on_result=on_result)
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


# ------------------------------------------------------------------ main --

def headline(args):
    """The scale-26 leg plus (mode all) the scale-22, batched and serving legs,
    as one JSON line."""
    import torch
    import paper_2009_07463_amd as gt

    gt.load_library(build_if_missing=True)
    torch.cuda.set_device(0)
    props = gt.device_props(0)
    ceiling = copy_ceiling()
    log("device %s, %d CUs; streaming copy %.0f GB/s; hipDeviceProp peak %.0f GB/s" % (
        props["arch"], props["compute_units"], ceiling["gbs"], props["peak_hbm_gbs"]))
    ow = OracleWorker() if args.cpu_baseline else None
    if ow is not None:
        ow.start()
    scale = args.scale
    leg = run_scale(args, scale, scale_variants(args, headline=True), ow, 8 if ow else 0,
                    full_checks=("split", "plain"), hint_ablation=args.hint_ablation)
    r = leg["results"]
    ref = "split" if "split" in r else next(iter(r))  # the handle of `value` and `roofline`
    sp = r[ref]
    numbering = core_numbering(args.hubs_first, hub_share_for(args))
    traffic = read_traffic_profile(scale, numbering)
    bu = sp["bu"]
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
                               "%s BFS" % (scale, args.edgefactor, len(leg["roots"]),
                                           "low-degree-split" if ref == "split" else "%s-handle" % ref),
                   "scale": scale, "edgefactor": args.edgefactor, "roots": len(leg["roots"]),
                   "graph_seed": args.seed, "root_seed": args.root_seed, "level_loop": args.loop,
                   "split_core_numbering": numbering},
        "plain_hmean_gteps": hm(r, "plain"),
        # like for like: both handles number their vertices in caller order
        "split_over_plain": ratio(r, "split_caller", "plain"),
        "split_caller_order_hmean_gteps": hm(r, "split_caller"),
        "hubs_first_ablation": {
            "split_hubs_first": hm(r, "split"),
            "plain_hubs_first": hm(r, "plain_hubs"),
            "split_over_plain_hubs_first": ratio(r, "split", "plain_hubs"),
            "split_caller_order": hm(r, "split_caller"),
            "plain_caller_order": hm(r, "plain")},
        "validated_roots": {k: v["validated_roots"] for k, v in leg["validation"].items()},
        "validation": leg["validation"],
        "mean_gteps": {k: round(v["mean_gteps"], 4) for k, v in r.items()},
        "latency_ms": {k: {"p50": round(v["p50_ms"], 4), "p99": round(v["p99_ms"], 4)} for k, v in r.items()},
        "phase_ms_per_root": {k: {p: round(t, 4) for p, t in v["phase_ms_per_root"].items()} for k, v in r.items()},
        "top_down_per_root": {k: {"examined": round(v["td"]["examined_per_root"]),
                                  "found": round(v["td"]["found_per_root"])} for k, v in r.items()},
        "tuning": leg["tuned"] or None,
        "edge_trees": edge_tree_report(args, leg["infos"], r),
        "degree_aware": leg["degree_aware"],
        "bottom_up_forms": leg["bu_forms"],
        "ablation": None if "rmzero" not in r or "plain_hubs" not in r else {
            "rmzero_hmean_gteps": round(r["rmzero"]["hmean_gteps"], 4),
            "rmzero_over_plain_hubs_first": round(r["rmzero"]["hmean_gteps"] / r["plain_hubs"]["hmean_gteps"], 4),
            "split_over_rmzero": round(sp["hmean_gteps"] / r["rmzero"]["hmean_gteps"], 4),
            "rmzero_core": leg["infos"]["rmzero"]["n_core"],
            "rmzero_core_entries": leg["infos"]["rmzero"]["n_core_entries"]},
        "graph": leg_summary(leg, scale)["graph"],
        "roofline": {"kernel": "k_bu (%s)" % ref, "bound": "hbm",
                     "achieved": round(bu["gbs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(bu["gbs"] / HBM_PEAK_GBS, 4),
                     "bytes_model": "2n/8 + 8S + 4.125Y + 8N' per bottom-up level (n core vertices, S tested, "
                                    "Y entries examined incl. the hint probe, N' found)",
                     "bytes_per_launch": round(bu["model_bytes_per_launch"]),
                     "layout_bytes_per_launch": round(bu["layout_bytes_per_launch"]),
                     "ms_per_launch": round(bu["ms_per_launch"], 5),
                     "launches": bu["launches"], "sums": bu["sums"],
                     "traffic": traffic,
                     "copy_ceiling_gbs": ceiling["gbs"],
                     "frac_of_copy_ceiling": round(bu["gbs"] / ceiling["gbs"], 4) if ceiling["gbs"] else None,
                     "hipdeviceprop_peak_gbs": round(props["peak_hbm_gbs"], 1),
                     "plain_achieved": round(r["plain"]["bu"]["gbs"], 2) if "plain" in r else None},
        "device": {k: props[k] for k in ("arch", "name", "compute_units", "clock_khz", "memory_clock_khz",
                                         "memory_bus_bits", "l2_bytes", "total_bytes")},
        "copy_ceiling": ceiling,
        "cpu_baseline": None,
        "configs": {},
    }
    if args.mode == "all":
        leg22 = run_scale(args_for_scale(args, 22), 22, scale_variants(args, headline=False), ow,
                          64 if ow else 0, full_checks=("split", "plain"), hint_ablation=False)
        out["configs"]["scale22_split_vs_plain"] = leg_summary(leg22, 22)
        out["configs"]["scale22_split_vs_plain"]["split_core_numbering"] = core_numbering(
            args.hubs_first, hub_share_for(args_for_scale(args, 22)))
        out["configs"]["scale22_split_vs_plain"]["tuning"] = leg22["tuned"] or None
        out["configs"]["scale24_batch"] = run_batch_leg(args, 24, 64, max(3, args.steps // 2), 1)
        out["configs"]["serving"] = run_serve_leg(args)
    if ow is not None:
        log("waiting for the CPU oracle")
        ow.finish()
        ow.join()
        res = ow.results.get("scale%d" % scale)
        if res is not None:
            out["cpu_baseline"] = oracle_summary(res, scale, "8 of the 64 timed roots (the first 8)")
            eq = [bool(np.array_equal(a, b)) for a, b in zip(res["levels"], leg["host_levels"])]
            out["cpu_baseline"]["levels_equal_gpu"] = "%d/%d" % (sum(eq), len(eq))
            out["cpu_baseline"]["edges_equal_gpu"] = bool(np.array_equal(np.asarray(res["edges"], np.float64),
                                                                        leg["m_r"][:len(res["edges"])]))
            if res.get("classes") and out["edge_trees"]:
                # Algorithm 8 classes of the whole graph by the oracle, against the device's
                et = out["edge_trees"]
                for h, cls in res["classes"].items():
                    key = "mh%d" % h
                    if key in et:
                        et[key]["oracle_classes"] = cls
                        et[key]["classes_equal_oracle"] = cls == et[key]["classes"]
        else:
            out["cpu_baseline"] = {"error": ow.errors.get("scale%d" % scale, "no result")}
        if args.mode == "all":
            res22 = ow.results.get("scale22")
            if res22 is not None:
                c22 = oracle_summary(res22, 22, "all 64 timed roots")
                eq = [bool(np.array_equal(a, b)) for a, b in zip(res22["levels"], leg22["host_levels"])]
                c22["levels_equal_gpu"] = "%d/%d" % (sum(eq), len(eq))
                out["configs"]["scale22_split_vs_plain"]["cpu_baseline"] = c22
    print(json.dumps(out), flush=True)


def args_for_scale(args, scale):
    a = argparse.Namespace(**vars(args))
    a.scale = scale
    return a


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=["all", "single", "batch", "serve"], default="all",
                    help="all: the scale-26 headline plus the scale-22, batched and serving workloads; "
                         "single / batch / serve: one workload alone")
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
                    help="one root at a time, hubs-first handles: at most n_core / 2^k hubs "
                         "(default: scale - 20, at least 2, so that the hubs' bits fit the LDS)")
    ap.add_argument("--batch-hub-share", type=int, default=5,
                    help="batch and serving handles: at most n_core / 2^k hubs (their pull reads the hubs' masks)")
    ap.add_argument("--no-hint-ablation", dest="hint_ablation", action="store_false",
                    help="skip timing the split handle with the degree-aware probe off")
    ap.add_argument("--form-roots", type=int, default=16,
                    help="roots of the bottom-up form comparison (0: skip it)")
    ap.add_argument("--no-rmzero", dest="rmzero", action="store_false",
                    help="skip the RmZero ablation handle (only isolated vertices removed)")
    ap.add_argument("--handles", type=lambda x: [v for v in x.split(",") if v], default=[],
                    help="one-root-at-a-time legs: build and time only these handles (comma list of split, plain, "
                         "split_caller, plain_hubs, rmzero, mh<h>; the first listed present is the reference); "
                         "default: all. For profiles of one handle's kernels")
    ap.add_argument("--serve-scales", default="18,20,22,24")
    ap.add_argument("--serve-loads", default="0.1,0.25,0.5")
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-seconds", type=float, default=1.5)
    ap.add_argument("--serve-budget-mb", type=int, default=None,
                    help="cap on the serving admission budget (default: free device memory less 4 GiB)")
    ap.add_argument("--serve-solo-max", type=int, default=16,
                    help="while at most this many queries wait for a graph, the first runs single-root")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported "
              "(multi-GPU sharding is described, not implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.mode in ("all", "single"):
        headline(args)
        return
    import torch
    import paper_2009_07463_amd as gt
    gt.load_library(build_if_missing=True)
    torch.cuda.set_device(0)
    if args.mode == "batch":
        scale = args.scale if "--scale" in sys.argv else 24
        res = run_batch_leg(args, scale, args.roots, args.steps, args.warmup)
        b = res["batched"]
        line = {"metric": "queries/s, %d-root batched BFS (scale %d)" % (res["roots"], scale),
                "value": b["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": b["batch_ms"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "u8", "data": "synthetic", "config": {"workload": res["workload"]},
                "roofline": res["pull_roofline"], "cpu_baseline": None, "batch": res}
    else:
        res = run_serve_leg(args)
        line = {"metric": "queries/s and p50/p99 latency, continuous-batching BFS server (scales %s)"
                          % args.serve_scales,
                "value": res["capacity"]["continuous_batching"]["qps"], "unit": "queries/s", "n_gpus": 1,
                "steps": 1, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "u8", "data": "synthetic", "config": {"workload": res["workload"]},
                "cpu_baseline": None, "serve": res}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
