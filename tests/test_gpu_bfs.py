"""GPU parity: gt_bfs (PLAIN and SPLIT) against the CPU oracle, through the C ABI.

Levels must equal the oracle's bit for bit; parents are not unique, so every
parent array must pass the oracle's validator (rules V1-V4) instead.
"""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests.et_table import edge_tree_table

pytestmark = pytest.mark.gpu

LOOP_HOST, LOOP_GRAPH, LOOP_DEVICE = 1, 2, 3
LOOPS = (LOOP_HOST, LOOP_GRAPH, LOOP_DEVICE)


def _gt():
    import paper_2009_07463_amd as gt
    gt.load_library()
    return gt


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


class Case:
    def __init__(self, n, src, dst):
        self.n = n
        self.src = np.ascontiguousarray(src, np.int32)
        self.dst = np.ascontiguousarray(dst, np.int32)
        self.g = oracle.build_csr(n, self.src, self.dst)
        gt = _gt()
        s, d = _dev(self.src), _dev(self.dst)
        self.plain = gt.Graph(s, d, n, split=False)
        self.split = gt.Graph(s, d, n, split=True)
        self.rmzero = gt.Graph(s, d, n, split=True, rmzero=True)
        # nothing split off, hubs first: plain BFS through the relabelling
        self.keepall = gt.Graph(s, d, n, split=True, keep_all=True, hubs_first=True, hub_share=2)

    def handles(self):
        return (("plain", self.plain), ("split", self.split), ("rmzero", self.rmzero), ("keepall", self.keepall))

    def check(self, roots, loops=LOOPS):
        """Every root on the three handles, with the host-driven and the
        device-driven (graph-captured) level loops."""
        for r in roots:
            r = int(r)
            _, lvl_ref = oracle.bfs(self.g, r)
            for name, h in self.handles():
                for loop in loops:
                    print("case n=%d root=%d %s loop=%d" % (self.n, r, name, loop), flush=True)
                    h.set_tuning(loop=loop)
                    p, l = h.bfs(r)
                    torch.cuda.synchronize()
                    p, l = p.cpu().numpy(), l.cpu().numpy()
                    np.testing.assert_array_equal(l, lvl_ref, err_msg="%s loop %d root %d levels" % (name, loop, r))
                    code, bad = oracle.validate(self.g, r, p, l)
                    assert code == 0, "%s loop %d root %d: rule V%d fails at vertex %d" % (name, loop, r, code, bad)

    def close(self):
        for _, h in self.handles():
            h.close()


def rmat_case(scale, ef=16, seed=1):
    src, dst = graphgen.kronecker_edges(scale, ef, seed=seed)
    return Case(1 << scale, src, dst), src, dst


def test_scale16_eight_seeded_roots():
    """Scale 16, edgefactor 16, 8 seeded roots of degree >= 1 (plain and split)."""
    c, src, dst = rmat_case(16)
    roots = graphgen.sample_roots(c.n, src, dst, 8, seed=2)
    c.check(roots)
    info = c.split.info()
    n0, n1, n2 = oracle.degree_counts(c.g)
    assert (info["n_zero"], info["n_leaf"], info["n_core"]) == (n0, n1, n2)
    assert info["n_entries"] == c.g.nnz
    assert c.plain.info()["n_entries"] == c.g.nnz
    assert info["max_degree"] == int(np.diff(c.g.off).max())
    # the RmZero ablation splits off only the isolated vertices
    rz = c.rmzero.info()
    assert (rz["n_zero"], rz["n_leaf"], rz["n_core"]) == (n0, 0, n1 + n2)
    assert rz["n_core_entries"] == c.g.nnz
    # the relabelled plain graph keeps every vertex
    ka = c.keepall.info()
    assert (ka["n_zero"], ka["n_leaf"], ka["n_core"]) == (0, 0, c.n)
    assert ka["n_core_entries"] == c.g.nnz
    c.close()


def test_degrees_match_oracle():
    c, _, _ = rmat_case(14, seed=3)
    for h in (c.plain, c.split):
        d = h.degrees().cpu().numpy()
        np.testing.assert_array_equal(d, np.diff(c.g.off))
    c.close()


def test_root_classes_leaf_pair_isolated_hub():
    c, src, dst = rmat_case(14, seed=4)
    deg = np.diff(c.g.off)
    leaves = np.flatnonzero(deg == 1)
    nbr = c.g.col[c.g.off[leaves]]
    pair_leaves = leaves[deg[nbr] == 1]            # two-vertex components
    core_leaves = leaves[deg[nbr] >= 2]
    roots = [int(np.argmax(deg)), int(np.flatnonzero(deg == 0)[0]), int(core_leaves[0]),
             int(core_leaves[-1]), 0, c.n - 1]
    if pair_leaves.size:
        roots.append(int(pair_leaves[0]))
    c.check(roots)
    c.close()


def test_long_path_many_levels():
    # 3000 levels: many more than one bitmap word and than GT_MAX_LEVELS stats
    n = 3001
    c = Case(n, *graphgen.path(n))
    c.check([0, 1500, n - 1, 7])
    c.close()


@pytest.mark.parametrize("name", ["star", "grid", "complete", "hypercube", "bintree", "cycle"])
def test_structured_graphs(name):
    edges = {"star": (130, graphgen.star(130)), "grid": (23 * 29, graphgen.grid(23, 29)),
             "complete": (70, graphgen.complete(70)), "hypercube": (1 << 9, graphgen.hypercube(9)),
             "bintree": (1000, graphgen.binary_tree(1000)), "cycle": (777, graphgen.cycle(777))}
    n, (src, dst) = edges[name]
    perm = np.random.default_rng(5).permutation(n).astype(np.int32)
    s2, d2 = graphgen.relabel(src, dst, perm)
    c = Case(n, s2, d2)
    c.check([int(perm[0]), int(perm[n // 2]), int(perm[n - 1])])
    c.close()


def test_ragged_sizes_isolated_tail_and_duplicates():
    # n not a multiple of 64; edges repeated, reversed and self-loops
    rng = np.random.default_rng(6)
    n = 1000 + 37
    m = 3000
    src = rng.integers(0, 900, m).astype(np.int32)
    dst = rng.integers(0, 900, m).astype(np.int32)
    src = np.concatenate([src, dst[:500], np.arange(50, dtype=np.int32)])
    dst = np.concatenate([dst, src[:500], np.arange(50, dtype=np.int32)])
    c = Case(n, src, dst)
    c.check([0, 899, n - 1, int(src[0])])
    c.close()


def test_empty_and_tiny_graphs():
    gt = _gt()
    # no edges at all: every root reaches only itself
    c = Case(65, np.zeros(0, np.int32), np.zeros(0, np.int32))
    c.check([0, 63, 64])
    c.close()
    # only self-loops
    c = Case(3, np.array([0, 1, 1], np.int32), np.array([0, 1, 1], np.int32))
    c.check([0, 1, 2])
    c.close()
    # one vertex
    c = Case(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    c.check([0])
    c.close()
    # K2 only
    c = Case(2, np.array([0], np.int32), np.array([1], np.int32))
    c.check([0, 1])
    c.close()


def test_invalid_arguments_are_rejected():
    gt = _gt()
    s = _dev(np.array([0, 5], np.int32))
    d = _dev(np.array([1, 1], np.int32))
    with pytest.raises(gt.GTError) as e:
        gt.Graph(s, d, 4)
    assert e.value.code == gt.GT_E_INVALID
    ok = gt.Graph(_dev(np.array([0], np.int32)), _dev(np.array([1], np.int32)), 4)
    with pytest.raises(gt.GTError) as e:
        ok.bfs(4)
    assert e.value.code == gt.GT_E_INVALID
    with pytest.raises(gt.GTError):
        ok.bfs(-1)
    ok.close()
    with pytest.raises(gt.GTError) as e:   # KEEP_LEAVES only with SPLIT
        gt.Graph(_dev(np.array([0], np.int32)), _dev(np.array([1], np.int32)), 4, split=False, rmzero=True)
    assert e.value.code == gt.GT_E_INVALID


def test_repeated_runs_levels_identical_parents_valid():
    c, src, dst = rmat_case(15, seed=8)
    roots = graphgen.sample_roots(c.n, src, dst, 2, seed=9)
    _, ref = oracle.bfs(c.g, int(roots[0]))
    for it in range(20):
        for h in (c.plain, c.split):
            h.set_tuning(loop=LOOPS[it % 3])
            p, l = h.bfs(int(roots[0]))
            l = l.cpu().numpy()
            np.testing.assert_array_equal(l, ref)
            assert oracle.validate(c.g, int(roots[0]), p.cpu().numpy(), l)[0] == 0
    c.close()


def test_graph_loop_stats_match_host_loop():
    """The device-driven loop takes the same direction decisions and counts
    the same frontier, discovered and scanned vertices as the host loop."""
    c, src, dst = rmat_case(16, seed=12)
    roots = list(graphgen.sample_roots(c.n, src, dst, 4, seed=13))
    for h in (c.plain, c.split):
        for r in roots:
            per = {}
            for loop in LOOPS:
                h.set_tuning(loop=loop)
                h.bfs(int(r))
                per[loop] = [(l["dir"], l["frontier"], l["found"]) + ((l["scanned"],) if l["dir"] == "BU" else ())
                             for l in h.last_stats().levels()]
            assert per[LOOP_HOST] == per[LOOP_GRAPH] == per[LOOP_DEVICE], (r, per)
    c.close()


def test_direction_switch_settings_do_not_change_levels():
    c, src, dst = rmat_case(15, seed=10)
    roots = graphgen.sample_roots(c.n, src, dst, 3, seed=11)
    settings = [
        dict(alpha=1, beta=1000000, bu_lane_edges=1, bu_hint=2, bu_list_div=1, td_flat=2),
        dict(alpha=1000000, beta=1, bu_lane_edges=4, bu_list_div=1 << 30, td_flat=1),
        dict(alpha=2, beta=2, bu_lane_edges=64, bu_hint=1),
        # second probe: degree <= 2 rows settled from the two probes alone
        dict(alpha=2, beta=1000000, bu_lane_edges=1, bu_hint=3, bu_list_div=1),
        dict(alpha=14, beta=24, bu_lane_edges=4, bu_hint=3, bu_list_div=1 << 30),
        # second probe only on levels whose frontier is under 1% of the
        # vertices: alpha = 1 starts bottom-up on a one-vertex frontier
        dict(alpha=1, beta=1000000, bu_lane_edges=2, bu_hint=4, bu_list_div=1 << 30),
        dict(alpha=14, beta=24, bu_lane_edges=4, bu_hint=4, bu_list_div=4),
        # every top-down level after the first claims in the bitmap and its
        # queue is compacted; many rows go to the long-row kernel
        dict(alpha=14, beta=24, bu_lane_edges=2, td_small_edges=1, bu_hub_deg=8, bu_hub_blocks=3,
             bu_blocks=7, td_blocks=5, td_flat=2),
        dict(alpha=14, beta=24, bu_lane_edges=2, td_small_edges=1, bu_hub_deg=8, bu_hub_blocks=3,
             bu_blocks=7, td_blocks=5, td_flat=1, td_hub_deg=256),
        dict(alpha=14, beta=24, bu_lane_edges=12, td_small_edges=100, bu_hub_deg=40, bu_hub_blocks=64,
             bu_blocks=4096, td_blocks=16384, bu_list_div=2),
        dict(alpha=14, beta=24, bu_lane_edges=4, td_small_edges=65536, bu_hub_deg=4096,
             bu_hub_blocks=4096, bu_blocks=4096, td_blocks=16384, bu_list_div=16),
        # device-driven loop: one level per graph replay, long top-down rows
        # cut into chunks from 256 entries on, a tiny grid
        dict(graph_levels=1, td_hub_deg=256, td_blocks=3, td_small_edges=1),
        dict(graph_levels=3, td_hub_deg=100000, td_blocks=16384, td_small_edges=65536),
        dict(graph_levels=8, td_hub_deg=256),
    ]
    for kw in settings:
        for h in (c.plain, c.split):
            h.set_tuning(**kw)
        c.check(roots)
    c.close()


def test_simple_bottom_up_forms_give_the_same_levels():
    """bu_form 2 (Algorithm 5 as written: a thread per 64-vertex word) and 3
    (a thread per vertex), with the hint probe and the LDS hub frontier on
    and off, in the host-driven loop; alpha = 1 sends every level after the
    first bottom-up."""
    c, src, dst = rmat_case(15, seed=10)
    roots = graphgen.sample_roots(c.n, src, dst, 3, seed=11)
    for form in (2, 3):
        for hint in (1, 2):
            for lds in (1, 2):
                for alpha, beta in ((1, 1000000), (14, 24)):
                    print("bu_form %d bu_hint %d bu_lds %d alpha %d" % (form, hint, lds, alpha), flush=True)
                    for _, h in c.handles():
                        h.set_tuning(bu_form=form, bu_hint=hint, bu_lds=lds, alpha=alpha, beta=beta)
                    c.check(roots, loops=(LOOP_HOST,))
    c.close()
    # ragged n (the last bitmap word part padding), repeated edges and
    # self-loops, every level after the first bottom-up
    rng = np.random.default_rng(16)
    n = 1000 + 37
    src = rng.integers(0, 900, 3000).astype(np.int32)
    dst = rng.integers(0, 900, 3000).astype(np.int32)
    src = np.concatenate([src, dst[:500], np.arange(50, dtype=np.int32)])
    dst = np.concatenate([dst, src[:500], np.arange(50, dtype=np.int32)])
    c = Case(n, src, dst)
    for form in (2, 3):
        print("ragged bu_form %d" % form, flush=True)
        for _, h in c.handles():
            h.set_tuning(bu_form=form, alpha=1, beta=1000000)
        c.check([0, 899, n - 1, int(src[0])], loops=(LOOP_HOST,))
    c.close()


def test_scale22_split_vs_plain_two_roots():
    """Scale 22, edgefactor 16 (the split-vs-plain workload), 2 seeded roots."""
    c, src, dst = rmat_case(22)
    roots = graphgen.sample_roots(c.n, src, dst, 2, seed=2)
    c.check(roots)
    info = c.split.info()
    assert info["n_core"] + info["n_leaf"] + info["n_zero"] == c.n
    c.close()


# ------------------------------------------------------------------ MH > 0
ET_CI, ET_CE, ET_TI, ET_TL, ET_VZ = 0, 1, 2, 3, 4


def _forest_on_cycle(seed):
    """A cycle (the core) with random trees hung on it, plus tree
    components of their own (paths, stars, pairs) and isolated vertices:
    TREE_INTERNAL vertices of several heights, and trees without a core."""
    rng = np.random.default_rng(seed)
    src, dst = [], []
    n = 0
    cyc = list(range(12))
    for i in cyc:
        src.append(i)
        dst.append((i + 1) % 12)
    n = 12
    for _ in range(60):                       # trees hanging from the cycle or from each other
        p = int(rng.integers(0, n))
        src.append(p)
        dst.append(n)
        n += 1
    for length in (2, 3, 5, 8):               # path components
        for i in range(length - 1):
            src.append(n + i)
            dst.append(n + i + 1)
        n += length
    for i in range(1, 6):                     # a star component
        src.append(n)
        dst.append(n + i)
    n += 6
    n += 5                                    # isolated vertices
    perm = rng.permutation(n).astype(np.int32)
    s2, d2 = graphgen.relabel(np.array(src, np.int32), np.array(dst, np.int32), perm)
    return n, s2, d2


def _et_cases():
    out = [("forest", *_forest_on_cycle(70)), ("forest2", *_forest_on_cycle(71))]
    n = 1 << 11
    s, d = graphgen.kronecker_edges(11, 2, seed=72)          # sparse: many small trees
    out.append(("rmat11ef2", n, s, d))
    s, d = graphgen.random_gnp(400, 1.6 / 400, seed=73)
    out.append(("gnp400", 400, s, d))
    s, d = graphgen.path(301)
    out.append(("path301", 301, s, d))
    s, d = graphgen.binary_tree(255)
    out.append(("bintree255", 255, s, d))
    # triangle with legs of three and four edges: MH 0, 1, 2 and unlimited
    # classify it differently (the oracle's hand-worked pin)
    out.append(("spider", 10, np.array([0, 1, 2, 0, 3, 4, 0, 6, 7, 8], np.int32),
                np.array([1, 2, 0, 3, 4, 5, 6, 7, 8, 9], np.int32)))
    return out


@pytest.mark.parametrize("mh", [1, 2, 255])
def test_edge_trees_classes_levels_and_parents(mh):
    """MH > 0 (Algorithm 8 rounds, Algorithm 10 tree pass, roots inside
    trees of Algorithm 9): vertex classes equal the oracle's Algorithm 8,
    levels equal the oracle BFS from every kind of root, parents pass V1-V4."""
    gt = _gt()
    for name, n, src, dst in _et_cases():
        g = oracle.build_csr(n, np.asarray(src, np.int32), np.asarray(dst, np.int32))
        types = oracle.etvca(g, -1 if mh == 255 else mh)
        h = gt.Graph(_dev(src), _dev(dst), n, split=True, mh=mh)
        info = h.info()
        cnt = np.bincount(types, minlength=5)
        assert info["n_core"] == cnt[ET_CI] + cnt[ET_CE], name
        assert info["n_core_edge"] == cnt[ET_CE], name
        assert info["n_tree_internal"] == cnt[ET_TI], name
        assert info["n_leaf"] == cnt[ET_TI] + cnt[ET_TL], name
        assert info["n_zero"] == cnt[ET_VZ], name
        # roots: every tree-internal vertex (up to 40), some leaves, core and isolated vertices
        rng = np.random.default_rng(n)
        roots = []
        for t in (ET_TI, ET_TL, ET_CE, ET_CI, ET_VZ):
            ids = np.flatnonzero(types == t)
            if ids.size:
                roots += [int(x) for x in rng.choice(ids, min(ids.size, 40 if t == ET_TI else 6), replace=False)]
        for loop in LOOPS:
            h.set_tuning(loop=loop)
            for r in roots:
                _, ref = oracle.bfs(g, r)
                print("mh=%d %s loop=%d root=%d type=%d" % (mh, name, loop, r, types[r]), flush=True)
                p, lv = h.bfs(r)
                p, lv = p.cpu().numpy(), lv.cpu().numpy()
                np.testing.assert_array_equal(lv, ref, err_msg="%s mh %d loop %d root %d levels" % (name, mh, loop, r))
                code, bad = oracle.validate(g, r, p, lv)
                assert code == 0, "%s mh %d loop %d root %d: rule V%d fails at vertex %d" % (name, mh, loop, r,
                                                                                             code, bad)
        h.close()


def test_edge_trees_at_scale14_match_oracle_classes_and_levels():
    gt = _gt()
    c, src, dst = rmat_case(14, seed=74)
    c.close()
    for mh in (1, 2):
        types = oracle.etvca(c.g, mh)
        h = gt.Graph(_dev(src), _dev(dst), c.n, split=True, mh=mh)
        info = h.info()
        assert info["n_tree_internal"] == int((types == ET_TI).sum())
        assert info["n_core_edge"] == int((types == ET_CE).sum())
        ti = np.flatnonzero(types == ET_TI)
        roots = [int(x) for x in ti[:6]] + [int(r) for r in graphgen.sample_roots(c.n, src, dst, 4, seed=75)]
        for r in roots:
            _, ref = oracle.bfs(c.g, r)
            p, lv = h.bfs(r)
            lv = lv.cpu().numpy()
            np.testing.assert_array_equal(lv, ref)
            assert oracle.validate(c.g, r, p.cpu().numpy(), lv)[0] == 0
        h.close()


@pytest.mark.parametrize("mh", [0, 1, 2, 255])
def test_edge_tree_table_matches_oracle_components(mh):
    """Edge trees per core-edge vertex (Table 3 columns: count, total, max,
    min) on the edge-tree test graphs and a scale-14 R-MAT, against
    connected components of the oracle's tree vertices."""
    gt = _gt()
    cases = list(_et_cases())
    s14, d14 = graphgen.kronecker_edges(14, 16, seed=74)
    cases.append(("rmat14", 1 << 14, s14, d14))
    for name, n, src, dst in cases:
        g = oracle.build_csr(n, np.asarray(src, np.int32), np.asarray(dst, np.int32))
        types = oracle.etvca(g, -1 if mh == 255 else mh)
        h = gt.Graph(_dev(src), _dev(dst), n, split=True, mh=mh)
        info = h.info()
        got = (info["n_edge_trees"], info["edge_tree_vertices"], info["edge_tree_max"], info["edge_tree_min"])
        assert got == edge_tree_table(g, types), "%s mh %d" % (name, mh)
        h.close()


def _u8(level):
    assert level.max() <= 254
    return np.where(level < 0, 255, level).astype(np.uint8)


def _tree_roots(types, rng, k_ti=30):
    roots = []
    for t, k in ((ET_TI, k_ti), (ET_TL, 10), (ET_CE, 6), (ET_CI, 6), (ET_VZ, 2)):
        ids = np.flatnonzero(types == t)
        if ids.size:
            roots += [int(x) for x in rng.choice(ids, min(ids.size, k), replace=False)]
    return roots[:64]


@pytest.mark.parametrize("mh", [1, 2, 255])
def test_edge_trees_batch_sessions_and_reconstruction(mh):
    """MH > 0 in the batched BFS, in sessions and in parent reconstruction:
    every slot's levels equal the oracle's (roots inside trees included) and
    reconstructed parents pass V1-V4."""
    from tests.test_gpu_batch import run_session
    gt = _gt()
    for name, n, src, dst in _et_cases()[:4]:
        g = oracle.build_csr(n, np.asarray(src, np.int32), np.asarray(dst, np.int32))
        types = oracle.etvca(g, -1 if mh == 255 else mh)
        h = gt.Graph(_dev(src), _dev(dst), n, split=True, mh=mh)
        roots = _tree_roots(types, np.random.default_rng(n + mh))
        refs = [oracle.bfs(g, r)[1] for r in roots]
        for ms_loop in (1, 3, 2):        # host, device-launched, graph-captured (the default, kept)
            print("mh=%d %s batch of %d, ms_loop %d" % (mh, name, len(roots), ms_loop), flush=True)
            h.set_tuning(ms_loop=ms_loop)
            lv = h.bfs_batch(roots)
            got = lv.cpu().numpy()
            for i, r in enumerate(roots):
                np.testing.assert_array_equal(got[i], _u8(refs[i]),
                                              err_msg="%s mh %d loop %d root %d" % (name, mh, ms_loop, r))
        for i, r in enumerate(roots[:12]):
            p = h.reconstruct_parent(r, lv[i].contiguous()).cpu().numpy()
            code, bad = oracle.validate(g, r, p, refs[i].astype(np.int32))
            assert code == 0, "%s mh %d root %d: rule V%d fails at vertex %d" % (name, mh, r, code, bad)
        plan = np.random.default_rng(mh).integers(0, 6, len(roots)).tolist()
        mixed = run_session(h, n, roots, plan, slots=8)
        for i, r in enumerate(roots):
            np.testing.assert_array_equal(mixed[i], _u8(refs[i]), err_msg="session %s mh %d root %d" % (name, mh, r))
        h.close()


def test_edge_tree_handle_needs_split():
    gt = _gt()
    n, src, dst = _forest_on_cycle(76)
    with pytest.raises(gt.GTError) as e:
        gt.Graph(_dev(src), _dev(dst), n, split=False, mh=2)
    assert e.value.code == gt.GT_E_INVALID


def test_edge_trees_degenerate_graphs():
    """MH > 0 on graphs with no tree at all, with nothing but trees, with no
    edges, and with one vertex: levels equal the oracle's."""
    gt = _gt()
    cases = [("complete", 40, *graphgen.complete(40)), ("cycle", 50, *graphgen.cycle(50)),
             ("star", 30, *graphgen.star(30)), ("k2", 2, np.array([0], np.int32), np.array([1], np.int32)),
             ("empty", 9, np.zeros(0, np.int32), np.zeros(0, np.int32)),
             ("one", 1, np.zeros(0, np.int32), np.zeros(0, np.int32))]
    for name, n, src, dst in cases:
        g = oracle.build_csr(n, np.asarray(src, np.int32), np.asarray(dst, np.int32))
        for mh in (1, 255):
            h = gt.Graph(_dev(src), _dev(dst), n, split=True, mh=mh)
            roots = sorted(set([0, n - 1, n // 2]))
            for r in roots:
                _, ref = oracle.bfs(g, r)
                p, lv = h.bfs(r)
                lv = lv.cpu().numpy()
                np.testing.assert_array_equal(lv, ref, err_msg="%s mh %d root %d" % (name, mh, r))
                assert oracle.validate(g, r, p.cpu().numpy(), lv)[0] == 0
            got = h.bfs_batch(roots).cpu().numpy()
            for i, r in enumerate(roots):
                np.testing.assert_array_equal(got[i], _u8(oracle.bfs(g, r)[1]), err_msg="%s batch %d" % (name, r))
            h.close()


@pytest.mark.parametrize("mh,rmzero,share", [(0, False, 0), (2, False, 0), (0, True, 0), (0, False, 2), (0, False, 6)])
def test_hubs_first_core(mh, rmzero, share):
    """GT_BUILD_HUBS_FIRST: the highest-degree core vertices numbered first
    (hubs are a class of their own in the output pass's groups); levels,
    parents, batched levels and reconstructed parents are checked as for the
    caller-order core, in every level loop, also on the RmZero handle."""
    gt = _gt()
    cases = [("rmat13", 1 << 13, *graphgen.kronecker_edges(13, 16, seed=80)), _et_cases()[0]]
    s15, d15 = graphgen.kronecker_edges(15, 16, seed=82)
    cases.append(("rmat15", 1 << 15, s15, d15))   # several tiles of class groups with hubs
    for name, n, src, dst in cases:
        g = oracle.build_csr(n, np.asarray(src, np.int32), np.asarray(dst, np.int32))
        h = gt.Graph(_dev(src), _dev(dst), n, split=True, mh=mh, hubs_first=True, rmzero=rmzero, hub_share=share)
        assert h.info()["n_core"] > 0
        roots = [int(r) for r in graphgen.sample_roots(n, np.asarray(src, np.int32), np.asarray(dst, np.int32), 6,
                                                       seed=81)]
        deg = np.diff(g.off)
        roots += [int(np.argmax(deg)), int(np.flatnonzero(deg == 1)[0])] if (deg == 1).any() else [int(np.argmax(deg))]
        refs = [oracle.bfs(g, r)[1] for r in roots]
        for loop in LOOPS:
            h.set_tuning(loop=loop)
            for r, ref in zip(roots, refs):
                p, lv = h.bfs(r)
                lv = lv.cpu().numpy()
                np.testing.assert_array_equal(lv, ref, err_msg="%s mh %d loop %d root %d" % (name, mh, loop, r))
                code, bad = oracle.validate(g, r, p.cpu().numpy(), lv)
                assert code == 0, "%s root %d: rule V%d fails at vertex %d" % (name, r, code, bad)
        lvb = h.bfs_batch(roots)
        got = lvb.cpu().numpy()
        for i, r in enumerate(roots):
            np.testing.assert_array_equal(got[i], _u8(refs[i]), err_msg="%s batch root %d" % (name, r))
            p = h.reconstruct_parent(r, lvb[i].contiguous()).cpu().numpy()
            assert oracle.validate(g, r, p, refs[i].astype(np.int32))[0] == 0
        h.close()
