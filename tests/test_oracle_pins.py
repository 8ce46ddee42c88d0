"""Pins of the CPU oracle to facts outside itself (no GPU).

Each test ties an oracle function to something independent of its own code:
all-pairs distances by boolean matrix powers, closed-form distances of
structured graphs, scipy's BFS and CSR construction, the paper's Table 2
counts (through the closed-form R-MAT expectation) and mutations that a
correct validator must reject.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import graphgen
import oracle
from tests.rmat_stats import degree01_expectation

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- helpers ---

def dense_adjacency(n, src, dst):
    a = np.zeros((n, n), dtype=bool)
    for s, d in zip(src.tolist(), dst.tolist()):
        if s != d:
            a[s, d] = True
            a[d, s] = True
    return a


def all_pairs_by_matrix_powers(a):
    """dist[r, v] = smallest k with ((I + A)^k)[r, v] > 0, else -1."""
    n = a.shape[0]
    reach = np.eye(n, dtype=bool)
    dist = np.where(reach, 0, -1).astype(np.int64)
    am = a.astype(np.int64)
    for k in range(1, n + 1):
        reach = reach | ((reach.astype(np.int64) @ am) > 0)
        newly = reach & (dist == -1)
        if not newly.any():
            break
        dist[newly] = k
    return dist


def check_all_roots(n, src, dst, expected_dist):
    g = oracle.build_csr(n, src, dst)
    for r in range(n):
        parent, level = oracle.bfs(g, r)
        np.testing.assert_array_equal(level, expected_dist[r], err_msg="root %d" % r)
        assert oracle.validate(g, r, parent, level) == (0, -1)


# ----------------------------------------------------------- brute force ---

def small_graphs():
    cases = []
    for seed in range(6):
        n = [1, 2, 7, 20, 41, 64][seed]
        cases.append(("gnp%d" % seed, n) + graphgen.random_gnp(n, 0.08 if n > 10 else 0.4, seed))
    for s in (3, 4, 5, 6):
        src, dst = graphgen.kronecker_edges(s, 4, seed=11 + s)
        cases.append(("rmat%d" % s, 1 << s, src, dst))
    # forest of K2s and isolated vertices, with repeated and reversed edges
    cases.append(("k2s", 12, np.array([0, 2, 4, 3, 0], np.int32), np.array([1, 3, 5, 2, 1], np.int32)))
    return cases


@pytest.mark.parametrize("name,n,src,dst", small_graphs(), ids=lambda x: x if isinstance(x, str) else "")
def test_levels_equal_matrix_power_distances(name, n, src, dst):
    a = dense_adjacency(n, src, dst)
    check_all_roots(n, src, dst, all_pairs_by_matrix_powers(a))


# ----------------------------------------------------------- closed forms ---

def _perm(n, seed):
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


def _closed_form_cases():
    out = []
    n = 17
    i = np.arange(n)
    out.append(("path", n, graphgen.path(n), lambda r: np.abs(i - r)))
    out.append(("cycle", n, graphgen.cycle(n), lambda r: np.minimum(np.abs(i - r), n - np.abs(i - r))))
    out.append(("star", 9, graphgen.star(9),
                lambda r: np.where(np.arange(9) == r, 0, np.where((np.arange(9) == 0) | (r == 0), 1, 2))))
    out.append(("complete", 8, graphgen.complete(8), lambda r: (np.arange(8) != r).astype(int)))
    a, b = 3, 5
    side = np.arange(a + b) < a
    out.append(("bipartite", a + b, graphgen.complete_bipartite(a, b),
                lambda r: np.where(np.arange(a + b) == r, 0, np.where(side == side[r], 2, 1))))
    rows, cols = 5, 7
    rr, cc = np.divmod(np.arange(rows * cols), cols)
    out.append(("grid", rows * cols, graphgen.grid(rows, cols),
                lambda r: np.abs(rr - rr[r]) + np.abs(cc - cc[r])))
    d = 5
    hv = np.arange(1 << d)
    out.append(("hypercube", 1 << d, graphgen.hypercube(d),
                lambda r: np.array([bin(int(x) ^ r).count("1") for x in hv])))
    nt = 31
    depth = np.floor(np.log2(np.arange(nt) + 1)).astype(int)

    def tree_dist(r):
        res = np.empty(nt, int)
        for v in range(nt):
            x, y = r, v
            while x != y:
                if x > y:
                    x = (x - 1) // 2
                else:
                    y = (y - 1) // 2
            res[v] = depth[r] + depth[v] - 2 * depth[x]
        return res
    out.append(("bintree", nt, graphgen.binary_tree(nt), tree_dist))
    return out


@pytest.mark.parametrize("name,n,edges,dist", _closed_form_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_closed_form_distances_under_relabelling(name, n, edges, dist):
    src, dst = edges
    perm = _perm(n, 3)              # old -> new label
    s2, d2 = graphgen.relabel(src, dst, perm)
    g = oracle.build_csr(n, s2, d2)
    for r in range(n):
        parent, level = oracle.bfs(g, int(perm[r]))
        expect = np.empty(n, np.int64)
        expect[perm] = dist(r)
        np.testing.assert_array_equal(level, expect, err_msg="%s root %d" % (name, r))
        assert oracle.validate(g, int(perm[r]), parent, level) == (0, -1)


def test_disjoint_union_unreached_is_minus_one():
    s1, d1 = graphgen.path(5)
    s2, d2 = graphgen.cycle(4)
    src = np.concatenate([s1, s2 + 5]).astype(np.int32)
    dst = np.concatenate([d1, d2 + 5]).astype(np.int32)
    n = 5 + 4 + 3  # three isolated vertices at the end
    g = oracle.build_csr(n, src, dst)
    parent, level = oracle.bfs(g, 2)
    np.testing.assert_array_equal(level, [2, 1, 0, 1, 2] + [-1] * 7)
    assert (parent[5:] == -1).all()
    parent, level = oracle.bfs(g, 11)
    np.testing.assert_array_equal(level, [-1] * 11 + [0])
    assert parent[11] == 11


# ------------------------------------------------------------ scipy cross ---

def scipy_csr(n, src, dst):
    keep = src != dst
    r = np.concatenate([src[keep], dst[keep]])
    c = np.concatenate([dst[keep], src[keep]])
    a = sp.csr_matrix((np.ones(r.size, np.int8), (r, c)), shape=(n, n))
    a.sum_duplicates()
    a.sort_indices()
    return a


@pytest.mark.parametrize("scale", [10, 14])
def test_csr_equals_scipy(scale):
    src, dst = graphgen.kronecker_edges(scale, 16, seed=5)
    n = 1 << scale
    g = oracle.build_csr(n, src, dst)
    a = scipy_csr(n, src, dst)
    np.testing.assert_array_equal(g.off, a.indptr.astype(np.int64))
    np.testing.assert_array_equal(g.col, a.indices.astype(np.int32))


@pytest.mark.parametrize("scale", [12, 16])
def test_levels_equal_scipy_bfs(scale):
    src, dst = graphgen.kronecker_edges(scale, 16, seed=7)
    n = 1 << scale
    g = oracle.build_csr(n, src, dst)
    a = scipy_csr(n, src, dst)
    roots = graphgen.sample_roots(n, src, dst, 4, seed=8)
    d = csgraph.shortest_path(a, unweighted=True, indices=roots)
    for i, r in enumerate(roots):
        parent, level = oracle.bfs(g, int(r))
        expect = np.where(np.isinf(d[i]), -1, d[i]).astype(np.int64)
        np.testing.assert_array_equal(level, expect)
        assert oracle.validate(g, int(r), parent, level) == (0, -1)
        assert oracle.reached_edges(g, level) * 2 == int(np.diff(g.off)[level >= 0].sum())


def test_reached_edges_closed_forms():
    """TEPS numerator (half the degree sum of the reached vertices of the
    simple graph) against edge counts known in closed form; the reached sets
    are written by hand, so no BFS is involved."""
    # K_7 given with every edge twice (once reversed) and a self-loop at each
    # vertex: 7 * 6 / 2 edges whatever the root
    ks, kd = graphgen.complete(7)
    src = np.concatenate([ks, kd, np.arange(7)]).astype(np.int32)
    dst = np.concatenate([kd, ks, np.arange(7)]).astype(np.int32)
    g = oracle.build_csr(7, src, dst)
    assert oracle.reached_edges(g, np.zeros(7, np.int32)) == 21
    # path 0-1-2-3-4 (4 edges), disjoint cycle 5..10 (6 edges), isolated 11
    ps, pd = graphgen.path(5)
    cs, cd = graphgen.cycle(6)
    src = np.concatenate([ps, cs + 5]).astype(np.int32)
    dst = np.concatenate([pd, cd + 5]).astype(np.int32)
    g = oracle.build_csr(12, src, dst)
    in_path = np.array([0] * 5 + [-1] * 7, np.int32)
    in_cycle = np.array([-1] * 5 + [0] * 6 + [-1], np.int32)
    alone = np.array([-1] * 11 + [0], np.int32)
    assert oracle.reached_edges(g, in_path) == 4
    assert oracle.reached_edges(g, in_cycle) == 6
    assert oracle.reached_edges(g, alone) == 0
    # star K_{1,5} with a repeated spoke: 5 edges
    ss, sd = graphgen.star(6)
    src = np.concatenate([ss, ss[:1]]).astype(np.int32)
    dst = np.concatenate([sd, sd[:1]]).astype(np.int32)
    g = oracle.build_csr(6, src, dst)
    assert oracle.reached_edges(g, np.zeros(6, np.int32)) == 5


def test_csr_hand_case_duplicates_and_loops():
    # edges: 0-1 twice (once reversed), loop at 2, 2-3, loop at 4 only
    src = np.array([0, 1, 2, 2, 4, 3], np.int32)
    dst = np.array([1, 0, 2, 3, 4, 2], np.int32)
    g = oracle.build_csr(6, src, dst)
    np.testing.assert_array_equal(g.off, [0, 1, 2, 3, 4, 4, 4])
    np.testing.assert_array_equal(g.col, [1, 0, 3, 2])
    assert oracle.degree_counts(g) == (2, 4, 0)
    with pytest.raises(ValueError):
        oracle.build_csr(4, np.array([0, 5], np.int32), np.array([1, 1], np.int32))


# ------------------------------------------------------ validator mutants ---

@pytest.fixture(scope="module")
def grid_result():
    src, dst = graphgen.grid(6, 6)
    g = oracle.build_csr(36 + 2, src, dst)   # vertices 36, 37 isolated
    parent, level = oracle.bfs(g, 0)
    return g, parent, level


def test_validator_accepts_alternative_parents(grid_result):
    g, parent, level = grid_result
    p = parent.copy()
    v = 7  # (1,1): parents (0,1)=1 or (1,0)=6 are both one level closer
    p[v] = 1 if p[v] == 6 else 6
    assert oracle.validate(g, 0, p, level) == (0, -1)


@pytest.mark.parametrize("mutation,rule", [
    ("root_parent", 1), ("root_level", 1), ("parent_without_level", 2), ("level_without_parent", 2),
    ("parent_not_neighbour", 3), ("level_off_by_one", 3), ("skip_component_vertex", 4),
    ("reach_isolated", 2),
])
def test_validator_rejects_planted_mistakes(grid_result, mutation, rule):
    g, parent, level = grid_result
    p, l = parent.copy(), level.copy()
    if mutation == "root_parent":
        p[0] = 1
    elif mutation == "root_level":
        l[0] = 1
    elif mutation == "parent_without_level":
        p[36] = 0
    elif mutation == "level_without_parent":
        l[36] = 3
    elif mutation == "parent_not_neighbour":
        p[35] = 0
    elif mutation == "level_off_by_one":
        l[35] += 1
    elif mutation == "skip_component_vertex":
        p[35] = -1
        l[35] = -1
    elif mutation == "reach_isolated":
        p[37] = 36
    code, _ = oracle.validate(g, 0, p, l)
    assert code == rule


def test_validator_rejects_shortcut_free_but_too_deep_levels():
    # path 0-1-2-3 plus edge 0-3: the levels of the plain path are consistent
    # with the parent rule but violate rule 4 on edge {0,3}
    src = np.array([0, 1, 2, 0], np.int32)
    dst = np.array([1, 2, 3, 3], np.int32)
    g = oracle.build_csr(4, src, dst)
    code, _ = oracle.validate(g, 0, np.array([0, 0, 1, 2], np.int32), np.array([0, 1, 2, 3], np.int32))
    assert code == 4


# --------------------------------------------- Table 2 and degree classes ---

def _golden_table2():
    rows = {}
    with open(os.path.join(HERE, "golden", "table2_scale26.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            mh, ci, ce, ti, tl, vz = map(int, line.split())
            rows[mh] = dict(CI=ci, CE=ce, TI=ti, TL=tl, VZ=vz)
    return rows


def test_table2_rows_sum_to_two_to_the_26():
    for row in _golden_table2().values():
        assert sum(row.values()) == 1 << 26


def test_table2_matches_closed_form_rmat_expectation():
    """The paper's scale-26 VZ and TL counts agree with plain R-MAT (no noise)."""
    ez, el, sz, sl = degree01_expectation(26)
    row = _golden_table2()[0]
    assert abs(row["VZ"] - ez) < 3 * sz
    assert abs(row["TL"] - el) < 3 * sl


@pytest.mark.parametrize("scale,seed", [(14, 1), (16, 1), (18, 3)])
def test_oracle_degree_classes_match_closed_form(scale, seed):
    src, dst = graphgen.kronecker_edges(scale, 16, seed=seed)
    g = oracle.build_csr(1 << scale, src, dst)
    n0, n1, n2 = oracle.degree_counts(g)
    ez, el, sz, sl = degree01_expectation(scale)
    assert abs(n0 - ez) < 5 * sz, (n0, ez, sz)
    assert abs(n1 - el) < 5 * sl, (n1, el, sl)
    assert n0 + n1 + n2 == 1 << scale


# ------------------------------------------------------------ Algorithm 8 ---

def _types(n, edges, mh):
    g = oracle.build_csr(n, *edges)
    return oracle.etvca(g, mh).tolist()


CI, CE, TI, TL, VZ = (oracle.CORE_INTERNAL, oracle.CORE_EDGE, oracle.TREE_INTERNAL,
                      oracle.TREE_LEAF, oracle.VERTEX_ZERO)


def test_etvca_hand_graphs():
    # triangle 0-1-2 with pendant 3 on vertex 2, and isolated vertex 4
    tri = (np.array([0, 1, 2, 2], np.int32), np.array([1, 2, 0, 3], np.int32))
    assert _types(5, tri, 0) == [CI, CI, CE, TL, VZ]
    assert _types(5, tri, -1) == [CI, CI, CE, TL, VZ]
    # K2: both ends are leaves at any height
    k2 = (np.array([0], np.int32), np.array([1], np.int32))
    assert _types(2, k2, 0) == [TL, TL]
    # path 0-1-2-3-4: MH=0 ends are leaves, 1 and 3 lose a neighbour
    p5 = graphgen.path(5)
    assert _types(5, p5, 0) == [TL, CE, CI, CE, TL]
    # MH=1: 1 and 3 fall to degree 1 and become tree-internal; 2 is then an
    # edge vertex of the core (its degree changed)
    assert _types(5, p5, 1) == [TL, TI, CE, TI, TL]
    # star: the centre keeps core status at MH=0 even with core degree 0
    st = graphgen.star(5)
    assert _types(5, st, 0) == [CE, TL, TL, TL, TL]
    assert _types(5, st, 1) == [TI, TL, TL, TL, TL]


def test_etvca_spider_heights_differ():
    """Triangle 0-1-2 with two legs hanging from vertex 0: 0-3-4-5 (three
    edges) and 0-6-7-8-9 (four). Each peeling round removes the current
    ends of the legs, so MH 0, 1, 2 and unlimited give four different
    answers, worked out by hand from Algorithm 8's rounds:
      round 0 marks the leaves 5, 9; round 1 marks 4, 8; round 2 marks 3, 7;
      round 3 marks 6; round 4 marks nothing (0 keeps 1 and 2).
    CORE_EDGE is a core vertex whose degree changed."""
    src = np.array([0, 1, 2, 0, 3, 4, 0, 6, 7, 8], np.int32)
    dst = np.array([1, 2, 0, 3, 4, 5, 6, 7, 8, 9], np.int32)
    e = (src, dst)
    assert _types(10, e, 0) == [CI, CI, CI, CI, CE, TL, CI, CI, CE, TL]
    assert _types(10, e, 1) == [CI, CI, CI, CE, TI, TL, CI, CE, TI, TL]
    assert _types(10, e, 2) == [CE, CI, CI, TI, TI, TL, CE, TI, TI, TL]
    assert _types(10, e, -1) == [CE, CI, CI, TI, TI, TL, TI, TI, TI, TL]
    assert _types(10, e, 3) == _types(10, e, -1)


def test_etvca_mh0_agrees_with_degree_counts():
    src, dst = graphgen.kronecker_edges(12, 16, seed=4)
    g = oracle.build_csr(1 << 12, src, dst)
    t = oracle.etvca(g, 0)
    n0, n1, n2 = oracle.degree_counts(g)
    assert (t == VZ).sum() == n0 and (t == TL).sum() == n1
    assert ((t == CI) | (t == CE)).sum() == n2
    deg = np.diff(g.off)
    # CE at MH=0: a core vertex with at least one degree-1 neighbour
    leaf = deg == 1
    has_leaf_nbr = np.zeros(g.n, bool)
    rows = np.repeat(np.arange(g.n), deg)
    has_leaf_nbr[rows[leaf[g.col]]] = True
    np.testing.assert_array_equal(t == CE, (deg >= 2) & has_leaf_nbr)


def test_edge_tree_table_on_hand_graphs():
    """Table 3 columns (trees, tree vertices, largest, smallest) of the test
    reference on graphs whose edge trees are known by construction."""
    from tests.et_table import edge_tree_table

    def table(n, edges, mh):
        g = oracle.build_csr(n, *edges)
        return edge_tree_table(g, oracle.etvca(g, mh))
    tri = (np.array([0, 1, 2, 2], np.int32), np.array([1, 2, 0, 3], np.int32))
    assert table(5, tri, 0) == (1, 1, 1, 1)          # pendant 3 on vertex 2
    p5 = graphgen.path(5)
    assert table(5, p5, 0) == (2, 2, 1, 1)           # ends on 1 and on 3
    assert table(5, p5, 1) == (1, 4, 4, 4)           # both halves hang from vertex 2
    assert table(5, p5, -1) == (0, 0, 0, 0)          # a path is a tree without a core
    st = graphgen.star(5)
    assert table(5, st, 0) == (1, 4, 4, 4)           # four leaves on the centre
    assert table(5, st, 1) == (0, 0, 0, 0)           # the centre joins the tree
    k2 = (np.array([0], np.int32), np.array([1], np.int32))
    assert table(2, k2, 0) == (0, 0, 0, 0)


@pytest.mark.parametrize("mh", [0, 1, 2])
def test_edge_tree_table_counts_every_core_edge_vertex(mh):
    """Every CORE_EDGE vertex lost a neighbour to a tree, and a tree touches
    at most one core vertex, so there are as many edge trees as CORE_EDGE
    vertices, and they hold every tree vertex except the trees without a
    core."""
    from tests.et_table import edge_tree_table
    src, dst = graphgen.kronecker_edges(12, 4, seed=6)
    g = oracle.build_csr(1 << 12, src, dst)
    t = oracle.etvca(g, mh)
    trees, total, mx, mn = edge_tree_table(g, t)
    assert trees == int((t == CE).sum()) > 0
    assert 1 <= mn <= mx <= total <= int(((t == TI) | (t == TL)).sum())


# ------------------------------------------------------------- generator ---

def test_generator_is_deterministic_and_chunkable():
    a = graphgen.kronecker_edges(12, 16, seed=9)
    b = graphgen.kronecker_edges(12, 16, seed=9)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    part = graphgen.kronecker_edges(12, 16, seed=9, first=1000, count=5000)
    np.testing.assert_array_equal(part[0], a[0][1000:6000])
    c = graphgen.kronecker_edges(12, 16, seed=10)
    assert not np.array_equal(a[0], c[0])


def test_scramble_is_a_bijection():
    for s in (1, 5, 10):
        img = {graphgen.scramble(s, 3, x) for x in range(1 << s)}
        assert img == set(range(1 << s))


def test_generator_bit_frequencies():
    """Unscrambled: each src bit is 1 with probability C+D, each dst bit with B+D,
    and both bits 0 with probability A."""
    src, dst = graphgen.kronecker_edges(10, 64, seed=2, permute=False)
    m = src.size
    for b in range(10):
        sb = (src >> b) & 1
        db = (dst >> b) & 1
        tol = 5 * np.sqrt(0.25 / m)
        assert abs(sb.mean() - 0.24) < tol
        assert abs(db.mean() - 0.24) < tol
        assert abs(((sb == 0) & (db == 0)).mean() - 0.57) < tol
        assert abs(((sb == 1) & (db == 1)).mean() - 0.05) < tol


def test_roots_have_degree_at_least_one():
    src, dst = graphgen.kronecker_edges(12, 16, seed=1)
    g = oracle.build_csr(1 << 12, src, dst)
    roots = graphgen.sample_roots(1 << 12, src, dst, 64, seed=2)
    assert len(set(roots.tolist())) == 64
    assert (np.diff(g.off)[roots] >= 1).all()
