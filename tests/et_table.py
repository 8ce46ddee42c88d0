"""Edge trees grouped by their core-edge vertex (the columns of the paper's
Table 3) from the oracle's Algorithm 8 classes, by connected components of
the tree vertices (scipy): the reference the GPU build's counts are checked
against. Test infrastructure."""
import numpy as np

import oracle


def edge_tree_table(g, types):
    """The paper's Table 3 columns from the oracle's Algorithm 8 classes:
    tree vertices (TREE_INTERNAL, TREE_LEAF) split into connected components
    of the subgraph they induce, each component credited to the core vertex
    it touches (none: a tree without a core). Returns (trees, vertices, max,
    min) over the core vertices credited with at least one vertex."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    tree = (types == oracle.TREE_INTERNAL) | (types == oracle.TREE_LEAF)
    core = (types == oracle.CORE_INTERNAL) | (types == oracle.CORE_EDGE)
    rows = np.repeat(np.arange(g.n), np.diff(g.off))
    cols = g.col
    keep = tree[rows] & tree[cols]
    a = csr_matrix((np.ones(int(keep.sum())), (rows[keep], cols[keep])), shape=(g.n, g.n))
    ncomp, lab = connected_components(a, directed=False)
    size = np.bincount(lab[tree], minlength=ncomp)
    touched = {}
    m = tree[rows] & core[cols]
    for t, c in zip(rows[m], cols[m]):
        touched.setdefault(int(lab[t]), set()).add(int(c))
    per = {}
    for comp, cs in touched.items():
        assert len(cs) == 1, "a tree component touches %d core vertices" % len(cs)
        c = cs.pop()
        per[c] = per.get(c, 0) + int(size[comp])
    v = np.array(list(per.values()), np.int64)
    if v.size == 0:
        return 0, 0, 0, 0
    return int(v.size), int(v.sum()), int(v.max()), int(v.min())
