"""The size-independent level checker (tests/level_check.py) on CPU tensors:
it accepts the oracle's results and rejects planted mistakes, including the
ones that only the "only the root has level 0" rule catches."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from tests.level_check import LevelCheckError, check_levels, u8_to_i32


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32))


@pytest.fixture(scope="module")
def rmat():
    scale = 10
    n = 1 << scale
    src, dst = graphgen.kronecker_edges(scale, 16, seed=5)
    g = oracle.build_csr(n, src, dst)
    root = int(graphgen.sample_roots(n, src, dst, 1, seed=6)[0])
    parent, level = oracle.bfs(g, root)
    return n, _t(src), _t(dst), g, root, parent, level


def test_accepts_oracle_result(rmat):
    n, s, d, g, root, parent, level = rmat
    reached = check_levels(s, d, n, root, _t(level), _t(parent), chunk=1000)
    assert reached == int((level >= 0).sum())
    assert check_levels(s, d, n, root, _t(level)) == reached


def test_second_level_zero_vertex_is_rejected():
    # path r - a - w labelled 0, 1, 0: every edge spans one level, a has a
    # closer neighbour, parents are edges; only "root alone at level 0" fails
    s, d = _t([0, 1]), _t([1, 2])
    with pytest.raises(LevelCheckError, match="other than the root"):
        check_levels(s, d, 3, 0, _t([0, 1, 0]), _t([0, 0, 1]))
    with pytest.raises(LevelCheckError, match="other than the root"):
        check_levels(s, d, 3, 0, _t([0, 1, 0]))
    # the correct answer passes
    assert check_levels(s, d, 3, 0, _t([0, 1, 2]), _t([0, 0, 1])) == 3


def test_too_shallow_without_closer_neighbour_is_rejected():
    # path r - a - b labelled 0, 1, 1: V4 holds on both edges, b has no
    # neighbour at level 0
    s, d = _t([0, 1]), _t([1, 2])
    with pytest.raises(LevelCheckError, match="closer"):
        check_levels(s, d, 3, 0, _t([0, 1, 1]))


def _mutations(n, g, root, parent, level):
    deg = np.diff(g.off)
    reached = np.nonzero((level > 0))[0]
    v = int(reached[len(reached) // 2])
    out = []
    lv = level.copy(); lv[v] += 1
    out.append(("level one too deep", parent, lv))
    lv = level.copy(); lv[v] = -1
    pa = parent.copy(); pa[v] = -1
    out.append(("reached vertex dropped", pa, lv))
    iso = int(np.nonzero(deg == 0)[0][0])
    lv = level.copy(); lv[iso] = 1
    pa = parent.copy(); pa[iso] = root
    out.append(("isolated vertex reached", pa, lv))
    pa = parent.copy()
    nbrs = set(g.col[g.off[v]:g.off[v + 1]].tolist())
    far = next(u for u in reached.tolist() if u not in nbrs and level[u] == level[v] - 1)
    pa[v] = far
    out.append(("parent not a neighbour", pa, level))
    pa = parent.copy()
    same = [u for u in g.col[g.off[v]:g.off[v + 1]].tolist() if level[u] == level[v]]
    if same:
        pa[v] = same[0]
        out.append(("parent on the same level", pa, level))
    pa = parent.copy(); pa[root] = v
    out.append(("root parent", pa, level))
    lv = level.copy(); lv[root] = 1
    out.append(("root level", parent, lv))
    return out


def test_rejects_planted_mistakes(rmat):
    n, s, d, g, root, parent, level = rmat
    for name, pa, lv in _mutations(n, g, root, parent, level):
        with pytest.raises(LevelCheckError):
            check_levels(s, d, n, root, _t(lv), _t(pa))
            pytest.fail("accepted: %s" % name)


def test_u8_levels_round_trip(rmat):
    n, s, d, g, root, parent, level = rmat
    u8 = torch.from_numpy(np.where(level < 0, 255, level).astype(np.uint8))
    lv = u8_to_i32(u8)
    assert torch.equal(lv, _t(level))
    assert check_levels(s, d, n, root, lv) == int((level >= 0).sum())
