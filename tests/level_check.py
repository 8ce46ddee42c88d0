"""Checks of a BFS result that hold at any size, by plain torch ops over the
generated edge list (duplicates and self-loops kept). They are independent of
the library's CSR, relabelling and kernels, and run on CPU or GPU tensors.

  V1  level[root] = 0, and no other vertex has level 0 (parent[root] = root);
  V2  parent[v] = -1 exactly where level[v] = -1 (and no level below -1);
  V3  a reached v != root has parent p with {p, v} an edge and
      level[p] = level[v] - 1;
  V4  every edge joins two unreached vertices or two reached ones whose
      levels differ by at most 1.

V4 bounds every level above by the hop distance (induction along a shortest
path from the root), and makes the reached set a union of components. "Every
reached v != root has a neighbour one level closer", applied down to level 0,
where only the root sits, gives a path to the root of length level[v], so the
levels are at least the hop distances. Together the levels are exactly the hop
distances and the reached set is exactly the root's component. Where there are
no parents (batched uint8 levels), the neighbour condition is checked on its
own; with parents, V3 implies it.

These are the Graph500 validation rules (the spanning-tree requirement of
Section 5.3) written over an edge list instead of a CSR.
"""
import torch

CHUNK = 1 << 27


class LevelCheckError(AssertionError):
    pass


def _need(cond, msg):
    if not cond:
        raise LevelCheckError(msg)


def check_levels(s, d, n, root, level, parent=None, chunk=CHUNK):
    """V1-V4 (V3 only with parents) for int32 levels; s, d: int32 tensors of
    the generated edges on the same device as level. Raises LevelCheckError
    naming the first rule that fails; returns the number of reached vertices."""
    _need(level.numel() == n, "level has %d entries, expected %d" % (level.numel(), n))
    _need(int(level[root]) == 0, "V1: level[root] = %d" % int(level[root]))
    _need(int((level == 0).sum()) == 1, "V1: a vertex other than the root has level 0")
    _need(int((level < -1).sum()) == 0, "a level below -1")
    has_lower = torch.zeros(n, dtype=torch.bool, device=level.device)
    par_edge = torch.zeros(n, dtype=torch.bool, device=level.device) if parent is not None else None
    for i in range(0, s.numel(), chunk):
        a = s[i:i + chunk].long()
        b = d[i:i + chunk].long()
        la, lb = level[a], level[b]
        _need(torch.equal(la >= 0, lb >= 0), "V4: an edge from a reached to an unreached vertex")
        _need(bool(((la - lb).abs() <= 1).all()), "V4: an edge spans more than one level")
        m = (lb >= 1) & (la == lb - 1)
        has_lower[b[m]] = True
        m = (la >= 1) & (lb == la - 1)
        has_lower[a[m]] = True
        if parent is not None:
            m = parent[b] == a
            par_edge[b[m]] = True
            m = parent[a] == b
            par_edge[a[m]] = True
        del a, b, la, lb, m
    reached = level > 0
    _need(bool(has_lower[reached].all()), "a reached vertex without a neighbour one level closer")
    if parent is not None:
        _need(parent.numel() == n, "parent has %d entries, expected %d" % (parent.numel(), n))
        _need(int(parent[root]) == root, "V1: parent[root] = %d" % int(parent[root]))
        _need(torch.equal(parent >= 0, level >= 0), "V2: parent and level disagree on reached vertices")
        _need(int((parent < -1).sum()) == 0 and int((parent >= n).sum()) == 0, "V2: parent out of range")
        v = reached.nonzero().squeeze(1)
        _need(bool((level[parent[v].long()] == level[v] - 1).all()), "V3: parent not one level closer")
        _need(bool(par_edge[v].all()), "V3: parent is not a neighbour")
    return int((level >= 0).sum())


def u8_to_i32(lv):
    """uint8 batch levels (255 = unreached) as int32 levels (-1 = unreached)."""
    out = lv.to(torch.int32)
    out[out == 255] = -1
    return out
