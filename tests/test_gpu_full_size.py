"""Parity at the benchmark sizes, in the configurations bench.py times
(autotuned handles): Kronecker scale 26 one root at a time, and scale 24 with
64 roots in one batch. The CPU oracle needs about a minute per root at these
sizes, so the outputs are checked by properties that hold at any size,
evaluated with plain torch ops over the generated edge list (independent of
the library's CSR, relabelling and kernels):

  V1  level[root] = 0 (and parent[root] = root);
  V2  parent[v] = -1 exactly where level[v] = -1;
  V3  a reached v != root has parent p with {p, v} an edge and
      level[p] = level[v] - 1;
  V4  every edge joins two unreached vertices or two reached ones whose
      levels differ by at most 1.

V1, V4 and "every reached v != root has a neighbour one level closer" make
the levels exactly the hop distances from the root (V4 bounds them above
along a shortest path, the closer neighbours give a path of that length), and
V4 makes the reached set exactly the root's component. Where there are no
parents (batched uint8 levels), that neighbour condition is checked on its
own."""
import pytest
import torch

import graphgen

pytestmark = pytest.mark.gpu

CHUNK = 1 << 27


def _gt():
    import paper_2009_07463_amd as gt
    gt.load_library()
    return gt


def check_levels(s, d, n, root, level, parent=None):
    """V1-V4 (V3 only with parents) for int32 levels on the GPU; s, d: the
    generated edges (int32 device tensors, duplicates and self-loops kept)."""
    assert int(level[root]) == 0
    has_lower = torch.zeros(n, dtype=torch.bool, device=level.device)
    par_edge = torch.zeros(n, dtype=torch.bool, device=level.device) if parent is not None else None
    for i in range(0, s.numel(), CHUNK):
        a = s[i:i + CHUNK].long()
        b = d[i:i + CHUNK].long()
        la, lb = level[a], level[b]
        assert torch.equal(la >= 0, lb >= 0), "V4: an edge from a reached to an unreached vertex"
        assert bool(((la - lb).abs() <= 1).all()), "V4: an edge spans more than one level"
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
    assert bool(has_lower[reached].all()), "a reached vertex without a neighbour one level closer"
    if parent is not None:
        assert int(parent[root]) == root
        assert torch.equal(parent >= 0, level >= 0), "V2"
        v = reached.nonzero().squeeze(1)
        assert bool((level[parent[v].long()] == level[v] - 1).all()), "V3: parent not one level closer"
        assert bool(par_edge[v].all()), "V3: parent is not a neighbour"
    return int((level >= 0).sum())


def u8_to_i32(lv):
    out = lv.to(torch.int32)
    out[out == 255] = -1
    return out


def special_roots(s, d, n):
    """A highest-count vertex and a vertex of degree exactly 1 (it appears in
    a single non-self-loop edge), from the edge list alone."""
    cnt = torch.zeros(n, dtype=torch.int64, device=s.device)
    for i in range(0, s.numel(), CHUNK):
        a, b = s[i:i + CHUNK], d[i:i + CHUNK]
        keep = a != b
        cnt += torch.bincount(a[keep].long(), minlength=n)
        cnt += torch.bincount(b[keep].long(), minlength=n)
    hub = int(torch.argmax(cnt))
    leaf = int(torch.nonzero(cnt == 1)[0])
    return hub, leaf


def test_scale26_single_source_split_and_plain():
    """The bench workload: scale 26, edgefactor 16, seed 1, autotuned split
    (hubs first, as the bench builds it) and plain handles; two of its roots
    plus a hub and a degree-1 root."""
    gt = _gt()
    scale, n = 26, 1 << 26
    src, dst = graphgen.kronecker_edges(scale, 16, seed=1)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 2, seed=2)]
    tune_roots = graphgen.sample_roots(n, src, dst, 16, seed=102)
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    del src, dst
    hub, leaf = special_roots(s, d, n)
    roots += [hub, leaf]
    split = gt.Graph(s, d, n, split=True, hubs_first=True, hub_share=2)
    plain = gt.Graph(s, d, n, split=False)
    for h in (split, plain):
        h.autotune(tune_roots)
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    level = torch.empty(n, dtype=torch.int32, device="cuda")
    level_plain = torch.empty_like(level)
    parent_plain = torch.empty_like(parent)
    for r in roots:
        print("scale 26 root %d" % r, flush=True)
        split.bfs(r, parent, level)
        plain.bfs(r, parent_plain, level_plain)
        torch.cuda.synchronize()
        reached = check_levels(s, d, n, r, level, parent)
        check_levels(s, d, n, r, level_plain, parent_plain)
        assert torch.equal(level, level_plain), "split and plain levels differ for root %d" % r
        assert reached >= 2
    split.close()
    plain.close()


def test_scale24_batch_of_64_and_reconstructed_parents():
    """The batch workload: scale 24, 64 roots (seed 2) in one batch on the
    autotuned hubs-first handle; every slot's levels, parents reconstructed
    for 8 of them, and two slots against the one-root path."""
    gt = _gt()
    scale, n = 24, 1 << 24
    src, dst = graphgen.kronecker_edges(scale, 16, seed=1)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 64, seed=2)]
    tune_roots = graphgen.sample_roots(n, src, dst, 64, seed=102)
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    del src, dst
    g = gt.Graph(s, d, n, split=True, hubs_first=True, hub_share=5)
    g.autotune(tune_roots, batch=True)
    lv = g.bfs_batch(roots)
    torch.cuda.synchronize()
    for i, r in enumerate(roots):
        check_levels(s, d, n, r, u8_to_i32(lv[i]))
    for i in range(0, 64, 8):
        print("scale 24 reconstruct slot %d root %d" % (i, roots[i]), flush=True)
        p = g.reconstruct_parent(roots[i], lv[i].contiguous())
        check_levels(s, d, n, roots[i], u8_to_i32(lv[i]), p)
    one = gt.Graph(s, d, n, split=True)
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    level = torch.empty(n, dtype=torch.int32, device="cuda")
    for i in (0, 37):
        one.bfs(roots[i], parent, level)
        assert torch.equal(u8_to_i32(lv[i]), level)
    one.close()
    g.close()
