"""Parity at the benchmark sizes, in the configurations bench.py times
(autotuned handles): Kronecker scale 26 one root at a time, and scale 24 with
64 roots in one batch. The CPU oracle needs about a minute per root at these
sizes, so the outputs are checked by the properties of tests/level_check.py
(V1-V4 plus "every reached vertex has a neighbour one level closer" and
"only the root has level 0"), which make the levels exactly the hop
distances at any size; they are evaluated with plain torch ops over the
generated edge list, independent of the library's CSR, relabelling and
kernels."""
import pytest
import torch

import graphgen
from tests.level_check import CHUNK, check_levels, u8_to_i32

pytestmark = pytest.mark.gpu


def _gt():
    import paper_2009_07463_amd as gt
    gt.load_library()
    return gt


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
