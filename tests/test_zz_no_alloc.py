"""gt_bfs_static (the single-source BFS without allocation) against gt_bfs.

gt_bfs_static runs the same traversal as gt_bfs with its working memory
taken from the library's static per-GPU array. Its levels must equal
gt_bfs's and the CPU oracle's bit for bit; parents are not unique, so each
parent array must pass the oracle's validator (rules V1-V4). The calls run
back to back, the second on a smaller graph, so the second call starts from
what the first one left in the shared array. Neither the library's device
memory (gt_memory_in_use) nor torch's changes during a call.
"""
import gc

import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _gt():
    import paper_2009_07463_amd as gt
    gt.load_library()
    return gt


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def _static_and_reference(gt, h, g_ref, root):
    """gt_bfs_static of root, checked against gt_bfs and the oracle."""
    n = h.n
    parent = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    level = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    # no garbage collection inside the window: a collection could free
    # tensors left by earlier tests and move torch's count
    gc.collect()
    gc.disable()
    try:
        lib_before = gt.memory_in_use()
        torch_before = torch.cuda.memory_allocated()
        h.bfs_static(root, parent, level)
        torch.cuda.synchronize()
        lib_after = gt.memory_in_use()
        torch_after = torch.cuda.memory_allocated()
    finally:
        gc.enable()
    assert lib_after == lib_before, "gt_bfs_static changed the library's device memory"
    assert torch_after == torch_before
    p_ref, l_ref = h.bfs(root)
    torch.cuda.synchronize()
    l = level.cpu().numpy()
    p = parent.cpu().numpy()
    np.testing.assert_array_equal(l, l_ref.cpu().numpy(), err_msg="levels differ from gt_bfs (root %d)" % root)
    np.testing.assert_array_equal(l, oracle.bfs(g_ref, root)[1], err_msg="levels differ from the oracle")
    code, bad = oracle.validate(g_ref, root, p, l)
    assert code == 0, "root %d: rule V%d fails at vertex %d" % (root, code, bad)
    code, bad = oracle.validate(g_ref, root, p_ref.cpu().numpy(), l)
    assert code == 0


def _special_roots(n, src, dst):
    """A leaf root and an isolated root of the graph (where it has them)."""
    deg = np.diff(oracle.build_csr(n, src, dst).off)
    out = []
    leaves = np.flatnonzero(deg == 1)
    if len(leaves):
        out.append(int(leaves[len(leaves) // 2]))
    zeros = np.flatnonzero(deg == 0)
    if len(zeros):
        out.append(int(zeros[-1]))
    return out


def test_bfs_static_matches_gt_bfs_on_two_calls_the_second_smaller():
    gt = _gt()
    cases = []
    for scale, seed in ((15, 71), (10, 72)):          # second call: a smaller graph
        n = 1 << scale
        src, dst = graphgen.kronecker_edges(scale, 16, seed=seed)
        roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 2, seed=seed + 100)]
        cases.append((n, src, dst, roots + _special_roots(n, src, dst)))
    for n, src, dst, roots in cases:
        g_ref = oracle.build_csr(n, src, dst)
        s, d = _dev(src), _dev(dst)
        for kw in (dict(split=True), dict(split=False), dict(split=True, hubs_first=True, hub_share=2)):
            with gt.Graph(s, d, n, **kw) as h:
                for r in roots:
                    print("gt_bfs_static n=%d root=%d %s" % (n, r, kw), flush=True)
                    _static_and_reference(gt, h, g_ref, r)


def test_bfs_static_ragged_and_tiny_graphs():
    gt = _gt()
    # a path with a pendant, a triangle, an isolated tail; 67 vertices: one
    # full bitmap word and a ragged one
    src = np.array([0, 1, 2, 3, 5, 6, 7, 10, 20, 64], np.int32)
    dst = np.array([1, 2, 3, 4, 6, 7, 5, 11, 21, 65], np.int32)
    n = 67
    g_ref = oracle.build_csr(n, src, dst)
    for split in (True, False):
        with gt.Graph(_dev(src), _dev(dst), n, split=split) as h:
            for r in (0, 2, 4, 5, 10, 64, 66):
                _static_and_reference(gt, h, g_ref, r)


def test_bfs_static_refuses_what_it_cannot_serve():
    gt = _gt()
    # working memory past the static array: a PLAIN handle of 2^22 vertices
    n = 1 << 22
    src = np.arange(0, 1000, dtype=np.int32)
    dst = src + 1
    parent = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    level = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with gt.Graph(_dev(src), _dev(dst), n, split=False) as h:
        with pytest.raises(gt.GTError) as e:
            h.bfs_static(0, parent, level)
        assert e.value.code == gt.GT_E_INVALID
        assert "static array holds" in str(e.value)
        torch.cuda.synchronize()
        assert int((parent != -7).sum()) == 0 and int((level != -7).sum()) == 0, "a refused call wrote outputs"
        with pytest.raises(gt.GTError) as e:
            h.bfs_static(n, parent, level)
        assert e.value.code == gt.GT_E_INVALID
    # edge-tree handles are not served
    m = 1 << 10
    s2, d2 = graphgen.kronecker_edges(10, 16, seed=73)
    with gt.Graph(_dev(s2), _dev(d2), m, split=True, mh=1) as h:
        with pytest.raises(gt.GTError) as e:
            h.bfs_static(0, parent, level)
        assert e.value.code == gt.GT_E_UNSUPPORTED
