"""Failure paths on the GPU: device memory running out.

The boundary promises GT_E_NOMEM with no handle and no leaked memory when an
allocation fails. The device's own free memory cannot be exhausted reliably
(the driver may evict allocations to host memory instead of failing), so the
library's memory cap (gt_set_memory_limit) stands in for a full device: an
allocation past the cap fails in the same code path as a failed hipMalloc.
gt_memory_in_use counts every byte the library holds, so a leak shows
exactly.
"""
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


def test_out_of_device_memory_leaves_no_handle_and_no_leak():
    gt = _gt()
    scale = 16
    n = 1 << scale
    src, dst = graphgen.kronecker_edges(scale, 16, seed=60)
    g_ref = oracle.build_csr(n, src, dst)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 4, seed=61)]
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    levels = torch.empty((len(roots), n), dtype=torch.uint8, device="cuda")
    base = gt.memory_in_use()
    h = gt.Graph(s, d, n, split=True)          # no batch state yet
    held = gt.memory_in_use() - base
    assert held >= h.info()["device_bytes"] > 0
    try:
        for split in (True, False):
            for frac in (0.0, 0.05, 0.2):      # the build fails at different allocations
                gt.set_memory_limit(base + held + max(1, int(frac * held)))
                before = gt.memory_in_use()
                with pytest.raises(gt.GTError) as e:
                    gt.Graph(s, d, n, split=split)
                assert e.value.code == gt.GT_E_NOMEM
                assert gt.memory_in_use() == before, "a failed build kept device memory"
        # the batched state of an existing handle does not fit either
        gt.set_memory_limit(base + held + 4096)
        for _ in range(2):
            with pytest.raises(gt.GTError) as e:
                h.bfs_batch(roots, levels)
            assert e.value.code == gt.GT_E_NOMEM
            assert gt.memory_in_use() == base + held, "a failed batch allocation kept device memory"
        # the single-root path needs nothing new
        p, l = h.bfs(roots[0])
        np.testing.assert_array_equal(l.cpu().numpy(), oracle.bfs(g_ref, roots[0])[1])
    finally:
        gt.set_memory_limit(0)
    # with the cap gone, the same handle allocates its batch state and is correct
    lv = h.bfs_batch(roots, levels).cpu().numpy()
    for i, r in enumerate(roots):
        ref = oracle.bfs(g_ref, r)[1]
        np.testing.assert_array_equal(lv[i], np.where(ref < 0, 255, ref).astype(np.uint8))
    h.close()
    assert gt.memory_in_use() == base
    with pytest.raises(gt.GTError) as e:
        gt.set_memory_limit(-1)
    assert e.value.code == gt.GT_E_INVALID
