"""Failure paths on the GPU: device memory running out.

The boundary promises GT_E_NOMEM with no handle and no leaked memory when an
allocation fails. Device memory is taken away by one large torch allocation
(leaving a few MiB free), so that the library's own allocations fail in the
ordinary way (hipMalloc returns an error); no kernel faults and nothing is
forced from inside the library.
"""
import numpy as np
import pytest
import torch

import graphgen
import oracle

pytestmark = pytest.mark.gpu

LEAVE = 2 << 20   # device bytes left free while memory is taken


def _gt():
    import paper_2009_07463_amd as gt
    gt.load_library()
    return gt


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_out_of_device_memory_leaves_no_handle_and_no_leak():
    gt = _gt()
    scale = 16
    n = 1 << scale
    src, dst = graphgen.kronecker_edges(scale, 16, seed=60)
    g_ref = oracle.build_csr(n, src, dst)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 4, seed=61)]
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    # load the library's code objects and warm the runtime first
    with gt.Graph(s, d, n, split=True) as warm:
        warm.bfs(roots[0])
        warm.bfs_batch(roots)
    h = gt.Graph(s, d, n, split=True)          # built before memory runs out; no batch state yet
    levels = torch.empty((len(roots), n), dtype=torch.uint8, device="cuda")
    torch.cuda.empty_cache()
    free0 = _free()
    hog_bytes = ((free0 - LEAVE) >> 21) << 21
    print("taking %d of %d free device bytes" % (hog_bytes, free0), flush=True)
    hog = torch.empty(hog_bytes, dtype=torch.uint8, device="cuda")
    try:
        with pytest.raises(gt.GTError) as e:
            gt.Graph(s, d, n, split=True)
        assert e.value.code == gt.GT_E_NOMEM
        free1 = _free()
        for _ in range(10):
            with pytest.raises(gt.GTError) as e:
                gt.Graph(s, d, n, split=False)
            assert e.value.code == gt.GT_E_NOMEM
        assert _free() == free1, "a failed build kept device memory"
        # the batched state of an existing handle does not fit either
        for _ in range(3):
            with pytest.raises(gt.GTError) as e:
                h.bfs_batch(roots, levels)
            assert e.value.code == gt.GT_E_NOMEM
        assert _free() == free1, "a failed batch allocation kept device memory"
    finally:
        del hog
        torch.cuda.empty_cache()
    # with memory back, the same handle allocates its batch state and is correct
    lv = h.bfs_batch(roots, levels).cpu().numpy()
    for i, r in enumerate(roots):
        ref = oracle.bfs(g_ref, r)[1]
        np.testing.assert_array_equal(lv[i], np.where(ref < 0, 255, ref).astype(np.uint8))
    h.close()
