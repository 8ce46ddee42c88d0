"""GPU: the autotuner (gt_autotune) through the C ABI. Tuning changes only
speed: under the chosen knobs every level array still equals the CPU
oracle's, and a second call takes the knobs from the cache file."""
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


def test_autotune_keeps_results_and_uses_the_cache(tmp_path):
    gt = _gt()
    scale = 14
    n = 1 << scale
    src, dst = graphgen.kronecker_edges(scale, 16, seed=31)
    g = oracle.build_csr(n, src, dst)
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 6, seed=32)]
    cache = str(tmp_path / "tuning.txt")
    sigs = []
    for split in (True, False):
        print("autotune split=%d" % split, flush=True)
        h = gt.Graph(_dev(src), _dev(dst), n, split=split)
        tun, rep = h.autotune(roots, cache_path=cache, batch=True)
        assert rep["from_cache"] == 0 and rep["trials"] >= 10
        assert rep["ms_best"] <= rep["ms_start"] and rep["ms_batch_best"] <= rep["ms_batch_start"]
        assert h.tuning().as_dict() == tun
        sigs.append(rep["signature"])
        for r in roots[:3]:
            p, l = h.bfs(r)
            _, ref = oracle.bfs(g, r)
            l = l.cpu().numpy()
            np.testing.assert_array_equal(l, ref)
            assert oracle.validate(g, r, p.cpu().numpy(), l)[0] == 0
        lv = h.bfs_batch(roots).cpu().numpy()
        for i, r in enumerate(roots):
            ref = oracle.bfs(g, r)[1]
            np.testing.assert_array_equal(lv[i], np.where(ref < 0, 255, ref).astype(np.uint8))
        h.set_tuning(alpha=3, bu_blocks=123, loop=gt.GT_LOOP_HOST)
        tun2, rep2 = h.autotune(roots, cache_path=cache)
        assert rep2["from_cache"] == 1 and rep2["trials"] == 0 and tun2 == tun
        assert h.tuning().as_dict() == tun
        h.close()
    lines = open(cache).read().splitlines()
    assert len(lines) == 2 and sigs[0] != sigs[1]
    assert all(l.split()[0] in sigs for l in lines)


def test_autotune_rejects_bad_arguments():
    gt = _gt()
    src, dst = graphgen.path(50)
    h = gt.Graph(_dev(src), _dev(dst), 50)
    for roots in ([], list(range(65)), [50], [-1]):
        with pytest.raises(gt.GTError) as e:
            h.autotune(roots)
        assert e.value.code == gt.GT_E_INVALID
    h.close()
