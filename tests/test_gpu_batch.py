"""GPU parity of the batched multi-source BFS, parent reconstruction and
continuous-batching sessions, through the C ABI, against the CPU oracle."""
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


def u8(level):
    """Oracle int32 levels as the batched uint8 encoding (255 = unreached)."""
    out = np.where(level < 0, 255, level)
    assert out.max() <= 255
    return out.astype(np.uint8)


@pytest.fixture(scope="module")
def rmat14():
    gt = _gt()
    src, dst = graphgen.kronecker_edges(14, 16, seed=21)
    n = 1 << 14
    g = oracle.build_csr(n, src, dst)
    s, d = _dev(src), _dev(dst)
    handles = {"plain": gt.Graph(s, d, n, split=False), "split": gt.Graph(s, d, n, split=True),
               "rmzero": gt.Graph(s, d, n, split=True, rmzero=True),
               # the core numbering the batch and serving benches use
               "split_hubs": gt.Graph(s, d, n, split=True, hubs_first=True, hub_share=5)}
    yield n, src, dst, g, handles
    for h in handles.values():
        h.close()


def special_roots(g):
    deg = np.diff(g.off)
    leaves = np.flatnonzero(deg == 1)
    nbr = g.col[g.off[leaves]]
    out = [int(np.argmax(deg)), int(np.flatnonzero(deg == 0)[0]), int(leaves[deg[nbr] >= 2][0])]
    pairs = leaves[deg[nbr] == 1]
    if pairs.size:
        out.append(int(pairs[0]))
    return out


MS_LOOPS = (1, 2, 3)   # host-driven steps, graph-captured steps, device-driven launches


def test_batch64_matches_oracle(rmat14):
    n, src, dst, g, handles = rmat14
    roots = list(graphgen.sample_roots(n, src, dst, 56, seed=22)) + special_roots(g)
    roots += [roots[0], roots[1]]                # duplicates are legal
    roots = [int(r) for r in roots[:64]]
    ref = np.stack([u8(oracle.bfs(g, r)[1]) for r in roots])
    for name, h in handles.items():
        for ms_loop in MS_LOOPS:
            print("batch 64 %s ms_loop %d" % (name, ms_loop), flush=True)
            h.set_tuning(ms_loop=ms_loop)
            lv = h.bfs_batch(roots).cpu().numpy()
            for i, r in enumerate(roots):
                np.testing.assert_array_equal(lv[i], ref[i], err_msg="%s loop %d slot %d root %d" % (name, ms_loop,
                                                                                                   i, r))
            st = h.last_stats()
            assert st.root_class == -1 and st.n_levels >= 1
        h.set_tuning(ms_loop=2)


def test_batch_graph_replays_across_calls_and_step_counts(rmat14):
    """The captured steps are replayed for batches of other roots, sizes and
    graph lengths (steps per replay), and give the same answers as the
    host-driven loop each time."""
    n, src, dst, g, handles = rmat14
    h = handles["split_hubs"]
    for j, (k, steps) in enumerate(((64, 8), (3, 8), (17, 4), (64, 1), (1, 12))):
        roots = [int(r) for r in graphgen.sample_roots(n, src, dst, k, seed=90 + j)]
        h.set_tuning(ms_loop=1)
        ref = h.bfs_batch(roots).cpu().numpy()
        h.set_tuning(ms_loop=2, graph_levels=steps)
        got = h.bfs_batch(roots).cpu().numpy()
        np.testing.assert_array_equal(got, ref, err_msg="k=%d steps=%d" % (k, steps))
        got2 = h.bfs_batch(roots).cpu().numpy()
        np.testing.assert_array_equal(got2, ref)
    h.set_tuning(ms_loop=2, graph_levels=8)


@pytest.mark.parametrize("k", [1, 5, 33])
def test_batch_partial_slots(rmat14, k):
    n, src, dst, g, handles = rmat14
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, k, seed=30 + k)]
    for name, h in handles.items():
        lv = h.bfs_batch(roots).cpu().numpy()
        assert lv.shape == (k, n)
        for i, r in enumerate(roots):
            np.testing.assert_array_equal(lv[i], u8(oracle.bfs(g, r)[1]))


def test_batch_push_only_and_pull_heavy_settings(rmat14):
    n, src, dst, g, handles = rmat14
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 20, seed=40)]
    ref = [u8(oracle.bfs(g, r)[1]) for r in roots]
    # alpha 1: push whenever possible; 10^6: pull after the first step.
    # ms_alpha > alpha: growing top-down slots join a step's pull early.
    for alpha, ms_alpha in ((1, 1), (1000000, 1), (1, 1000000), (14, 1000000)):
        for h in handles.values():
            for ms_loop in MS_LOOPS:
                h.set_tuning(alpha=alpha, ms_alpha=ms_alpha, ms_blocks=37, ms_loop=ms_loop)
                lv = h.bfs_batch(roots).cpu().numpy()
                for i in range(len(roots)):
                    np.testing.assert_array_equal(lv[i], ref[i])
            h.set_tuning(alpha=14, ms_alpha=50, ms_blocks=4096, ms_loop=2)


def test_reconstructed_parents_validate(rmat14):
    n, src, dst, g, handles = rmat14
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 6, seed=23)] + special_roots(g)
    for name, h in handles.items():
        lv = h.bfs_batch(roots)
        for i, r in enumerate(roots):
            p = h.reconstruct_parent(r, lv[i].contiguous()).cpu().numpy()
            l32 = lv[i].cpu().numpy().astype(np.int32)
            l32[l32 == 255] = -1
            code, bad = oracle.validate(g, r, p, l32)
            assert code == 0, "%s root %d: V%d at %d" % (name, r, code, bad)
            # first neighbour (ascending caller id) one level closer: the same
            # on every handle, whatever its core numbering
            if name != "plain":
                p_plain = handles["plain"].reconstruct_parent(r, lv[i].contiguous()).cpu().numpy()
                np.testing.assert_array_equal(p, p_plain)


def test_batch_depth_limit_is_reported():
    gt = _gt()
    n = 600
    src, dst = graphgen.path(n)
    with gt.Graph(_dev(src), _dev(dst), n, split=True) as h:
        for ms_loop in MS_LOOPS:
            h.set_tuning(ms_loop=ms_loop)
            with pytest.raises(gt.GTError) as e:
                h.bfs_batch([0])
            assert e.value.code == gt.GT_E_DEPTH
        # a root in the middle needs only 300 levels -> still too deep; a
        # short path works
    m = 200
    src, dst = graphgen.path(m)
    g = oracle.build_csr(m, src, dst)
    with gt.Graph(_dev(src), _dev(dst), m, split=True) as h:
        for ms_loop in MS_LOOPS:
            h.set_tuning(ms_loop=ms_loop)
            lv = h.bfs_batch([0, 100, 199]).cpu().numpy()
            for i, r in enumerate([0, 100, 199]):
                np.testing.assert_array_equal(lv[i], u8(oracle.bfs(g, r)[1]))


def test_batch_invalid_arguments(rmat14):
    gt = _gt()
    n, src, dst, g, handles = rmat14
    h = handles["split"]
    with pytest.raises(gt.GTError):
        h.bfs_batch([])
    with pytest.raises(gt.GTError):
        h.bfs_batch(list(range(65)))
    with pytest.raises(gt.GTError):
        h.bfs_batch([n])


def run_session(h, n, roots, admit_plan, slots=64):
    """admit_plan[i] = step at which roots[i] is admitted. Returns results."""
    gt = _gt()
    s = gt.Session(h, slots=slots)
    outs = {}
    pending = sorted(range(len(roots)), key=lambda i: admit_plan[i])
    step = 0
    running = {}
    while pending or running:
        while pending and admit_plan[pending[0]] <= step:
            i = pending[0]
            buf = torch.empty(n, dtype=torch.uint8, device="cuda")
            slot = s.try_admit(roots[i], buf)
            if slot is None:
                break
            running[slot] = (i, buf)
            pending.pop(0)
        done = s.step()
        for slot in list(running):
            if (done >> slot) & 1:
                i, buf = running.pop(slot)
                outs[i] = buf.cpu().numpy()
        step += 1
        assert step < 10000
    s.close()
    return outs


def test_session_results_equal_alone_and_in_the_mix(rmat14):
    n, src, dst, g, handles = rmat14
    roots = [int(r) for r in graphgen.sample_roots(n, src, dst, 40, seed=24)] + special_roots(g)
    rng = np.random.default_rng(25)
    plan = rng.integers(0, 12, len(roots)).tolist()
    for name, h in handles.items():
        print("session %s" % name, flush=True)
        mixed = run_session(h, n, roots, plan, slots=16)   # slots are reused
        for i, r in enumerate(roots):
            alone = h.bfs_batch([r]).cpu().numpy()[0]
            np.testing.assert_array_equal(mixed[i], alone, err_msg="%s root %d" % (name, r))
            np.testing.assert_array_equal(mixed[i], u8(oracle.bfs(g, r)[1]))


def test_session_busy_when_full(rmat14):
    gt = _gt()
    n, src, dst, g, handles = rmat14
    s = gt.Session(handles["split"], slots=2)
    bufs = [torch.empty(n, dtype=torch.uint8, device="cuda") for _ in range(3)]
    assert s.try_admit(1, bufs[0]) is not None
    assert s.try_admit(2, bufs[1]) is not None
    assert s.try_admit(3, bufs[2]) is None
    assert s.active() == 2
    for _ in range(200):
        s.step()
        if s.active() == 0:
            break
    assert s.active() == 0
    s.close()


def test_server_on_gpu_results_match_oracle():
    """The continuous-batching server with the GPU executor: every query's
    levels equal the oracle's, whatever it was batched with."""
    gt = _gt()
    from paper_2009_07463_amd import serve
    graphs, pools, refs = {}, {}, {}
    # caller-order and hubs-first handles (the served bench builds hubs first)
    for name, scale, hubs in (("a", 12, False), ("b", 14, True), ("c", 18, True)):
        n = 1 << scale
        src, dst = graphgen.kronecker_edges(scale, 16, seed=40 + scale)
        graphs[name] = (gt.Graph(_dev(src), _dev(dst), n, split=True, hubs_first=hubs, hub_share=5), n,
                        oracle.build_csr(n, src, dst))
        pools[name] = graphgen.sample_roots(n, src, dst, 200, seed=41)
    kept = {}

    def on_result(q):
        kept[q.qid] = q.result.cpu().numpy()       # synchronous: the buffer is recycled afterwards

    on_result.keeps_buffer = True
    # a burst (batched steps) and a trickle (mostly the single-root path)
    for rate, count, seed in ((50000.0, 150, 42), (300.0, 40, 43)):
        kept.clear()
        srv = serve.Server(hbm_budget_bytes=64 << 20, slots=16, on_result=on_result, solo_max=1)
        for name, (h, n, _) in graphs.items():
            srv.add_graph(name, h, n)
        sched = serve.poisson_arrivals(rate, count, sorted(graphs), pools, seed=seed)
        qs, _ = serve.run_open_loop(srv, sched)
        srv.join(timeout=120)
        assert len(kept) == count
        for q in qs:
            h, n, g = graphs[q.graph]
            np.testing.assert_array_equal(kept[q.qid], u8(oracle.bfs(g, q.root)[1]), err_msg="query %d" % q.qid)
        if rate < 1000:
            assert sum(srv.solo_counts().values()) > 0
    for h, _, _ in graphs.values():
        h.close()


def test_levels_to_u8_matches_numpy():
    gt = _gt()
    rng = np.random.default_rng(50)
    for n in (0, 1, 3, 4, 5, 63, 64, 1000, 4097):
        lv = rng.integers(-1, 255, n).astype(np.int32)
        out = gt.levels_to_u8(torch.from_numpy(lv).cuda()).cpu().numpy()
        np.testing.assert_array_equal(out, np.where(lv < 0, 255, lv).astype(np.uint8))
    # an unaligned view exercises the element-wise tail path
    lv = rng.integers(-1, 200, 1001).astype(np.int32)
    dev = torch.from_numpy(lv).cuda()
    out = torch.empty(1001, dtype=torch.uint8, device="cuda")
    gt.levels_to_u8(dev[1:], out[1:])
    np.testing.assert_array_equal(out[1:].cpu().numpy(), np.where(lv[1:] < 0, 255, lv[1:]).astype(np.uint8))
    with pytest.raises(gt.GTError) as e:
        gt.levels_to_u8(torch.tensor([0, 255, 3], dtype=torch.int32, device="cuda"))
    assert e.value.code == gt.GT_E_DEPTH
