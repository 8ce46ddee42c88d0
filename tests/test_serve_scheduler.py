"""The serving scheduler (paper_2009_07463_amd.serve) on the CPU.

A fake executor stands in for the GPU: its sessions answer each query with
the CPU oracle and finish it after as many steps as its BFS has levels, with
the same slot/busy semantics as gt_session_*. This checks queues, admission
by memory budget, slot refill and latency bookkeeping without a GPU.
"""
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle
from paper_2009_07463_amd import serve


class FakeSession:
    def __init__(self, g, slots):
        self.g = g
        self.slots = slots
        self.busy = {}
        self.max_busy = 0

    def try_admit(self, root, buf):
        free = [s for s in range(self.slots) if s not in self.busy]
        if not free:
            return None
        s = free[0]
        _, lvl = oracle.bfs(self.g, root)
        steps = int(lvl.max()) + 1
        self.busy[s] = [steps, buf, lvl]
        self.max_busy = max(self.max_busy, len(self.busy))
        return s

    def step(self):
        done = 0
        for s in list(self.busy):
            ent = self.busy[s]
            ent[0] -= 1
            if ent[0] <= 0:
                lvl = ent[2]
                ent[1][:] = np.where(lvl < 0, 255, lvl).astype(np.uint8)
                done |= 1 << s
                del self.busy[s]
        time.sleep(0.0005)
        return done


class FakeExecutor:
    def __init__(self, graphs):
        self.graphs = graphs
        self.sessions = []

    def new_stream(self):
        return None

    def session(self, graph, slots, stream):
        s = FakeSession(graph, slots)
        self.sessions.append(s)
        return s

    def buffer(self, n):
        return np.zeros(n, np.uint8)

    def synchronize(self, stream):
        pass

    def single_buffers(self, n):
        return np.zeros(n, np.int32), np.zeros(n, np.int32)

    def single_bfs(self, graph, root, parent, level, stream):
        p, l = oracle.bfs(graph, root)
        parent[:] = p
        level[:] = l

    def levels_to_u8(self, level, out, stream):
        out[:] = np.where(level < 0, 255, level).astype(np.uint8)


@pytest.fixture(scope="module")
def graphs():
    out = {}
    for name, scale in (("a", 9), ("b", 11)):
        src, dst = graphgen.kronecker_edges(scale, 16, seed=scale)
        n = 1 << scale
        out[name] = (oracle.build_csr(n, src, dst), n, graphgen.sample_roots(n, src, dst, 50, seed=1))
    return out


def _check(server_kw, graphs, rate=4000.0, count=300):
    results = {}
    lock = threading.Lock()
    peak = {"used": 0}

    def on_result(q):
        with lock:
            results[q.qid] = np.array(q.result, copy=True)
            peak["used"] = max(peak["used"], srv.budget.used)

    on_result.keeps_buffer = False
    ex = FakeExecutor(graphs)
    srv = serve.Server(executor=ex, on_result=on_result, **server_kw)
    for name, (g, n, _) in graphs.items():
        srv.add_graph(name, g, n)
    sched = serve.poisson_arrivals(rate, count, sorted(graphs), {k: v[2] for k, v in graphs.items()}, seed=3)
    qs, t0 = serve.run_open_loop(srv, sched)
    srv.join(timeout=120)
    assert len(srv.done) == count
    for q in qs:
        g, n, _ = graphs[q.graph]
        _, lvl = oracle.bfs(g, q.root)
        got = results[q.qid]
        if got.dtype == np.uint8:
            got = np.where(got == 255, -1, got.astype(np.int32))
        np.testing.assert_array_equal(got, lvl)
        assert q.t_done >= q.t_sched
    summ = serve.latency_summary(qs, t0)
    assert summ["queries"] == count and summ["p99_ms"] >= summ["p50_ms"] >= 0
    return srv, ex, peak


def test_continuous_batching_scheduler_results_and_slots(graphs):
    srv, ex, _ = _check(dict(hbm_budget_bytes=1 << 30, slots=4, solo_max=0), graphs)
    assert all(s.max_busy <= 4 for s in ex.sessions)
    assert any(s.max_busy > 1 for s in ex.sessions)      # queries were coalesced
    assert sum(srv.solo_counts().values()) == 0


def test_hybrid_solo_path_at_low_and_high_load(graphs):
    # low load: most queries find the session idle and run alone
    srv, ex, _ = _check(dict(hbm_budget_bytes=1 << 30, slots=4, solo_max=1), graphs, rate=200.0, count=60)
    assert sum(srv.solo_counts().values()) > 0
    # high load: queues build up and the session still coalesces queries
    srv, ex, _ = _check(dict(hbm_budget_bytes=1 << 30, slots=4, solo_max=1), graphs, rate=20000.0, count=300)
    assert any(s.max_busy > 1 for s in ex.sessions)


def test_admission_respects_memory_budget(graphs):
    # room for 3 level buffers of the larger graph only
    n_big = graphs["b"][1]
    srv, ex, peak = _check(dict(hbm_budget_bytes=3 * n_big, slots=8), graphs, count=120)
    assert peak["used"] <= 3 * n_big
    assert srv.budget.used == 0


def test_budget_from_free_device_memory(graphs):
    class WithFree(FakeExecutor):
        def free_bytes(self):
            return 10 << 20
    ex = WithFree(graphs)
    # free memory less the reserve, capped by an explicit budget if given
    assert serve.Server.derive_budget(ex, None, 4 << 20) == 6 << 20
    assert serve.Server.derive_budget(ex, 1 << 20, 4 << 20) == 1 << 20
    assert serve.Server.derive_budget(ex, None, 20 << 20) == 0
    # an executor that cannot tell free memory needs an explicit budget
    assert serve.Server.derive_budget(FakeExecutor(graphs), 5 << 20, 0) == 5 << 20
    with pytest.raises(ValueError):
        serve.Server.derive_budget(FakeExecutor(graphs), None, 0)
    srv = serve.Server(executor=WithFree(graphs), hbm_reserve_bytes=2 << 20)
    assert srv.budget.budget == 8 << 20


def test_sequential_baseline_scheduler(graphs):
    srv, ex, _ = _check(dict(hbm_budget_bytes=1 << 30, slots=4, sequential=True), graphs, count=80)


def test_short_queue_runs_solo_beside_a_busy_session(graphs):
    # a burst longer than solo_max goes into the session; a query arriving
    # while those are traversed finds a short queue and runs alone, between
    # the session's steps, and finishes before the burst does
    g, n, roots = graphs["b"]
    ex = FakeExecutor(graphs)
    srv = serve.Server(executor=ex, hbm_budget_bytes=1 << 30, slots=8, solo_max=2)
    srv.add_graph("b", g, n)
    burst = [(0.0, "b", int(r)) for r in roots[:6]]
    sched = burst + [(0.002, "b", int(roots[6]))]
    qs, t0 = serve.run_open_loop(srv, sched)
    srv.join(timeout=120)
    assert len(srv.done) == len(sched)
    assert srv.solo_counts()["b"] >= 1
    assert ex.sessions[0].max_busy >= 3          # the burst was batched
    late = qs[-1]
    assert late.t_done < max(q.t_done for q in qs[:6])


def test_solo_threshold_follows_measured_times(graphs):
    g, n, _ = graphs["a"]
    srv = serve.Server(executor=FakeExecutor(graphs), hbm_budget_bytes=1 << 30, slots=64, solo_max=4)
    srv.add_graph("a", g, n)
    w = srv.workers["a"]
    assert w.solo_threshold() == 4                  # nothing measured yet: solo_max
    w.t_solo, w.t_batch = 0.0004, 0.0064            # one session query takes 16 solo ones
    assert w.solo_threshold() == 16
    w.t_solo, w.t_batch = 0.0004, 0.0008            # never below solo_max
    assert w.solo_threshold() == 4
    srv.join(timeout=30)
