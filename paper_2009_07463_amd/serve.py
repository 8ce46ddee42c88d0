"""Query serving over resident graphs: continuous batching of BFS queries.

Several graphs stay resident in HBM. Queries (graph, root) arrive over time;
each graph has a worker that owns one continuous-batching session
(``gt_session_*``, up to 64 queries traversed together, one bit each). At
every level step the worker admits waiting queries into free slots -- if the
shared device-memory budget has room for their N-byte level buffers -- runs
one step for all active queries of that graph on the graph's own stream, and
hands finished results back. Workers of different graphs run concurrently,
so their steps overlap on the device.

The traversal itself is the library's (``gt_session_step``); this module only
schedules: queues, admission, slot refill, buffers and latency bookkeeping.
An ``executor`` object supplies sessions and buffers, so the scheduler can be
exercised without a GPU (the tests plug in a CPU executor).
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field


@dataclass
class Query:
    graph: str
    root: int
    t_sched: float                  # scheduled arrival (open-loop clock)
    t_admit: float = -1.0
    t_done: float = -1.0
    slot: int = -1
    result: object = None           # level buffer (executor-specific)
    qid: int = -1

    @property
    def latency(self) -> float:
        return self.t_done - self.t_sched


class MemoryBudget:
    """Admission by device memory: per-query level buffers must fit."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.used = 0
        self.lock = threading.Lock()

    def try_take(self, nbytes: int) -> bool:
        with self.lock:
            if self.used + nbytes > self.budget:
                return False
            self.used += nbytes
            return True

    def give_back(self, nbytes: int):
        with self.lock:
            self.used -= nbytes
            assert self.used >= 0


class GpuExecutor:
    """Sessions and level buffers on the GPU (gt C ABI through the binding)."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)

    def new_stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def session(self, graph, slots: int, stream):
        from . import Session
        return Session(graph, slots=slots, stream=stream)

    def buffer(self, n: int):
        return self.torch.empty(n, dtype=self.torch.uint8, device=self.device)

    def synchronize(self, stream):
        stream.synchronize()

    def single_buffers(self, n: int):
        t = self.torch
        return (t.empty(n, dtype=t.int32, device=self.device), t.empty(n, dtype=t.int32, device=self.device))

    def single_bfs(self, graph, root, parent, level, stream):
        graph.bfs(root, parent, level, stream=stream)

    def levels_to_u8(self, level, out, stream):
        from . import levels_to_u8
        levels_to_u8(level, out, stream=stream)

    def free_bytes(self):
        """Device memory free right now (hipMemGetInfo through torch)."""
        return int(self.torch.cuda.mem_get_info(self.device)[0])


class GraphWorker(threading.Thread):
    """Drives one graph's continuous-batching session.

    With solo_max > 0, the query at the head of the queue runs alone through
    the single-root BFS (gt_bfs, then the uint8 conversion) whenever at most
    solo_max queries wait, even while the session holds queries: a batched
    step costs about as much for one query as for 64, so a query that joins
    a session answers only after several such steps, while gt_bfs answers
    in about one. Only a longer queue is admitted into the session, which
    then takes every waiting query its free slots allow. Between two solo
    queries the session makes one step, so its queries keep moving.

    "Longer" adapts to the graph: once both are measured, the threshold is
    the number of queries that one after another take as long as one query
    takes through the session (running means of the solo service time and
    of a session query's time from admission to completion), and never
    below solo_max.
    """

    def __init__(self, server, name, graph, n, slots, stream):
        super().__init__(daemon=True)
        self.server = server
        self.name = name
        self.graph = graph
        self.n = n
        self.stream = stream
        self.session = server.executor.session(graph, slots, stream)
        self.queue = collections.deque()
        self.running = {}
        self.cv = threading.Condition()
        self.stop_flag = False
        self.steps = 0
        self.solo = 0
        self.error = None
        self.solo_max = server.solo_max
        self.t_solo = None     # running mean of a solo query's service time (s)
        self.t_batch = None    # ... of a session query's time from admission to completion (s)
        self.parent = self.level = None
        if self.solo_max > 0:
            self.parent, self.level = server.executor.single_buffers(n)

    @staticmethod
    def _mean(old, x, w=0.1):
        return x if old is None else (1.0 - w) * old + w * x

    def solo_threshold(self) -> int:
        """Longest queue served one query at a time."""
        if self.t_solo is None or self.t_batch is None or self.t_solo <= 0:
            return self.solo_max
        return max(self.solo_max, int(self.t_batch / self.t_solo))

    def _run_solo(self):
        """One waiting query through the single-root path; False if none ran."""
        srv = self.server
        with self.cv:
            if not self.queue or len(self.queue) > self.solo_threshold():
                return False
            q = self.queue[0]
        if not srv.budget.try_take(self.n):
            return False
        with self.cv:
            self.queue.popleft()
        buf = srv.buffers.get(self.n)
        q.t_admit = time.perf_counter()
        ex = srv.executor
        ex.single_bfs(self.graph, q.root, self.parent, self.level, self.stream)
        ex.levels_to_u8(self.level, buf, self.stream)
        q.result = buf
        srv.executor.synchronize(self.stream)
        q.t_done = time.perf_counter()
        self.t_solo = self._mean(self.t_solo, q.t_done - q.t_admit)
        self.solo += 1
        srv._finish(q)
        return True

    def submit(self, q: Query):
        with self.cv:
            self.queue.append(q)
            self.cv.notify()

    def _admit(self):
        srv = self.server
        while True:
            with self.cv:
                if not self.queue:
                    return
                q = self.queue[0]
            if not srv.budget.try_take(self.n):
                return                        # no device memory for another level buffer now
            buf = srv.buffers.get(self.n)
            slot = self.session.try_admit(q.root, buf)
            if slot is None:                  # all slots busy
                srv.buffers.put(self.n, buf)
                srv.budget.give_back(self.n)
                return
            with self.cv:
                self.queue.popleft()
            q.slot = slot
            q.result = buf
            q.t_admit = time.perf_counter()
            self.running[slot] = q

    def run(self):
        try:
            while True:
                with self.cv:
                    while not self.queue and not self.running and not self.stop_flag:
                        self.cv.wait(timeout=0.05)
                    if self.stop_flag and not self.queue and not self.running:
                        return
                if self.solo_max > 0 and self._run_solo():
                    if not self.running:
                        continue
                    # one step for the session's queries before the next solo one
                else:
                    self._admit()
                if not self.running:
                    time.sleep(0)             # waiting for memory or arrivals
                    continue
                done = self.session.step()
                self.steps += 1
                if done:
                    now = time.perf_counter()
                    for slot in list(self.running):
                        if (done >> slot) & 1:
                            q = self.running.pop(slot)
                            q.t_done = now
                            self.t_batch = self._mean(self.t_batch, q.t_done - q.t_admit)
                            self.server._finish(q)
        except Exception as e:  # surfaced by Server.join
            self.error = e

    def stop(self):
        with self.cv:
            self.stop_flag = True
            self.cv.notify()


class SequentialWorker(GraphWorker):
    """Baseline: one query at a time per graph (single-source gt_bfs), with
    the same result as the server's (uint8 levels in a pooled buffer)."""

    def __init__(self, server, name, graph, n, slots, stream):
        threading.Thread.__init__(self, daemon=True)
        self.server = server
        self.name = name
        self.graph = graph
        self.n = n
        self.stream = stream
        self.queue = collections.deque()
        self.running = {}
        self.cv = threading.Condition()
        self.stop_flag = False
        self.steps = 0
        self.solo = 0
        self.error = None
        self.parent, self.level = server.executor.single_buffers(n)

    def run(self):
        try:
            while True:
                with self.cv:
                    while not self.queue and not self.stop_flag:
                        self.cv.wait(timeout=0.05)
                    if self.stop_flag and not self.queue:
                        return
                    q = self.queue.popleft()
                q.t_admit = time.perf_counter()
                ex = self.server.executor
                buf = self.server.buffers.get(self.n)
                ex.single_bfs(self.graph, q.root, self.parent, self.level, self.stream)
                ex.levels_to_u8(self.level, buf, self.stream)
                ex.synchronize(self.stream)
                self.steps += 1
                q.t_done = time.perf_counter()
                q.result = buf
                self.server._finish_single(q)
        except Exception as e:
            self.error = e


class BufferPool:
    def __init__(self, executor):
        self.executor = executor
        self.free = collections.defaultdict(list)
        self.lock = threading.Lock()

    def get(self, n):
        with self.lock:
            if self.free[n]:
                return self.free[n].pop()
        return self.executor.buffer(n)

    def put(self, n, buf):
        with self.lock:
            self.free[n].append(buf)


class Server:
    """Continuous-batching BFS server over several resident graphs.

    on_result(q) is called from the graph's worker thread once q's level
    buffer is complete (its stream has been synchronised). The buffer goes
    back to the pool when on_result returns, so on_result must finish every
    use of q.result before returning (for a device buffer: copy it with a
    synchronous copy, or synchronise the stream it used).
    solo_max: while at most solo_max queries wait for a graph, the first
    runs through the single-root BFS, between the session's steps (0: every
    query joins the session).
    Admission: level buffers of admitted queries may take at most the device
    memory free at start-up minus hbm_reserve_bytes, capped by
    hbm_budget_bytes when given (Server.budget.budget holds the result).
    """

    def __init__(self, executor=None, hbm_budget_bytes: int | None = None, slots: int = 64,
                 on_result=None, sequential: bool = False, solo_max: int = 16,
                 hbm_reserve_bytes: int = 4 << 30):
        self.executor = executor if executor is not None else GpuExecutor()
        self.budget = MemoryBudget(self.derive_budget(self.executor, hbm_budget_bytes, hbm_reserve_bytes))
        self.buffers = BufferPool(self.executor)
        self.slots = slots
        self.workers = {}
        self.done = []
        self.lock = threading.Lock()
        self.on_result = on_result
        self.sequential = sequential
        self.solo_max = int(solo_max)

    @staticmethod
    def derive_budget(executor, cap_bytes, reserve_bytes):
        """Bytes of per-query level buffers admitted at once: the device
        memory free when the server starts, less a reserve for everything
        else (sessions' own state, other allocations), and at most cap_bytes
        if given. An executor that cannot tell free memory needs a cap."""
        free = executor.free_bytes() if hasattr(executor, "free_bytes") else None
        if free is None:
            if cap_bytes is None:
                raise ValueError("hbm_budget_bytes is required when free device memory is unknown")
            return int(cap_bytes)
        budget = max(0, int(free) - int(reserve_bytes))
        return budget if cap_bytes is None else min(budget, int(cap_bytes))

    def add_graph(self, name: str, graph, n: int):
        cls = SequentialWorker if self.sequential else GraphWorker
        w = cls(self, name, graph, n, self.slots, self.executor.new_stream())
        self.workers[name] = w
        w.start()

    def submit(self, q: Query):
        self.workers[q.graph].submit(q)

    def _finish(self, q: Query):
        w = self.workers[q.graph]
        self.executor.synchronize(w.stream)
        if self.on_result is not None:
            self.on_result(q)
        self.buffers.put(w.n, q.result)
        if self.on_result is None or not getattr(self.on_result, "keeps_buffer", False):
            q.result = None
        self.budget.give_back(w.n)
        with self.lock:
            self.done.append(q)

    def _finish_single(self, q: Query):
        if self.on_result is not None:
            self.on_result(q)
        self.buffers.put(self.workers[q.graph].n, q.result)
        q.result = None
        with self.lock:
            self.done.append(q)

    def join(self, timeout: float = 600.0):
        for w in self.workers.values():
            w.stop()
        t0 = time.perf_counter()
        for w in self.workers.values():
            w.join(max(0.0, timeout - (time.perf_counter() - t0)))
            if w.error is not None:
                raise w.error

    def steps(self):
        return {k: w.steps for k, w in self.workers.items()}

    def solo_counts(self):
        return {k: w.solo for k, w in self.workers.items()}


def poisson_arrivals(rate_qps: float, count: int, graphs, roots_by_graph, seed: int):
    """Open-loop schedule: exponential gaps, uniform graph, uniform root."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_qps, size=count))
    gsel = rng.integers(0, len(graphs), size=count)
    out = []
    for i in range(count):
        gname = graphs[gsel[i]]
        roots = roots_by_graph[gname]
        out.append((float(t[i]), gname, int(roots[rng.integers(0, len(roots))])))
    return out


def run_open_loop(server: Server, schedule, qid0: int = 0):
    """Submit queries at their scheduled times (relative to now); return them
    after all finished. Latency counts from the scheduled time, so a late
    submit (server busy) is charged to the server (no coordinated omission)."""
    t0 = time.perf_counter()
    qs = []
    for i, (ts, gname, root) in enumerate(schedule):
        when = t0 + ts
        while True:
            now = time.perf_counter()
            if now >= when:
                break
            time.sleep(min(when - now, 0.0005))
        q = Query(graph=gname, root=root, t_sched=when, qid=qid0 + i)
        qs.append(q)
        server.submit(q)
    return qs, t0


def latency_summary(qs, t0):
    import numpy as np
    lat = np.array([q.latency for q in qs]) * 1e3
    t_end = max(q.t_done for q in qs)
    return dict(queries=len(qs), qps=len(qs) / (t_end - t0), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()), max_ms=float(lat.max()))
