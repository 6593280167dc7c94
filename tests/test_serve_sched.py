"""Scheduling logic of the serving loop, on the CPU with a simulated executor."""
import threading
import time

import numpy as np
import pytest

from paper_2608_28183_amd.serve import Request, Server, percentile, run_stream


class SimExecutor:
    """Each request 'runs' for duration_s on its slot; records concurrency."""

    def __init__(self, need=None, duration=0.01, fail_ids=()):
        self.need = need or (lambda r: 1 << 30)
        self.duration = duration
        self.fail_ids = set(fail_ids)
        self.running = 0
        self.max_running = 0
        self.held = 0            # bytes of the requests started and not yet finished
        self.max_held = 0
        self.prepared = {}       # request object id -> submitting thread
        self.order = []
        self.lock = threading.Lock()

    def need_bytes(self, req):
        return self.need(req)

    def prepare(self, req):
        req.ready = ("ready", threading.get_ident())
        self.prepared[id(req)] = threading.get_ident()

    def start(self, req, slot):
        # the input was marked complete at submit, in the submitting thread
        assert req.ready is not None and id(req) in self.prepared
        if req.id in self.fail_ids:
            raise RuntimeError("injected launch failure")
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.held += self.need(req)
            self.max_held = max(self.max_held, self.held)
            self.order.append(req.id)
        return (time.perf_counter() + self.duration, self.need(req))

    def done(self, handle):
        return time.perf_counter() >= handle[0]

    def finish(self, req):
        with self.lock:
            self.running -= 1
            self.held -= req.handle[1]
        return ("result", req.id)


def test_percentile_matches_nearest_rank():
    xs = list(np.random.default_rng(0).random(101))
    assert percentile(xs, 50) == sorted(xs)[50]
    assert percentile(xs, 99) == sorted(xs)[99]
    assert percentile([3.0], 99) == 3.0


def test_slots_bound_concurrency_and_results_arrive():
    ex = SimExecutor(duration=0.02)
    srv = Server(ex, n_slots=3, hbm_budget=100 << 30).start()
    futs = [srv.submit(Request("fk", (8, 8, 8))) for _ in range(12)]
    res = [f.result(timeout=10) for f in futs]
    srv.stop()
    assert [r[1] for r in res] == list(range(12))
    assert ex.max_running == 3 and srv.stats.peak_inflight == 3
    assert ex.order == sorted(ex.order)  # FIFO admission


def test_memory_budget_is_never_exceeded():
    # sizes in GiB by the request's first dimension; the executor counts the bytes of the
    # requests it is actually running, independently of the scheduler's bookkeeping
    sizes = [6, 5, 3, 8, 2, 9]
    ex = SimExecutor(need=lambda r: sizes[r.shape[0] % 6] << 30, duration=0.01)
    srv = Server(ex, n_slots=8, hbm_budget=10 << 30).start()
    futs = [srv.submit(Request("rsd", (k % 6, 8, 8))) for k in range(30)]
    for f in futs:
        f.result(timeout=20)
    srv.stop()
    assert ex.max_held <= 10 << 30
    assert ex.max_held >= 8 << 30       # the budget was actually approached
    assert srv.stats.peak_bytes <= 10 << 30 and ex.held == 0
    assert srv.stats.completed == 30
    assert ex.order == sorted(ex.order)


def test_inputs_are_marked_ready_in_the_submitting_thread():
    ex = SimExecutor(duration=0.005)
    srv = Server(ex, n_slots=2, hbm_budget=100 << 30).start()
    reqs = [Request("fk", (8, 8, 8)) for _ in range(6)]
    futs = [srv.submit(r) for r in reqs]
    for f in futs:
        f.result(timeout=10)
    srv.stop()
    me = threading.get_ident()
    assert all(r.ready == ("ready", me) and ex.prepared[id(r)] == me for r in reqs)


def test_oversize_request_is_rejected_and_failure_frees_the_slot():
    ex = SimExecutor(need=lambda r: (20 << 30) if r.shape[0] == 99 else (1 << 30), fail_ids={1})
    srv = Server(ex, n_slots=1, hbm_budget=10 << 30).start()
    big = srv.submit(Request("fk", (99, 8, 8)))
    with pytest.raises(MemoryError):
        big.result(timeout=5)
    bad = srv.submit(Request("fk", (8, 8, 8)))   # id 1: launch fails
    ok = srv.submit(Request("fk", (8, 8, 8)))
    with pytest.raises(RuntimeError):
        bad.result(timeout=5)
    assert ok.result(timeout=5)[0] == "result"
    srv.stop()
    assert srv.used_bytes == 0 and srv.free_slots == [0]


def test_poisson_stream_latency_report():
    ex = SimExecutor(duration=0.005)
    srv = Server(ex, n_slots=2, hbm_budget=8 << 30).start()
    rng = np.random.default_rng(3)
    t = np.cumsum(rng.exponential(1 / 400.0, size=80))
    run_stream(srv, [(float(x), Request("fk", (8, 8, 8))) for x in t])
    srv.stop()
    s = srv.stats.summary()
    assert s["completed"] == 80 and s["p99_ms"] >= s["p50_ms"] >= 5.0
    assert s["volumes_per_s"] > 0
