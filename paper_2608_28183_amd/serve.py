"""Continuous-batching request loop for f-k and RSD reconstructions on one GPU.

The paper's streaming system (Section 4.1, producer-consumer pipeline) overlaps
capture and reconstruction; this loop is its serving analogue on one MI355X:

* requests arrive at any time (``submit`` returns a Future);
* a dispatcher admits queued requests, in arrival order, as soon as a slot (a HIP
  stream with its own nlos context) and enough HBM are free: a request's need is the
  exact workspace of its plan (``nlos_*_workspace_bytes``) plus its output volume and
  image, checked against the budget before anything is allocated;
* admitted requests run concurrently on their streams, so work from different
  requests overlaps on the device; completion is detected by polling a HIP event and
  frees the slot and the memory for the next admissions;
* plans (FFT tables, Stolt constants, radial kernels) are built once per
  (method, shape, precision) and stay resident; inputs are device tensors.

Latency is arrival -> completion observed on the host.  Results do not depend on the
mix: every kernel is deterministic and each request uses its own workspace.

The scheduling logic is independent of the GPU: ``Server`` drives an executor
object (``GpuExecutor`` here; tests use a simulated one).
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import threading
import time
from typing import Any, Callable, Deque, Dict, List, Optional, Tuple

# ---------------------------------------------------------------------------
# requests and statistics
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Request:
    method: str                      # "fk" or "rsd"
    shape: Tuple[int, int, int]      # (ny, nx, nt)
    precision: str = "fp32"          # storage precision of the intermediates
    tau: Any = None                  # device tensor [ny, nx, nt] float32
    id: int = 0
    arrival: float = 0.0             # perf_counter() at submit
    admitted: float = 0.0
    done: float = 0.0
    need_bytes: int = 0
    future: Optional[concurrent.futures.Future] = None
    slot: int = -1
    handle: Any = None
    ready: Any = None                # set at submit: marks the input complete on its stream


def percentile(xs: List[float], q: float) -> float:
    """Nearest-rank percentile (q in [0, 100])."""
    if not xs:
        return float("nan")
    s = sorted(xs)
    k = max(0, min(len(s) - 1, int(-(-q * len(s) // 100)) - 1))
    return s[k]


@dataclasses.dataclass
class Stats:
    latencies: List[float] = dataclasses.field(default_factory=list)
    queue_waits: List[float] = dataclasses.field(default_factory=list)
    completed: int = 0
    rejected: int = 0
    peak_bytes: int = 0
    peak_inflight: int = 0
    first_arrival: float = 0.0
    last_done: float = 0.0

    def summary(self) -> Dict[str, float]:
        span = max(self.last_done - self.first_arrival, 1e-9)
        return {
            "completed": self.completed,
            "rejected": self.rejected,
            "p50_ms": percentile(self.latencies, 50) * 1e3,
            "p99_ms": percentile(self.latencies, 99) * 1e3,
            "mean_ms": (sum(self.latencies) / len(self.latencies) * 1e3) if self.latencies else float("nan"),
            "queue_p99_ms": percentile(self.queue_waits, 99) * 1e3,
            "volumes_per_s": self.completed / span,
            "peak_bytes": self.peak_bytes,
            "peak_inflight": self.peak_inflight,
        }


# ---------------------------------------------------------------------------
# scheduler
# ---------------------------------------------------------------------------


class Server:
    """Admission by memory and slot, FIFO order, overlapped execution.

    executor must provide:
      need_bytes(req) -> int         exact device bytes the request will hold
      start(req, slot) -> handle     enqueue the request's work on slot's stream
      done(handle) -> bool           non-blocking completion check
      finish(req) -> result          release per-request buffers, return the result
    """

    def __init__(self, executor, n_slots: int = 4, hbm_budget: int = 16 << 30,
                 poll_s: float = 50e-6, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.n_slots = n_slots
        self.budget = hbm_budget
        self.poll_s = poll_s
        self.clock = clock
        self.queue: Deque[Request] = collections.deque()
        self.running: Dict[int, Request] = {}
        self.free_slots = list(range(n_slots))
        self.used_bytes = 0
        self.stats = Stats()
        self._lock = threading.Lock()
        self._wake = threading.Condition(self._lock)
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self._next_id = 0

    # -- client side -------------------------------------------------------
    def submit(self, req: Request) -> concurrent.futures.Future:
        req.future = concurrent.futures.Future()
        req.need_bytes = int(self.ex.need_bytes(req))
        prepare = getattr(self.ex, "prepare", None)
        if prepare is not None:
            prepare(req)     # in the submitting thread: sees the caller's current stream
        with self._lock:
            req.id = self._next_id
            self._next_id += 1
            req.arrival = self.clock()
            if not self.stats.first_arrival:
                self.stats.first_arrival = req.arrival
            if req.need_bytes > self.budget:
                self.stats.rejected += 1
                req.future.set_exception(MemoryError(
                    f"request needs {req.need_bytes} bytes, budget is {self.budget}"))
                return req.future
            self.queue.append(req)
            self._wake.notify()
        return req.future

    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._loop, name="nlos-serve", daemon=True)
        self._thread.start()
        return self

    def stop(self, drain: bool = True, timeout: float = 120.0) -> None:
        if drain:
            t0 = time.perf_counter()
            while True:
                with self._lock:
                    idle = not self.queue and not self.running
                if idle or time.perf_counter() - t0 > timeout:
                    break
                time.sleep(1e-3)
        with self._lock:
            self._stop = True
            self._wake.notify()
        if self._thread is not None:
            self._thread.join(timeout)

    # -- dispatcher ----------------------------------------------------------
    def step(self) -> int:
        """One scheduling round: retire finished work, then admit.  Returns the
        number of requests that changed state (for callers that drive the loop)."""
        changed = 0
        for slot, req in list(self.running.items()):
            if self.ex.done(req.handle):
                result = self.ex.finish(req)
                req.done = self.clock()
                with self._lock:
                    del self.running[slot]
                    self.free_slots.append(slot)
                    self.used_bytes -= req.need_bytes
                    self.stats.completed += 1
                    self.stats.latencies.append(req.done - req.arrival)
                    self.stats.queue_waits.append(req.admitted - req.arrival)
                    self.stats.last_done = req.done
                req.future.set_result(result)
                changed += 1
        while True:
            with self._lock:
                if not self.queue or not self.free_slots:
                    break
                req = self.queue[0]
                if self.used_bytes + req.need_bytes > self.budget:
                    break            # FIFO: the head waits for memory
                self.queue.popleft()
                slot = self.free_slots.pop(0)
                self.used_bytes += req.need_bytes
                self.running[slot] = req
                self.stats.peak_bytes = max(self.stats.peak_bytes, self.used_bytes)
                self.stats.peak_inflight = max(self.stats.peak_inflight, len(self.running))
            req.slot = slot
            req.admitted = self.clock()
            try:
                req.handle = self.ex.start(req, slot)
            except Exception as e:  # noqa: BLE001 - surfaced through the future
                with self._lock:
                    del self.running[slot]
                    self.free_slots.append(slot)
                    self.used_bytes -= req.need_bytes
                    self.stats.rejected += 1
                req.future.set_exception(e)
            changed += 1
        return changed

    def _loop(self) -> None:
        while True:
            with self._lock:
                if self._stop:
                    return
                if not self.queue and not self.running:
                    self._wake.wait(0.01)
                    continue
            if self.step() == 0:
                time.sleep(self.poll_s)


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------


def rsd_precisions(precision: str) -> Tuple[str, str]:
    """(data, kernel) storage of an RSD request: the reduced-precision forms store the
    complex intermediates and the radial kernel K_r (accumulated in FP64, rounded once on
    store) in FP16 or BF16, and propagate on the matrix cores.  An f-k request's
    precision is the storage of its complex intermediates (fp32, fp16, bf16)."""
    return (precision, precision)


class GpuExecutor:
    """Runs requests through libnlos on per-slot HIP streams.

    geometry(shape) -> dict with the physical parameters of a shape (wall size, bin
    width, padding, RSD frequency set and depths); plans are cached per
    (method, shape, precision)."""

    def __init__(self, n_slots: int, geometry: Callable[[Tuple[int, int, int]], dict], device: int = 0):
        import torch

        from . import runtime
        self.torch = torch
        self.runtime = runtime
        self.device = torch.device("cuda", device)
        self.geometry = geometry
        # default-priority streams (one nlos context per stream)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_slots)]
        self.ctxs = [runtime.Context(device, s) for s in self.streams]
        self.plans: Dict[tuple, Any] = {}
        self._plan_ctx = runtime.Context(device, torch.cuda.current_stream(self.device))

    def plan(self, method: str, shape, precision: str):
        key = (method, tuple(shape), precision)
        p = self.plans.get(key)
        if p is None:
            ny, nx, nt = shape
            g = self.geometry(tuple(shape))
            if method == "fk":
                p = self.runtime.FkPlan(self._plan_ctx, ny, nx, nt, g["wall_w"], g["wall_h"],
                                        g["bin_ps"], g["pad"], precision)
            else:
                r = g["rsd"]
                data_prec, kernel_prec = rsd_precisions(precision)
                p = self.runtime.RsdPlan(self._plan_ctx, ny, nx, nt, g["dx"], g["dy"], g["bin_ps"],
                                         g["pad"], r.freq_bins, r.weights, r.n_depth, r.depth0,
                                         r.depth_step, r.sigma_s, r.sigma_t, r.delta, data_prec,
                                         kernel_prec)
            self.plans[key] = p
        return p

    def need_bytes(self, req: Request) -> int:
        p = self.plan(req.method, req.shape, req.precision)
        ny, nx, nt = req.shape
        nz = nt if req.method == "fk" else p.n_depth
        return p.ws_bytes + 4 * ny * nx * nz + 4 * ny * nx

    def prepare(self, req: Request) -> None:
        """At submit time: an event on the submitting thread's current stream, after the
        work that produced req.tau, which the slot stream waits for before reading it."""
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.device))
        req.ready = ev

    def start(self, req: Request, slot: int):
        torch = self.torch
        p = self.plan(req.method, req.shape, req.precision)
        s = self.streams[slot]
        if req.ready is not None:
            s.wait_event(req.ready)
        # the input is in use on the slot stream until the reconstruction ends there
        req.tau.record_stream(s)
        ny, nx, nt = req.shape
        nz = nt if req.method == "fk" else p.n_depth
        with torch.cuda.stream(s):
            ws = torch.empty(p.ws_bytes, dtype=torch.uint8, device=self.device)
            vol = torch.empty((ny, nx, nz), dtype=torch.float32, device=self.device)
            img = torch.empty((ny, nx), dtype=torch.float32, device=self.device)
        ctx = self.ctxs[slot]
        if req.method == "fk":
            self.runtime.nlos.nlos_fk(ctx.handle, p.handle, req.tau, vol, img, ws)
        else:
            self.runtime.nlos.nlos_rsd(ctx.handle, p.handle, req.tau, vol, img, ws)
        ev = torch.cuda.Event()
        ev.record(s)
        return {"event": ev, "ws": ws, "vol": vol, "img": img}

    def done(self, handle) -> bool:
        return handle["event"].query()

    def finish(self, req: Request):
        h = req.handle
        h["ws"] = None  # the workspace returns to the allocator (stream-ordered)
        return h["vol"], h["img"]


# ---------------------------------------------------------------------------
# Poisson load driver
# ---------------------------------------------------------------------------


def run_stream(server: Server, arrivals: List[Tuple[float, Request]], timeout: float = 600.0):
    """Submits requests at their arrival offsets (seconds from now) and waits for all."""
    t0 = time.perf_counter()
    futures = []
    for off, req in arrivals:
        now = time.perf_counter() - t0
        if off > now:
            time.sleep(off - now)
        futures.append(server.submit(req))
    results = []
    for f in futures:
        try:
            results.append(f.result(timeout=timeout))
        except Exception as e:  # noqa: BLE001
            results.append(e)
    return results
