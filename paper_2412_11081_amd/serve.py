"""Serving loop: continuous batching of force/stress requests on one GPU.

Requests (structures with their block tensors) arrive at any time.  A
scheduler thread admits them in arrival order while the device-memory budget
allows (the footprint of a request is its input tensors plus the work buffers
the library sizes for it), and hands the admitted ones, up to ``max_batch``
at a time, to whichever worker is free.  Each worker evaluates its batch with
one ``lrx_evaluate_batch`` call on the stream of the batch's first context,
so batches of different workers overlap on the device, and requests that
arrive while a batch runs join the next one.  A finished request releases its
memory at once, which admits the next waiting ones.

The engine (what admits, evaluates and releases) is a small interface, so the
scheduling and the failure handling are tested on the CPU with a fake engine;
``LrxEngine`` is the real one.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import threading
import time
from typing import Any, Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    payload: Any                      # what the engine needs (e.g. a synth.Structure)
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    footprint: int = 0
    result: Any = None                # (E, F, sigma)
    error: Optional[str] = None
    batch_size: int = 0
    done: threading.Event = dataclasses.field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


class Engine:
    """What the server needs from a compute backend."""

    def estimate(self, payload) -> int:
        """Device bytes a request will hold while admitted (an upper estimate)."""
        raise NotImplementedError

    def admit(self, payload):
        """Bring the request's tensors to the device; returns (handle, bytes held)."""
        raise NotImplementedError

    def run(self, handles: List[Any]) -> List[Any]:
        """Evaluate a batch; one result per handle."""
        raise NotImplementedError

    def release(self, handle) -> None:
        raise NotImplementedError


class Server:
    """Continuous-batching request loop over an Engine."""

    def __init__(self, engine: Engine, hbm_budget: int, max_batch: int = 8, workers: int = 2, admitters: int = 2,
                 window: float = 0.0):
        assert hbm_budget > 0 and max_batch > 0 and workers > 0 and admitters > 0 and window >= 0
        self.engine = engine
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.n_workers = int(workers)
        # batching window: a free worker takes the admitted requests once
        # max_batch of them are ready, once the oldest has waited `window`
        # seconds, or once no other request is on its way (pending or being
        # admitted); 0 dispatches whatever is ready at once
        self.window = float(window)
        self._lock = threading.Condition()
        self._pending: collections.deque = collections.deque()      # submitted, not admitted
        self._ready: collections.deque = collections.deque()        # admitted, waiting for a worker
        self._handles: Dict[int, Any] = {}
        self._used = 0
        self._busy = 0
        self._admitting = 0
        self._stop = False
        self.max_used = 0
        self.batches: List[int] = []
        self.finished: List[Request] = []
        self._threads = [threading.Thread(target=self._schedule, name="lrx-sched", daemon=True)]
        self._threads += [threading.Thread(target=self._work, name=f"lrx-worker{i}", daemon=True)
                          for i in range(self.n_workers)]
        self._jobs: collections.deque = collections.deque()
        # admissions (tensors to the device, context set-up) run in a pool so
        # several requests are prepared while batches run
        self._admit_pool = concurrent.futures.ThreadPoolExecutor(max_workers=admitters,
                                                                 thread_name_prefix="lrx-admit")
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------------ API
    def submit(self, req: Request) -> Request:
        req.t_submit = time.perf_counter()
        try:
            req.footprint = int(self.engine.estimate(req.payload))
        except Exception as e:      # noqa: BLE001 - any estimate failure rejects the request
            self._finish(req, error=f"estimate failed: {e}")
            return req
        if req.footprint > self.budget:
            self._finish(req, error=f"request needs {req.footprint} bytes, more than the budget {self.budget}")
            return req
        with self._lock:
            self._pending.append(req)
            self._lock.notify_all()
        return req

    def drain(self, timeout: Optional[float] = None) -> bool:
        """Wait until every submitted request has finished."""
        end = None if timeout is None else time.perf_counter() + timeout
        with self._lock:
            while self._pending or self._ready or self._jobs or self._busy or self._admitting:
                left = None if end is None else end - time.perf_counter()
                if left is not None and left <= 0:
                    return False
                self._lock.wait(left if left is not None else 0.5)
        return True

    def reset_stats(self):
        """Forget finished requests and batch sizes (e.g. after a warm-up)."""
        with self._lock:
            self.finished = []
            self.batches = []
            self.max_used = self._used

    def close(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        for t in self._threads:
            t.join(timeout=30)
        self._admit_pool.shutdown(wait=True)

    def stats(self) -> Dict[str, float]:
        ok = [r for r in self.finished if r.error is None]
        lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
        t0 = min((r.t_submit for r in self.finished), default=0.0)
        t1 = max((r.t_done for r in self.finished), default=0.0)
        return {"completed": len(ok), "failed": len(self.finished) - len(ok),
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "span_s": t1 - t0,
                "evals_per_s": len(ok) / max(t1 - t0, 1e-9),
                "mean_batch": float(np.mean(self.batches)) if self.batches else 0.0,
                "max_batch_seen": max(self.batches, default=0), "max_bytes_held": self.max_used}

    # ------------------------------------------------------------ internals
    def _finish(self, req: Request, result=None, error=None):
        req.result, req.error = result, error
        req.t_done = time.perf_counter()
        with self._lock:
            self.finished.append(req)
            self._lock.notify_all()
        req.done.set()

    def _schedule(self):
        while True:
            with self._lock:
                while not self._stop and not self._pending and not (self._ready and self._busy < self.n_workers):
                    self._lock.wait(0.05)
                if self._stop:
                    return
                # admission: in arrival order, while the budget allows
                take = None
                if self._pending and self._used + self._pending[0].footprint <= self.budget:
                    take = self._pending.popleft()
                    self._admitting += 1
                    self._used += take.footprint
                    self.max_used = max(self.max_used, self._used)
                # dispatch: a free worker takes the admitted requests
                if self._ready and self._busy + len(self._jobs) < self.n_workers and self._dispatch_now():
                    batch = [self._ready.popleft() for _ in range(min(self.max_batch, len(self._ready)))]
                    self._jobs.append(batch)
                    self._lock.notify_all()
            if take is not None:
                self._admit_pool.submit(self._admit, take)
            else:
                with self._lock:
                    self._lock.wait(0.002)

    def _dispatch_now(self) -> bool:
        """Whether the ready requests go out now (called with the lock held)."""
        if self.window <= 0 or len(self._ready) >= self.max_batch:
            return True
        if not self._pending and not self._admitting:
            return True
        return time.perf_counter() - self._ready[0].t_admit >= self.window

    def _admit(self, req: Request):
        try:
            handle, held = self.engine.admit(req.payload)
        except Exception as e:      # noqa: BLE001 - the request fails, the server goes on
            with self._lock:
                self._used -= req.footprint
                self._admitting -= 1
            self._finish(req, error=f"admission failed: {e}")
            return
        req.t_admit = time.perf_counter()
        with self._lock:
            # keep the estimate as the reservation unless the request holds more
            if held > req.footprint:
                self._used += held - req.footprint
                req.footprint = held
                self.max_used = max(self.max_used, self._used)
            self._handles[req.rid] = handle
            self._ready.append(req)
            self._admitting -= 1
            self._lock.notify_all()

    def _work(self):
        while True:
            with self._lock:
                while not self._stop and not self._jobs:
                    self._lock.wait(0.05)
                if self._stop and not self._jobs:
                    return
                batch = self._jobs.popleft()
                self._busy += 1
                self.batches.append(len(batch))
            handles = [self._handles[r.rid] for r in batch]
            t = time.perf_counter()
            for r in batch:
                r.t_start, r.batch_size = t, len(batch)
            try:
                results = self.engine.run(handles)
                errors = [None] * len(batch)
            except Exception as e:      # noqa: BLE001 - every request of the batch fails
                results, errors = [None] * len(batch), [f"evaluation failed: {e}"] * len(batch)
            for r, h, res, err in zip(batch, handles, results, errors):
                try:
                    self.engine.release(h)
                except Exception:       # noqa: BLE001
                    pass
                with self._lock:
                    self._used -= r.footprint
                    del self._handles[r.rid]
                self._finish(r, result=res, error=err)
            with self._lock:
                self._busy -= 1
                self._lock.notify_all()


_PRECISION_INDEX = {"fp64": 0, "fp32": 1, "bf16x3": 2}


class LrxEngine(Engine):
    """The library as the server's engine: one context per admitted request,
    block tensors materialised on the device at admission, batches evaluated
    with lrx_evaluate_batch (no per-composition tuning or graph capture: every
    batch composition is new, so plans run eagerly with the persistent grid)."""

    def __init__(self, precision: str = "bf16x3", device: int = 0, work_ratio: float = 3.0):
        self.precision = precision
        self.device = device
        self.ratio = work_ratio      # device work buffers per input byte, refined as requests arrive
        self._rlock = threading.Lock()
        self._streams = threading.local()

    @staticmethod
    def input_bytes(st) -> int:
        nC = sum(int(st.nabf[f]) * int(st.nao[f]) * int(st.nao[s]) for f, s in zip(*st.keysC[:2]))
        nV = sum(int(st.nabf[f]) * int(st.nabf[s]) for f, s in zip(*st.keysV[:2]))
        return 32 * (nC + nV) + 8 * int(st.n_tot) ** 2

    def estimate(self, st) -> int:
        with self._rlock:
            return int(self.input_bytes(st) * (1.0 + self.ratio))

    def admit(self, st):
        import torch

        from . import lrx

        # each admitting thread materialises on its own stream, so admissions
        # do not wait for the batches running on the device
        if not hasattr(self._streams, "s"):
            self._streams.s = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(self._streams.s):
            mats = st.materialize(f"cuda:{self.device}")
            ctx = lrx.context_for(st, mats, device=self.device)
        stats = ctx.stats()
        p = _PRECISION_INDEX[self.precision]
        # what the context holds now, plus the work buffers its first
        # evaluation in the serving precision allocates
        held = int(stats["device_bytes"]) + self.input_bytes(st)
        if not stats["work_held"][p]:
            held += int(stats["work_bytes"][p])
        with self._rlock:
            self.ratio = max(self.ratio, held / max(1, self.input_bytes(st)) - 1.0)
        return (ctx, mats, st), held

    def run(self, handles):
        from . import lrx

        # one batched pass per distinct (theta, theta_cs): the thresholds are
        # options of the whole pass
        out = [None] * len(handles)
        groups = {}
        for i, h in enumerate(handles):
            groups.setdefault((h[2].theta, h[2].theta_cs), []).append(i)
        for (theta, theta_cs), idx in groups.items():
            E, F, S = lrx.evaluate_batch([handles[i][0] for i in idx], theta, theta_cs, precision=self.precision,
                                         eager=True, tune=False)
            for k, i in enumerate(idx):
                out[i] = (E[k], F[k], S[k])
        return out

    def release(self, handle):
        handle[0].close()


def poisson_arrivals(n: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of n requests at the given mean rate (per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def replay(server: Server, payloads: List[Any], arrivals: np.ndarray,
           prepare: Optional[Callable[[Any], Any]] = None) -> List[Request]:
    """Submit payloads at the given arrival times (relative to now)."""
    t0 = time.perf_counter()
    reqs = []
    for i, (p, t) in enumerate(zip(payloads, arrivals)):
        if prepare is not None:
            p = prepare(p)
        wait = t0 + float(t) - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        reqs.append(server.submit(Request(i, p)))
    return reqs
