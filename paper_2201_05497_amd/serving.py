"""Continuous-batching server for dynamic-frame LM-SPDHG reconstructions.

Requests (listmode frames of uneven size, each with its own image grid,
subset count and number of epochs) arrive at any time.  The server admits
them as GPU memory and slots free up, keeps every admitted reconstruction
resident in HBM (its plan, image and dual state), and interleaves their
work: each admitted request runs on its own HIP stream (default priority)
and the scheduler issues one epoch per request per tick, so kernels of
different requests overlap on the device.  Admission is first come, first
served against an HBM budget, using lm_plan_bytes for the plan's footprint
plus the request's own inputs.  Sensitivity images are computed once per
scanner and image geometry (lm_sens) and shared.  Plans allocate
stream-ordered, so admitting or finishing a request never waits for the
work of the others.

Every step of a reconstruction runs in the library's kernels; this module
only schedules them.  The method is unchanged: a served reconstruction is
the same sequence of LM-SPDHG updates as a plain solver run with the same
inputs, up to the summation order of float32 atomics.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from concurrent.futures import CancelledError, Future
from typing import Dict, List, Optional

import numpy as np
import torch

from . import Geometry, Plan, lm_plan_bytes, lm_sens
from .sequence import subset_sequence

__all__ = ["Request", "Result", "Server", "solve", "latency_stats"]


@dataclasses.dataclass
class Request:
    """One frame to reconstruct.  events: int16 [N, 5]; s: float32 [N];
    x0: float32 image [nz, ny, nx]; the subset sequence is drawn from
    ``seq_seed`` (SplitMix64, global update counter) unless ``seq`` lists the
    choices of every update explicitly."""
    geom: Geometry
    events: np.ndarray
    s: np.ndarray
    x0: np.ndarray
    n_subsets: int = 28
    epochs: int = 3
    beta: float = 0.03
    rho: float = 0.999
    gamma: Optional[float] = None
    seq_seed: int = 0
    seq: Optional[np.ndarray] = None
    name: str = ""

    def n_updates(self) -> int:
        return 2 * self.n_subsets * self.epochs

    def sequence(self) -> np.ndarray:
        if self.seq is not None:
            return np.asarray(self.seq, dtype=np.int32)
        return subset_sequence(self.seq_seed, 0, self.n_updates(), self.n_subsets)


@dataclasses.dataclass
class Result:
    name: str
    x: np.ndarray
    events: int
    epochs: int
    t_submit: float
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


def _gamma(req: Request) -> float:
    return float(req.gamma) if req.gamma is not None else float(np.float32(3.0 / float(np.max(req.x0))))


def _geom_key(g: Geometry):
    return (g.n_cry, g.n_ring, g.n, g.h, g.n_tof, g.tof_bin, g.tof_fwhm, g.tof_nsigma, g.tof_on,
            g.det.data_ptr())


class _SensCache:
    def __init__(self):
        self._c: Dict[tuple, torch.Tensor] = {}
        self._lock = threading.Lock()

    def get(self, geom: Geometry, g: Optional[torch.Tensor] = None) -> torch.Tensor:
        key = _geom_key(geom)
        with self._lock:
            if key not in self._c and g is not None:
                self._c[key] = g
            if key not in self._c:
                s = torch.cuda.Stream(device=geom.device)
                with torch.cuda.stream(s):
                    g = lm_sens(geom)
                s.synchronize()
                self._c[key] = g
            return self._c[key]

    def has(self, geom: Geometry) -> bool:
        with self._lock:
            return _geom_key(geom) in self._c

    def bytes(self) -> int:
        with self._lock:
            return sum(t.numel() * 4 for t in self._c.values())


def footprint(req: Request) -> int:
    """Device bytes a request holds while admitted: its plan (including the
    temporaries of plan creation), its events, contamination and image."""
    n = len(req.events)
    return lm_plan_bytes(req.geom, n, req.n_subsets) + n * (10 + 4) + 4 * req.geom.nvox


class _Active:
    def __init__(self, req: Request, fut: Future, t_submit: float):
        self.req, self.fut, self.t_submit = req, fut, t_submit
        self.t_admit = 0.0
        self.stream: Optional[torch.cuda.Stream] = None
        self.plan: Optional[Plan] = None
        self.x: Optional[torch.Tensor] = None
        self.inputs = ()
        self.seq = None
        self.issued = 0
        self.pending: collections.deque = collections.deque()  # events of queued epochs
        self.bytes = 0
        self.error: Optional[BaseException] = None
        self.cancel = False  # stop after the epochs in flight


class Server:
    """``Server(hbm_budget)``; ``submit(request) -> Future[Result]``.

    hbm_budget: device bytes the resident reconstructions may hold (shared
    sensitivity images included; the scheduler thread alone updates the
    plans' share).  max_active: most reconstructions admitted at once (being
    prepared or running).  epochs_in_flight: epochs queued ahead on each
    request's stream.  A request whose footprint alone exceeds the budget
    fails with MemoryError.  ``cancel(future)`` drops a waiting request or
    stops a running one after its epochs in flight, freeing its slot and
    memory.  ``close()`` waits for the admitted and queued work.

    Two threads: the scheduler admits requests, issues epochs and completes
    results; a preparation thread uploads each admitted request's inputs
    and builds its plan (plan creation is synchronous on the request's own
    stream), so that the scheduler keeps the running requests fed
    meanwhile."""

    def __init__(self, hbm_budget: int, device="cuda:0", max_active: int = 8, epochs_in_flight: int = 2):
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.in_flight = max(1, int(epochs_in_flight))
        self._q: "queue.Queue[tuple]" = queue.Queue()
        self._cancel_q: "queue.Queue[Future]" = queue.Queue()
        self._cancelled: set = set()  # ids of futures whose requests are being cancelled
        self._prep_q: "queue.Queue[Optional[_Active]]" = queue.Queue()
        self._ready: "queue.Queue[_Active]" = queue.Queue()
        self._waiting: collections.deque = collections.deque()
        self._active: List[_Active] = []
        self._preparing = 0
        self._sens = _SensCache()
        self._used = 0
        self.peak_bytes = 0
        self.results: List[Result] = []
        self._stop = False
        self._err: Optional[BaseException] = None
        self._thread = threading.Thread(target=self._loop, name="lm-serving", daemon=True)
        self._prep = threading.Thread(target=self._prep_loop, name="lm-serving-prep", daemon=True)
        self._prep.start()
        self._thread.start()

    # ------------------------------------------------------------ client API

    def warm(self, geom: Geometry, g: Optional[torch.Tensor] = None) -> None:
        """Compute (or take g as) the sensitivity image of a geometry and
        keep it, before requests for it arrive."""
        self._sens.get(geom, g)

    def submit(self, req: Request) -> Future:
        if self._stop:
            raise RuntimeError("server closed")
        fut: Future = Future()
        self._q.put((req, fut, time.perf_counter()))
        return fut

    def cancel(self, fut: Future) -> bool:
        """Cancels a request.  A waiting one is dropped (``fut.cancelled()``
        is then true).  A running one, being prepared or with epochs on the
        device, stops after the epochs already queued: its plan and memory
        are released and ``fut.result()`` raises CancelledError (a request
        that completes before the scheduler acts keeps its result).  Returns
        False if the request had already finished."""
        if fut.done():
            return False
        if fut.cancel():
            return True
        self._cancel_q.put(fut)
        return True

    def close(self, wait: bool = True) -> None:
        self._stop = True
        if wait:
            self._thread.join()
            self._prep.join()
        if self._err is not None:
            raise RuntimeError("serving loop failed") from self._err

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ scheduler

    def _loop(self):
        try:
            torch.cuda.set_device(self.device)
            while True:
                self._drain_queue()
                self._drain_cancels()
                self._collect_ready()
                self._admit()
                progressed = self._tick()
                progressed |= self._complete()
                if (self._stop and not self._waiting and not self._active and not self._preparing
                        and self._q.empty()):
                    break
                if not progressed:
                    time.sleep(0.0002)
        except BaseException as e:  # surface the failure to every waiting client
            self._err = e
            for a in list(self._active) + [w for w in self._waiting]:
                fut = a.fut if isinstance(a, _Active) else a[1]
                if not fut.done():
                    fut.set_exception(e)
        finally:
            self._prep_q.put(None)

    def _drain_queue(self):
        while True:
            try:
                req, fut, t = self._q.get_nowait()
            except queue.Empty:
                return
            self._waiting.append((req, fut, t))

    def _drain_cancels(self):
        while True:
            try:
                fut = self._cancel_q.get_nowait()
            except queue.Empty:
                return
            self._cancelled.add(id(fut))
            for a in self._active:
                if a.fut is fut:
                    a.cancel = True

    def _finish_cancelled(self, a: _Active):
        """Frees a cancelled request once its queued work is done."""
        self._cancelled.discard(id(a.fut))
        if a.stream is not None:
            a.stream.synchronize()
        self._release(a)
        if not a.fut.done():
            a.fut.set_exception(CancelledError(f"request {a.req.name} cancelled"))

    def _admit(self):
        while self._waiting and len(self._active) + self._preparing < self.max_active:
            req, fut, t = self._waiting[0]
            if fut.cancelled():
                self._waiting.popleft()
                continue
            need = footprint(req)
            need_sens = 0 if self._sens.has(req.geom) else 4 * req.geom.nvox
            shared = self._sens.bytes()
            if need + need_sens + shared > self.budget:
                self._waiting.popleft()
                fut.set_exception(MemoryError(f"request needs {need + need_sens} bytes, budget {self.budget}"))
                continue
            if self._used + need + need_sens + shared > self.budget:
                return  # first come, first served: wait for memory
            self._waiting.popleft()
            if not fut.set_running_or_notify_cancel():
                continue
            a = _Active(req, fut, t)
            a.bytes = need
            self._used += need
            self.peak_bytes = max(self.peak_bytes, self._used + shared + need_sens)
            self._preparing += 1
            self._prep_q.put(a)

    def _prep_loop(self):
        torch.cuda.set_device(self.device)
        while True:
            a = self._prep_q.get()
            if a is None:
                return
            try:
                self._start(a)
            except BaseException as e:
                a.error = e
            self._ready.put(a)

    def _start(self, a: _Active):
        """Preparation thread: inputs to the device, plan, initialisation."""
        req = a.req
        a.t_admit = time.perf_counter()
        g = self._sens.get(req.geom)
        a.stream = torch.cuda.Stream(device=self.device)
        with torch.cuda.stream(a.stream):
            ev = torch.from_numpy(np.ascontiguousarray(req.events, dtype=np.int16)).to(self.device)
            s = torch.from_numpy(np.ascontiguousarray(req.s, dtype=np.float32)).to(self.device)
            a.x = torch.from_numpy(np.ascontiguousarray(req.x0, dtype=np.float32)).to(self.device)
            a.plan = Plan(req.geom, ev, s, req.n_subsets, _gamma(req), req.rho, req.beta, g=g)
            a.plan.init(a.x)
        a.inputs = (ev, s)
        a.seq = req.sequence()

    def _collect_ready(self):
        while True:
            try:
                a = self._ready.get_nowait()
            except queue.Empty:
                return
            self._preparing -= 1
            if a.error is not None:
                self._cancelled.discard(id(a.fut))
                self._release(a)
                if not a.fut.done():
                    a.fut.set_exception(a.error)
                continue
            if id(a.fut) in self._cancelled:  # cancelled while being prepared
                self._finish_cancelled(a)
                continue
            self._active.append(a)

    def _tick(self) -> bool:
        progressed = False
        for a in self._active:
            if a.fut.cancelled() or a.cancel:
                continue
            while a.pending and a.pending[0].query():
                a.pending.popleft()
            step = 2 * a.req.n_subsets
            # keep up to `in_flight` epochs queued on the request's stream
            while a.issued < len(a.seq) and len(a.pending) < self.in_flight:
                with torch.cuda.stream(a.stream):
                    a.plan.epoch(a.x, a.seq[a.issued:a.issued + step])
                    ev = torch.cuda.Event()
                    ev.record(a.stream)
                a.pending.append(ev)
                a.issued += step
                progressed = True
        return progressed

    def _release(self, a: _Active):
        if a.plan is not None:
            a.plan.destroy()
        a.plan = a.x = None
        a.inputs = ()
        self._used -= a.bytes

    def _complete(self) -> bool:
        keep = []
        done_any = False
        for a in self._active:
            if a.cancel:
                if all(e.query() for e in a.pending):
                    self._finish_cancelled(a)
                    done_any = True
                else:
                    keep.append(a)
                continue
            done = a.issued >= len(a.seq) and all(e.query() for e in a.pending)
            if a.fut.cancelled():
                done = True
            if not done:
                keep.append(a)
                continue
            done_any = True
            a.stream.synchronize()
            if not a.fut.cancelled():
                with torch.cuda.stream(a.stream):
                    x = a.x.cpu().numpy()
                res = Result(a.req.name, x, len(a.req.events), a.req.epochs, a.t_submit, a.t_admit,
                             time.perf_counter())
                self.results.append(res)
                a.fut.set_result(res)
            self._release(a)
        self._active = keep
        return done_any


def solve(req: Request, device="cuda:0", g: Optional[torch.Tensor] = None) -> np.ndarray:
    """The plain solver: one reconstruction on the current stream, start to
    finish (the baseline the server is compared with).  g: the sensitivity
    image of the request's geometry if already computed (else lm_sens)."""
    dev = torch.device(device)
    ev = torch.from_numpy(np.ascontiguousarray(req.events, dtype=np.int16)).to(dev)
    s = torch.from_numpy(np.ascontiguousarray(req.s, dtype=np.float32)).to(dev)
    x = torch.from_numpy(np.ascontiguousarray(req.x0, dtype=np.float32)).to(dev)
    if g is None:
        g = lm_sens(req.geom)
    with Plan(req.geom, ev, s, req.n_subsets, _gamma(req), req.rho, req.beta, g=g) as plan:
        plan.init(x)
        plan.epoch(x, req.sequence())
        out = x.cpu().numpy()
    return out


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    t0 = min(r.t_submit for r in results)
    t1 = max(r.t_done for r in results)
    ev = sum(r.events * r.epochs for r in results)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": t1 - t0, "events_per_s": ev / (t1 - t0),
            "requests": len(results)}
