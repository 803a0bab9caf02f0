"""Serving loop over the batched persistent step (continuous batching).

Requests are ground-state solves (imaginary time, renormalised every step,
run until the chemical potential changes by less than ``mu_tol`` between two
observations) and dynamics solves (real time, a fixed number of steps) of
1D/2D/3D trap problems of different sizes, in the FP32 form.  The server
keeps every admitted wavefunction resident in device memory and advances all
of them together, ``tick_steps`` launches of the persistent step at a time.
Between ticks it retires finished requests (their slot and memory return to
the pool) and admits waiting ones.

Admission is first-come first-served by HBM footprint: the request at the
head of the queue is admitted when a slot is free and its footprint (state
plus workspace: the Thomas tables and the reduction partials) fits in what
the budget has left; nothing behind it overtakes it, so a large request
cannot be starved by a stream of small ones.  A request whose footprint
exceeds the whole budget is refused at submission.

An instance's results do not depend on what else is in the batch (tile
shapes depend only on its own shape, reductions have fixed slots and a fixed
order), so a request gives the same state alone and in any mix.

Latency is measured from ``submit`` to the poll that sees the request
finished.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import inputs
from .sscn import F32, IMAG, REAL, SLOT_RUNNING, Problem, batch_workspace_bytes, state_bytes

GROUND = "ground"
DYNAMICS = "dynamics"


@dataclass
class Job:
    """One solve: the problem, its initial state and its stop rule."""
    kind: str                 # GROUND or DYNAMICS
    prob: Problem
    psi0: object              # numpy array or device tensor, shape prob.shape
    mu_tol: float = 0.0       # > 0: stop when |mu - mu_prev| < mu_tol
    max_steps: int = 1 << 40  # stop after this many steps
    keep_state: bool = True   # keep the final state (device tensor) in the result
    tag: object = None        # caller's label, returned in the result


@dataclass
class Result:
    rid: int
    kind: str
    tag: object
    status: int               # SLOT_CONVERGED, SLOT_DONE, SLOT_NONFINITE
    steps: int
    obs: object               # sscn.Obs of the last observation
    psi: object               # final state (device tensor) or None
    points: int
    t_submit: float
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit

    @property
    def wait(self) -> float:
        return self.t_admit - self.t_submit


class ServerError(RuntimeError):
    pass


def footprint(prob: Problem) -> int:
    """HBM bytes a request keeps resident while admitted: its state plus its
    batch workspace (Thomas tables and reduction partials)."""
    return state_bytes(prob) + batch_workspace_bytes(prob)


# Work-item split of the serving batch: a serving batch usually holds a few
# tens of requests, so each instance is cut finer than in a batch that fills
# the device, which finishes the running requests sooner (sscn_batch_set_split).
SERVE_SPLIT = 64


class BatchExecutor:
    """The device side of the server: one ``sscn.Batch`` on its own stream."""

    def __init__(self, max_slots: int, max_items: int = 1 << 20, device: str = "cuda", split: int = SERVE_SPLIT):
        import torch
        from .sscn import Batch
        self.stream = torch.cuda.Stream(device=device)
        self.batch = Batch(max_slots, max_items=max_items, device=device, stream=self.stream, split=split)

    def footprint(self, prob: Problem) -> int:
        return footprint(prob)

    def admit(self, slot, prob, psi0, mu_tol, max_steps):
        self.batch.admit(slot, prob, psi0, mu_tol=mu_tol, max_steps=max_steps)

    def step(self, k: int):
        self.batch.step(k)

    def poll(self):
        return self.batch.poll(wait=True)

    def error(self) -> bool:
        return self.batch.error()

    def evict(self, slot):
        return self.batch.evict(slot)

    def close(self):
        self.batch.close()


@dataclass
class _Entry:
    rid: int
    job: Job
    fut: Future
    fp: int
    t_submit: float
    t_admit: float = 0.0
    slot: int = -1


class Server:
    """Continuous-batching server.  ``submit`` may be called from any thread;
    ``run`` (or the thread ``start`` launches) drives the device until
    ``close`` has been called and every accepted request has finished."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, tick_steps: int = 20,
                 executor=None, clock: Callable[[], float] = time.perf_counter, error_every: int = 16):
        if budget_bytes <= 0 or max_slots <= 0 or tick_steps <= 0:
            raise ValueError("budget, slots and tick must be positive")
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.tick = int(tick_steps)
        self.ex = executor if executor is not None else BatchExecutor(max_slots)
        self.clock = clock
        self.error_every = int(error_every)
        self._cv = threading.Condition()
        self._pending: collections.deque = collections.deque()
        self._free = list(range(self.max_slots - 1, -1, -1))
        self._running: dict = {}
        self._used = 0
        self._closed = False
        self._next = 0
        self._thread: Optional[threading.Thread] = None
        self.results: list = []
        self.admit_order: list = []   # rids in admission order
        self.ticks = 0
        self.peak_bytes = 0
        self.peak_running = 0

    # ---- client side -----------------------------------------------------
    def submit(self, job: Job) -> Future:
        fut: Future = Future()
        fp = int(self.ex.footprint(job.prob))
        with self._cv:
            if self._closed:
                raise ServerError("server is closed")
            rid = self._next
            self._next += 1
            if fp > self.budget:
                fut.set_exception(ServerError(f"request {rid} needs {fp} bytes, budget is {self.budget}"))
                return fut
            self._pending.append(_Entry(rid, job, fut, fp, self.clock()))
            self._cv.notify()
        return fut

    def close(self) -> None:
        """No more submissions; the loop ends once the accepted ones finish."""
        with self._cv:
            self._closed = True
            self._cv.notify()

    # ---- device side -----------------------------------------------------
    def start(self) -> None:
        self._thread = threading.Thread(target=self.run, name="sscn-serve", daemon=True)
        self._thread.start()

    def join(self, timeout: Optional[float] = None) -> None:
        if self._thread is not None:
            self._thread.join(timeout)

    def _admissible(self) -> list:
        """Head-of-queue admissions that fit (called with the lock held)."""
        out = []
        while self._pending and self._free:
            e = self._pending[0]
            if self._used + e.fp > self.budget:
                break
            self._pending.popleft()
            e.slot = self._free.pop()
            self._used += e.fp
            out.append(e)
        return out

    def _admit(self, e: _Entry) -> None:
        j = e.job
        try:
            self.ex.admit(e.slot, j.prob, j.psi0, j.mu_tol, j.max_steps)
        except Exception as exc:        # invalid problem, work list full, ...
            with self._cv:
                self._free.append(e.slot)
                self._used -= e.fp
            e.fut.set_exception(exc)
            return
        e.t_admit = self.clock()
        self._running[e.slot] = e
        self.admit_order.append(e.rid)
        self.peak_bytes = max(self.peak_bytes, self._used)
        self.peak_running = max(self.peak_running, len(self._running))

    def _retire(self, e: _Entry, st, now: float) -> None:
        psi = self.ex.evict(e.slot)
        r = Result(e.rid, e.job.kind, e.job.tag, st.state, st.steps, st.obs,
                   psi if e.job.keep_state else None, e.job.prob.points, e.t_submit, e.t_admit, now)
        del self._running[e.slot]
        with self._cv:
            self._free.append(e.slot)
            self._used -= e.fp
        self.results.append(r)
        e.fut.set_result(r)

    def _fail_running(self, exc: Exception) -> None:
        for slot, e in list(self._running.items()):
            try:
                self.ex.evict(slot)
            except Exception:
                pass
            e.fut.set_exception(exc)
        self._running.clear()

    def run(self) -> None:
        try:
            while True:
                with self._cv:
                    while not self._pending and not self._running and not self._closed:
                        self._cv.wait()
                    if self._closed and not self._pending and not self._running:
                        return
                    todo = self._admissible()
                for e in todo:
                    self._admit(e)
                if not self._running:
                    # every admission of this pass failed (their futures
                    # hold the errors): look at the queue again
                    continue
                self.ex.step(self.tick)
                st = self.ex.poll()
                self.ticks += 1
                now = self.clock()
                done = [(slot, e) for slot, e in self._running.items() if st[slot].state != SLOT_RUNNING]
                # the launch error flag (a bounded wait that gave up voids the
                # batch's results) is checked before anything is handed out,
                # and every error_every ticks otherwise
                if (done or (self.error_every and self.ticks % self.error_every == 0)) and self.ex.error():
                    raise ServerError("a bounded wait of the persistent step gave up; results of the batch are void")
                for slot, e in done:
                    self._retire(e, st[slot], now)
        except Exception as exc:
            self._fail_running(exc)
            with self._cv:
                pend = list(self._pending)
                self._pending.clear()
                self._closed = True
            for e in pend:
                e.fut.set_exception(exc)
            raise

    def shutdown(self) -> None:
        self.close()
        self.join()
        self.ex.close()


# ---------------------------------------------------------------------------
# the synthetic request mix
# ---------------------------------------------------------------------------

def job_from_request(req: inputs.Request, ground_tol: float = 1e-6, ground_cap: int = 300000,
                     dyn_steps: int = 2000, keep_state: bool = False) -> Job:
    """Ground-state requests: imaginary time from the noisy oscillator
    Gaussian, dt = 0.1 dx^2, observed every 10 steps, stopped at
    |delta mu| < ground_tol.  Dynamics requests: real time, dt = 0.02 dx^2,
    from the same kind of seeded Gaussian, dyn_steps steps, observed every
    100 steps and at the end."""
    d = req.draw
    h = min(d.dx[:d.dim])
    psi0 = inputs.ho_gaussian(d.dim, d.n, d.dx, d.omega, noise=1e-3, seed=d.seed)
    if req.kind == "ground":
        p = Problem(d.dim, d.n, d.dx[:d.dim], d.omega[:d.dim], d.g, 0.1 * h * h, IMAG, F32, 1, 10)
        return Job(GROUND, p, psi0, mu_tol=ground_tol, max_steps=ground_cap, keep_state=keep_state, tag=req.rid)
    p = Problem(d.dim, d.n, d.dx[:d.dim], d.omega[:d.dim], d.g, 0.02 * h * h, REAL, F32, 0, 100)
    return Job(DYNAMICS, p, psi0.astype(np.complex64), mu_tol=0.0, max_steps=dyn_steps,
               keep_state=keep_state, tag=req.rid)


def drive(server: Server, reqs, make_job=job_from_request, clock: Callable[[], float] = time.perf_counter,
          sleep: Callable[[float], None] = time.sleep):
    """Client: submit each request at its arrival time (seconds after the
    call), building its initial state just before.  Returns the futures and
    the lateness of each submission against its scheduled time."""
    t0 = clock()
    futs, late = [], []
    for r in reqs:
        job = make_job(r)
        dt = t0 + r.arrival - clock()
        if dt > 0:
            sleep(dt)
        late.append(max(0.0, clock() - (t0 + r.arrival)))
        futs.append(server.submit(job))
    return futs, late


def latency_stats(results, t0: float, t1: float) -> dict:
    lat = np.array([r.latency for r in results], dtype=np.float64)
    wait = np.array([r.wait for r in results], dtype=np.float64)
    ptsteps = float(sum(r.steps * r.points for r in results))
    el = max(t1 - t0, 1e-12)
    out = {
        "requests": len(results),
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_s": float(lat.mean()) if len(lat) else None,
        "max_s": float(lat.max()) if len(lat) else None,
        "wait_p50_s": float(np.percentile(wait, 50)) if len(wait) else None,
        "wait_p99_s": float(np.percentile(wait, 99)) if len(wait) else None,
        "req_per_s": len(results) / el,
        "ptsteps_per_s": ptsteps / el,
        "elapsed_s": el,
    }
    for kind in (GROUND, DYNAMICS):
        lk = np.array([r.latency for r in results if r.kind == kind])
        if len(lk):
            out[f"{kind}_p50_s"] = float(np.percentile(lk, 50))
            out[f"{kind}_p99_s"] = float(np.percentile(lk, 99))
    return out
