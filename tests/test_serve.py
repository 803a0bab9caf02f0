"""Admission and retirement policy of the serving loop, on a fake executor
(CPU only): budget and slot limits, first-come first-served order without
starvation, refusal of oversized requests, isolation of a failed request,
eviction of every retired slot, overlap of requests (continuous batching)."""
import threading
import time

import numpy as np
import pytest

from paper_1605_03958_amd import inputs, serve
from paper_1605_03958_amd.sscn import (IMAG, REAL, F32, SLOT_CONVERGED, SLOT_DONE, SLOT_EMPTY, SLOT_NONFINITE,
                                      SLOT_RUNNING, Obs, Problem, SlotStatus)


class FakeExecutor:
    """Each job's tag says how many steps it takes and how it ends; the
    footprint is 4 bytes per point.  Records every call."""

    def __init__(self, max_slots):
        self.max_slots = max_slots
        self.slots = {}
        self.calls = []
        self.evicted = []
        self.fail_admit = set()
        self.closed = False
        self.steps_total = 0

    def footprint(self, prob):
        return 4 * prob.points

    def admit(self, slot, prob, psi0, mu_tol, max_steps):
        assert slot not in self.slots, "slot admitted twice"
        tag = psi0["tag"]
        if tag in self.fail_admit:
            raise RuntimeError("admission refused")
        self.slots[slot] = dict(prob=prob, need=psi0["need"], end=psi0.get("end", SLOT_DONE), steps=0, tag=tag,
                                max_steps=max_steps)
        self.calls.append(("admit", slot, tag))

    def step(self, k):
        self.calls.append(("step", k, tuple(sorted(self.slots))))
        self.steps_total += k
        for s in self.slots.values():
            if s["steps"] < s["need"] and s["steps"] < s["max_steps"]:
                s["steps"] = min(s["need"], s["steps"] + k, s["max_steps"])

    def poll(self):
        out = []
        for i in range(self.max_slots):
            s = self.slots.get(i)
            if s is None:
                out.append(SlotStatus(SLOT_EMPTY, 0, 0.0, Obs(0, 0, 0, 0, 0, 0, 0)))
                continue
            st = SLOT_RUNNING if s["steps"] < min(s["need"], s["max_steps"]) else s["end"]
            out.append(SlotStatus(st, s["steps"], 1.0, Obs(s["steps"], 1.0, 0.5, 0.4, 0, 0, 0)))
        return out

    def error(self):
        return False

    def evict(self, slot):
        s = self.slots.pop(slot)
        self.evicted.append(s["tag"])
        self.calls.append(("evict", slot, s["tag"]))
        return ("state", s["tag"])

    def close(self):
        self.closed = True


def prob_of(points):
    return Problem(1, (points, 1, 1), (0.1,), (1.0,), 1.0, 1e-3, IMAG, F32, 1, 10)


def job(tag, points, need, end=SLOT_DONE, kind=serve.GROUND):
    return serve.Job(kind, prob_of(points), {"tag": tag, "need": need, "end": end}, max_steps=1 << 30, tag=tag)


def run_all(server, jobs):
    futs = [server.submit(j) for j in jobs]
    server.close()
    server.run()
    return futs


def test_budget_and_slots_bound_the_running_set():
    ex = FakeExecutor(8)
    srv = serve.Server(budget_bytes=4 * 3000, max_slots=8, tick_steps=10, executor=ex)
    jobs = [job(i, 1000, 30 + 10 * (i % 4)) for i in range(12)]
    futs = run_all(srv, jobs)
    res = [f.result() for f in futs]
    assert all(r.status == SLOT_DONE for r in res)
    assert srv.peak_bytes <= 4 * 3000 and srv.peak_running == 3
    for c in ex.calls:
        if c[0] == "step":
            assert len(c[2]) <= 3
    assert sorted(ex.evicted) == list(range(12))

    ex = FakeExecutor(2)
    srv = serve.Server(budget_bytes=1 << 40, max_slots=2, tick_steps=10, executor=ex)
    futs = run_all(srv, [job(i, 100, 20) for i in range(7)])
    assert all(f.result().status == SLOT_DONE for f in futs)
    assert srv.peak_running == 2


def test_first_come_first_served_without_starvation():
    ex = FakeExecutor(16)
    srv = serve.Server(budget_bytes=4 * 10000, max_slots=16, tick_steps=10, executor=ex)
    # a long small job occupies part of the budget; then a big job (needs the
    # whole budget) queues, followed by small jobs that would fit at once
    jobs = [job(0, 2000, 100)] + [job(1, 10000, 20)] + [job(2 + i, 500, 10) for i in range(6)]
    futs = run_all(srv, jobs)
    res = [f.result() for f in futs]
    assert srv.admit_order == list(range(8))
    big = res[1]
    assert all(r.t_admit >= big.t_admit for r in res[2:])
    assert big.t_admit >= res[0].t_done


def test_oversized_request_is_refused_and_others_run():
    ex = FakeExecutor(4)
    srv = serve.Server(budget_bytes=4 * 1000, max_slots=4, tick_steps=5, executor=ex)
    futs = run_all(srv, [job(0, 500, 10), job(1, 5000, 10), job(2, 500, 10)])
    assert futs[0].result().status == SLOT_DONE and futs[2].result().status == SLOT_DONE
    with pytest.raises(serve.ServerError):
        futs[1].result()
    assert ("admit", 0, 1) not in [c[:3] for c in ex.calls]


def test_failed_request_is_isolated():
    ex = FakeExecutor(4)
    ex.fail_admit.add(3)
    srv = serve.Server(budget_bytes=1 << 30, max_slots=4, tick_steps=5, executor=ex)
    jobs = [job(0, 100, 20), job(1, 100, 12, end=SLOT_NONFINITE), job(2, 100, 30), job(3, 100, 5), job(4, 100, 8)]
    futs = run_all(srv, jobs)
    assert futs[1].result().status == SLOT_NONFINITE
    with pytest.raises(RuntimeError):
        futs[3].result()
    for i in (0, 2, 4):
        r = futs[i].result()
        assert r.status == SLOT_DONE and r.steps == jobs[i].psi0["need"]
    # the refused admission gave its slot and bytes back
    assert srv._used == 0 and len(srv._free) == 4


def test_retired_requests_are_evicted_and_slots_reused():
    ex = FakeExecutor(2)
    srv = serve.Server(budget_bytes=1 << 30, max_slots=2, tick_steps=7, executor=ex)
    futs = run_all(srv, [job(i, 64, 7 * (1 + i % 3), end=SLOT_CONVERGED) for i in range(9)])
    res = [f.result() for f in futs]
    assert [r.psi for r in res] == [("state", i) for i in range(9)]
    assert sorted(ex.evicted) == list(range(9)) and not ex.slots
    used = {c[1] for c in ex.calls if c[0] == "admit"}
    assert used == {0, 1}
    srv.shutdown()
    assert ex.closed


def test_requests_overlap_on_the_device():
    """A request that arrives while another runs joins the running batch
    (continuous batching), instead of waiting for it to finish."""
    class Timed(FakeExecutor):
        def step(self, k):          # a tick takes device time (and frees the GIL)
            super().step(k)
            time.sleep(0.0005)

    ex = Timed(4)
    srv = serve.Server(budget_bytes=1 << 30, max_slots=4, tick_steps=10, executor=ex)
    srv.start()
    f0 = srv.submit(job(0, 100, 10 ** 4))
    while not any(c[0] == "step" for c in ex.calls):
        time.sleep(0.001)
    f1 = srv.submit(job(1, 100, 50))
    r1 = f1.result(timeout=30)
    assert not f0.done()
    steps_with_both = [c for c in ex.calls if c[0] == "step" and c[2] == (0, 1)]
    assert steps_with_both
    srv.close()
    srv.join(30)
    r0 = f0.result(timeout=30)
    assert r0.t_done > r1.t_done and r1.t_admit < r0.t_done


def test_submit_after_close_raises():
    srv = serve.Server(budget_bytes=100, max_slots=1, executor=FakeExecutor(1))
    srv.close()
    with pytest.raises(serve.ServerError):
        srv.submit(job(0, 10, 1))


def test_drive_follows_the_arrival_schedule():
    reqs = inputs.request_stream(40, rate=50.0, seed=3)
    now = [0.0]

    def clock():
        return now[0]

    def sleep(dt):
        now[0] += dt

    class Sink:
        def __init__(self):
            self.times = []

        def submit(self, j):
            self.times.append(clock())
            return j

    sink = Sink()
    futs, late = serve.drive(sink, reqs, make_job=lambda r: r.rid, clock=clock, sleep=sleep)
    assert futs == list(range(40))
    assert np.allclose(sink.times, [r.arrival for r in reqs]) and max(late) == 0.0


def test_request_mix_and_jobs():
    reqs = inputs.request_stream(600, rate=10.0, seed=200)
    kinds = [r.kind for r in reqs]
    frac = kinds.count("ground") / len(kinds)
    assert 0.65 <= frac <= 0.75
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 0.1) < 0.015 and np.all(gaps > 0)
    assert {r.draw.dim for r in reqs} == {1, 2, 3}
    assert inputs.request_stream(5, 10.0, seed=200)[3].draw == reqs[3].draw
    small = [r for r in reqs if r.draw.dim == 1][:2] + [r for r in reqs if r.draw.dim == 2][:1]
    for r in small:
        j = serve.job_from_request(r)
        assert j.prob.shape == np.asarray(j.psi0).shape
        h = r.draw.dx[0]
        if r.kind == "ground":
            assert j.prob.mode == IMAG and j.mu_tol == 1e-6 and abs(j.prob.dt - 0.1 * h * h) < 1e-15
        else:
            assert j.prob.mode == REAL and j.max_steps == 2000 and j.psi0.dtype == np.complex64
            assert abs(j.prob.dt - 0.02 * h * h) < 1e-15


def test_latency_stats():
    rs = [serve.Result(i, serve.GROUND if i % 3 else serve.DYNAMICS, None, SLOT_DONE, 10, None, None, 100,
                       t_submit=float(i), t_admit=float(i) + 0.5, t_done=float(i) + 1.0 + i / 100.0)
          for i in range(100)]
    s = serve.latency_stats(rs, 0.0, 10.0)
    lat = 1.0 + np.arange(100) / 100.0
    assert s["p50_s"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_s"] == pytest.approx(np.percentile(lat, 99))
    assert s["req_per_s"] == pytest.approx(10.0) and s["ptsteps_per_s"] == pytest.approx(100 * 10 * 100 / 10.0)
    assert s["wait_p50_s"] == pytest.approx(0.5)


def test_voided_launch_results_are_not_handed_out():
    """When the batch reports that a bounded wait gave up, the server hands
    out no result: running and queued requests fail with the error."""
    class Broken(FakeExecutor):
        def error(self):
            return any(s["steps"] >= 10 for s in self.slots.values())

    ex = Broken(1)
    srv = serve.Server(budget_bytes=1 << 30, max_slots=1, tick_steps=10, executor=ex)
    futs = [srv.submit(job(0, 100, 10)), srv.submit(job(1, 100, 10))]
    srv.close()
    with pytest.raises(serve.ServerError):
        srv.run()
    for f in futs:
        with pytest.raises(serve.ServerError):
            f.result(timeout=1)
    assert not srv.results
