"""GPU tests of the serving loop: requests that arrive while others run are
admitted as slots and memory free up, and each request's result is the same
(bitwise) whether it ran alone or in the mix; a request that blows up does
not disturb the others."""
import time

import numpy as np
import pytest

import oracle
from paper_1605_03958_amd import inputs, serve
from paper_1605_03958_amd.sscn import F32, IMAG, REAL, SLOT_CONVERGED, SLOT_DONE, SLOT_NONFINITE, Problem

pytestmark = pytest.mark.gpu


def small_jobs():
    """Ground-state and dynamics requests of all three dimensions, small
    enough for a test, in the request-mix parameter ranges."""
    jobs = []
    specs = [
        (1, (3000, 1, 1), 0.08, IMAG), (2, (96, 80, 1), 0.15, REAL), (3, (40, 36, 44), 0.2, IMAG),
        (1, (2048, 1, 1), 0.1, REAL), (2, (128, 128, 1), 0.12, IMAG), (3, (48, 48, 48), 0.18, REAL),
        (1, (5000, 1, 1), 0.05, IMAG), (2, (70, 150, 1), 0.2, IMAG), (3, (30, 50, 40), 0.25, IMAG),
        (2, (200, 64, 1), 0.1, REAL),
    ]
    rng = np.random.default_rng(77)
    for i, (dim, n, h, mode) in enumerate(specs):
        om = tuple(float(x) for x in rng.uniform(0.5, 4.0, size=dim))
        g = float(10 ** rng.uniform(0, 2))
        dx = (h,) * dim
        psi0 = inputs.ho_gaussian(dim, n, dx, om, noise=1e-3, seed=300 + i)
        if mode == IMAG:
            p = Problem(dim, n, dx, om, g, 0.1 * h * h, IMAG, F32, 1, 10)
            jobs.append(serve.Job(serve.GROUND, p, psi0, mu_tol=1e-5, max_steps=3000, tag=i))
        else:
            p = Problem(dim, n, dx, om, g, 0.02 * h * h, REAL, F32, 0, 50)
            jobs.append(serve.Job(serve.DYNAMICS, p, psi0.astype(np.complex64), max_steps=300, tag=i))
    return jobs


def serve_all(jobs, budget, gaps=None, tick=10, slots=8):
    srv = serve.Server(budget_bytes=budget, max_slots=slots, tick_steps=tick)
    srv.start()
    futs = []
    for k, j in enumerate(jobs):
        if gaps is not None:
            time.sleep(gaps[k])
        futs.append(srv.submit(j))
    srv.close()
    srv.join(120)
    res = [f.result(timeout=1) for f in futs]
    srv.ex.close()
    return srv, res


def test_each_request_is_the_same_alone_and_in_the_mix():
    jobs = small_jobs()
    fps = [serve.footprint(j.prob) for j in jobs]
    # a budget that holds about three requests at a time: later arrivals wait
    budget = int(sorted(fps)[-1] + sorted(fps)[-2] + sorted(fps)[-3])
    gaps = np.random.default_rng(5).exponential(0.01, size=len(jobs))
    srv, mix = serve_all(jobs, budget, gaps=gaps)
    print(f"mix: peak running {srv.peak_running}, peak bytes {srv.peak_bytes} of {budget}, ticks {srv.ticks}",
          flush=True)
    assert srv.peak_bytes <= budget and srv.peak_running >= 2
    assert srv.admit_order == sorted(srv.admit_order)
    # overlap: some request was admitted while an earlier one was still running
    assert any(b.t_admit < a.t_done for a, b in zip(mix, mix[1:]))
    for j, r in zip(jobs, mix):
        alone = serve_all([j], 1 << 40)[1][0]
        print(f"request {j.tag} dim={j.prob.dim} n={j.prob.n} {j.kind}: status {r.status} steps {r.steps} "
              f"latency {r.latency * 1e3:.1f} ms", flush=True)
        assert r.status == alone.status and r.steps == alone.steps
        assert r.status == (SLOT_CONVERGED if j.kind == serve.GROUND else SLOT_DONE) or r.steps == j.max_steps
        assert np.array_equal(r.psi.cpu().numpy(), alone.psi.cpu().numpy())
        assert r.obs.mu == alone.obs.mu and r.obs.energy == alone.obs.energy


def test_served_requests_match_the_oracle():
    jobs = [j for j in small_jobs() if j.prob.points <= 130000][:4]
    _, res = serve_all(jobs, 1 << 40)
    for j, r in zip(jobs, res):
        p = j.prob
        op = oracle.Problem(p.dim, p.n, p.dx, p.omega, p.g, p.dt, p.mode, p.renorm_every)
        ref = oracle.run(op, np.asarray(j.psi0, dtype=np.complex128), r.steps).psi
        got = r.psi.cpu().numpy().astype(np.complex128)
        err = np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel())
        print(f"request {j.tag}: {r.steps} steps, rel L2 vs oracle {err:.2e}", flush=True)
        assert err <= 5e-5


def test_blown_up_request_does_not_disturb_the_others():
    jobs = small_jobs()[:5]
    bad = jobs[4]
    psi = np.array(bad.psi0, copy=True)
    psi.flat[psi.size // 2] = np.nan
    broken = serve.Job(bad.kind, bad.prob, psi, bad.mu_tol, bad.max_steps, tag="bad")
    _, ref = serve_all(jobs[:4], 1 << 40)
    _, got = serve_all(jobs[:2] + [broken] + jobs[2:4], 1 << 40)
    assert got[2].status == SLOT_NONFINITE
    for a, b in zip(ref, got[:2] + got[3:]):
        assert a.status == b.status and a.steps == b.steps
        assert np.array_equal(a.psi.cpu().numpy(), b.psi.cpu().numpy())
