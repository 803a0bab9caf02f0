"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  FP64 bar: relative L2 of psi <= 1e-10 after 1000
steps (1e-12 for the short runs below), observables to 1e-10 relative."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1605_03958_amd import autotune, inputs, sscn
from paper_1605_03958_amd.sscn import F32, F64, IMAG, REAL, Problem

TILES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1605_03958_amd",
                     "tiles_gfx950.json")

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oprob(p: Problem) -> oracle.Problem:
    return oracle.Problem(p.dim, p.n, p.dx, p.omega, p.g, p.dt, p.mode, p.renorm_every)


def initial(p: Problem, seed=0):
    if p.mode == IMAG:
        return inputs.ho_gaussian(p.dim, p.n, p.dx, p.omega, noise=1e-3, seed=seed)
    return inputs.thomas_fermi(p.dim, p.n, p.dx, p.omega, 1.25 * p.g + 1.0, phase_sigma=0.05, seed=seed)


def run_both(p: Problem, steps: int, seed=0, chunks=None):
    psi0 = initial(p, seed)
    s = sscn.Solver(p, psi0)
    s.step(steps)
    got = s.state()
    ob = s.observe()
    s.close()
    ref = oracle.run(oprob(p), psi0, steps)
    return got, ref.psi, ob, oracle.observe(oprob(p), ref.psi)


SMALL = [
    # dim, n, dx, omega
    (1, (1, 1, 1), (0.3,), (1.0,)),
    (1, (2, 1, 1), (0.3,), (1.0,)),
    (1, (5, 1, 1), (0.3,), (1.0,)),
    (1, (63, 1, 1), (0.2,), (1.3,)),
    (1, (65, 1, 1), (0.2,), (1.3,)),
    (1, (257, 1, 1), (0.1,), (1.1,)),
    (1, (3000, 1, 1), (0.01,), (1.1,)),      # several waves per x line
    (2, (3, 2, 1), (0.4, 0.3), (1.0, 2.0)),
    (2, (65, 63, 1), (0.2, 0.25), (1.0, 1.7)),
    (2, (130, 257, 1), (0.1, 0.08), (1.0, 1.5)),
    (3, (5, 3, 2), (0.5, 0.4, 0.3), (1.0, 1.5, 2.0)),
    (3, (17, 33, 9), (0.3, 0.2, 0.4), (1.2, 1.0, 2.0)),
    (3, (64, 48, 40), (0.2, 0.25, 0.3), (1.0, 1.5, 2.0)),
    (3, (65, 70, 33), (0.2, 0.2, 0.3), (1.0, 1.5, 2.0)),
    (2, (48, 700, 1), (0.2, 0.02), (1.0, 1.5)),   # long y lines over 8 lanes (complex128)
    (2, (32, 2000, 1), (0.2, 0.01), (1.0, 1.5)),  # 2000-point y lines: 16 waves x 8 lanes x 16 (complex128)
]


@pytest.mark.parametrize("dim,n,dx,omega", SMALL)
@pytest.mark.parametrize("mode", [IMAG, REAL])
def test_fp64_matches_oracle_small(dim, n, dx, omega, mode):
    h = min(dx)
    dt = 0.1 * h * h if mode == IMAG else 0.02 * h * h
    p = Problem(dim, n, dx, omega, 7.0, dt, mode, F64, 1 if mode == IMAG else 0)
    print(f"case dim={dim} n={n} mode={mode}", flush=True)
    got, ref, ob, orf = run_both(p, 40, seed=3)
    assert rel_l2(got, ref) <= 1e-12
    for f in ("norm", "mu", "energy"):
        assert abs(getattr(ob, f) - getattr(orf, f)) <= 1e-11 * max(1.0, abs(getattr(orf, f))), f
    assert abs(ob.ekin - orf.K) <= 1e-11 * max(1.0, abs(orf.K))
    assert abs(ob.epot - orf.P) <= 1e-11 * max(1.0, abs(orf.P))
    assert abs(ob.eint - orf.I) <= 1e-11 * max(1.0, abs(orf.I))
    for a in range(3):
        assert abs(ob.mean[a] - orf.mean[a]) <= 1e-11
        assert abs(ob.msq[a] - orf.msq[a]) <= 1e-11 * max(1.0, orf.msq[a])


@pytest.mark.parametrize("dim,n", [(2, (64, 5000, 1)), (3, (16, 5000, 8)), (1, (200000, 1, 1))])
@pytest.mark.parametrize("mode", [IMAG, REAL])
def test_fp64_fallback_lines_match_oracle(dim, n, mode):
    """Lines too long for the register-resident kernels take the exact
    one-thread-per-line path."""
    dx = (0.05, 0.05, 0.1)[:dim]
    om = (1.0, 1.5, 2.0)[:dim]
    dt = 0.1 * 0.05 ** 2 if mode == IMAG else 0.02 * 0.05 ** 2
    p = Problem(dim, n, dx, om, 5.0, dt, mode, F64, 1 if mode == IMAG else 0)
    kinds = [a["kind"] for a in sscn.plan_info(p) if a]
    assert "stream" in kinds
    got, ref, ob, orf = run_both(p, 6, seed=4)
    assert rel_l2(got, ref) <= 1e-12


def test_renorm_every_k_and_continuation():
    """renorm_every = 3 and a run split over several calls equal one call."""
    p = Problem(3, (20, 18, 16), (0.3, 0.3, 0.3), (1.0, 1.5, 2.0), 10.0, 0.01, IMAG, F64, 3)
    psi0 = initial(p, 5)
    s = sscn.Solver(p, psi0)
    for k in (1, 4, 2, 3):
        s.step(k)
    got = s.state()
    ref = oracle.run(oprob(p), psi0, 10).psi
    assert rel_l2(got, ref) <= 1e-12


@pytest.mark.parametrize("chunks", [(1, 4, 2), (2, 8, 16), (4, 32, 4), (8, 16, 8)])
def test_tile_hints_give_the_same_result(chunks):
    p = Problem(3, (64, 64, 32), (0.2, 0.2, 0.3), (1.0, 1.5, 2.0), 22.0, 0.004, IMAG, F64, 1)
    psi0 = initial(p, 6)
    ref = oracle.run(oprob(p), psi0, 20).psi
    try:
        sscn.set_tile_hint(p, chunks)
        s = sscn.Solver(p, psi0)
        s.step(20)
        got = s.state()
    finally:
        sscn.clear_tile_hints()
    assert rel_l2(got, ref) <= 1e-12


@pytest.mark.parametrize("nx,chunk,lanes", [(37, 4, 16), (64, 4, 16), (2, 4, 16), (65, 2, 64)])
@pytest.mark.parametrize("mode,prec", [(IMAG, F64), (REAL, F64), (IMAG, F32), (REAL, F32)])
def test_x_lines_shorter_than_a_wave(nx, chunk, lanes, mode, prec):
    """x lines of at most 64 points over 16 lanes (four lines per wave),
    ragged lengths included, and the 64-lane form just above, against the
    oracle."""
    p = Problem(3, (nx, 12, 10), (0.05, 0.3, 0.3), (1.0, 1.5, 2.0), 9.0,
                0.1 * 0.05 ** 2 if mode == IMAG else 0.02 * 0.05 ** 2, mode, prec, 1 if mode == IMAG else 0)
    psi0 = initial(p, 13)
    try:
        if chunk != 4:
            sscn.set_tile_hint(p, (chunk, 0, 0))
        q = sscn.plan_info(p)[0]
        assert (q["kind"], q["chunk"], q["lanes"]) == ("row", chunk, lanes)
        s = sscn.Solver(p, psi0)
        s.step(25)
        got = s.state()
        s.close()
    finally:
        sscn.clear_tile_hints()
    ref = oracle.run(oprob(p), psi0, 25).psi
    err = rel_l2(got, ref)
    print(f"case nx={nx} chunk={chunk} mode={mode} prec={prec}: rel-L2 {err:.2e}", flush=True)
    assert err <= (1e-12 if prec == F64 else 1e-5)


@pytest.mark.parametrize("n,mode,prec,lanes", [(3000, IMAG, F64, 8), (4096, IMAG, F64, 8), (3000, REAL, F32, 8),
                                                (6000, IMAG, F32, 8), (2000, REAL, F64, 8)])
def test_long_column_lines_take_more_lanes(n, mode, prec, lanes):
    """y lines longer than 16 waves x the 128-byte-segment lane count cover
    (2048 points) take the longest chunk and up to 8 lanes instead of the
    one-thread-per-line form; against the oracle."""
    p = Problem(2, (16, n, 1), (0.2, 0.01), (1.0, 1.5), 6.0,
                0.1 * 0.01 ** 2 if mode == IMAG else 0.02 * 0.01 ** 2, mode, prec, 1 if mode == IMAG else 0)
    q = sscn.plan_info(p)[1]
    assert q["kind"] == "col" and q["lanes"] == lanes
    assert q["chunk"] * q["waves"] * q["lanes"] >= n
    psi0 = initial(p, 17)
    s = sscn.Solver(p, psi0)
    s.step(25)
    got = s.state()
    s.close()
    ref = oracle.run(oprob(p), psi0, 25).psi
    err = rel_l2(got, ref)
    print(f"case n={n} mode={mode} prec={prec}: rel-L2 {err:.2e}", flush=True)
    assert err <= (1e-12 if prec == F64 else 1e-5)


def test_ground64_1000_steps():
    """64^3 imaginary time, g = 22, FP64: rel-L2 <= 1e-10 after 500 and 1000
    steps, mu and E to 1e-10."""
    dx = 0.2
    p = Problem(3, (64, 64, 64), (dx,) * 3, (1.0, 1.5, 2.0), 22.0, 0.1 * dx * dx, IMAG, F64, 1)
    psi0 = inputs.ho_gaussian(3, p.n, p.dx, p.omega, noise=1e-3, seed=0)
    s = sscn.Solver(p, psi0)
    op = oprob(p)
    r500 = oracle.run(op, psi0, 500)
    s.step(500)
    assert rel_l2(s.state(), r500.psi) <= 1e-10
    ob = s.observe()
    orf = oracle.observe(op, r500.psi)
    assert abs(ob.mu - orf.mu) <= 1e-10 * abs(orf.mu)
    assert abs(ob.energy - orf.energy) <= 1e-10 * abs(orf.energy)
    r1000 = oracle.run(op, r500.psi, 500, first_step=501)
    s.step(500)
    assert rel_l2(s.state(), r1000.psi) <= 1e-10
    ob = s.observe()
    orf = oracle.observe(op, r1000.psi)
    assert abs(ob.mu - orf.mu) <= 1e-10 * abs(orf.mu)
    assert abs(ob.energy - orf.energy) <= 1e-10 * abs(orf.energy)


def cube256_problem(prec=F64):
    dx = 0.1
    return Problem(3, (256, 256, 256), (dx,) * 3, (1.0, 1.5, 2.0), 80.0, 0.02 * dx * dx, REAL, prec, 0)


def test_cube256_short_run_matches_oracle():
    """256^3 complex128 real time in the benchmark's launch configuration:
    10 steps against the oracle."""
    p = cube256_problem()
    psi0 = inputs.thomas_fermi(3, p.n, p.dx, p.omega, 100.0, phase_sigma=0.05, seed=1)
    s = sscn.Solver(p, psi0)
    s.step(10)
    got = s.state()
    ref = oracle.run(oprob(p), psi0, 10).psi
    assert rel_l2(got, ref) <= 1e-12


def test_cube256_norm_and_energy_over_1000_steps():
    """Properties that hold at any size: the real-time step conserves the
    discrete norm exactly (FP64 round-off), and the energy drift of the
    quenched state stays small."""
    p = cube256_problem()
    psi0 = inputs.thomas_fermi(3, p.n, p.dx, p.omega, 100.0, phase_sigma=0.05, seed=1)
    s = sscn.Solver(p, psi0)
    o0 = s.observe()
    s.step(1000)
    o1 = s.observe()
    assert abs(o1.norm / o0.norm - 1) <= 1e-12
    assert abs(o1.energy - o0.energy) <= 1e-3 * abs(o0.energy)


def test_run_stops_where_the_oracle_stops():
    p = Problem(2, (40, 36, 1), (0.25, 0.25), (1.0, 2.0), 5.0, 0.01, IMAG, F64, 1, observe_every=10)
    psi0 = initial(p, 9)
    s = sscn.Solver(p, psi0)
    rc, trace = s.run(100000, 1e-7)
    r = oracle.run(oprob(p), psi0, 100000, observe_every=10, mu_tol=1e-7)
    assert rc == sscn.OK and r.converged
    assert trace[-1].step == r.steps
    assert abs(trace[-1].mu - r.trace[-1, 2]) <= 1e-11


def test_quench_set_g():
    p = Problem(2, (48, 40, 1), (0.2, 0.2), (1.0, 1.3), 30.0, 0.001, REAL, F64, 0)
    psi0 = initial(p, 2)
    s = sscn.Solver(p, psi0)
    s.step(10)
    s.set_g(20.0)
    s.step(10)
    got = s.state()
    op = oprob(p)
    r1 = oracle.run(op, psi0, 10).psi
    op.g = 20.0
    r2 = oracle.run(op, r1, 10, first_step=11).psi
    assert rel_l2(got, r2) <= 1e-12


@pytest.mark.parametrize("dim,n,dx", [(1, (5000,), (0.01,)), (2, (300, 7), (0.05, 0.3)),
                                      (3, (70, 9, 5), (0.2, 0.3, 0.4))])
def test_density_along_x_matches_oracle(dim, n, dx):
    """n_1D keeping x (partial sums over row blocks) in 1D, 2D and 3D,
    line lengths above and below one block's threads."""
    om = (1.0, 1.5, 2.0)[:dim]
    p = Problem(dim, n, dx, om, 5.0, 0.1 * min(dx) ** 2, IMAG, F64, 1)
    s = sscn.Solver(p, initial(p, 2))
    s.step(3)
    psi = s.state()
    assert np.allclose(s.density_1d(0), oracle.density_1d(oprob(p), psi, 0), rtol=1e-12, atol=1e-14)
    s.close()


@pytest.mark.parametrize("mode", [IMAG, REAL])
def test_densities_of_fp32_states_match_oracle(mode):
    """The density kernels over float and complex64 states (FP64 sums): the
    oracle sums the same stored values in FP64."""
    p = Problem(3, (70, 36, 30), (0.25, 0.25, 0.3), (1.0, 1.5, 2.0), 10.0,
                0.01 if mode == IMAG else 0.002, mode, F32, 1 if mode == IMAG else 0)
    s = sscn.Solver(p, initial(p, 3))
    s.step(4)
    psi = s.state().astype(np.complex128 if mode == REAL else np.float64)
    op = oprob(p)
    for a in range(3):
        assert np.allclose(s.density_1d(a), oracle.density_1d(op, psi, a), rtol=1e-12, atol=1e-14)
        assert np.allclose(s.density_2d(a), oracle.density_2d(op, psi, a), rtol=1e-12, atol=1e-14)
    s.close()


def test_densities_with_more_x_lines_than_the_scratch_holds():
    """More than 256K x lines: n_1D keeping y or z takes the per-output
    kernel instead of the x-line sums (no scratch for them)."""
    p = Problem(3, (2, 600, 600), (0.3, 0.05, 0.05), (1.0, 1.5, 2.0), 5.0, 2.5e-4, IMAG, F64, 1)
    s = sscn.Solver(p, initial(p, 6))
    s.step(2)
    psi = s.state()
    op = oprob(p)
    for a in range(3):
        assert np.allclose(s.density_1d(a), oracle.density_1d(op, psi, a), rtol=1e-12, atol=1e-14)
        assert np.allclose(s.density_2d(a), oracle.density_2d(op, psi, a), rtol=1e-12, atol=1e-14)
    s.close()


def test_densities_are_ordered_on_the_solver_stream():
    """The density outputs are made on the solver's own stream: with torch's
    current stream still busy, the results are the kernel's (an output
    cleared on the current stream would land after it)."""
    import torch
    p = Problem(3, (40, 36, 30), (0.25, 0.25, 0.3), (1.0, 1.5, 2.0), 10.0, 0.01, IMAG, F64, 1)
    s = sscn.Solver(p, initial(p, 1))
    s.step(3)
    psi = s.state()
    op = oprob(p)
    big = torch.randn(4096, 4096, device="cuda")
    for a in range(3):
        busy = big @ big  # queued on the current stream, not waited for
        assert np.allclose(s.density_1d(a), oracle.density_1d(op, psi, a), rtol=1e-12, atol=1e-14)
        busy = big @ big
        assert np.allclose(s.density_2d(a), oracle.density_2d(op, psi, a), rtol=1e-12, atol=1e-14)
    torch.cuda.synchronize()
    del busy
    s.close()


def test_integrated_densities_match_oracle():
    p = Problem(3, (40, 36, 30), (0.25, 0.25, 0.3), (1.0, 1.5, 2.0), 10.0, 0.01, IMAG, F64, 1)
    psi0 = initial(p, 1)
    s = sscn.Solver(p, psi0)
    s.step(5)
    psi = s.state()
    op = oprob(p)
    for a in range(3):
        assert np.allclose(s.density_1d(a), oracle.density_1d(op, psi, a), rtol=1e-12, atol=1e-14)
        assert np.allclose(s.density_2d(a), oracle.density_2d(op, psi, a), rtol=1e-12, atol=1e-14)


def test_nonfinite_state_reported():
    p = Problem(1, (64, 1, 1), (0.2,), (1.0,), 1.0, 0.004, IMAG, F64, 1)
    psi0 = initial(p, 0)
    psi0[0, 0, 10] = np.nan
    s = sscn.Solver(p, psi0)
    ob = s.observe()
    assert ob.status == sscn.E_NONFINITE


@pytest.mark.parametrize("mode", [IMAG, REAL])
@pytest.mark.parametrize("tol", [0.0, 1e-300])
def test_run_without_convergence_test_equals_observing_by_hand(mode, tol):
    """mu_tol = 0 queues the observations without waits, a tolerance never
    met observes and tests after every interval; either way (with the
    renormalisation left pending between observations and applied in the
    observation's loads) the rows and the final state are those of stepping
    to each observation step and observing, bit for bit (observe_every = 7
    and a cap between observations)."""
    p = Problem(3, (40, 36, 30), (0.25, 0.25, 0.3), (1.0, 1.5, 2.0), 10.0,
                0.01 if mode == IMAG else 0.002, mode, F64, 1 if mode == IMAG else 0, 7)
    psi0 = initial(p, 5)
    a = sscn.Solver(p, psi0)
    rc, rows = a.run(103, tol)
    assert rc == sscn.NOT_CONVERGED
    b = sscn.Solver(p, psi0)
    want, done = [], 0
    while done < 103:
        k = min(7 - done % 7, 103 - done)
        b.step(k)
        done += k
        want.append(b.observe())
    assert [r.step for r in rows] == [w.step for w in want] == list(range(7, 103, 7)) + [103]
    for r, w in zip(rows, want):
        assert (r.norm, r.mu, r.energy, r.ekin, r.epot, r.eint, r.mean, r.msq, r.status) == \
               (w.norm, w.mu, w.energy, w.ekin, w.epot, w.eint, w.mean, w.msq, w.status)
    assert np.array_equal(a.state(), b.state())
    a.close()
    b.close()


def test_run_without_convergence_test_ends_its_trace_at_a_blow_up():
    p = Problem(1, (64, 1, 1), (0.2,), (1.0,), 1.0, 0.004, IMAG, F64, 1, 5)
    psi0 = initial(p, 0)
    psi0[0, 0, 10] = np.nan
    s = sscn.Solver(p, psi0)
    rc, rows = s.run(50, 0.0)
    assert rc == sscn.E_NONFINITE
    assert len(rows) == 1 and rows[0].step == 5 and rows[0].status == sscn.E_NONFINITE
    s.close()


@pytest.mark.parametrize("mode", [IMAG, REAL])
@pytest.mark.parametrize("sigma", [0.3, 10.0, 300.0])
def test_large_sigma_full_depth_scans(mode, sigma):
    """Large CN coefficients make |alpha| close to 1: the scans must then
    reach across many chunks (up to the full line)."""
    dx = (0.2, 0.25, 0.3)
    dt = sigma * 4 * 0.2 * 0.2
    # g = 0: with steps this long the nonlinear phase would amplify any
    # rounding difference step after step; the linear problem isolates the
    # line solves
    p = Problem(3, (130, 40, 24), dx, (1.0, 1.5, 2.0), 0.0, dt, mode, F64, 1 if mode == IMAG else 0)
    got, ref, ob, orf = run_both(p, 5, seed=8)
    # the CN matrix has condition number ~1 + 4 sigma, which scales the
    # rounding differences between the scan and the oracle's Thomas order
    assert rel_l2(got, ref) <= max(1e-12, 1e-13 * (1 + 4 * sigma))


def _golden_cube256():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube256_oracle_1000.json")
    with open(path) as f:
        return json.load(f)


def _golden_lines():
    """The stored oracle's line sums (every grid point enters three of them)
    and the function that defines them."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_cube256_reference",
                                                  os.path.join(here, "make_cube256_reference.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    ref = np.load(os.path.join(here, "cube256_oracle_1000_lines.npz"))
    return {k: ref[k] for k in ref.files}, mod.line_sums


def _line_errors(flat, shape):
    ref, line_sums = _golden_lines()
    got = line_sums(flat.astype(np.complex128).reshape(shape))
    out = {}
    for k, r in ref.items():
        d = got[k] - r
        out[k] = (float(np.linalg.norm(d) / np.linalg.norm(r)), float(np.max(np.abs(d)) / np.max(np.abs(r))))
    return out


def _cube256_run(prec, steps=1000):
    """The benchmark's 256^3 workload in its launch configuration: the
    stored tile choices for the shape apply, as in bench.py."""
    p = cube256_problem(prec)
    psi0 = inputs.thomas_fermi(3, p.n, p.dx, p.omega, 100.0, phase_sigma=0.05, seed=1)
    try:
        autotune.apply(p, "single", cache_path=TILES)
        s = sscn.Solver(p, psi0)
    finally:
        sscn.clear_tile_hints()
    s.step(steps)
    ob = s.observe()
    flat = s.state().reshape(-1)
    s.close()
    return ob, flat


def test_cube256_1000_steps_matches_stored_oracle():
    """256^3 complex128, 1000 steps, bench launch configuration, against the
    stored oracle run (tests/golden/make_cube256_reference.py): relative L2 over
    4096 seeded sample points <= 1e-10 and each sample within 1e-10 of the
    largest; every grid point through the x-, y- and z-line sums (relative
    L2 and largest deviation <= 1e-10 of each vector); observables <= 1e-10
    relative."""
    ref = _golden_cube256()
    ob, flat = _cube256_run(F64)
    idx = np.asarray(ref["sample_index"])
    exp = np.asarray(ref["sample_re"]) + 1j * np.asarray(ref["sample_im"])
    got = flat[idx].astype(np.complex128)
    err = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    emax = np.max(np.abs(got - exp)) / np.max(np.abs(exp))
    lines = _line_errors(flat, (256, 256, 256))
    print(f"256^3 FP64 sampled rel-L2 {err:.3e} max {emax:.3e}; line sums (rel-L2, max) "
          + " ".join(f"{k} {v[0]:.2e} {v[1]:.2e}" for k, v in lines.items()), flush=True)
    assert err <= 1e-10 and emax <= 1e-10
    for k, (l2, mx) in lines.items():
        assert l2 <= 1e-10 and mx <= 1e-10, k
    assert abs(np.sum(np.abs(flat) ** 2) / ref["l2sq"] - 1) <= 1e-12
    for f, g in (("norm", "norm"), ("mu", "mu"), ("energy", "energy"), ("ekin", "K"), ("epot", "P"),
                 ("eint", "I")):
        assert abs(getattr(ob, f) - ref["obs1"][g]) <= 1e-10 * abs(ref["obs1"][g]), f


def test_cube256_fp32_error_against_stored_oracle():
    """complex64 storage, FP32 sweeps, FP64 tables and reductions, 1000 steps:
    the stated errors against the FP64 oracle; gate |d mu| <= 1e-5."""
    ref = _golden_cube256()
    ob, flat = _cube256_run(F32)
    idx = np.asarray(ref["sample_index"])
    exp = np.asarray(ref["sample_re"]) + 1j * np.asarray(ref["sample_im"])
    got = flat[idx].astype(np.complex128)
    err = np.linalg.norm(got - exp) / np.linalg.norm(exp)
    emax = np.max(np.abs(got - exp)) / np.max(np.abs(exp))
    lines = _line_errors(flat, (256, 256, 256))
    o1 = ref["obs1"]
    dmu = abs(ob.mu - o1["mu"])
    dE = abs(ob.energy - o1["energy"]) / abs(o1["energy"])
    dN = abs(ob.norm - o1["norm"])
    print(f"256^3 FP32: psi sampled rel-L2 {err:.3e} max {emax:.3e}  |d mu| {dmu:.3e}  rel dE {dE:.3e}  "
          f"|d norm| {dN:.3e}; line sums (rel-L2, max) "
          + " ".join(f"{k} {v[0]:.2e} {v[1]:.2e}" for k, v in lines.items()), flush=True)
    assert dmu <= 1e-5
    assert err <= 1e-3 and emax <= 1e-4
    for k, (l2, mx) in lines.items():
        assert l2 <= 1e-3 and mx <= 1e-3, k
    assert dE <= 1e-5
    assert dN <= 1e-5


@pytest.mark.parametrize("mode,prec", [(IMAG, F64), (REAL, F64), (IMAG, F32), (REAL, F32)])
def test_checkpoint_and_resume_is_bitwise(mode, prec):
    """1000 steps in one solver equal, bit for bit, 500 steps, the state
    saved to host memory, a fresh solver created from it, and 500 more
    (imaginary time renormalises every step, so the phase of the
    renormalisation does not depend on where the run was cut)."""
    p = Problem(3, (40, 36, 30), (0.25, 0.25, 0.3), (1.0, 1.5, 2.0), 18.0,
                0.006 if mode == IMAG else 0.0012, mode, prec, 1 if mode == IMAG else 0)
    psi0 = initial(p, seed=9)
    s = sscn.Solver(p, psi0)
    s.step(1000)
    whole = s.state()
    s.close()
    a = sscn.Solver(p, psi0)
    a.step(500)
    saved = a.state().copy()
    a.close()
    b = sscn.Solver(p, saved)
    b.step(500)
    resumed = b.state()
    b.close()
    assert np.array_equal(whole, resumed)


def test_graph_replay_equals_direct_launches():
    """Runs of steps replayed from captured graphs give bitwise the state
    of direct launches: imaginary time with renormalisation every 3 steps
    (runs start at every phase) and every step (the x sweep forms the factor
    from the previous step's partials inside a run, the final-sum kernel
    ends each run: one-step runs never fold), real time with a quench between
    runs, and a solver on the legacy default stream (always direct)."""
    import torch
    p1 = Problem(3, (20, 24, 18), (0.2, 0.2, 0.2), (1.0, 1.5, 2.0), 8.0, 0.004, IMAG, F64, 1)
    assert sscn.plan_info(p1)[0]["lanes"] == 16
    for mode, every in ((IMAG, 3), (IMAG, 1), (REAL, 0)):
        p = Problem(3, (20, 24, 18), (0.2, 0.2, 0.2), (1.0, 1.5, 2.0), 8.0, 0.004 if mode == IMAG else 0.0008,
                    mode, F64, every)
        if mode == IMAG:
            psi0 = inputs.ho_gaussian(3, p.n, p.dx, p.omega, noise=1e-3, seed=5)
        else:
            psi0 = inputs.thomas_fermi(3, p.n, p.dx, p.omega, 10.0, phase_sigma=0.05, seed=5)
        # 70 = 32 + 32 + 4 + 2; quench; 101 = 3 x 32 + 4 + 1; 20 = 16 + 4
        # after sscn_prepare; 1 step
        plan = [(70, None), (101, 6.0), (20, None), (1, None)]
        outs = []
        for how in ("graph", "step1", "direct", "default"):
            s = sscn.Solver(p, psi0, stream=torch.cuda.default_stream() if how == "default" else None)
            for n, g in plan:
                if g is not None:
                    s.set_g(g)
                if how == "step1":                  # one-step graphs
                    for _ in range(n):
                        s.step(1)
                elif how == "direct":               # the timed path launches every kernel directly
                    s.step_timed(n)
                else:
                    if n == 20:
                        s.prepare(n)
                    s.step(n)
            outs.append(s.state())
            s.close()
        for k in range(1, len(outs)):
            assert np.array_equal(outs[0], outs[k]), (mode, k)
