"""GPU test of the imaginary -> real-time pipeline (ground state, quench,
rms sizes per step) against the same pipeline run by the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_1605_03958_amd import dynamics, inputs
from paper_1605_03958_amd.sscn import F64, IMAG, REAL, Problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,n,dx", [(1, (300,), (0.05,)), (2, (40, 34), (0.25, 0.25)),
                                      (3, (24, 20, 17), (0.35, 0.35, 0.4))])
def test_pipeline_matches_the_oracle(dim, n, dx):
    om = (1.0, 1.5, 2.0)[:dim]
    h = min(dx)
    p = Problem(dim, n, dx, om, 10.0, 0.1 * h * h, IMAG, F64, 1, 10)
    psi0 = inputs.ho_gaussian(dim, p.n, p.dx, p.omega, noise=1e-3, seed=4)
    dt_real, steps, factor = 0.02 * h * h, 300, 0.8
    d = dynamics.ground_state_then_dynamics(p, psi0, factor, steps, dt_real, mu_tol=1e-9)
    assert d.converged

    op = oracle.Problem(dim, p.n, p.dx, p.omega, p.g, p.dt, IMAG, 1)
    g = oracle.run(op, psi0, 10**6, observe_every=10, mu_tol=1e-9)
    assert g.converged and g.steps == d.ground_steps
    rp = oracle.Problem(dim, p.n, p.dx, p.omega, p.g * factor, dt_real, REAL, 0)
    psi_g = g.psi.astype(np.complex128)
    r = oracle.run(rp, psi_g, steps, observe_every=1)
    o0 = oracle.observe(rp, psi_g)
    msq = np.vstack([np.array(o0.msq[:dim])[None, :],
                     r.trace[:, [oracle.TRACE_COLS.index(c) for c in ("mx2", "my2", "mz2")[:dim]]]])
    t = np.arange(steps + 1) * dt_real
    want = np.column_stack([t, np.sqrt(msq), np.sqrt(msq.sum(axis=1))])

    assert d.table.shape == want.shape
    np.testing.assert_allclose(d.table, want, rtol=1e-9, atol=0)
    # the quench sets the cloud breathing: the rms size does change (by
    # 2e-5 relative over the 1D case's short time span, t = 0.015)
    assert np.ptp(d.table[:, -1]) > 1e-6 * d.table[0, -1]
