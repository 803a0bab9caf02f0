"""GPU tests of sscn_create_noalloc, the solver whose workspace is the
library's static device array: called through the C ABI, its results equal
those of a solver from sscn_create (same kernels), on two creations in a
row, the second with a smaller problem; the array is held by one solver per
device at a time; problems whose workspace does not fit are refused."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1605_03958_amd import inputs, sscn
from paper_1605_03958_amd.sscn import F32, F64, IMAG, REAL, Problem

pytestmark = pytest.mark.gpu


def _case(dim, n, mode, prec, every, seed):
    dx = (0.25, 0.3, 0.3)[:dim]
    om = (1.0, 1.5, 2.0)[:dim]
    p = Problem(dim, n, dx, om, 15.0, 0.006 if mode == IMAG else 0.0012, mode, prec, every)
    if mode == IMAG:
        psi0 = inputs.ho_gaussian(dim, p.n, p.dx, p.omega, noise=1e-3, seed=seed)
    else:
        psi0 = inputs.thomas_fermi(dim, p.n, p.dx, p.omega, 20.0, phase_sigma=0.05, seed=seed)
    return p, psi0


def _run(p, psi0, steps, noalloc):
    s = sscn.Solver(p, psi0, noalloc=noalloc)
    s.step(steps)
    ob = s.observe()
    rho = s.density_1d(0)
    st = s.state()
    s.close()
    return st, ob, rho


def test_noalloc_solver_equals_workspace_solver_on_two_calls():
    """Two solvers in a row on the static array (the second smaller, so the
    array still holds the first one's larger tables and partials): each
    equals a solver over a workspace tensor bit for bit -- state,
    observables and the x density, whose partial sums live in the array."""
    cases = [_case(3, (48, 40, 36), IMAG, F64, 3, 11), _case(2, (30, 20, 1), REAL, F32, 0, 12)]
    for p, psi0 in cases:
        print(f"noalloc vs workspace: dim={p.dim} n={p.n} mode={p.mode} prec={p.prec}", flush=True)
        a_state, a_obs, a_rho = _run(p, psi0, 37, True)
        b_state, b_obs, b_rho = _run(p, psi0, 37, False)
        assert np.array_equal(a_state, b_state)
        assert a_obs == b_obs
        assert np.array_equal(a_rho, b_rho)


def test_static_array_is_held_by_one_solver_at_a_time():
    p, psi0 = _case(1, (500, 1, 1), IMAG, F64, 1, 13)
    first = sscn.Solver(p, psi0, noalloc=True)
    try:
        with pytest.raises(sscn.SSCNError) as e:
            sscn.Solver(p, psi0, noalloc=True)
        assert e.value.code == sscn.E_NOSPACE
    finally:
        first.close()
    again = sscn.Solver(p, psi0, noalloc=True)      # released by the destroy
    again.step(3)
    again.close()


def test_problem_larger_than_the_static_array_is_refused():
    """A problem whose workspace exceeds SSCN_STATIC_WS_BYTES is refused
    before anything is touched (the state pointer is only checked)."""
    p = Problem(1, (1 << 20, 1, 1), (0.01,), (1.0,), 1.0, 1e-5, IMAG, F64, 1)
    assert sscn.workspace_bytes(p) > (4 << 20)
    dummy = torch.zeros(4, dtype=torch.float64, device="cuda")
    h = ctypes.c_void_p(0)
    pc = p.c()
    rc = sscn.lib().sscn_create_noalloc(ctypes.byref(pc), ctypes.c_void_p(dummy.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    assert rc == sscn.E_UNSUPPORTED and not h.value
