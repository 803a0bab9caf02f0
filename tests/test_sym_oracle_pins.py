"""Pins of the symmetric-trap oracle (circular, spherical and axial traps)
against facts that do not come from the oracle: a dense linear-algebra
solve, the symmetry of the discrete operator in its inner product, exact
norm conservation, closed forms of the harmonic trap (ground-state chemical
potentials with their second-order grid error, Gaussian integrals,
Thomas-Fermi limits), the exact 2D breathing frequency, the Kohn dipole
mode, exact separability of the axial trap at g = 0 into the circular and
the anisotropic Cartesian oracles, and agreement with the Cartesian 2D
oracle on an isotropic trap."""
import math

import numpy as np
import pytest

import oracle
from oracle import AXI, CIR, IMAG, REAL, SPH, SymProblem
from paper_1605_03958_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore::numpy.exceptions.ComplexWarning")


def _dense(prob, tau):
    l, d, u, _ = oracle.sym_coefs(prob)
    n = prob.n[0]
    H = np.diag(d).astype(np.complex128)
    for i in range(n - 1):
        H[i, i + 1] = -u[i]
        H[i + 1, i] = -l[i + 1]
    return np.eye(n) + tau * H, np.eye(n) - tau * H


@pytest.mark.parametrize("geom", [CIR, SPH])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 40])
@pytest.mark.parametrize("mode", [IMAG, REAL])
def test_radial_substep_matches_dense_solve(geom, n, mode):
    """The r substep (1 + tau H) v = (1 - tau H) u by Thomas equals a dense
    solve with the same coefficients (pins the elimination and the
    right-hand side, with the l_0 and outer-ghost ends)."""
    dt = 0.05
    prob = SymProblem(geom, (n, 1), (0.2, 1.0), (1.3, 0.0), 0.0, dt, mode, 1)
    rng = np.random.default_rng(n + 10 * geom)
    u = rng.normal(size=n) + 1j * rng.normal(size=n)
    tau = 0.5 * dt * (1j if mode == REAL else 1.0)
    A, B = _dense(prob, tau)
    ref = np.linalg.solve(A, B @ u)
    got = oracle.sym_substep(prob, u, 0).reshape(-1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("geom", [CIR, SPH])
def test_radial_operator_is_symmetric_in_its_inner_product(geom):
    """W H is symmetric (W_i u_i = W_{i+1} l_{i+1}), W > 0 and H has zero row
    sums apart from the outer edge: the flux form with the origin closed."""
    prob = SymProblem(geom, (50, 1), (0.1, 1.0), (1.0, 0.0), 0.0, 0.01)
    l, d, u, w = oracle.sym_coefs(prob)
    assert l[0] == 0.0
    assert np.all(w > 0)
    np.testing.assert_allclose(w[:-1] * u[:-1], w[1:] * l[1:], rtol=1e-14)
    np.testing.assert_allclose(d[:-1], l[:-1] + u[:-1], rtol=1e-15)


@pytest.mark.parametrize("geom", [CIR, SPH])
def test_kinetic_energy_is_the_operator_expectation(geom):
    """K (evaluated in its gradient form) equals Re <psi, H_r psi> with H_r
    the dense operator of the oracle's coefficients and the weighted inner
    product c dr sum W conj(a) b (summation by parts)."""
    n = 80
    h = 0.1
    prob = SymProblem(geom, (n, 1), (h, 1.0), (1.0, 0.0), 0.0, 0.01)
    l, d, u, w = oracle.sym_coefs(prob)
    H = np.diag(d) - np.diag(u[:-1], 1) - np.diag(l[1:], -1)
    rng = np.random.default_rng(geom)
    psi = (rng.normal(size=n) + 1j * rng.normal(size=n)) * np.exp(-0.02 * np.arange(n))
    c = 4 * math.pi if geom == SPH else 2 * math.pi
    want = c * h * np.real(np.sum(w * np.conj(psi) * (H @ psi)))
    assert abs(oracle.sym_observe(prob, psi).K - want) <= 1e-12 * abs(want)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_axial_kinetic_energy_of_a_z_sine_mode(k):
    """psi = a(rho) sin(pi k (j+1)/(n_z+1)): the z factor is an exact
    eigenvector of the Dirichlet 3-point Laplacian with eigenvalue
    tau_k = 2 - 2 cos(pi k/(n_z+1)), so the axial trap's kinetic energy per
    norm is the circular trap's for a(rho) plus tau_k/(2 dz^2) exactly."""
    nr, nz, h, hz = 30, 25, 0.15, 0.2
    rng = np.random.default_rng(k)
    a = np.exp(-0.5 * inputs.radial_coords(nr, h) ** 2) * (1 + 0.2 * rng.uniform(size=nr))
    j = np.arange(nz)
    b = np.sin(math.pi * k * (j + 1) / (nz + 1))
    ax = oracle.sym_observe(SymProblem(AXI, (nr, nz), (h, hz), (1.0, 1.0), 0.0, 0.01), b[:, None] * a[None, :])
    ci = oracle.sym_observe(SymProblem(CIR, (nr, 1), (h, 1.0), (1.0, 0.0), 0.0, 0.01), a)
    tau = 2 - 2 * math.cos(math.pi * k / (nz + 1))
    assert abs(ax.K / ax.norm - (ci.K / ci.norm + tau / (2 * hz * hz))) <= 1e-12 * (ax.K / ax.norm)


@pytest.mark.parametrize("geom", [CIR, SPH, AXI])
def test_real_time_conserves_the_weighted_norm(geom):
    n = (60, 1) if geom != AXI else (30, 40)
    dx = (0.15, 0.2)
    om = (1.0, 1.7)
    prob = SymProblem(geom, n, dx, om, 25.0, 0.004, REAL, 0)
    psi0 = inputs.sym_thomas_fermi(geom, n, dx, om, 30.0, phase_sigma=0.05, seed=3)
    n0 = oracle.sym_observe(prob, psi0).norm
    r = oracle.sym_run(prob, psi0, 1000)
    n1 = oracle.sym_observe(prob, r.psi).norm
    assert abs(n1 / n0 - 1) <= 1e-12


def _ground(geom, n, dx, om, g, dt, steps, psi0=None):
    prob = SymProblem(geom, n, dx, om, g, dt, IMAG, 1)
    if psi0 is None:
        psi0 = inputs.sym_gaussian(geom, n, dx, om, noise=0.0)
    r = oracle.sym_run(prob, psi0, steps, observe_every=max(1, steps // 4))
    return prob, r


@pytest.mark.parametrize("geom,om,exact", [(CIR, (1.3, 0.0), 1.3), (SPH, (1.1, 0.0), 1.65),
                                           (AXI, (1.0, 1.6), 1.0 + 0.8)])
def test_ground_state_mu_at_g0_is_second_order(geom, om, exact):
    """g = 0: mu converges to the oscillator's (w (2D), 3w/2 (3D), w_rho +
    w_z/2 (axial)) with an error that falls 4x when the grid spacing halves
    (dt scaled with it, so the splitting error falls alike)."""
    errs = []
    for h in (0.2, 0.1):
        R = 7.0 / math.sqrt(min(w for w in om if w > 0))
        n = (int(round(R / h)), int(round(2 * R / h)) if geom == AXI else 1)
        dx = (h, h)
        dt = 0.1 * h * h
        steps = int(round(6.0 / dt))
        _, r = _ground(geom, n, dx, om, 0.0, dt, steps)
        errs.append(r.trace[-1, 2] - exact)
    assert abs(errs[0]) < 2e-2 * exact
    assert 3.5 < errs[0] / errs[1] < 4.5, errs


@pytest.mark.parametrize("geom", [CIR, SPH])
def test_gaussian_integrals(geom):
    """For the oscillator Gaussian: N = 1, P = d w/4, K = d w/4 (the virial
    of the oscillator ground state), I = (w/2pi)^(d/2), <r^2> = d/(2w),
    <r> = sqrt(pi/(4w)) (2D) or 2/sqrt(pi w) (3D), each to O(dr^2) (errors
    falling ~4x when dr halves)."""
    w = 1.4
    d = 2 if geom == CIR else 3
    want = {"norm": 1.0, "P": d * w / 4, "K": d * w / 4, "I": (w / (2 * math.pi)) ** (d / 2),
            "r2": d / (2 * w), "r": math.sqrt(math.pi / (4 * w)) if d == 2 else 2 / math.sqrt(math.pi * w)}
    errs = {k: [] for k in want}
    for h in (0.1, 0.05):
        n = (int(round(9.0 / h)), 1)
        prob = SymProblem(geom, n, (h, 1.0), (w, 0.0), 0.0, 0.01)
        o = oracle.sym_observe(prob, inputs.sym_gaussian(geom, n, (h, 1.0), (w, 0.0), noise=0.0))
        got = {"norm": o.norm, "P": o.P, "K": o.K, "I": o.I, "r2": o.msq[0], "r": o.mean[0]}
        for k in want:
            errs[k].append(got[k] - want[k])
    for k in want:
        e0, e1 = errs[k]
        assert abs(e0) < 5e-3 * max(1.0, want[k]), (k, errs[k])
        assert abs(e1) < abs(e0) / 3.3, (k, errs[k])


def test_axial_gaussian_integrals():
    """Axial oscillator Gaussian displaced by z0 along z: N = 1,
    P = w_rho/2 + w_z/4 + w_z^2 z0^2/2, I = (w_rho/2pi) sqrt(w_z/2pi),
    <rho^2> = 1/w_rho, <z> = z0, <z^2> = 1/(2 w_z) + z0^2; the z parts are
    spectrally accurate, the radial ones O(d rho^2)."""
    om = (1.3, 2.1)
    z0 = 0.3
    h = 0.05
    n = (int(round(8.0 / h)), int(round(14.0 / h)))
    prob = SymProblem(AXI, n, (h, h), om, 0.0, 0.01)
    o = oracle.sym_observe(prob, inputs.sym_gaussian(AXI, n, (h, h), om, noise=0.0, z_shift=z0))
    assert abs(o.norm - 1) < 1e-3
    assert abs(o.P - (om[0] / 2 + om[1] / 4 + om[1] ** 2 * z0 ** 2 / 2)) < 2e-3
    assert abs(o.I - om[0] / (2 * math.pi) * math.sqrt(om[1] / (2 * math.pi))) < 2e-3
    assert abs(o.msq[0] - 1 / om[0]) < 2e-3
    assert abs(o.mean[1] - z0) < 1e-9
    assert abs(o.msq[1] - (1 / (2 * om[1]) + z0 ** 2)) < 1e-9


@pytest.mark.parametrize("geom,gs,tol_mu,tol_ratio", [(CIR, (20.0, 200.0, 2000.0), 3e-3, 3e-3),
                                                       (SPH, (20.0, 200.0, 2000.0), 2e-2, 1.5e-2)])
def test_thomas_fermi_limits(geom, gs, tol_mu, tol_ratio):
    """Large g: mu -> mu_TF (2D: w sqrt(g/pi); 3D: (15 g w^3/(4 pi))^(2/5)/2)
    and E/mu -> (d+2)/(d+4), errors decreasing in g."""
    w = 1.0
    d = 2 if geom == CIR else 3
    e_mu, e_ratio = [], []
    for g in gs:
        mu_tf = inputs.sym_mu_thomas_fermi(geom, g, (w, w))
        h = 0.1
        n = (int(round((math.sqrt(2 * mu_tf) / w + 3.0) / h)), 1)
        psi0 = inputs.sym_thomas_fermi(geom, n, (h, 1.0), (w, 0.0), g).real
        _, r = _ground(geom, n, (h, 1.0), (w, 0.0), g, 0.005, 800, psi0)
        mu, E = r.trace[-1, 2], r.trace[-1, 3]
        e_mu.append(abs(mu - mu_tf) / mu_tf)
        e_ratio.append(abs(E / mu - (d + 2) / (d + 4)))
    assert e_mu[0] > e_mu[1] > e_mu[2] and e_mu[2] < tol_mu, e_mu
    assert e_ratio[0] > e_ratio[1] > e_ratio[2] and e_ratio[2] < tol_ratio, e_ratio


def test_circular_trap_breathes_at_twice_the_trap_frequency():
    """2D isotropic trap with contact interaction: after a quench of g the
    mean square radius oscillates exactly at 2w for any g (the 2D scale
    symmetry of the GP equation).  A fit of A + B cos 2wt + C sin 2wt over
    one period leaves a residual below 1 % of the amplitude; the same fit at
    1.1 x 2w does not."""
    w = 1.0
    h = 0.05
    n = (int(round(8.0 / h)), 1)
    _, r = _ground(CIR, n, (h, 1.0), (w, 0.0), 20.0, 0.0025, 1600)
    dt = 0.001
    steps = int(round(math.pi / (w * dt)))
    prob = SymProblem(CIR, n, (h, 1.0), (w, 0.0), 8.0, dt, REAL, 0)
    tr = oracle.sym_run(prob, r.psi.astype(np.complex128), steps, observe_every=10).trace
    t = tr[:, 0] * dt
    y = tr[:, 10]

    def resid(freq):
        M = np.stack([np.ones_like(t), np.cos(freq * t), np.sin(freq * t)], axis=1)
        c, *_ = np.linalg.lstsq(M, y, rcond=None)
        return np.max(np.abs(M @ c - y)), math.hypot(c[1], c[2])

    res, amp = resid(2 * w)
    bad, _ = resid(2.2 * w)
    assert amp > 0.05
    assert res < 0.01 * amp, (res, amp)
    assert bad > 5 * res


def test_axial_trap_kohn_mode_along_z():
    """A ground state displaced along z by z0 oscillates as <z> = z0 cos(w_z t)
    at any g (the centre of mass decouples in a harmonic trap)."""
    om = (1.0, 1.5)
    dx = (0.15, 0.15)
    n = (40, 80)
    z0 = 0.4
    psi = inputs.sym_gaussian(AXI, n, dx, om, noise=0.0, z_shift=z0)
    prob = SymProblem(AXI, n, dx, om, 15.0, 0.0015, REAL, 0)
    steps = int(round(2 * math.pi / om[1] / 0.0015))
    # start from the interacting ground state shifted by z0: relax it first
    g_prob, gr = _ground(AXI, n, dx, om, 15.0, 0.005, 1200)
    shift = int(round(z0 / dx[1]))
    psi = np.roll(gr.psi.reshape(n[1], n[0]), shift, axis=0)
    tr = oracle.sym_run(prob, psi.astype(np.complex128), steps, observe_every=25).trace
    t = tr[:, 0] * 0.0015
    zc = tr[:, 8]
    z_start = oracle.sym_observe(prob, psi).mean[1]
    assert abs(z_start - shift * dx[1]) < 1e-3
    err = np.max(np.abs(zc - z_start * np.cos(om[1] * t)))
    assert err < 0.02 * abs(z_start), err


def test_axial_trap_separates_at_g0():
    """g = 0, real time: a product state rho-profile x z-profile evolves as
    the circular oracle's radial evolution times the anisotropic Cartesian
    oracle's 1D evolution along z (both pinned on their own), exactly up to
    rounding."""
    om = (1.2, 1.9)
    dx = (0.2, 0.17)
    n = (25, 31)
    dt = 0.003
    steps = 200
    rng = np.random.default_rng(4)
    a = np.exp(-0.6 * inputs.radial_coords(n[0], dx[0]) ** 2) * (1 + 0.1 * rng.uniform(size=n[0]))
    b = np.exp(-0.9 * inputs.coords(n[1], dx[1]) ** 2) * (1 + 0.1 * rng.uniform(size=n[1]))
    psi = (b[:, None] * a[None, :]).astype(np.complex128)
    got = oracle.sym_run(SymProblem(AXI, n, dx, om, 0.0, dt, REAL, 0), psi, steps).psi
    ra = oracle.sym_run(SymProblem(CIR, (n[0], 1), (dx[0], 1.0), (om[0], 0.0), 0.0, dt, REAL, 0),
                        a.astype(np.complex128), steps).psi.reshape(-1)
    rb = oracle.run(oracle.Problem(1, (n[1], 1, 1), (dx[1], 1.0, 1.0), (om[1], 0.0, 0.0), 0.0, dt, REAL, 0),
                    b.astype(np.complex128), steps).psi.reshape(-1)
    ref = rb[:, None] * ra[None, :]
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_circular_trap_agrees_with_the_cartesian_2d_oracle():
    """An isotropic 2D trap solved on the radial grid and on the Cartesian
    grid: both chemical potentials converge to the same continuum value, so
    their difference falls with the grid spacing and is small."""
    w, g = 1.0, 20.0
    diffs = []
    for h in (0.2, 0.1):
        R = 7.0
        _, rc = _ground(CIR, (int(round(R / h)), 1), (h, 1.0), (w, 0.0), g, 0.1 * h * h, int(6.0 / (0.1 * h * h)))
        m = int(round(2 * R / h))
        cp = oracle.Problem(2, (m, m, 1), (h, h, 1.0), (w, w, 0.0), g, 0.1 * h * h, IMAG, 1)
        steps = int(6.0 / (0.1 * h * h))
        rr = oracle.run(cp, inputs.ho_gaussian(2, (m, m, 1), (h, h), (w, w), noise=0.0), steps,
                        observe_every=steps // 2)
        diffs.append(abs(rc.trace[-1, 2] - rr.trace[-1, 2]))
    assert diffs[0] < 2e-2 and diffs[1] < diffs[0] / 3, diffs
