"""ctypes binding of the plain FP64 CPU oracle (``sscn_oracle.c`` for the
anisotropic Cartesian grids, ``sscn_sym_oracle.c`` for the circular,
spherical and axial traps).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package imports nothing from the product.

Every state crosses as a numpy array of shape ``(nz, ny, nx)`` (x fastest), of
dtype complex128; imaginary-time states are passed with zero imaginary part and
come back real-valued in complex storage.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

IMAG = 0
REAL = 1

TRACE_COLS = ("step", "norm", "mu", "energy", "K", "P", "I",
              "mx", "my", "mz", "mx2", "my2", "mz2")


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("dx", ctypes.c_double * 3),
        ("omega", ctypes.c_double * 3),
        ("g", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("mode", ctypes.c_int),
        ("renorm_every", ctypes.c_int),
    ]


@dataclass
class Problem:
    """Oracle-side problem description (unused axes: n = 1)."""
    dim: int
    n: tuple
    dx: tuple
    omega: tuple
    g: float
    dt: float
    mode: int = IMAG
    renorm_every: int = 1

    def c(self) -> _Problem:
        p = _Problem()
        p.dim = int(self.dim)
        n = list(self.n) + [1] * (3 - len(self.n))
        dx = list(self.dx) + [1.0] * (3 - len(self.dx))
        om = list(self.omega) + [0.0] * (3 - len(self.omega))
        for a in range(3):
            p.n[a] = int(n[a])
            p.dx[a] = float(dx[a])
            p.omega[a] = float(om[a])
        p.g = float(self.g)
        p.dt = float(self.dt)
        p.mode = int(self.mode)
        p.renorm_every = int(self.renorm_every)
        return p

    @property
    def shape(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        return (n[2], n[1], n[0])


CIR, SPH, AXI = 1, 2, 3
SYM_TRACE_COLS = ("step", "norm", "mu", "energy", "K", "P", "I", "mr", "mz", "unused", "mr2", "mz2",
                  "unused2")


class _SymProblem(ctypes.Structure):
    _fields_ = [
        ("geom", ctypes.c_int),
        ("n", ctypes.c_int * 2),
        ("dx", ctypes.c_double * 2),
        ("omega", ctypes.c_double * 2),
        ("g", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("mode", ctypes.c_int),
        ("renorm_every", ctypes.c_int),
    ]


@dataclass
class SymProblem:
    """Symmetric trap: geom CIR (2D circular, psi(r)), SPH (3D spherical,
    psi(r)) or AXI (3D axial, psi(rho, z)); n = (n_r, n_z), dx = (dr, dz),
    omega = (omega_r, omega_z); n_z = 1 unless axial."""
    geom: int
    n: tuple
    dx: tuple
    omega: tuple
    g: float
    dt: float
    mode: int = IMAG
    renorm_every: int = 1

    def c(self) -> _SymProblem:
        p = _SymProblem()
        p.geom = int(self.geom)
        n = list(self.n) + [1] * (2 - len(self.n))
        dx = list(self.dx) + [1.0] * (2 - len(self.dx))
        om = list(self.omega) + [0.0] * (2 - len(self.omega))
        for a in range(2):
            p.n[a] = int(n[a])
            p.dx[a] = float(dx[a])
            p.omega[a] = float(om[a])
        p.g = float(self.g)
        p.dt = float(self.dt)
        p.mode = int(self.mode)
        p.renorm_every = int(self.renorm_every)
        return p

    @property
    def shape(self):
        n = list(self.n) + [1] * (2 - len(self.n))
        return (n[1], n[0])


_lib = None
_lib_path = LIB_PATH


def use_library(path: str) -> str:
    """Load later calls from the oracle library at `path` (the benchmark's
    host-tuned copy of the same source); returns the previous path."""
    global _lib, _lib_path
    prev = _lib_path
    _lib_path = path
    _lib = None
    return prev


def load():
    """Load (never build) the oracle library; tests build it beforehand."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_lib_path):
        raise RuntimeError(f"oracle library missing: {_lib_path}; run oracle.build.build()")
    lib = ctypes.CDLL(_lib_path)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(_Problem)
    lib.orc_thomas.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.orc_cn_line.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
    lib.orc_observe.argtypes = [pp, dp, dp]
    lib.orc_potential.argtypes = [pp, dp]
    lib.orc_substep.argtypes = [pp, dp, ctypes.c_int]
    lib.orc_run.argtypes = [pp, dp, ctypes.c_long, ctypes.c_long, ctypes.c_int,
                            ctypes.c_double, dp, ctypes.c_long,
                            ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
    lib.orc_threads.argtypes = []
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_density_1d.argtypes = [pp, dp, ctypes.c_int, dp]
    lib.orc_density_2d.argtypes = [pp, dp, ctypes.c_int, dp]
    sp = ctypes.POINTER(_SymProblem)
    lib.ors_coefs.argtypes = [sp, dp, dp, dp, dp]
    lib.ors_observe.argtypes = [sp, dp, dp]
    lib.ors_substep.argtypes = [sp, dp, ctypes.c_int]
    lib.ors_run.argtypes = [sp, dp, ctypes.c_long, ctypes.c_long, ctypes.c_int,
                            ctypes.c_double, dp, ctypes.c_long,
                            ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
    for f in (lib.orc_thomas, lib.orc_cn_line, lib.orc_observe, lib.orc_potential,
              lib.orc_substep, lib.orc_run, lib.orc_threads, lib.orc_set_threads, lib.orc_density_1d,
              lib.orc_density_2d, lib.ors_coefs, lib.ors_observe, lib.ors_substep, lib.ors_run):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_state(prob: Problem, psi) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128).reshape(prob.shape))
    return a.copy()


def thomas(n: int, sigma: complex, rhs) -> np.ndarray:
    """Solve tridiag(-sigma, 1+2 sigma, -sigma) x = rhs (Thomas, FP64)."""
    r = np.ascontiguousarray(np.asarray(rhs, dtype=np.complex128))
    x = np.zeros(n, dtype=np.complex128)
    rc = load().orc_thomas(n, float(np.real(sigma)), float(np.imag(sigma)),
                           _ptr(r.view(np.float64)), _ptr(x.view(np.float64)))
    if rc:
        raise ValueError(f"orc_thomas rc={rc}")
    return x


def cn_line(n: int, sigma: complex, u) -> np.ndarray:
    """One CN kinetic substep (1+sT)v = (1-sT)u on a single line."""
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.complex128))
    v = np.zeros(n, dtype=np.complex128)
    rc = load().orc_cn_line(n, float(np.real(sigma)), float(np.imag(sigma)),
                            _ptr(uu.view(np.float64)), _ptr(v.view(np.float64)))
    if rc:
        raise ValueError(f"orc_cn_line rc={rc}")
    return v


def potential(prob: Problem) -> np.ndarray:
    v = np.zeros(prob.shape, dtype=np.float64)
    pc = prob.c()
    rc = load().orc_potential(ctypes.byref(pc), _ptr(v))
    if rc:
        raise ValueError(f"orc_potential rc={rc}")
    return v


def substep(prob: Problem, psi, which: int) -> np.ndarray:
    """which = -1: pointwise substep; 0/1/2: CN sweep along x/y/z."""
    a = _as_state(prob, psi)
    pc = prob.c()
    rc = load().orc_substep(ctypes.byref(pc), _ptr(a.view(np.float64)), int(which))
    if rc:
        raise ValueError(f"orc_substep rc={rc}")
    return a


@dataclass
class Observables:
    norm: float
    mu: float
    energy: float
    K: float
    P: float
    I: float
    mean: tuple = field(default=(0.0, 0.0, 0.0))
    msq: tuple = field(default=(0.0, 0.0, 0.0))


def observe(prob: Problem, psi) -> Observables:
    a = _as_state(prob, psi)
    out = np.zeros(12)
    pc = prob.c()
    rc = load().orc_observe(ctypes.byref(pc), _ptr(a.view(np.float64)), _ptr(out))
    if rc:
        raise ValueError(f"orc_observe rc={rc}")
    return Observables(*out[:6], tuple(out[6:9]), tuple(out[9:12]))


@dataclass
class RunResult:
    psi: np.ndarray
    trace: np.ndarray        # rows of TRACE_COLS
    steps: int
    converged: bool


def run(prob: Problem, psi, nsteps: int, observe_every: int = 0,
        mu_tol: float = 0.0, first_step: int = 1) -> RunResult:
    """Propagate nsteps SSCN steps (see sscn_oracle.c for the definition)."""
    a = _as_state(prob, psi)
    cap = (nsteps // observe_every + 2) if observe_every > 0 else 2
    trace = np.zeros((cap, len(TRACE_COLS)))
    rows = ctypes.c_long(0)
    done = ctypes.c_long(0)
    pc = prob.c()
    rc = load().orc_run(ctypes.byref(pc), _ptr(a.view(np.float64)), int(nsteps),
                        int(first_step), int(observe_every), float(mu_tol),
                        _ptr(trace), cap, ctypes.byref(rows), ctypes.byref(done))
    if rc < 0:
        raise ValueError(f"orc_run rc={rc}")
    return RunResult(a, trace[: rows.value].copy(), int(done.value), rc == 0)


def density_1d(prob: Problem, psi, keep: int) -> np.ndarray:
    a = _as_state(prob, psi)
    n = (list(prob.n) + [1, 1])[keep]
    out = np.zeros(n)
    pc = prob.c()
    rc = load().orc_density_1d(ctypes.byref(pc), _ptr(a.view(np.float64)), int(keep), _ptr(out))
    if rc:
        raise ValueError(f"orc_density_1d rc={rc}")
    return out


def density_2d(prob: Problem, psi, drop: int) -> np.ndarray:
    a = _as_state(prob, psi)
    n = list(prob.n)
    keep = [ax for ax in range(3) if ax != drop]
    out = np.zeros((n[keep[1]], n[keep[0]]))
    pc = prob.c()
    rc = load().orc_density_2d(ctypes.byref(pc), _ptr(a.view(np.float64)), int(drop),
                               _ptr(out.reshape(-1)))
    if rc:
        raise ValueError(f"orc_density_2d rc={rc}")
    return out


def threads() -> int:
    return int(load().orc_threads())


def set_threads(n: int) -> None:
    if load().orc_set_threads(int(n)):
        raise ValueError(f"orc_set_threads({n})")


# ---------------------------------------------------------------------------
# symmetric traps (sscn_sym_oracle.c)
# ---------------------------------------------------------------------------

def _as_sym_state(prob: SymProblem, psi) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(psi, dtype=np.complex128).reshape(prob.shape)).copy()


def sym_coefs(prob: SymProblem):
    """(l, d, u, W): H_r = -Lap_r/2 on radial cell i is
    d_i psi_i - l_i psi_{i-1} - u_i psi_{i+1}; W_i the cell weights."""
    n = prob.n[0]
    l, d, u, w = (np.zeros(n) for _ in range(4))
    pc = prob.c()
    rc = load().ors_coefs(ctypes.byref(pc), _ptr(l), _ptr(d), _ptr(u), _ptr(w))
    if rc:
        raise ValueError(f"ors_coefs rc={rc}")
    return l, d, u, w


def sym_observe(prob: SymProblem, psi) -> Observables:
    a = _as_sym_state(prob, psi)
    out = np.zeros(12)
    pc = prob.c()
    rc = load().ors_observe(ctypes.byref(pc), _ptr(a.view(np.float64)), _ptr(out))
    if rc:
        raise ValueError(f"ors_observe rc={rc}")
    return Observables(*out[:6], tuple(out[6:9]), tuple(out[9:12]))


def sym_substep(prob: SymProblem, psi, which: int) -> np.ndarray:
    """which = -1: pointwise substep; 0: the r substep; 1: the z substep."""
    a = _as_sym_state(prob, psi)
    pc = prob.c()
    rc = load().ors_substep(ctypes.byref(pc), _ptr(a.view(np.float64)), int(which))
    if rc:
        raise ValueError(f"ors_substep rc={rc}")
    return a


def sym_run(prob: SymProblem, psi, nsteps: int, observe_every: int = 0,
            mu_tol: float = 0.0, first_step: int = 1) -> RunResult:
    a = _as_sym_state(prob, psi)
    cap = (nsteps // observe_every + 2) if observe_every > 0 else 2
    trace = np.zeros((cap, len(SYM_TRACE_COLS)))
    rows = ctypes.c_long(0)
    done = ctypes.c_long(0)
    pc = prob.c()
    rc = load().ors_run(ctypes.byref(pc), _ptr(a.view(np.float64)), int(nsteps), int(first_step),
                        int(observe_every), float(mu_tol), _ptr(trace), cap, ctypes.byref(rows),
                        ctypes.byref(done))
    if rc < 0:
        raise ValueError(f"ors_run rc={rc}")
    return RunResult(a, trace[: rows.value].copy(), int(done.value), rc == 0)


# ---------------------------------------------------------------------------
# physical units -> dimensionless nonlinearity
# ---------------------------------------------------------------------------

def units_to_g(dim: int, atoms: float, scattering_length_bohr: float, mass_amu: float, omega: float,
               tight=(1.0, 1.0)):
    """The nonlinearity of the dimensionless GP equation from physical inputs
    (the paper's programs take the number of atoms, the scattering length
    and the trap's oscillator length; "Reasons for the new version").  In
    units of l = sqrt(hbar/(m omega)) the 3D coefficient is 4 pi N a / l; a
    problem of lower dimension keeps the frozen directions in their
    oscillator ground states and integrates |phi|^4 over them, here by
    numerical quadrature of the normalised Gaussians (no closed form).
    Parity unpinned against the paper's programs: it prints no formula.
    Returns (g, l in m, 1/omega in s)."""
    hbar, amu, bohr = 1.054571817e-34, 1.66053906660e-27, 5.29177210903e-11
    length = math.sqrt(hbar / (mass_amu * amu * omega))
    g = 4.0 * math.pi * atoms * scattering_length_bohr * bohr / length
    frozen = {3: (), 2: (tight[0],), 1: (tight[0], tight[1])}[int(dim)]
    for nu in frozen:
        # phi(z) = (nu/pi)^(1/4) exp(-nu z^2/2): integrate phi^4 on a grid
        # reaching 12 widths, trapezoid rule (spectrally accurate here)
        w = 1.0 / math.sqrt(nu)
        z = np.linspace(-12.0 * w, 12.0 * w, 20001)
        phi = (nu / math.pi) ** 0.25 * np.exp(-0.5 * nu * z * z)
        g *= float(np.trapezoid(phi ** 4, z))
    return g, length, 1.0 / omega
