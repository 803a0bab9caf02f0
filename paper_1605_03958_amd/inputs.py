"""Seeded synthetic inputs shared by the GPU path's tests, the oracle's tests
and the benchmark.

This module holds no arithmetic of the propagation method: it only draws
initial states and instance parameters.  The same FP64 arrays go to the
oracle and to the GPU library (FP32 runs receive them rounded), so both sides
start from identical data.  Every draw uses ``numpy.random.default_rng(seed)``
(PCG64) in a fixed order.

Grid convention (shared with both implementations by definition, not by
code): axis a has n_a points at x_a(i) = (i - (n_a - 1)/2) dx_a, layout x
fastest, arrays shaped (n_z, n_y, n_x).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def coords(n: int, dx: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * dx


def _pad3(v, fill):
    v = list(v)
    return v + [fill] * (3 - len(v))


def _mesh(dim, n, dx):
    n = _pad3(n, 1)
    dx = _pad3(dx, 1.0)
    axes = [coords(n[a], dx[a]) if a < dim else np.zeros(1) for a in range(3)]
    z, y, x = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return x, y, z


def _dvol(dim, dx):
    return float(np.prod(np.asarray(dx[:dim], dtype=np.float64)))


def trap_potential(dim, n, dx, omega) -> np.ndarray:
    """V = sum_a omega_a^2 x_a^2 / 2 on the grid (used to shape initial states)."""
    x, y, z = _mesh(dim, n, dx)
    om = _pad3(omega, 0.0)
    v = 0.5 * om[0] ** 2 * x ** 2
    if dim > 1:
        v = v + 0.5 * om[1] ** 2 * y ** 2
    if dim > 2:
        v = v + 0.5 * om[2] ** 2 * z ** 2
    return v


def ho_gaussian(dim, n, dx, omega, noise: float = 1e-3, seed: int = 0,
                shift=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Harmonic-oscillator ground-state Gaussian prod_a (w_a/pi)^(1/4)
    exp(-w_a (x_a - shift_a)^2 / 2), plus U[-noise, noise) per point, then
    normalised so that dV * sum psi^2 = 1.  Real FP64, shape (nz, ny, nx)."""
    nn = _pad3(n, 1)
    dd = _pad3(dx, 1.0)
    # per-axis coordinates broadcast against the (nz, ny, nx) array: the
    # same products in the same order as on a full mesh, without the mesh
    ax = [coords(nn[a], dd[a]) if a < dim else np.zeros(1) for a in range(3)]
    om = _pad3(omega, 1.0)
    sh = _pad3(shift, 0.0)
    psi = np.ones((1, 1, 1))
    for a, c in enumerate((ax[0][None, None, :], ax[1][None, :, None], ax[2][:, None, None])):
        if a < dim:
            w = om[a]
            psi = psi * (w / math.pi) ** 0.25 * np.exp(-0.5 * w * (c - sh[a]) ** 2)
    psi = np.broadcast_to(psi, (nn[2], nn[1], nn[0]))
    if noise > 0:
        rng = np.random.default_rng(seed)
        psi = psi + rng.uniform(-noise, noise, size=psi.shape)
    nrm = _dvol(dim, _pad3(dx, 1.0)) * np.sum(psi * psi)
    return psi / math.sqrt(nrm)


def mu_thomas_fermi(dim: int, g: float, omega) -> float:
    """Thomas-Fermi chemical potential of a unit-norm condensate."""
    om = _pad3(omega, 1.0)
    if dim == 1:
        return 0.5 * (1.5 * g * om[0]) ** (2.0 / 3.0)
    if dim == 2:
        return math.sqrt(g * om[0] * om[1] / math.pi)
    return 0.5 * (15.0 * g * om[0] * om[1] * om[2] / (4.0 * math.pi)) ** 0.4


def thomas_fermi(dim, n, dx, omega, g_init: float, phase_sigma: float = 0.0,
                 seed: int = 1) -> np.ndarray:
    """sqrt(max(mu_TF - V, 0) / g_init), normalised to dV * sum |psi|^2 = 1,
    times exp(i theta) with theta ~ N(0, phase_sigma^2) iid per point.
    Complex128, shape (nz, ny, nx)."""
    v = trap_potential(dim, n, dx, omega)
    mu = mu_thomas_fermi(dim, g_init, omega)
    amp = np.sqrt(np.maximum(mu - v, 0.0) / g_init)
    nrm = _dvol(dim, _pad3(dx, 1.0)) * np.sum(amp * amp)
    amp = amp / math.sqrt(nrm)
    if phase_sigma > 0:
        rng = np.random.default_rng(seed)
        theta = rng.normal(0.0, phase_sigma, size=amp.shape)
        return amp * np.exp(1j * theta)
    return amp.astype(np.complex128)


# ---------------------------------------------------------------------------
# Symmetric traps: circular (2D, psi(r)), spherical (3D, psi(r)), axial
# (3D, psi(rho, z)).  Radial grid convention (shared by both implementations
# by definition, not by code): n cells of width dr with values at the
# centres r_i = (i + 1/2) dr; z as a Cartesian axis.  Arrays are shaped
# (n_z, n_r), r fastest (n_z = 1 unless axial).
# ---------------------------------------------------------------------------

SYM_CIR, SYM_SPH, SYM_AXI = 1, 2, 3


def radial_coords(n: int, dr: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) * dr


def sym_gaussian(geom: int, n, dx, omega, noise: float = 1e-3, seed: int = 0,
                 z_shift: float = 0.0) -> np.ndarray:
    """The harmonic-oscillator ground state of the trap (continuum
    normalisation: (w/pi)^(d/4) exp(-w r^2/2) with d = 2 (circular) or 3
    (spherical); axial: (w_rho/pi)^(1/2) (w_z/pi)^(1/4) exp(-w_rho rho^2/2
    - w_z (z - z_shift)^2/2)), plus U[-noise, noise) per point.  Real FP64,
    shape (n_z, n_r).  Not renormalised on the grid."""
    nr = int(n[0])
    nz = int(n[1]) if geom == SYM_AXI else 1
    r = radial_coords(nr, dx[0])
    w = omega[0]
    if geom == SYM_CIR:
        psi = (w / math.pi) ** 0.5 * np.exp(-0.5 * w * r * r)[None, :]
    elif geom == SYM_SPH:
        psi = (w / math.pi) ** 0.75 * np.exp(-0.5 * w * r * r)[None, :]
    else:
        wz = omega[1]
        z = coords(nz, dx[1]) - z_shift
        psi = ((w / math.pi) ** 0.5 * np.exp(-0.5 * w * r * r)[None, :]
               * ((wz / math.pi) ** 0.25 * np.exp(-0.5 * wz * z * z))[:, None])
    psi = np.broadcast_to(psi, (nz, nr))
    if noise > 0:
        rng = np.random.default_rng(seed)
        psi = psi + rng.uniform(-noise, noise, size=psi.shape)
    return np.array(psi)


def sym_mu_thomas_fermi(geom: int, g: float, omega) -> float:
    """Thomas-Fermi chemical potential of a unit-norm condensate in the
    symmetric trap (2D isotropic for circular, 3D otherwise)."""
    w = omega[0]
    if geom == SYM_CIR:
        return math.sqrt(g * w * w / math.pi)
    wz = w if geom == SYM_SPH else omega[1]
    return 0.5 * (15.0 * g * w * w * wz / (4.0 * math.pi)) ** 0.4


def sym_thomas_fermi(geom: int, n, dx, omega, g_init: float, phase_sigma: float = 0.0,
                     seed: int = 1) -> np.ndarray:
    """sqrt(max(mu_TF - V, 0) / g_init) (continuum-normalised by the choice of
    mu_TF) times exp(i theta), theta ~ N(0, phase_sigma^2) iid per point.
    Complex128, shape (n_z, n_r)."""
    nr = int(n[0])
    nz = int(n[1]) if geom == SYM_AXI else 1
    r = radial_coords(nr, dx[0])
    v = 0.5 * omega[0] ** 2 * r * r
    if geom == SYM_AXI:
        z = coords(nz, dx[1])
        v = v[None, :] + (0.5 * omega[1] ** 2 * z * z)[:, None]
    else:
        v = v[None, :]
    mu = sym_mu_thomas_fermi(geom, g_init, omega)
    amp = np.sqrt(np.maximum(mu - v, 0.0) / g_init)
    if phase_sigma > 0:
        rng = np.random.default_rng(seed)
        return amp * np.exp(1j * rng.normal(0.0, phase_sigma, size=amp.shape))
    return amp.astype(np.complex128)


# ---------------------------------------------------------------------------
# Batch and serving draws
# ---------------------------------------------------------------------------

@dataclass
class InstanceDraw:
    index: int
    dim: int
    n: tuple
    dx: tuple
    omega: tuple
    g: float
    seed: int


def batch_draw(index: int, seed_base: int = 100, dims=None) -> InstanceDraw:
    """One instance of the uneven batch mix.  Index 0..21 are 1D, 22..42 2D,
    43..63 3D (for a 64-instance batch; ``dims`` overrides).  Sizes: 1D
    n ~ U{2048..16384}; 2D square n ~ U{256..1024}; 3D cube n ~ U{48..160}.
    Trap frequencies iid U[0.5, 4]; g = 10^U[0, 3]; dx ~ U[0.05, 0.25]."""
    if dims is None:
        dim = 1 if index < 22 else (2 if index < 43 else 3)
    else:
        dim = dims
    seed = seed_base + index
    rng = np.random.default_rng(seed)
    if dim == 1:
        m = int(rng.integers(2048, 16384, endpoint=True))
    elif dim == 2:
        m = int(rng.integers(256, 1024, endpoint=True))
    else:
        m = int(rng.integers(48, 160, endpoint=True))
    om = rng.uniform(0.5, 4.0, size=3)
    g = float(10.0 ** rng.uniform(0.0, 3.0))
    h = float(rng.uniform(0.05, 0.25))
    n = tuple([m] * dim + [1] * (3 - dim))
    dx = tuple([h] * dim + [1.0] * (3 - dim))
    omega = tuple(float(om[a]) if a < dim else 0.0 for a in range(3))
    return InstanceDraw(index, dim, n, dx, omega, g, seed)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    kind: str               # "ground" or "dynamics"
    draw: InstanceDraw


def request_stream(count: int, rate: float, seed: int = 200, ground_frac: float = 0.7):
    """Poisson arrivals at ``rate`` per second; 70 % ground-state requests,
    30 % real-time requests; sizes and parameters from the batch mix."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    kinds = rng.uniform(size=count)
    dims = rng.integers(1, 4, size=count)
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        kind = "ground" if kinds[i] < ground_frac else "dynamics"
        d = batch_draw(i, seed_base=seed * 1000, dims=int(dims[i]))
        out.append(Request(i, float(t[i]), kind, d))
    return out
