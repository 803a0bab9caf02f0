"""Dense numpy formulations used to pin the CPU oracle on tiny grids.

These build the whole linear operators as explicit matrices (numpy.linalg
solves and Kronecker products) instead of per-line Thomas sweeps, so a wrong
stride, axis, sign or coefficient in the oracle's line code shows up as a
mismatch.  The discretisation they encode is the one the oracle's header
states: Lie splitting, pointwise substep first, then Crank-Nicolson along x, y
and z with the 3-point Laplacian and zero Dirichlet ghosts.
"""
from __future__ import annotations

import numpy as np


def lap_T(n: int) -> np.ndarray:
    """T = tridiag(-1, 2, -1) (n x n): dx^2 times minus the 3-point Laplacian."""
    return 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def cn_matrix(n: int, sigma: complex) -> np.ndarray:
    """(I + sigma T)^-1 (I - sigma T) as a dense matrix."""
    T = lap_T(n)
    return np.linalg.solve(np.eye(n) + sigma * T, np.eye(n) - sigma * T)


def sigma_of(dt: float, dx: float, real_time: bool) -> complex:
    """Crank-Nicolson coefficient for H_a = -1/2 d^2/dx^2 over one step:
    imaginary time exp(-dt H) ~ (1 + dt H/2)^-1 (1 - dt H/2), real time
    exp(-i dt H) ~ (1 + i dt H/2)^-1 (1 - i dt H/2); dt H/2 = dt/(4 dx^2) T."""
    s = dt / (4.0 * dx * dx)
    return 1j * s if real_time else s


def full_step_operator(n3, dx3, dim, dt, real_time):
    """Dense kinetic operator of one step on the flattened grid (x fastest):
    L = (C_z x I x I)(I x C_y x I)(I x I x C_x), Kronecker order z, y, x."""
    nx, ny, nz = n3
    mats = []
    for a in range(3):
        na = n3[a]
        if a < dim:
            mats.append(cn_matrix(na, sigma_of(dt, dx3[a], real_time)))
        else:
            mats.append(np.eye(na))
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    Lx = np.kron(Iz, np.kron(Iy, mats[0]))
    Ly = np.kron(Iz, np.kron(mats[1], Ix))
    Lz = np.kron(mats[2], np.kron(Iy, Ix))
    return Lz @ Ly @ Lx


def dense_run(psi0, n3, dx3, dim, V, g, dt, real_time, nsteps, renorm_every=1):
    """Brute-force propagation on the flattened state with dense operators."""
    L = full_step_operator(n3, dx3, dim, dt, real_time)
    v = V.reshape(-1)
    dV = float(np.prod(dx3[:dim]))
    psi = np.asarray(psi0, dtype=np.complex128).reshape(-1).copy()
    for step in range(1, nsteps + 1):
        q = np.abs(psi) ** 2
        phi = dt * (v + g * q)
        psi = (np.exp(-1j * phi) if real_time else np.exp(-phi)) * psi
        psi = L @ psi
        if not real_time and renorm_every > 0 and step % renorm_every == 0:
            psi = psi / np.sqrt(dV * np.sum(np.abs(psi) ** 2))
    return psi.reshape(psi0.shape)


def hamiltonian_1d(n: int, dx: float, omega: float, x: np.ndarray) -> np.ndarray:
    """Dense 1D discrete Hamiltonian -1/2 Lap_h + omega^2 x^2 / 2 (Dirichlet)."""
    return lap_T(n) / (2.0 * dx * dx) + np.diag(0.5 * omega * omega * x * x)


def dominant_state_1d(n, dx, omega, dt, x):
    """Fixed point of the 1D imaginary-time map M = C diag(exp(-dt V)) at g=0:
    the eigenvector of M with the largest eigenvalue modulus."""
    C = cn_matrix(n, sigma_of(dt, dx, False))
    M = C @ np.diag(np.exp(-dt * 0.5 * omega * omega * x * x))
    w, vecs = np.linalg.eig(M)
    k = int(np.argmax(np.abs(w)))
    v = np.real(vecs[:, k])
    return v / np.linalg.norm(v)
