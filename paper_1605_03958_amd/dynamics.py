"""Ground state, then dynamics: the imaginary -> real-time pipeline.

The paper's real-time programs can start from the state that an
imaginary-time run converged to (the NSTP = 0 hand-off of its "Summary of
revisions" section), multiply the nonlinearity by a factor, and record the
rms sizes of the condensate over time (its dynamics output files, with time
in the first column and the rms sizes per axis and of r after it).

This module only orchestrates library calls (sscn_run, sscn_observe) on two
solvers; every step runs in the HIP kernels.  The hand-off stays on the
device: the converged real state is cast to the real-time dtype on the
imaginary-time solver's stream and copied into the real-time solver's
state.

rms sizes are taken about the trap centre (the origin of the coordinates):
rms_a = sqrt(<x_a^2>) per present axis and rms_r = sqrt(sum_a <x_a^2>).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, replace

import numpy as np

from . import sscn


def rms_sizes(obs: "sscn.Obs", dim: int):
    """(rms_x, ..., rms_r) from an observation's second moments."""
    msq = [max(float(obs.msq[a]), 0.0) for a in range(dim)]
    return tuple(math.sqrt(m) for m in msq) + (math.sqrt(sum(msq)),)


@dataclass
class Dynamics:
    ground: "sscn.Obs"          # last observation of the imaginary-time run
    ground_steps: int           # imaginary-time steps taken
    converged: bool             # |delta mu| fell below mu_tol
    table: np.ndarray           # rows: t, rms per present axis, rms_r
    trace: list                 # the real-time observations, t = 0 first
    imag_seconds: float = 0.0   # wall time of the imaginary-time run
    real_seconds: float = 0.0   # wall time of the real-time run


def ground_state_then_dynamics(prob: "sscn.Problem", psi0, g_factor: float, real_steps: int,
                               dt_real: float, mu_tol: float = 1e-7,
                               max_imag_steps: int = 1_000_000, observe_every: int = 1) -> Dynamics:
    """Imaginary-time propagation of prob (mode IMAG) from psi0 until
    |delta mu| < mu_tol between observations (or max_imag_steps), then
    real_steps real-time steps of size dt_real from the converged state with
    the nonlinearity g * g_factor, observed every observe_every steps."""
    if prob.mode != sscn.IMAG:
        raise ValueError("the pipeline starts from an imaginary-time problem")
    if real_steps < 0 or observe_every < 1:
        raise ValueError("real_steps >= 0 and observe_every >= 1 are required")
    import torch
    rp = replace(prob, g=prob.g * g_factor, dt=dt_real, mode=sscn.REAL, renorm_every=0,
                 observe_every=observe_every)
    s = sscn.Solver(prob, psi0)
    try:
        t0 = time.perf_counter()
        # no trace: the convergence test runs inside sscn_run, and the
        # last observation is read afterwards
        rc, _ = s.run(max_imag_steps, mu_tol, trace_cap=0)
        ground = s.observe()
        t_imag = time.perf_counter() - t0
        if ground.status != sscn.OK:
            raise sscn.SSCNError(ground.status, "imaginary-time run")
        with torch.cuda.stream(s.stream):
            psi_g = s.psi.to(rp.torch_dtype())
        s.stream.synchronize()
    finally:
        s.close()
    r = sscn.Solver(rp, psi_g)
    del psi_g
    try:
        trace = [r.observe()]
        t0 = time.perf_counter()
        if real_steps:
            _, rows = r.run(real_steps, 0.0, trace_cap=real_steps // observe_every + 2)
            trace += rows
        t_real = time.perf_counter() - t0
    finally:
        r.close()
    table = np.array([(o.step * dt_real,) + rms_sizes(o, prob.dim) for o in trace])
    return Dynamics(ground, ground.step, rc == sscn.OK, table, trace, t_imag, t_real)
