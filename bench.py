"""Benchmark: SSCN grid-point-steps/s at 256^3 on one MI355X.

Workload (one "step" = one full SSCN time step: pointwise substep + x, y, z
Crank-Nicolson sweeps): real-time 3D propagation of a 256^3 complex128 state,
dx = 0.1, dt = 0.02 dx^2, trap (1, 1.5, 2), initial Thomas-Fermi profile of
g = 100 times a seeded random phase (sigma 0.05), propagated with g = 80.
The same workload in complex64 (FP32 sweeps, FP64 tables and reductions) is
timed beside it.  Inputs are resident in HBM before the timed region.

Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSCN grid-point-steps/s at 256^3 FP64 vs FP32; p50/p99 batched solve latency"
HBM_PEAK_GBS = 8000.0


def c1_problem(prec):
    from paper_1605_03958_amd.sscn import Problem, REAL
    dx = 0.1
    return Problem(3, (256, 256, 256), (dx, dx, dx), (1.0, 1.5, 2.0), 80.0, 0.02 * dx * dx, REAL, prec, 0)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("sscn_dev.hpp", "sscn_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1605_03958_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_class: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, or
    None when it is absent or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel_class)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def time_steps(solver, steps, warmup):
    import torch
    solver.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def copy_bandwidth(nbytes: int, reps: int = 20):
    """Device-to-device copy rate (GB/s, read + write counted) of a plain
    torch copy kernel over nbytes, as a measured ceiling beside the peak."""
    import torch
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2 * nbytes / dt / 1e9


def cpu_baseline(target_s: float = 12.0):
    """The FP64 oracle on a bounded sample of the same workload: the full
    256^3 grid for as many steps as fit in about target_s seconds."""
    import oracle
    from paper_1605_03958_amd import inputs
    p = c1_problem(0)
    op = oracle.Problem(p.dim, p.n, p.dx, p.omega, p.g, p.dt, p.mode, p.renorm_every)
    psi0 = inputs.thomas_fermi(3, p.n, p.dx, p.omega, 100.0, phase_sigma=0.05, seed=1)
    t0 = time.perf_counter()
    r = oracle.run(op, psi0, 2)
    t2 = time.perf_counter() - t0
    steps = max(1, int(2 * target_s / max(t2, 1e-3)) - 2)
    t0 = time.perf_counter()
    oracle.run(op, r.psi, steps, first_step=3)
    dt = time.perf_counter() - t0
    total = steps + 2
    return {"value": p.points * total / (dt + t2), "unit": "grid-point-steps/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"256^3 complex128 real-time workload, first {total} steps ({dt + t2:.1f} s), "
                      f"FP64 C oracle with OpenMP over lines"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--only", choices=["fp64", "fp32"], default=None,
                    help="run only one precision (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent problems shard trivially across GPUs, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1605_03958_amd import inputs, sscn

    torch.cuda.set_device(0)
    out = {}
    precs = [sscn.F64, sscn.F32]
    if args.no_fp32 or args.only == "fp64":
        precs = [sscn.F64]
    if args.only == "fp32":
        precs = [sscn.F32]
    psi0 = inputs.thomas_fermi(3, (256, 256, 256), (0.1,) * 3, (1.0, 1.5, 2.0), 100.0, phase_sigma=0.05, seed=1)
    for prec in precs:
        p = c1_problem(prec)
        s = sscn.Solver(p, psi0)
        el = time_steps(s, args.steps, args.warmup)
        kms = s.step_timed(args.steps)
        S = 16 if prec == sscn.F64 else 8
        out[prec] = dict(elapsed=el, pts=p.points * args.steps / el, kernels=kms, S=S, points=p.points)
        s.close()
        del s
        torch.cuda.empty_cache()

    main_prec = precs[0]
    m = out[main_prec]
    # dominant kernel: the sweep class with the largest mean duration
    sweeps = {k: v for k, v in m["kernels"].items() if k in ("x_sweep_pointwise", "y_sweep", "z_sweep_norm")}
    dom = max(sweeps, key=sweeps.get)
    alg_bytes = 2 * m["S"] * m["points"]            # one read + one write of psi per sweep
    achieved = alg_bytes / (sweeps[dom] * 1e-3) / 1e9
    workload = "c1_256cube_c128" if main_prec == sscn.F64 else "c2_256cube_c64"
    traffic = load_traffic(dom, workload)
    res = {
        "metric": METRIC,
        "value": m["pts"],
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * m["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == sscn.F64 else "f32",
        "data": "synthetic",
        "config": {"workload": "real-time 3D SSCN, 256^3 complex128, dx=0.1, dt=0.02*dx^2, trap (1,1.5,2), "
                               "Thomas-Fermi(g=100) x random phase sigma 0.05 (seed 1), g quenched to 80",
                   "grid": [256, 256, 256], "state": "complex128" if main_prec == sscn.F64 else "complex64",
                   "mode": "real-time"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes, "mean_launch_ms": sweeps[dom]},
        "kernel_ms": {k: round(v, 5) for k, v in m["kernels"].items()},
        "step_hbm_frac": (6 * m["S"] * m["points"] * args.steps / m["elapsed"]) / (HBM_PEAK_GBS * 1e9),
    }
    if sscn.F32 in out and main_prec == sscn.F64:
        f = out[sscn.F32]
        res["fp32"] = {"value": f["pts"], "ms_per_step": 1e3 * f["elapsed"] / args.steps,
                       "speedup_vs_fp64": f["pts"] / m["pts"], "kernel_ms": {k: round(v, 5) for k, v in f["kernels"].items()},
                       "state": "complex64"}
    res["copy_gbs"] = copy_bandwidth(m["S"] * m["points"])
    if not args.no_cpu and args.only is None:
        res["cpu_baseline"] = cpu_baseline()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
