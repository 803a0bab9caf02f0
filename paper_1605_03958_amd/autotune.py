"""Tile autotuner.

For one problem shape it measures the candidate points-per-thread choices of
each axis and keeps the fastest, then records the choice in a JSON cache so
later runs apply it without measuring.  Two targets:

* ``single``: the single-problem kernels (``sscn_set_tile_hint``); the cost of
  a candidate is the mean duration of the sweeps over a few steps, from the
  per-kernel HIP events of ``Solver.step_timed``.
* ``batch``: the persistent batched kernel (``sscn_batch_set_tile_hint``);
  the cost is the time per launch of a batch holding enough copies of the
  shape to fill the device (the copies share the shape, hence the tiles).

The search is coordinate-wise: axis by axis, every candidate of that axis
with the other axes at their current best, starting from the library's own
choice, which is always a candidate, so the result is never slower than the
default as measured.  A hint depends on the shape only, so an instance's
geometry (and its results) stays independent of what else runs.

Cache key: ``target|arch|dim|nx,ny,nz|mode|prec``.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Optional

import numpy as np

from . import inputs, sscn
from .sscn import F32, IMAG, Problem

SINGLE_CHUNKS = (1, 2, 4, 8, 16, 32, 64)
BATCH_ROW_CHUNKS = {False: (1, 2, 3, 4, 6, 8, 12, 16), True: (1, 2, 3, 4, 6, 8)}
BATCH_COL_CHUNKS = {False: (2, 3, 4, 5, 6, 8, 10, 12, 16), True: (2, 3, 4, 5, 6, 8)}


def device_arch() -> str:
    import torch
    if not torch.cuda.is_available():
        return "cpu"
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def cache_key(target: str, prob: Problem, arch: str) -> str:
    n = ",".join(str(int(v)) for v in prob.n)
    return f"{target}|{arch}|{prob.dim}|{n}|{prob.mode}|{prob.prec}"


def load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(path: str, cache: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _state(prob: Problem, seed: int = 0):
    psi = inputs.ho_gaussian(prob.dim, prob.n, prob.dx, prob.omega, noise=1e-3, seed=seed)
    if prob.mode != IMAG:
        psi = psi.astype(np.complex128)
    return psi


# ---------------------------------------------------------------------------
# measurement
# ---------------------------------------------------------------------------

def measure_single(prob: Problem, chunks, steps: int = 300, psi0=None, warm: int = 100) -> float:
    """Wall-clock time (ms) per step with these chunks, over `steps` graph-
    replayed steps after `warm` untimed ones (per-kernel event timing adds
    its own overhead to short kernels and moved the choice by noise)."""
    import torch
    sscn.set_tile_hint(prob, chunks)
    s = sscn.Solver(prob, _state(prob) if psi0 is None else psi0)
    try:
        s.step(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        s.close()
    return 1e3 * el / steps


def measure_batch(prob: Problem, chunks, launches: int = 10, target_points: float = 2.0e7, psi0=None) -> float:
    """Time (ms) per launch of a batch of copies of prob with these chunks."""
    import torch
    sscn.batch_set_tile_hint(prob, chunks)
    copies = int(max(1, min(64, target_points // max(1, prob.points))))
    st = torch.cuda.Stream()
    b = sscn.Batch(copies, stream=st)
    try:
        psi = _state(prob) if psi0 is None else psi0
        for i in range(copies):
            b.admit(i, prob, psi, mu_tol=0.0, max_steps=1 << 40)
        b.step(launches)
        b.poll()
        t0 = time.perf_counter()
        b.step(launches)
        b.poll()
        dt = (time.perf_counter() - t0) / launches
        if b.error():
            raise RuntimeError("batch wait gave up while tuning")
    finally:
        b.close()
    return 1e3 * dt


# ---------------------------------------------------------------------------
# search
# ---------------------------------------------------------------------------

def candidates(target: str, prob: Problem):
    """Per-axis candidate chunks (0 = the library's own choice)."""
    out = []
    cplx = prob.mode != IMAG
    for a in range(3):
        if a >= prob.dim:
            out.append([0])
            continue
        if target == "single":
            out.append([0] + list(SINGLE_CHUNKS))
        elif a == 0:
            # single-wave x lines of 2D and 3D instances take at most 4 points per thread
            out.append([0] + [c for c in BATCH_ROW_CHUNKS[cplx] if c * 64 >= prob.n[0] and (prob.dim == 1 or c <= 4)])
        else:
            # at most 16 waves x 8 lanes of chunks cover a line
            out.append([0] + [c for c in BATCH_COL_CHUNKS[cplx] if c * 128 >= prob.n[a]])
    return out


def _settable(target: str, prob: Problem, chunks) -> bool:
    try:
        if target == "single":
            sscn.set_tile_hint(prob, chunks)
        else:
            sscn.batch_set_tile_hint(prob, chunks)
        return True
    except sscn.SSCNError:
        return False


def _clear(target: str) -> None:
    if target == "single":
        sscn.clear_tile_hints()
    else:
        sscn.batch_clear_tile_hints()


def tune(prob: Problem, target: str = "batch", cache_path: Optional[str] = None, measure: Optional[Callable] = None,
         reps: int = 2, force: bool = False, arch: Optional[str] = None, log: Callable = lambda *_: None,
         margin: float = 0.02) -> dict:
    """Search the chunks of prob's shape, store and return the record
    {"chunks": [...], "ms": best, "default_ms": ..., "tried": {...}}.  A
    candidate replaces the best so far only when it is faster by more than
    `margin` (relative), so timing noise does not move the choice."""
    if target not in ("single", "batch"):
        raise ValueError(target)
    if target == "batch" and prob.prec != F32:
        raise ValueError("the batch runs the FP32 forms")
    arch = arch or device_arch()
    cache = load_cache(cache_path)
    key = cache_key(target, prob, arch)
    if key in cache and not force:
        return cache[key]
    if measure is None:
        psi0 = _state(prob)                  # one initial state for every candidate
        base = measure_single if target == "single" else measure_batch

        def meas(p, ch):
            return base(p, ch, psi0=psi0)
    else:
        meas = measure

    tried = {}

    def cost(ch):
        k = ",".join(str(c) for c in ch)
        if k not in tried:
            if not _settable(target, prob, ch):
                tried[k] = None
            else:
                tried[k] = min(meas(prob, list(ch)) for _ in range(reps))
            log(f"{target} {prob.n} chunks {ch}: {tried[k]}")
        return tried[k]

    try:
        best = [0, 0, 0]
        default_ms = cost(best)
        best_ms = default_ms
        for a, cand in enumerate(candidates(target, prob)):
            for c in cand:
                ch = list(best)
                ch[a] = c
                t = cost(ch)
                if t is not None and t < best_ms * (1.0 - margin):
                    best, best_ms = ch, t
    finally:
        _clear(target)
    rec = {"chunks": best, "ms": best_ms, "default_ms": default_ms,
           "tried": {k: v for k, v in tried.items() if v is not None}}
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = rec
        save_cache(cache_path, cache)
    return rec


def apply(prob: Problem, target: str = "batch", cache_path: Optional[str] = None, arch: Optional[str] = None) -> bool:
    """Set the cached hint of prob's shape, if there is one; True if set."""
    rec = load_cache(cache_path).get(cache_key(target, prob, arch or device_arch()))
    if not rec or not any(rec["chunks"]):
        return False
    if target == "single":
        sscn.set_tile_hint(prob, rec["chunks"])
    else:
        sscn.batch_set_tile_hint(prob, rec["chunks"])
    return True


# ---------------------------------------------------------------------------
# command line: tune the shapes of the standard workloads
# ---------------------------------------------------------------------------

def mix_problems():
    """The 64 shapes of the uneven batch mix (imaginary time, FP32)."""
    out = []
    for i in range(64):
        d = inputs.batch_draw(i)
        h = d.dx[0]
        out.append(Problem(d.dim, d.n, d.dx[:d.dim], d.omega[:d.dim], d.g, 0.1 * h * h, IMAG, F32, 1, 10))
    return out


def cube_problems():
    """The 256^3 real-time workload in FP64 and FP32."""
    from .sscn import F64, REAL
    dx = 0.1
    return [Problem(3, (256, 256, 256), (dx, dx, dx), (1.0, 1.5, 2.0), 80.0, 0.02 * dx * dx, REAL, prec, 0)
            for prec in (F64, F32)]


def imag_problems():
    """The imaginary-time workloads of the benchmark: the 64^3 FP64 ground
    state (dx = 0.2) and its physics at 256^3 (dx = 0.05) in FP64 and FP32."""
    from .sscn import F64
    out = [Problem(3, (64, 64, 64), (0.2,) * 3, (1.0, 1.5, 2.0), 22.0, 0.1 * 0.2 * 0.2, IMAG, F64, 1)]
    out += [Problem(3, (256, 256, 256), (0.05,) * 3, (1.0, 1.5, 2.0), 22.0, 0.1 * 0.05 * 0.05, IMAG, prec, 1)
            for prec in (F64, F32)]
    return out


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune tile shapes and store them in a JSON cache")
    ap.add_argument("--cache", required=True)
    ap.add_argument("--mix", action="store_true", help="the 64 shapes of the uneven batch mix (batch kernel)")
    ap.add_argument("--cube", action="store_true", help="the 256^3 workload (single-problem kernels)")
    ap.add_argument("--imag", action="store_true",
                    help="the 64^3 and 256^3 imaginary-time workloads (single-problem kernels)")
    ap.add_argument("--force", action="store_true")
    args = ap.parse_args(argv)
    jobs = []
    if args.mix:
        seen = set()
        for p in mix_problems():
            if p.dim == 1 or (p.dim, p.n) in seen:      # 1D lines run as one item: nothing to choose
                continue
            seen.add((p.dim, p.n))
            jobs.append(("batch", p))
    if args.cube:
        jobs += [("single", p) for p in cube_problems()]
    if args.imag:
        jobs += [("single", p) for p in imag_problems()]
    t0 = time.perf_counter()
    for k, (target, p) in enumerate(jobs):
        rec = tune(p, target, cache_path=args.cache, reps=3 if target == "single" else 1, force=args.force)
        print(f"[{k + 1}/{len(jobs)} {time.perf_counter() - t0:.0f}s] {target} dim={p.dim} n={p.n} "
              f"prec={p.prec}: chunks {rec['chunks']} {rec['ms']:.4f} ms (default {rec['default_ms']:.4f})",
              flush=True)


if __name__ == "__main__":
    main()
