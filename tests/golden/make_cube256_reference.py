"""Write the FP64 CPU oracle's result for the 256^3 real-time workload after
1000 steps:

* ``cube256_oracle_1000.json``: the observables before and after, the state at
  a seeded sample of 4096 grid points, and the state's sum of |psi|^2;
* ``cube256_oracle_1000_lines.npz``: line sums that together touch every grid
  point -- per x line sum_i psi and sum_i (i + 1) psi / n_x, per y line
  sum_j psi, per z line sum_k psi (complex128, 65536 lines each).  A wrong
  value at any single point moves at least three of them.

Calls only the oracle and the seeded input generator.  Takes about 11 min on
8 cores.  Workload: dx = 0.1, dt = 0.02 dx^2, trap (1, 1.5, 2), initial
Thomas-Fermi profile of g = 100 times a random phase of sigma 0.05 (seed 1),
propagated with g = 80.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1605_03958_amd import inputs  # noqa: E402

N = 256
DX = 0.1
STEPS = 1000
NSAMPLE = 4096
SAMPLE_SEED = 12345


def line_sums(psi: np.ndarray) -> dict:
    """Line sums of a (nz, ny, nx) state; the GPU parity test applies this
    same definition to the GPU's state."""
    a = np.asarray(psi, dtype=np.complex128)
    nx = a.shape[2]
    w = (np.arange(nx, dtype=np.float64) + 1.0) / nx
    return {
        "x_sum": a.sum(axis=2).reshape(-1),
        "x_wsum": (a * w[None, None, :]).sum(axis=2).reshape(-1),
        "y_sum": a.sum(axis=1).reshape(-1),
        "z_sum": a.sum(axis=0).reshape(-1),
    }


def main(out=os.path.join(HERE, "cube256_oracle_1000.json"),
         out_lines=os.path.join(HERE, "cube256_oracle_1000_lines.npz")):
    n = (N, N, N)
    om = (1.0, 1.5, 2.0)
    prob = oracle.Problem(3, n, (DX,) * 3, om, 80.0, 0.02 * DX * DX, oracle.REAL, 0)
    psi0 = inputs.thomas_fermi(3, n, (DX,) * 3, om, 100.0, phase_sigma=0.05, seed=1)
    o0 = oracle.observe(prob, psi0)
    t0 = time.time()
    r = oracle.run(prob, psi0, STEPS)
    el = time.time() - t0
    o1 = oracle.observe(prob, r.psi)
    idx = np.random.default_rng(SAMPLE_SEED).choice(N ** 3, size=NSAMPLE, replace=False)
    idx.sort()
    flat = r.psi.reshape(-1)
    rec = {
        "workload": "real-time 3D SSCN 256^3, dx=0.1, dt=0.02*dx^2, trap (1,1.5,2), TF(g=100) x phase "
                    "sigma 0.05 seed 1, g=80",
        "steps": STEPS,
        "oracle_seconds": el,
        "oracle_threads": oracle.threads(),
        "obs0": {k: getattr(o0, k) for k in ("norm", "mu", "energy", "K", "P", "I")},
        "obs1": {k: getattr(o1, k) for k in ("norm", "mu", "energy", "K", "P", "I")},
        "sample_seed": SAMPLE_SEED,
        "sample_index": idx.tolist(),
        "sample_re": flat[idx].real.tolist(),
        "sample_im": flat[idx].imag.tolist(),
        "l2sq": float(np.sum(np.abs(flat) ** 2)),
    }
    with open(out, "w") as f:
        json.dump(rec, f)
    np.savez(out_lines, **line_sums(r.psi))
    print(f"wrote {out} and {out_lines} ({el:.0f} s)")


if __name__ == "__main__":
    main()
