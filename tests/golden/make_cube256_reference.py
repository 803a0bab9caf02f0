"""Write tests/golden/cube256_oracle_1000.json: the FP64 CPU oracle's result for
the 256^3 real-time workload after 1000 steps (observables before and after,
and the state at a seeded sample of grid points).

Calls only the oracle and the seeded input generator.  Takes about 15 min on
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


def main(out=os.path.join(HERE, "cube256_oracle_1000.json")):
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
    print(f"wrote {out} ({el:.0f} s)")


if __name__ == "__main__":
    main()
