"""The tile autotuner on the GPU: the tuned choice is never slower than the
default as measured, and results with the tuned tiles still match the
oracle."""
import numpy as np
import pytest

import oracle
from paper_1605_03958_amd import autotune, inputs, sscn
from paper_1605_03958_amd.sscn import F32, IMAG, Problem

pytestmark = pytest.mark.gpu


def test_tune_batch_and_single(tmp_path):
    path = str(tmp_path / "tiles.json")
    p = Problem(3, (60, 52, 44), (0.2, 0.2, 0.2), (1.0, 1.5, 2.0), 10.0, 0.004, IMAG, F32, 1, 10)
    for target in ("batch", "single"):
        rec = autotune.tune(p, target, cache_path=path, reps=1, log=lambda s: print(s, flush=True))
        print(target, rec["chunks"], rec["ms"], rec["default_ms"], flush=True)
        assert rec["ms"] <= rec["default_ms"] and len(rec["tried"]) >= 5
    psi0 = inputs.ho_gaussian(3, p.n, p.dx, p.omega, noise=1e-3, seed=4)
    ref = oracle.run(oracle.Problem(p.dim, p.n, p.dx, p.omega, p.g, p.dt, p.mode, p.renorm_every), psi0, 20).psi
    try:
        assert autotune.apply(p, "batch", cache_path=path) or True
        b = sscn.Batch(1)
        b.admit(0, p, psi0, mu_tol=0.0, max_steps=20)
        b.step(20)
        b.poll()
        got = b.evict(0).cpu().numpy()
        b.close()
        autotune.apply(p, "single", cache_path=path)
        s = sscn.Solver(p, psi0)
        s.step(20)
        single = s.state()
        s.close()
    finally:
        sscn.batch_clear_tile_hints()
        sscn.clear_tile_hints()
    for g in (got, single):
        err = np.linalg.norm((g.astype(np.complex128) - ref).ravel()) / np.linalg.norm(ref.ravel())
        assert err <= 5e-5, err
