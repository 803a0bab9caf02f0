"""Tile autotuner search and cache logic with a stand-in cost (CPU); the
hints it sets are the library's own (validated by the library)."""
import json

import pytest

from paper_1605_03958_amd import autotune, sscn
from paper_1605_03958_amd.sscn import F32, F64, IMAG, REAL, Problem


def prob(mode=IMAG, prec=F32, n=(48, 40, 36)):
    return Problem(3, n, (0.1, 0.1, 0.1), (1.0, 1.5, 2.0), 5.0, 1e-3, mode, prec, 1 if mode == IMAG else 0, 10)


def fake_cost(best):
    """Cost with a unique minimum at `best` per axis (0 = default costs 5)."""
    calls = []

    def measure(p, chunks):
        calls.append(tuple(chunks))
        return 10.0 + sum(5.0 if c == 0 else abs(c - b) for c, b in zip(chunks, best))
    return measure, calls


@pytest.mark.parametrize("target,best", [("batch", [3, 10, 5]), ("single", [2, 8, 4])])
def test_search_finds_the_minimum_and_caches_it(tmp_path, target, best):
    path = str(tmp_path / "tiles.json")
    p = prob()
    meas, calls = fake_cost(best)
    rec = autotune.tune(p, target, cache_path=path, measure=meas, reps=1, arch="gfx950")
    assert rec["chunks"] == best and rec["ms"] == 10.0 and rec["default_ms"] == 25.0
    assert calls[0] == (0, 0, 0)                   # the default is measured first
    n = len(calls)
    with open(path) as f:
        cache = json.load(f)
    assert list(cache) == [autotune.cache_key(target, p, "gfx950")]
    # cached: no measurement the second time
    rec2 = autotune.tune(p, target, cache_path=path, measure=meas, reps=1, arch="gfx950")
    assert rec2 == rec and len(calls) == n
    # hints are cleared after tuning; apply() sets the cached one
    info = sscn.batch_plan_info if target == "batch" else sscn.plan_info
    before = info(p)
    try:
        assert autotune.apply(p, target, cache_path=path, arch="gfx950")
        after = info(p)
        assert [after[a]["chunk"] for a in range(3)] == best
    finally:
        sscn.batch_clear_tile_hints()
        sscn.clear_tile_hints()
    assert info(p) == before
    assert not autotune.apply(prob(n=(50, 40, 36)), target, cache_path=path, arch="gfx950")


def test_unsettable_candidates_are_skipped(tmp_path):
    p = prob(mode=REAL)
    meas, calls = fake_cost([4, 12, 12])             # 12 is not a complex chunk: never measured
    rec = autotune.tune(p, "batch", cache_path=None, measure=meas, reps=1, arch="gfx950")
    assert all(12 not in c for c in calls)
    assert rec["chunks"] == [4, 8, 8]               # the closest complex chunks


def test_batch_target_needs_fp32():
    with pytest.raises(ValueError):
        autotune.tune(prob(prec=F64), "batch", measure=lambda p, c: 1.0, arch="gfx950")
