"""CPU bounds check of the single-problem sweep kernels' index arithmetic.

For every plan the planner reports (sscn_plan_info) on a range of shapes --
x lines over 16 or 64 lanes and several waves, column sweeps with 1 to 8
lanes per line including lines longer than 2048 points -- this test
re-evaluates the index formulas of k_row and k_col for every thread of a
block and checks that each table slot, exchange slot, LDS byte and state
index stays inside its buffer, that every point of a line is held by one
thread, and that the blocks cover every line once.  It also checks the norm
partials the next x sweep reads when it forms the renormalisation factor
(at most 256).  No kernel is launched."""
import numpy as np
import pytest

from paper_1605_03958_amd import sscn
from paper_1605_03958_amd.sscn import F32, F64, IMAG, REAL, Problem

LDS_MAX = 160 * 1024 - 1024        # a COL block's dynamic LDS at most


def _sizes(mode, prec):
    S = {(IMAG, F64): 8, (REAL, F64): 16, (IMAG, F32): 4, (REAL, F32): 8}[(mode, prec)]
    ltab = {(IMAG, F64): 16, (REAL, F64): 32, (IMAG, F32): 16, (REAL, F32): 32}[(mode, prec)]
    return S, ltab


def _check_row(q, n, nlines, S, ltab):
    C, wpl, seg = q["chunk"], q["waves"], q["lanes"]
    block, grid = q["block"], q["grid"]
    assert seg in (16, 64) and (seg == 64 or wpl == 1)
    G = 64 * wpl if seg == 64 else seg
    lpb = block // G
    assert lpb * G == block and block == 64 * wpl * max(1, 4 // wpl)
    assert C * G >= n                                   # thread t holds points t*C .. t*C+C-1
    tid = np.arange(block)
    lb, t = tid // G, tid % G
    slots = np.arange(C)[:, None] * G + t[None, :]      # lane-major table slots
    assert slots.max() < C * G
    if wpl == 1:
        tab = C * G * ltab
        if seg == 64 and S >= 16 and tab + lpb * (C * 64 + 64) * S <= 65536:
            # per-wave regrouping buffer after the table (row_load_tr)
            e = np.arange(C)[:, None] * 64 + (tid & 63)[None, :]
            buf = lb * (C * 64 + 64) + e + e // C
            assert tab + (buf.max() + 1) * S <= 65536
    else:
        assert (lb * wpl * 4 + (t >> 6) * 4 + 3).max() < lpb * wpl * 4
    # grid-stride over line groups: every line once
    seen = np.zeros(nlines, dtype=np.int64)
    for b in range(grid):
        gb = b * lpb
        while gb < nlines:
            lines = gb + np.arange(lpb)
            np.add.at(seen, lines[lines < nlines], 1)
            gb += grid * lpb
    assert np.all(seen == 1)


def _check_col(q, n, nlines, npts, stride, m1, s1, s2, S, ltab):
    C, W, L, grid, block = q["chunk"], q["waves"], q["lanes"], q["grid"], q["block"]
    assert L in (1, 2, 4, 8) and 1 <= W <= 16 and block == 64 * W
    nch, LPB = W * L, 64 // L
    assert nch * C >= n
    assert W * L * C * ltab + 2 * W * 64 * S <= LDS_MAX
    tid = np.arange(block)
    lane, w = tid & 63, tid >> 6
    sub, li = lane // LPB, lane % LPB
    ch = w * L + sub
    assert ch.max() < nch and li.max() < LPB
    assert (ch * LPB + li).max() < nch * LPB            # exchange slots
    assert (ch[None, :] * C + np.arange(C)[:, None]).max() < nch * C
    lines = (np.arange(grid)[:, None] * LPB + li[None, :]).ravel()
    covered = np.unique(lines[lines < nlines])
    assert covered.size == nlines and grid == -(-nlines // LPB)
    base = (covered % m1) * s1 + (covered // m1) * s2
    assert base.max() + (n - 1) * stride < npts


SHAPES = [(1, (64, 1, 1)), (1, (5000, 1, 1)), (1, (16384, 1, 1)),
          (2, (1, 7, 1)), (2, (37, 20, 1)), (2, (64, 700, 1)), (2, (32, 2000, 1)), (2, (16, 3000, 1)),
          (2, (16, 4096, 1)), (2, (8, 6000, 1)), (2, (8, 8192, 1)), (2, (1024, 1024, 1)),
          (3, (5, 3, 2)), (3, (48, 40, 9)), (3, (64, 64, 64)), (3, (65, 70, 33)), (3, (96, 96, 96)),
          (3, (128, 128, 128)), (3, (256, 256, 256)), (3, (16, 16, 3000))]


@pytest.mark.parametrize("mode,prec", [(IMAG, F64), (REAL, F64), (IMAG, F32), (REAL, F32)])
@pytest.mark.parametrize("dim,n", SHAPES)
def test_single_problem_plans_stay_in_bounds(dim, n, mode, prec):
    p = Problem(dim, n, (0.1,) * dim, (1.0, 1.5, 2.0)[:dim], 5.0, 1e-4, mode, prec, 1 if mode == IMAG else 0)
    info = sscn.plan_info(p)
    npts = n[0] * n[1] * n[2]
    S, ltab = _sizes(mode, prec)
    for a in range(dim):
        q = info[a]
        nl = npts // n[a]
        if q["kind"] == "row":
            _check_row(q, n[a], nl, S, ltab)
        elif q["kind"] == "col":
            stride = n[0] if a == 1 else n[0] * n[1]
            s2 = n[0] * n[1] if a == 1 else n[0]
            _check_col(q, n[a], nl, npts, stride, n[0], 1, s2, S, ltab)
        else:
            assert q["kind"] == "stream"
    # the renormalisation factor formed in the x sweep reads the last
    # sweep's partials w*64 + lane for w < 4 only when there are at most 256
    last = info[dim - 1]
    if mode == IMAG and dim >= 2 and info[0]["kind"] == "row" and info[0]["lanes"] == 16 and last["kind"] == "col":
        if last["grid"] <= 256:
            w, lane = np.meshgrid(np.arange(4), np.arange(64))
            idx = (w * 64 + lane)[(w * 64 + lane) < last["grid"]]
            assert idx.size == last["grid"] and idx.max() < last["grid"]
