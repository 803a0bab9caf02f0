"""CPU bounds check of the persistent batch kernel's index arithmetic.

The x-line (ROW) and y/z-line (COL) items of k_batch_step compute every
state, table and LDS index from the instance geometry the planner reports
(sscn_batch_plan_info) and the block shape (1024 threads, 64 KB of dynamic
LDS).  This test re-evaluates those index formulas for every thread of a
block, for every 1D line length up to 16384 points in both modes (float and
complex<float>) and for 2D and 3D shapes of the batch mix, and checks that
each access stays inside its buffer and that the items cover every line of
an instance exactly once.  It runs on the host: no kernel is launched."""
import numpy as np
import pytest

from paper_1605_03958_amd import sscn
from paper_1605_03958_amd.sscn import F32, IMAG, REAL, Problem

BLOCK = 1024          # threads per persistent block
LDS = 64 * 1024       # dynamic LDS bytes per block
pytestmark = pytest.mark.filterwarnings("ignore")


def _vbytes(mode):
    return 4 if mode == IMAG else 8            # float / complex<float>


def _ltab(mode):
    return 16 if mode == IMAG else 32           # staged (alpha, m) hi/lo pairs


def _check_row_threads(C, wpl, mode):
    """Per-thread ROW indices of one block (batch_row / row_solve)."""
    S = _vbytes(mode)
    G = 64 * wpl
    lpb = 16 // wpl
    assert lpb * wpl == 16
    tid = np.arange(BLOCK)
    lb, t = tid // G, tid % G
    wl = t >> 6
    assert lb.max() < lpb and wl.max() < wpl
    k = np.arange(C)[:, None]
    slots = k * G + t[None, :]                  # lane-major table slot of chunk point k
    assert slots.min() >= 0 and slots.max() < C * 64 * wpl
    if wpl > 1:
        xs = lb * wpl * 4 + wl * 4               # 4 exchange values per wave of each line group
        assert (xs + 3).max() < 16 * 4
        assert 16 * 4 * S <= LDS
    else:
        assert C * 64 * _ltab(mode) <= LDS       # table staged in LDS
    return G, lpb


def _check_lines_covered(nlines, ntiles, rep, per_set, line_of):
    """Items (tile, r) and their slots cover [0, nlines) exactly once."""
    seen = np.zeros(nlines, dtype=np.int64)
    for tile in range(ntiles):
        for r in range(rep):
            lines = line_of(tile, r)
            lines = lines[lines < nlines]
            np.add.at(seen, lines, 1)
    assert np.all(seen == 1)


@pytest.mark.parametrize("mode", [IMAG, REAL])
def test_row_items_of_every_1d_line_length(mode):
    """Every 1D line of 1..16384 points: the chunk covers the line, the
    table and LDS indices of every thread stay inside their buffers (the
    multi-wave form's 4 exchange slots per wave included)."""
    seen_geom = set()
    for n in range(1, 16385):
        p = Problem(1, (n, 1, 1), (0.05,), (1.0,), 5.0, 1e-4, mode, F32, 1 if mode == IMAG else 0, 10)
        x = sscn.batch_plan_info(p)[0]
        assert x["kind"] == "row"
        C, wpl = x["chunk"], x["waves"]
        assert wpl in (1, 2, 4, 8, 16)
        assert C * 64 * wpl >= n                 # thread t holds points t*C .. t*C+C-1
        assert (C * 64 * (wpl // 2) < n) if wpl > 1 else True
        if (C, wpl) not in seen_geom:
            seen_geom.add((C, wpl))
            _check_row_threads(C, wpl, mode)
        assert x["items"] == 1                   # a 1D instance has one line
    assert len(seen_geom) >= 6


SHAPES = [(2, (256, 256, 1)), (2, (300, 517, 1)), (2, (1015, 1015, 1)), (2, (1024, 1024, 1)),
          (3, (48, 48, 48)), (3, (61, 77, 50)), (3, (159, 159, 159)), (3, (160, 160, 160)),
          (3, (100, 33, 129))]


@pytest.mark.parametrize("mode", [IMAG, REAL])
@pytest.mark.parametrize("dim,n", SHAPES)
def test_items_of_2d_and_3d_instances(dim, n, mode):
    """x items (ROW) and y/z items (COL) of mix-sized instances: every
    index inside its buffer and every line of every pass covered once."""
    p = Problem(dim, n, (0.1,) * dim, (1.0, 1.5, 2.0)[:dim], 5.0, 1e-4, mode, F32, 1 if mode == IMAG else 0, 10)
    info = sscn.batch_plan_info(p)
    npts = n[0] * n[1] * n[2]
    S = _vbytes(mode)
    for a in range(dim):
        g = info[a]
        nl = npts // n[a]
        C, rep, ntiles = g["chunk"], g["rep"], g["items"]
        if g["kind"] == "row":
            wpl = g["waves"]
            assert C * 64 * wpl >= n[a]
            G, lpb = _check_row_threads(C, wpl, mode)
            lb = np.arange(BLOCK) // G
            _check_lines_covered(nl, ntiles, rep, lpb,
                                 lambda tile, r: np.unique(tile * rep * lpb + lb + r * lpb))
        else:
            W, L = g["waves"], g["lanes"]
            assert W in (1, 2, 4, 8, 16) and L in (1, 2, 4, 8)
            nch, LPB, tpi = W * L, 64 // L, 16 // W
            assert nch * C >= n[a]                            # chunks cover the line
            assert W * L * C * _ltab(mode) + tpi * 2 * W * 64 * S <= LDS
            tid = np.arange(BLOCK)
            wave, lane = tid >> 6, tid & 63
            st_i, w = wave // W, wave % W
            sub, li = lane // LPB, lane % LPB
            ch = w * L + sub
            assert st_i.max() < tpi and ch.max() < nch and li.max() < LPB
            # exchange slots: this sub-tile's two arrays of nch x LPB values
            # after the staged table
            tab_bytes = nch * C * _ltab(mode)
            off = tab_bytes + (st_i * 2 * nch * LPB + nch * LPB + ch * LPB + li) * S
            assert off.max() + S <= LDS
            assert (ch[None, :] * C + np.arange(C)[:, None]).max() < nch * C   # table entries
            _check_lines_covered(nl, ntiles, rep, tpi * LPB,
                                 lambda tile, r: np.unique(((tile * rep + r) * tpi + st_i) * LPB + li))
            # state: line l starts at (l % m1) s1 + (l / m1) s2, points stride apart
            m1 = n[0]
            stride = n[0] if a == 1 else n[0] * n[1]
            s1, s2 = 1, (n[0] * n[1] if a == 1 else n[0])
            lines = np.arange(nl)
            base = (lines % m1) * s1 + (lines // m1) * s2
            assert base.max() + (n[a] - 1) * stride < npts
