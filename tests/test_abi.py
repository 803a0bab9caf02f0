"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/sscn.h declares, validates problems before any side
effect, sizes the state and workspace, and plans kernel geometries."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1605_03958_amd import sscn
from paper_1605_03958_amd.sscn import Problem, IMAG, REAL, F64, F32

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sscn_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = sscn.lib()
    names = _declared("sscn.h")
    assert "sscn_create" in names and "sscn_step" in names
    for name in names:
        assert hasattr(L, name), name
    # and the binding declares a signature for each of them
    missing = [n for n in names if n not in sscn.EXPORTS]
    assert not missing, missing


def test_abi_version_and_status_strings():
    L = sscn.lib()
    assert L.sscn_abi_version() == 2
    for code in (0, 1, -1, -2, -3, -4, -5, 99):
        assert isinstance(sscn.status_string(code), str) and sscn.status_string(code)


def _good():
    return Problem(3, (8, 6, 5), (0.2, 0.2, 0.2), (1, 1.5, 2), 22.0, 0.004, IMAG, F64, 1, 10)


@pytest.mark.parametrize("field,value", [
    ("dim", 0), ("dim", 4), ("n", (0, 6, 5)), ("dx", (0.0, 0.2, 0.2)), ("dx", (float("nan"), 0.2, 0.2)),
    ("omega", (-1.0, 1, 1)), ("omega", (float("inf"), 1, 1)), ("g", float("nan")), ("dt", 0.0),
    ("dt", -1.0), ("mode", 2), ("prec", 5), ("renorm_every", 0), ("observe_every", -1),
])
def test_validate_rejects(field, value):
    p = _good()
    setattr(p, field, value)
    p.__post_init__()
    assert sscn.validate(p) == sscn.E_INVALID


def test_validate_unused_axis_and_real_renorm():
    p = Problem(2, (8, 6, 2), (0.2, 0.2, 1), (1, 1, 0), 1.0, 0.01, IMAG, F64, 1)
    assert sscn.validate(p) == sscn.E_INVALID        # n_z must be 1 in 2D
    p = Problem(2, (8, 6, 1), (0.2, 0.2, 1), (1, 1, 0), 1.0, 0.01, REAL, F64, 1)
    assert sscn.validate(p) == sscn.E_INVALID        # no renormalisation in real time
    p.renorm_every = 0
    assert sscn.validate(p) == sscn.OK
    huge = Problem(3, (20000, 20000, 20000), (0.1,) * 3, (1, 1, 1), 1.0, 0.01, IMAG, F64, 1)
    assert sscn.validate(huge) == sscn.E_UNSUPPORTED


def test_state_bytes_by_dtype():
    for mode, prec, size in ((IMAG, F64, 8), (IMAG, F32, 4), (REAL, F64, 16), (REAL, F32, 8)):
        p = Problem(3, (7, 5, 3), (0.2,) * 3, (1, 1, 1), 1.0, 0.01, mode, prec, 1 if mode == IMAG else 0)
        assert sscn.state_bytes(p) == 7 * 5 * 3 * size
        assert sscn.workspace_bytes(p) % 256 == 0 and sscn.workspace_bytes(p) > 0


def test_null_arguments_rejected_without_side_effects():
    L = sscn.lib()
    pc = _good().c()
    h = ctypes.c_void_p(0)
    assert L.sscn_create(ctypes.byref(pc), None, None, None, ctypes.byref(h)) == sscn.E_INVALID
    assert h.value is None
    assert L.sscn_create(ctypes.byref(pc), ctypes.c_void_p(256), ctypes.c_void_p(260), None,
                         ctypes.byref(h)) == sscn.E_INVALID   # misaligned workspace
    assert L.sscn_step(None, 1) == sscn.E_INVALID
    assert L.sscn_set_g(None, 1.0) == sscn.E_INVALID
    assert L.sscn_destroy(None) == sscn.E_INVALID
    assert L.sscn_validate(None) == sscn.E_INVALID


def test_plan_geometries():
    # 256^3 complex128: x lines in registers (4 points per lane), y/z 16 x 16
    p = Problem(3, (256, 256, 256), (0.1,) * 3, (1, 1.5, 2), 80.0, 2e-4, REAL, F64, 0)
    info = sscn.plan_info(p)
    assert info[0]["kind"] == "row" and info[0]["chunk"] == 4 and info[0]["waves"] == 1
    assert info[1]["kind"] == "col" and info[1]["chunk"] * info[1]["waves"] * info[1]["lanes"] >= 256
    assert info[1]["chunk"] == 4 and info[1]["lanes"] == 4
    assert info[2]["kind"] == "col"
    # long x lines use several waves per line; too long falls back
    p = Problem(1, (5000, 1, 1), (0.1,), (1,), 1.0, 1e-3, IMAG, F64, 1)
    info = sscn.plan_info(p)
    assert info[0]["kind"] == "row" and info[0]["waves"] == 8
    assert info[1] is None
    p = Problem(1, (300000, 1, 1), (0.1,), (1,), 1.0, 1e-3, IMAG, F64, 1)
    assert sscn.plan_info(p)[0]["kind"] == "stream"
    # x lines of at most 64 points: chunks of 4 over 16 lanes, four lines
    # per wave (16 per 256-thread block), scans of at most 4 steps
    for nx in (1, 5, 63, 64):
        for prec in (F64, F32):
            for mode in (IMAG, REAL):
                p = Problem(3, (nx, 64, 64), (0.2,) * 3, (1, 1.5, 2), 22.0, 0.004, mode, prec, 1 if mode == IMAG else 0)
                q = sscn.plan_info(p)[0]
                assert (q["kind"], q["chunk"], q["lanes"], q["block"]) == ("row", 4, 16, 256), (nx, prec, mode)
                assert q["grid"] == 64 * 64 // 16 and q["depth"] <= 4
    p = Problem(3, (65, 64, 64), (0.2,) * 3, (1, 1.5, 2), 22.0, 0.004, IMAG, F64, 1)
    q = sscn.plan_info(p)[0]
    assert (q["chunk"], q["lanes"]) == (2, 64)
    # a tile hint of another chunk length keeps 64 lanes per line
    p = Problem(3, (64, 64, 64), (0.2,) * 3, (1, 1.5, 2), 22.0, 0.004, IMAG, F64, 1)
    try:
        sscn.set_tile_hint(p, (1, 0, 0))
        q = sscn.plan_info(p)[0]
        assert (q["chunk"], q["lanes"], q["grid"]) == (1, 64, 64 * 64 // 4)
    finally:
        sscn.clear_tile_hints()
    # (complex128: up to 8 lanes, a 128-byte row segment, when the sweep
    # would launch fewer than 256 blocks)
    p = Problem(2, (64, 700, 1), (0.1, 0.1), (1, 1), 1.0, 1e-3, REAL, F64, 0)
    assert sscn.plan_info(p)[1]["kind"] == "col" and sscn.plan_info(p)[1]["lanes"] == 8
    assert sscn.plan_info(p)[1]["chunk"] == 8 and sscn.plan_info(p)[1]["grid"] == 8
    p = Problem(2, (64, 5000, 1), (0.1, 0.1), (1, 1), 1.0, 1e-3, REAL, F64, 0)
    assert sscn.plan_info(p)[1]["kind"] == "stream"


@pytest.mark.parametrize("prec", [F64, F32])
def test_small_grid_column_sweeps_take_more_lanes(prec):
    # a y/z sweep of fewer than 256 blocks takes more lanes per line (up to
    # 4 for 8-byte values, 2 for 4-byte ones) so that it launches more blocks
    lmax = 4 if prec == F64 else 2
    p = Problem(3, (64, 64, 64), (0.2,) * 3, (1, 1.5, 2), 22.0, 0.004, IMAG, prec, 1)
    for q in sscn.plan_info(p)[1:]:
        assert q["kind"] == "col" and q["lanes"] == lmax
        assert q["grid"] == 64 * 64 // (64 // lmax)
        assert q["chunk"] * q["waves"] * q["lanes"] >= 64
    # a sweep that already has 256 blocks keeps the lanes its line length
    # asks for (128 points: 32 chunks of 4 over 16 waves, 2 lanes)
    p = Problem(3, (128, 128, 128), (0.2,) * 3, (1, 1.5, 2), 22.0, 0.004, IMAG, prec, 1)
    for q in sscn.plan_info(p)[1:]:
        assert (q["chunk"], q["waves"], q["lanes"], q["grid"]) == (4, 16, 2, 512)
    # never more lanes than chunks: a short line keeps covering itself
    p = Problem(2, (40, 6, 1), (0.2, 0.2), (1, 1.5), 1.0, 0.004, IMAG, prec, 1)
    q = sscn.plan_info(p)[1]
    assert q["kind"] == "col" and q["lanes"] <= max(1, -(-6 // q["chunk"]))
    assert q["chunk"] * q["waves"] * q["lanes"] >= 6


def test_tile_hints_change_the_plan():
    p = Problem(3, (64, 64, 64), (0.2,) * 3, (1, 1.5, 2), 22.0, 0.004, IMAG, F64, 1)
    try:
        sscn.set_tile_hint(p, (2, 8, 16))
        info = sscn.plan_info(p)
        assert info[0]["chunk"] == 2 and info[1]["chunk"] == 8 and info[2]["chunk"] == 16
        assert info[1]["waves"] * info[1]["lanes"] == 8 and info[2]["waves"] * info[2]["lanes"] == 4
        with pytest.raises(sscn.SSCNError):
            sscn.set_tile_hint(p, (3, 0, 0))
    finally:
        sscn.clear_tile_hints()
    assert sscn.plan_info(p)[1]["chunk"] == 4


@pytest.mark.parametrize("sigma", [0.005, 0.025, 0.3, 10.0])
@pytest.mark.parametrize("mode", [IMAG, REAL])
def test_scan_depth_bounds_neglected_terms(sigma, mode):
    """The scan depth chosen by the plan is the smallest that keeps every
    neglected term below 2^-64 of the largest (FP64): a term from k chunks
    back carries a product of k chunk factors prod |alpha|."""
    import numpy as np
    n = 256
    dx = 0.1
    dt = sigma * 4 * dx * dx
    p = Problem(2, (n, n, 1), (dx, dx), (1, 1), 1.0, dt, mode, F64, 1 if mode == IMAG else 0)
    info = sscn.plan_info(p)
    s = sigma if mode == IMAG else 1j * sigma
    m = np.zeros(n, dtype=complex)
    m[0] = 1 / (1 + 2 * s)
    for i in range(1, n):
        m[i] = 1 / (1 + 2 * s - s * s * m[i - 1])
    al = np.abs(s * m)
    for ax in (0, 1):
        C = info[ax]["chunk"]
        amax = max(np.prod(al[c:c + C]) for c in range(0, n - C + 1, C))
        covered = (2 ** info[ax]["depth"]) if info[ax]["kind"] == "row" else info[ax]["depth"]
        nchunks = -(-n // C)
        if covered < nchunks - 1:
            assert amax ** covered <= 2.0 ** -64
            assert amax ** (covered // 2 if info[ax]["kind"] == "row" else covered - 1) > 2.0 ** -64 or covered == 1
        # the tail the kernels read as one constant is constant to round-off
        ic = info[ax]["i_conv"]
        assert np.all(np.abs(m[ic:] - m[-1]) <= 4e-16 * abs(m[-1]))


def test_batch_sizes_and_validation():
    assert sscn.batch_ctl_bytes(64, 100000) >= 100000 * 8
    with pytest.raises(sscn.SSCNError):
        sscn.batch_ctl_bytes(0, 10)
    p = Problem(3, (64, 48, 40), (0.2,) * 3, (1, 1.5, 2), 10.0, 0.004, IMAG, F32, 1, 10)
    assert sscn.batch_workspace_bytes(p) % 256 == 0
    with pytest.raises(sscn.SSCNError) as e:   # the batch runs the FP32 forms only
        sscn.batch_workspace_bytes(Problem(3, (8, 8, 8), (0.2,) * 3, (1, 1, 1), 1.0, 0.004, IMAG, F64, 1, 10))
    assert e.value.code == sscn.E_UNSUPPORTED
    with pytest.raises(sscn.SSCNError) as e:   # observation interval needed
        sscn.batch_workspace_bytes(Problem(1, (64, 1, 1), (0.2,), (1,), 1.0, 0.004, IMAG, F32, 1, 0))
    assert e.value.code == sscn.E_INVALID
    # uneven sizes of the batch mix all fit the persistent tiles
    from paper_1605_03958_amd import inputs
    for i in range(64):
        d = inputs.batch_draw(i)
        for mode in (IMAG, REAL):
            q = Problem(d.dim, d.n, d.dx, d.omega, d.g, 0.1 * d.dx[0] ** 2, mode, F32,
                        1 if mode == IMAG else 0, 10)
            assert sscn.batch_workspace_bytes(q) > 0


def test_one_hip_runtime_in_the_process():
    """Loading the library before anything imports torch must not bring a
    second HIP runtime into the process (torch's tensors and streams belong
    to torch's runtime)."""
    import subprocess
    import sys
    code = ("from paper_1605_03958_amd import sscn\n"
            "sscn.lib()\n"
            "import torch\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


ROW_CHUNKS = {False: [1, 2, 3, 4, 6, 8, 12, 16], True: [1, 2, 3, 4, 6, 8]}
COL_CHUNKS = {False: [2, 3, 4, 5, 6, 8, 10, 12, 16], True: [2, 3, 4, 5, 6, 8]}


@pytest.mark.parametrize("dim,n", [(3, (152, 152, 152)), (3, (48, 49, 50)), (3, (17, 160, 3)), (2, (919, 919, 1)),
                                   (2, (267, 1024, 1)), (2, (64, 2048, 1)), (1, (9912, 1, 1)), (1, (700, 1, 1))])
@pytest.mark.parametrize("mode", [sscn.IMAG, sscn.REAL])
def test_batch_geometry_covers_lines(dim, n, mode):
    cplx = mode == sscn.REAL
    p = sscn.Problem(dim, n, (0.1,) * dim, (1.0, 1.5, 2.0)[:dim], 5.0, 1e-3, mode, sscn.F32,
                     1 if mode == sscn.IMAG else 0, 10)
    if cplx and dim == 2 and n[1] > 1024:
        with pytest.raises(sscn.SSCNError):
            sscn.batch_plan_info(p)
        return
    info = sscn.batch_plan_info(p)
    for a in range(3):
        g = info[a]
        if a >= dim:
            assert g is None
            continue
        if g["kind"] == "row":
            assert g["chunk"] * 64 * g["waves"] >= n[a]
            if g["waves"] == 1:
                assert g["chunk"] in ROW_CHUNKS[cplx]
                assert (g["chunk"] - 1) * 64 < n[a] or g["chunk"] == 1 or ROW_CHUNKS[cplx].index(g["chunk"]) == 0 \
                    or ROW_CHUNKS[cplx][ROW_CHUNKS[cplx].index(g["chunk"]) - 1] * 64 < n[a]
        else:
            assert a > 0 and g["chunk"] in COL_CHUNKS[cplx]
            assert g["chunk"] * g["waves"] * g["lanes"] >= n[a]
            assert 16 % g["waves"] == 0 and g["lanes"] in (1, 2, 4, 8)
        assert g["items"] >= 1 and g["rep"] >= 1
    # a 1D instance whose line fits one block runs its whole step as one item
    if dim == 1:
        assert info[0]["items"] == 1


def test_batch_tile_hints():
    p = sscn.Problem(3, (40, 44, 36), (0.1,) * 3, (1.0, 1.5, 2.0), 5.0, 1e-3, sscn.IMAG, sscn.F32, 1, 10)
    q = sscn.Problem(3, (40, 44, 37), (0.1,) * 3, (1.0, 1.5, 2.0), 5.0, 1e-3, sscn.IMAG, sscn.F32, 1, 10)
    base = sscn.batch_plan_info(p)
    qbase = sscn.batch_plan_info(q)

    def geo(g):
        return {k: v for k, v in g.items() if k != "big"}
    try:
        sscn.batch_set_tile_hint(p, (2, 3, 12))
        h = sscn.batch_plan_info(p)
        assert [h[0]["chunk"], h[1]["chunk"], h[2]["chunk"]] == [2, 3, 12]
        # x lines of 2D and 3D instances take at most 4 points per thread in
        # one wave: a larger hint is accepted but not taken
        sscn.batch_set_tile_hint(p, (6, 3, 12))
        assert sscn.batch_plan_info(p)[0] == base[0]
        assert h[1]["chunk"] * h[1]["waves"] * h[1]["lanes"] >= 44
        assert sscn.batch_plan_info(q) == qbase      # other shapes untouched
        sscn.batch_set_tile_hint(p, (0, 16, 0))
        h = sscn.batch_plan_info(p)
        assert h[1]["chunk"] == 16 and h[1]["big"]
        assert geo(h[0]) == geo(base[0]) and geo(h[2]) == geo(base[2])
        for bad in ((5, 0, 0), (0, 7, 0), (0, 0, 32), (-1, 0, 0)):
            with pytest.raises(sscn.SSCNError) as e:
                sscn.batch_set_tile_hint(p, bad)
            assert e.value.code == sscn.E_INVALID
        r = sscn.Problem(3, (40, 44, 36), (0.1,) * 3, (1.0, 1.5, 2.0), 5.0, 1e-3, sscn.REAL, sscn.F32, 0, 10)
        with pytest.raises(sscn.SSCNError):
            sscn.batch_set_tile_hint(r, (12, 0, 0))      # complex lines take at most 8 per thread
        d2 = sscn.Problem(2, (40, 44, 1), (0.1,) * 2, (1.0, 1.5), 5.0, 1e-3, sscn.IMAG, sscn.F32, 1, 10)
        with pytest.raises(sscn.SSCNError):
            sscn.batch_set_tile_hint(d2, (0, 0, 4))      # no z axis
    finally:
        sscn.batch_clear_tile_hints()
    assert sscn.batch_plan_info(p) == base


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus above 1 exits with a message before
    touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 2 and "one GPU" in out.stderr and out.stdout == ""


def test_dynamics_pipeline_host_checks():
    # argument checks happen before any device work; rms from the moments
    from paper_1605_03958_amd import dynamics
    p = Problem(1, (64,), (0.1,), (1.0,), 1.0, 1e-3, REAL, F64, 0, 1)
    with pytest.raises(ValueError):
        dynamics.ground_state_then_dynamics(p, np.zeros(64), 0.5, 10, 1e-3)
    q = Problem(1, (64,), (0.1,), (1.0,), 1.0, 1e-3, IMAG, F64, 1, 10)
    with pytest.raises(ValueError):
        dynamics.ground_state_then_dynamics(q, np.zeros(64), 0.5, -1, 1e-3)
    o = sscn.Obs(0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, (0.0, 0.0, 0.0), (4.0, 9.0, 0.0))
    assert dynamics.rms_sizes(o, 2) == (2.0, 3.0, math.sqrt(13.0))


def test_symmetric_trap_validation_and_plan():
    """Circular and spherical traps store one radial axis, the axial trap
    two (rho, z); radial axes are limited to SSCN_RADIAL_MAX cells; the
    batch, the densities' shapes and the tile hints are Cartesian only; the
    plan puts the radial axis on the line-per-block kernel."""
    G = sscn
    ok = Problem(1, (500, 1, 1), (0.02,), (1.0,), 5.0, 1e-4, IMAG, F64, 1, geom=G.GEOM_CIR)
    assert sscn.validate(ok) == sscn.OK
    for bad in (Problem(2, (50, 40, 1), (0.1, 0.1), (1.0, 1.0), 5.0, 1e-4, IMAG, F64, 1, geom=G.GEOM_SPH),
                Problem(1, (50, 1, 1), (0.1,), (1.0,), 5.0, 1e-4, IMAG, F64, 1, geom=G.GEOM_AXI),
                Problem(1, (50, 1, 1), (0.1,), (1.0,), 5.0, 1e-4, IMAG, F64, 1, geom=7)):
        assert sscn.validate(bad) == sscn.E_INVALID
    big = Problem(1, (16385, 1, 1), (0.01,), (1.0,), 5.0, 1e-4, IMAG, F64, 1, geom=G.GEOM_SPH)
    assert sscn.validate(big) == sscn.E_UNSUPPORTED
    ax = Problem(2, (100, 70, 1), (0.1, 0.2), (1.0, 2.0), 5.0, 1e-4, REAL, F64, 0, geom=G.GEOM_AXI)
    info = sscn.plan_info(ax)
    assert info[0]["kind"] == "rad" and info[0]["grid"] == 70 and info[0]["block"] * info[0]["chunk"] >= 100
    assert info[1]["kind"] == "col"
    assert sscn.workspace_bytes(ax) > 0
    batch = Problem(1, (500, 1, 1), (0.02,), (1.0,), 5.0, 1e-4, IMAG, F32, 1, 10, geom=G.GEOM_CIR)
    with pytest.raises(sscn.SSCNError) as e:
        sscn.batch_workspace_bytes(batch)
    assert e.value.code == sscn.E_UNSUPPORTED
    with pytest.raises(sscn.SSCNError) as e:
        sscn.set_tile_hint(ok, (4, 0, 0))
    assert e.value.code == sscn.E_UNSUPPORTED
