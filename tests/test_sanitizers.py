"""CPU sanitizer builds (no GPU): the oracle compiled with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer, and the library's host
runtime (the C-ABI sources: validation, planning, table and geometry
set-up, the units front end) compiled with the same sanitizers on hipcc's
host pass, each driven through its host-side calls in a child process that
preloads the sanitizer runtime.  Any report ends the child with a non-zero
status; the child's output names it."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_BASE = {
    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=23:halt_on_error=1",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
}


def _runtime(compiler, name):
    try:
        p = subprocess.run([compiler, f"-print-file-name={name}"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run_child(code, preload, tmp_path):
    env = dict(os.environ, **ENV_BASE)
    env["LD_PRELOAD"] = preload
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    script = tmp_path / "child.py"
    script.write_text(textwrap.dedent(code))
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True,
                       timeout=600, cwd=str(tmp_path))
    assert r.returncode == 0 and "CHILD OK" in r.stdout, (r.returncode, r.stdout[-3000:], r.stderr[-6000:])


ORACLE_CHILD = """
import math, sys
import numpy as np
import oracle
from oracle import Problem, SymProblem, IMAG, REAL, CIR, SPH, AXI
oracle.use_library(sys.argv[0].replace("child.py", "liboracle_san.so"))
oracle.set_threads(2)
rng = np.random.default_rng(5)
for dim, n in ((1, (37,)), (2, (13, 9)), (3, (7, 6, 5)), (3, (1, 1, 1)), (1, (1,)), (1, (2,))):
    for mode in (IMAG, REAL):
        p = Problem(dim, n, (0.3,) * dim, (1.0, 1.5, 2.0)[:dim], 7.0, 0.01, mode, 1 if mode == IMAG else 0)
        shape = tuple(reversed(n))
        psi = rng.standard_normal(shape) + (1j * rng.standard_normal(shape) if mode == REAL else 0)
        out = oracle.run(p, psi, 3, observe_every=1)
        oracle.observe(p, out.psi)
        for a in range(dim):
            oracle.density_1d(p, psi, a)
            oracle.substep(p, psi, a)
        if dim == 3:
            for d in range(3):
                oracle.density_2d(p, psi, d)
        oracle.substep(p, psi, -1)
        oracle.potential(p)
for n in (1, 2, 3, 17):
    oracle.thomas(n, 0.3 + 0.2j, np.ones(n, complex))
    oracle.cn_line(n, 0.1j, np.ones(n, complex))
for geom, n, dx, om in ((CIR, (40,), (0.2,), (1.0,)), (SPH, (33,), (0.25,), (1.0,)),
                        (AXI, (12, 20), (0.3, 0.25), (1.0, 1.7)), (CIR, (1,), (0.5,), (1.0,)),
                        (AXI, (1, 1), (0.5, 0.5), (1.0, 1.0))):
    for mode in (IMAG, REAL):
        q = SymProblem(geom, n, dx, om, 5.0, 0.005, mode, 1 if mode == IMAG else 0)
        shape = (n[1], n[0]) if geom == AXI else (n[0],)
        psi = rng.standard_normal(shape) + (1j * rng.standard_normal(shape) if mode == REAL else 0)
        oracle.sym_coefs(q)
        oracle.sym_run(q, psi, 3, observe_every=1)
        oracle.sym_observe(q, psi)
        for w in range(-1, 2 if geom == AXI else 1):
            oracle.sym_substep(q, psi, w)
for dim in (1, 2, 3):
    oracle.units_to_g(dim, 1e4, 100.4, 86.909, 2 * math.pi * 100, (6.0, 9.0))
print("CHILD OK")
"""


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    preload = _runtime("gcc", "libasan.so")
    if preload is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    from oracle import build as obuild
    obuild.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    _run_child(ORACLE_CHILD, preload, tmp_path)


HOST_CHILD = """
import ctypes, math, sys
from paper_1605_03958_amd import sscn
from paper_1605_03958_amd.sscn import Problem, IMAG, REAL, F64, F32
L = ctypes.CDLL(sys.argv[0].replace("child.py", "libsscn_san.so"))
for name, (args, res) in sscn.EXPORTS.items():
    f = getattr(L, name)
    f.argtypes = args
    f.restype = res
sscn._lib = L
assert L.sscn_abi_version() == 2
for code in range(-8, 8):
    sscn.status_string(code)
# validation: every field out of range, before any side effect
base = dict(dim=3, n=(8, 6, 5), dx=(0.2,) * 3, omega=(1, 1.5, 2), g=22.0, dt=0.004, mode=IMAG, prec=F64,
            renorm_every=1, observe_every=10)
bad = [("dim", 0), ("dim", 4), ("n", (0, 6, 5)), ("n", (-3, 6, 5)), ("dx", (0.0, 0.2, 0.2)),
       ("dx", (float("nan"), 0.2, 0.2)), ("omega", (-1.0, 1, 1)), ("omega", (float("inf"), 1, 1)),
       ("g", float("nan")), ("dt", 0.0), ("dt", -1.0), ("mode", 2), ("prec", 5), ("renorm_every", 0),
       ("observe_every", -1), ("n", (20000, 20000, 20000))]
for field, value in bad:
    kw = dict(base)
    kw[field] = value
    assert sscn.validate(Problem(**kw)) != sscn.OK, field
for geom in (sscn.GEOM_CIR, sscn.GEOM_SPH, sscn.GEOM_AXI):
    for n in ((1, 1, 1), (4096, 1, 1), (16384, 1, 1), (16385, 1, 1), (512, 1024, 1), (64, 64, 64)):
        dim = 2 if geom == sscn.GEOM_AXI else 1
        for mode, prec in ((IMAG, F64), (REAL, F64), (IMAG, F32), (REAL, F32)):
            p = Problem(dim, n, (0.01, 0.02, 1.0)[:dim], (1.0, 1.6)[:dim], 30.0, 1e-5, mode, prec,
                        1 if mode == IMAG else 0, 10, geom=geom)
            if sscn.validate(p) == sscn.OK:
                sscn.state_bytes(p)
                sscn.workspace_bytes(p)
                sscn.plan_info(p)
# planning across shapes, both modes and precisions
shapes = [(1, (n, 1, 1)) for n in (1, 2, 3, 63, 64, 65, 255, 256, 1000, 4096, 5000, 9912, 16384, 70000, 300000)]
shapes += [(2, (a, b, 1)) for a in (1, 2, 17, 64, 256, 700) for b in (1, 3, 64, 700, 5000)]
shapes += [(3, n) for n in ((1, 1, 1), (2, 3, 4), (7, 5, 3), (64, 64, 64), (61, 77, 50), (256, 256, 256),
                            (160, 160, 160), (1024, 8, 8), (8, 8, 1024))]
for dim, n in shapes:
    for mode, prec in ((IMAG, F64), (REAL, F64), (IMAG, F32), (REAL, F32)):
        p = Problem(dim, n, (0.1,) * dim, (1.0, 1.5, 2.0)[:dim], 5.0, 1e-3, mode, prec,
                    1 if mode == IMAG else 0, 10)
        if sscn.validate(p) != sscn.OK:
            continue
        sscn.state_bytes(p)
        sscn.workspace_bytes(p)
        sscn.plan_info(p)
        if prec == F32:
            try:
                sscn.batch_workspace_bytes(p)
                sscn.batch_plan_info(p)
            except sscn.SSCNError:
                pass
# tile hints: set, plan, clear (single-problem and batch tables)
p = Problem(3, (64, 64, 64), (0.1,) * 3, (1, 1.5, 2), 5.0, 1e-3, IMAG, F64, 1, 10)
for hint in ((2, 8, 16), (4, 4, 4), (3, 0, 0)):
    try:
        sscn.set_tile_hint(p, hint)
        sscn.plan_info(p)
    except sscn.SSCNError:
        pass
sscn.clear_tile_hints()
q = Problem(3, (40, 44, 36), (0.1,) * 3, (1.0, 1.5, 2.0), 5.0, 1e-3, IMAG, F32, 1, 10)
for hint in ((6, 3, 12), (0, 16, 0), (100, 100, 100)):
    try:
        sscn.batch_set_tile_hint(q, hint)
        sscn.batch_plan_info(q)
    except sscn.SSCNError:
        pass
sscn.batch_clear_tile_hints()
for slots, cap in ((1, 1), (64, 100000), (4096, 1 << 20)):
    sscn.batch_ctl_bytes(slots, cap)
# null and misaligned arguments
pc = Problem(**base).c()
h = ctypes.c_void_p(0)
assert L.sscn_create(ctypes.byref(pc), None, None, None, ctypes.byref(h)) == sscn.E_INVALID
assert L.sscn_create(ctypes.byref(pc), ctypes.c_void_p(256), ctypes.c_void_p(260), None,
                     ctypes.byref(h)) == sscn.E_INVALID
assert L.sscn_step(None, 1) == sscn.E_INVALID
assert L.sscn_set_g(None, 1.0) == sscn.E_INVALID
assert L.sscn_destroy(None) == sscn.E_INVALID
assert L.sscn_validate(None) == sscn.E_INVALID
# physical units
for dim in (1, 2, 3):
    sscn.units_to_g(dim, 1e4, 100.4, 86.909, 2 * math.pi * 100, (6.0, 9.0))
for bad_args in ((0, 1e4, 100.4, 86.9, 600.0), (3, 0.0, 100.4, 86.9, 600.0), (3, 1e4, 100.4, -1.0, 600.0)):
    try:
        sscn.units_to_g(*bad_args)
    except sscn.SSCNError:
        pass
print("CHILD OK")
"""


def test_host_runtime_under_address_and_ub_sanitizers(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc is not installed")
    preload = _runtime("/opt/rocm/llvm/bin/clang", "libclang_rt.asan-x86_64.so")
    if preload is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    from paper_1605_03958_amd import build as pbuild
    pbuild.build_host_sanitized(str(tmp_path / "libsscn_san.so"))
    _run_child(HOST_CHILD, preload, tmp_path)
