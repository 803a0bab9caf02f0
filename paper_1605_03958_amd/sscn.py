"""Thin ctypes binding of libsscn.so (include/sscn.h).

Argument marshalling only: every step of the propagation runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory (the state and the
workspace are torch tensors the binding owns) and the current HIP stream.
The library must be built (``paper_1605_03958_amd/build.py``); importing
this module without it raises.
"""
from __future__ import annotations

import ctypes
import gc
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsscn.so")

OK, NOT_CONVERGED, BUSY = 0, 1, 2
E_INVALID, E_HIP, E_NONFINITE, E_NOSPACE, E_UNSUPPORTED = -1, -2, -3, -4, -5
IMAG, REAL = 0, 1
F64, F32 = 0, 1
GEOM_CART, GEOM_CIR, GEOM_SPH, GEOM_AXI = 0, 1, 2, 3
NKERNELS = 5
KERNEL_CLASSES = ("x_sweep_pointwise", "y_sweep", "z_sweep_norm", "norm_final", "scale_pass")


class SSCNError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


class CProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("omega", ctypes.c_double * 3),
        ("g", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("renorm_every", ctypes.c_int32),
        ("observe_every", ctypes.c_int32),
        ("geom", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


class CObs(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("norm", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("ekin", ctypes.c_double),
        ("epot", ctypes.c_double),
        ("eint", ctypes.c_double),
        ("mean", ctypes.c_double * 3),
        ("msq", ctypes.c_double * 3),
        ("status", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
    ]


class CBatchSlot(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("steps", ctypes.c_int64),
        ("last_norm", ctypes.c_double),
        ("obs", CObs),
    ]


SLOT_EMPTY, SLOT_RUNNING, SLOT_CONVERGED, SLOT_DONE, SLOT_NONFINITE = 0, 1, 2, 3, 4


class CUnits(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("atoms", ctypes.c_double),
        ("scattering_length", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("tight", ctypes.c_double * 2),
    ]

EXPORTS = {
    "sscn_abi_version": ([], ctypes.c_int),
    "sscn_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "sscn_validate": ([ctypes.POINTER(CProblem)], ctypes.c_int),
    "sscn_units_to_g": ([ctypes.POINTER(CUnits), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "sscn_state_bytes": ([ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sscn_workspace_bytes": ([ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sscn_create": ([ctypes.POINTER(CProblem), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "sscn_create_noalloc": ([ctypes.POINTER(CProblem), ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "sscn_step": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "sscn_prepare": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "sscn_observe": ([ctypes.c_void_p, ctypes.POINTER(CObs)], ctypes.c_int),
    "sscn_run": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(CObs),
                  ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "sscn_set_g": ([ctypes.c_void_p, ctypes.c_double], ctypes.c_int),
    "sscn_step_timed": ([ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "sscn_set_tile_hint": ([ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "sscn_clear_tile_hints": ([], ctypes.c_int),
    "sscn_plan_info": ([ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32],
                       ctypes.c_int),
    "sscn_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "sscn_density_1d": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "sscn_density_2d": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "sscn_batch_ctl_bytes": ([ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sscn_batch_workspace_bytes": ([ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sscn_batch_set_tile_hint": ([ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "sscn_batch_clear_tile_hints": ([], ctypes.c_int),
    "sscn_batch_plan_info": ([ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32],
                             ctypes.c_int),
    "sscn_batch_set_split": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "sscn_batch_create": ([ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                           ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "sscn_batch_admit": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(CProblem), ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_double, ctypes.c_int64], ctypes.c_int),
    "sscn_batch_evict": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "sscn_batch_step": ([ctypes.c_void_p, ctypes.c_int32], ctypes.c_int),
    "sscn_batch_poll": ([ctypes.c_void_p, ctypes.POINTER(CBatchSlot), ctypes.c_int32, ctypes.c_int32],
                        ctypes.c_int),
    "sscn_batch_error": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "sscn_batch_destroy": ([ctypes.c_void_p], ctypes.c_int),
}

_lib = None


def lib():
    """Load libsscn.so (never builds it); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsscn.so is not built ({LIB_PATH}); run paper_1605_03958_amd/build.py")
    # torch first: its HIP runtime then satisfies the library's dependency
    # (same soname), so the tensors and streams torch hands over belong to
    # the runtime the library calls.  Loaded the other way round, torch
    # would bring a second copy of the runtime into the process.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in EXPORTS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def status_string(code: int) -> str:
    try:
        return lib().sscn_status_string(int(code)).decode()
    except Exception:  # pragma: no cover - only when the library is absent
        return "unknown"


def _check(rc: int, what: str, allow=(OK,)):
    if rc not in allow:
        raise SSCNError(rc, what)
    return rc


@dataclass
class Problem:
    dim: int
    n: tuple
    dx: tuple
    omega: tuple
    g: float
    dt: float
    mode: int = IMAG
    prec: int = F64
    renorm_every: int = 1
    observe_every: int = 0
    geom: int = GEOM_CART

    def __post_init__(self):
        self.n = tuple(int(v) for v in (list(self.n) + [1, 1, 1])[:3])
        self.dx = tuple(float(v) for v in (list(self.dx) + [1.0, 1.0, 1.0])[:3])
        self.omega = tuple(float(v) for v in (list(self.omega) + [0.0, 0.0, 0.0])[:3])

    def c(self) -> CProblem:
        p = CProblem()
        p.dim = int(self.dim)
        for a in range(3):
            p.n[a] = self.n[a]
            p.dx[a] = self.dx[a]
            p.omega[a] = self.omega[a]
        p.g = float(self.g)
        p.dt = float(self.dt)
        p.mode = int(self.mode)
        p.prec = int(self.prec)
        p.renorm_every = int(self.renorm_every)
        p.observe_every = int(self.observe_every)
        p.geom = int(self.geom)
        p.pad_ = 0
        return p

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def points(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def dvol(self) -> float:
        return float(np.prod(self.dx[: self.dim]))

    def torch_dtype(self):
        import torch
        if self.mode == IMAG:
            return torch.float64 if self.prec == F64 else torch.float32
        return torch.complex128 if self.prec == F64 else torch.complex64

    def numpy_dtype(self):
        if self.mode == IMAG:
            return np.float64 if self.prec == F64 else np.float32
        return np.complex128 if self.prec == F64 else np.complex64


def units_to_g(dim: int, atoms: float, scattering_length_bohr: float, mass_amu: float, omega: float,
               tight=(1.0, 1.0)):
    """The dimensionless nonlinearity of a condensate of `atoms` atoms of
    mass `mass_amu` (u) and scattering length `scattering_length_bohr`
    (Bohr radii) in a trap of reference angular frequency `omega` (rad/s);
    `tight`: the frozen directions' frequencies over omega (dim < 3).
    Returns (g, length unit in m, time unit in s)."""
    u = CUnits()
    u.dim = int(dim)
    u.pad_ = 0
    u.atoms = float(atoms)
    u.scattering_length = float(scattering_length_bohr)
    u.mass = float(mass_amu)
    u.omega = float(omega)
    u.tight[0] = float(tight[0])
    u.tight[1] = float(tight[1])
    g, l, t = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().sscn_units_to_g(ctypes.byref(u), ctypes.byref(g), ctypes.byref(l), ctypes.byref(t)),
           "sscn_units_to_g")
    return g.value, l.value, t.value


def validate(prob: Problem) -> int:
    pc = prob.c()
    return lib().sscn_validate(ctypes.byref(pc))


def state_bytes(prob: Problem) -> int:
    pc = prob.c()
    v = ctypes.c_size_t(0)
    _check(lib().sscn_state_bytes(ctypes.byref(pc), ctypes.byref(v)), "sscn_state_bytes")
    return int(v.value)


def workspace_bytes(prob: Problem) -> int:
    pc = prob.c()
    v = ctypes.c_size_t(0)
    _check(lib().sscn_workspace_bytes(ctypes.byref(pc), ctypes.byref(v)), "sscn_workspace_bytes")
    return int(v.value)


def plan_info(prob: Problem):
    pc = prob.c()
    info = (ctypes.c_int32 * 24)()
    _check(lib().sscn_plan_info(ctypes.byref(pc), info, 24), "sscn_plan_info")
    kinds = {0: "row", 1: "col", 2: "stream", 3: "rad", -1: None}
    out = []
    for a in range(3):
        o = info[8 * a: 8 * a + 8]
        out.append(None if o[0] < 0 else dict(kind=kinds[o[0]], chunk=o[1], waves=o[2], lanes=o[3],
                                              grid=o[4], block=o[5], i_conv=o[6], depth=o[7]))
    return out


def set_tile_hint(prob: Problem, chunks) -> None:
    pc = prob.c()
    arr = (ctypes.c_int32 * 3)(*[int(c) for c in chunks])
    _check(lib().sscn_set_tile_hint(ctypes.byref(pc), arr), "sscn_set_tile_hint")


def clear_tile_hints() -> None:
    lib().sscn_clear_tile_hints()


@dataclass
class Obs:
    step: int
    norm: float
    mu: float
    energy: float
    ekin: float
    epot: float
    eint: float
    mean: tuple = field(default=(0.0, 0.0, 0.0))
    msq: tuple = field(default=(0.0, 0.0, 0.0))
    status: int = OK

    @staticmethod
    def from_c(o: CObs) -> "Obs":
        return Obs(int(o.step), o.norm, o.mu, o.energy, o.ekin, o.epot, o.eint,
                   tuple(o.mean), tuple(o.msq), int(o.status))

    @staticmethod
    def rows(buf, n: int) -> list:
        """Obs of the first n entries of a CObs array, read through one numpy
        view."""
        if n <= 0:
            return []
        a = np.ctypeslib.as_array(buf)[:n]
        # a burst of small objects: the cyclic collector is held off for it
        # (a full collection over a process holding torch took ~60 ms)
        was = gc.isenabled()
        gc.disable()
        try:
            return Obs._rows_of(a)
        finally:
            if was:
                gc.enable()

    @staticmethod
    def _rows_of(a) -> list:
        return [Obs(int(st), float(nm), float(mu), float(en), float(ek), float(ep), float(ei),
                    (float(m[0]), float(m[1]), float(m[2])), (float(q[0]), float(q[1]), float(q[2])), int(sta))
                for st, nm, mu, en, ek, ep, ei, m, q, sta in
                zip(a["step"].tolist(), a["norm"].tolist(), a["mu"].tolist(), a["energy"].tolist(),
                    a["ekin"].tolist(), a["epot"].tolist(), a["eint"].tolist(), a["mean"].tolist(),
                    a["msq"].tolist(), a["status"].tolist())]


class Solver:
    """One SSCN problem bound to torch-owned device memory on a stream.

    Without a stream argument the solver gets a stream of its own (not the
    legacy default stream, so the library can replay its steps from captured
    graphs); state(), observe() and the densities wait for it."""

    def __init__(self, prob: Problem, psi0=None, device: str = "cuda", stream=None, noalloc: bool = False):
        """noalloc: create through sscn_create_noalloc (the library's static
        workspace on the device; no workspace tensor)."""
        import torch
        L = lib()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.prob = prob
        self._pc = prob.c()
        _check(L.sscn_validate(ctypes.byref(self._pc)), "sscn_validate")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.psi = torch.zeros(prob.shape, dtype=prob.torch_dtype(), device=self.device)
        self.ws = None
        if not noalloc:
            wsb = workspace_bytes(prob)
            self.ws = torch.zeros(wsb // 8 + 32, dtype=torch.float64, device=self.device)
            if self.ws.data_ptr() % 256:
                raise RuntimeError("workspace tensor is not 256-byte aligned")
        if psi0 is not None:
            self.set_state(psi0)
        h = ctypes.c_void_p(0)
        torch.cuda.synchronize(self.device)
        if noalloc:
            with torch.cuda.device(self.device):
                _check(L.sscn_create_noalloc(ctypes.byref(self._pc), ctypes.c_void_p(self.psi.data_ptr()),
                                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                       "sscn_create_noalloc")
        else:
            _check(L.sscn_create(ctypes.byref(self._pc), ctypes.c_void_p(self.psi.data_ptr()),
                                 ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h)), "sscn_create")
        self._h = h

    # -- state ---------------------------------------------------------------
    def set_state(self, psi0) -> None:
        """psi0: a host array, or a device tensor ready on torch's current
        stream (converted to the state's dtype by the copy)."""
        import torch
        if isinstance(psi0, torch.Tensor):
            src = psi0.reshape(self.prob.shape)
            self.stream.wait_stream(torch.cuda.current_stream(self.device))
            with torch.cuda.stream(self.stream):
                self.psi.copy_(src)
            self.stream.synchronize()
            return
        a = np.ascontiguousarray(np.asarray(psi0).reshape(self.prob.shape))
        if self.prob.mode == IMAG and np.iscomplexobj(a):
            a = a.real
        a = a.astype(self.prob.numpy_dtype())
        with torch.cuda.stream(self.stream):
            self.psi.copy_(torch.from_numpy(a))
        self.stream.synchronize()

    def state(self) -> np.ndarray:
        self.stream.synchronize()
        return self.psi.cpu().numpy()

    # -- propagation ---------------------------------------------------------
    def step(self, nsteps: int) -> None:
        _check(lib().sscn_step(self._h, int(nsteps)), "sscn_step")

    def prepare(self, nsteps: int) -> None:
        """Capture the graphs a following step(nsteps) replays (no launch)."""
        _check(lib().sscn_prepare(self._h, int(nsteps)), "sscn_prepare")

    def step_timed(self, nsteps: int):
        ms = (ctypes.c_double * NKERNELS)()
        _check(lib().sscn_step_timed(self._h, int(nsteps), ms), "sscn_step_timed")
        return dict(zip(KERNEL_CLASSES, list(ms)))

    def observe(self) -> Obs:
        o = CObs()
        rc = lib().sscn_observe(self._h, ctypes.byref(o))
        _check(rc, "sscn_observe", allow=(OK, E_NONFINITE))
        return Obs.from_c(o)

    def run(self, max_steps: int, mu_tol: float, trace_cap: int = 100000):
        """sscn_run; trace_cap = 0 keeps no trace (the rows are not copied)."""
        cap = int(trace_cap)
        buf = (CObs * cap)() if cap > 0 else None
        rows = ctypes.c_int64(0)
        rc = lib().sscn_run(self._h, int(max_steps), float(mu_tol), buf, cap, ctypes.byref(rows))
        _check(rc, "sscn_run", allow=(OK, NOT_CONVERGED, E_NONFINITE))
        return rc, Obs.rows(buf, rows.value)

    def set_g(self, g: float) -> None:
        _check(lib().sscn_set_g(self._h, float(g)), "sscn_set_g")

    def density_1d(self, keep: int) -> np.ndarray:
        import torch
        # allocated on the solver's stream, which the kernel writes it on
        # (every element)
        with torch.cuda.stream(self.stream):
            out = torch.empty(self.prob.n[keep], dtype=torch.float64, device=self.device)
        _check(lib().sscn_density_1d(self._h, int(keep), ctypes.c_void_p(out.data_ptr())), "sscn_density_1d")
        self.stream.synchronize()
        return out.cpu().numpy()

    def density_2d(self, drop: int) -> np.ndarray:
        import torch
        keep = [a for a in range(3) if a != drop]
        with torch.cuda.stream(self.stream):
            out = torch.empty((self.prob.n[keep[1]], self.prob.n[keep[0]]), dtype=torch.float64, device=self.device)
        _check(lib().sscn_density_2d(self._h, int(drop), ctypes.c_void_p(out.data_ptr())), "sscn_density_2d")
        self.stream.synchronize()
        return out.cpu().numpy()

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().sscn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batch
# ---------------------------------------------------------------------------

def batch_ctl_bytes(max_slots: int, max_items: int) -> int:
    v = ctypes.c_size_t(0)
    _check(lib().sscn_batch_ctl_bytes(int(max_slots), int(max_items), ctypes.byref(v)), "sscn_batch_ctl_bytes")
    return int(v.value)


def batch_workspace_bytes(prob: Problem) -> int:
    pc = prob.c()
    v = ctypes.c_size_t(0)
    _check(lib().sscn_batch_workspace_bytes(ctypes.byref(pc), ctypes.byref(v)), "sscn_batch_workspace_bytes")
    return int(v.value)


@dataclass
class SlotStatus:
    state: int
    steps: int
    last_norm: float
    obs: Obs


def batch_plan_info(prob: Problem):
    """Geometry of prob's instances in the persistent kernel, per axis."""
    pc = prob.c()
    info = (ctypes.c_int32 * 24)()
    _check(lib().sscn_batch_plan_info(ctypes.byref(pc), info, 24), "sscn_batch_plan_info")
    kinds = {0: "row", 1: "col", -1: None}
    out = []
    for a in range(3):
        o = info[8 * a: 8 * a + 8]
        out.append(None if o[0] < 0 else dict(kind=kinds[o[0]], chunk=o[1], waves=o[2], lanes=o[3], items=o[4],
                                              rep=o[5], depth=o[6], big=bool(o[7])))
    return out


def batch_set_tile_hint(prob: Problem, chunks) -> None:
    pc = prob.c()
    arr = (ctypes.c_int32 * 3)(*[int(c) for c in chunks])
    _check(lib().sscn_batch_set_tile_hint(ctypes.byref(pc), arr), "sscn_batch_set_tile_hint")


def batch_clear_tile_hints() -> None:
    lib().sscn_batch_clear_tile_hints()


class Batch:
    """A batch of FP32 instances advanced by one persistent launch per step
    (1D lines that fit one block take whole steps in a solo kernel, several
    per launch; on a stream of its own beside the persistent launches).

    Owns (as torch tensors) the control block and, per admitted slot, the
    instance state and workspace."""

    def __init__(self, max_slots: int, max_items: int = 1 << 20, device: str = "cuda", stream=None,
                 split: int = 0):
        """split > 0: the work-item split (sscn_batch_set_split); 0 keeps
        the library's default."""
        import torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.max_slots = int(max_slots)
        nb = batch_ctl_bytes(max_slots, max_items)
        self.ctl = torch.zeros(nb // 8 + 64, dtype=torch.float64, device=self.device)
        self.psi = [None] * self.max_slots
        self.ws = [None] * self.max_slots
        self.prob = [None] * self.max_slots
        h = ctypes.c_void_p(0)
        torch.cuda.synchronize(self.device)
        _check(lib().sscn_batch_create(self.max_slots, int(max_items), ctypes.c_void_p(self.ctl.data_ptr()),
                                       ctypes.c_size_t(nb), ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h)), "sscn_batch_create")
        self._h = h
        if split:
            _check(lib().sscn_batch_set_split(self._h, int(split)), "sscn_batch_set_split")

    def footprint(self, prob: Problem) -> int:
        """HBM bytes a slot of this problem keeps resident (state + workspace)."""
        return state_bytes(prob) + batch_workspace_bytes(prob)

    def admit(self, slot: int, prob: Problem, psi0, mu_tol: float = 0.0, max_steps: int = 1 << 40):
        import torch
        wsb = batch_workspace_bytes(prob)
        if isinstance(psi0, torch.Tensor):
            src = psi0.to(device=self.device, dtype=prob.torch_dtype()).reshape(prob.shape)
        else:
            a = np.ascontiguousarray(np.asarray(psi0).reshape(prob.shape))
            if prob.mode == IMAG and np.iscomplexobj(a):
                a = a.real
            src = torch.from_numpy(a.astype(prob.numpy_dtype())).to(self.device)
        # src is ready on the caller's stream; the slot's tensors are made
        # on the batch stream, which the library then works on
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            psi = torch.empty(prob.shape, dtype=prob.torch_dtype(), device=self.device)
            psi.copy_(src)
            ws = torch.zeros(wsb // 8 + 32, dtype=torch.float64, device=self.device)
        self.stream.synchronize()
        pc = prob.c()
        _check(lib().sscn_batch_admit(self._h, int(slot), ctypes.byref(pc), ctypes.c_void_p(psi.data_ptr()),
                                      ctypes.c_void_p(ws.data_ptr()), float(mu_tol), int(max_steps)),
               "sscn_batch_admit")
        self.psi[slot], self.ws[slot], self.prob[slot] = psi, ws, prob

    def evict(self, slot: int):
        """Release a slot; returns its (renormalised) state tensor."""
        _check(lib().sscn_batch_evict(self._h, int(slot)), "sscn_batch_evict")
        psi = self.psi[slot]
        self.psi[slot] = self.ws[slot] = self.prob[slot] = None
        return psi

    def step(self, nsteps: int) -> None:
        _check(lib().sscn_batch_step(self._h, int(nsteps)), "sscn_batch_step")

    def poll(self, wait: bool = True):
        buf = (CBatchSlot * self.max_slots)()
        rc = lib().sscn_batch_poll(self._h, buf, self.max_slots, 1 if wait else 0)
        if rc == BUSY:
            return None
        _check(rc, "sscn_batch_poll")
        return [SlotStatus(buf[i].state, int(buf[i].steps), buf[i].last_norm, Obs.from_c(buf[i].obs))
                for i in range(self.max_slots)]

    def error(self) -> bool:
        f = ctypes.c_int32(0)
        _check(lib().sscn_batch_error(self._h, ctypes.byref(f)), "sscn_batch_error")
        return bool(f.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().sscn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
