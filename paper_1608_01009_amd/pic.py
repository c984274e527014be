"""Python binding of ``libpic_hip.so`` (the C ABI declared in ``include/pic.h``).

Argument marshalling only: every step of the PIC path runs in the library's
HIP kernels.  The functions keep the ABI's names.  Arrays may be NumPy arrays
(host memory) or PyTorch tensors (host or device memory of the context's
GPU); PyTorch is used only as an allocator and for its stream handle.

If the shared library has not been built, :func:`library` raises: there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libpic_hip.so")

PIC_OK = 0
PIC_EINVAL = -1
PIC_FP64 = 0
PIC_FP32_MIXED = 1
_PRECISION = {"fp64": PIC_FP64, "mixed": PIC_FP32_MIXED, PIC_FP64: PIC_FP64,
              PIC_FP32_MIXED: PIC_FP32_MIXED}
PIC_BC_PERIODIC = 0
PIC_BC_ABSORBING = 1
_BC = {"periodic": PIC_BC_PERIODIC, "absorbing": PIC_BC_ABSORBING, PIC_BC_PERIODIC: 0,
       PIC_BC_ABSORBING: 1}
PIC_ENOMEM = -2
PIC_EDEVICE = -3
PIC_ECAPACITY = -4
PIC_ENONFINITE = -5
PIC_ESTATE = -6
STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EDEVICE",
                -4: "PIC_ECAPACITY", -5: "PIC_ENONFINITE", -6: "PIC_ESTATE"}

# the entry points declared in include/pic.h
ABI_SYMBOLS = ("pic_create", "pic_load_particles", "pic_set_fields", "pic_step",
               "pic_get_fields", "pic_get_particles", "pic_diagnostics", "pic_enable_timers",
               "pic_get_timers", "pic_get_counters", "pic_record", "pic_backward", "pic_set_laser",
               "pic_eval_sqrt_div", "pic_eval_sqrt_div_f32", "pic_eval_sqrt_div_noalloc",
               "pic_last_error", "pic_destroy")


class PicGrid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("supercell", C.c_int32), ("rebin_every", C.c_int32),
                ("halo", C.c_int32), ("precision", C.c_int32), ("deterministic_j", C.c_int32),
                ("bc_x", C.c_int32), ("reserved", C.c_int32), ("stream", C.c_void_p)]


class PicSpecies(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("weight", C.c_double),
                ("capacity", C.c_int64)]


class PicError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code
        self.message = message


_lib = None


def library():
    """Load libpic_hip.so; raises if it is missing (build it first).

    PyTorch (the allocator and stream provider) ships its own HIP runtime.
    It is imported first so that the library binds to that same runtime by
    soname; two HIP runtimes in one process do not share the device."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_1608_01009_amd.build)")
        L = C.CDLL(LIB_PATH)
        V = C.c_void_p
        D = C.POINTER(C.c_double)
        L.pic_create.argtypes = [C.POINTER(PicGrid), D, C.c_double, C.POINTER(PicSpecies),
                                 C.c_int32, C.POINTER(V)]
        L.pic_load_particles.argtypes = [V, C.c_int32, C.c_int64] + [V] * 7
        L.pic_set_fields.argtypes = [V, C.POINTER(V)]
        L.pic_step.argtypes = [V, C.c_int32]
        L.pic_get_fields.argtypes = [V, C.POINTER(V)]
        L.pic_get_particles.argtypes = [V, C.c_int32, C.c_int64, C.POINTER(C.c_int64)] + [V] * 7
        L.pic_diagnostics.argtypes = [V, D]
        L.pic_enable_timers.argtypes = [V, C.c_int32]
        L.pic_get_timers.argtypes = [V, D]
        L.pic_get_counters.argtypes = [V, C.POINTER(C.c_int64)]
        L.pic_record.argtypes = [V, C.c_int32]
        L.pic_set_laser.argtypes = [V, C.c_double, C.c_double, C.c_double, C.c_int32]
        L.pic_backward.argtypes = [V, C.POINTER(V), C.POINTER(V), C.POINTER(V), C.POINTER(V)]
        L.pic_eval_sqrt_div.argtypes = [C.c_int64, V, V, V, V, V]
        L.pic_eval_sqrt_div_noalloc.argtypes = [C.c_int64, V, V, V, V, V]
        L.pic_eval_sqrt_div_f32.argtypes = [C.c_int64, V, V, V, V, V]
        L.pic_last_error.argtypes = [V]
        L.pic_last_error.restype = C.c_char_p
        L.pic_destroy.argtypes = [V]
        L.pic_destroy.restype = None
        for name in ABI_SYMBOLS:
            if name not in ("pic_last_error", "pic_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _addr(a, n: int, dtype) -> Optional[int]:
    """Address of a contiguous array of at least n elements of dtype."""
    if a is None:
        return None
    if _is_torch(a):
        import torch
        want = torch.float64 if dtype == np.float64 else torch.int64
        if a.dtype != want or not a.is_contiguous() or a.numel() < n:
            raise ValueError(f"tensor must be contiguous {want} with >= {n} elements")
        return a.data_ptr()
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags.c_contiguous or a.size < n:
        raise ValueError(f"array must be a contiguous {np.dtype(dtype)} ndarray with >= {n} elements")
    return a.ctypes.data


def _check(ctx, code: int):
    if code != PIC_OK:
        msg = library().pic_last_error(ctx)
        raise PicError(code, msg.decode() if msg else "")


def _torch_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def pic_create(n: Sequence[int], dx: Sequence[float], dt: float, species, *, supercell: int = 4,
               rebin_every: int = 20, halo: int = 0, stream=None, precision="fp64",
               deterministic_j: bool = False, bc_x="periodic"):
    """``species``: sequence of ``(charge, mass, weight, capacity)``.
    ``stream``: None (library-owned stream), ``"torch"`` (torch's current
    stream) or a raw ``hipStream_t`` integer.  ``precision``: "fp64" or
    "mixed" (PIC_FP32_MIXED).  ``deterministic_j``: bit-reproducible current
    accumulation.  Returns the context handle."""
    L = library()
    g = PicGrid()
    for d in range(3):
        g.n[d] = int(n[d])
    g.supercell = int(supercell)
    g.rebin_every = int(rebin_every)
    g.halo = int(halo)
    g.precision = _PRECISION[precision] if precision in _PRECISION else int(precision)
    g.deterministic_j = int(deterministic_j)
    g.bc_x = _BC[bc_x] if bc_x in _BC else int(bc_x)
    if stream == "torch":
        stream = _torch_stream()
    g.stream = stream
    sp = (PicSpecies * len(species))()
    for i, s in enumerate(species):
        sp[i].charge, sp[i].mass, sp[i].weight = float(s[0]), float(s[1]), float(s[2])
        sp[i].capacity = int(s[3])
    dxa = (C.c_double * 3)(*[float(v) for v in dx])
    out = C.c_void_p()
    code = L.pic_create(C.byref(g), dxa, float(dt), sp, len(species), C.byref(out))
    if code != PIC_OK:
        raise PicError(code, L.pic_last_error(None).decode())
    return out


def pic_load_particles(ctx, species: int, x, y, z, ux, uy, uz, ids=None):
    n = int(x.shape[0]) if x is not None else 0
    ptrs = [_addr(a, n, np.float64) for a in (x, y, z, ux, uy, uz)]
    ip = _addr(ids, n, np.int64)
    _check(ctx, library().pic_load_particles(ctx, int(species), n, *ptrs, ip))


def pic_set_fields(ctx, EB: Sequence, ncell: Optional[int] = None):
    nc = ncell if ncell is not None else int(EB[0].shape[0])
    arr = (C.c_void_p * 6)(*[_addr(a, nc, np.float64) for a in EB])
    _check(ctx, library().pic_set_fields(ctx, arr))


def pic_set_laser(ctx, amplitude: float, omega: float, duration: float, plane: int):
    _check(ctx, library().pic_set_laser(ctx, float(amplitude), float(omega), float(duration),
                                        int(plane)))


def pic_step(ctx, n_steps: int = 1):
    _check(ctx, library().pic_step(ctx, int(n_steps)))


def pic_get_fields(ctx, ncell: int, out: Optional[List] = None) -> List:
    """Returns [Ex, Ey, Ez, Bx, By, Bz, Jx, Jy, Jz]; into ``out`` if given
    (None entries are skipped)."""
    if out is None:
        out = [np.empty(ncell) for _ in range(9)]
    arr = (C.c_void_p * 9)(*[_addr(a, ncell, np.float64) for a in out])
    _check(ctx, library().pic_get_fields(ctx, arr))
    return out


def pic_get_particles(ctx, species: int, capacity: Optional[int] = None,
                      out: Optional[Dict] = None) -> Dict:
    L = library()
    n = C.c_int64(0)
    if out is None:
        code = L.pic_get_particles(ctx, int(species), 0, C.byref(n), *([None] * 7))
        if code not in (PIC_OK, PIC_ECAPACITY):
            _check(ctx, code)
        cnt = int(n.value)
        out = {k: np.empty(cnt) for k in ("x", "y", "z", "ux", "uy", "uz")}
        out["id"] = np.empty(cnt, dtype=np.int64)
        capacity = cnt
    keys = ("x", "y", "z", "ux", "uy", "uz")
    cap = int(capacity if capacity is not None else len(out["x"]))
    ptrs = [_addr(out.get(k), 0, np.float64) for k in keys]
    ip = _addr(out.get("id"), 0, np.int64)
    _check(ctx, L.pic_get_particles(ctx, int(species), cap, C.byref(n), *ptrs, ip))
    out["n"] = int(n.value)
    return out


def pic_diagnostics(ctx) -> np.ndarray:
    out = np.zeros(8)
    _check(ctx, library().pic_diagnostics(ctx, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def pic_enable_timers(ctx, on=True):
    """on: False/0 off, True/1 every stage, 2 the stored-order push+deposit only,
    3 that kernel on one timed step in seven."""
    _check(ctx, library().pic_enable_timers(ctx, int(on)))


def pic_get_timers(ctx) -> np.ndarray:
    """ms[0] push+deposit in stored order, ms[1] its launches, ms[2] push+deposit
    through a re-sort order, ms[3] its launches, ms[4] far movers, ms[5] Yee
    update, ms[6] re-sort, ms[7] total, ms[8] steps, ms[9] zero."""
    out = np.zeros(10)
    _check(ctx, library().pic_get_timers(ctx, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def pic_get_counters(ctx) -> np.ndarray:
    out = np.zeros(4, dtype=np.int64)
    _check(ctx, library().pic_get_counters(ctx, out.ctypes.data_as(C.POINTER(C.c_int64))))
    return out


def pic_record(ctx, checkpoint_every: int):
    _check(ctx, library().pic_record(ctx, int(checkpoint_every)))


def pic_backward(ctx, ncell: int, counts: Sequence[int], seed_fields=None, seed_particles=None,
                 grad_fields=None, grad_particles=None):
    """Reverse sweep over the recorded run.  ``seed_fields``: six arrays or
    None; ``seed_particles``: per species None or six arrays (x, y, z, ux, uy,
    uz); ``grad_fields`` / ``grad_particles`` the same shapes as outputs
    (allocated as NumPy arrays when None).  ``counts``: particles per species.
    Returns (grad_fields, grad_particles)."""
    ns = len(counts)
    if grad_fields is None:
        grad_fields = [np.empty(ncell) for _ in range(6)]
    if grad_particles is None:
        grad_particles = [[np.empty(int(n)) for _ in range(6)] for n in counts]
    sf = None
    if seed_fields is not None:
        sf = (C.c_void_p * 6)(*[_addr(a, ncell, np.float64) for a in seed_fields])
    sp = None
    if seed_particles is not None:
        flat = []
        for s in range(ns):
            arrs = seed_particles[s] if seed_particles[s] is not None else [None] * 6
            flat += [_addr(a, int(counts[s]), np.float64) for a in arrs]
        sp = (C.c_void_p * (6 * ns))(*flat)
    gf = (C.c_void_p * 6)(*[_addr(a, ncell, np.float64) for a in grad_fields])
    flat = []
    for s in range(ns):
        arrs = grad_particles[s] if grad_particles[s] is not None else [None] * 6
        flat += [_addr(a, int(counts[s]), np.float64) for a in arrs]
    gp = (C.c_void_p * (6 * ns))(*flat)
    _check(ctx, library().pic_backward(ctx, sf, sp, gf, gp))
    return grad_fields, grad_particles


def pic_eval_sqrt_div(x=None, a=None, b=None, noalloc=False, f32=False):
    """The push's square root of x (>= 1) and quotient a / b (1 <= b < 2^1000)
    evaluated by the library (host or device arrays of equal length); returns
    (sqrt, quotient) as new arrays of the inputs' kind, None where not asked.
    noalloc: through pic_eval_sqrt_div_noalloc (no device allocation in the
    library; n at most 209,696).  f32: the mixed-precision push's FP32
    versions (float32 arrays; pic_eval_sqrt_div_f32)."""
    n = len(x) if x is not None else len(a)
    like = x if x is not None else a
    dt = np.float32 if f32 else np.float64

    def new():
        if _is_torch(like):
            import torch
            return torch.empty(n, dtype=torch.float32 if f32 else torch.float64,
                               device=like.device)
        return np.empty(n, dtype=dt)

    def addr(v):
        if v is None:
            return None
        if _is_torch(v):
            import torch
            want = torch.float32 if f32 else torch.float64
            if v.dtype != want or not v.is_contiguous() or v.numel() < n:
                raise ValueError(f"tensor must be contiguous {want} with >= {n} elements")
            return v.data_ptr()
        if not isinstance(v, np.ndarray) or v.dtype != dt or not v.flags.c_contiguous or v.size < n:
            raise ValueError(f"array must be a contiguous {np.dtype(dt)} ndarray with >= {n} "
                             f"elements")
        return v.ctypes.data
    sq = new() if x is not None else None
    dv = new() if a is not None else None
    L = library()
    fn = L.pic_eval_sqrt_div_f32 if f32 else (L.pic_eval_sqrt_div_noalloc if noalloc
                                              else L.pic_eval_sqrt_div)
    if f32 and noalloc:
        raise ValueError("the no-allocation variant is FP64 only")
    _check(None, fn(n, addr(x), addr(a), addr(b), addr(sq), addr(dv)))
    return sq, dv


def pic_last_error(ctx=None) -> str:
    m = library().pic_last_error(ctx)
    return m.decode() if m else ""


def pic_destroy(ctx):
    if ctx is not None:
        library().pic_destroy(ctx)


class Simulation:
    """Owning convenience wrapper around one context."""

    def __init__(self, n, dx, dt, species, *, supercell=4, rebin_every=20, halo=0, stream=None,
                 precision="fp64", deterministic_j=False, bc_x="periodic"):
        self.n = tuple(int(v) for v in n)
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        self.species = [tuple(s) for s in species]
        self.precision = precision
        self.ctx = pic_create(n, dx, dt, species, supercell=supercell, rebin_every=rebin_every,
                              halo=halo, stream=stream, precision=precision,
                              deterministic_j=deterministic_j, bc_x=bc_x)

    @classmethod
    def from_workload(cls, wl, capacity_factor=1.0, **kw):
        species = [(s.charge, s.mass, s.weight, int(s.n * capacity_factor)) for s in wl.species]
        bc = getattr(wl, "bc_x", "periodic")
        sim = cls(wl.n, wl.dx, wl.dt, species, supercell=wl.S, rebin_every=wl.R, bc_x=bc, **kw)
        for i, s in enumerate(wl.species):
            sim.load_particles(i, *s.arrays())
        sim.set_fields(wl.fields)
        if getattr(wl, "laser", None) is not None:
            sim.set_laser(*wl.laser)
        return sim

    def load_particles(self, species, x, y, z, ux, uy, uz, ids=None):
        pic_load_particles(self.ctx, species, x, y, z, ux, uy, uz, ids)

    def set_fields(self, EB):
        pic_set_fields(self.ctx, EB, self.ncell)

    def step(self, n=1):
        pic_step(self.ctx, n)

    def fields(self, out=None):
        return pic_get_fields(self.ctx, self.ncell, out)

    def particles(self, species=0, out=None):
        return pic_get_particles(self.ctx, species, out=out)

    def diagnostics(self):
        return pic_diagnostics(self.ctx)

    def counters(self):
        return pic_get_counters(self.ctx)

    def counts(self):
        """Particles per species."""
        return [self._count(s) for s in range(len(self.species))]

    def _count(self, s):
        L = library()
        n = C.c_int64(0)
        code = L.pic_get_particles(self.ctx, int(s), 0, C.byref(n), *([None] * 7))
        if code not in (PIC_OK, PIC_ECAPACITY):
            _check(self.ctx, code)
        return int(n.value)

    def set_laser(self, amplitude, omega, duration, plane):
        pic_set_laser(self.ctx, amplitude, omega, duration, plane)

    def record(self, checkpoint_every=20):
        pic_record(self.ctx, checkpoint_every)

    def backward(self, seed_fields=None, seed_particles=None, grad_fields=None,
                 grad_particles=None):
        return pic_backward(self.ctx, self.ncell, self.counts(), seed_fields, seed_particles,
                            grad_fields, grad_particles)

    def close(self):
        if self.ctx is not None:
            pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
