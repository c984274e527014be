"""CPU FP64 oracle of the PIC step (and of its mixed-precision variant) --
TEST INFRASTRUCTURE, not product code.

Thin ctypes wrapper around ``liborc.so`` (built from ``pic_oracle.c``).  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library: the two meet
only through NumPy arrays.

The stepping semantics (Section 2 of arXiv:1608.01009 gives the stage order;
Section 4.3 the supercell grouping):

* ``load_particles`` stores the particles and stable-sorts them by the
  supercell key; the rebin counter restarts.
* ``step`` clears J, runs the particle loop of every species in array order
  (gather, Boris, advance, deposit, wrap), applies the Yee update, and after
  every ``R``-th step since the last sort stable-sorts every species again.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("PIC_ORACLE_LIB") or os.path.join(_HERE, "liborc.so")
_lib = None

_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


class OrcGrid(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("dx", C.c_double * 3), ("dt", C.c_double),
                ("S", C.c_int64), ("absorb_x", C.c_int64)]


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        G = C.POINTER(OrcGrid)
        PP6 = _D * 6
        PP3 = _D * 3
        L.orc_gather.argtypes = [G, PP6, _D, _D]
        L.orc_boris.argtypes = [C.c_double, C.c_double, C.c_double, _D, _D]
        L.orc_advance.argtypes = [G, _D, _D, _D]
        L.orc_deposit_vb.argtypes = [G, PP3, _D, _D, C.c_double]
        L.orc_wrap.argtypes = [G, _D]
        L.orc_fdtd.argtypes = [G, PP3, PP3, PP3]
        L.orc_sort_key.argtypes = [G, _D]
        L.orc_sort_key.restype = C.c_int64
        L.orc_rebin.argtypes = [G, C.c_int64, _D, _D, _D, _D, _D, _D, _I64]
        L.orc_rebin.restype = C.c_int64
        L.orc_laser_field.argtypes = [C.c_double] * 4
        L.orc_laser_field.restype = C.c_double
        L.orc_add_laser.argtypes = [G, _D, C.c_int64, C.c_double, C.c_double, C.c_double,
                                    C.c_double]
        L.orc_push_deposit.argtypes = [G, C.c_double, C.c_double, C.c_double, C.c_int64,
                                       _D, _D, _D, _D, _D, _D, PP6, PP3]
        L.orc_mixed_round_pos.argtypes = [C.c_double, C.c_int64]
        L.orc_mixed_round_pos.restype = C.c_double
        L.orc_push_deposit_mixed.argtypes = [G, C.c_double, C.c_double, C.c_double, C.c_int64,
                                             _D, _D, _D, _D, _D, _D, PP6, PP3, C.c_void_p,
                                             C.c_void_p]
        L.orc_fdtd_adjoint.argtypes = [G, PP3, PP3, PP3]
        L.orc_adjoint_particles.argtypes = [G, C.c_double, C.c_double, C.c_double, C.c_int64,
                                            _D, _D, _D, _D, _D, _D, PP6, PP3,
                                            _D, _D, _D, _D, _D, _D, PP6]
        L.orc_rho.argtypes = [G, C.c_double, C.c_double, C.c_int64, _D, _D, _D, _D]
        L.orc_gauss.argtypes = [G, PP3, _D, _D]
        L.orc_divb.argtypes = [G, PP3, _D]
        L.orc_kinetic.argtypes = [C.c_double, C.c_double, C.c_int64, _D, _D, _D]
        L.orc_kinetic.restype = C.c_double
        L.orc_field_energy.argtypes = [G, C.POINTER(_D), C.c_int]
        L.orc_field_energy.restype = C.c_double
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(_I64)


def _ptrs(arrs):
    return (_D * len(arrs))(*[_dp(a) for a in arrs])


def make_grid(n, dx=(1.0, 1.0, 1.0), dt=None, S=1, absorb_x=False) -> OrcGrid:
    g = OrcGrid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.dx[d] = float(dx[d])
    g.dt = float(dt)
    g.S = int(S)
    g.absorb_x = int(bool(absorb_x))
    return g


# ---- per-particle primitives (for the pins) --------------------------------

def gather(g: OrcGrid, EB, xp):
    EB = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in EB]
    xp = np.ascontiguousarray(xp, dtype=np.float64)
    out = np.zeros(6)
    lib().orc_gather(C.byref(g), _ptrs(EB), _dp(xp), _dp(out))
    return out


def boris(q, m, dt, EB, u):
    EB = np.ascontiguousarray(EB, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    lib().orc_boris(q, m, dt, _dp(EB), _dp(u))
    return u


def advance(g: OrcGrid, u, x):
    u = np.ascontiguousarray(u, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_advance(C.byref(g), _dp(u), _dp(x), _dp(out))
    return out


def wrap(g: OrcGrid, x):
    x = np.array(x, dtype=np.float64)
    lib().orc_wrap(C.byref(g), _dp(x))
    return x


def deposit_vb(g: OrcGrid, J, x0, x1, qw):
    """Accumulate one move into J (list of three flat arrays), in place."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    x1 = np.ascontiguousarray(x1, dtype=np.float64)
    lib().orc_deposit_vb(C.byref(g), _ptrs(J), _dp(x0), _dp(x1), float(qw))


def fdtd(g: OrcGrid, E, B, J):
    lib().orc_fdtd(C.byref(g), _ptrs(E), _ptrs(B), _ptrs(J))


def sort_key(g: OrcGrid, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    return int(lib().orc_sort_key(C.byref(g), _dp(x)))


def rho(g: OrcGrid, q, w, x, y, z, out=None):
    nc = g.n[0] * g.n[1] * g.n[2]
    if out is None:
        out = np.zeros(nc)
    lib().orc_rho(C.byref(g), q, w, len(x), _dp(x), _dp(y), _dp(z), _dp(out))
    return out


def gauss(g: OrcGrid, E, rho_arr):
    out = np.zeros_like(rho_arr)
    lib().orc_gauss(C.byref(g), _ptrs(E), _dp(rho_arr), _dp(out))
    return out


def divb(g: OrcGrid, B):
    out = np.zeros_like(B[0])
    lib().orc_divb(C.byref(g), _ptrs(B), _dp(out))
    return out


def fdtd_adjoint(g: OrcGrid, lE, lB):
    """Transposed Yee update in place on (lE, lB); returns lJ."""
    nc = len(lE[0])
    lJ = [np.zeros(nc) for _ in range(3)]
    lib().orc_fdtd_adjoint(C.byref(g), _ptrs(lE), _ptrs(lB), _ptrs(lJ))
    return lJ


def adjoint_particles(g: OrcGrid, q, m, w, state, EB, lJ, lam, lEB):
    """One species' particle loop reversed.  state: x, y, z, ux, uy, uz at the
    start of the step; lam: six adjoint arrays, end of step -> start of step
    (in place); lEB: six arrays, accumulated."""
    n = len(state[0])
    lib().orc_adjoint_particles(C.byref(g), q, m, w, n, *[_dp(a) for a in state[:6]],
                                _ptrs(EB), _ptrs(lJ), *[_dp(a) for a in lam], _ptrs(lEB))


def laser_field(E0, omega, T, t):
    return lib().orc_laser_field(float(E0), float(omega), float(T), float(t))


def add_laser(g: OrcGrid, Jy, plane, E0, omega, T, t):
    """Jy += -2 E_L(t) / dx on the node plane x = plane (in place)."""
    lib().orc_add_laser(C.byref(g), _dp(Jy), int(plane), float(E0), float(omega), float(T),
                        float(t))


def mixed_round_pos(x, n):
    """Positions as the mixed-precision variant stores them (integer cell +
    FP32 offset), as FP64 values."""
    f = lib().orc_mixed_round_pos
    x = np.asarray(x, dtype=np.float64)
    return np.array([f(float(v), int(n)) for v in x.ravel()]).reshape(x.shape)


def push_deposit_mixed(g: OrcGrid, q, m, w, x, y, z, ux, uy, uz, EB, J, Jabs=None, Jcnt=None):
    """Mixed-precision particle loop (in place on the six FP64 arrays, which
    must hold values of the variant); J, Jabs (FP64) and Jcnt (int64) are
    lists of three flat arrays or None."""
    ja = _ptrs(Jabs) if Jabs is not None else None
    jn = (_I64 * 3)(*[_ip(a) for a in Jcnt]) if Jcnt is not None else None
    lib().orc_push_deposit_mixed(C.byref(g), q, m, w, len(x), _dp(x), _dp(y), _dp(z), _dp(ux),
                                 _dp(uy), _dp(uz), _ptrs(EB), _ptrs(J),
                                 C.cast(ja, C.c_void_p) if ja is not None else None,
                                 C.cast(jn, C.c_void_p) if jn is not None else None)


# ---- whole-state simulator -------------------------------------------------

FIELD_NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz")


class OracleSim:
    """Plain FP64 PIC state advanced by the oracle.

    ``species`` is a list of ``(charge, mass, weight)``.  Positions are in
    cell units.  Field arrays are flat, x-fastest, ``n[0]*n[1]*n[2]`` long.
    """

    def __init__(self, n, dx, dt, species, S=4, R=20, precision="fp64", absorb_x=False,
                 laser=None):
        """``absorb_x``: absorbing x boundaries with particle removal (FP64
        only).  ``laser``: None or (E0, omega, T, plane), the soft current
        sheet of ``orc_add_laser`` added every step at t = (step + 1/2) dt."""
        assert precision in ("fp64", "mixed")
        assert not (absorb_x and precision != "fp64")
        self.absorb_x = bool(absorb_x)
        self.laser = None if laser is None else tuple(float(v) for v in laser[:3]) + (int(laser[3]),)
        self.precision = precision
        self.n = tuple(int(v) for v in n)
        self.dx = tuple(float(v) for v in dx)
        self.dt = float(dt)
        self.S = int(S)
        self.R = int(R)
        self.g = make_grid(self.n, self.dx, self.dt, self.S, self.absorb_x)
        self.species = [tuple(float(v) for v in s) for s in species]
        nc = self.n[0] * self.n[1] * self.n[2]
        self.F = [np.zeros(nc) for _ in range(9)]
        self.P = [None] * len(self.species)
        self.steps_since_sort = 0
        self.step_count = 0
        # mixed precision only: when True, each step also records per J node
        # the sum of |contribution| (Jabs) and the number of contributions (Jcnt)
        self.collect_abs = False
        self.Jabs = None
        self.Jcnt = None

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * self.n[2]

    def load_particles(self, s, x, y, z, ux, uy, uz, ids=None):
        arrs = [np.array(a, dtype=np.float64).ravel() for a in (x, y, z, ux, uy, uz)]
        if self.precision == "mixed":
            arrs = self.to_mixed(arrs)
        n = len(arrs[0])
        ids = np.arange(n, dtype=np.int64) if ids is None else np.array(ids, dtype=np.int64)
        self.P[s] = arrs + [ids]
        self._sort(s)
        self.steps_since_sort = 0

    def set_state(self, particles, EB, steps_since_sort, step_count=None):
        """Install a full state exactly as given (no sort): per species the
        arrays (x, y, z, ux, uy, uz, id) in stored order, the six E/B arrays
        and the number of steps since the last sort.  Used to take one step
        from a state read back from another implementation."""
        for s, arrs in enumerate(particles):
            self.P[s] = [np.array(a, dtype=np.float64).ravel().copy() for a in arrs[:6]] + \
                        [np.array(arrs[6], dtype=np.int64).ravel().copy()]
        for c in range(6):
            self.F[c] = np.array(EB[c], dtype=np.float64).ravel().copy()
        self.steps_since_sort = int(steps_since_sort)
        if step_count is not None:
            self.step_count = int(step_count)       # the laser's clock

    def to_mixed(self, arrs):
        """x, y, z, ux, uy, uz as the mixed-precision variant stores them."""
        out = [mixed_round_pos(arrs[d], self.n[d]) for d in range(3)]
        return out + [np.asarray(a, dtype=np.float32).astype(np.float64) for a in arrs[3:6]]

    def _sort(self, s):
        x, y, z, ux, uy, uz, ids = self.P[s]
        kept = lib().orc_rebin(C.byref(self.g), len(x), _dp(x), _dp(y), _dp(z), _dp(ux),
                               _dp(uy), _dp(uz), _ip(ids))
        if kept < len(x):              # removed particles (absorbing x) dropped
            self.P[s] = [np.ascontiguousarray(a[:kept]) for a in self.P[s]]

    def set_fields(self, EB):
        for c in range(6):
            self.F[c] = np.array(EB[c], dtype=np.float64).ravel().copy()
        for c in range(6, 9):
            self.F[c] = np.zeros(self.ncells)

    def step(self, nsteps=1):
        L = lib()
        for _ in range(int(nsteps)):
            for c in range(6, 9):
                self.F[c][:] = 0.0
            EB = _ptrs(self.F[:6])
            J = _ptrs(self.F[6:9])
            ja = jn = None
            if self.precision == "mixed" and self.collect_abs:
                self.Jabs = [np.zeros(self.ncells) for _ in range(3)]
                self.Jcnt = [np.zeros(self.ncells, dtype=np.int64) for _ in range(3)]
                ja_arr = _ptrs(self.Jabs)                 # kept alive for the calls below
                jn_arr = (_I64 * 3)(*[_ip(a) for a in self.Jcnt])
                ja = C.cast(ja_arr, C.c_void_p)
                jn = C.cast(jn_arr, C.c_void_p)
            for s, (q, m, w) in enumerate(self.species):
                if self.P[s] is None or len(self.P[s][0]) == 0:
                    continue
                x, y, z, ux, uy, uz, _ = self.P[s]
                if self.precision == "mixed":
                    L.orc_push_deposit_mixed(C.byref(self.g), q, m, w, len(x), _dp(x), _dp(y),
                                             _dp(z), _dp(ux), _dp(uy), _dp(uz), EB, J, ja, jn)
                else:
                    L.orc_push_deposit(C.byref(self.g), q, m, w, len(x), _dp(x), _dp(y), _dp(z),
                                       _dp(ux), _dp(uy), _dp(uz), EB, J)
            if self.laser is not None:
                E0, om, T, plane = self.laser
                L.orc_add_laser(C.byref(self.g), _dp(self.F[7]), plane, E0, om, T,
                                (self.step_count + 0.5) * self.dt)
            L.orc_fdtd(C.byref(self.g), _ptrs(self.F[0:3]), _ptrs(self.F[3:6]),
                       _ptrs(self.F[6:9]))
            self.step_count += 1
            self.steps_since_sort += 1
            if self.steps_since_sort % self.R == 0:
                for s in range(len(self.species)):
                    if self.P[s] is not None:
                        self._sort(s)
                self.steps_since_sort = 0

    def run_recorded(self, nsteps):
        """Advance ``nsteps`` steps (FP64 only), keeping the full state at the
        start of every step: a tape for :meth:`adjoint`."""
        assert self.precision == "fp64"
        tape = []
        for _ in range(int(nsteps)):
            tape.append(([None if P is None else [a.copy() for a in P] for P in self.P],
                         [f.copy() for f in self.F[:6]]))
            self.step(1)
        return tape

    def adjoint(self, tape, seed_EB, seed_P):
        """Reverse-mode gradient of a scalar of the current state with respect
        to the state at the start of ``tape``.  ``seed_EB``: six arrays (dL/dE,
        dL/dB now); ``seed_P``: per species six arrays (dL/dx .. dL/duz, stored
        order now) or None.  Returns (six field gradients, per species six
        gradient arrays in the stored order at the start of the tape).  A
        re-sort only reorders particles: its transpose moves each adjoint back
        to the slot of the same particle id."""
        lEB = [np.array(a, dtype=np.float64).copy() for a in seed_EB]
        lam = []
        for s, P in enumerate(self.P):
            if P is None:
                lam.append(None)
                continue
            sd = None if seed_P is None else seed_P[s]
            lam.append([np.zeros(len(P[0])) if sd is None else np.array(sd[k], dtype=np.float64).copy()
                        for k in range(6)])
        ids_after = [None if P is None else P[6] for P in self.P]
        for j in range(len(tape) - 1, -1, -1):
            Pj, EBj = tape[j]
            for s, P in enumerate(Pj):
                if P is None:
                    continue
                if not np.array_equal(P[6], ids_after[s]):
                    order = np.argsort(P[6], kind="stable")
                    slot = order[np.searchsorted(P[6][order], ids_after[s])]
                    for k in range(6):
                        moved = np.empty_like(lam[s][k])
                        moved[slot] = lam[s][k]
                        lam[s][k] = moved
            lJ = fdtd_adjoint(self.g, lEB[0:3], lEB[3:6])
            for s, (q, m, w) in enumerate(self.species):
                if Pj[s] is None or len(Pj[s][0]) == 0:
                    continue
                adjoint_particles(self.g, q, m, w, Pj[s], EBj, lJ, lam[s], lEB)
            ids_after = [None if P is None else P[6] for P in Pj]
        return lEB, lam

    def fields(self):
        return {k: self.F[i] for i, k in enumerate(FIELD_NAMES)}

    def particles(self, s):
        x, y, z, ux, uy, uz, ids = self.P[s]
        return {"x": x, "y": y, "z": z, "ux": ux, "uy": uy, "uz": uz, "id": ids}

    def rho(self):
        out = np.zeros(self.ncells)
        for s, (q, m, w) in enumerate(self.species):
            if self.P[s] is None:
                continue
            x, y, z = self.P[s][:3]
            rho(self.g, q, w, x, y, z, out)
        return out

    def gauss(self):
        return gauss(self.g, self.F[0:3], self.rho())

    def divb(self):
        return divb(self.g, self.F[3:6])

    def kinetic(self):
        K = 0.0
        for s, (q, m, w) in enumerate(self.species):
            if self.P[s] is None:
                continue
            live = self.P[s][0] >= 0.0           # removed particles carry x = -1
            ux, uy, uz = [np.ascontiguousarray(a[live]) for a in self.P[s][3:6]]
            K += lib().orc_kinetic(m, w, len(ux), _dp(ux), _dp(uy), _dp(uz))
        return K

    def field_energy(self):
        L = lib()
        E = (_D * 3)(*[_dp(a) for a in self.F[0:3]])
        B = (_D * 3)(*[_dp(a) for a in self.F[3:6]])
        return (L.orc_field_energy(C.byref(self.g), E, 3),
                L.orc_field_energy(C.byref(self.g), B, 3))

    def total_charge(self):
        return sum(q * w * (0 if self.P[s] is None else int(np.sum(self.P[s][0] >= 0.0)))
                   for s, (q, m, w) in enumerate(self.species))
