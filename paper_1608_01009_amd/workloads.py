"""Seeded synthetic inputs for the PIC step.

This module only draws random numbers and lays out arrays; it contains none
of the method's arithmetic, so both the GPU library's tests and the CPU
oracle's tests can take their inputs from it.

The benchmark problem of arXiv:1608.01009 (Section 3) is itself synthetic: a
plasma on a periodic grid with a fixed number of particles per cell, run in
double precision.  The generators below build plasmas of that shape:

* positions: for every cell in linear order (x fastest), ``ppc`` particles at
  ``(i + U, j + U, k + U)`` with ``U ~ U[0, 1)``;
* momenta ``u = gamma v / c``: each component ``N(0, v_th^2)``;
* optional sinusoidal x-density perturbation of amplitude ``eps`` applied as
  the displacement ``x <- x - (eps / k) sin(k x)``, ``k = 2 pi / L_x``, then
  wrapped into ``[0, L_x)``;
* optional field noise: every stored E/B value uniform in ``[-a, a]``.

Draw order: positions, then momenta, then fields, from
``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

ELECTRON = (-1.0, 1.0)   # (charge in e, mass in m_e)
PROTON = (1.0, 1836.0)


def courant_dt(dx=(1.0, 1.0, 1.0), fraction=0.5) -> float:
    """``fraction`` of the 3D Yee stability limit c dt <= 1/sqrt(sum 1/dx_d^2)."""
    return fraction / math.sqrt(sum(1.0 / (d * d) for d in dx))


@dataclass
class Species:
    charge: float
    mass: float
    weight: float
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return (self.x, self.y, self.z, self.ux, self.uy, self.uz)


@dataclass
class Workload:
    name: str
    n: Tuple[int, int, int]
    dx: Tuple[float, float, float]
    dt: float
    S: int
    R: int
    steps: int
    species: List[Species]
    fields: List[np.ndarray]            # Ex, Ey, Ez, Bx, By, Bz (flat, x-fastest)
    meta: dict = field(default_factory=dict)
    bc_x: str = "periodic"              # or "absorbing"
    laser: Optional[Tuple[float, float, float, int]] = None   # (E0, omega, T, plane)

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nparticles(self) -> int:
        return sum(s.n for s in self.species)


def _wrap(a: np.ndarray, L: float) -> np.ndarray:
    a = np.where(a < 0.0, a + L, a)
    a = np.where(a >= L, a - L, a)
    a[a == L] = 0.0
    return a


def uniform_positions(rng, n, ppc):
    """``ppc`` particles per cell, cells in linear (x-fastest) order."""
    nx, ny, nz = n
    nc = nx * ny * nz
    U = rng.random((nc * ppc, 3))
    cell = np.repeat(np.arange(nc, dtype=np.int64), ppc)
    i = cell % nx
    j = (cell // nx) % ny
    k = cell // (nx * ny)
    x = i + U[:, 0]
    y = j + U[:, 1]
    z = k + U[:, 2]
    # i + U can round up to i + 1 when U is within half an ulp of 1
    x = _wrap(np.minimum(x, np.nextafter(i + 1.0, 0.0)), float(nx))
    y = _wrap(np.minimum(y, np.nextafter(j + 1.0, 0.0)), float(ny))
    z = _wrap(np.minimum(z, np.nextafter(k + 1.0, 0.0)), float(nz))
    return x, y, z


def quiet_positions(n, per_dim=2):
    """Regular lattice of ``per_dim**3`` particles per cell (quiet start)."""
    nx, ny, nz = n
    off = (np.arange(per_dim) + 0.5) / per_dim
    gx = (np.arange(nx)[:, None] + off[None, :]).ravel()
    gy = (np.arange(ny)[:, None] + off[None, :]).ravel()
    gz = (np.arange(nz)[:, None] + off[None, :]).ravel()
    Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
    return X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()


def perturb_x(x, Lx, eps, mode=1):
    k = 2.0 * math.pi * mode / Lx
    return _wrap(x - (eps / k) * np.sin(k * x), float(Lx))


def plasma(name, n, ppc, vth, seed, *, eps=0.0, noise=0.0, S=4, R=20, steps=100,
           dx=(1.0, 1.0, 1.0), dt=None, n0=1.0, species=ELECTRON) -> Workload:
    """Uniform (optionally perturbed) thermal plasma of one mobile species over
    an immobile neutralising background."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = uniform_positions(rng, n, ppc)
    u = rng.normal(0.0, vth, size=(x.shape[0], 3)) if vth > 0 else np.zeros((x.shape[0], 3))
    if eps != 0.0:
        x = perturb_x(x, n[0], eps)
    nc = n[0] * n[1] * n[2]
    if noise > 0.0:
        F = rng.uniform(-noise, noise, size=(6, nc))
        fields = [np.ascontiguousarray(F[c]) for c in range(6)]
    else:
        fields = [np.zeros(nc) for _ in range(6)]
    dv = dx[0] * dx[1] * dx[2]
    w = n0 * dv / ppc
    q, m = species
    sp = Species(q, m, w, np.ascontiguousarray(x), np.ascontiguousarray(y),
                 np.ascontiguousarray(z), np.ascontiguousarray(u[:, 0]),
                 np.ascontiguousarray(u[:, 1]), np.ascontiguousarray(u[:, 2]))
    return Workload(name, tuple(n), tuple(dx), courant_dt(dx) if dt is None else dt, S, R,
                    steps, [sp], fields,
                    meta=dict(ppc=ppc, vth=vth, seed=seed, eps=eps, noise=noise, n0=n0))


# ---- the named workloads ----------------------------------------------------

# recipe: grid, particles per cell, v_th, seed, keyword arguments of plasma()
RECIPES = {
    1: dict(name="uniform-16c-8ppc-perturbed", n=(16, 16, 16), ppc=8, vth=0.01, seed=1001,
            eps=0.01, steps=100),
    2: dict(name="uniform-64c-50ppc", n=(64, 64, 64), ppc=50, vth=0.05, seed=1002,
            noise=1e-3, steps=200),
    4: dict(name="uniform-128c-32ppc-perturbed", n=(128, 128, 128), ppc=32, vth=0.01,
            seed=1004, eps=0.01, steps=200),
    5: dict(name="uniform-32c-16ppc-modes", n=(32, 32, 32), ppc=16, vth=0.02, seed=1005,
            steps=400),
}


def from_recipe(r: dict, **override) -> Workload:
    r = dict(r, **override)
    name, n, ppc, vth, seed = r.pop("name"), r.pop("n"), r.pop("ppc"), r.pop("vth"), r.pop("seed")
    return plasma(name, n, ppc, vth, seed, **r)


def config1() -> Workload:
    """16^3 periodic, 8 electrons per cell (32,768), v_th = 0.01 c, x-density
    perturbation 0.01, E = B = 0, 100 steps."""
    return from_recipe(RECIPES[1])


def config2() -> Workload:
    """64^3 periodic, 50 electrons per cell (13,107,200), v_th = 0.05 c, E/B
    noise 1e-3, supercells 4^3, rebin every 20 steps, 200 steps."""
    return from_recipe(RECIPES[2])


def config4() -> Workload:
    """128^3 periodic, 32 electrons per cell (67,108,864), v_th = 0.01 c,
    x-density perturbation 0.01, 200 steps."""
    return from_recipe(RECIPES[4])


def config5(amplitudes: Optional[np.ndarray] = None) -> Workload:
    """32^3 periodic, 16 electrons per cell (524,288), v_th = 0.02 c, E_x a sum of
    the eight lowest x-modes, 400 steps."""
    wl = from_recipe(RECIPES[5])
    a = np.full(8, 1e-3) if amplitudes is None else np.asarray(amplitudes, dtype=np.float64)
    nx, ny, nz = wl.n
    xi = np.arange(nx) + 0.5
    prof = sum(a[m - 1] * np.cos(2.0 * math.pi * m * xi / nx) for m in range(1, 9))
    wl.fields[0] = np.ascontiguousarray(np.broadcast_to(prof[None, None, :], (nz, ny, nx)).ravel())
    wl.meta["amplitudes"] = a.tolist()
    return wl


def laser_slab(n=(256, 128, 128), slab=(96, 224), ppc=8, seed=1003, a0=1.0, wavelength=32.0,
               envelope_steps=200, plane=2, density=0.5, S=4, R=20, steps=1000,
               name="laser-slab-256x128x128") -> Workload:
    """Laser-plasma slab: absorbing x boundaries, periodic y and z; cold
    electrons and protons (mass 1836) at ``ppc`` particles per cell each, at
    the same positions (a neutral start, E = B = 0), filling the cells
    slab[0] <= x < slab[1] with density ``density`` times the critical
    density of the laser (n_crit = omega^2 with m_e = e = 1); a linearly
    polarised (E_y) laser of wavelength ``wavelength`` cells, normalised
    amplitude a0 (E0 = a0 omega) and a sin^2 envelope ``envelope_steps`` steps
    long, launched from the node plane x = ``plane``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = n
    sub = (slab[1] - slab[0], ny, nz)
    x, y, z = uniform_positions(rng, sub, ppc)
    x = x + float(slab[0])
    dt = courant_dt()
    omega = 2.0 * math.pi / wavelength
    n0 = density * omega * omega
    w = n0 / ppc
    zeros = np.zeros(x.shape[0])
    species = []
    for q, m in (ELECTRON, PROTON):
        species.append(Species(q, m, w, x.copy(), y.copy(), z.copy(), zeros.copy(),
                               zeros.copy(), zeros.copy()))
    nc = nx * ny * nz
    fields = [np.zeros(nc) for _ in range(6)]
    return Workload(name, tuple(n), (1.0, 1.0, 1.0), dt, S, R, steps, species, fields,
                    meta=dict(ppc=ppc, seed=seed, slab=tuple(slab), a0=a0,
                              wavelength=wavelength, density=density, n0=n0),
                    bc_x="absorbing",
                    laser=(a0 * omega, omega, envelope_steps * dt, int(plane)))


def config3() -> Workload:
    """Laser-plasma slab on 256 x 128 x 128 cells (absorbing x), electrons and
    protons at 8 per cell each in 96 <= x < 224 (33,554,432 particles), 0.5 n_crit,
    a0 = 1, wavelength 32 cells, 200-step sin^2 envelope, 1000 steps.  Particles
    are re-sorted every 10 steps: once the pulse drives the electrons to
    0.5-0.8 c they outrun the one-cell halo of the tiles within a few steps, and
    the global-memory path of those far movers costs more than the extra
    re-sorts."""
    return laser_slab(R=10)


def scaled(cfg: int, n, ppc, seed=7, **kw) -> Workload:
    """The recipe of a named workload on another grid / particles per cell (for
    parity tests at sizes the oracle finishes in seconds)."""
    r = dict(RECIPES[cfg])
    r["name"] = r["name"] + f"-at-{n[0]}x{n[1]}x{n[2]}-{ppc}ppc"
    r.update(n=tuple(n), ppc=ppc, seed=seed)
    r.update(kw)
    return from_recipe(r)
