"""Pins of the oracle's energy sums against exact special values.

* Kinetic energy w m (gamma - 1): u = 0.75 gives gamma = 1.25 exactly; u = 2.4
  gives gamma = 2.6; for slow particles (|u| = 1e-3 .. 1e-9) gamma - 1 keeps
  full relative accuracy against a 50-digit evaluation (the form
  sqrt(1 + u^2) - 1 loses it to cancellation).
* Field energy 1/2 sum F^2 dV: a cosine of one full period on the lattice sums
  to exactly half the number of points (discrete orthogonality).
"""
import math

import numpy as np


def test_kinetic_exact_gammas(orc):
    L = orc.lib()
    ux = np.array([0.75, 0.0, 0.0, 1.8])
    uy = np.array([0.0, 0.75, 0.0, 0.0])
    uz = np.array([0.0, 0.0, 0.75, 1.0])       # (1.8, 0, 1.0): |u|^2 = 4.24, gamma = sqrt(5.24)
    K = L.orc_kinetic(3.0, 0.5, 4, orc._dp(ux), orc._dp(uy), orc._dp(uz))
    want = 0.5 * 3.0 * (3 * 0.25 + (math.sqrt(5.24) - 1.0))
    assert abs(K - want) < 1e-14
    u = np.array([2.4])
    z = np.zeros(1)
    assert abs(L.orc_kinetic(1.0, 1.0, 1, orc._dp(u), orc._dp(z), orc._dp(z)) - 1.6) < 1e-15


def test_kinetic_small_u_limit(orc):
    L = orc.lib()
    u = np.array([1e-4])
    z = np.zeros(1)
    K = L.orc_kinetic(2.0, 1.5, 1, orc._dp(u), orc._dp(z), orc._dp(z))
    assert abs(K - 0.5 * 3.0 * 1e-8) < 1e-16


def test_kinetic_slow_particles_full_relative_accuracy(orc):
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    L = orc.lib()
    for u0 in (1e-3, 3.7e-5, 1e-7, 2.2e-9):
        u = np.array([u0, 0.6 * u0, 0.0])
        ux, uy, uz = (np.ascontiguousarray(u[i:i + 1]) for i in range(3))
        K = L.orc_kinetic(1.0, 1.0, 1, orc._dp(ux), orc._dp(uy), orc._dp(uz))
        u2 = Decimal(float(u[0])) ** 2 + Decimal(float(u[1])) ** 2
        want = float((1 + u2).sqrt() - 1)
        assert abs(K - want) <= 4e-16 * want, (u0, K, want)


def test_field_energy_of_a_lattice_cosine(orc):
    n = (8, 6, 4)
    dx = (0.5, 1.0, 2.0)
    g = orc.make_grid(n, dx, 0.1, 1)
    K, J, I = np.meshgrid(np.arange(4), np.arange(6), np.arange(8), indexing="ij")
    F = [np.ascontiguousarray((3.0 * np.cos(2 * math.pi * I / 8)).ravel()),
         np.ascontiguousarray((2.0 * np.cos(2 * math.pi * 2 * J / 6 + 0.3)).ravel()),
         np.zeros(192)]
    arr = (orc._D * 3)(*[orc._dp(a) for a in F])
    W = orc.lib().orc_field_energy(g, arr, 3)
    dv = 0.5 * 1.0 * 2.0
    want = 0.5 * dv * (9.0 * 192 / 2 + 4.0 * 192 / 2)
    assert abs(W - want) < 1e-12 * want
