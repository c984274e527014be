"""Pins of the oracle's Maxwell integration (Section 2 stage 1) on the Yee
lattice with the split-B leapfrog.

* A discrete transverse standing wave E^0 = e cos(k r), B^0 = 0 evolves as
  E^n = cos(omega n dt) E^0 exactly, with the Yee dispersion relation
  sin(omega dt / 2) = dt sqrt(sum_d sin^2(k_d dx_d / 2) / dx_d^2)
  (B^{1/2} = -(dt/2) curl E^0 is exactly the discrete mode's own half-step
  value, so the split start excites no second mode).  A wrong stagger, sign
  or missing half step changes omega or breaks the cos law.
* div B is constant for arbitrary E, B, J (div curl = 0 on the lattice).
* div E changes by exactly -dt div J per step (the J term's sign and place).
"""
import math

import numpy as np
import pytest

STAG = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5],
                 [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def _mode(n, dx, m):
    k = np.array([2 * math.pi * m[d] / (n[d] * dx[d]) for d in range(3)])
    sk = np.array([math.sin(k[d] * dx[d] / 2) / dx[d] for d in range(3)])
    # polarisation orthogonal to the discrete wave vector sk
    trial = np.array([1.0, 0.0, 0.0]) if abs(sk[0]) < 0.9 * np.linalg.norm(sk) else np.array([0.0, 1.0, 0.0])
    e = np.cross(sk, trial)
    e /= np.linalg.norm(e)
    K, J, I = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    E = []
    for c in range(3):
        r = [(I + STAG[c][0]) * dx[0], (J + STAG[c][1]) * dx[1], (K + STAG[c][2]) * dx[2]]
        E.append((e[c] * np.cos(k[0] * r[0] + k[1] * r[1] + k[2] * r[2])).ravel())
    return k, sk, E


@pytest.mark.parametrize("m,omega_printed", [((1, 0, 0), 0.390387194059),
                                             ((1, 1, 1), 0.676889047562),
                                             ((4, 0, 0), 1.424223332915)])
def test_standing_wave_dispersion_16cubed(orc, m, omega_printed):
    n, dx = (16, 16, 16), (1.0, 1.0, 1.0)
    dt = 0.5 / math.sqrt(3.0)
    k, sk, E0 = _mode(n, dx, m)
    omega = 2.0 / dt * math.asin(dt * np.linalg.norm(sk))
    assert abs(omega - omega_printed) < 1e-11
    g = orc.make_grid(n, dx, dt, 1)
    E = [a.copy() for a in E0]
    B = [np.zeros_like(E0[0]) for _ in range(3)]
    J = [np.zeros_like(E0[0]) for _ in range(3)]
    for step in range(1, 81):
        orc.fdtd(g, E, B, J)
        for c in range(3):
            np.testing.assert_allclose(E[c], math.cos(omega * step * dt) * E0[c], rtol=0, atol=1e-12)


def test_standing_wave_anisotropic_dx(orc):
    n, dx = (8, 12, 10), (1.0, 0.5, 2.0)
    dt = 0.45 / math.sqrt(sum(1 / d ** 2 for d in dx))
    k, sk, E0 = _mode(n, dx, (1, 2, 1))
    omega = 2.0 / dt * math.asin(dt * np.linalg.norm(sk))
    g = orc.make_grid(n, dx, dt, 1)
    E = [a.copy() for a in E0]
    B = [np.zeros_like(E0[0]) for _ in range(3)]
    J = [np.zeros_like(E0[0]) for _ in range(3)]
    for step in range(1, 61):
        orc.fdtd(g, E, B, J)
    for c in range(3):
        np.testing.assert_allclose(E[c], math.cos(omega * 60 * dt) * E0[c], rtol=0, atol=1e-12)


def _dive(n, dx, E):
    nx, ny, nz = n
    Ex, Ey, Ez = (a.reshape(nz, ny, nx) for a in E)
    return ((Ex - np.roll(Ex, 1, 2)) / dx[0] + (Ey - np.roll(Ey, 1, 1)) / dx[1]
            + (Ez - np.roll(Ez, 1, 0)) / dx[2]).ravel()


def test_div_b_constant_and_gauss_update(orc):
    n, dx = (6, 7, 5), (1.0, 0.8, 1.3)
    dt = 0.4
    g = orc.make_grid(n, dx, dt, 1)
    rng = np.random.default_rng(4)
    nc = n[0] * n[1] * n[2]
    E = [rng.standard_normal(nc) for _ in range(3)]
    B = [rng.standard_normal(nc) for _ in range(3)]
    J = [rng.standard_normal(nc) for _ in range(3)]
    db0 = orc.divb(g, B)
    for _ in range(10):
        de0 = _dive(n, dx, E)
        orc.fdtd(g, E, B, J)
        np.testing.assert_allclose(_dive(n, dx, E) - de0, -dt * _dive(n, dx, J), rtol=0, atol=1e-12)
        np.testing.assert_allclose(orc.divb(g, B), db0, rtol=0, atol=1e-12)
    # and the oracle's divB is the plain cell-centred difference
    nx, ny, nz = n
    Bx, By, Bz = (a.reshape(nz, ny, nx) for a in B)
    want = ((np.roll(Bx, -1, 2) - Bx) / dx[0] + (np.roll(By, -1, 1) - By) / dx[1]
            + (np.roll(Bz, -1, 0) - Bz) / dx[2]).ravel()
    np.testing.assert_allclose(orc.divb(g, B), want, rtol=0, atol=1e-13)
