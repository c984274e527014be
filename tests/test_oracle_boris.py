"""Pins of the oracle's relativistic equations of motion (Section 2) and
position advance, against closed forms of the Boris scheme:

* pure magnetic field: |u| is conserved exactly (the rotation is orthogonal),
  each step rotates u by theta = 2 atan(|q| B dt / (2 m gamma)) in the sense
  fixed by the sign of q, and the discrete orbit is a circle of radius
  r = (|u_perp| / gamma) dt / (2 sin(theta / 2));
* pure electric field: u^n = u^0 + (q E dt / m) n;
* crossed fields: the mean velocity is the E x B drift.

Worked example (B = 0.5 z, |u_perp| = 0.1, q = -1, m = 1, dt at half the 3D
Courant limit): gamma = 1.00498756, omega_c = 0.497518595,
theta = 0.143375135, omega_num = 0.496666036, r = 0.200515013.
"""
import math

import numpy as np
import pytest

DT = 0.5 / math.sqrt(3.0)


def _eb(E=(0, 0, 0), B=(0, 0, 0)):
    return np.array(list(E) + list(B), dtype=np.float64)


def test_worked_example_constants():
    g = math.sqrt(1.0 + 0.1 ** 2)
    theta = 2.0 * math.atan(0.5 * DT / (2.0 * g))
    assert abs(g - 1.00498756) < 1e-8
    assert abs(0.5 / g - 0.497518595) < 1e-9
    assert abs(theta - 0.143375135) < 1e-9
    assert abs(theta / DT - 0.496666036) < 1e-9
    assert abs((0.1 / g) * DT / (2.0 * math.sin(theta / 2.0)) - 0.200515013) < 1e-9


@pytest.mark.parametrize("q", [-1.0, 1.0])
def test_pure_b_rotation_angle_and_speed(orc, q):
    B0 = 0.5
    u = np.array([0.1, 0.0, 0.03])          # with a parallel component
    eb = _eb(B=(0, 0, B0))
    speed0 = np.linalg.norm(u)
    gam = math.sqrt(1.0 + speed0 ** 2)
    theta = 2.0 * math.atan(abs(q) * B0 * DT / (2.0 * gam))
    ang_prev = math.atan2(u[1], u[0])
    for n in range(500):
        u = orc.boris(q, 1.0, DT, eb, u)
        assert abs(np.linalg.norm(u) - speed0) <= 1e-15 * 4
        assert abs(u[2] - 0.03) <= 1e-17              # parallel momentum untouched
        ang = math.atan2(u[1], u[0])
        d = (ang - ang_prev + math.pi) % (2 * math.pi) - math.pi
        # dv/dt = (q/m) v x B: for B along +z a negative charge turns
        # counter-clockwise (positive angle), a positive charge clockwise
        assert abs(d - (-np.sign(q)) * theta) < 1e-12
        ang_prev = ang


def test_pure_b_orbit_radius(orc):
    g = orc.make_grid((64, 64, 64), (1.0, 1.0, 1.0), DT, 1)
    eb = _eb(B=(0, 0, 0.5))
    u = np.array([0.1, 0.0, 0.0])
    x = np.array([32.0, 32.0, 32.0])
    pts = []
    for n in range(120):
        u = orc.boris(-1.0, 1.0, DT, eb, u)
        x = orc.advance(g, u, x)
        pts.append(x[:2].copy())
    pts = np.array(pts)
    # circle through three well separated points
    a, b, c = pts[0], pts[7], pts[15]
    A = np.array([[b[0] - a[0], b[1] - a[1]], [c[0] - a[0], c[1] - a[1]]]) * 2.0
    rhs = np.array([b @ b - a @ a, c @ c - a @ a])
    ctr = np.linalg.solve(A, rhs)
    r = np.linalg.norm(pts - ctr, axis=1)
    assert np.max(np.abs(r - 0.200515013470470)) < 1e-11


def test_pure_e_linear_in_time(orc):
    E = np.array([0.02, -0.01, 0.005])
    u0 = np.array([0.01, 0.02, -0.03])
    u = u0.copy()
    q, m = -1.0, 1.0
    for n in range(1, 201):
        u = orc.boris(q, m, DT, _eb(E=E), u)
        np.testing.assert_allclose(u, u0 + (q * E * DT / m) * n, rtol=0, atol=1e-15 * n + 1e-16)


@pytest.mark.parametrize("start_at_drift", [True, False])
def test_e_cross_b_drift(orc, start_at_drift):
    g = orc.make_grid((1 << 20, 1 << 20, 1 << 20), (1.0, 1.0, 1.0), DT, 1)
    E0, B0 = 0.01, 1.0
    eb = _eb(E=(0, E0, 0), B=(0, 0, B0))
    vd = E0 / B0                               # E x B / B^2 = +0.01 x
    if start_at_drift:
        u = np.array([vd / math.sqrt(1 - vd * vd), 0.0, 0.0])
    else:
        u = np.zeros(3)
    x0 = np.array([1000.0, 1000.0, 1000.0])
    x = x0.copy()
    # an integer number of numerical gyro periods
    gam = 1.0
    theta = 2.0 * math.atan(B0 * DT / (2.0 * gam))
    nsteps = int(round(200 * 2 * math.pi / theta))
    for _ in range(nsteps):
        u = orc.boris(-1.0, 1.0, DT, eb, u)
        x = orc.advance(g, u, x)
    vmean = (x - x0) / (nsteps * DT)
    tol = 1e-4 if start_at_drift else 2e-3
    assert abs(vmean[0] - vd) < tol * vd
    assert abs(vmean[1]) < tol * vd and abs(vmean[2]) < 1e-18


def test_advance_and_wrap(orc):
    g = orc.make_grid((8, 8, 8), (1.0, 1.0, 1.0), DT, 1)
    # gamma = sqrt(1 + 0.75^2) = 1.25, v = 0.6 along x
    x = orc.advance(g, np.array([0.75, 0.0, 0.0]), np.array([7.9, 0.1, 0.2]))
    assert abs(x[0] - (7.9 + DT * 0.6)) < 1e-15 and x[1] == 0.1 and x[2] == 0.2
    w = orc.wrap(g, x)
    assert abs(w[0] - (7.9 + DT * 0.6 - 8.0)) < 1e-14
    # a tiny negative coordinate rounds to L on wrapping: stored as 0, never L
    w = orc.wrap(g, np.array([-1e-300, 8.0, -0.25]))
    assert w[0] == 0.0 and w[1] == 0.0 and w[2] == 7.75
    rng = np.random.default_rng(5)
    for _ in range(2000):
        p = rng.random(3) * 8.0 + rng.uniform(-0.3, 0.3, 3)
        w = orc.wrap(g, p)
        assert np.all(w >= 0.0) and np.all(w < 8.0)


def test_dx_scaling_of_advance(orc):
    g = orc.make_grid((8, 8, 8), (0.5, 1.0, 2.0), 0.1, 1)
    u = np.array([0.3, 0.3, 0.3])
    gi = 1.0 / math.sqrt(1 + 0.27)
    x = orc.advance(g, u, np.array([1.0, 1.0, 1.0]))
    np.testing.assert_allclose(x - 1.0, [0.1 / 0.5 * 0.3 * gi, 0.1 * 0.3 * gi, 0.1 / 2.0 * 0.3 * gi],
                               rtol=1e-14)
