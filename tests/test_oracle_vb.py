"""Pins of the oracle's Villasenor-Buneman current deposition (Section 3 names
the charge-conserving scheme with the cloud-in-cell form factor).

* Continuity, particle by particle: the CIC charge moved from x0 to x1,
  computed here independently with tent weights, equals -dt div J at every
  node, for moves crossing 0, 1, 2 and 3 cell planes, across the periodic
  seam, and with endpoints exactly on planes.
* Brute force of the plain definition: J_x at edge (i+1/2, j, k) is
  (q w / (dt * face)) * integral of xdot * [floor x(t) = i] W(y(t)-j) W(z(t)-k)
  over the straight path, evaluated here by splitting the path at every plane
  crossing and integrating each piece with 2-point Gauss-Legendre (exact, as
  the integrand is quadratic on each piece).
* Special cases: pure-x motion gives transverse weights (1-y)(1-z), y(1-z),
  (1-y)z, yz; no motion gives J = 0.
"""
import math

import numpy as np
import pytest


def _tent(r):
    return np.maximum(0.0, 1.0 - np.abs(r))


def _lin(n, i, j, k):
    return (i % n[0]) + n[0] * ((j % n[1]) + n[1] * (k % n[2]))


def cic_rho(n, dx, qw, x):
    rho = np.zeros(n[0] * n[1] * n[2])
    c = np.floor(x).astype(np.int64)
    dv = dx[0] * dx[1] * dx[2]
    for a in range(2):
        for b in range(2):
            for cc in range(2):
                w = _tent(x[0] - (c[0] + a)) * _tent(x[1] - (c[1] + b)) * _tent(x[2] - (c[2] + cc))
                rho[_lin(n, c[0] + a, c[1] + b, c[2] + cc)] += qw * w / dv
    return rho


def div_j(n, dx, J):
    nx, ny, nz = n
    Jx, Jy, Jz = (a.reshape(nz, ny, nx) for a in J)
    d = ((Jx - np.roll(Jx, 1, axis=2)) / dx[0] + (Jy - np.roll(Jy, 1, axis=1)) / dx[1]
         + (Jz - np.roll(Jz, 1, axis=0)) / dx[2])
    return d.ravel()


def bruteforce_j(n, dx, dt, qw, x0, x1):
    d = x1 - x0
    ts = {0.0, 1.0}
    for dim in range(3):
        if d[dim] == 0.0:
            continue
        lo, hi = min(x0[dim], x1[dim]), max(x0[dim], x1[dim])
        for p in range(math.ceil(lo), math.floor(hi) + 1):
            t = (p - x0[dim]) / d[dim]
            if 0.0 < t < 1.0:
                ts.add(t)
    ts = sorted(ts)
    J = [np.zeros(n[0] * n[1] * n[2]) for _ in range(3)]
    gq = [0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]
    for ta, tb in zip(ts[:-1], ts[1:]):
        mid = x0 + 0.5 * (ta + tb) * d
        cell = np.floor(mid).astype(np.int64)
        for gpt in gq:
            tg = ta + (tb - ta) * gpt
            p = x0 + tg * d
            wq = 0.5 * (tb - ta)
            for dim in range(3):
                e1, e2 = [e for e in range(3) if e != dim]
                area = dx[e1] * dx[e2]
                for o1 in range(2):
                    for o2 in range(2):
                        node = cell.copy()
                        node[e1] += o1
                        node[e2] += o2
                        Wt = _tent(p[e1] - node[e1]) * _tent(p[e2] - node[e2])
                        J[dim][_lin(n, *node)] += qw / (dt * area) * d[dim] * Wt * wq
    return J


def _moves(rng, n, count):
    """Random moves, |displacement| < 1 per axis, including forced 1/2/3-plane
    crossings, the periodic seam, and endpoints exactly on planes."""
    L = np.array(n, dtype=np.float64)
    out = []
    for i in range(count):
        kind = i % 6
        x0 = rng.random(3) * L
        dlt = rng.uniform(-0.95, 0.95, 3)
        if kind == 1:      # near a corner: likely 3 crossings
            x0 = np.floor(x0) + rng.choice([0.02, 0.98], 3)
            dlt = np.where(x0 - np.floor(x0) < 0.5, -1, 1) * rng.uniform(0.05, 0.9, 3)
        elif kind == 2:    # endpoint exactly on a plane
            x0 = np.floor(x0) + np.array([0.0, 0.5, 0.25])
        elif kind == 3:    # arrival exactly on a plane
            x1 = np.round(x0 + dlt)
            dlt = x1 - x0
            dlt = np.where(np.abs(dlt) >= 1.0, 0.0, dlt)
        elif kind == 4:    # across the periodic seam
            x0 = np.array([L[0] - 0.1, 0.05, L[2] - 0.3])
            dlt = np.array([0.4, -0.2, 0.6])
        elif kind == 5:    # small moves inside one cell
            dlt = rng.uniform(-0.01, 0.01, 3)
        out.append((x0, x0 + dlt))
    return out


@pytest.mark.parametrize("dx", [(1.0, 1.0, 1.0), (0.5, 1.5, 2.0)])
def test_continuity_per_particle(orc, dx):
    n = (6, 5, 7)
    dt = 0.3
    g = orc.make_grid(n, dx, dt, 1)
    rng = np.random.default_rng(11)
    nc = n[0] * n[1] * n[2]
    qw = -0.37
    worst = 0.0
    for x0, x1 in _moves(rng, n, 600):
        J = [np.zeros(nc) for _ in range(3)]
        orc.deposit_vb(g, J, x0, x1, qw)
        x1w = orc.wrap(g, x1)
        r0 = cic_rho(n, dx, qw, x0)
        r1 = cic_rho(n, dx, qw, x1w)
        res = (r1 - r0) / dt + div_j(n, dx, J)
        worst = max(worst, np.max(np.abs(res)))
    assert worst < 1e-13


def test_matches_bruteforce_definition(orc):
    n = (6, 5, 7)
    dx = (1.0, 1.0, 1.0)
    dt = 0.3
    g = orc.make_grid(n, dx, dt, 1)
    rng = np.random.default_rng(12)
    nc = n[0] * n[1] * n[2]
    for x0, x1 in _moves(rng, n, 300):
        J = [np.zeros(nc) for _ in range(3)]
        orc.deposit_vb(g, J, x0, x1, 1.0)
        Jb = bruteforce_j(n, dx, dt, 1.0, x0, x1)
        for d in range(3):
            np.testing.assert_allclose(J[d], Jb[d], rtol=0, atol=1e-14)


def test_pure_x_motion_weights(orc):
    n = (8, 8, 8)
    dt = 0.25
    g = orc.make_grid(n, (1.0, 1.0, 1.0), dt, 1)
    nc = 512
    x0 = np.array([3.2, 4.3, 5.6])
    x1 = np.array([3.7, 4.3, 5.6])
    J = [np.zeros(nc) for _ in range(3)]
    orc.deposit_vb(g, J, x0, x1, 1.0)
    fy, fz = 0.3, 0.6
    want = {(3, 4, 5): (1 - fy) * (1 - fz), (3, 5, 5): fy * (1 - fz),
            (3, 4, 6): (1 - fy) * fz, (3, 5, 6): fy * fz}
    for (i, j, k), w in want.items():
        assert abs(J[0][_lin(n, i, j, k)] - 0.5 / dt * w) < 1e-15
    assert abs(J[0].sum() - 0.5 / dt) < 1e-15
    assert np.all(J[1] == 0.0) and np.all(J[2] == 0.0)


def test_no_motion_no_current(orc):
    g = orc.make_grid((4, 4, 4), (1.0, 1.0, 1.0), 0.2, 1)
    for x0 in (np.array([1.3, 2.7, 0.1]), np.array([2.0, 3.0, 0.0])):
        J = [np.zeros(64) for _ in range(3)]
        orc.deposit_vb(g, J, x0, x0.copy(), 2.0)
        assert all(np.all(a == 0.0) for a in J)
