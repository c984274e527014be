"""The oracle's evaluation order against the textbook forms (Section 3:
cloud-in-cell interpolation and the relativistic push, in double precision).

The paper fixes no evaluation order.  The oracle interpolates by nested
linear interpolation with fused multiply-adds and evaluates the Boris push
and the position advance as chains of fused multiply-adds.  These pins show
that those forms are admissible roundings of the textbook expressions:
* gather: the nested-lerp value and the plain tent sum
  sum_abc w_a(fx) w_b(fy) w_c(fz) F (every product and sum rounded
  separately) both lie within a few ulp of the exactly evaluated tent sum
  (rational arithmetic), measured in ulp of the largest stencil value;
* Boris push and advance: the fused chain and the separately rounded
  textbook expressions both lie within a few ulp of the exact result
  (50-digit decimal arithmetic), in ulp of the largest momentum component
  or coordinate involved;
so the two forms agree to a few ulp, on random inputs and on positions at
the periodic seam and on integer and half-integer planes.
"""
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

STAG = ((0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0))
GATHER_ULP = 6
PUSH_ULP = 8


def _ulp(v):
    return float(np.spacing(np.float64(abs(v))))


def _stencil(x, s):
    xi = x - s
    fl = math.floor(xi)
    return int(fl), xi - fl


def _positions(n, rng, count):
    P = list(rng.random((count, 3)) * np.array(n))
    L = [float(v) for v in n]
    seam = [0.0, 0.5, 1.0, 1.5, L[0] - 0.5, np.nextafter(L[0], 0.0), np.nextafter(0.5, 1.0),
            np.nextafter(0.5, 0.0), 1e-300, 3.0, 2.5]
    for a in seam:
        for b in (0.0, 0.5, np.nextafter(L[1], 0.0), 1.25):
            P.append(np.array([a, b, np.nextafter(L[2], 0.0)]))
    return P


@pytest.mark.parametrize("seed", [1, 2])
def test_gather_nested_lerp_and_tent_sum_within_ulps_of_exact(orc, seed):
    n = (6, 5, 4)
    rng = np.random.default_rng(seed)
    nc = n[0] * n[1] * n[2]
    EB = [rng.uniform(-1.0, 1.0, nc) * 10.0 ** rng.integers(-3, 3) for _ in range(6)]
    g = orc.make_grid(n, (1.0, 1.0, 1.0), 0.3, 1)
    worst_fma = worst_plain = 0.0
    for xp in _positions(n, rng, 150):
        got = orc.gather(g, EB, np.asarray(xp, dtype=np.float64))
        for c in range(6):
            i, f = zip(*[_stencil(float(xp[d]), STAG[c][d]) for d in range(3)])
            exact = Fraction(0)
            plain = 0.0
            vmax = 0.0
            for a in (0, 1):
                for b in (0, 1):
                    for cc in (0, 1):
                        idx = ((i[0] + a) % n[0]) + n[0] * (((i[1] + b) % n[1]) +
                                                            n[1] * ((i[2] + cc) % n[2]))
                        F = float(EB[c][idx])
                        vmax = max(vmax, abs(F))
                        w = [(1 - Fraction(f[d])) if o == 0 else Fraction(f[d])
                             for d, o in enumerate((a, b, cc))]
                        exact += w[0] * w[1] * w[2] * Fraction(F)
                        wp = [(1.0 - f[d]) if o == 0 else f[d] for d, o in enumerate((a, b, cc))]
                        plain = plain + ((wp[0] * wp[1]) * wp[2]) * F
            ex = float(exact)
            u = _ulp(vmax)
            worst_fma = max(worst_fma, abs(got[c] - ex) / u)
            worst_plain = max(worst_plain, abs(plain - ex) / u)
            assert abs(got[c] - ex) <= GATHER_ULP * u, (xp, c, got[c], ex)
            assert abs(plain - ex) <= GATHER_ULP * u, (xp, c, plain, ex)
            assert abs(got[c] - plain) <= 2 * GATHER_ULP * u
    print(f"gather: nested lerp {worst_fma:.2f} ulp, tent sum {worst_plain:.2f} ulp of the exact")


def _boris_plain(q, m, dt, EB, u):
    """Textbook Boris, every operation rounded separately (numpy float64)."""
    E = [float(v) for v in EB[:3]]
    B = [float(v) for v in EB[3:]]
    h = (q * dt) / (2.0 * m)
    um = [u[d] + h * E[d] for d in range(3)]
    gm = math.sqrt(1.0 + ((um[0] * um[0] + um[1] * um[1]) + um[2] * um[2]))
    t = [(h / gm) * B[d] for d in range(3)]
    sf = 2.0 / (1.0 + ((t[0] * t[0] + t[1] * t[1]) + t[2] * t[2]))
    s = [sf * t[d] for d in range(3)]
    cr = lambda a, b: [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],  # noqa: E731
                       a[0] * b[1] - a[1] * b[0]]
    c1 = cr(um, t)
    up = [um[d] + c1[d] for d in range(3)]
    c2 = cr(up, s)
    upl = [um[d] + c2[d] for d in range(3)]
    return [upl[d] + h * E[d] for d in range(3)]


def _boris_exact(q, m, dt, EB, u):
    getcontext().prec = 50
    D = lambda v: Decimal(float(v))  # noqa: E731  (exact conversion of a double)
    E = [D(v) for v in EB[:3]]
    B = [D(v) for v in EB[3:]]
    h = D((q * dt) / (2.0 * m))      # the rounded constant that both forms use
    um = [D(u[d]) + h * E[d] for d in range(3)]
    gm = (1 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]).sqrt()
    t = [(h / gm) * B[d] for d in range(3)]
    sf = 2 / (1 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2])
    s = [sf * t[d] for d in range(3)]
    cr = lambda a, b: [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],  # noqa: E731
                       a[0] * b[1] - a[1] * b[0]]
    c1 = cr(um, t)
    up = [um[d] + c1[d] for d in range(3)]
    c2 = cr(up, s)
    upl = [um[d] + c2[d] for d in range(3)]
    return [float(upl[d] + h * E[d]) for d in range(3)], [float(v) for v in um]


@pytest.mark.parametrize("q,m", [(-1.0, 1.0), (1.0, 1836.0)])
def test_boris_fused_chain_and_textbook_within_ulps_of_exact(orc, q, m):
    rng = np.random.default_rng(5 if q < 0 else 6)
    dt = 0.5 / math.sqrt(3.0)
    worst_fma = worst_plain = 0.0
    for k in range(400):
        su = 10.0 ** rng.uniform(-3, 1)
        sf = 10.0 ** rng.uniform(-4, 0.5)
        u = rng.standard_normal(3) * su
        EB = rng.standard_normal(6) * sf
        if k % 10 == 0:
            EB[:3] = 0.0            # pure rotation
        if k % 10 == 1:
            EB[3:] = 0.0            # pure kick
        got = orc.boris(q, m, dt, EB, u)
        plain = _boris_plain(q, m, dt, EB, list(u))
        ex, um = _boris_exact(q, m, dt, EB, u)
        scale = max(np.max(np.abs(u)), np.max(np.abs(ex)), np.max(np.abs(um)))
        ul = _ulp(scale)
        for d in range(3):
            worst_fma = max(worst_fma, abs(got[d] - ex[d]) / ul)
            worst_plain = max(worst_plain, abs(plain[d] - ex[d]) / ul)
            assert abs(got[d] - ex[d]) <= PUSH_ULP * ul, (k, d, got[d], ex[d])
            assert abs(plain[d] - ex[d]) <= PUSH_ULP * ul, (k, d, plain[d], ex[d])
    print(f"boris: fused chain {worst_fma:.2f} ulp, textbook {worst_plain:.2f} ulp of the exact")


def test_advance_fused_and_textbook_within_ulps_of_exact(orc):
    rng = np.random.default_rng(7)
    dt = 0.5 / math.sqrt(3.0)
    getcontext().prec = 50
    for dx in ((1.0, 1.0, 1.0), (0.5, 1.0, 2.0)):
        g = orc.make_grid((64, 64, 64), dx, dt, 4)
        for k in range(300):
            x = rng.random(3) * 64.0
            if k % 5 == 0:
                x = np.floor(x) + (0.5 if k % 2 else 0.0)
            u = rng.standard_normal(3) * 10.0 ** rng.uniform(-3, 1)
            got = orc.advance(g, u, x)
            gi = 1.0 / math.sqrt(1.0 + ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]))
            D = Decimal
            ge = 1 / (1 + D(float(u[0])) ** 2 + D(float(u[1])) ** 2 + D(float(u[2])) ** 2).sqrt()
            for d in range(3):
                cdt = dt / dx[d]
                plain = x[d] + (cdt * u[d]) * gi
                ex = float(D(float(x[d])) + D(cdt) * D(float(u[d])) * ge)
                scale = max(abs(x[d]), abs(ex - x[d]), 1e-300)
                ul = _ulp(scale)
                assert abs(got[d] - ex) <= 4 * ul, (k, d, got[d], ex)
                assert abs(plain - ex) <= 4 * ul, (k, d, plain, ex)
