"""Pins of the oracle's cloud-in-cell field interpolation (Section 2 stage
"field interpolation"; Section 3 names the cloud-in-cell form factor).

Each pin is independent of the oracle's own code: a constant field (partition
of unity), a field linear in one coordinate on each component's own staggered
lattice (linear exactness, which fails for a wrong stagger), and a brute-force
sum of the tent kernel over every lattice point (which fails for a wrong index
order or a transposed axis).
"""
import numpy as np
import pytest

STAG = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5],
                 [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


def _grid(orc, n=(8, 6, 5)):
    return orc.make_grid(n, (1.0, 1.0, 1.0), 0.2, 1)


def test_partition_of_unity(orc):
    g = _grid(orc)
    rng = np.random.default_rng(1)
    nc = 8 * 6 * 5
    EB = [np.full(nc, 1.0 + c) for c in range(6)]
    for _ in range(200):
        xp = rng.random(3) * np.array([8, 6, 5])
        out = orc.gather(g, EB, xp)
        np.testing.assert_allclose(out, 1.0 + np.arange(6), rtol=2e-15, atol=0)
    # positions on the periodic seam and on integer / half-integer planes
    for xp in ([0.0, 0.0, 0.0], [7.999999999999999, 5.5, 0.5], [0.5, 0.25, 4.75]):
        out = orc.gather(g, EB, np.array(xp))
        np.testing.assert_allclose(out, 1.0 + np.arange(6), rtol=2e-15, atol=0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_field_exact_on_own_lattice(orc, axis):
    """F_c(r) = alpha * r_axis + beta sampled at the component's own staggered
    points is reproduced exactly (to rounding) away from the seam."""
    n = (12, 12, 12)
    g = orc.make_grid(n, (1.0, 1.0, 1.0), 0.2, 1)
    k, j, i = np.meshgrid(np.arange(12), np.arange(12), np.arange(12), indexing="ij")
    idx = [i, j, k]
    EB = []
    alpha = [0.3, -1.7, 2.5, 0.9, -0.4, 1.1]
    for c in range(6):
        coord = idx[axis] + STAG[c][axis]
        EB.append((alpha[c] * coord + 10.0 + c).ravel().astype(np.float64))
    rng = np.random.default_rng(2)
    for _ in range(300):
        xp = 2.0 + rng.random(3) * 8.0   # stays away from the wrap in every axis
        out = orc.gather(g, EB, xp)
        want = np.array([alpha[c] * xp[axis] + 10.0 + c for c in range(6)])
        np.testing.assert_allclose(out, want, rtol=0, atol=2e-14)


def _tent(r):
    return np.maximum(0.0, 1.0 - np.abs(r))


def test_brute_force_tent_sum(orc):
    """F_p = sum over every lattice point of W(x-X) W(y-Y) W(z-Z) F, with the
    minimum-image distance on the periodic lattice."""
    n = (7, 5, 6)
    g = orc.make_grid(n, (1.0, 1.0, 1.0), 0.2, 1)
    rng = np.random.default_rng(3)
    nc = n[0] * n[1] * n[2]
    EB = [rng.standard_normal(nc) for _ in range(6)]
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    L = np.array(n, dtype=np.float64)
    for _ in range(16):
        xp = rng.random(3) * L
        out = orc.gather(g, EB, xp)
        for c in range(6):
            X = (i + STAG[c][0]).ravel()
            Y = (j + STAG[c][1]).ravel()
            Z = (k + STAG[c][2]).ravel()
            d = []
            for dim, P in enumerate((X, Y, Z)):
                r = xp[dim] - P
                r = r - L[dim] * np.round(r / L[dim])
                d.append(r)
            w = _tent(d[0]) * _tent(d[1]) * _tent(d[2])
            want = np.sum(w * EB[c])
            assert abs(out[c] - want) <= 1e-14 * max(1.0, np.sum(np.abs(w * EB[c])))
