"""GPU parity on the edge cases of the CIC gather and the VB split (Section 3:
CIC form factor, charge-conserving Villasenor-Buneman deposition).

The oracle pins of these cases (tests/test_oracle_vb.py, test_oracle_gather.py,
test_oracle_mixed.py) exercise the oracle alone; here the same kinds of moves
run through the HIP kernels and are compared with the oracle's step from the
same state (the protocol of gpu_parity_util):

* moves that end exactly on a cell plane (one, two and three axes), that start
  exactly on a plane, that cross two or three planes at the same time (ties,
  resolved in axis order), corner crossings, crossings of the periodic seam,
  and moves that end exactly on x = L (stored as 0) or exactly on x = 0;
* particles whose interpolation stencil switches: positions exactly on
  integer and half-integer planes, with non-zero fields;
* FP32-mixed: positions whose FP32 offset rounds to 1 (the guard that moves
  them to the next cell with offset 0), and the same plane cases.

The exact end positions are built with the oracle's own per-particle advance
(zero fields leave the momentum unchanged), searching the momentum until the
end position is the wanted plane bit for bit; the inputs therefore come from
the oracle, never from the GPU library.
"""
import numpy as np
import pytest

import oracle
from paper_1608_01009_amd import workloads as W

from gpu_parity_util import one_step_parity
from test_gpu_mixed import _against_mixed_oracle, _run

pytestmark = pytest.mark.gpu

N = (8, 8, 8)
DT = W.courant_dt()


def _grid():
    return oracle.make_grid(N, (1.0, 1.0, 1.0), DT, 4)


def _end(g, x0, u):
    return oracle.advance(g, np.asarray(u, dtype=np.float64), np.asarray(x0, dtype=np.float64))


def _hit(g, x0, u, d, target):
    """Momentum with u[d] adjusted so that the advance of x0 ends exactly on
    target along axis d (the other components fixed): bisection on u[d] for
    one value that lands, then for the ends of the interval of values that
    land (the advance rounds a range of momenta to the same position); the
    middle of that interval is returned, so that the small change of gamma
    from adjusting another component keeps this one on target."""
    u = np.array(u, dtype=np.float64)
    sgn = 1.0 if target > x0[d] else -1.0

    def f(v):
        uu = u.copy()
        uu[d] = v
        return _end(g, x0, uu)[d]

    def below(v):   # f(v) on the near side of the target
        return (f(v) < target) if sgn > 0 else (f(v) > target)

    lo, hi = 0.0, sgn * 50.0
    hit = None
    while True:
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        fm = f(mid)
        if fm == target:
            hit = mid
            break
        if below(mid):
            lo = mid
        else:
            hi = mid
    assert hit is not None, f"no momentum reaches {target} from {x0[d]} on axis {d}"
    a, b = lo, hit          # first value that lands: in (a, b]
    while True:
        mid = 0.5 * (a + b)
        if mid == a or mid == b:
            break
        if f(mid) == target:
            b = mid
        else:
            a = mid
    first = b
    a, b = hit, hi          # last value that lands: in [a, b)
    while True:
        mid = 0.5 * (a + b)
        if mid == a or mid == b:
            break
        if f(mid) == target:
            a = mid
        else:
            b = mid
    u[d] = 0.5 * (first + a)
    assert f(u[d]) == target
    return u


def _cases():
    g = _grid()
    P = []   # (x0, u)

    def add(x0, u):
        P.append((np.array(x0, dtype=np.float64), np.array(u, dtype=np.float64)))

    # end exactly on a plane: along each axis, upwards (into the next cell)
    # and downwards (onto the cell's own lower plane)
    for d in range(3):
        x0 = np.array([2.875, 3.6875, 4.8125])
        x0[d] = 2.875
        add(x0, _hit(g, x0, [0.01, -0.02, 0.015], d, 3.0))
        x0[d] = 2.125
        add(x0, _hit(g, x0, [0.01, -0.02, 0.015], d, 2.0))
    # all three axes end on planes (a corner): the three components are
    # adjusted in turn until every one lands (each changes gamma)
    x0 = np.array([2.875, 3.8125, 4.9375])
    target = np.floor(x0) + 1.0
    v = (target - x0) / DT
    u = v / np.sqrt(1.0 - v @ v)        # the momentum of the straight move
    for _ in range(50):
        for d in range(3):
            u = _hit(g, x0, u, d, target[d])
        if np.array_equal(_end(g, x0, u), target):
            break
    assert np.array_equal(_end(g, x0, u), target)
    add(x0, u)
    # start exactly on a plane, moving down (crossing it at t = 0) and up
    add([3.0, 4.5, 5.25], [-0.4, 0.1, 0.05])
    add([3.0, 4.0, 5.0], [-0.3, -0.3, -0.3])
    add([3.0, 4.0, 5.0], [0.3, 0.3, 0.3])
    # ties: identical fractional offsets and momenta in one binade ([4, 8))
    add([4.875, 5.875, 6.5], [0.9, 0.9, 0.01])        # x and y cross together
    add([4.875, 5.875, 6.875], [0.9, 0.9, 0.9])       # x, y and z together
    add([4.125, 5.125, 6.125], [-0.9, -0.9, -0.9])    # downwards, three together
    add([4.875, 5.875, 6.95], [0.9, 0.9, 0.9])        # x, y tie, z earlier
    add([4.875, 5.5, 6.875], [0.9, 0.02, 0.9])        # x, z tie
    # corner crossing with distinct times
    add([4.9, 5.85, 6.8], [1.1, 1.1, 1.1])
    add([4.1, 5.15, 6.2], [-1.1, -1.1, -1.1])
    # the periodic seam, crossed up and down in every axis
    add([7.9, 0.05, 7.95], [0.9, -0.9, 0.9])
    add([0.03, 7.96, 0.02], [-0.9, 0.9, -0.9])
    # ending exactly on x = L (stored as 0), and just below 0 by less than
    # half a unit of L (the wrap x + L rounds to L: also stored as 0)
    for d in range(3):
        x0 = np.array([3.5, 3.5, 3.5])
        x0[d] = 7.875
        add(x0, _hit(g, x0, [0.0, 0.0, 0.0], d, 8.0))
        x0 = np.array([3.5, 3.5, 3.5])
        x0[d] = 0.125
        add(x0, _just_below_zero(g, x0, d))
    return P


def _just_below_zero(g, x0, d):
    """Momentum along -d whose advance of x0 ends in (-ulp(L)/2, 0)."""
    def f(v):
        u = np.zeros(3)
        u[d] = v
        return _end(g, x0, u)[d]
    lo, hi = 0.0, -50.0          # f(lo) > 0 >= f(hi)
    while True:
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    v = hi
    while f(v) == 0.0:
        v = np.nextafter(v, -np.inf)
    e = f(v)
    assert e < 0.0 and e + N[d] == N[d], e
    u = np.zeros(3)
    u[d] = v
    return u


def _workload(parts, fields, name):
    x0 = np.array([p[0] for p in parts])
    u = np.array([p[1] for p in parts])
    sp = W.Species(-1.0, 1.0, 0.3, x0[:, 0].copy(), x0[:, 1].copy(), x0[:, 2].copy(),
                   u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy())
    return W.Workload(name, N, (1.0, 1.0, 1.0), DT, 4, 20, 4, [sp], fields)


def _check_targets(parts):
    # the constructed endpoints are what they claim, by the oracle's advance
    g = _grid()
    ends = [_end(g, x0, u) for x0, u in parts]
    on_plane = sum(int(np.any(e == np.round(e))) for e in ends)
    assert on_plane >= 10, on_plane
    assert any(e[0] == 8.0 for e in ends)
    assert any(e[0] < 0.0 and e[0] + 8.0 == 8.0 for e in ends)


def test_vb_edge_moves_fp64():
    parts = _cases()
    _check_targets(parts)
    zero = [np.zeros(512) for _ in range(6)]
    reps, sim = one_step_parity(_workload(parts, zero, "vb-edges"), [0, 1])
    sim.close()


def test_gather_on_stencil_planes_fp64():
    # integer and half-integer planes switch the lower index of the two
    # staggers; non-zero fields make a wrong stencil visible
    pos = []
    for a in (3.0, 3.5, 0.0, 7.5, 4.25):
        for b in (4.0, 4.5, 0.0, 7.5):
            for c in (5.0, 5.5, 0.0):
                pos.append([a, b, c])
    rng = np.random.default_rng(90)
    parts = [(np.array(p), rng.normal(0.0, 0.05, 3)) for p in pos]
    fields = [rng.uniform(-0.05, 0.05, 512) for _ in range(6)]
    reps, sim = one_step_parity(_workload(parts, fields, "gather-planes"), [0])
    sim.close()


def test_vb_edge_moves_and_offset_guard_mixed():
    parts = _cases()
    # offsets that round to 1 in FP32 at load (moved to the next cell with
    # offset 0), in every axis and at the seam
    for x0 in ([3.0 + (1.0 - 2.0 ** -25), 4.5, 5.5], [2.5, 4.0 + (1.0 - 2.0 ** -30), 5.5],
               [2.5, 4.5, 7.0 + (1.0 - 2.0 ** -26)], [7.0 + (1.0 - 2.0 ** -40), 0.5, 0.5]):
        parts.append((np.array(x0), np.array([0.05, -0.03, 0.02])))
    # offsets just below 1 moving up by less than an FP32 unit of the offset
    for k in range(8):
        parts.append((np.array([2.0 + (1.0 - 2.0 ** -24 * (k + 1)), 4.5, 5.5]),
                      np.array([1e-7 * (k + 1), 0.0, 0.0])))
    rng = np.random.default_rng(91)
    fields = [rng.uniform(-1e-3, 1e-3, 512) for _ in range(6)]
    _run(_workload(parts, fields, "mixed-edges"), [0, 1], _against_mixed_oracle)
