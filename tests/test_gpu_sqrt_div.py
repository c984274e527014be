"""The push's square root and division (the relativistic Boris step of
Section 2 takes sqrt(1 + |u|^2) and divides by it) against numpy's correctly
rounded IEEE FP64 square root and division, bit for bit, through the C ABI
(pic_eval_sqrt_div).

Operands: 2^24 random ones over the ranges the push uses (log-uniform
x in [1, 2^100], b in [1, 2^100], |a| in [2^-100, 2^100] with both signs),
plus 2^21 hard ones each, whose exact results lie within a few units of
2^-53 relative of a rounding boundary (the midpoint between two doubles):
  sqrt: x = the double nearest m^2 for a midpoint m = y + ulp(y) / 2,
  div:  a = the double nearest m * b for a midpoint m,
computed in numpy's extended precision.  Exact cases (perfect squares, b = 1,
a = 0, powers of two) are included too.
"""
import numpy as np
import pytest

from paper_1608_01009_amd import pic

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(2024)


def _loguniform(n, lo_exp, hi_exp):
    return np.exp2(RNG.uniform(lo_exp, hi_exp, n))


def _midpoints(n, lo_exp, hi_exp):
    y = _loguniform(n, lo_exp, hi_exp)
    return y, np.nextafter(y, np.inf)


def _hard_sqrt(n):
    y, y1 = _midpoints(n, 0.0, 50.0)
    m = (y.astype(np.longdouble) + y1.astype(np.longdouble)) / 2     # exact in 64 bits
    x = (m * m).astype(np.float64)
    return x[x >= 1.0]


def _hard_div(n):
    q, q1 = _midpoints(n, -60.0, 60.0)
    m = (q.astype(np.longdouble) + q1.astype(np.longdouble)) / 2
    b = _loguniform(n, 0.0, 40.0)
    a = (m * b.astype(np.longdouble)).astype(np.float64)
    sign = np.where(RNG.random(n) < 0.5, -1.0, 1.0)
    return a * sign, b


def test_sqrt_and_div_bit_exact():
    assert np.finfo(np.longdouble).nmant >= 63, "needs 64-bit extended precision"
    n = 1 << 24
    x = np.concatenate([_loguniform(n, 0.0, 100.0), _hard_sqrt(1 << 21),
                        np.arange(1.0, 4097.0) ** 2, [1.0, 2.0, 4.0, 2.0 ** 100]])
    a = np.concatenate([_loguniform(n, -100.0, 100.0) * np.where(RNG.random(n) < 0.5, -1, 1),
                        np.zeros(4)])
    b = np.concatenate([_loguniform(n, 0.0, 100.0), [1.0, 3.0, 2.0 ** 99, 1.5]])
    ha, hb = _hard_div(1 << 21)
    a = np.concatenate([a, ha, [1.0, -7.0, 2.0 ** -99, 2.0 ** 99]])
    b = np.concatenate([b, hb, [1.0, 1.0, 2.0, 4.0]])
    m = min(len(x), len(a))
    x, a, b = x[:m], a[:m], b[:m]
    sq, dv = pic.pic_eval_sqrt_div(x, a, b)
    ref_sq = np.sqrt(x)
    ref_dv = a / b
    bad_sq = np.flatnonzero(sq.view(np.int64) != ref_sq.view(np.int64))
    bad_dv = np.flatnonzero(dv.view(np.int64) != ref_dv.view(np.int64))
    assert bad_sq.size == 0, (bad_sq.size, x[bad_sq[:5]], sq[bad_sq[:5]], ref_sq[bad_sq[:5]])
    assert bad_dv.size == 0, (bad_dv.size, a[bad_dv[:5]], b[bad_dv[:5]], dv[bad_dv[:5]])
    print(f"sqrt and division bit for bit on {m} operands each")


def test_f32_sqrt_and_div_bit_exact():
    """The FP32 versions used by the mixed-precision push, against numpy's
    IEEE float32 square root and division: 2^24 random operands over their
    ranges (x in [1, 2^60], b in [1, 2^63], |a| in [2^-60, 2^60]) plus 2^21
    near-midpoint ones each (midpoints of two floats are exact in float64)."""
    n = 1 << 24
    x = np.exp2(RNG.uniform(0.0, 60.0, n)).astype(np.float32)
    y = np.exp2(RNG.uniform(0.0, 30.0, 1 << 21)).astype(np.float32)
    m = (y.astype(np.float64) + np.nextafter(y, np.float32(np.inf)).astype(np.float64)) / 2
    xh = (m * m).astype(np.float32)
    x = np.concatenate([x, xh[xh >= 1.0], np.arange(1, 4097, dtype=np.float32) ** 2,
                        np.array([1.0, 2.0, 4.0, 2.0 ** 60], dtype=np.float32)])
    a = (np.exp2(RNG.uniform(-60.0, 60.0, n)) *
         np.where(RNG.random(n) < 0.5, -1.0, 1.0)).astype(np.float32)
    b = np.exp2(RNG.uniform(0.0, 63.0, n)).astype(np.float32)
    q = np.exp2(RNG.uniform(-30.0, 30.0, 1 << 21)).astype(np.float32)
    qm = (q.astype(np.float64) + np.nextafter(q, np.float32(np.inf)).astype(np.float64)) / 2
    bh = np.exp2(RNG.uniform(0.0, 25.0, 1 << 21)).astype(np.float32)
    ah = (qm * bh.astype(np.float64)).astype(np.float32)
    a = np.concatenate([a, ah, np.array([0.0, 1.0, 2.0, -1.0], dtype=np.float32)])
    b = np.concatenate([b, bh, np.array([1.0, 3.0, 1.5, 2.0 ** 62], dtype=np.float32)])
    mlen = min(len(x), len(a))
    x, a, b = x[:mlen], a[:mlen], b[:mlen]
    sq, dv = pic.pic_eval_sqrt_div(x, a, b, f32=True)
    ref_sq = np.sqrt(x)
    ref_dv = a / b
    assert ref_sq.dtype == np.float32 and ref_dv.dtype == np.float32
    bad_sq = np.flatnonzero(sq.view(np.int32) != ref_sq.view(np.int32))
    bad_dv = np.flatnonzero(dv.view(np.int32) != ref_dv.view(np.int32))
    assert bad_sq.size == 0, (bad_sq.size, x[bad_sq[:5]], sq[bad_sq[:5]], ref_sq[bad_sq[:5]])
    assert bad_dv.size == 0, (bad_dv.size, a[bad_dv[:5]], b[bad_dv[:5]], dv[bad_dv[:5]])
    print(f"FP32 sqrt and division bit for bit on {mlen} operands each")
