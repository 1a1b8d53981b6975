"""The device sin/cos of the orbital phase (track_sincos in csrc/bsh_internal.h) pinned to the
mathematics: its constants are read from the source and checked against pi/2 and 1/n! computed
here from first principles, and its method (Cody-Waite reduction by pi/2, Taylor series on
[-pi/4, pi/4], quadrant selection), evaluated with those constants in float64, is checked
against numpy's sin/cos over the phases the tracks use.  The GPU kernels' bins are checked
against the oracle by the parity tests; this pins the constants a typo could spoil."""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1904_04873_amd", "csrc", "bsh_internal.h")


def _pi() -> Fraction:
    # Machin: pi = 16 atan(1/5) - 4 atan(1/239), to 70 digits
    getcontext().prec = 80

    def atan_inv(n):
        x = Decimal(1) / n
        x2, s, t, k = x * x, x, x, 1
        while True:
            t *= -x2
            k += 2
            if abs(t / k) < Decimal(10) ** -75:
                return s
            s += t / k

    return Fraction(16 * atan_inv(5) - 4 * atan_inv(239))


def _constants():
    body = open(SRC).read()
    body = body[body.index("void track_sincos("):]
    body = body[: body.index("\n}\n")]
    lits = re.findall(r"(-?0x[0-9a-f.]+p[-+]?\d+|-0\.5)", body)
    vals = [float.fromhex(v) if "x" in v else float(v) for v in lits]
    assert len(vals) == 4 + 7 + 8, len(vals)
    return vals[0], vals[1:4], vals[4:11], vals[11:19]


def _significant_bits(x: float) -> int:
    m, _ = math.frexp(abs(x))
    f = Fraction(m)
    bits = 0
    while f.denominator != 1:
        f *= 2
        bits += 1
    return bits


def test_reduction_constants():
    two_over_pi, (p1, p2, p3), _, _ = _constants()
    pi = _pi()
    assert two_over_pi == float(2 / pi)
    assert _significant_bits(p1) <= 33 and _significant_bits(p2) <= 33
    assert abs(Fraction(p1) + Fraction(p2) + Fraction(p3) - pi / 2) < Fraction(1, 10 ** 33)


def test_taylor_coefficients():
    _, _, ps, pc = _constants()
    # ps: -1/15!, 1/13!, ..., -1/3!; pc: 1/16!, -1/14!, ..., -1/2!
    want_s = [(-1) ** ((n - 1) // 2) / math.factorial(n) for n in (15, 13, 11, 9, 7, 5, 3)]
    want_c = [(-1) ** (n // 2) / math.factorial(n) for n in (16, 14, 12, 10, 8, 6, 4, 2)]
    assert ps == [float(Fraction((-1) ** ((n - 1) // 2), math.factorial(n))) for n in (15, 13, 11, 9, 7, 5, 3)]
    assert pc == [float(Fraction((-1) ** (n // 2), math.factorial(n))) for n in (16, 14, 12, 10, 8, 6, 4, 2)]
    assert np.allclose(ps, want_s, rtol=1e-15) and np.allclose(pc, want_c, rtol=1e-15)


def _method(x, consts):
    two_over_pi, (p1, p2, p3), ps_c, pc_c = consts
    k = np.rint(x * two_over_pi)
    r = x - k * p1          # exact: k p1 has at most 53 bits and cancels against x
    r = r - k * p2
    r = r - k * p3
    r2 = r * r
    ps = np.full_like(r, ps_c[0])
    for a in ps_c[1:]:
        ps = ps * r2 + a
    sr = r + (r * r2) * ps
    pc = np.full_like(r, pc_c[0])
    for a in pc_c[1:]:
        pc = pc * r2 + a
    cr = 1.0 + r2 * pc
    q = k.astype(np.int64) & 3
    s0 = np.where(q & 1, cr, sr)
    c0 = np.where(q & 1, sr, cr)
    return np.where(q & 2, -s0, s0), np.where((q + 1) & 2, -c0, c0)


def test_method_accuracy_over_track_phases():
    consts = _constants()
    rng = np.random.default_rng(190404873)
    # W t for P in [15, 45] d and |t| up to 240 d, plus multiples of pi/2 and their neighbours
    x = np.concatenate([rng.uniform(-110.0, 110.0, 400_000), rng.uniform(-1.0, 1.0, 50_000),
                        np.arange(-70, 71) * (np.pi / 2),
                        np.nextafter(np.arange(-70, 71) * (np.pi / 2), np.inf)])
    s, c = _method(x, consts)
    assert np.max(np.abs(s - np.sin(x))) < 4e-16
    assert np.max(np.abs(c - np.cos(x))) < 4e-16
    # the reduction is exact in its first step, so the error does not grow with |x| in range
    big = rng.uniform(900.0, 1000.0, 50_000)
    s, c = _method(big, consts)
    assert np.max(np.abs(s - np.sin(big))) < 1e-15 and np.max(np.abs(c - np.cos(big))) < 1e-15
