"""Exact rational model of IEEE-754 binary32 round-to-nearest-even.

Used to check that the compiled float32 oracle evaluates its point-distance
expression exactly as written: every operation is computed exactly with
fractions and rounded once to binary32 (the explicit fused multiply-adds are
rounded once for the whole a*b+c).  No compiler, no hardware rounding mode.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

_EMIN = -126
_P = 24


def _floor_log2(q: Fraction) -> int:
    # q > 0
    e = q.numerator.bit_length() - q.denominator.bit_length()
    if Fraction(2) ** e > q:
        e -= 1
    elif Fraction(2) ** (e + 1) <= q:
        e += 1
    return e


def round32(q: Fraction) -> Fraction:
    """Round a rational to the nearest binary32 value, ties to even."""
    if q == 0:
        return Fraction(0)
    s = -1 if q < 0 else 1
    a = -q if q < 0 else q
    e = max(_floor_log2(a), _EMIN)
    ulp = Fraction(2) ** (e - (_P - 1))
    m = a / ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * ulp
    if r > Fraction(np.finfo(np.float32).max.item()):
        raise OverflowError("outside binary32 range")
    return s * r


def f(x) -> Fraction:
    """Exact value of a float32 (or float) number."""
    return Fraction(float(np.float32(x)))


def d2(a, b) -> Fraction:
    """dx = fl(ax-bx), ...; fl(dz*dz + fl(dy*dy + fl(dx*dx)))."""
    dx = round32(f(a[0]) - f(b[0]))
    dy = round32(f(a[1]) - f(b[1]))
    dz = round32(f(a[2]) - f(b[2]))
    t = round32(dx * dx)
    t = round32(dy * dy + t)
    return round32(dz * dz + t)


def pair(a, b):
    """(direct max, inverse max) of the float32 squared point distances."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    md = max(d2(a[i], b[i]) for i in range(21))
    mi = max(d2(a[i], b[20 - i]) for i in range(21))
    return md, mi


def to_f32(q: Fraction) -> np.float32:
    v = np.float32(float(q))
    assert Fraction(float(v)) == q, "value is not a binary32 number"
    return v
