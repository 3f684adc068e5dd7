"""Exact-arithmetic reference for tiny inputs: TEST INFRASTRUCTURE ONLY.

Binary32 coordinates are dyadic rationals, so every quantity of Definition 1 has
an exact value that Python's ``fractions.Fraction`` can hold.  This module gives
two independent things:

* the real-number certificate (exact squared distances, nearest neighbour with
  exact ties to the lowest index, exact second smallest squared distance);
* an emulation of the binary32 certificate formula in which every operation is
  done exactly and then rounded to the nearest binary32 value (ties to even) by
  ``round_f32`` below, so that the C oracle's arithmetic can be checked bit by bit
  without trusting any floating-point unit.

It is slow on purpose and meant for N of a few dozen at most.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

_EMIN = -126          # smallest normal exponent of binary32
_P = 24               # significand bits
_MAXF = Fraction((2 ** _P - 1) * 2 ** (127 - _P + 1))


def exact(x) -> Fraction:
    """Exact value of a binary32 (or any finite float)."""
    return Fraction(float(x))


def round_f32(x: Fraction) -> Fraction:
    """Round an exact rational to the nearest binary32 value, ties to even."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = -x if x < 0 else x
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, _EMIN)                      # subnormals share the smallest quantum
    quantum = Fraction(2) ** (e - _P + 1)
    q = a / quantum
    lo = q.numerator // q.denominator
    rem = q - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    r = lo * quantum
    if r > _MAXF:
        raise OverflowError("binary32 overflow")
    return sign * r


def _next_up(r: Fraction) -> Fraction:
    return exact(np.nextafter(np.float32(float(r)), np.float32(np.inf)))


def _next_down(r: Fraction) -> Fraction:
    return exact(np.nextafter(np.float32(float(r)), np.float32(-np.inf)))


def sqrt_f32(s: Fraction) -> Fraction:
    """Correctly rounded binary32 square root of a non-negative binary32 value.

    The result r is the unique binary32 with (r_prev + r)/2 < sqrt(s) < (r + r_next)/2,
    checked by squaring the midpoints exactly (the square root of a binary32 is
    never a binary32 midpoint, so there are no ties)."""
    if s == 0:
        return Fraction(0)
    guess = np.float32(np.sqrt(float(s)))
    cands = [exact(guess)]
    cands.append(_next_up(cands[0]))
    cands.append(_next_down(cands[0]))
    hits = []
    for r in cands:
        lo = (_next_down(r) + r) / 2
        hi = (r + _next_up(r)) / 2
        if lo * lo < s < hi * hi:
            hits.append(r)
    if len(hits) != 1:
        raise ArithmeticError("square root bracketing failed")
    return hits[0]


def coords(pos: np.ndarray):
    """Exact coordinates, list over axes of lists over points."""
    return [[exact(v) for v in axis] for axis in np.asarray(pos, dtype=np.float32)]


def sqdist_real(P, i: int, j: int) -> Fraction:
    return sum(((ax[j] - ax[i]) ** 2 for ax in P), Fraction(0))


def sqdist_f32(P, i: int, j: int) -> Fraction:
    """The binary32 formula, each operation rounded: ((dx*dx) + (dy*dy)) + (dz*dz)."""
    s = None
    for ax in P:
        dk = round_f32(ax[j] - ax[i])
        sq = round_f32(dk * dk)
        s = sq if s is None else round_f32(s + sq)
    return s


def _top2(P, i: int, dist):
    n = len(P[0])
    best = []
    for j in range(n):
        if j != i:
            best.append((dist(P, i, j), j))
    if not best:
        return -1, None, None
    best.sort()                    # by value, then index: ties go to the lowest index
    s1, nn = best[0]
    s2 = best[1][0] if len(best) > 1 else None
    return nn, s1, s2


def top2_real(P, i: int):
    """(nn, S1, S2) with exact squared distances; None stands for +inf."""
    return _top2(P, i, sqdist_real)


def top2_f32(P, i: int):
    """(nn, d1, d2) under the binary32 formula, d = correctly rounded sqrt; None = +inf."""
    nn, s1, s2 = _top2(P, i, sqdist_f32)
    d1 = None if s1 is None else sqrt_f32(s1)
    d2 = None if s2 is None else sqrt_f32(s2)
    return nn, d1, d2
