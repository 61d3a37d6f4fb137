"""Pins of the oracle's scalar arithmetic (oracle/mpnum.py, oracle/c/mpref.c).

The oracle's rounding is checked against two things it does not share code
with:

* brute force: at p = 4, 5 and 6 every p-bit value over a wide exponent range
  is listed, and the nearest one to the exact result (ties to the even
  mantissa) is looked up in that list;
* mpmath.libmp, an independent implementation of round-to-nearest-even
  binary arithmetic, at p = 128, 256 and 512 on random and adversarial
  operands.
"""

import bisect
import random
from fractions import Fraction

import numpy as np
import pytest
from mpmath import libmp

from oracle import mpnum, cref
from paper_1410_1599_amd import inputs as I

from helpers import adversarial_pairs, random_value


# ------------------------------------------------------------- brute force

def all_values(p, emin, emax):
    """Every positive p-bit value M 2**(e-p), sorted, with its mantissa."""
    vals = []
    for e in range(emin, emax + 1):
        for M in range(1 << (p - 1), 1 << p):
            vals.append((Fraction(M) * Fraction(2) ** (e - p), M, e))
    vals.sort()
    return vals


def brute_nearest(x, table, keys):
    """Nearest entry of the table to the Fraction x, ties to even mantissa."""
    if x == 0:
        return (0, 0)
    a = abs(x)
    i = bisect.bisect_left(keys, a)
    cands = [table[j] for j in (i - 1, i) if 0 <= j < len(table)]
    best = None
    for v, M, e in cands:
        d = abs(v - a)
        key = (d, M & 1)
        if best is None or key < best[0]:
            best = (key, M, e)
    _, M, e = best
    return (-M if x < 0 else M, e)


@pytest.mark.parametrize("p", [4, 5, 6])
def test_brute_force_small_p(p):
    table = all_values(p, -3 * p - 8, 3 * p + 8)
    keys = [t[0] for t in table]
    mants = list(range(1 << (p - 1), 1 << p))
    rng = random.Random(p)
    F = lambda v: mpnum.to_fraction(v, p)
    count = 0
    for mx in mants:
        for my in mants:
            for gap in list(range(0, p + 6)):
                for sx in (1, -1):
                    for sy in (1, -1):
                        x = (sx * mx, 0)
                        y = (sy * my, -gap)
                        for xx, yy in ((x, y), (y, x)):
                            assert mpnum.add(xx, yy, p) == brute_nearest(F(xx) + F(yy), table, keys)
                            assert mpnum.sub(xx, yy, p) == brute_nearest(F(xx) - F(yy), table, keys)
                        assert mpnum.mul(x, y, p) == brute_nearest(F(x) * F(y), table, keys)
                        assert mpnum.div(x, y, p) == brute_nearest(F(x) / F(y), table, keys)
                        count += 1
    assert count == len(mants) ** 2 * (p + 6) * 4
    # zero operands
    z = mpnum.ZERO
    x = (mants[-1], 2)
    assert mpnum.add(z, x, p) == x and mpnum.add(x, z, p) == x
    assert mpnum.sub(x, x, p) == z and mpnum.mul(x, z, p) == z and mpnum.div(z, x, p) == z


def test_rn_of_integers_brute():
    p = 5
    table = all_values(p, -2, 14)
    keys = [t[0] for t in table]
    for v in range(-3000, 3001):
        assert mpnum.from_int(v, p) == brute_nearest(Fraction(v), table, keys), v


def test_from_fraction_brute():
    p = 6
    table = all_values(p, -20, 12)
    keys = [t[0] for t in table]
    for q in range(1, 400):
        for num in (1, 3, -7, 1000):
            x = Fraction(num, q)
            assert mpnum.from_fraction(x, p) == brute_nearest(x, table, keys), (num, q)


# ------------------------------------------------------------- mpmath

def to_mpf(v, p):
    sig, e = v
    return libmp.from_man_exp(sig, e - p) if sig else libmp.fzero


@pytest.mark.parametrize("p", [128, 256, 512])
def test_against_mpmath(p):
    rng = random.Random(1000 + p)
    pairs = adversarial_pairs(rng, p) + [(random_value(rng, p), random_value(rng, p)) for _ in range(3000)]
    for x, y in pairs:
        X, Y = to_mpf(x, p), to_mpf(y, p)
        assert to_mpf(mpnum.add(x, y, p), p) == libmp.mpf_add(X, Y, p, "n")
        assert to_mpf(mpnum.sub(x, y, p), p) == libmp.mpf_sub(X, Y, p, "n")
        assert to_mpf(mpnum.mul(x, y, p), p) == libmp.mpf_mul(X, Y, p, "n")
        if y[0]:
            assert to_mpf(mpnum.div(x, y, p), p) == libmp.mpf_div(X, Y, p, "n")


def test_mpmath_rounds_ties_to_even():
    # the property the mpmath pin relies on: at p = 2, 1 + 1/4 -> 1 and 1 + 3/4 -> 2
    one = libmp.from_int(1)
    assert libmp.mpf_add(one, libmp.from_man_exp(1, -2), 2, "n") == one
    assert libmp.mpf_add(one, libmp.from_man_exp(3, -2), 2, "n") == libmp.from_int(2)


@pytest.mark.parametrize("p", [128, 256])
def test_add_shortcut_matches_exact_sum(p):
    """add() returns the larger operand for a gap >= p + 3; compare with the
    exact aligned sum rounded once."""
    rng = random.Random(7)
    one = 1 << (p - 1)
    for gap in range(p + 3, p + 12):
        for mx in (one, one + 1, (1 << p) - 1, rng.randrange(one, 1 << p)):
            for s in (1, -1):
                x = (mx, 0)
                y = (s * rng.randrange(one, 1 << p), -gap)
                n = (x[0] << gap) + y[0]
                assert mpnum.add(x, y, p) == mpnum.rn(n, -gap - p, p)
                assert mpnum.add(y, x, p) == mpnum.rn(n, -gap - p, p)


# ------------------------------------------------------------- C oracle

def rec(v, p):
    a = I.empty(1, 1, p)
    I.set_entry(a, 0, 0, v, p)
    return a.reshape(-1).copy()


def unrec(r, p):
    return I.entry(r.reshape(p // 32 + 2, 1, 1), 0, 0, p)


@pytest.mark.parametrize("p", [128, 256, 512])
def test_c_oracle_scalar_matches_python(p):
    rng = random.Random(77 + p)
    pairs = adversarial_pairs(rng, p)[:400] + [(random_value(rng, p), random_value(rng, p)) for _ in range(400)]
    for x, y in pairs:
        for op, f in (("mul", mpnum.mul), ("add", mpnum.add), ("sub", mpnum.sub), ("div", mpnum.div)):
            if op == "div" and y[0] == 0:
                continue
            got = unrec(cref.scalar(op, p, rec(x, p), rec(y, p)), p)
            assert got == f(x, y, p), (op, x, y)
