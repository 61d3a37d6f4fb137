"""Helpers shared by the tests: adversarial scalar operands and plane packing."""

import random

import numpy as np

from paper_1410_1599_amd import inputs as I


def random_value(rng, p, emin=-8, emax=8):
    return (rng.choice((1, -1)) * rng.randrange(1 << (p - 1), 1 << p), rng.randint(emin, emax))


def adversarial_pairs(rng, p):
    """Operand pairs at the corners of rounding code: exponent gaps around 0,
    32 and p, extreme mantissas, exact ties, few-bit mantissas (exact
    products and ties), and full or near-full cancellation."""
    one = 1 << (p - 1)
    top = (1 << p) - 1
    out = []
    for gap in [0, 1, 2, 31, 32, 33, 63, 64, 65, p - 33, p - 32, p - 1, p, p + 1, p + 2, p + 3, p + 4,
                p + 31, p + 32, p + 33, 2 * p, 10 * p]:
        for mx in (one, top, rng.randrange(one, 1 << p)):
            for my in (one, top, rng.randrange(one, 1 << p), one | 1, top - 1):
                for s in (1, -1):
                    out.append(((mx, 5), (s * my, 5 - gap)))
    for mx in (one, one + 1, top, top - 1):
        out.append(((mx, 0), (one, -p)))
        out.append(((mx, 0), (-one, -p)))
    for _ in range(300):
        a = one | (1 << rng.randrange(0, p - 1))
        b = one | (1 << rng.randrange(0, p - 1)) | (1 << rng.randrange(0, p - 1))
        out.append(((rng.choice((1, -1)) * a, rng.randint(-3, 3)), (rng.choice((1, -1)) * b, rng.randint(-3, 3))))
    # products near a rounding midpoint: a * b with b = 2^(p-1) + small, a
    # with trailing ones, so the low half of the product is close to 1/2
    for _ in range(200):
        a = top - rng.randrange(0, 1 << 20)
        b = one + rng.randrange(0, 1 << 20)
        out.append(((a, 0), (b, 0)))
        out.append(((one + (1 << rng.randrange(0, p - 1)), 0), (top, 0)))
    for _ in range(60):
        m = rng.randrange(one, 1 << p)
        out.append(((m, 1), (-m, 1)))
        out.append(((m, 1), (-(m - 1 if m > one else m + 1), 1)))
        out.append(((m, 1), (-(m >> 1 | one), 0)))
    # gaps d = 32 + t past the guard limb where the aligned operand leaves the
    # guard limb empty below its top two bits, so that the bits shifted out
    # below the window (present or not) decide a tie or an exact result
    for t in (1, 2, 5, 31, 32, 33, 64, p - 64, p - 33, p - 32, p - 31, p - 2, p - 1):
        if t < 1 or t >= p:
            continue
        for top2 in (0, 1, 2, 3):
            for lost in (0, 1, 1 << (t - 1), rng.randrange(1, 1 << t)):
                my = one | lost
                if t + 30 < p:
                    my |= ((top2 & 1) << (t + 30))
                if t + 31 < p:
                    my |= ((top2 >> 1) << (t + 31))
                    my |= (rng.randrange(0, 1 << max(p - t - 32, 1)) << (t + 32)) & (top - ((1 << (t + 32)) - 1))
                my &= top
                my |= one
                for mx in (one, top, rng.randrange(one, 1 << p)):
                    for s in (1, -1):
                        out.append(((mx, 7), (s * my, 7 - 32 - t)))
    # zeros
    out.append(((0, 0), (one, 3)))
    out.append(((one, 3), (0, 0)))
    out.append(((0, 0), (0, 0)))
    return out


def vec_planes(vals, p):
    """A 1 x N matrix of the given (sig, e) values."""
    a = I.empty(1, len(vals), p)
    for j, v in enumerate(vals):
        I.set_entry(a, 0, j, v, p)
    return a


def planes_equal(X, Y):
    return X.shape == Y.shape and bool(np.array_equal(X, Y))


def first_mismatch(X, Y, p):
    """(i, j, got, want) of the first differing element, for messages."""
    L = p // 32
    diff = np.any(X != Y, axis=0)
    pos = np.argwhere(diff)
    if len(pos) == 0:
        return None
    i, j = (int(v) for v in pos[0])
    return (i, j, I.entry(X, i, j, p), I.entry(Y, i, j, p), int(diff.sum()))
