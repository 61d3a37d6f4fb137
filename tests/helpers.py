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


def division_stress_matrix(p, n, K, seed):
    """First K columns lower triangular: a_jj is a divisor built to strain the
    radix-2^32 digit estimate, the entries below it are dividends of smaller
    magnitude, the entries above it zero (so no earlier step changes column j
    and its pivot is row j).  Columns from K on are uniform in [-1, 1)."""
    rng = random.Random(seed)
    A = I.uniform_pm1(n, n, p, seed)
    one, full = 1 << (p - 1), (1 << p) - 1
    zero = (0, 0)
    top_equal = 0
    for j in range(K):
        run = rng.randrange(1, p - 64)
        kind = j % 3
        if kind == 0:                    # 1 0...0 1...1: top limbs 2^31, 0
            my = one | ((1 << run) - 1)
        elif kind == 1:                  # 1...1 0...0
            my = full ^ ((1 << run) - 1)
        else:
            my = rng.randrange(one + 1, 1 << p)
        ey = rng.randrange(-3, 4)
        I.set_entry(A, j, j, (my if rng.random() < 0.5 else -my, ey), p)
        for i in range(j):
            I.set_entry(A, i, j, zero, p)
        for i in range(j + 1, n):
            pick = (i + j) % 5
            if pick == 0:                # just below the divisor: the same top limbs
                mx, ex = max(one, my - rng.randrange(1, 1 << 16)), ey
            elif pick == 1:              # 1 0...0 over a divisor with ones below its top bit
                mx, ex = one, ey
            elif pick == 2:
                mx, ex = rng.randrange(one, 1 << p), ey - 1
            elif pick == 3:              # the divisor's top 64 bits over smaller low bits
                low = my & ((1 << (p - 64)) - 1)
                mx, ex = (my ^ low) | rng.randrange(0, low + 1), ey
                mx = mx if mx < my else my - 1
            else:
                mx, ex = 0, 0
            if mx == 0:
                I.set_entry(A, i, j, zero, p)
                continue
            assert one <= mx < (1 << p) and (ex < ey or mx < my)     # |a_ij| < |a_jj|
            top_equal += (mx >> (p - 64)) == (my >> (p - 64))
            I.set_entry(A, i, j, (mx if rng.random() < 0.5 else -mx, ex), p)
    return A, top_equal
