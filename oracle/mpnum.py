"""Reference p-bit binary floating-point arithmetic, round to nearest, ties to even.

TEST INFRASTRUCTURE ONLY.  This package is the oracle that the GPU path is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import it; the library never does.

The paper computes every scalar operation with MPFR at a fixed mantissa
length, rounding to nearest (Section 3, test environment).  A value here is a
pair ``(sig, e)`` of Python ints with

    value = sig * 2**(e - p),   2**(p-1) <= |sig| < 2**p,   or  (0, 0) for zero.

This is MPFR's normalisation (mantissa in [1/2, 1), exponent e).  There is a
single zero, +0 (the paper is silent on signed zeros).  The exponent is
unbounded: no overflow or underflow exists in this model.

Every operation forms the exact result as an integer times a power of two and
rounds it once with :func:`rn`.  Nothing here is fast; everything is meant to
be checked by eye.

Parity pins (tests/test_oracle_scalar.py): brute-force nearest search over all
p-bit candidates for p = 4..8, and mpmath.libmp's independent round-to-nearest
at p = 128..512.
"""

ZERO = (0, 0)


def rn(n, f, p):
    """Round the exact value n * 2**f (n, f ints) to the nearest p-bit value.

    Ties go to the even mantissa.  Returns ``(sig, e)``.
    """
    if n == 0:
        return ZERO
    neg = n < 0
    a = -n if neg else n
    b = a.bit_length()
    if b > p:
        s = b - p                       # bits that do not fit
        q = a >> s                      # kept p bits
        r = a - (q << s)                # dropped bits
        half = 1 << (s - 1)
        if r > half or (r == half and (q & 1)):
            q += 1
            if q == 1 << p:             # rounded up to the next binade
                q >>= 1
                s += 1
        a, f = q, f + s
    else:
        a, f = a << (p - b), f - (p - b)
    # now value = a * 2**f with 2**(p-1) <= a < 2**p, so e - p = f
    return (-a if neg else a, f + p)


def is_zero(x):
    return x[0] == 0


def neg(x):
    return (-x[0], x[1])


def mul(x, y, p):
    """RN(x * y): the exact product has at most 2p bits."""
    if x[0] == 0 or y[0] == 0:
        return ZERO
    return rn(x[0] * y[0], (x[1] - p) + (y[1] - p), p)


def add(x, y, p):
    """RN(x + y).

    The exact sum is formed by aligning both mantissas to the smaller
    exponent.  When the exponent gap is p + 3 or more the smaller operand is
    below a quarter of an ulp of the larger one (a quarter, not a half, so
    that the case where the larger operand is a power of two and the smaller
    one is subtracted is covered too), and the rounded result is the larger
    operand itself; this keeps the integers small for wildly different
    magnitudes.  tests/test_oracle_scalar.py checks this shortcut against the
    exact computation.
    """
    if x[0] == 0:
        return y
    if y[0] == 0:
        return x
    if x[1] - y[1] >= p + 3:
        return x
    if y[1] - x[1] >= p + 3:
        return y
    e0 = min(x[1], y[1])
    n = (x[0] << (x[1] - e0)) + (y[0] << (y[1] - e0))
    return rn(n, e0 - p, p)


def sub(x, y, p):
    """RN(x - y)."""
    return add(x, neg(y), p)


def div(x, y, p):
    """RN(x / y), correctly rounded (not reciprocal then multiply).

    The integer quotient of the mantissas is taken with p + 2 or more bits and
    the remainder is folded into one extra sticky bit below them, so the
    single rounding in :func:`rn` sees the same side of every midpoint as the
    exact quotient does.
    """
    if y[0] == 0:
        raise ZeroDivisionError("oracle div by zero")
    if x[0] == 0:
        return ZERO
    ax, ay = abs(x[0]), abs(y[0])
    k = p + 3
    q, r = divmod(ax << k, ay)          # q has p + 3 or p + 4 bits
    n = (q << 1) | (1 if r else 0)
    if (x[0] < 0) != (y[0] < 0):
        n = -n
    # x / y = (ax / ay) * 2**(ex - ey);  ax / ay ~ n * 2**-(k + 1)
    return rn(n, x[1] - y[1] - k - 1, p)


def cmp_abs(x, y):
    """Compare |x| and |y| exactly; returns -1, 0 or 1."""
    if x[0] == 0 or y[0] == 0:
        ax, ay = (x[0] != 0), (y[0] != 0)
        return (ax > ay) - (ax < ay)
    if x[1] != y[1]:
        return 1 if x[1] > y[1] else -1
    a, b = abs(x[0]), abs(y[0])
    return (a > b) - (a < b)


def from_int(v, p):
    """Nearest p-bit value to the integer v."""
    return rn(v, 0, p)


def from_fraction(q, p):
    """Nearest p-bit value to the rational q (a fractions.Fraction)."""
    num, den = q.numerator, q.denominator
    if num == 0:
        return ZERO
    if den == 1:
        return rn(num, 0, p)
    # scale so the integer quotient has at least p + 2 bits, then fold the
    # remainder into a sticky bit, exactly as div() does
    k = max(0, p + 3 - (abs(num).bit_length() - den.bit_length()))
    qq, r = divmod(abs(num) << k, den)
    n = (qq << 1) | (1 if r else 0)
    if num < 0:
        n = -n
    return rn(n, -k - 1, p)


def to_fraction(x, p):
    from fractions import Fraction
    sig, e = x
    if sig == 0:
        return Fraction(0)
    sh = e - p
    return Fraction(sig * (1 << sh)) if sh >= 0 else Fraction(sig, 1 << (-sh))


def to_float(x, p):
    """Nearest double (for reporting only)."""
    return float(to_fraction(x, p))


def ulp(x, p):
    """Exponent of one ulp of x: ulp(x) = 2**(e - p) for nonzero x."""
    return x[1] - p
