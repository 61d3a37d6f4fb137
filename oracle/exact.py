"""Exact products and ulp error, the yardstick for the INT8-slice path.

TEST INFRASTRUCTURE ONLY (see oracle/mpnum.py).

The slice path does not follow the paper's per-operation rounding; it is
judged against the mathematically exact product, rounded once:
c_ij = RN_p(sum_k a_ik b_kj) with the sum taken exactly.  The error of a
result x in units in the last place is |x - c_ij| / ulp_p(c_ij) where
ulp_p(y) = 2**(floor(log2|y|) - p + 1).
"""

from fractions import Fraction

from . import mpnum


def exact_dot(row, col, p):
    """sum_k row[k] * col[k] exactly, as (n, f) with value n * 2**f."""
    terms = []
    for x, y in zip(row, col):
        if x[0] and y[0]:
            terms.append((x[0] * y[0], x[1] + y[1] - 2 * p))
    if not terms:
        return 0, 0
    f0 = min(f for _, f in terms)
    return sum(n << (f - f0) for n, f in terms), f0


def exact_entry(A, B, i, j, p):
    """RN_p of the exact c_ij."""
    n, f = exact_dot(A[i], [B[k][j] for k in range(len(B))], p)
    return mpnum.rn(n, f, p)


def ulp_error(x, n, f, p):
    """|x - n 2**f| in ulps of the exact value n 2**f (a Fraction).

    For an exact zero the error is reported as 0 when x is zero and as
    infinity otherwise.
    """
    exact = Fraction(n) * (Fraction(2) ** f)
    if n == 0:
        return Fraction(0) if x[0] == 0 else float("inf")
    # floor(log2|exact|) = bitlen(|n|) - 1 + f
    e_floor = abs(n).bit_length() - 1 + f
    ulp = Fraction(2) ** (e_floor - p + 1)
    return abs(mpnum.to_fraction(x, p) - exact) / ulp


def window_widths(A, B, p, extra):
    """The slice path's windows: W = p + min(largest exponent spread among the
    nonzero entries of a row of A (a column of B), extra)."""
    def spread(vectors):
        s = 0
        for v in vectors:
            es = [x[1] for x in v if x[0] != 0]
            if es:
                s = max(s, max(es) - min(es))
        return s
    cols = [[B[k][j] for k in range(len(B))] for j in range(len(B[0]))]
    return p + min(spread(A), extra), p + min(spread(cols), extra)


def _window_int(x, emax, W, p):
    """trunc(x * 2^(W - emax)) as an integer (toward zero)."""
    sig, e = x
    if sig == 0:
        return 0
    sh = e - p + W - emax
    mag = abs(sig) << sh if sh >= 0 else abs(sig) >> (-sh)
    return -mag if sig < 0 else mag


def slice_model_entry(A, B, i, j, p, WA, WB):
    """What the INT8-slice path computes for c_ij, step by step: scale row i
    of A by its largest exponent and column j of B by its own, keep each entry
    as an integer in a window of WA (WB) bits, truncating toward zero, form the
    exact integer dot product, and round once to p bits."""
    row = A[i]
    col = [B[k][j] for k in range(len(B))]
    ea = max((x[1] for x in row if x[0]), default=0)
    fb = max((x[1] for x in col if x[0]), default=0)
    z = sum(_window_int(a, ea, WA, p) * _window_int(b, fb, WB, p) for a, b in zip(row, col))
    return mpnum.rn(z, ea + fb - WA - WB, p)
