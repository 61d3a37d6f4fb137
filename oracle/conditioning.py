"""Exact condition numbers of the paper's test matrices (Section 4).

TEST INFRASTRUCTURE ONLY (see oracle/mpnum.py).

The paper quotes ||A||_1 ||A^-1||_1 of its Lotkin matrix at n = 1024 (first
row all ones, a_ij = 1 / (i + j - 1) below it) to show why 8192 bits are
needed.  Here that number is computed exactly, in rational arithmetic:

* The Hilbert matrix H (h_ij = 1 / (i + j - 1)) has an integer inverse with
  the classical closed form (1-based indices)
      (H^-1)_ij = (-1)^(i+j) (i+j-1) C(n+i-1, n-j) C(n+j-1, n-i) C(i+j-2, i-1)^2.
* The Lotkin matrix differs from H in its first row only: A = H + e_1 w^T
  with w_j = 1 - 1/j.  By the Sherman-Morrison formula
      A^-1 = H^-1 - (H^-1 e_1)(w^T H^-1) / (1 + w^T H^-1 e_1).
  With Ln = lcm(1..n), W = Ln w is an integer vector, c = H^-1 e_1,
  R = H^-1 W (H^-1 is symmetric) and D = Ln + W^T c, every entry of A^-1 is
  (D (H^-1)_ij - c_i R_j) / D, an exact integer over D.
* ||A||_1 is the largest column sum of |a_ij|; every entry of a column
  shrinks as j grows, so it is the first column's, 1 + sum_{i=2..n} 1/i;
  ||A||_inf is the first row's, n.

Each column of H^-1 is walked with exact integer recurrences of the three
binomials, so no n x n matrix of big integers is ever held.
"""

from fractions import Fraction
from math import comb, gcd


def hilbert_inverse_entry(n, i, j):
    """(H^-1)_ij of the n x n Hilbert matrix, 1-based, from the closed form."""
    s = -1 if (i + j) % 2 else 1
    return s * (i + j - 1) * comb(n + i - 1, n - j) * comb(n + j - 1, n - i) * comb(i + j - 2, i - 1) ** 2


def _hilbert_inverse_column(n, j):
    """Column j (1-based) of H^-1 as a list of n integers, by recurrences in i."""
    X = comb(n, j)                 # C(n + i - 1, n - j) at i = 1
    Y = comb(n + j - 1, n - 1)     # C(n + j - 1, n - i) at i = 1
    Z = 1                          # C(i + j - 2, i - 1) at i = 1
    col = []
    for i in range(1, n + 1):
        v = (i + j - 1) * X * Y * Z * Z
        col.append(-v if (i + j) % 2 else v)
        if i < n:
            X = X * (n + i) // (i + j)
            Y = Y * (n - i) // (j + i)
            Z = Z * (i + j - 1) // i
    return col


def lotkin(n):
    """The n x n Lotkin matrix as Fractions (row 1 ones, then Hilbert rows)."""
    return [[Fraction(1) if i == 1 else Fraction(1, i + j - 1) for j in range(1, n + 1)] for i in range(1, n + 1)]


def lotkin_conditions(n):
    """(||A||_1 ||A^-1||_1, ||A||_inf ||A^-1||_inf) of the n x n Lotkin
    matrix, exactly (Fractions).  ||A||_inf = n (the first row)."""
    Ln = 1
    for k in range(2, n + 1):
        Ln = Ln * k // gcd(Ln, k)
    W = [Ln - Ln // j for j in range(1, n + 1)]          # Ln * (1 - 1/j)
    c = _hilbert_inverse_column(n, 1)
    D = Ln + sum(w * ci for w, ci in zip(W, c))
    # R_j = sum_i (H^-1)_ji W_i = sum_i (H^-1)_ij W_i, column by column
    R = [sum(w * h for w, h in zip(W, _hilbert_inverse_column(n, j))) for j in range(1, n + 1)]
    col_best = 0
    row_sums = [0] * n
    for j in range(1, n + 1):
        Rj = R[j - 1]
        vals = [abs(D * h - ci * Rj) for h, ci in zip(_hilbert_inverse_column(n, j), c)]
        col_best = max(col_best, sum(vals))
        for i, v in enumerate(vals):
            row_sums[i] += v
    norm1_a = 1 + sum(Fraction(1, i) for i in range(2, n + 1))
    return norm1_a * Fraction(col_best, abs(D)), n * Fraction(max(row_sums), abs(D))


def lotkin_cond1(n):
    """||A||_1 ||A^-1||_1 of the n x n Lotkin matrix, exactly (a Fraction)."""
    return lotkin_conditions(n)[0]


def inverse_fraction(M):
    """Exact inverse of a small square Fraction matrix by Gauss-Jordan (pins)."""
    n = len(M)
    A = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(M)]
    for c in range(n):
        r = next(i for i in range(c, n) if A[i][c] != 0)
        A[c], A[r] = A[r], A[c]
        piv = A[c][c]
        A[c] = [v / piv for v in A[c]]
        for i in range(n):
            if i != c and A[i][c] != 0:
                f = A[i][c]
                A[i] = [a - f * b for a, b in zip(A[i], A[c])]
    return [row[n:] for row in A]


def cond1(M):
    """||M||_1 ||M^-1||_1 of a small Fraction matrix, exactly."""
    n = len(M)
    inv = inverse_fraction(M)
    n1 = lambda X: max(sum(abs(X[i][j]) for i in range(n)) for j in range(n))
    return n1(M) * n1(inv)


def cond_inf(M):
    """||M||_inf ||M^-1||_inf of a small Fraction matrix, exactly."""
    inv = inverse_fraction(M)
    ni = lambda X: max(sum(abs(v) for v in row) for row in X)
    return ni(M) * ni(inv)


def decimal_mantissa_exponent(q, digits=2):
    """(mantissa rounded to `digits` significant digits, decimal exponent) of
    a positive Fraction, exactly (no floating point)."""
    e = len(str(q.numerator // q.denominator)) - 1 if q >= 1 else -len(str(q.denominator // q.numerator))
    while Fraction(10) ** e > q:
        e -= 1
    while Fraction(10) ** (e + 1) <= q:
        e += 1
    scaled = q / Fraction(10) ** (e - digits + 1)                 # in [10^(d-1), 10^d)
    m = (scaled.numerator * 2 + scaled.denominator) // (2 * scaled.denominator)   # round half up
    if m == 10 ** digits:
        m, e = m // 10, e + 1
    return m / 10 ** (digits - 1), e
