"""Reference blocked LU with partial pivoting, and the solve that follows it.

TEST INFRASTRUCTURE ONLY (see oracle/mpnum.py).

Section 4 factors A in blocks of K columns: A11 = L11 U11, A12 -> U12,
A21 -> L21, then A22 := A22 - L21 U12 with the product formed by one of the
matrix-multiplication algorithms, and repeats on A22.  The paper's LU does
not pivot; this one adds row partial pivoting, with these readings:

* pivot row = the smallest index i >= c that maximises |a_ic| (exact
  comparison);
* the row swap covers all n columns; piv[c] records the row swapped with c
  (0-based, LAPACK getrf style); a zero pivot sets info = c + 1 (first one
  only) and skips that column's division and update;
* the multipliers are true quotients RN(a_ic / a_cc);
* U12 is formed by unit-lower forward substitution, column by column;
* the trailing update forms P = L21 U12 with the chosen algorithm first and
  then subtracts it elementwise (Section 4, step 3);
* the last panel may be narrower than K.
"""

from . import mpnum
from . import gemm as G


def lu(A, p, panel=64, algo=G.WINOGRAD, cutoff=32, policy=G.PEEL, pivot=True):
    """Factor a copy of A in place.  Returns (LU, piv, info).

    pivot=False is the paper's LU as published (Section 4): no row
    exchanges, every pivot the diagonal entry, piv the identity; a zero
    diagonal entry sets info and skips that column like a zero pivot."""
    n = len(A)
    a = [list(r) for r in A]
    piv = list(range(n))
    info = 0
    ar = G.Arith(p)
    for j0 in range(0, n, panel):
        kb = min(panel, n - j0)
        je = j0 + kb
        # 1. panel: unblocked right-looking elimination on columns j0..je-1
        for c in range(j0, je):
            r = c
            for i in range(c + 1, n if pivot else c + 1):
                if mpnum.cmp_abs(a[i][c], a[r][c]) > 0:
                    r = i
            piv[c] = r
            if r != c:
                a[c], a[r] = a[r], a[c]
            if a[c][c][0] == 0:
                if info == 0:
                    info = c + 1
                continue
            for i in range(c + 1, n):
                a[i][c] = mpnum.div(a[i][c], a[c][c], p)
            for i in range(c + 1, n):
                lic = a[i][c]
                for j in range(c + 1, je):
                    a[i][j] = ar.sub(a[i][j], ar.mul(lic, a[c][j]))
        if je >= n:
            break
        # 2. U12 := L11^{-1} A12 (unit lower triangular, forward substitution)
        for t in range(kb):
            for r in range(t + 1, kb):
                lrt = a[j0 + r][j0 + t]
                for j in range(je, n):
                    a[j0 + r][j] = ar.sub(a[j0 + r][j], ar.mul(lrt, a[j0 + t][j]))
        # 3. A22 := A22 - L21 U12, the product formed first
        L21 = [row[j0:je] for row in a[je:]]
        U12 = [row[je:] for row in a[j0:je]]
        P = G.gemm(L21, U12, p, algo=algo, cutoff=cutoff, policy=policy)
        for i in range(je, n):
            for j in range(je, n):
                a[i][j] = ar.sub(a[i][j], P[i - je][j - je])
    return a, piv, info


def rhs_ones(A, p):
    """b = A * ones by Simple (j ascending): b_i = sum_j a_ij."""
    one = mpnum.from_int(1, p)
    col = [[one] for _ in range(len(A))]
    return [r[0] for r in G.gemm(A, col, p, algo=G.SIMPLE)]


def solve(LU, piv, b, p):
    """x from the factors: apply the swaps, then Ly = Pb, then Ux = y."""
    n = len(LU)
    y = list(b)
    for k in range(n):
        r = piv[k]
        if r != k:
            y[k], y[r] = y[r], y[k]
    for t in range(n):
        for r in range(t + 1, n):
            y[r] = mpnum.sub(y[r], mpnum.mul(LU[r][t], y[t], p), p)
    x = [mpnum.ZERO] * n
    for t in range(n - 1, -1, -1):
        x[t] = mpnum.div(y[t], LU[t][t], p)
        for r in range(t):
            y[r] = mpnum.sub(y[r], mpnum.mul(LU[r][t], x[t], p), p)
    return x


def permute_rows(A, piv):
    """P A for the sequential swaps in piv."""
    a = [list(r) for r in A]
    for k, r in enumerate(piv):
        if r != k:
            a[k], a[r] = a[r], a[k]
    return a


def residual_exact(A, LU, piv, p):
    """||PA - L U||_inf / ||A||_inf with exact rational arithmetic (small n)."""
    from fractions import Fraction
    n = len(A)
    F = lambda v: mpnum.to_fraction(v, p)
    PA = permute_rows(A, piv)
    num = Fraction(0)
    den = Fraction(0)
    for i in range(n):
        rs = Fraction(0)
        ra = Fraction(0)
        for j in range(n):
            s = Fraction(0)
            for k in range(min(i, j) + 1):
                lik = Fraction(1) if k == i else F(LU[i][k])
                s += lik * F(LU[k][j])
            rs += abs(F(PA[i][j]) - s)
            ra += abs(F(A[i][j]))
        num = max(num, rs)
        den = max(den, ra)
    return num / den if den else Fraction(0)
