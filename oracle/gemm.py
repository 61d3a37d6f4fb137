"""Reference MP matrix products: Simple, Block, Strassen, Winograd's variant.

TEST INFRASTRUCTURE ONLY (see oracle/mpnum.py).

A matrix is a list of rows; an entry is an ``(sig, e)`` pair of
oracle.mpnum.  Every scalar operation rounds once (mpnum.mul, mpnum.add,
mpnum.sub), so Strassen and Winograd reach a *different* rounded result from
Simple; the functions below fix the order of every operation.

Readings of the paper used here:

* Simple, eq. (1): c_ij starts at exact zero and takes add(c_ij,
  mul(a_ik, b_kj)) for k ascending (a product is rounded, then the sum is
  rounded: two roundings per term, as a sequence of MPFR multiply and add
  calls does).
* Block, eq. (2): each product a_ik b_kj goes straight into c_ij, k-blocks
  ascending and k ascending inside a block, so Block equals Simple bit for bit
  for every block size.  The block loops are written out anyway.
* Strassen, Section 2 (P1..P7 and the C quadrants): sums as printed, left to
  right.
* Winograd's variant, eqs. (winograd_mod1)-(winograd_mod3) and the C
  quadrants that follow them: S1..S8, M1..M7, T1, T2 in the printed order and
  association.
* Recursion, Section 2 (last paragraph): recurse while min(m, l, n) exceeds
  the cutoff n_min, else Simple.  This strict reading is the one under which
  Table 1 reproduces.
* Odd sizes, same paragraph ("a mixture of dynamic padding and peeling"):
  policy ``peel`` (default), ``pad``, or ``mixed`` (pad a dimension d with
  d = 3 mod 4, peel one with d = 1 mod 4, which reproduces all of Table 1).
"""

from . import mpnum

ZERO = mpnum.ZERO

SIMPLE, BLOCK, STRASSEN, WINOGRAD = "simple", "block", "strassen", "winograd"
PEEL, PAD, MIXED = "peel", "pad", "mixed"


class Counter:
    """Counts scalar multiplications and additions/subtractions."""

    def __init__(self):
        self.mul = 0
        self.addsub = 0


class Arith:
    """The scalar operations at precision p, optionally counted."""

    def __init__(self, p, counter=None):
        self.p = p
        self.c = counter

    def mul(self, x, y):
        if self.c is not None:
            self.c.mul += 1
        return mpnum.mul(x, y, self.p)

    def add(self, x, y):
        if self.c is not None:
            self.c.addsub += 1
        return mpnum.add(x, y, self.p)

    def sub(self, x, y):
        if self.c is not None:
            self.c.addsub += 1
        return mpnum.sub(x, y, self.p)


# ---------------------------------------------------------------- helpers

def zeros(m, n):
    return [[ZERO] * n for _ in range(m)]


def shape(A):
    return len(A), (len(A[0]) if A else 0)


def sub_block(A, r0, r1, c0, c1):
    return [row[c0:c1] for row in A[r0:r1]]


def mat_add(ar, X, Y):
    return [[ar.add(x, y) for x, y in zip(rx, ry)] for rx, ry in zip(X, Y)]


def mat_sub(ar, X, Y):
    return [[ar.sub(x, y) for x, y in zip(rx, ry)] for rx, ry in zip(X, Y)]


# ---------------------------------------------------------------- eq. (1)

def simple(ar, A, B, m, l, n):
    """Simple, eq. (1): c_ij = sum_k a_ik b_kj, k ascending from exact 0."""
    C = zeros(m, n)
    for i in range(m):
        for j in range(n):
            c = ZERO
            for k in range(l):
                c = ar.add(c, ar.mul(A[i][k], B[k][j]))
            C[i][j] = c
    return C


# ---------------------------------------------------------------- eq. (2)

def block(ar, A, B, m, l, n, bs):
    """Block, eq. (2), with bs x bs blocks.

    C_ij accumulates A_ik B_kj over k-blocks ascending; inside a block pair
    each product is added straight into c_ij with k ascending.
    """
    C = zeros(m, n)
    for i0 in range(0, m, bs):
        for j0 in range(0, n, bs):
            for k0 in range(0, l, bs):
                for i in range(i0, min(i0 + bs, m)):
                    for j in range(j0, min(j0 + bs, n)):
                        c = C[i][j]
                        for k in range(k0, min(k0 + bs, l)):
                            c = ar.add(c, ar.mul(A[i][k], B[k][j]))
                        C[i][j] = c
    return C


# ------------------------------------------------------- one even level

def strassen_level(ar, A, B, m, l, n, rec):
    """One Strassen level on even m, l, n (P1..P7, then the C quadrants)."""
    h, g, w = m // 2, l // 2, n // 2
    A11, A12 = sub_block(A, 0, h, 0, g), sub_block(A, 0, h, g, l)
    A21, A22 = sub_block(A, h, m, 0, g), sub_block(A, h, m, g, l)
    B11, B12 = sub_block(B, 0, g, 0, w), sub_block(B, 0, g, w, n)
    B21, B22 = sub_block(B, g, l, 0, w), sub_block(B, g, l, w, n)
    P1 = rec(mat_add(ar, A11, A22), mat_add(ar, B11, B22), h, g, w)
    P2 = rec(mat_add(ar, A21, A22), B11, h, g, w)
    P3 = rec(A11, mat_sub(ar, B12, B22), h, g, w)
    P4 = rec(A22, mat_sub(ar, B21, B11), h, g, w)
    P5 = rec(mat_add(ar, A11, A12), B22, h, g, w)
    P6 = rec(mat_sub(ar, A21, A11), mat_add(ar, B11, B12), h, g, w)
    P7 = rec(mat_sub(ar, A12, A22), mat_add(ar, B21, B22), h, g, w)
    C11 = mat_add(ar, mat_sub(ar, mat_add(ar, P1, P4), P5), P7)
    C12 = mat_add(ar, P3, P5)
    C21 = mat_add(ar, P2, P4)
    C22 = mat_add(ar, mat_sub(ar, mat_add(ar, P1, P3), P2), P6)
    return assemble(C11, C12, C21, C22)


def winograd_level(ar, A, B, m, l, n, rec):
    """One level of Winograd's variant on even m, l, n."""
    h, g, w = m // 2, l // 2, n // 2
    A11, A12 = sub_block(A, 0, h, 0, g), sub_block(A, 0, h, g, l)
    A21, A22 = sub_block(A, h, m, 0, g), sub_block(A, h, m, g, l)
    B11, B12 = sub_block(B, 0, g, 0, w), sub_block(B, 0, g, w, n)
    B21, B22 = sub_block(B, g, l, 0, w), sub_block(B, g, l, w, n)
    S1 = mat_add(ar, A21, A22)
    S2 = mat_sub(ar, S1, A11)
    S3 = mat_sub(ar, A11, A21)
    S4 = mat_sub(ar, A12, S2)
    S5 = mat_sub(ar, B12, B11)
    S6 = mat_sub(ar, B22, S5)
    S7 = mat_sub(ar, B22, B12)
    S8 = mat_sub(ar, S6, B21)
    M1 = rec(S2, S6, h, g, w)
    M2 = rec(A11, B11, h, g, w)
    M3 = rec(A12, B21, h, g, w)
    M4 = rec(S3, S7, h, g, w)
    M5 = rec(S1, S5, h, g, w)
    M6 = rec(S4, B22, h, g, w)
    M7 = rec(A22, S8, h, g, w)
    T1 = mat_add(ar, M1, M2)
    T2 = mat_add(ar, T1, M4)
    C11 = mat_add(ar, M2, M3)
    C12 = mat_add(ar, mat_add(ar, T1, M5), M6)
    C21 = mat_sub(ar, T2, M7)
    C22 = mat_add(ar, T2, M5)
    return assemble(C11, C12, C21, C22)


def assemble(C11, C12, C21, C22):
    top = [r1 + r2 for r1, r2 in zip(C11, C12)]
    bot = [r1 + r2 for r1, r2 in zip(C21, C22)]
    return top + bot


# ------------------------------------------------------- odd dimensions

def odd_actions(m, l, n, policy):
    """For each of m, l, n: 'even', 'peel' or 'pad'."""
    out = []
    for d in (m, l, n):
        if d % 2 == 0:
            out.append("even")
        elif policy == PEEL:
            out.append("peel")
        elif policy == PAD:
            out.append("pad")
        elif policy == MIXED:
            out.append("pad" if d % 4 == 3 else "peel")
        else:
            raise ValueError(policy)
    return out


def recursive(ar, A, B, m, l, n, algo, cutoff, policy=PEEL):
    """R(A, B): Strassen or Winograd down to the cutoff, Simple below it.

    Recurse iff min(m, l, n) > cutoff.  Odd dimensions are made even by
    peeling or padding before each level:

    * pad: append an exact zero row/column, run the level, crop.
    * peel m (odd): rows 0..m-2 come from the level; row m-1 (all n columns)
      is Simple over the full l.
    * peel n (odd): columns 0..n-2 come from the level; column n-1 for rows
      0..m'-1 is Simple over the full l.
    * peel l (odd): the level runs on inner size l-1 and each entry of its
      m' x n' result then takes c := add(c, mul(a_{i,l-1}, b_{l-1,j})).
    """
    if m == 0 or n == 0:
        return zeros(m, n)
    if min(m, l, n) <= cutoff:
        return simple(ar, A, B, m, l, n)
    level = strassen_level if algo == STRASSEN else winograd_level

    def rec(X, Y, mm, ll, nn):
        return recursive(ar, X, Y, mm, ll, nn, algo, cutoff, policy)

    act_m, act_l, act_n = odd_actions(m, l, n, policy)
    # padded / peeled even core sizes
    me = m + 1 if act_m == "pad" else (m - 1 if act_m == "peel" else m)
    le = l + 1 if act_l == "pad" else (l - 1 if act_l == "peel" else l)
    ne = n + 1 if act_n == "pad" else (n - 1 if act_n == "peel" else n)
    # operands of the even core: crop the peeled parts, pad with exact zeros
    Ae = [[A[i][k] if (i < m and k < l) else ZERO for k in range(le)] for i in range(me)]
    Be = [[B[k][j] if (k < l and j < n) else ZERO for j in range(ne)] for k in range(le)]
    Ce = level(ar, Ae, Be, me, le, ne, rec)
    mi, ni = min(m, me), min(n, ne)            # rows/cols the core delivers
    C = zeros(m, n)
    for i in range(mi):
        for j in range(ni):
            C[i][j] = Ce[i][j]
    if act_l == "peel":
        k = l - 1
        for i in range(mi):
            for j in range(ni):
                C[i][j] = ar.add(C[i][j], ar.mul(A[i][k], B[k][j]))
    if act_n == "peel":
        j = n - 1
        for i in range(mi):
            c = ZERO
            for k in range(l):
                c = ar.add(c, ar.mul(A[i][k], B[k][j]))
            C[i][j] = c
    if act_m == "peel":
        i = m - 1
        for j in range(n):
            c = ZERO
            for k in range(l):
                c = ar.add(c, ar.mul(A[i][k], B[k][j]))
            C[i][j] = c
    return C


def gemm(A, B, p, algo=SIMPLE, cutoff=32, policy=PEEL, block_size=16, counter=None):
    """C := AB at precision p with the chosen algorithm (entry point)."""
    m, l = len(A), (len(A[0]) if A else 0)
    n = len(B[0]) if B else 0
    if m and len(B) != l:
        raise ValueError("inner dimensions differ")
    ar = Arith(p, counter)
    if algo == SIMPLE:
        return simple(ar, A, B, m, l, n)
    if algo == BLOCK:
        return block(ar, A, B, m, l, n, block_size)
    if algo in (STRASSEN, WINOGRAD):
        return recursive(ar, A, B, m, l, n, algo, cutoff, policy)
    raise ValueError(algo)


# ------------------------------------------------- operation counts

def op_counts(m, l, n, algo, cutoff, policy=PEEL):
    """(Mul, Addsub) that gemm() performs, counted without arithmetic.

    Follows recursive() step for step, so a peeled index costs one multiply
    and one add per product that touches it and a padded zero is counted
    like any other operand.  The paper's recurrences (Section 2) are the
    even case: Mul = 7 Mul(m/2, l/2, n/2) and Addsub = 7 Addsub(m/2, l/2, n/2)
    + cA (m/2)(l/2) + cB (l/2)(n/2) + cC (m/2)(n/2), (cA, cB, cC) = (5, 5, 8)
    for Strassen and (4, 4, 7) for Winograd; the printed recurrences leave the
    7 Addsub(m/2, l/2, n/2) term of the sub-products out.
    """
    if m == 0 or n == 0:
        return 0, 0
    if algo in (SIMPLE, BLOCK) or min(m, l, n) <= cutoff:
        return m * l * n, m * l * n
    act_m, act_l, act_n = odd_actions(m, l, n, policy)
    me = m + 1 if act_m == "pad" else (m - 1 if act_m == "peel" else m)
    le = l + 1 if act_l == "pad" else (l - 1 if act_l == "peel" else l)
    ne = n + 1 if act_n == "pad" else (n - 1 if act_n == "peel" else n)
    h, g, w = me // 2, le // 2, ne // 2
    sm, sa = op_counts(h, g, w, algo, cutoff, policy)
    ca, cb, cc = (5, 5, 8) if algo == STRASSEN else (4, 4, 7)
    mul = 7 * sm
    addsub = 7 * sa + ca * h * g + cb * g * w + cc * h * w
    mi, ni = min(m, me), min(n, ne)
    if act_l == "peel":
        mul += mi * ni
        addsub += mi * ni
    if act_n == "peel":
        mul += mi * l
        addsub += mi * l
    if act_m == "peel":
        mul += n * l
        addsub += n * l
    return mul, addsub


def depth(m, l, n, cutoff, policy=PEEL):
    """Number of recursion levels R() takes on an m x l x n product."""
    d = 0
    while min(m, l, n) > cutoff:
        act = odd_actions(m, l, n, policy)
        dims = []
        for dd, a in zip((m, l, n), act):
            dims.append((dd + 1 if a == "pad" else (dd - 1 if a == "peel" else dd)) // 2)
        m, l, n = dims
        d += 1
    return d
