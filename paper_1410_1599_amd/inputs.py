"""Seeded synthetic inputs and the plane layout of an MP matrix.

This module is shared by the tests, the benchmark and the oracle's callers.
It holds no arithmetic of the method (no rounded multiply, add or divide):
it draws exact p-bit values and packs or unpacks them.

Plane layout (the library's matrix format, see include/mpgemm.h): an
r x c matrix at precision p (L = p / 32 limbs) is a uint32 array of shape
(L + 2, r, ld) with ld >= c:

* planes 0 .. L-1: the mantissa limbs, plane 0 the least significant;
* plane L: the exponent e as an int32;
* plane L + 1: the sign, 0 or 1.

The value is (-1)**sign * M * 2**(e - p) with 2**(p-1) <= M < 2**p, and zero
is all words 0.  In Python a value is the pair (sig, e) with sig = +-M, the
same pair oracle.mpnum uses.
"""

import math

import numpy as np

MASK32 = 0xFFFFFFFF


def nlimbs(p):
    if p % 32 or p <= 0:
        raise ValueError("precision must be a positive multiple of 32")
    return p // 32


def empty(rows, cols, p, ld=None):
    L = nlimbs(p)
    return np.zeros((L + 2, rows, ld if ld is not None else cols), dtype=np.uint32)


# ------------------------------------------------------------ packing

def to_planes(M, p, ld=None):
    """Pack a list of rows of (sig, e) pairs into the plane layout."""
    L = nlimbs(p)
    rows = len(M)
    cols = len(M[0]) if rows else 0
    out = empty(rows, cols, p, ld)
    for i, row in enumerate(M):
        for j, (sig, e) in enumerate(row):
            set_entry(out, i, j, (sig, e), p)
    return out


def set_entry(arr, i, j, v, p):
    L = nlimbs(p)
    sig, e = v
    mag = -sig if sig < 0 else sig
    if sig != 0 and not (1 << (p - 1)) <= mag < (1 << p):
        raise ValueError("mantissa not normalised to p bits")
    for k in range(L):
        arr[k, i, j] = (mag >> (32 * k)) & MASK32
    arr[L, i, j] = np.uint32(e & MASK32)
    arr[L + 1, i, j] = 1 if sig < 0 else 0


def entry(arr, i, j, p):
    """Unpack one element as (sig, e)."""
    L = nlimbs(p)
    mag = 0
    for k in range(L - 1, -1, -1):
        mag = (mag << 32) | int(arr[k, i, j])
    e = int(np.int32(np.uint32(arr[L, i, j])))
    if mag == 0:
        return (0, 0)
    return (-mag if arr[L + 1, i, j] else mag, e)


def from_planes(arr, p, rows=None, cols=None):
    """Unpack a whole matrix (small matrices: this is a Python loop)."""
    r = arr.shape[1] if rows is None else rows
    c = arr.shape[2] if cols is None else cols
    return [[entry(arr, i, j, p) for j in range(c)] for i in range(r)]


def row(arr, i, p, cols=None):
    c = arr.shape[2] if cols is None else cols
    return [entry(arr, i, j, p) for j in range(c)]


def col(arr, j, p, rows=None):
    r = arr.shape[1] if rows is None else rows
    return [entry(arr, i, j, p) for i in range(r)]


# ------------------------------------------------------------ generators

def _words(rng, L, shape):
    return rng.integers(0, 1 << 32, size=(L,) + tuple(shape), dtype=np.uint64).astype(np.uint32)


def _normalise_planes(W, p):
    """Left-justify the p-bit magnitudes W (L limb planes, uint32).

    Returns (mantissa planes, shift z) with M = W << z normalised; z is the
    leading-zero count, or -1 for W = 0.  Elements whose top limb is zero
    (probability 2**-32 each) are redone one by one with Python ints.
    """
    L = W.shape[0]
    top = W[L - 1].astype(np.uint64)
    z = np.zeros(top.shape, dtype=np.int64)
    t = top.copy()
    for b in (16, 8, 4, 2, 1):
        hi = t < (np.uint64(1) << np.uint64(32 - b))
        z = np.where(hi, z + b, z)
        t = np.where(hi, t << np.uint64(b), t)
    z = np.where(top == 0, 32, z)
    M = np.empty_like(W)
    zz = np.minimum(z, 31).astype(np.uint64)
    for k in range(L - 1, -1, -1):
        cur = W[k].astype(np.uint64) << zz
        low = (W[k - 1].astype(np.uint64) >> (np.uint64(32) - zz)) if k > 0 else np.zeros_like(cur)
        low = np.where(zz == 0, np.uint64(0), low)
        M[k] = ((cur | low) & np.uint64(MASK32)).astype(np.uint32)
    slow = np.argwhere(top == 0)
    for idx in slow:
        idx = tuple(idx)
        mag = 0
        for k in range(L - 1, -1, -1):
            mag = (mag << 32) | int(W[(k,) + idx])
        if mag == 0:
            z[idx] = -1
            for k in range(L):
                M[(k,) + idx] = 0
            continue
        zz1 = p - mag.bit_length()
        mag <<= zz1
        z[idx] = zz1
        for k in range(L):
            M[(k,) + idx] = (mag >> (32 * k)) & MASK32
    return M, z


def uniform_pm1(rows, cols, p, seed, ld=None):
    """Exact p-bit entries uniform on (-1, 1).

    x = (-1)**s * W * 2**-p with the sign s and W in [0, 2**p) uniform and
    independent, drawn from numpy's PCG64 seeded with `seed` (L words per
    entry, then one sign word).  Such x has at most p significant bits, so it
    is stored exactly; W = 0 gives the single zero.
    """
    L = nlimbs(p)
    rng = np.random.Generator(np.random.PCG64(seed))
    W = _words(rng, L, (rows, cols))
    s = (rng.integers(0, 2, size=(rows, cols), dtype=np.uint8)).astype(np.uint32)
    M, z = _normalise_planes(W, p)
    out = empty(rows, cols, p, ld)
    out[:L, :, :cols] = M
    e = np.where(z < 0, 0, -z).astype(np.int64)
    out[L, :, :cols] = (e & MASK32).astype(np.uint32)
    out[L + 1, :, :cols] = np.where(z < 0, 0, s)
    return out


def log_uniform(rows, cols, p, seed, emin=-20, emax=20, ld=None):
    """Sign uniform, exponent E uniform on [emin, emax], M uniform in [2**(p-1), 2**p).

    The value (-1)**s * M * 2**(E - p) lies in [2**(E-1), 2**E): log-uniform
    across binades, uniform inside one.
    """
    L = nlimbs(p)
    rng = np.random.Generator(np.random.PCG64(seed))
    W = _words(rng, L, (rows, cols))
    W[L - 1] |= np.uint32(0x80000000)
    E = rng.integers(emin, emax + 1, size=(rows, cols), dtype=np.int64)
    s = rng.integers(0, 2, size=(rows, cols), dtype=np.uint8).astype(np.uint32)
    out = empty(rows, cols, p, ld)
    out[:L, :, :cols] = W
    out[L, :, :cols] = (E & MASK32).astype(np.uint32)
    out[L + 1, :, :cols] = s
    return out


def sparse_bits(rows, cols, p, seed, nbits=3, emin=-3, emax=3, ld=None):
    """Mantissas with only a few set bits (the top bit and nbits-1 random
    others), small random exponents, random signs, and some zeros.

    Products and sums of such values are often exact or exact ties, which is
    where rounding code goes wrong; uniform random inputs almost never reach
    those paths.
    """
    L = nlimbs(p)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = empty(rows, cols, p, ld)
    for i in range(rows):
        for j in range(cols):
            if rng.integers(0, 16) == 0:
                continue
            mag = 1 << (p - 1)
            for _ in range(nbits - 1):
                mag |= 1 << int(rng.integers(0, p - 1))
            e = int(rng.integers(emin, emax + 1))
            sig = -mag if rng.integers(0, 2) else mag
            set_entry(out, i, j, (sig, e), p)
    return out


def integers(rows, cols, p, seed, bits=10):
    """Small integers |v| < 2**bits (as p-bit values): with p >= 64 no sum or
    product met in a product of modest size rounds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = empty(rows, cols, p)
    vals = rng.integers(-(1 << bits) + 1, 1 << bits, size=(rows, cols))
    for i in range(rows):
        for j in range(cols):
            v = int(vals[i, j])
            if v:
                mag = abs(v)
                sh = p - mag.bit_length()
                set_entry(out, i, j, ((-1 if v < 0 else 1) * (mag << sh), mag.bit_length()), p)
    return out


def hilbert(n, p, ld=None):
    """a_ij = the p-bit value nearest 1 / (i + j - 1) (1-based i, j)."""
    out = empty(n, n, p, ld)
    if n == 0:
        return out
    # the 2n - 1 distinct values 1/q, q = 1 .. 2n - 1, as plane columns, then
    # gathered by q = i + j + 1
    V = empty(1, 2 * n, p)
    for q in range(1, 2 * n):
        set_entry(V, 0, q, _recip_value(q, p), p)
    idx = np.add.outer(np.arange(n), np.arange(n)) + 1
    out[:, :, :n] = V[:, 0, :][:, idx]
    return out


def _rn_sqrt_times(c, k, p):
    """(sig, e) of the p-bit value nearest k * sqrt(c) (k >= 1, c not a square):
    integer square roots only; the value is irrational, so there is no tie."""
    v = c * k * k
    e = math.isqrt(v).bit_length()
    s = 2 * (p + 1 - e)
    r = math.isqrt(v << s) if s >= 0 else math.isqrt(v >> -s)
    M = (r >> 1) + (r & 1)
    if M == 1 << p:
        M >>= 1
        e += 1
    return (M, e)


def sqrt_workload(m, l, n, p):
    """The paper's benchmark matrices (Section 3): A (m x l) with
    a_ij = sqrt5 (i + j - 1), B (l x n) with b_ij = sqrt3 (n - i + 1), 1-based,
    each the nearest p-bit value (n is the column count of B and C, l <= n).
    c_ij = sqrt15 [(i - 1) l (2n - l + 1) / 2 + sum_k k (n - k + 1)]."""
    if l > n:
        raise ValueError("b_ij = sqrt3 (n - i + 1) needs l <= n")
    A = empty(m, l, p)
    B = empty(l, n, p)
    VA = empty(1, m + l, p)
    for q in range(1, m + l):
        set_entry(VA, 0, q, _rn_sqrt_times(5, q, p), p)
    A[:] = VA[:, 0, :][:, np.add.outer(np.arange(m), np.arange(l)) + 1]
    VB = empty(1, l, p)
    for i in range(l):
        set_entry(VB, 0, i, _rn_sqrt_times(3, n - i, p), p)
    B[:] = VB[:, 0, :][:, :, None]
    return A, B


def lotkin(n, p, ld=None):
    """The Lotkin matrix: the first row all ones, a_ij = the p-bit value
    nearest 1 / (i + j - 1) below it (1-based i, j)."""
    out = hilbert(n, p, ld)
    for j in range(n):
        set_entry(out, 0, j, (1 << (p - 1), 1), p)
    return out


def arange_column(n, p):
    """The n x 1 column x = [0, 1, ..., n - 1] (exact p-bit integers)."""
    out = empty(n, 1, p)
    for i in range(n):
        if i:
            e = i.bit_length()
            set_entry(out, i, 0, (i << (p - e), e), p)
    return out


def _recip_value(q, p):
    """(sig, e) of the nearest p-bit value to 1/q, by integer division only."""
    # 1/q lies in [2**(e-1), 2**e) with e = -(bitlen(q-1)) for q >= 2, e = 1 for q = 1
    e = 1 - (q - 1).bit_length() if q > 1 else 1
    # mantissa target: M = 1/q * 2**(p - e), in [2**(p-1), 2**p)
    num = 1 << (p - e)
    m, r = divmod(num, q)
    if 2 * r > q or (2 * r == q and (m & 1)):
        m += 1
    if m == 1 << p:
        m >>= 1
        e += 1
    return (m, e)


def ones_column(n, p):
    """An n x 1 column of ones (1 = 2**(p-1) * 2**(1 - p))."""
    out = empty(n, 1, p)
    for i in range(n):
        set_entry(out, i, 0, (1 << (p - 1), 1), p)
    return out
