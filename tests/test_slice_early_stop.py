"""The INT8-slice product's early stop, checked on the host (no GPU).

The slice product's exact sum is Z = sum_u 256^u G_u over digit-pair
diagonals u.  Its first pass sums only the diagonals u >= u0 into V and keeps
V's rounding when the omitted part E, |E| < 2^D, cannot change it.  Two facts
carry that step; both are checked here against exact integer arithmetic and
the oracle's round-to-nearest-even:

1. the decision rule: with sh = bitlen(|V|) - p > D + 1 and the bits D .. sh-2
   of |V| neither all zero nor all one, RN_p(V + E) = RN_p(V) for every
   |E| < 2^D (exhaustive over E on small p and D);
2. the bound: sum_{u<u0} pairs(u) 256^u l 2^14 < 2^D for
   D = 8 u0 + 7 + ceil(log2 l) + ceil(log2 min(u0, S_A, S_B)), pairs(u) being
   the digit pairs (s, u - s) with 0 <= s < S_A, 0 <= u - s < S_B, and 2^14 the
   largest product of two balanced digits in [-128, 127].
"""

import random

from oracle import mpnum


def certain(V, D, p, lowest=None):
    """The decision rule (lowest: first bit of the tested field, D unless a
    test plants a mistake)."""
    lo = D if lowest is None else lowest
    a = abs(V)
    if a == 0:
        return False
    sh = a.bit_length() - p
    if sh - 1 <= D:
        return False
    w = sh - 1 - lo
    field = (a >> lo) & ((1 << w) - 1)
    return field != 0 and field != (1 << w) - 1


def violations(p, D, values, lowest=None):
    bad = []
    for V in values:
        if not certain(V, D, p, lowest):
            continue
        want = mpnum.from_int(V, p)
        for E in range(-(1 << D) + 1, 1 << D):
            if mpnum.from_int(V + E, p) != want:
                bad.append((V, E))
                break
    return bad


def edge_values(p, D, rng):
    """Values whose tail sits next to 0, the midpoint or a full unit, at the
    smallest exponents the rule accepts, and random ones."""
    out = []
    for sh in (D + 2, D + 3, D + 5):
        unit, half = 1 << sh, 1 << (sh - 1)
        for K in ((1 << (p - 1)), (1 << (p - 1)) + 1, (1 << p) - 1, rng.randrange(1 << (p - 1), 1 << p)):
            base = K * unit
            for t in (0, 1, (1 << D) - 1, 1 << D, (1 << D) + 1, half - (1 << D) - 1, half - (1 << D),
                      half - 1, half, half + 1, half + (1 << D), unit - (1 << D) - 1, unit - (1 << D), unit - 1):
                if 0 <= t < unit:
                    out += [base + t, -(base + t)]
    for _ in range(300):
        b = rng.randrange(p + D + 2, p + D + 12)
        v = rng.randrange(1 << (b - 1), 1 << b)
        out.append(v if rng.random() < 0.5 else -v)
    return out


def test_decision_rule_exhaustive_small():
    rng = random.Random(5)
    decided = 0
    for p in (4, 6, 8):
        for D in (0, 1, 3, 6):
            vals = edge_values(p, D, rng)
            assert violations(p, D, vals) == [], (p, D)
            decided += sum(certain(v, D, p) for v in vals)
    assert decided > 1000          # the rule accepts most values, not a vacuous few


def test_decision_rule_with_a_planted_mistake_fails():
    """Testing one bit too few (the field starting at D - 1) accepts values
    whose tail is within 2^D of a boundary: the exhaustive check must catch it."""
    rng = random.Random(6)
    found = False
    for p in (4, 6, 8):
        for D in (1, 3, 6):
            if violations(p, D, edge_values(p, D, rng), lowest=D - 1):
                found = True
    assert found


def pairs(u, SA, SB):
    return min(u, SA - 1) - max(0, u - SB + 1) + 1


def ceil_log2(v):
    r = 0
    while (1 << r) < v:
        r += 1
    return r


def test_omitted_diagonals_bound():
    for SA, SB in ((1, 1), (3, 40), (17, 17), (37, 37), (38, 37), (69, 5), (133, 133)):
        ndiag = SA + SB - 1
        for l in (1, 2, 7, 64, 2048, 131008, 262143):
            for u0 in sorted({1, 2, 3, min(SA, SB), ndiag // 2, ndiag - 1} - {0}):
                if u0 >= ndiag:
                    continue
                omitted = sum(pairs(u, SA, SB) * 256 ** u for u in range(u0)) * l * 2 ** 14
                D = 8 * u0 + 7 + ceil_log2(l) + ceil_log2(min(u0, SA, SB))
                assert omitted < 2 ** D, (SA, SB, l, u0)
                # and not loose by more than a few bits
                assert omitted >= 2 ** (D - 4 - 8), (SA, SB, l, u0)
