"""Host checks (no GPU) of the two facts the one-value-per-wavefront
arithmetic rests on, for every supported width (L = 64 R limbs over 64 lanes):

1. the product's work map: lane t, step s, column slot k takes the term
   a_(s+k) b_((R t - s) mod L), which belongs to column R t + k while s <= R t and
   to column L + R t + k after; over all lanes, steps and slots every term
   a_i b_j is taken exactly once, in the column i + j, and every lane takes
   exactly L R terms (no idle multiplies);
2. the carry lookahead: with G the lanes whose own limb sums carry out and P
   the lanes whose sums are all ones (never both), the carry into lane t is
   bit t of ((G|P) + G + cin) xor (G|P) xor G, and the carry out of lane 63 is
   the overflow of that 64-bit sum -- checked against a lane-by-lane ripple.
"""

import random

import pytest


@pytest.mark.parametrize("R", [1, 2, 4, 5])
def test_product_work_map_covers_every_term_once(R):
    L = 64 * R
    nb = (L + R - 1 + R - 1) // R                 # blocks of R steps from s = 1 - R
    seen = {}
    per_lane = [0] * 64
    for t in range(64):
        for q in range(nb):
            for u in range(R):
                s = R * (q - 1) + 1 + u
                for k in range(R):
                    i = s + k
                    if not 0 <= i < L:
                        continue                 # a_(s+k) outside the value: a zero operand
                    j = (R * t - s) % L
                    col = R * t + k if s <= R * t else L + R * t + k
                    assert i + j == col, (t, s, k)
                    assert (i, j) not in seen, (i, j)
                    seen[(i, j)] = col
                    per_lane[t] += 1
                # the switch from low to high columns falls on a block start
                if s == R * t + 1:
                    assert u == 0
    assert len(seen) == L * L
    assert all(c == L * R for c in per_lane)


def ripple(G, P, cin):
    carries, c = 0, cin
    for t in range(64):
        if c:
            carries |= 1 << t
        g, p = (G >> t) & 1, (P >> t) & 1
        c = 1 if (g or (p and c)) else 0
    return carries, c


def lookahead(G, P, cin):
    M = (1 << 64) - 1
    GP = G | P
    u = (GP + G) & M
    s = (u + cin) & M
    cout = 1 if (u < GP or s < u) else 0
    return (s ^ GP ^ G) & M, cout


def test_carry_lookahead_matches_ripple():
    rng = random.Random(11)
    cases = [(0, 0), (0, (1 << 64) - 1), (1, (1 << 64) - 2), (1 << 63, 0), ((1 << 64) - 1, 0)]
    for _ in range(5000):
        G = rng.getrandbits(64) & rng.getrandbits(64)
        P = rng.getrandbits(64) & ~G
        if rng.random() < 0.3:
            P = ((1 << 64) - 1) & ~G               # long propagate runs
        cases.append((G, P))
    for G, P in cases:
        for cin in (0, 1):
            assert lookahead(G, P, cin) == ripple(G, P, cin), (hex(G), hex(P), cin)
