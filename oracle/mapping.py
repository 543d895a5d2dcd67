"""Constant-weight codes and the paper's mappings onto them (test infrastructure only).

Section 3: a binary constant-weight code CW(m, k) has C(m, k) codewords; for n identifiers the
code length is the smallest m with C(m, k) >= n.  A codeword is represented here by the ascending
list of its one positions.
"""
from __future__ import annotations

import math

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def binom(a: int, b: int) -> int:
    """C(a, b), zero when a < b (the convention the mapping algorithms rely on)."""
    return math.comb(a, b) if 0 <= b <= a else 0


def code_length(n: int, k: int) -> int:
    """Smallest m with C(m, k) >= n (Section 3)."""
    m = k
    while binom(m, k) < n:
        m += 1
    return m


def perfect_map(x: int, m: int, k: int) -> list:
    """Perfect mapping (Algorithm 3): identifier x in [C(m,k)] -> the one positions of the x-th
    codeword of CW(m, k) in colexicographic order.

    Written as the inverse of the colex rank that Algorithm 7 computes, x = sum_h C(p_h, h) over
    the ascending positions p_1 < ... < p_k (the combinatorial number system): the top position
    p_k is the largest p with C(p, k) <= x, since the codewords whose top one is below p number
    C(p, k); the rest x - C(p_k, k) is the rank of the remaining k - 1 positions below p_k, so the
    same rule gives p_{k-1}, and so on down to p_1."""
    if not 0 <= x < binom(m, k):
        raise ValueError("identifier outside the code")
    ones = []
    r, hi = x, m - 1                       # p_h lies in [h - 1, hi]
    for h in range(k, 0, -1):
        lo = h - 1                          # C(h - 1, h) = 0 <= r, so lo always qualifies
        while lo < hi:                      # largest p in [lo, hi] with C(p, h) <= r
            mid = (lo + hi + 1) // 2
            if binom(mid, h) <= r:
                lo = mid
            else:
                hi = mid - 1
        ones.append(lo)
        r -= binom(lo, h)
        hi = lo - 1
    assert r == 0
    return sorted(ones)


def inverse_perfect_map(ones, m: int) -> int:
    """Inverse perfect mapping (Algorithm 7): sum over the ascending one positions m'_h (h = 1..k)
    of C(m'_h, h)."""
    x, h = 0, 1
    for mp in range(m):
        if mp in ones:
            x += binom(mp, h)
            h += 1
    return x


def mix64(z: int) -> int:
    """SplitMix64 output function (Steele, Lea and Flood 2014)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def lossy_hash(seed: int, x: int, i: int, m: int) -> int:
    """H_i(x) = mix64(seed XOR x XOR i * golden-gamma) mod m, i = 1, 2, ..."""
    return mix64((seed ^ x ^ ((i * GOLDEN_GAMMA) & MASK64)) & MASK64) % m


def lossy_map(x: int, m: int, k: int, seed: int) -> list:
    """Lossy mapping (Algorithm 8): draw H_1(x), H_2(x), ... and keep the first k distinct
    positions; the codeword is returned as its sorted one positions."""
    ones = set()
    i = 1
    while len(ones) < k:
        ones.add(lossy_hash(seed, x, i, m))
        i += 1
    return sorted(ones)


def codeword_bits(ones, m: int) -> list:
    bits = [0] * m
    for p in ones:
        bits[p] = 1
    return bits
