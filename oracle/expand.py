"""Query packing and server-side query expansion (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg may use this
module; the product path never does.

What it computes (paper, Section 3.3.2 "Query" and Section 3.3.3 "Query Expansion"):
  * pack_query   Algorithm 4 with compression factor c: the codeword bits E_q are cut into
                 h = ceil(m / 2^c) groups of 2^c; group i becomes the plaintext
                 m_i(x) = sum_j (2^-c mod t) E_q[i 2^c + j] x^j, encrypted with the secret key.
  * expand       Algorithm 5: every packed ciphertext is expanded into 2^c ciphertexts with one
                 substitution per (level a, slot b) and two monomial products; the outputs are
                 concatenated and the first m kept.  No final scaling: the client's 2^-c cancels
                 the gain of 2^c.
  * expand_sealpir  Algorithm 1 (SealPIR's expansion, the form the paper proves Algorithm 5
                 equivalent to): two substitutions per (a, b), then a plaintext product by
                 2^-c mod t.  Fed an unscaled packing, it must decrypt to the same bits.

Readings.  Sub_g is the automorphism x -> x^g followed by a key switch of the second polynomial
back to s with the same per-limb digits as relinearization (Galois key b_i = -a_i s + e_i +
g_i s(x^g)).  The Galois element at level a is N / 2^a + 1.  Algorithm 1's printed monomial
x^{2^{-a}} is read as x^{-2^a}, the monomial Algorithm 5 uses.  x^{-e} is x^{2N - e}.
"""
from __future__ import annotations

import math

import numpy as np

import datagen
from .core import Oracle


def galois_elements(N: int, c: int) -> list:
    """Galois element of each expansion level a in [c]: N / 2^a + 1 (Algorithm 5)."""
    return [N // (1 << a) + 1 for a in range(c)]


def galois_keys(orc: Oracle, sk: np.ndarray, c: int, seed: int) -> dict:
    """Galois keys {g: [L][2][L][N]} for the c levels, from the seeded key stream."""
    per = orc.rnd_words_rlk()
    return {g: orc.galois_keygen(sk, g, datagen.words(seed, datagen.S_GALOIS, per, offset=a * per))
            for a, g in enumerate(galois_elements(orc.N, c))}


def packed_count(m: int, c: int) -> int:
    return -(-m // (1 << c))


def pack_messages(bits, c: int, N: int, t: int, prescale: bool = True) -> np.ndarray:
    """Algorithm 4, packing: the h plaintexts [h][N]; plaintext i holds 2^-c (mod t) times bit
    i 2^c + j in coefficient j.  With prescale=False the coefficients are the bits themselves (the
    input of Algorithm 1)."""
    bits = [int(b) for b in bits]
    m = len(bits)
    if (1 << c) > N:
        raise ValueError("2^c must not exceed N")
    h = packed_count(m, c)
    inv = pow(2, -c, t) if prescale else 1
    msgs = np.zeros((h, N), dtype=np.uint64)
    for i in range(h):
        for j in range(1 << c):
            if i * (1 << c) + j < m:
                msgs[i, j] = (inv * bits[i * (1 << c) + j]) % t
    return msgs


def pack_query(orc: Oracle, sk: np.ndarray, bits, c: int, seed: int, draw: int = 0, prescale: bool = True):
    """Algorithm 4, packing and encryption: h packed ciphertexts [h][2][L][N], the encryptions of
    pack_messages."""
    msgs = pack_messages(bits, c, orc.N, orc.t, prescale)
    h = len(msgs)
    per = orc.rnd_words_encrypt()
    out = np.empty((h, 2, orc.L, orc.N), dtype=np.uint64)
    for i in range(h):
        rnd = datagen.words(seed, datagen.S_PACKED, per, offset=(draw * h + i) * per)
        out[i] = orc.encrypt(sk, msgs[i], rnd)
    return out


def split_level(orc: Oracle, key, ct: np.ndarray, a: int) -> tuple:
    """What level a of Algorithm 5 does to one ciphertext, derived from its effect on the plaintext.

    Before level a the plaintext has terms only at exponents that are multiples of 2^a, say
    u_j x^{j 2^a}.  The substitution with g = N / 2^a + 1 sends x^{j 2^a} to x^{j 2^a g} =
    x^{j N} x^{j 2^a} = (-1)^j x^{j 2^a}: even j are fixed, odd j negated.  So ct + Sub_g(ct) keeps
    the even-j terms (doubled) and ct - Sub_g(ct) the odd-j terms (doubled), which the monomial
    x^{-2^a} moves down to multiples of 2^{a+1}.  Returns (ct + Sub_g(ct), x^{-2^a} (ct - Sub_g(ct)))."""
    N = orc.N
    g = N // (1 << a) + 1
    s = orc.sub(key, ct, g)
    even = orc.add(ct, s)
    odd = orc.mul_monomial(_sub(orc, ct, s), 2 * N - (1 << a))   # x^{-2^a} = x^{2N - 2^a}
    return even, odd


def expand(orc: Oracle, gkeys: dict, packed: np.ndarray, m: int, c: int) -> np.ndarray:
    """Algorithm 5: [h][2][L][N] -> the first m of the h 2^c expanded ciphertexts, [m][2][L][N].

    Each packed ciphertext goes through c levels of split_level; at level a the 2^a ciphertexts
    b < 2^a become 2^{a+1}, the even part staying at b and the odd part going to b + 2^a, so that
    after the last level ciphertext b carries plaintext coefficient b (times 2^c, which the client's
    2^-c pre-scale cancels)."""
    N = orc.N
    keys = {g: orc.load_key(gk) if isinstance(gk, np.ndarray) else gk for g, gk in gkeys.items()}
    out = []
    for ct in packed:
        cts = [np.array(ct, dtype=np.uint64)]
        for a in range(c):
            halves = [split_level(orc, keys[N // (1 << a) + 1], x, a) for x in cts]
            cts = [e for e, _ in halves] + [o for _, o in halves]
        out.extend(cts)
    return np.stack(out[:m])


def expand_sealpir(orc: Oracle, gkeys: dict, packed: np.ndarray, m: int, c: int) -> np.ndarray:
    """Algorithm 1 on each packed ciphertext, then the product by 2^-c mod t; first m outputs."""
    N, t = orc.N, orc.t
    keys = {g: orc.load_key(gk) if isinstance(gk, np.ndarray) else gk for g, gk in gkeys.items()}
    inv = np.zeros(N, dtype=np.uint64)
    inv[0] = pow(2, -c, t)
    out = []
    for ct in packed:
        cts = [np.array(ct, dtype=np.uint64)] + [None] * ((1 << c) - 1)
        for a in range(c):
            g = N // (1 << a) + 1
            for b in range(1 << a):
                c0 = cts[b]
                c1 = orc.mul_monomial(c0, 2 * N - (1 << a))
                cts[b] = orc.add(c0, orc.sub(keys[g], c0, g))
                cts[b + (1 << a)] = orc.add(c1, orc.sub(keys[g], c1, g))
        out.extend(orc.pm(x, inv) for x in cts)
    return np.stack(out[:m])


def _sub(orc: Oracle, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """a - b mod q (as a + (-1) b, with the negation done residue by residue)."""
    neg = np.empty_like(b)
    for j, p in enumerate(orc.primes):
        x = b[:, j, :]
        neg[:, j, :] = np.where(x == 0, np.uint64(0), np.uint64(p) - x)
    return orc.add(a, neg)


def noise_budget_bits(orc: Oracle) -> float:
    return math.log2((orc.q // orc.t) / 2)
