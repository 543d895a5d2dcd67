"""Seeded query ciphertexts: the compressed upload of secret-key encryption (test infrastructure).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg may use this
module; the product path never does.

What it computes (paper, Section 2, the optimisations of SealPIR: encrypting the query with the
secret key instead of the public key compresses the uploaded ciphertexts; the upload column of the
communication-cost table).  A secret-key ciphertext ([-a s + e + Delta m]_q, a) carries a uniform
second polynomial a that the client need not send: it sends c0 and a 64-bit seed, and the server
regenerates a from the seed.

Reading (the paper names no generator).  The seed is the starting state of SplitMix64 (Steele, Lea
and Flood, OOPSLA 2014): output number v + 1 of that sequence is
    W(v) = mix64(seed + (v + 1) gamma mod 2^64),   gamma = 0x9E3779B97F4A7C15,
and ciphertext i of a seeded batch takes the residue of limb j, coefficient c from the two words at
u = (i L + j) N + c, the same two-word uniform draw as the encryption routine:
    a_i[j][c] = (W(2u) 2^64 + W(2u + 1)) mod q_j.
The 128-bit value is reduced once, so each residue is within 2^-(128 - log2 q_j) of uniform.
"""
from __future__ import annotations

import numpy as np

import datagen
from .core import Oracle
from .mapping import codeword_bits, mix64

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


def splitmix_words(seed: int, start: int, count: int) -> list:
    """W(start), ..., W(start + count - 1) of the sequence started from state `seed`."""
    return [mix64((seed + (v + 1) * GAMMA) & MASK64) for v in range(start, start + count)]


def splitmix_words_np(seed: int, start: int, count: int) -> np.ndarray:
    """The same words, computed with wrapping uint64 arithmetic (for large counts)."""
    v = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + v * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def seeded_a(primes, N: int, seed: int, count: int) -> np.ndarray:
    """The second polynomials a_i, i < count, of a seeded batch: uint64 [count][L][N]."""
    L = len(primes)
    out = np.empty((count, L, N), dtype=np.uint64)
    for i in range(count):
        for j, q in enumerate(primes):
            u0 = (i * L + j) * N
            w = splitmix_words_np(seed, 2 * u0, 2 * N).tolist()
            out[i, j] = [((w[2 * c] << 64) | w[2 * c + 1]) % q for c in range(N)]
    return out


def unseed(primes, N: int, c0: np.ndarray, seed: int) -> np.ndarray:
    """Full ciphertexts [count][2][L][N] from their first polynomials c0 [count][L][N] and the seed."""
    c0 = np.asarray(c0, dtype=np.uint64)
    out = np.empty((c0.shape[0], 2) + c0.shape[1:], dtype=np.uint64)
    out[:, 0] = c0
    out[:, 1] = seeded_a(primes, N, seed, c0.shape[0])
    return out


def encrypt_seeded(orc: Oracle, sk: np.ndarray, messages, seed: int, err_seed: int) -> np.ndarray:
    """Secret-key encryptions of the plaintexts `messages` [count][N] whose a polynomials come from
    `seed`: returns the full ciphertexts [count][2][L][N] (the client sends only [:, 0] and the
    seed).  Errors come from the seeded-query stream of `err_seed`."""
    L, N = orc.L, orc.N
    out = np.empty((len(messages), 2, L, N), dtype=np.uint64)
    for i, msg in enumerate(messages):
        ra = splitmix_words_np(seed, i * 2 * L * N, 2 * L * N)
        re = datagen.words(err_seed, datagen.S_SEEDED, N, offset=i * N)
        out[i] = orc.encrypt(sk, np.asarray(msg, dtype=np.uint64), np.concatenate([ra, re]))
    return out


def seeded_query(orc: Oracle, sk: np.ndarray, positions, m: int, seed: int, err_seed: int) -> np.ndarray:
    """A constant-weight query (one ciphertext per codeword bit, the constant polynomial of the bit)
    encrypted with seeded a polynomials: full ciphertexts [m][2][L][N]."""
    msgs = np.zeros((m, orc.N), dtype=np.uint64)
    msgs[:, 0] = codeword_bits(positions, m)
    return encrypt_seeded(orc, sk, msgs, seed, err_seed)


def seeded_pack(orc: Oracle, sk: np.ndarray, bits, c: int, seed: int, err_seed: int) -> np.ndarray:
    """A packed query (Algorithm 4) encrypted with seeded a polynomials: [h][2][L][N]."""
    from .expand import pack_messages
    return encrypt_seeded(orc, sk, pack_messages(bits, c, orc.N, orc.t), seed, err_seed)
