"""Folklore PIR with the plain folklore equality operator (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg may use this
module; the product path never does.

The plain folklore operator (Section 2.4, equation of f_PF) compares an encrypted l-bit string x with
a public one y: f_PF(x, y) = prod_{y[i]=0} (1 - x[i]) prod_{y[i]=1} x[i], multiplicative depth
ceil(log2 l).  In index PIR the query is the l = ceil(log2 n) bits of the target index, one
ciphertext per bit (the constant polynomial of the bit); the server forms 1 - x[i] homomorphically.

Readings.  Bit i of index j is (j >> i) & 1 (least significant first).  The 2l leaves are ordered
leaf 2i = 1 - x[i], leaf 2i + 1 = x[i], so element j's factors are the leaves 2i + bit_i(j),
ascending in i, and the product is the same tree as the constant-weight operator's (neighbours
paired level by level, an odd last factor carried up, a relinearization after every
multiplication): f_PF is the constant-weight product over a weight-l word of length 2l.
"""
from __future__ import annotations

import numpy as np

import datagen
from .core import Oracle


def index_bits(n: int) -> int:
    """l = ceil(log2 n), at least 1."""
    return max(1, (n - 1).bit_length())


def folklore_codewords(n: int, ell: int) -> np.ndarray:
    """uint32 [n][ell]: element j's leaf positions 2i + bit_i(j)."""
    j = np.arange(n, dtype=np.uint64)[:, None]
    i = np.arange(ell, dtype=np.uint64)[None, :]
    return (2 * i + ((j >> i) & np.uint64(1))).astype(np.uint32)


def folklore_query(orc: Oracle, sk: np.ndarray, target: int, ell: int, seed: int, draw: int = 0) -> np.ndarray:
    """The client's query: ell ciphertexts [ell][2][L][N], ciphertext i encrypting bit i of target."""
    per = orc.rnd_words_encrypt()
    out = np.empty((ell, 2, orc.L, orc.N), dtype=np.uint64)
    for i in range(ell):
        msg = np.zeros(orc.N, dtype=np.uint64)
        msg[0] = (target >> i) & 1
        out[i] = orc.encrypt(sk, msg, datagen.words(seed, datagen.S_QUERY, per, offset=(draw * ell + i) * per))
    return out


def folklore_leaves(orc: Oracle, query: np.ndarray) -> np.ndarray:
    """The server's 2 ell leaves: [1 - x[0], x[0], 1 - x[1], x[1], ...]."""
    out = np.empty((2 * query.shape[0],) + query.shape[1:], dtype=np.uint64)
    for i, ct in enumerate(query):
        out[2 * i] = orc.one_minus(ct)
        out[2 * i + 1] = ct
    return out
