"""Pins of the oracle's arithmetic constant-weight equality (Algorithm 2) on batch-encoded
ciphertexts, CPU only.

* Slots: psi is a primitive 2N-th root of unity mod t; decoding inverts encoding; the negacyclic
  product of two encodings (schoolbook, mod t) decodes to the slot-wise product.
* The algorithm itself (plaintext closed form): over every pair of codewords of CW(6, 2) and
  CW(7, 3), e = 1 exactly when the codewords are equal.
* On ciphertexts: N comparisons per evaluation, random codeword pairs per slot (about half equal),
  decrypt and decode to the indicator of equality (tiny, k = 2, depth 2; mid, k = 4, depth 3).
"""
import math

import numpy as np
import pytest

import datagen
from oracle import arith as A
from oracle.core import Oracle, negacyclic_mul_schoolbook
from oracle.mapping import codeword_bits, perfect_map

T = 65537


def test_slot_encoding():
    for N in (16, 4096):
        psi = A.slot_root(N, T)
        assert pow(psi, 2 * N, T) == 1 and pow(psi, N, T) == T - 1
        rng = np.random.default_rng(N)
        a, b = rng.integers(0, T, N, dtype=np.uint64), rng.integers(0, T, N, dtype=np.uint64)
        pa, pb = A.encode(a, N, T), A.encode(b, N, T)
        assert np.array_equal(A.decode(pa, T), a)
        prod = negacyclic_mul_schoolbook(T, pa.copy(), pb.copy())
        assert np.array_equal(A.decode(prod, T), a * b % np.uint64(T))


@pytest.mark.parametrize("m,k", [(6, 2), (7, 3)])
def test_algorithm2_is_an_equality_operator(m, k):
    codes = [codeword_bits(perfect_map(i, m, k), m) for i in range(math.comb(m, k))]
    n = len(codes)
    xs = np.array([codes[i] for i in range(n) for _ in range(n)]).T  # [m][pairs]
    ys = np.array([codes[j] for _ in range(n) for j in range(n)]).T
    e = A.plain_equality(xs, ys, k, T)
    want = np.array([int(i == j) for i in range(n) for j in range(n)])
    assert np.array_equal(e, want)


def _run(name, m, k, seed):
    cfg = datagen.CONFIGS[name]
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    sk = orc.keygen(datagen.words(seed, datagen.S_SECRET, cfg.N))
    key = orc.load_key(orc.relin_keygen(sk, datagen.words(seed, datagen.S_RLK, orc.rnd_words_rlk())))
    rng = np.random.default_rng(seed)
    ncodes = math.comb(m, k)
    xi = rng.integers(0, ncodes, cfg.N)
    yi = np.where(rng.integers(0, 2, cfg.N) == 1, xi, rng.integers(0, ncodes, cfg.N))
    xb = np.array([codeword_bits(perfect_map(int(i), m, k), m) for i in xi]).T  # [m][N]
    yb = np.array([codeword_bits(perfect_map(int(i), m, k), m) for i in yi]).T
    per = orc.rnd_words_encrypt()
    enc = lambda bits, off: np.stack([orc.encrypt(sk, A.encode(bits[i], cfg.N, cfg.t),  # noqa: E731
                                                  datagen.words(seed, datagen.S_QUERY, per, offset=(off + i) * per))
                                      for i in range(m)])
    x, y = enc(xb, 0), enc(yb, m)
    e = A.arith_equality(orc, key, x, y, k)
    msg, noise = orc.decrypt(sk, e)
    return A.decode(msg, cfg.t), (xi == yi).astype(np.uint64), noise, orc.log2_half_delta(), (x, y, e)


def test_arith_equality_tiny_k2():
    # depth 2 with full-slot plaintexts is at the edge of the tiny budget (the paper's table has no
    # N = 4096 entry at depth 2); the decoded result is still exact
    got, want, noise, budget, _ = _run("tiny", 6, 2, 71)
    assert np.array_equal(got, want)
    assert noise < budget - 2


def test_arith_equality_mid_k4():
    got, want, noise, budget, _ = _run("mid", 8, 4, 72)
    assert np.array_equal(got, want)
    assert noise < budget - 10
