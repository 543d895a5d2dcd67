"""Pins of the oracle's folklore PIR and of product trees beyond k = 4, CPU only.

* 1 - ct decrypts to 1 - m (mod t) for random messages, and is bit-identical to the Python
  micro-oracle's (Delta - c0, -c1).
* The folklore codeword of element j has weight l and selects leaf 2i + bit_i(j), ascending.
* The plain folklore equality operator, evaluated as the product tree over the 2l leaves, decrypts
  to 1 exactly at the queried index and to 0 at every other index (brute force over all 16
  elements, l = 4, depth 2, mid parameters), and a 64-element answer (l = 6, depth 3) decrypts to
  the queried payload.
* Constant-weight trees with k = 5 and k = 8 (depth 3, mid parameters): the answer over every
  codeword of CW(8, 5) and CW(10, 8) with random payloads decrypts to the target's payload.
"""
import math

import numpy as np

import datagen
from oracle.client import encrypt_query
from oracle.core import Oracle
from oracle.folklore import folklore_codewords, folklore_leaves, folklore_query, index_bits
from oracle.mapping import perfect_map
from oracle.micro import Micro
from test_oracle_pins import _primes_1_mod

TINY = datagen.CONFIGS["tiny"]


def _keys(orc, seed):
    sk = orc.keygen(datagen.words(seed, datagen.S_SECRET, orc.N))
    rlk = orc.relin_keygen(sk, datagen.words(seed, datagen.S_RLK, orc.rnd_words_rlk()))
    return sk, orc.load_key(rlk)


def test_one_minus_decrypts_and_matches_micro():
    N = 32
    primes = _primes_1_mod(2 * N, 44, 3)
    orc, mic = Oracle(N, primes), Micro(N, primes)
    sk = orc.keygen(datagen.words(5, datagen.S_SECRET, N))
    msg = np.random.default_rng(1).integers(0, 65537, N, dtype=np.uint64)
    ct = orc.encrypt(sk, msg, datagen.words(5, datagen.S_QUERY, orc.rnd_words_encrypt()))
    om = orc.one_minus(ct)
    want = [(1 - int(m)) % 65537 if i == 0 else (-int(m)) % 65537 for i, m in enumerate(msg)]
    assert list(orc.decrypt(sk, om)[0]) == want
    c0, c1 = mic.to_int(ct[0]), mic.to_int(ct[1])
    ref = np.stack([mic.to_res([((mic.delta if i == 0 else 0) - v) % mic.q for i, v in enumerate(c0)]),
                    mic.to_res([(-v) % mic.q for v in c1])])
    assert np.array_equal(om, ref)


def test_folklore_codewords():
    cw = folklore_codewords(40, 6)
    assert cw.shape == (40, 6)
    for j in range(40):
        assert list(cw[j]) == [2 * i + ((j >> i) & 1) for i in range(6)]
    assert index_bits(64) == 6 and index_bits(65) == 7 and index_bits(2) == 1


MID = datagen.CONFIGS["mid"]  # a depth-3 folklore tree needs more than the tiny noise budget


def test_folklore_equality_brute_force_depth2():
    n = 16
    ell = index_bits(n)
    orc = Oracle(MID.N, MID.primes, MID.t)
    sk, key = _keys(orc, 41)
    target = 11
    leaves = folklore_leaves(orc, folklore_query(orc, sk, target, ell, 41))
    cw = folklore_codewords(n, ell)
    for j in range(n):
        msg, noise = orc.decrypt(sk, orc.selector(key, leaves, cw[j]))
        assert int(msg[0]) == (j == target) and not msg[1:].any(), j
        assert noise < orc.log2_half_delta() - 10


def test_folklore_answer_depth3_decrypts_to_the_payload():
    n = 64
    ell = index_bits(n)
    orc = Oracle(MID.N, MID.primes, MID.t)
    sk, key = _keys(orc, 42)
    target = 45
    leaves = folklore_leaves(orc, folklore_query(orc, sk, target, ell, 42))
    pay = datagen.payload(MID.with_n(n), n)
    ans = orc.answer(key, leaves, folklore_codewords(n, ell), pay)
    msg, noise = orc.decrypt(sk, ans[0])  # = sum_j sel_j P_j: only the target's selector is 1
    assert np.array_equal(msg, pay[target][0].astype(np.uint64))
    assert noise < orc.log2_half_delta() - 10


def test_constant_weight_trees_k5_k8_answers():
    """Every element's selector enters the answer; with random payloads the answer decrypts to the
    target's payload only if the selector is 1 at the target and 0 at every other codeword."""
    orc = Oracle(MID.N, MID.primes, MID.t)
    sk, key = _keys(orc, 43)
    for k, m in ((5, 8), (8, 10)):
        codes = np.array([perfect_map(i, m, k) for i in range(math.comb(m, k))], dtype=np.uint32)
        target = len(codes) // 3
        query = encrypt_query(orc, sk, [int(v) for v in codes[target]], m, 43, draw=k)
        pay = datagen.payload(MID.with_n(len(codes)), len(codes))
        msg, noise = orc.decrypt(sk, orc.answer(key, query, codes, pay)[0])
        assert np.array_equal(msg, pay[target][0].astype(np.uint64)), k
        assert noise < orc.log2_half_delta() - 10, (k, noise)
