"""Pins of the oracle's seeded query ciphertexts (compressed upload of secret-key encryption), CPU only.

* The generator: the first SplitMix64 outputs from state 0 equal the published known-answer values
  (tests/golden/splitmix64_state0.txt), in both the scalar and the vectorised form, so the counter
  offset (output number v + 1 for word v) and the mix are fixed.
* The residues: the oracle's Python big-integer reduction of the two-word draw equals the a
  polynomial that the C++ oracle's encryption routine builds from the same words (a second,
  independent implementation of (w1 2^64 + w2) mod q_j), for every limb and ciphertext of a batch.
* Uniformity: a chi-square test over the top bits of the residues of every limb.
* The protocol: a seeded query decrypts bit for bit to its codeword, and the PIR answer computed
  from the unseeded query decrypts to the queried payload.
"""
import os

import numpy as np
import pytest

import datagen
from oracle import seeded as S
from oracle.client import build_instance
from oracle.core import Oracle
from oracle.mapping import codeword_bits

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "splitmix64_state0.txt")) as f:
        return [int(x, 16) for x in f if x.strip() and not x.startswith("#")]


def test_splitmix_known_answers():
    want = _golden()
    assert S.splitmix_words(0, 0, len(want)) == want
    assert S.splitmix_words_np(0, 0, len(want)).tolist() == want
    # a later window of the same sequence agrees between the two forms
    assert S.splitmix_words(0x0123456789ABCDEF, 1000, 7) == S.splitmix_words_np(0x0123456789ABCDEF, 1000, 7).tolist()


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_residues_match_the_encryption_routine(name):
    cfg = datagen.CONFIGS[name]
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    sk = orc.keygen(datagen.words(cfg.seed, datagen.S_SECRET, cfg.N))
    seed = 0xC0FFEE1234567890
    msgs = np.zeros((3, cfg.N), dtype=np.uint64)
    cts = S.encrypt_seeded(orc, sk, msgs, seed, err_seed=cfg.seed)
    a = S.seeded_a(cfg.primes, cfg.N, seed, 3)
    assert np.array_equal(cts[:, 1], a)
    assert np.array_equal(S.unseed(cfg.primes, cfg.N, cts[:, 0], seed), cts)
    assert all(int(a[:, j].max()) < q for j, q in enumerate(cfg.primes))


def test_residues_are_uniform():
    cfg = datagen.CONFIGS["tiny"]
    a = S.seeded_a(cfg.primes, cfg.N, 77, 4)  # 4 ciphertexts x 3 limbs x 4096 residues
    bins = 16
    for j, q in enumerate(cfg.primes):
        x = a[:, j].reshape(-1).astype(np.float64)
        counts = np.bincount((x * bins / q).astype(np.int64), minlength=bins)
        e = x.size / bins
        chi2 = float(((counts - e) ** 2 / e).sum())
        assert chi2 < 40.0, (j, chi2)  # 15 degrees of freedom: P(chi2 > 40) < 1e-3


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_seeded_query_decrypts_and_answers(name):
    cfg = datagen.CONFIGS[name]
    inst = build_instance(cfg.with_n(12))
    q = S.seeded_query(inst.orc, inst.sk, inst.positions, cfg.m, seed=99, err_seed=cfg.seed)
    bits = codeword_bits(inst.positions, cfg.m)
    for i in range(cfg.m):
        msg, noise = inst.orc.decrypt(inst.sk, q[i])
        assert int(msg[0]) == bits[i] and not msg[1:].any()
        assert noise < inst.orc.log2_half_delta() - 10
    full = S.unseed(cfg.primes, cfg.N, q[:, 0], 99)
    assert np.array_equal(full, q)
    ans = inst.orc.answer(inst.key, full, inst.codewords, inst.payload)
    msg, _ = inst.orc.decrypt(inst.sk, ans[0])
    assert np.array_equal(msg, inst.payload[inst.target][0].astype(np.uint64))
