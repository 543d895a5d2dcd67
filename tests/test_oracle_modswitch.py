"""Pins of the oracle's response compression (modulus switching from q to q' = q_0 ... q_{keep-1}).

* The C++ oracle and the pure-Python micro-oracle agree bit for bit (random residues and
  encryptions, every keep).
* Closed forms: coefficients that are multiples of r = q / q' divide exactly; constants at
  k r +- (r - 1)/2 and k r +- (r + 1)/2 round to the nearer integer on either side of zero
  (no ties: r is odd); keep = L is the identity.
* Decryption is preserved: a PIR answer (tiny, mid) switched to one or two primes decrypts under q'
  to the same message, with the switched noise below Delta'/2.
"""
import math

import numpy as np
import pytest

import datagen
from oracle.core import Oracle
from oracle.micro import Micro
from test_oracle_pins import _primes_1_mod


def _constant(primes, N, values):
    """residues [len(values)][L][N] of the integers `values` placed in coefficient 0"""
    out = np.zeros((len(values), len(primes), N), np.uint64)
    for r, v in enumerate(values):
        for j, p in enumerate(primes):
            out[r, j, 0] = v % p
    return out


@pytest.mark.parametrize("N,bits,L", [(16, 36, 3), (32, 44, 5), (16, 55, 4)])
def test_mod_switch_matches_micro_oracle(N, bits, L):
    primes = _primes_1_mod(2 * N, bits, L)
    orc, mic = Oracle(N, primes), Micro(N, primes)
    u = datagen.uniform_residues(primes, (2,), N, seed=3 * N + L)
    sk = orc.keygen(datagen.words(N + bits, datagen.S_SECRET, N))
    msg = np.random.default_rng(N).integers(0, 65537, N, dtype=np.uint64)
    ct = orc.encrypt(sk, msg, datagen.words(N + bits, datagen.S_QUERY, orc.rnd_words_encrypt()))
    for keep in range(1, L + 1):
        assert np.array_equal(orc.mod_switch(u, keep), mic.mod_switch(u, keep)), keep
        assert np.array_equal(orc.mod_switch(ct, keep), mic.mod_switch(ct, keep)), keep
    assert np.array_equal(orc.mod_switch(u, L), u)


def test_mod_switch_closed_forms():
    cfg = datagen.CONFIGS["mid"]
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    q = math.prod(cfg.primes)
    for keep in (1, 2, 4):
        qk = math.prod(cfg.primes[:keep])
        r = q // qk
        k = 123456789
        vals = [r * 7, -r * 7, k * r + (r - 1) // 2, k * r + (r + 1) // 2, -(k * r + (r - 1) // 2),
                -(k * r + (r + 1) // 2), (qk // 2) * r]
        want = [7, -7, k, k + 1, -k, -(k + 1), qk // 2]
        got = orc.mod_switch(_constant(cfg.primes, cfg.N, vals), keep)
        for i, w in enumerate(want):
            for j, p in enumerate(cfg.primes[:keep]):
                assert int(got[i, j, 0]) == w % p, (keep, i)
            assert not got[i, :, 1:].any()


@pytest.mark.parametrize("name,keeps", [("tiny", (1, 2)), ("mid", (1, 2))])
def test_switched_answer_decrypts_to_the_payload(instances, name, keeps):
    n = 8
    ins = instances(name, n=n)
    cfg = ins.cfg
    ans = ins.orc.answer(ins.key, ins.query, ins.codewords[:n], ins.payload[:n])
    want = ins.payload[ins.target][0].astype(np.uint64) if ins.target < n else None
    msg_full, _ = ins.orc.decrypt(ins.sk, ans[0])
    for keep in keeps:
        small = Oracle(cfg.N, cfg.primes[:keep], cfg.t)
        sw = ins.orc.mod_switch(ans[0], keep)
        msg, noise = small.decrypt(ins.sk, sw)
        assert np.array_equal(msg, msg_full), keep
        if want is not None:
            assert np.array_equal(msg, want)
        # the switched noise includes (q' mod t) m / t < 2^16 from the change of Delta
        assert noise < small.log2_half_delta() - 2, (keep, noise)
