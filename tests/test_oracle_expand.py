"""Pins of the oracle's query packing and expansion (Algorithms 4, 5 and 1), CPU only.

* The automorphism x -> x^g equals polynomial composition over Z (the Python micro-oracle builds
  (x^g)^i by repeated negacyclic products), composes as sigma_g sigma_h = sigma_{g h mod 2N}, and
  the monomial product equals a schoolbook product by x^e.
* Sub_g is bit-identical between the C++ oracle and the micro-oracle, and decrypts to sigma_g of
  the message (key switching from s(x^g) back to s).
* Expansion: every expanded ciphertext decrypts to its codeword bit, brute force over all bits and
  several codewords (tiny and mid parameters, several compression factors), and Algorithm 1 fed an
  unscaled packing decrypts to the same bits (the appendix's equivalence, at the plaintext level).
* c = 0 packs one bit per ciphertext as the constant polynomial of that bit, as the c = 0 query.
"""
import numpy as np
import pytest

import datagen
from oracle import expand as X
from oracle.core import Oracle, negacyclic_mul_schoolbook
from oracle.mapping import codeword_bits
from oracle.micro import Micro
from test_oracle_pins import _primes_1_mod


def _bits_of(ct_list, orc, sk):
    out = []
    for ct in ct_list:
        msg, noise = orc.decrypt(sk, ct)
        out.append((msg, noise))
    return out


@pytest.mark.parametrize("N,bits,L", [(16, 36, 3), (32, 44, 2)])
def test_automorphism_and_monomial_match_polynomial_arithmetic(N, bits, L):
    primes = _primes_1_mod(2 * N, bits, L)
    orc, mic = Oracle(N, primes), Micro(N, primes)
    u = datagen.uniform_residues(primes, (2,), N, seed=N + bits)
    for g in (3, 5, N + 1, N // 2 + 1, 2 * N - 1):
        assert np.array_equal(orc.automorphism(u, g), mic.automorphism(u, g)), g
    for g, h in ((3, 5), (N + 1, N // 2 + 1), (7, 2 * N - 1)):
        lhs = orc.automorphism(orc.automorphism(u, h), g)
        assert np.array_equal(lhs, orc.automorphism(u, g * h % (2 * N)))
    for e in (0, 1, N - 1, N, N + 3, 2 * N - 2):
        got = orc.mul_monomial(u, e)
        assert np.array_equal(got, mic.mul_monomial(u, e))
        mono = np.zeros(N, np.uint64)
        for j, p in enumerate(primes):  # x^e as a residue polynomial, then a schoolbook product
            mono[:] = 0
            mono[e % N] = 1 if e < N else p - 1
            assert np.array_equal(got[0, j], negacyclic_mul_schoolbook(p, u[0, j].copy(), mono.copy()))


@pytest.mark.parametrize("N,bits,L", [(16, 36, 3), (32, 44, 3), (16, 55, 2)])
def test_substitution_matches_micro_oracle_and_decrypts(N, bits, L):
    primes = _primes_1_mod(2 * N, bits, L)
    orc, mic = Oracle(N, primes), Micro(N, primes)
    seed = 7 * N + bits
    sk = orc.keygen(datagen.words(seed, datagen.S_SECRET, N))
    rng = np.random.default_rng(seed)
    msg = rng.integers(0, 65537, N, dtype=np.uint64)
    ct = orc.encrypt(sk, msg, datagen.words(seed, datagen.S_QUERY, orc.rnd_words_encrypt()))
    for a, g in enumerate((N + 1, N // 2 + 1, 3)):
        gk = orc.galois_keygen(sk, g, datagen.words(seed, datagen.S_GALOIS, orc.rnd_words_rlk(), offset=a))
        got = orc.sub(orc.load_key(gk), ct, g)
        assert np.array_equal(got, mic.sub(gk, ct, g)), g
        want = [0] * N  # sigma_g(msg) mod t
        for i, v in enumerate(msg):
            pos = i * g % (2 * N)
            if pos < N:
                want[pos] = int(v)
            else:
                want[pos - N] = (-int(v)) % 65537
        assert list(orc.decrypt(sk, got)[0]) == want, g


def _instance(name):
    cfg = datagen.CONFIGS[name]
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    sk = orc.keygen(datagen.words(cfg.seed, datagen.S_SECRET, cfg.N))
    return cfg, orc, sk


@pytest.mark.parametrize("c", [0, 1, 3, 5])
def test_expansion_decrypts_to_every_codeword_bit_tiny(c):
    cfg, orc, sk = _instance("tiny")
    gk = X.galois_keys(orc, sk, c, cfg.seed)
    for draw, pos in enumerate(([0, 1], [3, 17], [22, 23])):
        bits = codeword_bits(pos, cfg.m)
        packed = X.pack_query(orc, sk, bits, c, cfg.seed, draw=draw)
        assert packed.shape[0] == -(-cfg.m // (1 << c))
        ex = X.expand(orc, gk, packed, cfg.m, c)
        assert ex.shape == (cfg.m, 2, cfg.L, cfg.N)
        for i, (msg, noise) in enumerate(_bits_of(ex, orc, sk)):
            want = np.zeros(cfg.N, np.uint64)
            want[0] = bits[i]
            assert np.array_equal(msg, want), (c, pos, i)
            assert noise < X.noise_budget_bits(orc) - 10


def test_c0_packing_is_one_constant_per_bit():
    cfg, orc, sk = _instance("tiny")
    bits = codeword_bits([2, 9], cfg.m)
    packed = X.pack_query(orc, sk, bits, 0, cfg.seed)
    assert np.array_equal(X.expand(orc, {}, packed, cfg.m, 0), packed)
    for i, (msg, _) in enumerate(_bits_of(packed, orc, sk)):
        assert int(msg[0]) == bits[i] and not msg[1:].any()


def test_algorithm1_and_algorithm5_decrypt_alike_tiny():
    cfg, orc, sk = _instance("tiny")
    c = 3
    gk = X.galois_keys(orc, sk, c, cfg.seed)
    bits = codeword_bits([5, 11], cfg.m)
    e5 = X.expand(orc, gk, X.pack_query(orc, sk, bits, c, cfg.seed), cfg.m, c)
    e1 = X.expand_sealpir(orc, gk, X.pack_query(orc, sk, bits, c, cfg.seed, prescale=False), cfg.m, c)
    d5 = [m for m, _ in _bits_of(e5, orc, sk)]
    d1 = [m for m, _ in _bits_of(e1, orc, sk)]
    for i in range(cfg.m):
        assert np.array_equal(d5[i], d1[i]) and int(d5[i][0]) == bits[i]


@pytest.mark.slow
def test_expansion_mid_parameters_c5():
    cfg, orc, sk = _instance("mid")
    c = 5
    gk = X.galois_keys(orc, sk, c, cfg.seed)
    bits = codeword_bits([1, 8, 20, 26], cfg.m)
    ex = X.expand(orc, gk, X.pack_query(orc, sk, bits, c, cfg.seed), cfg.m, c)
    for i, (msg, noise) in enumerate(_bits_of(ex, orc, sk)):
        assert int(msg[0]) == bits[i] and not msg[1:].any(), i
        assert noise < X.noise_budget_bits(orc) - 100
