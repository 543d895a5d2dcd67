"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names what it pins:
  P1 code length rule          printed tables of the paper (golden file)
  P2 perfect mapping           brute-force sorted enumeration, Algorithm 7 round trip, order
  P3 lossy mapping             weight, range, uniformity over the code (collision Theorem)
  P4 polynomial products       schoolbook negacyclic convolution
  P5 exact Mult rounding       closed form on constant polynomials, near-half vectors
  P6 FV homomorphism           decryption of Enc, Mult, Relin, PM, Add
  P7 equality operator         decrypted selector is 1 exactly at the queried codeword
  P8 PIR answer                decrypted answer is the queried payload, zero when absent
  P9 linearity                 answer over a database = sum of answers over a split
  -- second implementation     pure-Python FV (oracle.micro) agrees bit for bit at tiny N
"""
import itertools
import math
import os
import random

import numpy as np
import pytest

import datagen
from oracle import (binom, code_length, divmod_big, inverse_perfect_map, lossy_map,
                    negacyclic_mul_ntt, negacyclic_mul_schoolbook, perfect_map)
from oracle.client import build_instance
from oracle.core import Oracle
from oracle.micro import Micro

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _is_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _primes_1_mod(mod, bits, count):
    out, c = [], ((1 << bits) - 1) // mod * mod + 1
    while len(out) < count:
        if c < (1 << bits) and _is_prime(c):
            out.append(c)
        c -= mod
    return out


def _golden_code_lengths():
    rows = []
    with open(os.path.join(GOLDEN, "code_lengths.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            src, k, lg, m = line.split()
            rows.append((src, int(k), int(lg), int(m)))
    return rows


# ---------------------------------------------------------------------------------------------
# P1
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("src,k,lg,m", _golden_code_lengths())
def test_code_length_matches_paper_tables(src, k, lg, m):
    assert code_length(1 << lg, k) == m


def test_workload_code_lengths():
    c = datagen.CONFIGS
    assert c["tiny"].m == code_length(c["tiny"].n, 2) == 24
    assert c["mid"].m == code_length(c["mid"].n, 4) == 27
    assert c["keyword"].m == code_length(1 << 32, 4) == 569
    assert c["large"].m == code_length(c["large"].n, 2) == 725
    for cfg in datagen.batched_configs():
        assert binom(cfg.m, cfg.k) >= cfg.n > binom(cfg.m - 1, cfg.k)


def test_workload_primes():
    """Every ciphertext prime is prime, 1 mod 2N, and the listed ones are the largest such below
    their bit bound (the reading for the unspecified moduli)."""
    for cfg in (datagen.CONFIGS["tiny"], datagen.CONFIGS["mid"], datagen.CONFIGS["keyword"]):
        for p in cfg.primes:
            assert _is_prime(p) and p % (2 * cfg.N) == 1
    assert list(datagen.Q_N4096) == _primes_1_mod(2 * 4096, 36, 3)
    assert list(datagen.Q_N8192[:2]) == _primes_1_mod(2 * 8192, 43, 2)
    assert list(datagen.Q_N8192[2:]) == _primes_1_mod(2 * 8192, 44, 3)
    assert list(datagen.Q_N16384[:2]) == _primes_1_mod(2 * 16384, 54, 2)
    assert list(datagen.Q_N16384[2:]) == _primes_1_mod(2 * 16384, 55, 6)
    assert math.prod(datagen.Q_N8192).bit_length() == 218
    assert math.prod(datagen.Q_N16384).bit_length() == 438


# ---------------------------------------------------------------------------------------------
# P2
# ---------------------------------------------------------------------------------------------
def test_perfect_map_is_the_sorted_enumeration():
    """Algorithm 3 assigns the i-th codeword of the sorted list of CW(m, k) to i (sorted as binary
    numbers with position m' worth 2^m'); Algorithm 7 inverts it."""
    for m in range(1, 11):
        for k in range(1, m + 1):
            code = sorted(itertools.combinations(range(m), k), key=lambda c: sum(1 << p for p in c))
            assert len(code) == binom(m, k)
            for i, c in enumerate(code):
                assert perfect_map(i, m, k) == list(c)
                assert inverse_perfect_map(list(c), m) == i


def test_perfect_map_round_trip_and_order_at_workload_sizes():
    rng = random.Random(7)
    for m, k in ((24, 2), (27, 4), (725, 2), (569, 4)):
        size = binom(m, k)
        xs = sorted(rng.randrange(size) for _ in range(200)) + [0, size - 1]
        prev = -1
        for x in sorted(set(xs)):
            ones = perfect_map(x, m, k)
            assert len(ones) == k and len(set(ones)) == k and all(0 <= p < m for p in ones)
            assert inverse_perfect_map(ones, m) == x
            val = sum(1 << p for p in ones)
            assert val > prev          # order preserving
            prev = val
    with pytest.raises(ValueError):
        perfect_map(binom(24, 2), 24, 2)


# ---------------------------------------------------------------------------------------------
# P3
# ---------------------------------------------------------------------------------------------
def test_lossy_map_weight_and_range():
    for x in range(500):
        ones = lossy_map(x * 0x1234567 + 11, 569, 4, seed=99)
        assert len(ones) == 4 and ones == sorted(set(ones)) and all(0 <= p < 569 for p in ones)


def test_lossy_map_uniform_over_the_code():
    """Collision Theorem for Algorithm 8: every codeword has probability 1/C(m, k).  Chi-square
    over CW(10, 3) (120 codewords) and the empirical pair-collision rate."""
    m, k, trials = 10, 3, 60000
    counts = {}
    for x in range(trials):
        cw = tuple(lossy_map(x, m, k, seed=0xC0FFEE))
        counts[cw] = counts.get(cw, 0) + 1
    size = binom(m, k)
    assert len(counts) == size
    exp = trials / size
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    dof = size - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    coll = sum(c * (c - 1) for c in counts.values()) / (trials * (trials - 1))
    assert abs(coll - 1 / size) < 0.1 / size


# ---------------------------------------------------------------------------------------------
# big integers
# ---------------------------------------------------------------------------------------------
def test_big_division_matches_python_integers():
    rng = random.Random(3)
    for _ in range(300):
        a = rng.getrandbits(rng.randrange(1, 960))
        b = rng.getrandbits(rng.randrange(1, 480)) | 1
        assert divmod_big(a, b) == divmod(a, b)
    assert divmod_big((1 << 900) - 1, (1 << 64) + 1) == divmod((1 << 900) - 1, (1 << 64) + 1)


# ---------------------------------------------------------------------------------------------
# P4
# ---------------------------------------------------------------------------------------------
def _rand_poly(rng, N, p):
    return np.array([rng.randrange(p) for _ in range(N)], dtype=np.uint64)


@pytest.mark.parametrize("N,p", [(16, 97), (64, 7681), (1024, _primes_1_mod(2048, 62, 1)[0])]
                         + [(4096, p) for p in datagen.Q_N4096] + [(8192, datagen.Q_N8192[2])])
def test_ntt_product_equals_schoolbook(N, p):
    rng = random.Random(N ^ p)
    a, b = _rand_poly(rng, N, p), _rand_poly(rng, N, p)
    assert np.array_equal(negacyclic_mul_ntt(p, a, b), negacyclic_mul_schoolbook(p, a, b))


def test_ntt_product_at_n16384_sampled_coefficients():
    N, p = 16384, datagen.Q_N16384[2]
    rng = random.Random(11)
    a, b = _rand_poly(rng, N, p), _rand_poly(rng, N, p)
    out = negacyclic_mul_ntt(p, a, b)
    A, B = [int(v) for v in a], [int(v) for v in b]
    for k in (0, 1, 777, N // 2, N - 1):
        v = sum(A[i] * B[k - i] for i in range(k + 1)) - sum(A[i] * B[N + k - i] for i in range(k + 1, N))
        assert int(out[k]) == v % p


# ---------------------------------------------------------------------------------------------
# P5
# ---------------------------------------------------------------------------------------------
def _const_ct(orc, c0, c1):
    ct = np.zeros((2, orc.L, orc.N), dtype=np.uint64)
    for j, p in enumerate(orc.primes):
        ct[0, j, 0] = c0 % p
        ct[1, j, 0] = c1 % p
    return ct


def _centred(x, q):
    x %= q
    return x - q if x > q // 2 else x


def _closed_form(orc, a, b):
    q, t = orc.q, orc.t
    A = [_centred(v, q) for v in a]
    B = [_centred(v, q) for v in b]
    X = [A[0] * B[0], A[0] * B[1] + A[1] * B[0], A[1] * B[1]]
    return [((2 * t * x + q) // (2 * q)) % q for x in X]


def _const_of(orc, ct_poly):
    q = orc.q
    x = 0
    for j, p in enumerate(orc.primes):
        Mj = q // p
        x += int(ct_poly[j][0]) * Mj * pow(Mj, -1, p)
    return x % q


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_mult_closed_form_on_constants(name):
    cfg = datagen.CONFIGS[name]
    orc = Oracle(cfg.N, cfg.primes, cfg.t) if name == "tiny" else Oracle(1024, _primes_1_mod(2048, 44, 5))
    q, t = orc.q, orc.t
    rng = random.Random(5)
    inv_t = pow(t, -1, q)
    cases = [(rng.randrange(q), rng.randrange(q), rng.randrange(q), rng.randrange(q)) for _ in range(4)]
    # near-half vectors: t * a0 = j q + (q -/+ 1)/2, paired with b = (1, 0)
    cases += [((q - 1) // 2 * inv_t % q, rng.randrange(q), 1, 0), ((q + 1) // 2 * inv_t % q, rng.randrange(q), 1, 0),
              ((q - (q - 1) // 2) * inv_t % q, 3, 1, 0), (q - 1, q - 1, q - 1, q - 1), (0, 0, 5, 7)]
    for a0, a1, b0, b1 in cases:
        out = orc.mult(_const_ct(orc, a0, a1), _const_ct(orc, b0, b1))
        exp = _closed_form(orc, (a0, a1), (b0, b1))
        for r in range(3):
            assert _const_of(orc, out[r]) == exp[r]
            assert not out[r][:, 1:].any()
    # the near-half pair rounds down and up respectively
    lo = _closed_form(orc, ((q - 1) // 2 * inv_t % q, 0), (1, 0))[0]
    hi = _closed_form(orc, ((q + 1) // 2 * inv_t % q, 0), (1, 0))[0]
    a_lo = _centred((q - 1) // 2 * inv_t % q, q)
    assert (t * a_lo - (q - 1) // 2) % q == 0
    assert lo == ((t * a_lo - (q - 1) // 2) // q) % q
    a_hi = _centred((q + 1) // 2 * inv_t % q, q)
    assert hi == ((t * a_hi - (q + 1) // 2) // q + 1) % q


# ---------------------------------------------------------------------------------------------
# second implementation (pure Python FV) at tiny N
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("N,bits,L", [(16, 36, 3), (32, 44, 5), (16, 55, 2)])
def test_cpp_oracle_matches_python_micro_oracle(N, bits, L):
    primes = _primes_1_mod(2 * N, bits, L)
    orc, mic = Oracle(N, primes), Micro(N, primes)
    seed = N * 1000 + bits
    sk = orc.keygen(datagen.words(seed, 1, N))
    rlk = orc.relin_keygen(sk, datagen.words(seed, 2, orc.rnd_words_rlk()))
    key = orc.load_key(rlk)
    rng = np.random.default_rng(seed)
    m1 = rng.integers(0, 65537, N, dtype=np.uint64)
    m2 = rng.integers(0, 65537, N, dtype=np.uint64)
    r1 = datagen.words(seed, 3, orc.rnd_words_encrypt())
    r2 = datagen.words(seed, 3, orc.rnd_words_encrypt(), offset=orc.rnd_words_encrypt())
    c1, c2 = orc.encrypt(sk, m1, r1), orc.encrypt(sk, m2, r2)
    assert np.array_equal(c1, mic.encrypt(sk, m1, r1))
    assert np.array_equal(c2, mic.encrypt(sk, m2, r2))
    assert list(orc.decrypt(sk, c1)[0]) == mic.decrypt(sk, c1) == [int(v) for v in m1]
    prod = orc.mult(c1, c2)
    assert np.array_equal(prod, mic.mult(c1, c2))
    assert list(orc.decrypt(sk, prod)[0]) == mic.decrypt(sk, prod)
    rel = orc.relin(key, prod)
    assert np.array_equal(rel, mic.relin(rlk, prod))
    assert list(orc.decrypt(sk, rel)[0]) == mic.decrypt(sk, prod)
    pt = rng.integers(0, 1 << 16, N, dtype=np.uint64)
    assert np.array_equal(orc.pm(c1, pt), mic.pm(c1, pt))
    # arbitrary residues (not encryptions) exercise every lift
    u = datagen.uniform_residues(primes, (2, 2), N, seed)
    assert np.array_equal(orc.mult(u[0], u[1]), mic.mult(u[0], u[1]))


# ---------------------------------------------------------------------------------------------
# P6
# ---------------------------------------------------------------------------------------------
def test_fv_homomorphism_tiny(instances):
    inst = instances("tiny", n=16)
    orc, sk = inst.orc, inst.sk
    N, t = orc.N, orc.t
    rng = np.random.default_rng(1)
    m1 = rng.integers(0, t, N, dtype=np.uint64)
    m2 = rng.integers(0, t, N, dtype=np.uint64)
    per = orc.rnd_words_encrypt()
    c1 = orc.encrypt(sk, m1, datagen.words(77, 3, per))
    c2 = orc.encrypt(sk, m2, datagen.words(77, 3, per, offset=per))
    d1, n1 = orc.decrypt(sk, c1)
    assert np.array_equal(d1, m1) and n1 < 8
    assert np.array_equal(orc.decrypt(sk, orc.add(c1, c2))[0], (m1 + m2) % t)
    want = negacyclic_mul_schoolbook(t, m1, m2)
    prod = orc.mult(c1, c2)
    d3, n3 = orc.decrypt(sk, prod)
    assert np.array_equal(d3, want)
    rel = orc.relin(inst.key, prod)
    d2, n2 = orc.decrypt(sk, rel)
    assert np.array_equal(d2, want)
    assert n2 < orc.log2_half_delta() - 10
    pt = rng.integers(0, 1 << 16, N, dtype=np.uint64)
    assert np.array_equal(orc.decrypt(sk, orc.pm(c1, pt))[0], negacyclic_mul_schoolbook(t, m1, pt))


# ---------------------------------------------------------------------------------------------
# P7
# ---------------------------------------------------------------------------------------------
def test_equality_is_one_exactly_at_the_query_tiny_all_elements(instances):
    cfg = datagen.CONFIGS["tiny"].with_n(64, m=code_length(64, 2))
    inst = instances(cfg)
    ones = np.zeros(inst.orc.N, dtype=np.uint64)
    ones[0] = 1
    zero = np.zeros(inst.orc.N, dtype=np.uint64)
    worst = 0.0
    for j in range(cfg.n):
        sel = inst.orc.selector(inst.key, inst.query, inst.codewords[j])
        msg, noise = inst.orc.decrypt(inst.sk, sel)
        worst = max(worst, noise)
        assert np.array_equal(msg, ones if j == inst.target else zero), j
    assert worst < inst.orc.log2_half_delta() - 30


def test_equality_depth2_all_elements_k4():
    """k = 4 (depth 2) on the 4096-degree parameters, every element of a 15-element code."""
    cfg = datagen.Config("tiny-k4", 4096, datagen.Q_N4096, 65537, 4, 6, 15, 1, 21)
    inst = build_instance(cfg)
    for j in range(cfg.n):
        msg, noise = inst.orc.decrypt(inst.sk, inst.orc.selector(inst.key, inst.query, inst.codewords[j]))
        assert int(msg[0]) == (1 if j == inst.target else 0) and not msg[1:].any()
        assert noise < inst.orc.log2_half_delta() - 8


@pytest.mark.slow
def test_equality_mid_parameters(instances):
    inst = instances("mid", n=8)
    for j in (inst.target, (inst.target + 1) % 8):
        msg, noise = inst.orc.decrypt(inst.sk, inst.orc.selector(inst.key, inst.query, inst.codewords[j]))
        assert int(msg[0]) == (1 if j == inst.target else 0) and not msg[1:].any()
        assert noise < inst.orc.log2_half_delta() - 80


# ---------------------------------------------------------------------------------------------
# P8, P9
# ---------------------------------------------------------------------------------------------
def test_answer_decrypts_to_the_payload_tiny_full(instances):
    inst = instances("tiny")
    ans = inst.orc.answer(inst.key, inst.query, inst.codewords, inst.payload, threads=0)
    msg, noise = inst.orc.decrypt(inst.sk, ans[0])
    assert np.array_equal(msg, inst.payload[inst.target][0].astype(np.uint64))
    assert noise < inst.orc.log2_half_delta() - 12


KW_SMALL = datagen.Config("kw-small", 4096, datagen.Q_N4096, 65537, 2, 24, 16, 2, 7, keyword=True)


def test_keyword_answer_present_and_absent(instances):
    inst = instances(KW_SMALL)
    ans = inst.orc.answer(inst.key, inst.query, inst.codewords, inst.payload)
    for r in range(KW_SMALL.s):
        assert np.array_equal(inst.orc.decrypt(inst.sk, ans[r])[0], inst.payload[inst.target][r].astype(np.uint64))
    absent = instances(KW_SMALL, absent=True)
    assert absent.target == -1
    assert not any(list(cw) == absent.positions for cw in absent.codewords.tolist())
    ans = absent.orc.answer(absent.key, absent.query, absent.codewords, absent.payload)
    for r in range(KW_SMALL.s):
        assert not absent.orc.decrypt(absent.sk, ans[r])[0].any()


def test_answer_is_linear_over_a_split(instances):
    inst = instances("tiny", n=40)
    q = np.array(inst.orc.primes, dtype=np.uint64).reshape(1, 1, -1, 1)
    full = inst.orc.answer(inst.key, inst.query, inst.codewords, inst.payload)
    a = inst.orc.answer(inst.key, inst.query, inst.codewords[:23], inst.payload[:23])
    b = inst.orc.answer(inst.key, inst.query, inst.codewords[23:], inst.payload[23:])
    assert np.array_equal(full, (a + b) % q)


def test_unary_k1_selector_is_the_query_ciphertext():
    cfg = datagen.Config("unary", 4096, datagen.Q_N4096, 65537, 1, 8, 8, 1, 9)
    inst = build_instance(cfg)
    for j in range(cfg.n):
        assert np.array_equal(inst.orc.selector(inst.key, inst.query, inst.codewords[j]),
                              inst.query[inst.codewords[j][0]])
    ans = inst.orc.answer(inst.key, inst.query, inst.codewords, inst.payload)
    assert np.array_equal(inst.orc.decrypt(inst.sk, ans[0])[0], inst.payload[inst.target][0].astype(np.uint64))
