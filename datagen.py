"""Seeded synthetic inputs for constant-weight PIR.

This module is the single source of random inputs for both the CPU oracle tests and the HIP path.
It holds random-number generation and workload recipes only: no FV arithmetic and no codeword
mapping (those belong to the two implementations being compared).

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014).  Output number i (i = 1, 2, ...) of a stream with starting state z0 is
mix(z0 + i * 0x9E3779B97F4A7C15 mod 2^64), which makes every stream counter-based and lets numpy
produce it in one vectorised pass.  A stream is keyed by (config seed, stream id):
z0 = mix(mix(seed) XOR stream_id).

Stream ids: 1 secret key, 2 relinearization key, 3 query encryption, 4 payload, 5 identifier
permutation, 6 target, 7 keywords, 8 lossy-map hash seed, 9 arrivals, 10 database choice,
11 synthetic ciphertexts, 12 Galois keys, 13 packed query encryptions, 14 seeded query errors.

Workloads follow the paper's evaluation: random synthetic databases of n elements, each element s
FV plaintexts of N coefficients (Section 5.1 and the keyword-PIR application in Section 5.3); the
constant-weight code length m is the smallest with C(m, k) >= n (Section 3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

S_SECRET, S_RLK, S_QUERY, S_PAYLOAD, S_PERM, S_TARGET, S_KEYWORDS, S_HASH, S_ARRIVALS, \
    S_DBCHOICE, S_SYNTH, S_GALOIS, S_PACKED, S_SEEDED = range(1, 15)


def mix64(z: int) -> int:
    """SplitMix64 output function on one Python integer."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return z


def stream_state(seed: int, stream_id: int) -> int:
    return mix64(mix64(seed) ^ stream_id)


def words(seed: int, stream_id: int, count: int, offset: int = 0) -> np.ndarray:
    """`count` consecutive 64-bit outputs of stream (seed, stream_id), starting after `offset`."""
    z0 = np.uint64(stream_state(seed, stream_id))
    idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64_np(z0 + idx * np.uint64(GAMMA))


# --------------------------------------------------------------------------------------------
# Workload configurations.  The ciphertext primes are the largest primes congruent to 1 mod 2N
# below 2^b, with the bit splits stated per configuration; every listed prime is a ciphertext
# prime (no key-switching-only prime).  t = 65537.
# --------------------------------------------------------------------------------------------

Q_N4096 = (0xffffee001, 0xffffc4001, 0xffffbe001)                       # 3 x 36 bits = 108
Q_N8192 = (0x7fffffd8001, 0x7fffffc8001, 0xfffffffc001, 0xffffff6c001,
           0xfffffebc001)                                                 # 43,43,44,44,44 = 218
Q_N16384 = (0x3fffffffef8001, 0x3fffffffeb8001, 0x7fffffffe90001, 0x7fffffffd58001,
            0x7fffffffbf0001, 0x7fffffffbd0001, 0x7fffffffba0001, 0x7fffffffb58001)  # 438


def code_length(n: int, k: int) -> int:
    """Smallest m with C(m, k) >= n (Section 3, constant-weight code size)."""
    m = k
    while math.comb(m, k) < n:
        m += 1
    return m


@dataclass(frozen=True)
class Config:
    name: str
    N: int
    primes: tuple
    t: int
    k: int
    m: int
    n: int
    s: int
    seed: int
    keyword: bool = False

    @property
    def L(self) -> int:
        return len(self.primes)

    def with_n(self, n: int, m: int | None = None) -> "Config":
        """Same parameters on a smaller database (for oracle-sized parity cases)."""
        return Config(self.name + f"-n{n}", self.N, self.primes, self.t, self.k,
                      self.m if m is None else m, n, self.s, self.seed, self.keyword)


CONFIGS = {
    "tiny": Config("tiny", 4096, Q_N4096, 65537, 2, 24, 256, 1, 1),
    "mid": Config("mid", 8192, Q_N8192, 65537, 4, 27, 16384, 1, 2),
    "keyword": Config("keyword", 16384, Q_N16384, 65537, 4, code_length(1 << 32, 4), 65536, 2, 3,
                      keyword=True),
    "large": Config("large", 8192, Q_N8192, 65537, 2, 725, 262144, 1, 5),
}

# Batched serving mix: (n, s, k) per resident database; m from the code-length rule.
BATCHED_DBS = [(4096, 1, 2), (16384, 1, 4), (32768, 2, 2), (65536, 4, 4)]


def batched_configs(seed: int = 4) -> list:
    return [Config(f"batched-db{i}", 8192, Q_N8192, 65537, k, code_length(n, k), n, s, seed * 16 + i)
            for i, (n, s, k) in enumerate(BATCHED_DBS)]


# --------------------------------------------------------------------------------------------
# Recipes
# --------------------------------------------------------------------------------------------

def payload(cfg: Config, n: int | None = None, offset_elems: int = 0) -> np.ndarray:
    """uint16 payload [n][s][N], uniform over [0, 2^16) (below t = 65537)."""
    n = cfg.n if n is None else n
    per_elem = cfg.s * cfg.N
    cnt = n * per_elem
    w = words(cfg.seed, S_PAYLOAD, (cnt + 3) // 4, offset=offset_elems * per_elem // 4)
    return w.view(np.uint16)[:cnt].reshape(n, cfg.s, cfg.N).copy()


def identifier_permutation(cfg: Config, n: int | None = None) -> np.ndarray:
    """Identifiers pi(0..n-1): the first n entries of a seeded Fisher-Yates shuffle of [C(m,k)].

    Element j of the database carries identifier pi(j); its codeword is the perfect mapping of it.
    """
    n = cfg.n if n is None else n
    size = math.comb(cfg.m, cfg.k)
    if n > size:
        raise ValueError("database larger than the code")
    w = words(cfg.seed, S_PERM, n)
    # Sparse inside-out shuffle: only the touched positions are materialised.
    pos: dict = {}
    out = np.empty(n, dtype=np.int64)
    for i in range(n):
        j = i + int(w[i]) % (size - i)
        vi, vj = pos.get(i, i), pos.get(j, j)
        pos[i], pos[j] = vj, vi
        out[i] = vj
    return out


def target_index(cfg: Config, n: int | None = None, draw: int = 0) -> int:
    n = cfg.n if n is None else n
    return int(words(cfg.seed, S_TARGET, 1, offset=draw)[0]) % n


def keywords(cfg: Config, count: int, offset: int = 0) -> np.ndarray:
    """Uniform 64-bit keywords (duplicates are removed by the caller's redraw policy)."""
    return words(cfg.seed, S_KEYWORDS, count, offset=offset)


def hash_seed(cfg: Config) -> int:
    return int(words(cfg.seed, S_HASH, 1)[0])


def uniform_residues(primes, shape_prefix, N: int, seed: int, stream_id: int = S_SYNTH) -> np.ndarray:
    """Random residues [*shape_prefix, L, N], limb i uniform below primes[i] (bias < 2^-9).

    Used where the timing of the server path is measured on statistically ciphertext-like inputs
    that nobody decrypts.
    """
    L = len(primes)
    shape = tuple(shape_prefix) + (L, N)
    w = words(seed, stream_id, int(np.prod(shape))).reshape(shape)
    q = np.array(primes, dtype=np.uint64).reshape((1,) * len(shape_prefix) + (L, 1))
    return w % q


def poisson_arrivals(seed: int, count: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process: exponential gaps -ln(u)/rate, u in (0, 1]."""
    w = words(seed, S_ARRIVALS, count)
    u = ((w >> np.uint64(11)).astype(np.float64) + 1.0) / float(1 << 53)
    return np.cumsum(-np.log(u) / rate_per_s)


def uniform_choice(seed: int, stream_id: int, count: int, bound: int) -> np.ndarray:
    return (words(seed, stream_id, count) % np.uint64(bound)).astype(np.int64)
