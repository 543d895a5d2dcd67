"""Client side of constant-weight PIR for tests (test infrastructure only).

Builds one PIR instance from a workload configuration: secret key, relinearization key, the
database's codewords and payload (Setup, Section 3.3.1) and an encrypted query with compression
factor c = 0, i.e. one ciphertext per codeword bit, each encrypting the constant polynomial of
that bit (Query, Algorithm 4 with c = 0).  All randomness comes from the seeded generators.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

import datagen
from .core import Oracle
from .mapping import codeword_bits, lossy_map, perfect_map


@dataclass
class Instance:
    cfg: object
    orc: Oracle
    sk: np.ndarray
    rlk: np.ndarray
    codewords: np.ndarray      # uint32 [n][k], ascending one positions
    payload: np.ndarray        # uint16 [n][s][N]
    target: int                # element index queried (-1: absent keyword)
    positions: list            # the queried codeword's one positions
    query: np.ndarray          # uint64 [m][2][L][N]
    keywords: np.ndarray | None = None

    _key: object = None

    @property
    def key(self):
        if self._key is None:
            self._key = self.orc.load_key(self.rlk)
        return self._key


def encrypt_query(orc: Oracle, sk: np.ndarray, positions, m: int, seed: int, draw: int = 0) -> np.ndarray:
    bits = codeword_bits(positions, m)
    per = orc.rnd_words_encrypt()
    out = np.empty((m, 2, orc.L, orc.N), dtype=np.uint64)
    msg = np.zeros(orc.N, dtype=np.uint64)
    for i, b in enumerate(bits):
        msg[0] = b
        rnd = datagen.words(seed, datagen.S_QUERY, per, offset=(draw * m + i) * per)
        out[i] = orc.encrypt(sk, msg, rnd)
    return out


def keyword_codewords(cfg, n: int):
    """Distinct uniform 64-bit keywords whose lossy-mapped codewords do not collide; a keyword
    that collides with an earlier one is replaced by the next draw of the keyword stream."""
    seed = datagen.hash_seed(cfg)
    kws, cws, seen = [], [], set()
    offset = 0
    while len(kws) < n:
        batch = datagen.keywords(cfg, n - len(kws) + 16, offset=offset)
        offset += len(batch)
        for x in batch:
            x = int(x)
            cw = tuple(lossy_map(x, cfg.m, cfg.k, seed))
            if cw in seen:
                continue
            seen.add(cw)
            kws.append(x)
            cws.append(cw)
            if len(kws) == n:
                break
    return np.array(kws, dtype=np.uint64), np.array(cws, dtype=np.uint32), seen, offset


def build_instance(cfg, n: int | None = None, absent: bool = False, orc: Oracle | None = None) -> Instance:
    n = cfg.n if n is None else n
    orc = orc or Oracle(cfg.N, cfg.primes, cfg.t)
    sk = orc.keygen(datagen.words(cfg.seed, datagen.S_SECRET, cfg.N))
    rlk = orc.relin_keygen(sk, datagen.words(cfg.seed, datagen.S_RLK, orc.rnd_words_rlk()))
    kws = None
    if cfg.keyword:
        kws, codewords, seen, offset = keyword_codewords(cfg, n)
    else:
        ids = datagen.identifier_permutation(cfg, n)
        codewords = np.array([perfect_map(int(x), cfg.m, cfg.k) for x in ids], dtype=np.uint32)
    payload = datagen.payload(cfg, n)
    if absent:
        if not cfg.keyword:
            raise ValueError("absent queries are defined for keyword databases")
        seed = datagen.hash_seed(cfg)
        while True:
            x = int(datagen.keywords(cfg, 1, offset=offset)[0])
            offset += 1
            pos = lossy_map(x, cfg.m, cfg.k, seed)
            if tuple(pos) not in seen:
                break
        target, draw = -1, 1
    else:
        target = datagen.target_index(cfg, n)
        pos = [int(v) for v in codewords[target]]
        draw = 0
    query = encrypt_query(orc, sk, pos, cfg.m, cfg.seed, draw=draw)
    return Instance(cfg, orc, sk, rlk, codewords, payload, target, list(pos), query, kws)
