"""Parity with the oracle at prime sets other than the workloads', bit for bit.

* mixed: N = 4096, primes of 46, 40 and 31 bits.  Every prime is below 2^48, so the key switch runs
  its lazy transforms, and digits of a much larger prime (q_i > 2.5 q_j) take the branch that
  reduces them before their transform.
* wide: N = 4096, primes of 49, 49 and 45 bits.  Primes at or above 2^48 put the key switch on its
  non-lazy fp64 path (every intermediate reduced).
Each set runs a key switch and a multiplication on random residues and a PIR answer over 24
elements, which must also decrypt to the queried payload.  The primes are the largest primes
congruent to 1 mod 2N below 2^b.
"""
import dataclasses

import numpy as np
import pytest

import datagen
from conftest import cached_instance
from oracle.core import Oracle

pytestmark = pytest.mark.gpu
PRIME_SETS = {
    "mixed": (0x3ffffff84001, 0xfffffdc001, 0x7ffe6001),
    "wide": (0x1fffffffce001, 0x1fffffff96001, 0x1ffffffce001),
}
_ctx = {}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _cfg(name):
    return dataclasses.replace(datagen.CONFIGS["tiny"], name=f"tiny-{name}", primes=PRIME_SETS[name])


def _context(cfg):
    from paper_2202_07569_amd import Context
    if cfg.name not in _ctx:
        _ctx[cfg.name] = Context(cfg.N, cfg.primes, cfg.t)
    return _ctx[cfg.name]


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name", list(PRIME_SETS))
def test_relin_and_mult_match_oracle(name):
    cfg = _cfg(name)
    orc, ctx = Oracle(cfg.N, cfg.primes), _context(cfg)
    sk = orc.keygen(datagen.words(cfg.seed, datagen.S_SECRET, cfg.N))
    rlk = orc.relin_keygen(sk, datagen.words(cfg.seed, datagen.S_RLK, orc.rnd_words_rlk()))
    c3 = datagen.uniform_residues(cfg.primes, (3,), cfg.N, seed=211)
    _say(f"relin {name}")
    assert np.array_equal(_host(ctx.relin(ctx.load_key(rlk), _dev(c3))), orc.relin(orc.load_key(rlk), c3))
    a, b = datagen.uniform_residues(cfg.primes, (2, 2), cfg.N, seed=213)
    _say(f"mult {name}")
    assert np.array_equal(_host(ctx.mult(_dev(a), _dev(b))), orc.mult(a, b))


@pytest.mark.parametrize("name", list(PRIME_SETS))
def test_answer_matches_oracle_and_decrypts(name):
    cfg = _cfg(name).with_n(24)
    ins = cached_instance(cfg)
    ctx = _context(cfg)
    _say(f"answer {name} n=24")
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    got = _host(ctx.answer(ctx.load_key(ins.rlk), db, _dev(ins.query)))
    assert np.array_equal(got, ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload))
    msg, _ = ins.orc.decrypt(ins.sk, got[0])
    assert np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64))
