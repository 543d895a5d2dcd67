"""The deferred key switch of the root products against per-element relinearization and the oracle.

The answer (Eq. (1), Section 3.3.3) is linear in every selector, so the library may multiply each
element's root product into its payload before relinearizing and relinearize the digit sums once
per answer (pir_set_defer_relin; mode 2 forces it on these small databases, which the default mode
leaves per element).  The answers must be bit-identical to relinearizing every selector
and to the oracle's, for every shape the deferred path takes: k = 2 and k = 4 trees, one, two,
three and four plaintexts per element (row pairs for s = 1, single rows with payload pairs above),
ragged chunks, several queries per launch, the tiny, mid and wide prime sets on the fp64
transforms, and the keyword parameters (s = 1, 2, 3) and 52-55-bit primes on the integer transforms.
"""
import numpy as np
import pytest

import datagen
from conftest import cached_instance
from oracle.client import encrypt_query

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[gpu-deferred] {msg}", flush=True)


def _diff(got, want):
    bad = np.argwhere(got != want)
    return f"{len(bad)} residues differ, first at {tuple(bad[0]) if len(bad) else None}"


def _answers(cfg, ins, defer, queries, chunk, qg=8):
    from paper_2202_07569_amd import Context
    ctx = Context(cfg.N, cfg.primes, cfg.t, chunk_elems=chunk)
    ctx.defer_relin = 2 if defer else 0  # 2: deferred wherever allowed, whatever the database size
    ctx.set_schedule(chunk, min(qg, len(queries)), 0)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    outs = ctx.answer_batch([key] * len(queries), [db] * len(queries), [_dev(q) for q in queries])
    return [_host(o) for o in outs]


CASES = {
    "tiny-k2-s1": datagen.CONFIGS["tiny"].with_n(70),
    "mid-k4-s1": datagen.CONFIGS["mid"].with_n(90),
    "mid-k2-s2": datagen.Config("mid-k2-s2", 8192, datagen.Q_N8192, 65537, 2, 16, 50, 2, 71),
    "mid-k4-s3": datagen.Config("mid-k4-s3", 8192, datagen.Q_N8192, 65537, 4, 9, 40, 3, 72),
    # k = 3 (depth 2) needs the mid modulus for the answer to decrypt (tiny's 108 bits run out)
    "mid-k3-s4": datagen.Config("mid-k3-s4", 8192, datagen.Q_N8192, 65537, 3, 8, 30, 4, 73),
    # keyword parameters: N = 16384, eight 54/55-bit primes, integer transforms: s = 2 (single rows
    # with payload pairs), s = 1 (row pairs) and s = 3 (a payload pair, then a single payload row)
    "kw-k4-s2": datagen.Config("kw-k4-s2", 16384, datagen.Q_N16384, 65537, 4, 12, 24, 2, 75),
    "kw-k2-s1": datagen.Config("kw-k2-s1", 16384, datagen.Q_N16384, 65537, 2, 12, 20, 1, 76),
    "kw-k2-s3": datagen.Config("kw-k2-s3", 16384, datagen.Q_N16384, 65537, 2, 12, 18, 3, 77),
}


@pytest.mark.parametrize("name", list(CASES))
def test_deferred_equals_per_element_and_oracle(name):
    cfg = CASES[name]
    ins = cached_instance(cfg)
    other = (ins.target + 3) % cfg.n
    q2 = encrypt_query(ins.orc, ins.sk, [int(v) for v in ins.codewords[other]], cfg.m, cfg.seed, draw=7)
    queries = [ins.query, q2]
    _say(f"{name}: deferred and per-element answers, chunk 16, two queries")
    on = _answers(cfg, ins, True, queries, 16)
    off = _answers(cfg, ins, False, queries, 16)
    for a, b in zip(on, off):
        assert np.array_equal(a, b), _diff(a, b)
    want = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
    assert np.array_equal(on[0], want), _diff(on[0], want)
    for r in range(cfg.s):
        msg, _ = ins.orc.decrypt(ins.sk, on[1][r])
        assert np.array_equal(msg, ins.payload[other][r].astype(np.uint64)), r
    # one query per launch and a chunk that covers the database in one ragged piece
    _say(f"{name}: one query per launch, one chunk")
    one = _answers(cfg, ins, True, queries, 64 if cfg.n > 64 else cfg.n + 7, qg=1)
    for a, b in zip(one, off):
        assert np.array_equal(a, b), _diff(a, b)


@pytest.mark.parametrize("primes", [(0x1fffffffce001, 0x1fffffff96001, 0x1ffffffce001),
                                    (0x3ffffff84001, 0xfffffdc001, 0x7ffe6001),
                                    (0x7ffffffffb4001, 0x3ffffffffd6001, 0xffffffffca001)],
                         ids=["wide", "mixed", "int55"])
def test_deferred_with_other_primes(primes):
    """49/49/45-bit primes (digits close to the auxiliary primes, which may be smaller than a
    digit's prime: such digits are reduced before their transform), 46/40/31-bit primes, and
    55/54/52-bit primes (at or above 2^50: integer transforms at N = 4096, digit-sum primes below
    2^61)."""
    cfg = datagen.Config("defer-primes", 4096, primes, 65537, 2, 10, 33, 1, 74)
    ins = cached_instance(cfg)
    _say(f"primes {[p.bit_length() for p in primes]}: deferred against the oracle")
    on = _answers(cfg, ins, True, [ins.query], 8)
    off = _answers(cfg, ins, False, [ins.query], 8)
    assert np.array_equal(on[0], off[0]), _diff(on[0], off[0])
    want = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
    assert np.array_equal(on[0], want), _diff(on[0], want)


def test_mode_switch_rules():
    from paper_2202_07569_amd import Context, PirError
    cfg = datagen.CONFIGS["tiny"].with_n(8)
    ins = cached_instance(cfg)
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    assert ctx.defer_relin == 1  # default: where it pays
    ctx.defer_relin = 0
    assert ctx.defer_relin == 0
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    assert not db.root_deferred
    with pytest.raises(PirError):
        ctx.defer_relin = 2
    db.close()
    ctx.defer_relin = 2
    assert ctx.defer_relin == 2
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    assert db.root_deferred  # k = 2, and eight elements fit the digit-sum bound
    db.close()
    ctx.defer_relin = 1
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    assert not db.root_deferred  # too small to repay the per-answer work
    db.close()
    with pytest.raises(PirError):
        ctx.defer_relin = 3
