"""Whole answers at the keyword and large parameter sets, element by element against the oracle.

The full keyword (65,536 elements) and large (262,144 elements) databases are beyond what the
oracle answers in seconds, so their parameters are exercised here on small databases that still
take every branch the full size takes (Section 3.3.3, Algorithm 6 and Eq. (1)):

* keyword parameters: N = 16384, eight 54/55-bit primes (the integer transforms and the staged key
  switch), k = 4 (depth 2), m = 569, s = 2 (two plaintexts per element, two accumulators), lossy-map
  codewords, a present and an absent keyword; 50 elements in chunks of 16 (a ragged last chunk of
  2), with inner tree nodes shared by the whole database and, under a small memo budget, within
  each chunk only (the way the full keyword database runs);
* large parameters: N = 8192, k = 2, m = 725, 64 elements, under the benchmark's cached schedules
  for one query and for the batch of 32 (one ragged chunk) and in chunks of 24.
"""
import numpy as np
import pytest

import datagen
from conftest import cached_instance

pytestmark = pytest.mark.gpu

KW50 = datagen.CONFIGS["keyword"].with_n(50)
LARGE64 = datagen.CONFIGS["large"].with_n(64)
_want = {}


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[gpu-params] {msg}", flush=True)


def _oracle(cfg, ins):
    k = (cfg.name, ins.target)
    if k not in _want:
        _want[k] = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
    return _want[k]


def _diff(got, want):
    bad = np.argwhere(got != want)
    return f"{len(bad)} residues differ, first at {tuple(bad[0]) if len(bad) else None}"


def _answer(cfg, ins, schedule=None, **ctxkw):
    from paper_2202_07569_amd import Context
    ctx = Context(cfg.N, cfg.primes, cfg.t, **ctxkw)
    if schedule is not None:
        ctx.set_schedule(schedule["chunk_elems"], schedule["query_group"], schedule["relin_group"])
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    return _host(ctx.answer(key, db, _dev(ins.query))), db


@pytest.mark.parametrize("absent", [False, True])
@pytest.mark.parametrize("memo", ["database", "chunk"])
def test_keyword_parameters_answer(memo, absent):
    cfg = KW50
    ins = cached_instance(cfg, absent=absent)
    kw = dict(chunk_elems=16) if memo == "database" else dict(chunk_elems=16, memo_bytes=1 << 20)
    _say(f"keyword parameters n={cfg.n} chunk=16 memo={memo} absent={absent}")
    got, db = _answer(cfg, ins, **kw)
    if memo == "database":
        assert 0 < db.pair_count <= 2 * cfg.n
    want = _oracle(cfg, ins)
    assert np.array_equal(got, want), _diff(got, want)
    for r in range(cfg.s):
        msg, _ = ins.orc.decrypt(ins.sk, got[r])
        expect = np.zeros(cfg.N, np.uint64) if absent else ins.payload[ins.target][r].astype(np.uint64)
        assert np.array_equal(msg, expect), r


def test_keyword_parameters_batch():
    """Two queries (present and absent keyword) in one call under the benchmark's cached batch-of-2
    schedule equal the oracle's answers."""
    from paper_2202_07569_amd import Context
    from paper_2202_07569_amd.binding import lookup_schedule
    cfg = KW50
    a, b = cached_instance(cfg), cached_instance(cfg, absent=True)
    ctx = Context(cfg.N, cfg.primes, cfg.t, chunk_elems=16)
    sched = lookup_schedule(cfg.N, cfg.primes, 2, cfg.k, cfg.s)
    if sched is not None:
        ctx.set_schedule(16, sched["query_group"], sched["relin_group"])
    key = ctx.load_key(a.rlk)
    db = ctx.encode_db(a.codewords, a.payload, cfg.m)
    _say(f"keyword parameters batch of 2 under {ctx.schedule()}")
    outs = ctx.answer_batch([key, key], [db, db], [_dev(a.query), _dev(b.query)])
    for ins, out in zip((a, b), outs):
        got, want = _host(out), _oracle(cfg, ins)
        assert np.array_equal(got, want), _diff(got, want)


@pytest.mark.parametrize("batch", [1, 32, None])
def test_large_parameters_answer(batch):
    from paper_2202_07569_amd.binding import lookup_schedule
    cfg = LARGE64
    ins = cached_instance(cfg)
    if batch is None:
        sched = dict(chunk_elems=24, query_group=1, relin_group=0)
    else:
        sched = lookup_schedule(cfg.N, cfg.primes, batch, cfg.k, cfg.s)
        assert sched is not None
        sched = dict(sched, query_group=1)
    _say(f"large parameters n={cfg.n} schedule={sched}")
    got, _ = _answer(cfg, ins, schedule=sched)
    want = _oracle(cfg, ins)
    assert np.array_equal(got, want), _diff(got, want)
    msg, _ = ins.orc.decrypt(ins.sk, got[0])
    assert np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64))
