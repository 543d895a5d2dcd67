"""Captured answers (HIP graphs): every replay answers the query the buffer holds at that time.

A graph is captured once, then replayed after new query ciphertexts are written into the captured
buffer, with the program's own eager work (an eager answer of the same query) between replays.
Each replay is compared with the eager answer, and the first with the oracle and by decryption.
"""
import numpy as np
import pytest

import datagen
from conftest import cached_instance

pytestmark = pytest.mark.gpu

TINY64 = datagen.CONFIGS["tiny"].with_n(64, m=12)
KW_SMALL = datagen.Config("kw-small", 4096, datagen.Q_N4096, 65537, 2, 24, 40, 2, 7, keyword=True)


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("defer", [1, 2], ids=["default", "deferred"])
def test_graph_replays_answer_new_queries(defer):
    """Mode 2 puts the root products' deferred key switch (accumulators cleared by a fill kernel,
    digit sums relinearized once per answer) under capture."""
    import torch
    from oracle.client import encrypt_query
    from paper_2202_07569_amd import Context
    cfg = TINY64
    ins = cached_instance(cfg)
    ctx = Context(cfg.N, cfg.primes, cfg.t, chunk_elems=24)
    ctx.defer_relin = defer
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    qbuf = torch.from_numpy(ins.query).cuda()
    _say(f"graph capture tiny n=64, deferral mode {defer}")
    g = ctx.capture([key], [db], [qbuf])
    want = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
    assert np.array_equal(_host(g.outs[0]), want)  # the capture's own eager run
    for r, target in enumerate([5, 17, 63, 5]):
        q = encrypt_query(ins.orc, ins.sk, [int(v) for v in ins.codewords[target]], cfg.m, cfg.seed, draw=10 + r)
        qbuf.copy_(torch.from_numpy(q).cuda())
        _say(f"graph replay {r} target {target}")
        got = _host(g.launch()[0]).copy()
        eager = _host(ctx.answer(key, db, torch.from_numpy(q).cuda()))
        assert np.array_equal(got, eager), r
        msg, _ = ins.orc.decrypt(ins.sk, got[0])
        assert np.array_equal(msg, ins.payload[target][0].astype(np.uint64)), r
        if r == 0:
            assert np.array_equal(got, ins.orc.answer(ins.key, q, ins.codewords, ins.payload))
    g.close()


def test_graph_of_a_batch_over_two_databases():
    import torch
    from paper_2202_07569_amd import Context
    a, b = cached_instance(TINY64), cached_instance(KW_SMALL)
    ctx = Context(TINY64.N, TINY64.primes, TINY64.t, chunk_elems=16)
    ka, kb = ctx.load_key(a.rlk), ctx.load_key(b.rlk)
    da, db = ctx.encode_db(a.codewords, a.payload, TINY64.m), ctx.encode_db(b.codewords, b.payload, KW_SMALL.m)
    qs = [torch.from_numpy(x).cuda() for x in (a.query, b.query, a.query)]
    _say("graph capture batch of 3 on two databases")
    g = ctx.capture([ka, kb, ka], [da, db, da], qs)
    for rep in range(3):
        outs = [_host(o).copy() for o in g.launch()]
        singles = [_host(ctx.answer(k, d, q)) for k, d, q in zip([ka, kb, ka], [da, db, da], qs)]
        for o, s in zip(outs, singles):
            assert np.array_equal(o, s), rep
    g.close()


def test_schedule_is_fixed_while_a_graph_exists():
    import torch
    from paper_2202_07569_amd import Context, PirError
    cfg = TINY64
    ins = cached_instance(cfg)
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    g = ctx.capture([key], [db], [torch.from_numpy(ins.query).cuda()])
    db.close()
    with pytest.raises(PirError):
        ctx.set_schedule(32, 1, 0)
    g.close()
    ctx.set_schedule(32, 1, 0)
