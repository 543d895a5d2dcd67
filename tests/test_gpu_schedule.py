"""Launch schedules and the autotuner: any schedule gives the same bits.

The schedule only cuts the work into launches (chunk size, queries per selector launch, order of
the key-switching workgroups) and groups the transform stages into passes (shape variants that
leave the same transformed layout).  These tests run the mid parameters (N = 8192, five primes,
k = 4) on a small database under several schedules and every shape, including the schedule the
autotuner picks, and compare every answer with the oracle's; the keyword parameters
(N = 16384, integer path) under both of their shapes.
"""
import numpy as np
import pytest

import datagen
from conftest import cached_instance

pytestmark = pytest.mark.gpu

MID72 = datagen.CONFIGS["mid"].with_n(72)
_want = {}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _oracle_answer(ins):
    k = id(ins)
    if k not in _want:
        _want[k] = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
    return _want[k]


def _answers(ctx, ins, nq):
    import torch
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, MID72.m)
    q = torch.from_numpy(ins.query).cuda()
    outs = ctx.answer_batch([key] * nq, [db] * nq, [q] * nq)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in outs]
    db.close()
    key.close()
    return res


@pytest.mark.parametrize("chunk,qb,rg", [(16, 1, 0), (40, 3, 8), (72, 2, 5), (7, 3, 1)])
def test_schedules_give_identical_answers(chunk, qb, rg):
    from paper_2202_07569_amd import Context
    cfg = MID72
    ins = cached_instance(cfg)
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    ctx.set_schedule(chunk, qb, rg)
    assert ctx.schedule()["chunk_elems"] == chunk and ctx.schedule()["query_group"] == qb
    _say(f"schedule chunk={chunk} query_group={qb} relin_group={rg}")
    want = _oracle_answer(ins)
    for got in _answers(ctx, ins, 3):
        assert np.array_equal(got, want)


@pytest.mark.parametrize("defer", [0, 2])
def test_every_ntt_shape_gives_identical_answers(defer):
    from paper_2202_07569_amd import Context
    cfg = MID72
    ins = cached_instance(cfg)
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    shapes = ctx.ntt_shapes()
    assert shapes == [[3, 3, 3, 2, 2], [3, 3, 2, 3, 2], [3, 2, 3, 3, 2]]
    want = _oracle_answer(ins)
    for v in range(len(shapes)):
        c = Context(cfg.N, cfg.primes, cfg.t)
        c.defer_relin = defer
        c.set_schedule(24, 2, 0, v)
        assert c.schedule()["ntt_shape"] == v
        _say(f"mid shape {v} {shapes[v]} defer mode {defer}")
        for got in _answers(c, ins, 2):
            assert np.array_equal(got, want)
    from paper_2202_07569_amd import PirError
    with pytest.raises(PirError):
        ctx.set_schedule(24, 2, 0, len(shapes))
    tiny = datagen.CONFIGS["tiny"]
    t = Context(tiny.N, tiny.primes, tiny.t)
    assert t.ntt_shapes() == [[3, 3, 3, 3]]  # one shape at N = 4096
    with pytest.raises(PirError):
        t.set_schedule(24, 2, 0, 1)


def test_keyword_parameters_under_both_shapes():
    """N = 16384, eight 54/55-bit primes (integer transforms, staged key switch), s = 2."""
    import torch
    from paper_2202_07569_amd import Context
    kw = datagen.CONFIGS["keyword"]
    cfg = datagen.Config("kw-shapes", kw.N, kw.primes, kw.t, 4, 12, 20, 2, 91)
    ins = cached_instance(cfg)
    want = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    assert ctx.ntt_shapes() == [[4, 4, 3, 3], [4, 3, 4, 3]]
    for v in range(2):
        c = Context(cfg.N, cfg.primes, cfg.t)
        c.set_schedule(8, 1, 0, v)
        _say(f"keyword parameters, shape {v}")
        key = c.load_key(ins.rlk)
        db = c.encode_db(ins.codewords, ins.payload, cfg.m)
        out = c.answer(key, db, torch.from_numpy(ins.query).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want)
        db.close()
        key.close()


def test_autotune_picks_a_measured_schedule_and_stays_exact():
    from paper_2202_07569_amd import Context
    cfg = MID72
    ins = cached_instance(cfg)
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    _say("autotune mid batch=2 k=4")
    res = ctx.autotune(batch=2, k=4, s=1)
    best, cands = res["best"], res["candidates"]
    assert cands and best in cands
    assert best["ns_per_elem"] == min(c["ns_per_elem"] for c in cands) > 0
    assert ctx.schedule()["chunk_elems"] == best["chunk_elems"]
    assert ctx.schedule()["query_group"] == best["query_group"]
    assert ctx.schedule()["relin_group"] == best["relin_group"]
    assert ctx.schedule()["ntt_shape"] == best["ntt_shape"]
    assert {c["ntt_shape"] for c in cands} == {0, 1, 2}  # the tuner tried every shape
    want = _oracle_answer(ins)
    for got in _answers(ctx, ins, 2):
        assert np.array_equal(got, want)


def test_schedule_is_fixed_once_a_database_exists():
    from paper_2202_07569_amd import Context, PirError
    cfg = datagen.CONFIGS["tiny"]
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    db = ctx.encode_db(np.array([[0, 1]], np.uint32), np.zeros((1, 1, cfg.N), np.uint16), cfg.m)
    with pytest.raises(PirError):
        ctx.set_schedule(64, 2, 0)
    with pytest.raises(PirError):
        ctx.autotune(batch=1, k=2, s=1)
    db.close()
    ctx.set_schedule(64, 2, 0)  # allowed again once the database is gone
    with pytest.raises(PirError):
        ctx.set_schedule(64, 9, 0)  # more queries per launch than a launch holds
