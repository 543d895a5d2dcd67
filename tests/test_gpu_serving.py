"""Serving with continuous batching on the HIP path (pir_serve_*).

A mixed trace of real encrypted queries from three clients (three secret keys) on three resident
databases, submitted while earlier queries are mid-scan and with fewer slots than queries: every
answer must equal the same query answered alone (pir_answer) bit for bit and decrypt to the
queried payload; one is also compared with the oracle's answer element for element.
"""
import numpy as np
import pytest

import datagen
from oracle.client import build_instance, encrypt_query

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
    print(f"[gpu-serve] {msg}", flush=True)


@pytest.fixture(scope="module")
def mix():
    from paper_2202_07569_amd import Context
    cfgs = datagen.batched_configs()
    # three databases of several 32-element chunks each (ragged last chunks), k = 2, 4, 2; s = 1, 1, 2
    insts = [build_instance(cfgs[0].with_n(200)), build_instance(cfgs[1].with_n(120)),
             build_instance(cfgs[2].with_n(90))]
    ctx = Context(8192, datagen.Q_N8192, chunk_elems=32)
    keys = [ctx.load_key(i.rlk) for i in insts]
    dbs = [ctx.encode_db(i.codewords, i.payload, i.cfg.m) for i in insts]
    return insts, ctx, keys, dbs


def _query(insts, ki, di, target, draw):
    ci, db = insts[ki], insts[di]
    pos = [int(v) for v in db.codewords[target]]
    return encrypt_query(ci.orc, ci.sk, pos, db.cfg.m, ci.cfg.seed, draw=draw)


@pytest.mark.parametrize("policy", [0, 1, 2], ids=["round_robin", "oldest_first", "size_aged"])
def test_serving_mix_equals_single_answers(mix, policy):
    from paper_2202_07569_amd import PirError, Server
    insts, ctx, keys, dbs = mix
    # (client key, database, element)
    plan = [(0, 0, 17), (1, 1, 119), (2, 0, 199), (0, 2, 45), (1, 0, 0), (2, 2, 89), (0, 1, 64), (1, 2, 3)]
    qs = [_query(insts, ki, di, j, draw=10 + n) for n, (ki, di, j) in enumerate(plan)]
    srv = Server(ctx, max_slots=4, policy=policy, aging_ns_per_element=1e6 if policy == 2 else 0.0)
    tickets = []
    _say("submit 2, step 2")
    for n in range(2):
        tickets.append(srv.submit(keys[plan[n][0]], dbs[plan[n][1]], _dev(qs[n])))
    srv.step()
    srv.step()
    _say("submit 2 mid-scan, step 1")
    for n in range(2, 4):
        tickets.append(srv.submit(keys[plan[n][0]], dbs[plan[n][1]], _dev(qs[n])))
    srv.step()
    _say("submit 4 more than the free slots, drain")
    for n in range(4, len(plan)):
        tickets.append(srv.submit(keys[plan[n][0]], dbs[plan[n][1]], _dev(qs[n])))
    st = srv.stats()
    assert st["active"] <= 4 and st["pending"] >= 1
    srv.drain(tickets)
    outs = [_host(srv.result(t)) for t in tickets]
    st = srv.stats()
    assert st["completed"] == len(plan) and st["admitted"] == len(plan) and st["active"] == 0
    with pytest.raises(PirError):
        srv.poll(tickets[0])  # released
    srv.close()
    for n, (ki, di, j) in enumerate(plan):
        _say(f"query {n}: key {ki} db {di} element {j}")
        alone = _host(ctx.answer(keys[ki], dbs[di], _dev(qs[n])))
        assert np.array_equal(outs[n], alone), n
        for r in range(insts[di].cfg.s):
            msg, _ = insts[ki].orc.decrypt(insts[ki].sk, outs[n][r])
            assert np.array_equal(msg, insts[di].payload[j][r].astype(np.uint64)), (n, r)
    if policy == 0:
        _say("oracle answer of query 0")
        i0 = insts[0]
        want = i0.orc.answer(i0.key, qs[0], i0.codewords, i0.payload)
        assert np.array_equal(outs[0], want)


def test_serving_rounds_are_chunks(mix):
    """One query on a database of c chunks completes after exactly c rounds."""
    from paper_2202_07569_amd import Server
    insts, ctx, keys, dbs = mix
    q = _query(insts, 0, 2, 5, draw=30)
    srv = Server(ctx, max_slots=2)
    t = srv.submit(keys[0], dbs[2], _dev(q))
    steps = 1
    while srv.step() > 0:  # the step that runs the last chunk leaves the server idle
        steps += 1
        assert steps < 10
    assert steps == (90 + 31) // 32
    srv.drain([t])
    assert np.array_equal(_host(srv.result(t)), _host(ctx.answer(keys[0], dbs[2], _dev(q))))
    srv.close()


def test_batch_wider_than_one_launch(mix):
    """More queries on one database than one selector launch holds: equal to the single answers."""
    insts, ctx, keys, dbs = mix
    B = 11
    qs = [_query(insts, b % 3, 0, (37 * b) % 200, draw=40 + b) for b in range(B)]
    outs = ctx.answer_batch([keys[b % 3] for b in range(B)], [dbs[0]] * B, [_dev(q) for q in qs])
    for b in range(B):
        assert np.array_equal(_host(outs[b]), _host(ctx.answer(keys[b % 3], dbs[0], _dev(qs[b])))), b


def test_oldest_first_runs_one_database_at_a_time(mix):
    """Oldest first: the newer query's database does not advance until the older query is done, so
    it needs all of its own chunks afterwards; both answers equal the single answers."""
    from paper_2202_07569_amd import Server
    insts, ctx, keys, dbs = mix
    qa, qb = _query(insts, 0, 2, 7, draw=50), _query(insts, 1, 0, 33, draw=51)
    srv = Server(ctx, max_slots=2, policy=Server.OLDEST_FIRST)
    ta = srv.submit(keys[0], dbs[2], _dev(qa))  # 90 elements: 3 chunks of 32
    tb = srv.submit(keys[1], dbs[0], _dev(qb))  # 200 elements: 7 chunks
    import torch
    for _ in range(3):
        srv.step()
    torch.cuda.synchronize()
    assert srv.poll(ta)  # done after its own 3 rounds
    steps = 1
    while srv.step() > 0:  # b has not advanced: it needs all 7 of its rounds now
        steps += 1
        assert steps <= 8
    assert steps == 7
    srv.drain([tb])
    assert np.array_equal(_host(srv.result(ta)), _host(ctx.answer(keys[0], dbs[2], _dev(qa))))
    assert np.array_equal(_host(srv.result(tb)), _host(ctx.answer(keys[1], dbs[0], _dev(qb))))
    srv.close()


@pytest.mark.parametrize("aging", [0.0, 1e9])
def test_size_aged_order(mix, aging):
    """Size aged: one query per round along its own chunk cursor.  With no aging the first query
    submitted runs first; with a large aging the query on the smaller database (90 elements, 3
    chunks) overtakes the one on the larger (200 elements, 7 chunks).  Answers equal the singles."""
    import torch
    from paper_2202_07569_amd import Server
    from paper_2202_07569_amd.binding import PIR_E_BUSY, lib
    insts, ctx, keys, dbs = mix
    qa, qb = _query(insts, 0, 0, 33, draw=60), _query(insts, 1, 2, 7, draw=61)
    srv = Server(ctx, max_slots=2, policy=Server.SIZE_AGED, aging_ns_per_element=aging)
    ta = srv.submit(keys[0], dbs[0], _dev(qa))  # 200 elements: 7 chunks of 32
    tb = srv.submit(keys[1], dbs[2], _dev(qb))  # 90 elements: 3 chunks
    assert lib().pir_serve_set_policy(srv._h, Server.ROUND_ROBIN) == PIR_E_BUSY
    first, n_first = (tb, 3) if aging else (ta, 7)
    second, n_second = (ta, 7) if aging else (tb, 3)
    _say(f"size aged, aging {aging}: {n_first} rounds for the first query")
    for _ in range(n_first):
        srv.step()
    torch.cuda.synchronize()
    assert srv.poll(first) and not srv.poll(second)
    steps = 0
    while srv.step() > 0:  # the other query has not advanced: all of its rounds remain
        steps += 1
        assert steps <= n_second
    assert steps + 1 == n_second
    srv.drain([second])
    assert np.array_equal(_host(srv.result(ta)), _host(ctx.answer(keys[0], dbs[0], _dev(qa))))
    assert np.array_equal(_host(srv.result(tb)), _host(ctx.answer(keys[1], dbs[2], _dev(qb))))
    srv.close()
