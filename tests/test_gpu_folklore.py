"""Parity of product trees beyond k = 4 and of folklore PIR with the oracle, bit for bit.

The engine memoises the inner nodes of every element's product tree depth by depth; these tests
run depth-3 trees (constant-weight k = 5 and k = 8, folklore with l = 6) at the mid parameters,
with the nodes shared by the whole database and shared per chunk, and compare the answers with
the oracle's per-element trees.  Folklore leaves (1 - x_i, x_i) are formed on the GPU.
"""
import math

import numpy as np
import pytest

import datagen
from oracle.client import encrypt_query
from oracle.core import Oracle
from oracle.folklore import folklore_codewords, folklore_leaves, folklore_query, index_bits
from oracle.mapping import perfect_map

pytestmark = pytest.mark.gpu
MID = datagen.CONFIGS["mid"]
_cache = {}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _keys():
    if "keys" not in _cache:
        orc = Oracle(MID.N, MID.primes, MID.t)
        sk = orc.keygen(datagen.words(61, datagen.S_SECRET, MID.N))
        rlk = orc.relin_keygen(sk, datagen.words(61, datagen.S_RLK, orc.rnd_words_rlk()))
        _cache["keys"] = (orc, sk, rlk, orc.load_key(rlk))
    return _cache["keys"]


def _gpu_answer(query, codewords, payload, m, **ctxkw):
    import torch
    from paper_2202_07569_amd import Context
    orc, sk, rlk, _ = _keys()
    ctx = Context(MID.N, MID.primes, MID.t, **ctxkw)
    key = ctx.load_key(rlk)
    db = ctx.encode_db(codewords, payload, m)
    out = ctx.answer(key, db, torch.from_numpy(query).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy(), db.pair_count


@pytest.mark.parametrize("k,m", [(5, 8), (8, 10)])
@pytest.mark.parametrize("memo", ["database", "chunk"])
def test_deep_constant_weight_trees(k, m, memo):
    orc, sk, rlk, key = _keys()
    codes = np.array([perfect_map(i, m, k) for i in range(math.comb(m, k))], dtype=np.uint32)
    target = len(codes) // 3
    query = encrypt_query(orc, sk, [int(v) for v in codes[target]], m, 61, draw=k)
    pay = datagen.payload(MID.with_n(len(codes)), len(codes))
    want_key = (k, m)
    if want_key not in _cache:
        _cache[want_key] = orc.answer(key, query, codes, pay)
    kw = dict(chunk_elems=16) if memo == "database" else dict(chunk_elems=16, memo_bytes=1 << 20)
    _say(f"answer k={k} m={m} n={len(codes)} memo={memo}")
    got, nodes = _gpu_answer(query, codes, pay, m, **kw)
    assert np.array_equal(got, _cache[want_key])
    msg, _ = orc.decrypt(sk, got[0])
    assert np.array_equal(msg, pay[target][0].astype(np.uint64))


@pytest.mark.parametrize("n,chunk,memo", [(64, 24, 0), (50, 16, 1 << 20)])
def test_folklore_pir(n, chunk, memo):
    import torch
    from paper_2202_07569_amd import Context
    orc, sk, rlk, key = _keys()
    ell = index_bits(n)
    target = (7 * n) // 9
    q = folklore_query(orc, sk, target, ell, 61, draw=n)
    want_leaves = folklore_leaves(orc, q)
    ctx = Context(MID.N, MID.primes, MID.t, chunk_elems=chunk, memo_bytes=memo)
    _say(f"folklore leaves l={ell}")
    leaves = ctx.folklore_leaves(torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(leaves.cpu().numpy(), want_leaves)
    cw = folklore_codewords(n, ell)
    pay = datagen.payload(MID.with_n(n), n)
    gkey = ctx.load_key(rlk)
    db = ctx.encode_db(cw, pay, 2 * ell)
    _say(f"folklore answer n={n} chunk={chunk}")
    got = ctx.answer(gkey, db, leaves)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got, orc.answer(key, want_leaves, cw, pay))
    msg, _ = orc.decrypt(sk, got[0])
    assert np.array_equal(msg, pay[target][0].astype(np.uint64))
