"""Parity of the HIP path with the CPU oracle (bit-exact: every result is an exact integer).

Unit level (single FV operations through the C ABI), selector level (Algorithm 6) and answer level
(Eq. (1) over whole databases), at sizes the oracle finishes in seconds that still span several
chunks and a ragged tail, plus edge cases: k = 1 and k = 3 trees, an empty database, an absent
keyword, near-half rounding inputs, level-1 products shared per database and per chunk.
"""
import math

import numpy as np
import pytest

import datagen
from conftest import cached_instance
from oracle.client import build_instance
from oracle.core import Oracle
from oracle.mapping import lossy_map, perfect_map

pytestmark = pytest.mark.gpu

PARAMS = {name: datagen.CONFIGS[name] for name in ("tiny", "mid", "keyword")}
_ctxs = {}


def _torch():
    import torch
    return torch


def ctx_for(cfg, **kw):
    from paper_2202_07569_amd import Context
    key = (cfg.N, cfg.primes, tuple(sorted(kw.items())))
    if key not in _ctxs:
        _ctxs[key] = Context(cfg.N, cfg.primes, cfg.t, **kw)
    return _ctxs[key]


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


# ---------------------------------------------------------------------------------------------
# unit level
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(PARAMS))
def test_pm_matches_oracle(name):
    cfg = PARAMS[name]
    orc, ctx = Oracle(cfg.N, cfg.primes), ctx_for(cfg)
    ct = datagen.uniform_residues(cfg.primes, (2,), cfg.N, seed=101)
    pt = (datagen.words(102, 4, cfg.N) % np.uint64(1 << 16)).astype(np.uint16)
    _say(f"pm {name}")
    assert np.array_equal(_host(ctx.pm(_dev(ct), _dev(pt))), orc.pm(ct, pt.astype(np.uint64)))


@pytest.mark.parametrize("name", list(PARAMS))
def test_mult_matches_oracle_random(name):
    cfg = PARAMS[name]
    orc, ctx = Oracle(cfg.N, cfg.primes), ctx_for(cfg)
    u = datagen.uniform_residues(cfg.primes, (2, 2), cfg.N, seed=103)
    _say(f"mult {name}")
    assert np.array_equal(_host(ctx.mult(_dev(u[0]), _dev(u[1]))), orc.mult(u[0], u[1]))


def _const_ct(primes, N, c0, c1):
    ct = np.zeros((2, len(primes), N), dtype=np.uint64)
    for j, p in enumerate(primes):
        ct[0, j, 0], ct[1, j, 0] = c0 % p, c1 % p
    return ct


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_mult_near_half_rounding(name):
    """Inputs whose centred lift (extension) or whose [t X]_q (rounding) sits next to q/2: the
    conversions decide them through the exact fallback."""
    cfg = PARAMS[name]
    orc, ctx = Oracle(cfg.N, cfg.primes), ctx_for(cfg)
    q, t = math.prod(cfg.primes), cfg.t
    it = pow(t, -1, q)
    cases = [((q - 1) // 2, (q + 1) // 2, 1, 0), ((q + 1) // 2, (q - 1) // 2, (q - 1) // 2, 1),
             ((q - 1) // 2 * it % q, 5, 1, 0), ((q + 1) // 2 * it % q, 7, 1, 0),
             ((q - 1) // 2 * it % q, (q + 1) // 2 * it % q, 1, 1)]
    for a0, a1, b0, b1 in cases:
        a = _const_ct(cfg.primes, cfg.N, a0, a1)
        b = _const_ct(cfg.primes, cfg.N, b0, b1)
        # spread the adversarial coefficient over the whole polynomial as well
        a[:, :, 1::3] = a[:, :, :1]
        _say(f"near-half mult {name}")
        assert np.array_equal(_host(ctx.mult(_dev(a), _dev(b))), orc.mult(a, b))


def _keys(cfg, orc, seed):
    sk = orc.keygen(datagen.words(seed, datagen.S_SECRET, cfg.N))
    return sk, orc.relin_keygen(sk, datagen.words(seed, datagen.S_RLK, orc.rnd_words_rlk()))


@pytest.mark.parametrize("name", list(PARAMS))
def test_relin_matches_oracle(name):
    cfg = PARAMS[name]
    orc, ctx = Oracle(cfg.N, cfg.primes), ctx_for(cfg)
    sk, rlk = _keys(cfg, orc, 104)
    c3 = datagen.uniform_residues(cfg.primes, (3,), cfg.N, seed=105)
    _say(f"relin {name}")
    gk = ctx.load_key(rlk)
    assert np.array_equal(_host(ctx.relin(gk, _dev(c3))), orc.relin(orc.load_key(rlk), c3))


# ---------------------------------------------------------------------------------------------
# codeword tables
# ---------------------------------------------------------------------------------------------
def test_map_perfect_matches_algorithm3():
    cfg = PARAMS["tiny"]
    ctx = ctx_for(cfg)
    for m, k in ((24, 2), (27, 4), (725, 2), (12, 8)):
        size = math.comb(m, k)
        ids = np.unique(np.concatenate([datagen.words(m * 31 + k, 5, 300) % np.uint64(size),
                                        np.array([0, size - 1], dtype=np.uint64)]))
        _say(f"map_perfect m={m} k={k}")
        got = _host(ctx.map_perfect(ids, m, k))
        want = np.array([perfect_map(int(x), m, k) for x in ids], dtype=np.uint32)
        assert np.array_equal(got, want)


def test_map_lossy_matches_algorithm8():
    cfg = PARAMS["tiny"]
    ctx = ctx_for(cfg)
    kws = datagen.words(7, datagen.S_KEYWORDS, 500)
    for m, k, seed in ((569, 4, 0x1234), (24, 2, 99), (10, 3, 5)):
        _say(f"map_lossy m={m} k={k}")
        got = _host(ctx.map_lossy(kws, m, k, seed))
        want = np.array([lossy_map(int(x), m, k, seed) for x in kws], dtype=np.uint32)
        assert np.array_equal(got, want)


# ---------------------------------------------------------------------------------------------
# selectors and answers
# ---------------------------------------------------------------------------------------------
_inst = {}


def inst(cfg, absent=False):
    key = (cfg, absent)
    if key not in _inst:
        _inst[key] = build_instance(cfg, absent=absent)
    return _inst[key]


def _gpu_answer(cfg, ins, **ctxkw):
    ctx = ctx_for(cfg, **ctxkw)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    return _host(ctx.answer(key, db, _dev(ins.query))), db


_want = {}


def oracle_answer(cfg, ins):
    k = (cfg, ins.target)
    if k not in _want:
        _want[k] = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
    return _want[k]


TINY64 = datagen.CONFIGS["tiny"].with_n(64, m=12)


def test_selectors_tiny_all_elements():
    cfg = TINY64
    ins = inst(cfg)
    ctx = ctx_for(cfg)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    _say("selectors tiny n=64")
    got = _host(ctx.selectors(key, db, _dev(ins.query), np.arange(cfg.n)))
    for j in range(cfg.n):
        assert np.array_equal(got[j], ins.orc.selector(ins.key, ins.query, ins.codewords[j])), j


def test_answer_tiny_full_config():
    cfg = datagen.CONFIGS["tiny"]
    ins = inst(cfg)
    _say("answer tiny n=256")
    got, _ = _gpu_answer(cfg, ins)
    assert np.array_equal(got, oracle_answer(cfg, ins))
    msg, noise = ins.orc.decrypt(ins.sk, got[0])
    assert np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64))


def test_answer_tiny_ragged_chunks():
    cfg = datagen.CONFIGS["tiny"].with_n(200)
    ins = inst(cfg)
    _say("answer tiny n=200 chunk=48")
    got, _ = _gpu_answer(cfg, ins, chunk_elems=48)
    assert np.array_equal(got, oracle_answer(cfg, ins))


MID96 = datagen.CONFIGS["mid"].with_n(96)


@pytest.mark.parametrize("memo", ["database", "chunk"])
def test_answer_mid_k4_ragged(memo):
    cfg = MID96
    ins = inst(cfg)
    kw = dict(chunk_elems=40) if memo == "database" else dict(chunk_elems=40, memo_bytes=1 << 20)
    _say(f"answer mid n=96 memo={memo}")
    got, db = _gpu_answer(cfg, ins, **kw)
    if memo == "database":
        assert db.pair_count < 2 * cfg.n      # shared across the whole database
    assert np.array_equal(got, oracle_answer(cfg, ins))
    msg, _ = ins.orc.decrypt(ins.sk, got[0])
    assert np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64))


KW_SMALL = datagen.Config("kw-small", 4096, datagen.Q_N4096, 65537, 2, 24, 40, 2, 7, keyword=True)


@pytest.mark.parametrize("absent", [False, True])
def test_answer_keyword_small(absent):
    cfg = KW_SMALL
    ins = inst(cfg, absent=absent)
    _say(f"answer keyword-small absent={absent}")
    got, _ = _gpu_answer(cfg, ins, chunk_elems=16)
    assert np.array_equal(got, oracle_answer(cfg, ins))
    for r in range(cfg.s):
        msg, _ = ins.orc.decrypt(ins.sk, got[r])
        want = np.zeros(cfg.N, np.uint64) if absent else ins.payload[ins.target][r].astype(np.uint64)
        assert np.array_equal(msg, want)


@pytest.mark.parametrize("k,m,n", [(1, 20, 20), (3, 9, 70)])
def test_answer_tree_shapes(k, m, n):
    cfg = datagen.Config(f"tiny-k{k}", 4096, datagen.Q_N4096, 65537, k, m, n, 1, 30 + k)
    ins = inst(cfg)
    _say(f"answer k={k}")
    got, _ = _gpu_answer(cfg, ins, chunk_elems=32)
    assert np.array_equal(got, oracle_answer(cfg, ins))


def test_answer_empty_database_is_zero():
    cfg = datagen.CONFIGS["tiny"]
    ctx = ctx_for(cfg)
    ins = inst(TINY64)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(np.zeros((0, 2), np.uint32), np.zeros((0, 1, cfg.N), np.uint16), 12)
    _say("answer empty db")
    assert not _host(ctx.answer(key, db, _dev(ins.query))).any()


def test_batch_equals_single_answers():
    cfg = TINY64
    ctx = ctx_for(cfg, chunk_elems=24)
    a, b = inst(cfg), inst(KW_SMALL)
    ka, kb = ctx.load_key(a.rlk), ctx.load_key(b.rlk)
    da = ctx.encode_db(a.codewords, a.payload, cfg.m)
    db = ctx.encode_db(b.codewords, b.payload, KW_SMALL.m)
    qa, qb = _dev(a.query), _dev(b.query)
    # a second query on database a: the codeword of another element
    other = (a.target + 5) % cfg.n
    from oracle.client import encrypt_query
    qa2 = _dev(encrypt_query(a.orc, a.sk, [int(v) for v in a.codewords[other]], cfg.m, cfg.seed, draw=3))
    _say("batch of 3")
    outs = ctx.answer_batch([ka, kb, ka], [da, db, da], [qa, qb, qa2])
    singles = [ctx.answer(ka, da, qa), ctx.answer(kb, db, qb), ctx.answer(ka, da, qa2)]
    for o, s in zip(outs, singles):
        assert np.array_equal(_host(o), _host(s))
    assert np.array_equal(_host(outs[0]), oracle_answer(cfg, a))
    msg, _ = a.orc.decrypt(a.sk, _host(outs[2])[0])
    assert np.array_equal(msg, a.payload[other][0].astype(np.uint64))


def test_encode_db_rejects_bad_codewords():
    from paper_2202_07569_amd import PirError
    cfg = datagen.CONFIGS["tiny"]
    ctx = ctx_for(cfg)
    pay = np.zeros((2, 1, cfg.N), np.uint16)
    for cw in (np.array([[3, 3], [0, 1]]), np.array([[4, 2], [0, 1]]), np.array([[0, 24], [0, 1]])):
        with pytest.raises(PirError):
            ctx.encode_db(cw.astype(np.uint32), pay, 24)


def test_answer_and_seeded_rebuild_on_a_side_stream_with_host_inputs():
    """Host arrays are copied to the device on torch's current stream; a call on another stream
    must wait for that copy and keep the copies alive until it has run."""
    import torch
    from oracle import seeded as S
    cfg = PARAMS["tiny"].with_n(40)
    ins = cached_instance(cfg)
    ctx = ctx_for(cfg)
    key, db = ctx.load_key(ins.rlk), ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    side = torch.cuda.Stream()  # default priority
    _say("answer tiny n=40 on a side stream, host query")
    got = ctx.answer(key, db, ins.query, stream=side)
    c0 = datagen.uniform_residues(cfg.primes, (3,), cfg.N, seed=17)
    full = ctx.seeded_query(c0, 99, stream=side)
    side.synchronize()
    assert np.array_equal(got.cpu().numpy(), ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload))
    assert np.array_equal(full.cpu().numpy(), S.unseed(cfg.primes, cfg.N, c0, 99))
