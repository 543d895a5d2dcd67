"""Parity of the HIP query expansion (Algorithm 5) with the oracle, bit for bit.

Packed queries (Algorithm 4) and Galois keys come from the oracle; the GPU expands them through the
C ABI (pir_expand) and the result must equal the oracle's expansion exactly.  At the mid parameters
a packed query is then answered end to end and must equal the oracle's answer on the oracle's
expansion and decrypt to the queried payload.  The N = 16384 parameters exercise the staged key
switch.
"""
import numpy as np
import pytest

import datagen
from conftest import cached_instance
from oracle import expand as X
from oracle.core import Oracle
from oracle.mapping import codeword_bits

pytestmark = pytest.mark.gpu
_ctx = {}


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _context(cfg):
    from paper_2202_07569_amd import Context
    k = (cfg.N, cfg.primes)
    if k not in _ctx:
        _ctx[k] = Context(cfg.N, cfg.primes, cfg.t)
    return _ctx[k]


def _setup(cfg, c, m, positions, draw=0, sk=None, orc=None):
    orc = orc or Oracle(cfg.N, cfg.primes, cfg.t)
    if sk is None:
        sk = orc.keygen(datagen.words(cfg.seed, datagen.S_SECRET, cfg.N))
    gk = X.galois_keys(orc, sk, c, cfg.seed)
    packed = X.pack_query(orc, sk, codeword_bits(positions, m), c, cfg.seed, draw=draw)
    return orc, sk, gk, packed


def _gpu_expand(cfg, gk, c, packed, m):
    import torch
    ctx = _context(cfg)
    keys = [ctx.load_galois_key(g, gk[g]) for g in X.galois_elements(cfg.N, c)]
    out = ctx.expand(keys, c, torch.from_numpy(packed).cuda(), m)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("c", [0, 1, 3, 5])
def test_expand_tiny_matches_oracle(c):
    cfg = datagen.CONFIGS["tiny"]
    orc, sk, gk, packed = _setup(cfg, c, cfg.m, [4, 19], draw=c)
    _say(f"expand tiny c={c}")
    got = _gpu_expand(cfg, gk, c, packed, cfg.m)
    assert np.array_equal(got, X.expand(orc, gk, packed, cfg.m, c))


def test_expand_ragged_last_packed_ciphertext():
    cfg = datagen.CONFIGS["tiny"]
    m, c = 21, 3  # h = 3, the last packed ciphertext holds 5 of 8 slots
    orc, sk, gk, packed = _setup(cfg, c, m, [0, 20])
    _say("expand tiny m=21 c=3")
    got = _gpu_expand(cfg, gk, c, packed, m)
    assert np.array_equal(got, X.expand(orc, gk, packed, m, c))


def test_expand_n16384_staged_key_switch():
    cfg = datagen.CONFIGS["keyword"]
    m, c = 40, 3
    orc, sk, gk, packed = _setup(cfg, c, m, [1, 9, 30, 39])
    _say("expand N=16384 m=40 c=3")
    got = _gpu_expand(cfg, gk, c, packed, m)
    assert np.array_equal(got, X.expand(orc, gk, packed, m, c))


def test_packed_query_answer_mid_end_to_end():
    import torch
    cfg = datagen.CONFIGS["mid"].with_n(48)
    ins = cached_instance(cfg)
    c = 5
    orc, sk = ins.orc, ins.sk
    gk = X.galois_keys(orc, sk, c, cfg.seed)
    packed = X.pack_query(orc, sk, codeword_bits(ins.positions, cfg.m), c, cfg.seed)
    want_query = X.expand(orc, gk, packed, cfg.m, c)
    _say("expand mid m=27 c=5, then answer n=48")
    ctx = _context(cfg)
    keys = [ctx.load_galois_key(g, gk[g]) for g in X.galois_elements(cfg.N, c)]
    q = ctx.expand(keys, c, torch.from_numpy(packed).cuda(), cfg.m)
    torch.cuda.synchronize()
    assert np.array_equal(q.cpu().numpy(), want_query)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    got = ctx.answer(key, db, q)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert np.array_equal(got, orc.answer(ins.key, want_query, ins.codewords, ins.payload))
    msg, noise = orc.decrypt(sk, got[0])
    assert np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64))
    assert noise < orc.log2_half_delta() - 10


def test_expand_rejects_bad_keys_and_shapes():
    import torch
    from paper_2202_07569_amd import PirError
    cfg = datagen.CONFIGS["tiny"]
    orc, sk, gk, packed = _setup(cfg, 2, cfg.m, [0, 1])
    ctx = _context(cfg)
    g0, g1 = X.galois_elements(cfg.N, 2)
    k0, k1 = ctx.load_galois_key(g0, gk[g0]), ctx.load_galois_key(g1, gk[g1])
    dev = torch.from_numpy(packed).cuda()
    with pytest.raises(PirError):
        ctx.expand([k1, k0], 2, dev, cfg.m)        # levels out of order
    with pytest.raises(PirError):
        ctx.expand([k0, k1], 2, dev[:-1], cfg.m)   # h != ceil(m / 2^c)
    with pytest.raises(PirError):
        ctx.load_galois_key(2, gk[g0])             # even Galois element
