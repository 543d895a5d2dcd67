"""Parity of the HIP modulus switching (response compression) with the oracle, bit for bit.

Random residues at the three parameter sets and every `keep`, constants next to the rounding
boundary (they take the exact fallback of the conversion), and a PIR answer computed on the GPU,
switched on the GPU and decrypted under the smaller modulus.
"""
import math

import numpy as np
import pytest

import datagen
from conftest import cached_instance
from oracle.core import Oracle

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


def _switch(cfg, x, keep):
    import torch
    out = _context(cfg).mod_switch(torch.from_numpy(x).cuda(), keep)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name", ["tiny", "mid", "keyword"])
def test_mod_switch_random_residues(name):
    cfg = datagen.CONFIGS[name]
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    x = datagen.uniform_residues(cfg.primes, (3,), cfg.N, seed=77)
    for keep in sorted({1, 2, cfg.L - 1, cfg.L}):
        _say(f"mod switch {name} keep={keep}")
        assert np.array_equal(_switch(cfg, x, keep), orc.mod_switch(x, keep)), keep


def test_mod_switch_near_half_takes_the_exact_path():
    cfg = datagen.CONFIGS["mid"]
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    q = math.prod(cfg.primes)
    rng = np.random.default_rng(5)
    for keep in (1, 3):
        r = q // math.prod(cfg.primes[:keep])
        vals = []
        for _ in range(cfg.N):  # k r +- (r -+ 1) / 2 for random k, both signs
            k = int(rng.integers(0, 1 << 40))
            v = k * r + ((r - 1) // 2 if rng.integers(2) else (r + 1) // 2)
            vals.append(-v if rng.integers(2) else v)
        x = np.array([[v % p for v in vals] for p in cfg.primes], dtype=np.uint64)[None]
        _say(f"mod switch near-half keep={keep}")
        assert np.array_equal(_switch(cfg, x, keep), orc.mod_switch(x, keep)), keep


def test_switched_gpu_answer_decrypts_mid():
    import torch
    cfg = datagen.CONFIGS["mid"].with_n(48)
    ins = cached_instance(cfg)
    ctx = _context(cfg)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    _say("answer mid n=48, then switch to one prime")
    ans = ctx.answer(key, db, torch.from_numpy(ins.query).cuda())
    sw = ctx.mod_switch(ans, 1)
    torch.cuda.synchronize()
    got = sw.cpu().numpy()
    want = ins.orc.mod_switch(ans.cpu().numpy().reshape(-1, cfg.L, cfg.N), 1).reshape(got.shape)
    assert np.array_equal(got, want)
    small = Oracle(cfg.N, cfg.primes[:1], cfg.t)
    msg, _ = small.decrypt(ins.sk, got[0])
    assert np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64))
