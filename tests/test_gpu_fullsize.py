"""Full-size checks of the HIP path in the configuration the benchmark times.

At the mid size (the workload the benchmark times) the GPU answer is compared element by element
with the oracle's full answer, which a committed script computes from `oracle/` alone
(`tests/golden/make_mid_answer.py`, stored in `tests/golden/mid_answer.npz`): under the plain
loop's schedule and as query 0 of the benchmark's batch of 8.  The oracle cannot compute a whole
answer over the large and keyword databases in seconds, so there the checks use what holds at any
size: the decrypted answer is the queried payload (zero for an absent keyword), sampled selectors
equal the oracle's bit for bit, the answer is linear over a split of the database, and a batch
equals the single answers (their parameters are compared with the oracle's whole answer on small
databases in `test_gpu_params_parity.py`).  Contexts take the launch schedules the benchmark uses
(the package's tuning cache): the plain loop's for single answers and, at the mid size, the
batch-of-8 schedule for the benchmark's batched step.
"""
import hashlib
import os

import numpy as np
import pytest

import datagen
from oracle.client import build_instance, encrypt_query

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _torch():
    import torch
    return torch


def _dev(a):
    return _torch().from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[gpu-full] {msg}", flush=True)


def _context(cfg, batch=1):
    """A context with the launch schedule the benchmark uses for `batch` queries per call (the
    package's tuning cache), or the library default when the cache has none."""
    from paper_2202_07569_amd import Context
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    sched = ctx.cached_schedule(batch, cfg.k, cfg.s)
    if sched is not None:
        ctx.set_schedule(sched["chunk_elems"], min(sched["query_group"], batch), sched["relin_group"])
    return ctx


def _check(cfg, ins, samples, absent=False, split=None):
    ctx = _context(cfg)
    key = ctx.load_key(ins.rlk)
    db = ctx.encode_db(ins.codewords, ins.payload, cfg.m)
    _say(f"{cfg.name}: answer over n={cfg.n}")
    ans = _host(ctx.answer(key, db, _dev(ins.query)))
    for r in range(cfg.s):
        msg, noise = ins.orc.decrypt(ins.sk, ans[r])
        want = np.zeros(cfg.N, np.uint64) if absent else ins.payload[ins.target][r].astype(np.uint64)
        assert np.array_equal(msg, want), r
        assert noise < ins.orc.log2_half_delta() - 8
    _say(f"{cfg.name}: sampled selectors {list(samples)}")
    sel = _host(ctx.selectors(key, db, _dev(ins.query), np.array(samples, dtype=np.uint64)))
    for i, j in enumerate(samples):
        assert np.array_equal(sel[i], ins.orc.selector(ins.key, ins.query, ins.codewords[j])), j
    if split:
        _say(f"{cfg.name}: linearity at {split}")
        q = np.array(cfg.primes, dtype=np.uint64).reshape(1, 1, -1, 1)
        da = ctx.encode_db(ins.codewords[:split], ins.payload[:split], cfg.m)
        dbb = ctx.encode_db(ins.codewords[split:], ins.payload[split:], cfg.m)
        a = _host(ctx.answer(key, da, _dev(ins.query)))
        b = _host(ctx.answer(key, dbb, _dev(ins.query)))
        assert np.array_equal(ans, (a + b) % q)
    return ctx, key, db, ans


GOLDEN_MID = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mid_answer.npz")


def _golden_mid(target):
    """The oracle's full mid answer from the committed golden file (checked against its digest)."""
    with np.load(GOLDEN_MID, allow_pickle=False) as z:
        want, digest, tgt = z["answer"], str(z["sha256"]), int(z["target"])
    assert hashlib.sha256(np.ascontiguousarray(want).tobytes()).hexdigest() == digest
    assert tgt == target
    return want


def _diff(got, want):
    bad = np.argwhere(got != want)
    return f"{len(bad)} residues differ, first at {tuple(bad[0]) if len(bad) else None}"


def test_mid_full_size():
    cfg = datagen.CONFIGS["mid"]
    ins = build_instance(cfg)
    ctx, key, db, ans = _check(cfg, ins, [ins.target, 0, cfg.n - 1], split=9001)
    assert db.pair_count <= 351
    _say(f"mid: plain answer under schedule {ctx.schedule()} against the oracle's full answer")
    want = _golden_mid(ins.target)
    assert ans.shape == want.shape
    assert np.array_equal(ans, want), _diff(ans, want)
    # the benchmark's batched step: 8 queries for 8 elements under the batch-8 schedule; query 0
    # equals the plain answer bit for bit and every answer decrypts to its element's payload
    ctx8 = _context(cfg, batch=8)
    key8, db8 = ctx8.load_key(ins.rlk), ctx8.encode_db(ins.codewords, ins.payload, cfg.m)
    others = [(ins.target + 777 * b) % cfg.n for b in range(1, 8)]
    qs = [ins.query] + [encrypt_query(ins.orc, ins.sk, [int(v) for v in ins.codewords[o]], cfg.m, cfg.seed,
                                      draw=4 + b) for b, o in enumerate(others)]
    _say(f"mid: batch of 8 under schedule {ctx8.schedule()}")
    outs = ctx8.answer_batch([key8] * 8, [db8] * 8, [_dev(q) for q in qs])
    got0 = _host(outs[0])
    assert np.array_equal(got0, want), _diff(got0, want)
    for o, out in zip(others, outs[1:]):
        msg, _ = ins.orc.decrypt(ins.sk, _host(out)[0])
        assert np.array_equal(msg, ins.payload[o][0].astype(np.uint64)), o


def test_large_full_size():
    cfg = datagen.CONFIGS["large"]
    ins = build_instance(cfg)
    _check(cfg, ins, [ins.target, 1, cfg.n - 1])


@pytest.mark.parametrize("absent", [False, True])
def test_keyword_full_size(absent):
    cfg = datagen.CONFIGS["keyword"]
    ins = build_instance(cfg, absent=absent)
    samples = [0, cfg.n - 1] if absent else [ins.target, cfg.n - 1]
    _check(cfg, ins, samples, absent=absent)
