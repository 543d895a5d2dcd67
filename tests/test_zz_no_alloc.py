"""The no-allocation response compression (pir_mod_switch_noalloc) against pir_mod_switch.

Both entry points switch polynomials from q to q' = q_0 ... q_{keep-1} (the modulus switching of
responses, Section 2.2); the no-allocation one keeps its fixup list in a fixed per-GPU array.  Its
output must equal the allocating entry point's bit for bit, on two calls in a row (the second with
fewer polynomials, a different keep and a smaller ring, so that it runs over what the first left in
the shared array), with inputs that take the exact fallback; it must leave the library's device
bytes unchanged, refuse requests beyond its limit and leave the context usable.
"""
import math

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)


def _near_half(cfg, keep, count, seed):
    """count polynomials whose coefficients sit next to the rounding boundary of the switch to
    keep primes (k r +- (r -+ 1)/2, both signs), so every coefficient takes the exact fallback."""
    q = math.prod(cfg.primes)
    r = q // math.prod(cfg.primes[:keep])
    rng = np.random.default_rng(seed)
    out = np.empty((count, cfg.L, cfg.N), dtype=np.uint64)
    for c in range(count):
        ks = rng.integers(0, 1 << 40, size=cfg.N)
        up = rng.integers(0, 2, size=cfg.N)
        sign = rng.integers(0, 2, size=cfg.N)
        vals = [(-1 if sg else 1) * (int(k) * r + ((r - 1) // 2 if u else (r + 1) // 2))
                for k, u, sg in zip(ks, up, sign)]
        for j, p in enumerate(cfg.primes):
            out[c, j] = np.array([v % p for v in vals], dtype=np.uint64)
    return out


def _pair(ctx, x, keep):
    import torch
    a = ctx.mod_switch(x, keep)
    out = ctx.empty(*x.shape[:-2], keep, ctx.N)
    before = ctx.device_bytes
    b = ctx.mod_switch_noalloc(x, keep, out=out)
    torch.cuda.synchronize()
    assert ctx.device_bytes == before
    return a.cpu().numpy(), b.cpu().numpy()


def test_mod_switch_noalloc_equals_mod_switch():
    import torch
    from paper_2202_07569_amd import Context, PirError
    mid, tiny = datagen.CONFIGS["mid"], datagen.CONFIGS["tiny"]
    cm = Context(mid.N, mid.primes, mid.t)
    # first call: 24 polynomials at N = 8192 (half random, half next to the boundary), keep 1
    x1 = np.concatenate([datagen.uniform_residues(mid.primes, (12,), mid.N, seed=41),
                         _near_half(mid, 1, 12, seed=42)])
    _say("noalloc mod switch: mid, 24 polynomials, keep 1")
    a, b = _pair(cm, torch.from_numpy(x1).cuda(), 1)
    assert np.array_equal(a, b)
    # second call right after, smaller: 3 polynomials of another context (N = 4096), keep 2
    ct = Context(tiny.N, tiny.primes, tiny.t)
    x2 = np.concatenate([datagen.uniform_residues(tiny.primes, (1,), tiny.N, seed=43),
                         _near_half(tiny, 2, 2, seed=44)])
    _say("noalloc mod switch: tiny, 3 polynomials, keep 2")
    a, b = _pair(ct, torch.from_numpy(x2).cuda(), 2)
    assert np.array_equal(a, b)
    # keep = L is the identity; count = 0 does nothing
    _say("noalloc mod switch: keep = L, count = 0")
    a, b = _pair(cm, torch.from_numpy(x1[:2]).cuda(), mid.L)
    assert np.array_equal(a, b) and np.array_equal(b, x1[:2])
    empty = cm.empty(0, mid.L, mid.N)
    assert cm.mod_switch_noalloc(empty, 1).shape == (0, 1, mid.N)
    # beyond the limit (2^19 coefficients): refused, nothing enqueued, the context still works
    big = cm.empty(65, mid.L, mid.N)
    with pytest.raises(PirError) as err:
        cm.mod_switch_noalloc(big, 1)
    assert "2^19" in str(err.value)
    _say("noalloc mod switch: after a refused call")
    a, b = _pair(cm, torch.from_numpy(x1[:5]).cuda(), 3)
    assert np.array_equal(a, b)
