"""Parity of the HIP arithmetic constant-weight equality (Algorithm 2) with the oracle, bit for bit.

Batch-encoded ciphertexts of random codeword pairs (about half of the N slots equal); the GPU result
must equal the oracle's ciphertext and decrypt and decode to the equality indicator.  k = 1 and
k = 3 check the tree's edge shapes bit for bit (k = 3 exceeds the tiny noise budget, so only the
bits are compared there).
"""
import numpy as np
import pytest

import datagen
from oracle import arith as A
from test_oracle_arith import _run

pytestmark = pytest.mark.gpu


def _gpu(name, x, y, k):
    import torch
    from paper_2202_07569_amd import Context
    cfg = datagen.CONFIGS[name]
    seed = {"tiny": 71, "mid": 72}.get(name, 73)
    from oracle.core import Oracle
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    sk = orc.keygen(datagen.words(seed, datagen.S_SECRET, cfg.N))
    rlk = orc.relin_keygen(sk, datagen.words(seed, datagen.S_RLK, orc.rnd_words_rlk()))
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    key = ctx.load_key(rlk)
    out = ctx.arith_equality(key, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), k)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name,m,k,seed", [("tiny", 6, 2, 71), ("mid", 8, 4, 72)])
def test_arith_equality_matches_oracle(name, m, k, seed):
    got_slots, want, noise, budget, (x, y, e) = _run(name, m, k, seed)
    print(f"[gpu] arith equality {name} m={m} k={k}", flush=True)
    assert np.array_equal(_gpu(name, x, y, k), e)
    assert np.array_equal(got_slots, want)


@pytest.mark.parametrize("m,k", [(4, 1), (7, 3)])
def test_arith_equality_tree_shapes(m, k):
    from oracle.core import Oracle
    cfg = datagen.CONFIGS["tiny"]
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    sk = orc.keygen(datagen.words(71, datagen.S_SECRET, cfg.N))
    key = orc.load_key(orc.relin_keygen(sk, datagen.words(71, datagen.S_RLK, orc.rnd_words_rlk())))
    x = datagen.uniform_residues(cfg.primes, (m, 2), cfg.N, seed=90 + k)
    y = datagen.uniform_residues(cfg.primes, (m, 2), cfg.N, seed=95 + k)
    print(f"[gpu] arith equality shape m={m} k={k}", flush=True)
    assert np.array_equal(_gpu("tiny", x, y, k), A.arith_equality(orc, key, x, y, k))
