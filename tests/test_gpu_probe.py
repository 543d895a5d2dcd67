"""The issue-rate probes (pir_probe_fp64, pir_probe_int): each reports a positive duration and the
number of wave-instructions of the timed operation that its launch issues (waves x iterations x
chains; the assembly of the probe loops holds exactly one such instruction per chain and
iteration), and rejects out-of-range arguments."""
import pytest

import datagen

pytestmark = pytest.mark.gpu


def test_probe_counts_and_arguments():
    from paper_2202_07569_amd import Context, PirError
    cfg = datagen.CONFIGS["tiny"]
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    for op in range(4):
        ms, wi = ctx.probe_fp64(op, blocks=64, iters=128)
        assert ms > 0.0
        assert wi == 64 * 4 * 128 * 8 * (2 if op == 3 else 1)  # waves x iterations x chains
    for bad in (dict(op=4), dict(op=0, blocks=0), dict(op=0, iters=(1 << 20) + 1)):
        with pytest.raises(PirError):
            ctx.probe_fp64(**bad)


def test_integer_probe_counts_and_arguments():
    from paper_2202_07569_amd import Context, PirError
    cfg = datagen.CONFIGS["tiny"]
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    for op in range(4):
        ms, wi = ctx.probe_int(op, blocks=64, iters=128)
        assert ms > 0.0
        assert wi == 64 * 4 * 128 * 8  # waves x iterations x chains
    for bad in (dict(op=4), dict(op=-1), dict(op=0, blocks=(1 << 20) + 1), dict(op=0, iters=0)):
        with pytest.raises(PirError):
            ctx.probe_int(**bad)
