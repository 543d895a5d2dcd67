"""Host code under sanitizers, CPU only (g++; no GPU code is built with them).

* The library's host-side parameter construction (csrc/host_params.cpp) with AddressSanitizer and
  UndefinedBehaviorSanitizer, driven over the workload prime sets (tests/sanitize).
* The C++ oracle with UndefinedBehaviorSanitizer (abort on the first report), running a tiny PIR
  answer and a key switch in a child process.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_07569_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def test_host_params_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_params_check")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", CSRC, os.path.join(ROOT, "tests", "sanitize", "host_params_check.cpp"),
                    os.path.join(CSRC, "host_params.cpp"), "-o", exe], check=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")


CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import oracle.build as ob
ob.LIB = {lib!r}
import numpy as np
import datagen
from oracle.client import build_instance
cfg = datagen.CONFIGS["tiny"].with_n(6)
ins = build_instance(cfg)
ans = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload)
msg, _ = ins.orc.decrypt(ins.sk, ans[0])
assert np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64))
c3 = datagen.uniform_residues(cfg.primes, (3,), cfg.N, seed=3)
ins.orc.relin(ins.key, c3)
print("ok")
"""


def test_oracle_under_ubsan(tmp_path):
    lib = str(tmp_path / "libcwpir_oracle.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fsanitize=undefined",
                    "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "cwpir_oracle.cpp"), "-o", lib],
                   check=True, timeout=300)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib)], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("ok")
