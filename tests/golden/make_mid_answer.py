"""Write the oracle's full answer for the mid index-PIR workload to tests/golden/mid_answer.npz.

The workload is N = 8192, five primes (218 bits), t = 65537, k = 4, m = 27, n = 16384, s = 1, with
the seeded keys, database and query of `oracle.client.build_instance` (query for the seeded
target).  The answer is Eq. (1) with the selection vector of Algorithm 6 (Section 3.3.3), every
element's product tree evaluated in full by the C++ oracle.  Only `oracle/` and `datagen` are
called: no value here comes from the GPU library.

The file holds the answer [s][2][L][N] (uint64 residues), its SHA-256, the instance's target and the
oracle's wall time with the number of threads it used.  Run from the repository root:

    python tests/golden/make_mid_answer.py [--threads T]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import datagen  # noqa: E402
from oracle.client import build_instance  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mid_answer.npz")


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0 = all)")
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    cfg = datagen.CONFIGS["mid"]
    ins = build_instance(cfg)
    threads = args.threads or os.cpu_count() or 1
    print(f"oracle answer: mid n={cfg.n} k={cfg.k} m={cfg.m} on {threads} threads", flush=True)
    t0 = time.perf_counter()
    ans = ins.orc.answer(ins.key, ins.query, ins.codewords, ins.payload, threads=threads)
    secs = time.perf_counter() - t0
    msg, noise = ins.orc.decrypt(ins.sk, ans[0])
    if not np.array_equal(msg, ins.payload[ins.target][0].astype(np.uint64)):
        raise SystemExit("the oracle's answer does not decrypt to the queried payload")
    digest = hashlib.sha256(np.ascontiguousarray(ans).tobytes()).hexdigest()
    np.savez_compressed(args.out, answer=ans, sha256=np.array(digest), target=np.array(ins.target),
                        oracle_seconds=np.array(secs), oracle_threads=np.array(threads),
                        host=np.array(f"{platform.processor() or platform.machine()}, {os.cpu_count()} cpus"),
                        noise_log2=np.array(noise))
    print(f"wrote {args.out}: sha256 {digest}, {secs:.1f} s on {threads} threads "
          f"({cfg.n / secs:.1f} elements/s), noise 2^{noise:.1f}", flush=True)


if __name__ == "__main__":
    main()
