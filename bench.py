"""Benchmark of the constant-weight PIR server path on one MI355X.

Workload: index PIR, N = 8192, five ciphertext primes (218 bits), t = 65537, k = 4 (depth-2
equality tree), m = 27, n = 16384 elements of one uint16 plaintext each (Section 5's synthetic
databases at the parameters of the mid configuration).  One step is one pass of the whole server
path (Section 3.3.3: selection vector by the plain constant-weight equality operator, Algorithm 6,
then the inner product with the database, Eq. (1)) for a batch of B queries against the resident
database; B = 1 is the plain one-query-at-a-time loop.  `value` is DB elements answered per
second for the batched step; the plain step, per-step latency percentiles, the dominant kernel's
roofline and the CPU oracle on a bounded sample are reported beside it.

Inputs are synthetic and seeded: payload uniform uint16, identifiers a seeded permutation mapped
to codewords on the GPU (Algorithm 3), and query ciphertexts and relinearization key as uniform
residues modulo each prime (statistically like real encryptions; the arithmetic and its cost do
not depend on the values, and nobody decrypts them).  Everything is resident in HBM before timing.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402

MI355X_HBM_GBPS = 8000.0
MI355X_CUS, MI355X_CLOCK_HZ = 256, 2.4e9
# Integer ALU roof: the 32-bit multiplies (v_mul_lo_u32, v_mul_hi_u32, v_mad_u64_u32) issue at one
# wave-instruction (64 lanes) per CU per clock while the CUs are busy (pir_probe_int, counters
# SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES = 0.94-0.96): 256 x 64 x 2.4 GHz = 39.3 T/s (timed 32-34 T/s
# at the lower clock of dense multiply chains).
MI355X_INT_MUL_PER_S = 256 * 64 * 2.4e9
MULS_PER_BUTTERFLY = 10  # 64-bit Shoup butterfly: hi64(a w') 5 mads, lo64(a w) and lo64(q p) 4 muls + 1 mul_hi
# fp64 roof: 78.6 TFLOP/s counting an FMA as two flops = 39.3 T fp64 instructions/s.  The fp64
# butterfly (primes below 2^50) needs 8: y*w, fma, h*(1/p), rint, fma, + l, X + T, X - T.
MI355X_FP64_INSTR_PER_S = 78.6e12 / 2
FP64_OPS_PER_BUTTERFLY = 8
FP_PRIME_BOUND = 1 << 50
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mid_answer_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2202_07569_amd", "csrc", f) for f in ("kernels.hip", "arith.h", "consts.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=8, help="queries per batched step")
    ap.add_argument("--workload", default="mid", choices=["mid", "tiny", "large", "keyword"])
    ap.add_argument("--n", type=int, default=0, help="override the database size")
    ap.add_argument("--cpu-sample", type=int, default=-1, help="oracle sample elements (0: skip)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--autotune", type=int, default=-1, choices=[-1, 0, 1],
                    help="1: tune the launch schedule per batch size before encoding; 0: never; "
                         "-1: use the package's tuning cache when it has the workload, else tune")
    ap.add_argument("--record-schedule", default="", help="write tuned schedules into this cache file")
    ap.add_argument("--schedule", default="",
                    help="fixed schedule 'chunk,query_group,relin_group[,ntt_shape]' for both loops instead of tuning")
    ap.add_argument("--chunk", type=int, default=0, help="elements per processing chunk (0: library default)")
    ap.add_argument("--defer-relin", type=int, default=1, choices=[0, 1, 2],
                    help="when root products are relinearized after the inner product (pir_set_defer_relin): "
                         "0 never, 1 where it pays (library default), 2 wherever allowed")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (reference for rocprofv3 byte counters)")
    ap.add_argument("--serve", type=int, default=-1, choices=[-1, 0, 1],
                    help="also replay the batched-serving trace (4 resident databases, Poisson arrivals)")
    ap.add_argument("--serve-queries", type=int, default=256)
    ap.add_argument("--serve-rates", default="0.8,2.0",
                    help="arrival rates as multiples of 1/S (S: mean plain service time): below and above capacity")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-schedule", default="cache", choices=["cache", "default"],
                    help="launch schedule of the serving context: the tuning cache's for the mid parameters "
                         "in batches of 8, or the library default")
    ap.add_argument("--serve-only", action="store_true", help="skip the mid workload")
    ap.add_argument("--probe", action="store_true",
                    help="only the fp64 issue-rate probe (pir_probe_fp64): wave-instructions per CU per clock")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the batched step (no plain loop, graph replay, expansion, folklore or "
                         "arithmetic timings): the launches a counter pass attributes to each kernel family "
                         "are then the batched step's")
    return ap.parse_args()


DISTINCT_QUERIES = 8  # larger batches reuse these query ciphertexts (the work does not depend on values)


def synthetic_inputs(cfg, n, B):
    rlk = datagen.uniform_residues(cfg.primes, (cfg.L, 2), cfg.N, seed=cfg.seed * 100 + 1)
    queries = [datagen.uniform_residues(cfg.primes, (cfg.m, 2), cfg.N, seed=cfg.seed * 100 + 10 + b)
               for b in range(min(B, DISTINCT_QUERIES))]
    payload = datagen.payload(cfg, n)
    return rlk, queries, payload


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; sharding the database rows over several "
                                   "GPUs is described in the design notes but not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2202_07569_amd import Context

    if args.probe:
        cfg = datagen.CONFIGS[args.workload]
        ctx = Context(cfg.N, cfg.primes, cfg.t)
        res = {"cus": MI355X_CUS, "clock_hz": MI355X_CLOCK_HZ}
        for key, ops, fn in (("probe_fp64", Context.PROBE_OPS, ctx.probe_fp64),
                             ("probe_int", Context.PROBE_INT_OPS, ctx.probe_int)):
            rows = []
            for op, name in enumerate(ops):
                ms, wi = fn(op)
                rate = wi / (ms * 1e-3) / (MI355X_CUS * MI355X_CLOCK_HZ)
                log(f"probe {name}: {ms:.3f} ms, {rate:.3f} wave-instructions per CU per clock at 2.4 GHz, "
                    f"{wi * 64 / (ms * 1e-3) / 1e12:.1f} T lane-ops/s")
                rows.append({"op": name, "ms": ms, "wave_instructions": wi, "per_cu_per_clock": rate,
                             "lane_ops_per_s": wi * 64 / (ms * 1e-3)})
            res[key] = rows
        print(json.dumps(res), flush=True)
        return

    serve = args.serve == 1 or (args.serve == -1 and args.workload == "mid")
    if args.serve_only:
        res = serve_bench(args, torch)
        first = res["rates"][0]["batched"]
        print(json.dumps({"metric": "DB elements answered/sec + p50/p99 query latency, batched serving vs plain",
                          "value": first["elements_per_s"], "unit": "elements/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": res["workload"]}, "serving": res}), flush=True)
        return

    cfg = datagen.CONFIGS[args.workload]
    n = args.n or cfg.n
    B = max(1, args.batch)
    log(f"workload {cfg.name}: N={cfg.N} L={cfg.L} k={cfg.k} m={cfg.m} n={n} s={cfg.s} batch={B}")
    rlk, queries, payload = synthetic_inputs(cfg, n, B)

    def make_ctx(batch):
        """A context with the launch schedule for `batch` queries per call: fixed by --schedule or
        --chunk, else the package's tuning cache, else (or with --autotune 1) the autotuner."""
        c = Context(cfg.N, cfg.primes, cfg.t, chunk_elems=args.chunk)
        c.defer_relin = args.defer_relin
        tune, source = None, "default"
        cached = c.cached_schedule(batch, cfg.k, cfg.s)
        if args.schedule:
            ch, qg, rg, *sh = (int(x) for x in args.schedule.split(","))
            c.set_schedule(ch, min(qg, batch), rg, sh[0] if sh else 0)
            source = "--schedule"
        elif args.chunk:
            source = "--chunk"
        elif cached is not None and args.autotune != 1:
            c.set_schedule(cached["chunk_elems"], cached["query_group"], cached["relin_group"],
                           cached.get("ntt_shape", 0))
            source = "tuning cache"
        elif args.autotune != 0:
            tune = c.autotune(batch=batch, k=cfg.k, s=cfg.s)
            source = "autotune"
            log(f"autotune batch={batch}: {tune['best']} ({len(tune['candidates'])} candidates)")
            if args.record_schedule:
                from paper_2202_07569_amd.binding import record_schedule
                b = tune["best"]
                record_schedule(cfg.N, cfg.primes, batch, cfg.k, cfg.s,
                                {k: b[k] for k in ("chunk_elems", "query_group", "relin_group", "ntt_shape")},
                                f"pir_autotune on MI355X, {b['ns_per_elem']:.0f} ns per element-query",
                                path=args.record_schedule)
        log(f"schedule batch={batch} ({source}): {c.schedule()}")
        return c, {"source": source, "tuning": tune}

    ctx_plain, tune_plain = make_ctx(1)
    ctx, tune = make_ctx(B)
    ids = datagen.identifier_permutation(cfg, n) if not cfg.keyword else None
    if cfg.keyword:
        kws = datagen.keywords(cfg, n)
        cw = ctx.map_lossy(kws, cfg.m, cfg.k, datagen.hash_seed(cfg))
    else:
        cw = ctx.map_perfect(ids.astype(np.uint64), cfg.m, cfg.k)
    torch.cuda.synchronize()
    codewords = cw.cpu().numpy()
    key, key_plain = ctx.load_key(rlk), ctx_plain.load_key(rlk)
    db, db_plain = ctx.encode_db(codewords, payload, cfg.m), ctx_plain.encode_db(codewords, payload, cfg.m)
    dq = [torch.from_numpy(q).cuda() for q in queries]
    dq = [dq[b % len(dq)] for b in range(B)]
    outs = [ctx.empty(cfg.s, 2, cfg.L, cfg.N) for _ in range(B)]
    out_plain = ctx.empty(cfg.s, 2, cfg.L, cfg.N)
    stream = torch.cuda.current_stream()
    log(f"resident: payload {payload.nbytes / 2**20:.0f} MiB, pairs {db.pair_count}, "
        f"library HBM {ctx.device_bytes / 2**30:.2f} GiB")

    def step_plain():
        ctx_plain.answer(key_plain, db_plain, dq[0], out=out_plain, stream=stream)

    def step_batch():
        ctx.answer_batch([key] * B, [db] * B, dq, outs=outs, stream=stream)

    def timed(fn, steps, warmup, profile):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        if profile:
            ctx.profile(True)
            ctx.profile_read(reset=True)
        per = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            a = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            per.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        prof = ctx.profile_read(reset=True) if profile else {}
        ctx.profile(False)
        return total, per, prof

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calibration_mib} MiB")
        del src, dst

    graph = None
    if not args.batched_only:
        log("plain loop")
        t_plain, per_plain, _ = timed(step_plain, args.steps, args.warmup, False)
        log(f"plain {t_plain / args.steps * 1e3:.1f} ms/query")
        graph = ctx_plain.capture([key_plain], [db_plain], [dq[0]], outs=[out_plain])
        t_graph, per_graph, _ = timed(lambda: graph.launch(stream=stream), args.steps, args.warmup, False)
        log(f"plain, captured graph {t_graph / args.steps * 1e3:.1f} ms/query")
    log(f"batched B={B}")
    t_b, per_b, _ = timed(step_batch, args.steps, args.warmup, False)
    ms_step = t_b / args.steps * 1e3
    value = B * n * args.steps / t_b
    log(f"batched {ms_step:.1f} ms/step -> {value:.0f} elements/s")
    # the roofline's per-family launch times: the same step again, with HIP events around every
    # kernel family's launches on the launching stream (they add a little time of their own)
    prof, prof_steps, t_bp = {}, 0, 0.0
    if not args.no_profile:
        prof_steps = args.steps
        t_bp, _, prof = timed(step_batch, prof_steps, 1, True)
        log(f"batched with kernel-family events {t_bp / prof_steps * 1e3:.1f} ms/step")
    torch.cuda.synchronize()
    extras = not args.batched_only
    if extras and not np.array_equal(out_plain.cpu().numpy(), outs[0].cpu().numpy()):
        raise SystemExit("the batched answer of query 0 differs from the plain answer")

    expansion = expansion_bench(args, ctx, cfg, torch, stream) if extras else None
    seeded = seeded_bench(args, ctx, cfg, torch, stream) if extras else None
    folklore = folklore_bench(args, cfg, torch, stream) if extras and args.workload == "mid" else None
    arith = arith_bench(args, ctx, key, cfg, torch, stream) if extras and args.workload == "mid" else None

    fp = cfg.N <= 8192 and all(p < FP_PRIME_BOUND for p in tuple(cfg.primes) + ctx.aux_primes)
    roof = roofline(prof, prof_steps, fp, traffic_table(cfg, n, B, ctx.schedule())) if prof else None
    if roof is not None:
        roof["events_ms_per_step"] = t_bp / prof_steps * 1e3

    cpu = None
    sample = args.cpu_sample if args.cpu_sample >= 0 else (256 if cfg.N <= 8192 else 32)
    if sample:
        cpu = cpu_baseline(cfg, rlk, queries[0], codewords[:sample], payload[:sample])

    lat = lambda xs: {"p50_ms": float(np.percentile(xs, 50) * 1e3), "p99_ms": float(np.percentile(xs, 99) * 1e3)}  # noqa
    out = {
        "metric": "DB elements answered/sec (N=8192, k=4) + p50/p99 query latency, batched vs plain",
        "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if fp else "u64", "data": "synthetic",
        "config": {"workload": f"index PIR {cfg.name}: N={cfg.N}, {cfg.L} primes ({math.prod(cfg.primes).bit_length()}"
                               f" bits), t={cfg.t}, k={cfg.k}, m={cfg.m}, n={n}, s={cfg.s}",
                   "batch_queries": B},
        "schedule": {"batched": ctx.schedule(), "plain": ctx_plain.schedule(),
                     "source": {"batched": tune, "plain": tune_plain}},
        "root_keyswitch": "deferred past the inner product" if db.root_deferred else "per element",
        "plain": {"value": n * args.steps / t_plain, "unit": "elements/s", "ms_per_query": t_plain / args.steps * 1e3,
                  **lat(per_plain)} if extras else None,
        "plain_graph": {"value": n * args.steps / t_graph, "unit": "elements/s",
                        "ms_per_query": t_graph / args.steps * 1e3, **lat(per_graph)} if extras else None,
        "batched": {"value": value, "ms_per_step": ms_step, **lat(per_b)},
        "expansion": expansion,
        "seeded_query": seeded,
        "folklore": folklore,
        "arith_equality": arith,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if graph is not None:
        graph.close()
    if serve and extras:
        del graph, db, dq, outs, key, ctx, db_plain, key_plain, ctx_plain, out_plain
        torch.cuda.empty_cache()
        out["serving"] = serve_bench(args, torch)
    print(json.dumps(out), flush=True)


NTT_FAMILIES = ("ntt_fwd", "ntt_inv", "ntt_inv_tensor", "ntt_digits", "relin", "payload_ntt", "root_pm")


def traffic_table(cfg, n, B, schedule):
    """Calibrated HBM bytes per launch from the committed rocprofv3 counter summary, when it was
    taken on this workload, batch size and launch schedule and the kernel sources have not changed
    since (else None)."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    data = json.load(open(TRAFFIC_FILE))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    sched = {k: schedule.get(k, 0) for k in ("chunk_elems", "query_group", "relin_group", "ntt_shape")}
    taken = {**{"ntt_shape": 0}, **data.get("schedule", {})}
    if (data.get("kernel_source_sha256") != h.hexdigest() or data.get("workload") != cfg.name
            or data.get("n") != n or data.get("batch") != B or taken != sched):
        return None
    return dict(data["families"])


def roofline(prof, steps, fp, traffic):
    """Roofline entry of the kernel family with the largest share of the timed region.

    Transforms are ALU-bound.  Integer path: one lazy Shoup butterfly on 64-bit words takes
    MULS_PER_BUTTERFLY 32-bit multiplies; fp64 path (every prime below 2^50): FP64_OPS_PER_BUTTERFLY
    fp64 instructions.  peak = the unit's rate / that count; achieved = algorithmic butterflies of
    one launch (rows x N/2 x log2 N) / the launch's average duration from HIP events on its stream.
    Every family also gets its fraction of the butterfly roof (transform families) and, where the
    committed counter summary has its bytes per launch, its HBM rate and fraction of 8 TB/s.
    """
    name, (tot_ms, launches, work) = max(prof.items(), key=lambda kv: kv[1][0])
    avg_ms = tot_ms / launches
    fam = {k: {"ms_per_step": v[0] / steps, "launches_per_step": v[1] / steps,
               "work_per_s": (v[2] / (v[0] * 1e-3)) if v[0] else None} for k, v in sorted(prof.items())}
    bfly_peak = (MI355X_FP64_INSTR_PER_S / FP64_OPS_PER_BUTTERFLY) if fp else (MI355X_INT_MUL_PER_S / MULS_PER_BUTTERFLY)
    for k, v in fam.items():  # every family's fraction of its roof: butterflies, and HBM where counted
        if k in NTT_FAMILIES and v["work_per_s"]:
            v["alu_frac"] = v["work_per_s"] / bfly_peak
        tr = traffic.get(k, {}).get("bytes_per_launch") if traffic else None
        if tr and v["launches_per_step"]:
            gbps = tr / (v["ms_per_step"] / v["launches_per_step"] * 1e-3) / 1e9
            v.update({"hbm_GBps": gbps, "hbm_frac": gbps / MI355X_HBM_GBPS})
    out = {"kernel": name, "avg_launch_ms": avg_ms, "launches_per_step": launches / steps, "families": fam}
    if name in NTT_FAMILIES:
        per_launch = work / launches
        achieved = per_launch / (avg_ms * 1e-3)
        peak = (MI355X_FP64_INSTR_PER_S / FP64_OPS_PER_BUTTERFLY) if fp else (MI355X_INT_MUL_PER_S / MULS_PER_BUTTERFLY)
        tr = traffic.get(name, {}).get("bytes_per_launch") if traffic else None
        out.update({"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "Tbutterfly/s",
                    "frac": achieved / peak, "traffic": tr, "arith": "fp64" if fp else "int64",
                    "butterflies_per_launch": per_launch,
                    "hbm_GBps_at_traffic": (tr / (avg_ms * 1e-3) / 1e9) if tr else None})
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, rlk, query, codewords, payload):
    """The CPU oracle (plain textbook FV, OpenMP over elements) on a bounded sample, on all host
    threads and, over a smaller sample, on one thread."""
    from oracle.core import Oracle
    orc = Oracle(cfg.N, cfg.primes, cfg.t)
    key = orc.load_key(rlk)
    threads = os.cpu_count() or 1
    log(f"cpu oracle: {len(codewords)} elements on {threads} threads")
    t0 = time.perf_counter()
    orc.answer(key, query, codewords, payload, threads=threads)
    dt = time.perf_counter() - t0
    one = max(1, len(codewords) // 16)
    log(f"cpu oracle: {one} elements on one thread")
    t1 = time.perf_counter()
    orc.answer(key, query, codewords[:one], payload[:one], threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": len(codewords) / dt, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(codewords)} of {cfg.n} elements of the same workload, one query, {dt:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "one_thread": {"value": one / dt1, "unit": "elements/s",
                           "sample": f"{one} elements of the same workload, one query, {dt1:.1f} s"},
            "full_tiny": cpu_full_tiny(threads), "full_mid_recorded": full_mid_record()}


def cpu_full_tiny(threads):
    """The oracle's whole answer for the tiny index-PIR configuration (N = 4096, 3 primes, k = 2,
    m = 24, n = 256), on all host threads: synthetic key and query, the configuration's database."""
    from oracle.core import Oracle
    from oracle.mapping import perfect_map
    c = datagen.CONFIGS["tiny"]
    orc = Oracle(c.N, c.primes, c.t)
    key = orc.load_key(datagen.uniform_residues(c.primes, (c.L, 2), c.N, seed=c.seed * 100 + 1))
    q = datagen.uniform_residues(c.primes, (c.m, 2), c.N, seed=c.seed * 100 + 10)
    cw = np.array([perfect_map(int(x), c.m, c.k) for x in datagen.identifier_permutation(c, c.n)], dtype=np.uint32)
    pay = datagen.payload(c, c.n)
    log(f"cpu oracle: whole tiny answer ({c.n} elements) on {threads} threads")
    t0 = time.perf_counter()
    orc.answer(key, q, cw, pay, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": c.n / dt, "unit": "elements/s", "seconds": dt, "threads": threads,
            "workload": f"tiny: N={c.N}, {c.L} primes, k={c.k}, m={c.m}, n={c.n}, one query"}


def full_mid_record():
    """The oracle's whole mid answer (n = 16384), as timed when the golden file was written (by
    tests/golden/make_mid_answer.py, on the machine named in the record, not this host)."""
    path = os.path.join(ROOT, "tests", "golden", "mid_answer.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        secs, thr, host = float(z["oracle_seconds"]), int(z["oracle_threads"]), str(z["host"])
    return {"value": 16384 / secs, "unit": "elements/s", "seconds": secs, "threads": thr, "host": host,
            "where": "recorded when the golden answer was written, not measured in this run"}


def expansion_bench(args, ctx, cfg, torch, stream):
    """Server-side expansion (Algorithm 5) of a query packed with compression factor c (the smallest
    c with 2^c >= m, at most 5): h = ceil(m / 2^c) packed ciphertexts -> m.  Synthetic uniform
    residues stand in for the packed ciphertexts and Galois keys (the arithmetic does not depend
    on the values)."""
    c = min(5, max(0, (cfg.m - 1).bit_length()))
    h = -(-cfg.m // (1 << c))
    keys = [ctx.load_galois_key(cfg.N // (1 << a) + 1,
                                datagen.uniform_residues(cfg.primes, (cfg.L, 2), cfg.N, seed=cfg.seed * 100 + 50 + a))
            for a in range(c)]
    packed = torch.from_numpy(datagen.uniform_residues(cfg.primes, (h, 2), cfg.N, seed=cfg.seed * 100 + 60)).cuda()
    out = ctx.empty(cfg.m, 2, cfg.L, cfg.N)
    for _ in range(max(1, args.warmup)):
        ctx.expand(keys, c, packed, cfg.m, out=out, stream=stream)
    torch.cuda.synchronize()
    per = []
    for _ in range(max(3, args.steps)):
        a = time.perf_counter()
        ctx.expand(keys, c, packed, cfg.m, out=out, stream=stream)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - a)
    for k in keys:
        k.close()
    log(f"expansion c={c} h={h} m={cfg.m}: {np.median(per) * 1e3:.2f} ms")
    return {"c": c, "packed_ciphertexts": h, "m": cfg.m, "substitutions": h * ((1 << c) - 1),
            "ms_median": float(np.median(per) * 1e3), "ms_p99": float(np.percentile(per, 99) * 1e3)}


def seeded_bench(args, ctx, cfg, torch, stream):
    """Rebuild of a seeded c = 0 query (m ciphertexts: c0 uploaded, a regenerated from the seed)
    and the upload sizes of the query forms (64-bit residues; a seed is 8 bytes)."""
    c0 = torch.from_numpy(datagen.uniform_residues(cfg.primes, (cfg.m,), cfg.N, seed=cfg.seed * 100 + 70)).cuda()
    out = ctx.empty(cfg.m, 2, cfg.L, cfg.N)
    for _ in range(max(1, args.warmup)):
        ctx.seeded_query(c0, 12345, out=out, stream=stream)
    torch.cuda.synchronize()
    per = []
    for _ in range(max(3, args.steps)):
        a = time.perf_counter()
        ctx.seeded_query(c0, 12345, out=out, stream=stream)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - a)
    poly = cfg.L * cfg.N * 8
    c = min(5, max(0, (cfg.m - 1).bit_length()))
    h = -(-cfg.m // (1 << c))
    log(f"seeded query rebuild m={cfg.m}: {np.median(per) * 1e3:.3f} ms")
    return {"m": cfg.m, "ms_median": float(np.median(per) * 1e3),
            "upload_bytes": {"query": cfg.m * 2 * poly, "seeded_query": cfg.m * poly + 8,
                             f"packed_c{c}": h * 2 * poly, f"seeded_packed_c{c}": h * poly + 8}}


def arith_bench(args, ctx, key, cfg, torch, stream, m=37, k=4):
    """Arithmetic constant-weight equality (Algorithm 2) on batch-encoded ciphertexts: N comparisons
    per evaluation, for the paper's n = 2^16, k = 4 row (code length m = 37).  Synthetic uniform
    residues stand in for the two encrypted codewords."""
    x = torch.from_numpy(datagen.uniform_residues(cfg.primes, (m, 2), cfg.N, seed=cfg.seed * 100 + 80)).cuda()
    y = torch.from_numpy(datagen.uniform_residues(cfg.primes, (m, 2), cfg.N, seed=cfg.seed * 100 + 81)).cuda()
    out = ctx.empty(2, cfg.L, cfg.N)
    for _ in range(max(1, args.warmup)):
        ctx.arith_equality(key, x, y, k, out=out, stream=stream)
    per = []
    for _ in range(max(3, args.steps)):
        a = time.perf_counter()
        ctx.arith_equality(key, x, y, k, out=out, stream=stream)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - a)
    t = float(np.median(per))
    log(f"arithmetic equality m={m} k={k}: {t * 1e3:.2f} ms per {cfg.N} comparisons")
    return {"m": m, "k": k, "slots": cfg.N, "ms_per_evaluation": t * 1e3, "comparisons_per_s": cfg.N / t}


def folklore_bench(args, cfg, torch, stream):
    """Folklore PIR (plain folklore operator) on the same parameters and database size: the query is
    the l = ceil(log2 n) index bits, the server forms the 2l leaves (1 - x_i, x_i) and evaluates the
    depth-ceil(log2 l) product per element with the memoised tree.  One query at a time."""
    from paper_2202_07569_amd import Context
    n = cfg.n
    ell = max(1, (n - 1).bit_length())
    j = np.arange(n, dtype=np.uint64)[:, None]
    i = np.arange(ell, dtype=np.uint64)[None, :]
    cw = (2 * i + ((j >> i) & np.uint64(1))).astype(np.uint32)  # leaf 2i + bit_i(j)
    ctx = Context(cfg.N, cfg.primes, cfg.t)
    key = ctx.load_key(datagen.uniform_residues(cfg.primes, (cfg.L, 2), cfg.N, seed=cfg.seed * 100 + 70))
    db = ctx.encode_db(cw, datagen.payload(cfg, n), 2 * ell)
    q = torch.from_numpy(datagen.uniform_residues(cfg.primes, (ell, 2), cfg.N, seed=cfg.seed * 100 + 71)).cuda()
    out = ctx.empty(cfg.s, 2, cfg.L, cfg.N)

    def one():
        ctx.answer(key, db, ctx.folklore_leaves(q, stream=stream), out=out, stream=stream)

    for _ in range(max(1, args.warmup)):
        one()
    torch.cuda.synchronize()
    per = []
    for _ in range(max(3, args.steps)):
        a = time.perf_counter()
        one()
        torch.cuda.synchronize()
        per.append(time.perf_counter() - a)
    t = float(np.median(per))
    log(f"folklore l={ell} (k={ell}, {db.pair_count} shared nodes): {t * 1e3:.1f} ms/query -> {n / t:.0f} elements/s")
    res = {"ell": ell, "shared_nodes": db.pair_count, "ms_per_query": t * 1e3, "elements_per_s": n / t,
           "p99_ms": float(np.percentile(per, 99) * 1e3)}
    db.close()
    key.close()
    return res


# --------------------------------------------------------------------------------------------
# Batched serving: four resident databases, Poisson arrivals, plain loop vs continuous batching
# --------------------------------------------------------------------------------------------
QUERY_POOL = 4  # distinct synthetic query ciphertexts per database, reused round-robin


def serve_bench(args, torch):
    """Replay one seeded arrival trace through (i) the plain loop, which answers one query at a time
    in arrival order with pir_answer, and (ii) the continuous-batching server (pir_serve_*) under
    its three policies (round robin, oldest first, size aged).

    Latency runs from a query's arrival (host clock) to its answer being complete on the device,
    and includes the upload of its ciphertexts: the client's query sits in pinned host memory until
    it arrives, and is then copied to a device buffer of its own and submitted (plain loop: copied
    and answered).  Elements/s = sum of the queried databases' sizes / time from the first arrival
    to the last completion.  The rate is a multiple of 1/S, S the plain loop's mean service time
    (query resident) over the uniform database mix, measured first.
    """
    from paper_2202_07569_amd import Context, Server
    cfgs = datagen.batched_configs()
    c0 = cfgs[0]
    ctx = Context(c0.N, c0.primes, c0.t, hbm_budget_bytes=96 << 30)
    # the launch schedule the tuning cache holds for these parameters in batches of 8 (the plain
    # loop and the server share the context, so both run it)
    cached = ctx.cached_schedule(8, 4, 1)
    if cached is not None and args.serve_schedule == "cache":
        ctx.set_schedule(cached["chunk_elems"], cached["query_group"], cached["relin_group"],
                         cached.get("ntt_shape", 0))
    log(f"serving schedule ({args.serve_schedule}): {ctx.schedule()}")
    keys = [ctx.load_key(datagen.uniform_residues(c0.primes, (c0.L, 2), c0.N, seed=c0.seed * 100 + 1 + i))
            for i in range(2)]
    dbs, pools = [], []
    for c in cfgs:
        log(f"serving db {c.name}: n={c.n} s={c.s} k={c.k} m={c.m}")
        cw = ctx.map_perfect(datagen.identifier_permutation(c).astype(np.uint64), c.m, c.k)
        torch.cuda.synchronize()
        pay = datagen.payload(c)
        dbs.append(ctx.encode_db(cw.cpu().numpy(), pay, c.m))
        del pay
        pools.append([torch.from_numpy(datagen.uniform_residues(c.primes, (c.m, 2), c.N,
                                                                seed=c.seed * 100 + 20 + i)).pin_memory()
                      for i in range(QUERY_POOL)])
    resident = [[q.cuda() for q in pool] for pool in pools]  # for the service-time measurement
    stream = torch.cuda.current_stream()
    Q = args.serve_queries
    seed = cfgs[0].seed
    dbc = datagen.uniform_choice(seed, datagen.S_DBCHOICE, Q, len(cfgs))
    keyc = np.arange(Q) % len(keys)
    outs = [ctx.empty(cfgs[d].s, 2, c0.L, c0.N) for d in dbc]
    elems = float(sum(cfgs[d].n for d in dbc))

    # S: plain service time per database (after a warm-up answer on each)
    svc = []
    for d, c in enumerate(cfgs):
        ctx.answer(keys[0], dbs[d], resident[d][0], out=outs[0] if dbc[0] == d else ctx.empty(c.s, 2, c0.L, c0.N))
        torch.cuda.synchronize()
        reps = []
        for r in range(3):
            a = time.perf_counter()
            ctx.answer(keys[r % 2], dbs[d], resident[d][r % QUERY_POOL], out=ctx.empty(c.s, 2, c0.L, c0.N))
            torch.cuda.synchronize()
            reps.append(time.perf_counter() - a)
        svc.append(float(np.median(reps)))
    del resident
    S = float(np.mean(svc))
    log(f"plain service times {[round(x * 1e3, 1) for x in svc]} ms, S = {S * 1e3:.1f} ms")
    # size-aged order: priority = arrival + aging * elements, aging twice the plain cost per element
    aging = 2.0 * float(np.mean([svc[d] / cfgs[d].n for d in range(len(cfgs))])) * 1e9

    def plain(arr):
        lat = np.zeros(Q)
        t0 = time.perf_counter()
        done = 0.0
        for i in range(Q):
            now = time.perf_counter() - t0
            if now < arr[i]:
                time.sleep(arr[i] - now)
            d = dbc[i]
            q = pools[d][i % QUERY_POOL].to(ctx.device, non_blocking=True)  # the upload, on `stream`
            ctx.answer(keys[keyc[i]], dbs[d], q, out=outs[i], stream=stream)
            stream.synchronize()
            del q
            done = time.perf_counter() - t0
            lat[i] = done - arr[i]
        return lat, done - arr[0]

    def batched(arr, policy=Server.ROUND_ROBIN, aging=0.0):
        srv = Server(ctx, max_slots=args.serve_slots, policy=policy, aging_ns_per_element=aging)
        lat = np.zeros(Q)
        live = {}
        i = nd = 0
        t0 = time.perf_counter()
        done = 0.0
        while nd < Q:
            now = time.perf_counter() - t0
            while i < Q and arr[i] <= now:
                d = dbc[i]
                q = pools[d][i % QUERY_POOL].to(ctx.device, non_blocking=True)  # upload; submit waits for it
                live[srv.submit(keys[keyc[i]], dbs[d], q, out=outs[i])] = i
                i += 1
            if not live:
                time.sleep(max(0.0, arr[i] - (time.perf_counter() - t0)))
                continue
            busy = srv.step()
            for t in [t for t in live if srv.poll(t)]:
                done = time.perf_counter() - t0
                j = live.pop(t)
                lat[j] = done - arr[j]
                srv.result(t)
                nd += 1
            if busy == 0 and live:
                time.sleep(2e-4)  # only completion events outstanding
        st = srv.stats()
        srv.close()
        return lat, done - arr[0], st

    res = {"workload": "batched serving: 4 resident databases (n, s, k) = "
                       + ", ".join(f"({c.n}, {c.s}, {c.k})" for c in cfgs)
                       + f"; N={c0.N}, {c0.L} primes, t={c0.t}; {Q} queries, uniform database choice, "
                         f"{len(keys)} keys",
           "plain_service_ms": [x * 1e3 for x in svc], "S_ms": S * 1e3, "slots": args.serve_slots,
           "schedule": {k: v for k, v in ctx.schedule().items() if k != "ns_per_elem"}, "rates": []}
    for mult in [float(x) for x in args.serve_rates.split(",")]:
        rate = mult / S
        arr = datagen.poisson_arrivals(seed + int(mult * 1000), Q, rate)
        arr = arr - arr[0]
        log(f"rate {mult}/S: plain loop")
        lp, tp = plain(arr)
        log(f"rate {mult}/S: continuous batching")
        lb, tb, st = batched(arr)
        log(f"rate {mult}/S: continuous batching, oldest first")
        lf, tf, stf = batched(arr, Server.OLDEST_FIRST)
        log(f"rate {mult}/S: size-aged order, aging {aging:.0f} ns per element")
        lg, tg, stg = batched(arr, Server.SIZE_AGED, aging)
        pct = lambda x: {"p50_ms": float(np.percentile(x, 50) * 1e3),  # noqa: E731
                         "p99_ms": float(np.percentile(x, 99) * 1e3), "mean_ms": float(x.mean() * 1e3)}
        entry = {"rate_per_s": rate, "rate_over_S": mult,
                 "plain": {"elements_per_s": elems / tp, "wall_s": tp, **pct(lp)},
                 "batched": {"elements_per_s": elems / tb, "wall_s": tb, **pct(lb), "rounds": st["rounds"]},
                 "batched_oldest_first": {"elements_per_s": elems / tf, "wall_s": tf, **pct(lf),
                                          "rounds": stf["rounds"]},
                 "size_aged": {"elements_per_s": elems / tg, "wall_s": tg, **pct(lg), "rounds": stg["rounds"],
                               "aging_ns_per_element": aging}}
        log(f"rate {mult}/S: plain {entry['plain']['elements_per_s']:.0f} el/s p50 {entry['plain']['p50_ms']:.0f} "
            f"p99 {entry['plain']['p99_ms']:.0f} ms | batched {entry['batched']['elements_per_s']:.0f} el/s "
            f"p50 {entry['batched']['p50_ms']:.0f} p99 {entry['batched']['p99_ms']:.0f} ms | oldest first "
            f"{entry['batched_oldest_first']['elements_per_s']:.0f} el/s p50 {entry['batched_oldest_first']['p50_ms']:.0f} "
            f"p99 {entry['batched_oldest_first']['p99_ms']:.0f} ms | size aged {entry['size_aged']['elements_per_s']:.0f} "
            f"el/s p50 {entry['size_aged']['p50_ms']:.0f} p99 {entry['size_aged']['p99_ms']:.0f} ms")
        res["rates"].append(entry)
    return res


# --------------------------------------------------------------------------------------------
# Counter summary: rocprofv3 FETCH_SIZE / WRITE_SIZE passes -> calibrated HBM bytes per launch
# --------------------------------------------------------------------------------------------
FAMILY_OF_KERNEL = [("k_relin", "relin"), ("k_ntt_inv_tensor", "ntt_inv_tensor"), ("k_scale_fix", None),
                    ("k_scale", "scale"), ("k_accumulate", "accumulate"), ("k_ntt_payload", "payload_ntt"),
                    ("k_root_pm", "root_pm"), ("k_root_reduce", "root_reduce"), ("copyBuffer", "copy")]


def summarize_traffic(fetch_csv, write_csv, copy_mib, workload, n, batch, schedule, out_json):
    """Per kernel family and grid size: average FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each
    scaled by the factor that makes the same counter read the known size of the plain device copy
    kernels of the run (copy_mib MiB per copy, split over its dispatches), for the grid size with
    the most dispatches of each family."""
    import collections
    import csv
    import hashlib

    def family(name):
        for key, fam in FAMILY_OF_KERNEL:
            if key in name:
                return fam
        return None

    def per_dispatch(path, counter):
        vals = collections.defaultdict(float)
        meta = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            fam = family(r["Kernel_Name"])
            if fam:
                d = r["Dispatch_Id"]
                vals[d] += float(r["Counter_Value"])
                meta[d] = (fam, int(r["Grid_Size"]))
        groups = collections.defaultdict(list)
        for d, v in vals.items():
            groups[meta[d]].append(v)
        return groups

    fetch, write = per_dispatch(fetch_csv, "FETCH_SIZE"), per_dispatch(write_csv, "WRITE_SIZE")

    def calib(groups):  # the run's three copies of copy_mib MiB are its three largest copy dispatches
        top = sorted((v for k, vs in groups.items() if k[0] == "copy" for v in vs), reverse=True)[:3]
        return copy_mib * 1024 / (sum(top) / 3)

    f_factor, w_factor, ncopy = calib(fetch), calib(write), 3
    fams = {}
    for fam in sorted({k[0] for k in fetch if k[0] != "copy"}):
        grid = max((k for k in fetch if k[0] == fam), key=lambda k: len(fetch[k]))
        fk = sum(fetch[grid]) / len(fetch[grid])
        wk = sum(write.get(grid, [0.0])) / max(1, len(write.get(grid, [])))
        fams[fam] = {"grid_size": grid[1], "dispatches": len(fetch[grid]), "fetch_kib_raw": fk, "write_kib_raw": wk,
                     "bytes_per_launch": (fk * f_factor + wk * w_factor) * 1024}
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    data = {"kernel_source_sha256": h.hexdigest(), "workload": workload, "n": n, "batch": batch,
            "schedule": schedule, "fetch_factor": f_factor, "write_factor": w_factor, "families": fams}
    with open(out_json, "w") as f:
        json.dump(data, f, indent=1)
    print(f"calibration: fetch x{f_factor:.3f}, write x{w_factor:.3f} ({ncopy} copy dispatches)")
    print("| Kernel family | Grid | Dispatches | FETCH_SIZE KiB/dispatch (raw) | WRITE_SIZE KiB/dispatch (raw) "
          "| HBM MB/launch (calibrated) |")
    print("|---|---|---|---|---|---|")
    for fam, v in fams.items():
        print(f"| `{fam}` | {v['grid_size']} | {v['dispatches']} | {v['fetch_kib_raw']:,.0f} | {v['write_kib_raw']:,.0f} "
              f"| {v['bytes_per_launch'] / 1e6:,.0f} |")


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-traffic":
        # bench.py --summarize-traffic FETCH_CSV WRITE_CSV COPY_MIB WORKLOAD N BATCH CHUNK,QG,RG[,SHAPE] OUT_JSON
        a = sys.argv[2:]
        ch, qg, rg, *sh = (int(x) for x in a[6].split(","))
        summarize_traffic(a[0], a[1], int(a[2]), a[3], int(a[4]), int(a[5]),
                          {"chunk_elems": ch, "query_group": qg, "relin_group": rg, "ntt_shape": sh[0] if sh else 0},
                          a[7])
    else:
        main()
