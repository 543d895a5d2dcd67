"""Host-side checks of the HIP library that need no GPU: it loads, exports every declared entry
point, and rejects unsupported parameters before touching a device."""
import ctypes
import os
import re

import pytest

import datagen
from paper_2202_07569_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:[\w\*]+\s+)+\**(pir_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == declared


def _setup(N, primes, t=65537, chunk=0):
    q = (ctypes.c_uint64 * len(primes))(*primes)
    p = binding._Params(N, len(primes), q, t, 0, 0, chunk, 0)
    h = ctypes.c_void_p()
    rc = binding.lib().pir_setup(ctypes.byref(p), ctypes.byref(h))
    return rc, binding.lib().pir_last_error().decode()


@pytest.mark.parametrize("N,primes,t,code,text", [
    (2048, datagen.Q_N4096, 65537, binding.PIR_E_UNSUPPORTED, "N must be"),
    (4096, (), 65537, binding.PIR_E_UNSUPPORTED, "L out of range"),
    (4096, datagen.Q_N4096[:2] + (datagen.Q_N4096[0],), 65537, binding.PIR_E_INVALID, "distinct"),
    (4096, (0xffffee001 + 8192,), 65537, binding.PIR_E_INVALID, "not prime"),
    (8192, datagen.Q_N4096, 65537, binding.PIR_E_INVALID, "1 mod 2N"),
    (4096, ((1 << 61) + 1,), 65537, binding.PIR_E_INVALID, "(2^30, 2^61)"),
    (4096, datagen.Q_N4096, 1, binding.PIR_E_INVALID, "t must be"),
])
def test_setup_rejects_bad_parameters(N, primes, t, code, text):
    rc, msg = _setup(N, primes, t)
    assert rc == code and text in msg


def test_setup_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, msg = _setup(4096, datagen.Q_N4096)
    assert rc == binding.PIR_E_DEVICE and "device" in msg


def test_context_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(binding.PirError):
        binding.Context(4096, datagen.Q_N4096)


def test_serving_calls_reject_null_server():
    L = binding.lib()
    t = ctypes.c_uint64()
    assert L.pir_serve_step(None) == binding.PIR_E_INVALID
    assert L.pir_serve_poll(None, 1) == binding.PIR_E_INVALID
    assert L.pir_serve_submit(None, None, None, None, None, ctypes.byref(t)) == binding.PIR_E_INVALID
    assert L.pir_serve_stats(None, None, None, None, None, None) == binding.PIR_E_INVALID
    assert "null server" in L.pir_last_error().decode()
    L.pir_serve_close(None)  # no-op


def test_schedule_calls_reject_null_context():
    L = binding.lib()
    s = binding._Schedule(64, 2, 0, 0, 0.0)
    assert L.pir_get_schedule(None, ctypes.byref(s)) == binding.PIR_E_INVALID
    assert L.pir_set_schedule(None, ctypes.byref(s)) == binding.PIR_E_INVALID
    assert L.pir_autotune(None, 1, 2, 1, None, 0, None) == binding.PIR_E_INVALID
    assert "null context" in L.pir_last_error().decode()
    st = (ctypes.c_uint32 * 8)()
    assert L.pir_ntt_shape_count(None) == 0
    assert L.pir_db_root_deferred(None) == 0
    assert L.pir_ntt_shape_stages(None, 0, st) == 0


def test_seeded_query_rejects_null_context():
    L = binding.lib()
    assert L.pir_seeded_query(None, None, 1, 7, None, None) == binding.PIR_E_INVALID
    assert "null context" in L.pir_last_error().decode()


def test_schedule_cache_round_trip(tmp_path):
    from paper_2202_07569_amd.binding import lookup_schedule, record_schedule
    path = str(tmp_path / "cache.json")
    primes = (0x7fffffd8001, 0x7fffffc8001)
    assert lookup_schedule(8192, primes, 8, 4, 1, path=path) is None
    a = {"chunk_elems": 512, "query_group": 1, "relin_group": 0}
    b = {"chunk_elems": 256, "query_group": 2, "relin_group": 32}
    record_schedule(8192, primes, 8, 4, 1, a, "first", path=path)
    record_schedule(8192, primes, 1, 4, 1, b, "batch 1", path=path)
    assert lookup_schedule(8192, primes, 8, 4, 1, path=path) == a
    assert lookup_schedule(8192, primes, 1, 4, 1, path=path) == b
    assert lookup_schedule(8192, primes, 8, 2, 1, path=path) is None        # other k
    assert lookup_schedule(8192, primes[::-1], 8, 4, 1, path=path) is None  # other prime order
    record_schedule(8192, primes, 8, 4, 1, b, "replaced", path=path)        # replaces, no duplicate
    assert lookup_schedule(8192, primes, 8, 4, 1, path=path) == b
    import json
    assert len(json.load(open(path))["entries"]) == 2


def test_package_tuning_cache_is_well_formed():
    import json
    from paper_2202_07569_amd.binding import SCHEDULE_CACHE
    for e in json.load(open(SCHEDULE_CACHE))["entries"]:
        sch = e["schedule"]
        assert 1 <= sch["chunk_elems"] <= 4096 and 1 <= sch["query_group"] <= 8 and sch["relin_group"] >= 0
        assert 0 <= sch.get("ntt_shape", 0) < {4096: 1, 8192: 3, 16384: 2}[e["N"]]
        assert all(p % (2 * e["N"]) == 1 for p in e["primes"])


def test_serving_aging_rejects_null_server():
    L = binding.lib()
    assert L.pir_serve_set_aging(None, 1.0) == binding.PIR_E_INVALID
    assert "null server" in L.pir_last_error().decode()


def test_probe_rejects_null_context():
    L = binding.lib()
    ms, wi = ctypes.c_double(), ctypes.c_double()
    assert L.pir_probe_fp64(None, 0, 1, 1, ctypes.byref(ms), ctypes.byref(wi), None) == binding.PIR_E_INVALID
