"""Python binding of libcwpir (include/cwpir.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels.  PyTorch supplies device memory and
streams: device buffers are torch tensors on the context's device (uint64 residues, uint16
payloads), and asynchronous calls run on torch's current stream unless one is given.  There is
no CPU fallback: without the built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

PIR_OK, PIR_E_INVALID, PIR_E_NOMEM, PIR_E_DEVICE, PIR_E_BUSY, PIR_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5

EXPORTS = [
    "pir_setup", "pir_load_key", "pir_encode_db", "pir_answer", "pir_answer_batch", "pir_mult", "pir_relin",
    "pir_pm", "pir_selectors", "pir_map_perfect", "pir_map_lossy", "pir_ctx_aux_primes", "pir_ctx_device_bytes",
    "pir_db_pair_count", "pir_profile_enable", "pir_profile_read", "pir_db_free", "pir_key_free", "pir_free",
    "pir_last_error", "pir_serve_open", "pir_serve_submit", "pir_serve_step", "pir_serve_poll", "pir_serve_stats",
    "pir_serve_close", "pir_get_schedule", "pir_set_schedule", "pir_autotune", "pir_graph_capture",
    "pir_graph_launch", "pir_graph_free", "pir_load_galois_key", "pir_expand", "pir_mod_switch",
    "pir_folklore_leaves", "pir_arith_equality", "pir_serve_set_policy", "pir_seeded_query",
    "pir_serve_set_aging", "pir_probe_fp64", "pir_mod_switch_noalloc", "pir_check_query", "pir_probe_int",
    "pir_set_defer_relin", "pir_get_defer_relin", "pir_ntt_shape_count", "pir_ntt_shape_stages",
    "pir_db_root_deferred",
]


class PirError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cwpir error {code}: {msg}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("L", ctypes.c_uint32), ("q", ctypes.POINTER(ctypes.c_uint64)),
                ("t", ctypes.c_uint64), ("hbm_budget_bytes", ctypes.c_uint64), ("device", ctypes.c_int32),
                ("chunk_elems", ctypes.c_uint32), ("memo_bytes", ctypes.c_uint64)]


class _Schedule(ctypes.Structure):
    _fields_ = [("chunk_elems", ctypes.c_uint32), ("query_group", ctypes.c_uint32), ("relin_group", ctypes.c_uint32),
                ("ntt_shape", ctypes.c_uint32), ("ns_per_elem", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {"chunk_elems": self.chunk_elems, "query_group": self.query_group, "relin_group": self.relin_group,
                "ntt_shape": self.ntt_shape, "ns_per_elem": self.ns_per_elem}


_lib = None


def library_path() -> str:
    return _build.LIB


def lib():
    """Load the built library (building it first only when nothing is built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        pp = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "pir_setup": (i32, [ctypes.POINTER(_Params), pp]),
            "pir_load_key": (i32, [vp, vp, pp]),
            "pir_encode_db": (i32, [vp, u64, u32, u32, u32, vp, vp, pp]),
            "pir_answer": (i32, [vp, vp, vp, vp, vp, vp]),
            "pir_answer_batch": (i32, [vp, u32, pp, pp, pp, pp, vp]),
            "pir_mult": (i32, [vp, vp, vp, vp, vp]),
            "pir_relin": (i32, [vp, vp, vp, vp, vp]),
            "pir_pm": (i32, [vp, vp, vp, vp, vp]),
            "pir_selectors": (i32, [vp, vp, vp, vp, vp, u32, vp, vp]),
            "pir_map_perfect": (i32, [vp, vp, u64, u32, u32, vp, vp]),
            "pir_map_lossy": (i32, [vp, vp, u64, u32, u32, u64, vp, vp]),
            "pir_ctx_aux_primes": (u32, [vp, vp]),
            "pir_ctx_device_bytes": (u64, [vp]),
            "pir_db_pair_count": (u64, [vp]),
            "pir_db_root_deferred": (i32, [vp]),
            "pir_ntt_shape_count": (u32, [vp]),
            "pir_ntt_shape_stages": (u32, [vp, u32, ctypes.POINTER(ctypes.c_uint32)]),
            "pir_profile_enable": (i32, [vp, i32]),
            "pir_profile_read": (i32, [vp, u32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double), i32]),
            "pir_db_free": (None, [vp]),
            "pir_key_free": (None, [vp]),
            "pir_free": (None, [vp]),
            "pir_last_error": (ctypes.c_char_p, []),
            "pir_serve_open": (i32, [vp, u32, pp]),
            "pir_serve_submit": (i32, [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)]),
            "pir_serve_step": (i32, [vp]),
            "pir_serve_poll": (i32, [vp, u64]),
            "pir_serve_stats": (i32, [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_uint32)]),
            "pir_serve_close": (None, [vp]),
            "pir_get_schedule": (i32, [vp, ctypes.POINTER(_Schedule)]),
            "pir_set_schedule": (i32, [vp, ctypes.POINTER(_Schedule)]),
            "pir_autotune": (i32, [vp, u32, u32, u32, ctypes.POINTER(_Schedule), u32, ctypes.POINTER(_Schedule)]),
            "pir_graph_capture": (i32, [vp, u32, pp, pp, pp, pp, pp]),
            "pir_graph_launch": (i32, [vp, vp]),
            "pir_graph_free": (None, [vp]),
            "pir_load_galois_key": (i32, [vp, u32, vp, pp]),
            "pir_expand": (i32, [vp, pp, u32, vp, u32, u32, vp, vp]),
            "pir_mod_switch": (i32, [vp, vp, u32, u32, vp, vp]),
            "pir_mod_switch_noalloc": (i32, [vp, vp, u32, u32, vp, vp]),
            "pir_check_query": (i32, [vp, vp, u32, vp]),
            "pir_set_defer_relin": (i32, [vp, i32]),
            "pir_get_defer_relin": (i32, [vp]),
            "pir_folklore_leaves": (i32, [vp, vp, u32, vp, vp]),
            "pir_arith_equality": (i32, [vp, vp, vp, vp, u32, u32, vp, vp]),
            "pir_serve_set_policy": (i32, [vp, i32]),
            "pir_seeded_query": (i32, [vp, vp, u32, ctypes.c_uint64, vp, vp]),
            "pir_serve_set_aging": (i32, [vp, ctypes.c_double]),
            "pir_probe_fp64": (i32, [vp, i32, u32, u32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), vp]),
            "pir_probe_int": (i32, [vp, i32, u32, u32, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PIR_OK:
        raise PirError(rc, lib().pir_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream, *tensors):
    """HIP stream handle for an asynchronous call on `stream` (default: torch's current stream of
    the tensors' device).  Inputs the binding copied to the device and outputs it allocated belong
    to torch's current stream; on another stream the call first waits for the current stream's
    queued work, and the tensors are marked as used by that stream, so that torch's caching
    allocator does not hand their memory to other work before the call has run."""
    torch = _torch()
    dev = tensors[0].device if tensors else None
    cur = torch.cuda.current_stream(dev)
    if stream is None:
        return ctypes.c_void_p(cur.cuda_stream)
    s = torch.cuda.ExternalStream(stream, device=dev) if isinstance(stream, int) else stream
    if s.cuda_stream != cur.cuda_stream:
        s.wait_stream(cur)
        for t in tensors:
            t.record_stream(s)
    return ctypes.c_void_p(s.cuda_stream)


def _dev_u64(x, device):
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint64))
    if x.dtype != torch.uint64:
        raise TypeError("expected uint64 residues")
    x = x.to(device).contiguous()
    return x


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Key:
    def __init__(self, ctx: "Context", handle):
        self.ctx, self._h = ctx, handle

    def close(self):
        if self._h:
            lib().pir_key_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Database:
    def __init__(self, ctx: "Context", handle, n, s, m, k):
        self.ctx, self._h = ctx, handle
        self.n, self.s, self.m, self.k = n, s, m, k

    @property
    def pair_count(self) -> int:
        return lib().pir_db_pair_count(self._h)

    @property
    def root_deferred(self) -> bool:
        """Whether answers relinearize the root products after the inner product
        (pir_db_root_deferred)."""
        return bool(lib().pir_db_root_deferred(self._h))

    def close(self):
        if self._h:
            lib().pir_db_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One FV parameter set on one device (pir_setup)."""

    def __init__(self, N: int, primes, t: int = 65537, hbm_budget_bytes: int = 0, device: int = 0,
                 chunk_elems: int = 0, memo_bytes: int = 0):
        torch = _torch()
        if not torch.cuda.is_available():
            raise PirError(PIR_E_DEVICE, "no GPU visible to torch")
        self.N, self.t, self.primes = int(N), int(t), tuple(int(p) for p in primes)
        self.L = len(self.primes)
        self.device = torch.device("cuda", device)
        q = (ctypes.c_uint64 * self.L)(*self.primes)
        p = _Params(self.N, self.L, q, self.t, hbm_budget_bytes, device, chunk_elems, memo_bytes)
        h = ctypes.c_void_p()
        _check(lib().pir_setup(ctypes.byref(p), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().pir_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def aux_primes(self) -> tuple:
        n = lib().pir_ctx_aux_primes(self._h, None)
        out = (ctypes.c_uint64 * n)()
        lib().pir_ctx_aux_primes(self._h, out)
        return tuple(out)

    @property
    def device_bytes(self) -> int:
        return lib().pir_ctx_device_bytes(self._h)

    def schedule(self) -> dict:
        out = _Schedule()
        _check(lib().pir_get_schedule(self._h, ctypes.byref(out)))
        return out.as_dict()

    @property
    def defer_relin(self) -> int:
        """When root products are relinearized after the inner product (pir_set_defer_relin):
        0 never, 1 where it pays (default), 2 wherever allowed."""
        rc = lib().pir_get_defer_relin(self._h)
        if rc < 0:
            _check(rc)
        return rc

    @defer_relin.setter
    def defer_relin(self, mode: int):
        _check(lib().pir_set_defer_relin(self._h, int(mode)))

    def set_schedule(self, chunk_elems: int, query_group: int, relin_group: int = 0, ntt_shape: int = 0):
        x = _Schedule(chunk_elems, query_group, relin_group, ntt_shape, 0.0)
        _check(lib().pir_set_schedule(self._h, ctypes.byref(x)))

    def ntt_shapes(self) -> list:
        """Stage counts of the passes of every transform shape variant of this ring degree
        (pir_ntt_shape_count / pir_ntt_shape_stages)."""
        out = []
        for v in range(lib().pir_ntt_shape_count(self._h)):
            st = (ctypes.c_uint32 * 8)()
            npass = lib().pir_ntt_shape_stages(self._h, v, st)
            out.append([int(st[i]) for i in range(npass)])
        return out

    def autotune(self, batch: int = 8, k: int = 4, s: int = 1) -> dict:
        """Time candidate launch schedules on synthetic inputs and apply the fastest (before any
        database is encoded).  Returns {"best": schedule, "candidates": [schedule, ...]}."""
        recs = (_Schedule * 64)()
        best = _Schedule()
        rc = lib().pir_autotune(self._h, batch, k, s, recs, 64, ctypes.byref(best))
        if rc < 0:
            _check(rc)
        return {"best": best.as_dict(), "candidates": [recs[i].as_dict() for i in range(min(rc, 64))]}

    def cached_schedule(self, batch: int, k: int, s: int):
        """The schedule the autotuner chose earlier for these parameters and call shape, from the
        package's tuning cache (schedules.json), or None."""
        return lookup_schedule(self.N, self.primes, batch, k, s)

    def empty(self, *shape, dtype=None):
        torch = _torch()
        return torch.empty(shape, dtype=dtype or torch.uint64, device=self.device)

    # ---- Setup ----
    def load_galois_key(self, g: int, gk) -> Key:
        gk = _dev_u64(gk, self.device)
        assert tuple(gk.shape) == (self.L, 2, self.L, self.N)
        h = ctypes.c_void_p()
        _check(lib().pir_load_galois_key(self._h, int(g), _ptr(gk), ctypes.byref(h)))
        return Key(self, h)

    def expand(self, gkeys, c: int, packed, m: int, out=None, stream=None):
        """Algorithm 5: packed [h][2][L][N] -> query [m][2][L][N]; gkeys[a] for g = N/2^a + 1."""
        packed = _dev_u64(packed, self.device)
        h = packed.shape[0]
        if out is None:
            out = self.empty(m, 2, self.L, self.N)
        arr = (ctypes.c_void_p * max(1, c))(*([k._h.value for k in gkeys[:c]] or [None]))
        _check(lib().pir_expand(self._h, arr, c, _ptr(packed), h, m, _ptr(out), _stream(stream, packed, out)))
        return out

    def arith_equality(self, key: Key, x, y, k: int, out=None, stream=None):
        """Algorithm 2: encrypted codewords x, y [m][2][L][N] of weight k -> e [2][L][N] (synchronous)."""
        x, y = _dev_u64(x, self.device), _dev_u64(y, self.device)
        assert x.shape == y.shape and tuple(x.shape[1:]) == (2, self.L, self.N)
        if out is None:
            out = self.empty(2, self.L, self.N)
        _check(lib().pir_arith_equality(self._h, key._h, _ptr(x), _ptr(y), x.shape[0], k, _ptr(out),
                                        _stream(stream, x, y, out)))
        return out

    def folklore_leaves(self, query, out=None, stream=None):
        """Folklore PIR: the l query bits [l][2][L][N] -> the 2l leaves (1 - x_i, x_i)."""
        query = _dev_u64(query, self.device)
        ell = query.shape[0]
        if out is None:
            out = self.empty(2 * ell, 2, self.L, self.N)
        _check(lib().pir_folklore_leaves(self._h, _ptr(query), ell, _ptr(out), _stream(stream, query, out)))
        return out

    def mod_switch(self, x, keep: int, out=None, stream=None):
        """Response compression: [..., L, N] residues mod q -> [..., keep, N] mod q_0 ... q_{keep-1}."""
        x = _dev_u64(x, self.device)
        lead = tuple(x.shape[:-2])
        assert tuple(x.shape[-2:]) == (self.L, self.N)
        count = int(np.prod(lead)) if lead else 1
        if out is None:
            out = self.empty(*lead, keep, self.N)
        _check(lib().pir_mod_switch(self._h, _ptr(x), count, keep, _ptr(out), _stream(stream, x, out)))
        return out

    def mod_switch_noalloc(self, x, keep: int, out=None, stream=None):
        """mod_switch through the entry point that allocates no device memory (at most 2^19
        coefficients per call); `out` may be preallocated so that nothing is allocated at all."""
        x = _dev_u64(x, self.device)
        lead = tuple(x.shape[:-2])
        assert tuple(x.shape[-2:]) == (self.L, self.N)
        count = int(np.prod(lead)) if lead else 1
        if out is None:
            out = self.empty(*lead, keep, self.N)
        _check(lib().pir_mod_switch_noalloc(self._h, _ptr(x), count, keep, _ptr(out), _stream(stream, x, out)))
        return out

    def seeded_query(self, c0, seed: int, out=None, stream=None):
        """Seeded query ciphertexts: c0 [count, L, N] plus the client's 64-bit seed -> the full
        ciphertexts [count, 2, L, N], whose a polynomials the library regenerates from the seed."""
        c0 = _dev_u64(c0, self.device)
        assert c0.dim() == 3 and tuple(c0.shape[1:]) == (self.L, self.N)
        count = int(c0.shape[0])
        if out is None:
            out = self.empty(count, 2, self.L, self.N)
        _check(lib().pir_seeded_query(self._h, _ptr(c0), count, int(seed) & (2**64 - 1), _ptr(out),
                                      _stream(stream, c0, out)))
        return out

    def load_key(self, rlk) -> Key:
        rlk = _dev_u64(rlk, self.device)
        assert tuple(rlk.shape) == (self.L, 2, self.L, self.N)
        h = ctypes.c_void_p()
        _check(lib().pir_load_key(self._h, _ptr(rlk), ctypes.byref(h)))
        return Key(self, h)

    def encode_db(self, codewords: np.ndarray, payload, m: int) -> Database:
        torch = _torch()
        cw = np.ascontiguousarray(codewords, dtype=np.uint32)
        n, k = cw.shape
        if isinstance(payload, np.ndarray):
            payload = torch.from_numpy(np.ascontiguousarray(payload, dtype=np.uint16))
        payload = payload.contiguous()
        assert payload.dtype == torch.uint16 and payload.shape[0] == n and payload.shape[2] == self.N
        s = payload.shape[1]
        h = ctypes.c_void_p()
        _check(lib().pir_encode_db(self._h, n, s, m, k, cw.ctypes.data_as(ctypes.c_void_p),
                                   ctypes.c_void_p(payload.data_ptr()) if n else None, ctypes.byref(h)))
        return Database(self, h, n, s, m, k)

    # ---- Process ----
    def answer(self, key: Key, db: Database, query, out=None, stream=None):
        query = _dev_u64(query, self.device)
        assert tuple(query.shape) == (db.m, 2, self.L, self.N)
        if out is None:
            out = self.empty(db.s, 2, self.L, self.N)
        _check(lib().pir_answer(self._h, key._h, db._h, _ptr(query), _ptr(out), _stream(stream, query, out)))
        return out

    def check_query(self, query, stream=None):
        """Range check of ciphertexts [count, 2, L, N] (pir_check_query): raises PirError
        (PIR_E_INVALID) if a residue is not below its prime."""
        query = _dev_u64(query, self.device)
        assert query.dim() == 4 and tuple(query.shape[1:]) == (2, self.L, self.N)
        _check(lib().pir_check_query(self._h, _ptr(query), int(query.shape[0]), _stream(stream, query)))

    def answer_batch(self, keys, dbs, queries, outs=None, stream=None):
        B = len(queries)
        queries = [_dev_u64(q, self.device) for q in queries]
        if outs is None:
            outs = [self.empty(db.s, 2, self.L, self.N) for db in dbs]
        arr = lambda xs: (ctypes.c_void_p * B)(*xs)  # noqa: E731
        _check(lib().pir_answer_batch(self._h, B, arr([k._h.value for k in keys]), arr([d._h.value for d in dbs]),
                                      arr([q.data_ptr() for q in queries]), arr([o.data_ptr() for o in outs]),
                                      _stream(stream, *queries, *outs)))
        return outs

    def capture(self, keys, dbs, queries, outs=None) -> "Graph":
        """Record pir_answer_batch for these buffers into a HIP graph (see Graph).  queries must be
        device tensors; they and outs are held by the graph and answered at every replay."""
        B = len(queries)
        for q in queries:
            if not (hasattr(q, "is_cuda") and q.is_cuda and q.is_contiguous()):
                raise TypeError("captured queries must be contiguous device tensors")
        if outs is None:
            outs = [self.empty(db.s, 2, self.L, self.N) for db in dbs]
        arr = lambda xs: (ctypes.c_void_p * B)(*xs)  # noqa: E731
        h = ctypes.c_void_p()
        _check(lib().pir_graph_capture(self._h, B, arr([k._h.value for k in keys]), arr([d._h.value for d in dbs]),
                                       arr([q.data_ptr() for q in queries]), arr([o.data_ptr() for o in outs]),
                                       ctypes.byref(h)))
        return Graph(self, h, list(keys), list(dbs), list(queries), outs)

    def selectors(self, key: Key, db: Database, query, elems, out=None, stream=None):
        query = _dev_u64(query, self.device)
        el = np.ascontiguousarray(elems, dtype=np.uint64)
        if out is None:
            out = self.empty(len(el), 2, self.L, self.N)
        _check(lib().pir_selectors(self._h, key._h, db._h, _ptr(query), el.ctypes.data_as(ctypes.c_void_p), len(el),
                                   _ptr(out), _stream(stream, query, out)))
        return out

    def mult(self, a, b, stream=None):
        a, b = _dev_u64(a, self.device), _dev_u64(b, self.device)
        out = self.empty(3, self.L, self.N)
        _check(lib().pir_mult(self._h, _ptr(a), _ptr(b), _ptr(out), _stream(stream, a, b, out)))
        return out

    def relin(self, key: Key, c3, stream=None):
        c3 = _dev_u64(c3, self.device)
        out = self.empty(2, self.L, self.N)
        _check(lib().pir_relin(self._h, key._h, _ptr(c3), _ptr(out), _stream(stream, c3, out)))
        return out

    def pm(self, ct, pt, stream=None):
        torch = _torch()
        ct = _dev_u64(ct, self.device)
        if isinstance(pt, np.ndarray):
            pt = torch.from_numpy(np.ascontiguousarray(pt, dtype=np.uint16))
        pt = pt.to(self.device).contiguous()
        out = self.empty(2, self.L, self.N)
        _check(lib().pir_pm(self._h, _ptr(ct), _ptr(pt), _ptr(out), _stream(stream, ct, pt, out)))
        return out

    # ---- codeword tables ----
    def map_perfect(self, ids, m: int, k: int, stream=None):
        torch = _torch()
        ids = _dev_u64(np.asarray(ids, dtype=np.uint64), self.device)
        out = torch.empty((ids.shape[0], k), dtype=torch.uint32, device=self.device)
        _check(lib().pir_map_perfect(self._h, _ptr(ids), ids.shape[0], m, k, _ptr(out), _stream(stream, ids, out)))
        return out

    def map_lossy(self, keywords, m: int, k: int, seed: int, stream=None):
        torch = _torch()
        kw = _dev_u64(np.asarray(keywords, dtype=np.uint64), self.device)
        out = torch.empty((kw.shape[0], k), dtype=torch.uint32, device=self.device)
        _check(lib().pir_map_lossy(self._h, _ptr(kw), kw.shape[0], m, k, seed, _ptr(out), _stream(stream, kw, out)))
        return out

    # ---- profiling ----
    PROBE_OPS = ("v_fma_f64", "v_mul_f64", "v_add_f64", "v_rndne_f64 + v_add_f64")

    def probe_fp64(self, op: int, blocks: int = 4096, iters: int = 4096, stream=None):
        """Issue-rate probe (pir_probe_fp64): (milliseconds, wave-instructions) of one timed launch."""
        ms, wi = ctypes.c_double(), ctypes.c_double()
        _check(lib().pir_probe_fp64(self._h, op, blocks, iters, ctypes.byref(ms), ctypes.byref(wi),
                                    _stream(stream)))
        return ms.value, wi.value

    PROBE_INT_OPS = ("v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32", "v_lshl_add_u64")

    def probe_int(self, op: int, blocks: int = 4096, iters: int = 4096, stream=None):
        """Integer issue-rate probe (pir_probe_int): (milliseconds, wave-instructions) of one timed
        launch."""
        ms, wi = ctypes.c_double(), ctypes.c_double()
        _check(lib().pir_probe_int(self._h, op, blocks, iters, ctypes.byref(ms), ctypes.byref(wi), _stream(stream)))
        return ms.value, wi.value

    def profile(self, on: bool = True):
        _check(lib().pir_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, reset: bool = True) -> dict:
        """{family: (total_ms, launches, work)} since the last reset."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_uint64 * cap)()
        work = (ctypes.c_double * cap)()
        n = lib().pir_profile_read(self._h, cap, names, ms, cnt, work, 1 if reset else 0)
        if n < 0:
            _check(n)
        return {names[i].decode(): (ms[i], int(cnt[i]), work[i]) for i in range(min(n, cap))}


SCHEDULE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules.json")


def _schedule_key(N, primes, batch, k, s):
    return {"N": int(N), "primes": [int(p) for p in primes], "batch": int(batch), "k": int(k), "s": int(s)}


def lookup_schedule(N, primes, batch, k, s, path=SCHEDULE_CACHE):
    """Tuning cache lookup: {"chunk_elems", "query_group", "relin_group", ...} or None."""
    import json
    if not os.path.exists(path):
        return None
    key = _schedule_key(N, primes, batch, k, s)
    for e in json.load(open(path)).get("entries", []):
        if {kk: e.get(kk) for kk in key} == key:
            return e["schedule"]
    return None


def record_schedule(N, primes, batch, k, s, schedule, note, path=SCHEDULE_CACHE):
    """Add or replace a tuning-cache entry."""
    import json
    data = json.load(open(path)) if os.path.exists(path) else {"entries": []}
    key = _schedule_key(N, primes, batch, k, s)
    data["entries"] = [e for e in data["entries"] if {kk: e.get(kk) for kk in key} != key]
    data["entries"].append({**key, "schedule": schedule, "note": note})
    with open(path, "w") as f:
        json.dump(data, f, indent=1)


class Graph:
    """A captured answer: launch() replays the recorded pir_answer_batch, answering what the captured
    query tensors hold at that time into the captured output tensors (self.outs)."""

    def __init__(self, ctx: Context, handle, keys, dbs, queries, outs):
        self.ctx, self._h = ctx, handle
        self._keep = (keys, dbs, queries)  # must outlive the graph
        self.queries, self.outs = queries, outs

    def launch(self, stream=None):
        _check(lib().pir_graph_launch(self._h, _stream(stream, *self.queries, *self.outs)))
        return self.outs

    def close(self):
        if getattr(self, "_h", None):
            lib().pir_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over one context's resident databases (pir_serve_*).

    submit() queues a query and returns its ticket; step() admits waiting queries and runs one
    round; poll(ticket) is True once that answer is complete, after which result(ticket) hands
    back the answer tensor.  The binding keeps each query and answer tensor alive until then.
    """

    ROUND_ROBIN, OLDEST_FIRST, SIZE_AGED = 0, 1, 2

    def __init__(self, ctx: Context, max_slots: int = 16, policy: int = 0, aging_ns_per_element: float = 0.0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().pir_serve_open(ctx._h, max_slots, ctypes.byref(h)))
        self._h = h
        if aging_ns_per_element:
            _check(lib().pir_serve_set_aging(h, float(aging_ns_per_element)))
        if policy:
            _check(lib().pir_serve_set_policy(h, policy))
        self._live = {}   # ticket -> (query, answer) while queued or running
        self._done = {}   # ticket -> answer once complete

    def submit(self, key: Key, db: Database, query, out=None) -> int:
        ctx = self.ctx
        query = _dev_u64(query, ctx.device)
        assert tuple(query.shape) == (db.m, 2, ctx.L, ctx.N)
        if out is None:
            out = ctx.empty(db.s, 2, ctx.L, ctx.N)
        _torch().cuda.current_stream(ctx.device).synchronize()  # the query must be on the device
        t = ctypes.c_uint64()
        _check(lib().pir_serve_submit(self._h, key._h, db._h, _ptr(query), _ptr(out), ctypes.byref(t)))
        self._live[t.value] = (query, out)
        return t.value

    def step(self) -> int:
        rc = lib().pir_serve_step(self._h)
        if rc < 0:
            _check(rc)
        return rc

    def poll(self, ticket: int) -> bool:
        if ticket in self._done:
            return True
        rc = lib().pir_serve_poll(self._h, ticket)
        if rc < 0:
            _check(rc)
        if rc == 1:
            self._done[ticket] = self._live.pop(ticket)[1]
        return rc == 1

    def result(self, ticket: int):
        return self._done.pop(ticket)

    def stats(self) -> dict:
        r, a, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        act, pend = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().pir_serve_stats(self._h, ctypes.byref(r), ctypes.byref(a), ctypes.byref(c), ctypes.byref(act),
                                     ctypes.byref(pend)))
        return {"rounds": r.value, "admitted": a.value, "completed": c.value, "active": act.value,
                "pending": pend.value}

    def drain(self, tickets=None):
        """Step until every given ticket (default: all submitted) is complete."""
        want = list(self._live) if tickets is None else list(tickets)
        while True:
            if all(self.poll(t) for t in want):
                return
            self.step()

    def close(self):
        if getattr(self, "_h", None):
            lib().pir_serve_close(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
