"""ctypes binding of the C++ oracle (test infrastructure only).

Layouts follow the library's interface: a polynomial limb is N uint64 residues in coefficient
order; a ciphertext is [2][L][N]; a 3-polynomial product is [3][L][N]; a relinearization key is
[L digits][2 (b, a)][L limbs][N]; the payload is uint16 [n][s][N]; codewords are uint32 [n][k].
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_u64p = ctypes.POINTER(ctypes.c_uint64)


def _ptr(a: np.ndarray, ctype=ctypes.c_uint64):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        vp = ctypes.c_void_p
        u32, u64 = ctypes.c_uint32, ctypes.c_uint64
        P64 = _u64p
        P32 = ctypes.POINTER(ctypes.c_uint32)
        P16 = ctypes.POINTER(ctypes.c_uint16)
        P8 = ctypes.POINTER(ctypes.c_int8)
        sig = {
            "orc_new": (vp, [u32, u32, P64, u64]),
            "orc_free": (None, [vp]),
            "orc_num_product_primes": (u32, [vp]),
            "orc_negacyclic_mul_ntt": (None, [u32, u64, P64, P64, P64]),
            "orc_negacyclic_mul_schoolbook": (None, [u32, u64, P64, P64, P64]),
            "orc_divmod_words": (None, [P64, u32, P64, u32, P64, P64]),
            "orc_keygen": (None, [vp, P64, P8]),
            "orc_encrypt": (None, [vp, P8, P64, P64, P64, P64]),
            "orc_relin_keygen": (None, [vp, P8, P64, P64, P64]),
            "orc_decrypt": (ctypes.c_double, [vp, P8, P64, u32, P64]),
            "orc_mult": (None, [vp, P64, P64, P64]),
            "orc_load_rlk": (vp, [vp, P64]),
            "orc_key_free": (None, [vp]),
            "orc_relin": (None, [vp, vp, P64, P64]),
            "orc_pm": (None, [vp, P64, P64, P64]),
            "orc_add": (None, [vp, P64, P64, u32, P64]),
            "orc_selector": (None, [vp, vp, P64, P32, u32, P64]),
            "orc_answer": (None, [vp, vp, P64, u32, u64, u32, P32, P16, P64, ctypes.c_int]),
            "orc_automorphism": (None, [vp, P64, u32, u32, P64]),
            "orc_mul_monomial": (None, [vp, P64, u32, u32, P64]),
            "orc_galois_keygen": (None, [vp, P8, u32, P64, P64, P64]),
            "orc_sub": (None, [vp, vp, P64, u32, P64]),
            "orc_mod_switch": (None, [vp, P64, u32, u32, P64]),
            "orc_one_minus": (None, [vp, P64, P64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def negacyclic_mul_ntt(p: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().orc_negacyclic_mul_ntt(len(a), p, _ptr(a), _ptr(b), _ptr(out))
    return out


def negacyclic_mul_schoolbook(p: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().orc_negacyclic_mul_schoolbook(len(a), p, _ptr(a), _ptr(b), _ptr(out))
    return out


def _to_words(x: int, n: int) -> np.ndarray:
    return np.array([(x >> (64 * i)) & ((1 << 64) - 1) for i in range(n)], dtype=np.uint64)


def _from_words(w: np.ndarray) -> int:
    return sum(int(v) << (64 * i) for i, v in enumerate(w))


def divmod_big(a: int, b: int) -> tuple:
    na = max(1, (a.bit_length() + 63) // 64)
    nb = max(1, (b.bit_length() + 63) // 64)
    A, B = _to_words(a, na), _to_words(b, nb)
    Q, R = np.zeros(na, np.uint64), np.zeros(nb, np.uint64)
    lib().orc_divmod_words(_ptr(A), na, _ptr(B), nb, _ptr(Q), _ptr(R))
    return _from_words(Q), _from_words(R)


class Key:
    def __init__(self, orc: "Oracle", rlk: np.ndarray):
        self._orc = orc
        self.rlk = np.ascontiguousarray(rlk, dtype=np.uint64)
        self._h = lib().orc_load_rlk(orc._h, _ptr(self.rlk))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_key_free(self._h)
            self._h = None


class Oracle:
    """Textbook FV and constant-weight PIR on the CPU for one parameter set (N, q_0..q_{L-1}, t)."""

    def __init__(self, N: int, primes, t: int = 65537):
        self.N, self.t = int(N), int(t)
        self.primes = tuple(int(p) for p in primes)
        self.L = len(self.primes)
        q = np.array(self.primes, dtype=np.uint64)
        self._h = lib().orc_new(self.N, self.L, _ptr(q), self.t)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_free(self._h)
            self._h = None

    @property
    def q(self) -> int:
        r = 1
        for p in self.primes:
            r *= p
        return r

    @property
    def num_product_primes(self) -> int:
        return lib().orc_num_product_primes(self._h)

    def ct_shape(self, size: int = 2) -> tuple:
        return (size, self.L, self.N)

    # ---- client side ------------------------------------------------------------------------
    def keygen(self, rnd: np.ndarray) -> np.ndarray:
        rnd = np.ascontiguousarray(rnd[: self.N], dtype=np.uint64)
        sk = np.empty(self.N, dtype=np.int8)
        lib().orc_keygen(self._h, _ptr(rnd), _ptr(sk, ctypes.c_int8))
        return sk

    def rnd_words_encrypt(self) -> int:
        return 2 * self.L * self.N + self.N

    def encrypt(self, sk: np.ndarray, msg: np.ndarray, rnd: np.ndarray) -> np.ndarray:
        """rnd: rnd_words_encrypt() words: 2 L N for the uniform a, then N for the error."""
        msg = np.ascontiguousarray(msg, dtype=np.uint64)
        ra = np.ascontiguousarray(rnd[: 2 * self.L * self.N], dtype=np.uint64)
        re = np.ascontiguousarray(rnd[2 * self.L * self.N: 2 * self.L * self.N + self.N], dtype=np.uint64)
        ct = np.empty(self.ct_shape(), dtype=np.uint64)
        lib().orc_encrypt(self._h, _ptr(sk, ctypes.c_int8), _ptr(msg), _ptr(ra), _ptr(re), _ptr(ct))
        return ct

    def rnd_words_rlk(self) -> int:
        return self.L * 2 * self.L * self.N + self.L * self.N

    def relin_keygen(self, sk: np.ndarray, rnd: np.ndarray) -> np.ndarray:
        na = self.L * 2 * self.L * self.N
        ra = np.ascontiguousarray(rnd[:na], dtype=np.uint64)
        re = np.ascontiguousarray(rnd[na: na + self.L * self.N], dtype=np.uint64)
        rlk = np.empty((self.L, 2, self.L, self.N), dtype=np.uint64)
        lib().orc_relin_keygen(self._h, _ptr(sk, ctypes.c_int8), _ptr(ra), _ptr(re), _ptr(rlk))
        return rlk

    def galois_keygen(self, sk: np.ndarray, g: int, rnd: np.ndarray) -> np.ndarray:
        """Key switching from s(x^g) to s (same randomness layout as relin_keygen)."""
        na = self.L * 2 * self.L * self.N
        ra = np.ascontiguousarray(rnd[:na], dtype=np.uint64)
        re = np.ascontiguousarray(rnd[na: na + self.L * self.N], dtype=np.uint64)
        gk = np.empty((self.L, 2, self.L, self.N), dtype=np.uint64)
        lib().orc_galois_keygen(self._h, _ptr(sk, ctypes.c_int8), int(g), _ptr(ra), _ptr(re), _ptr(gk))
        return gk

    def decrypt(self, sk: np.ndarray, ct: np.ndarray) -> tuple:
        """Returns (message mod t [N], largest log2 noise)."""
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        size = ct.shape[0]
        msg = np.empty(self.N, dtype=np.uint64)
        noise = lib().orc_decrypt(self._h, _ptr(sk, ctypes.c_int8), _ptr(ct), size, _ptr(msg))
        return msg, noise

    def log2_half_delta(self) -> float:
        import math
        return math.log2((self.q // self.t) / 2)

    # ---- server side ------------------------------------------------------------------------
    def load_key(self, rlk: np.ndarray) -> Key:
        return Key(self, rlk)

    def mult(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.empty(self.ct_shape(3), dtype=np.uint64)
        lib().orc_mult(self._h, _ptr(a), _ptr(b), _ptr(out))
        return out

    def relin(self, key: Key, c3: np.ndarray) -> np.ndarray:
        c3 = np.ascontiguousarray(c3, dtype=np.uint64)
        out = np.empty(self.ct_shape(2), dtype=np.uint64)
        lib().orc_relin(self._h, key._h, _ptr(c3), _ptr(out))
        return out

    def pm(self, ct: np.ndarray, pt: np.ndarray) -> np.ndarray:
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        pt = np.ascontiguousarray(pt, dtype=np.uint64)
        out = np.empty(self.ct_shape(2), dtype=np.uint64)
        lib().orc_pm(self._h, _ptr(ct), _ptr(pt), _ptr(out))
        return out

    def add(self, a: np.ndarray, b: np.ndarray) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint64)
        b = np.ascontiguousarray(b, dtype=np.uint64)
        out = np.empty_like(a)
        lib().orc_add(self._h, _ptr(a), _ptr(b), a.shape[0], _ptr(out))
        return out

    def automorphism(self, ct: np.ndarray, g: int) -> np.ndarray:
        """x -> x^g (g odd) on every polynomial of ct [npoly][L][N]."""
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty_like(ct)
        lib().orc_automorphism(self._h, _ptr(ct), ct.shape[0], int(g), _ptr(out))
        return out

    def mul_monomial(self, ct: np.ndarray, e: int) -> np.ndarray:
        """Multiply every polynomial of ct [npoly][L][N] by x^e (0 <= e < 2N)."""
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty_like(ct)
        lib().orc_mul_monomial(self._h, _ptr(ct), ct.shape[0], int(e) % (2 * self.N), _ptr(out))
        return out

    def sub(self, gk: Key, ct: np.ndarray, g: int) -> np.ndarray:
        """Substitution Sub_g: automorphism, then key switch back to s with the Galois key gk."""
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty(self.ct_shape(2), dtype=np.uint64)
        lib().orc_sub(self._h, gk._h, _ptr(ct), int(g), _ptr(out))
        return out

    def one_minus(self, ct: np.ndarray) -> np.ndarray:
        """The plaintext constant 1 minus the ciphertext: (Delta - c0, -c1) mod q."""
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty_like(ct)
        lib().orc_one_minus(self._h, _ptr(ct), _ptr(out))
        return out

    def mod_switch(self, ct: np.ndarray, keep: int) -> np.ndarray:
        """Response compression: [npoly][L][N] mod q -> [npoly][keep][N] mod q' = q_0 ... q_{keep-1},
        each coefficient round(q' x / q) of its centred representative x."""
        ct = np.ascontiguousarray(ct, dtype=np.uint64)
        out = np.empty((ct.shape[0], keep, self.N), dtype=np.uint64)
        lib().orc_mod_switch(self._h, _ptr(ct), ct.shape[0], int(keep), _ptr(out))
        return out

    def selector(self, key: Key, query: np.ndarray, positions) -> np.ndarray:
        query = np.ascontiguousarray(query, dtype=np.uint64)
        pos = np.ascontiguousarray(positions, dtype=np.uint32)
        out = np.empty(self.ct_shape(2), dtype=np.uint64)
        lib().orc_selector(self._h, key._h, _ptr(query), _ptr(pos, ctypes.c_uint32), len(pos), _ptr(out))
        return out

    def answer(self, key: Key, query: np.ndarray, codewords: np.ndarray, payload: np.ndarray,
               threads: int = 0) -> np.ndarray:
        query = np.ascontiguousarray(query, dtype=np.uint64)
        cw = np.ascontiguousarray(codewords, dtype=np.uint32)
        pl = np.ascontiguousarray(payload, dtype=np.uint16)
        n, k = cw.shape
        s = pl.shape[1]
        assert pl.shape == (n, s, self.N)
        out = np.empty((s, 2, self.L, self.N), dtype=np.uint64)
        lib().orc_answer(self._h, key._h, _ptr(query), k, n, s, _ptr(cw, ctypes.c_uint32),
                         _ptr(pl, ctypes.c_uint16), _ptr(out), threads)
        return out
