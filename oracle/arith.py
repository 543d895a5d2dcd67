"""Arithmetic constant-weight equality (Algorithm 2) on batch-encoded ciphertexts (test infrastructure).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg may use this
module; the product path never does.

What it computes (paper, Section 3.1 "Arithmetic Constant-weight Equality Operator", Algorithm 2,
and the SIMD evaluation of Section 4): for two encrypted constant-weight codewords x, y of CW(m, k),
    k' = sum_{i in [m]} x[i] y[i],    e = (1 / k!) prod_{i in [k]} (k' - i),
which is 1 when x = y and 0 otherwise.  The ciphertexts are batch encoded: slot s of every
plaintext holds one comparison, so N pairs are compared at once.

Readings.
* Slots: plaintext p in Z_t[x]/(x^N + 1) holds the values p(w_s), w_s = psi^(2s+1), s in [N], where
  psi = 3^((t-1)/(2N)) mod t is a primitive 2N-th root of unity (3 generates Z_t^* for t = 65537,
  and 2N divides t - 1).  Encoding is interpolation at those points, decoding is evaluation.
* Order of operations: the m products are Mult (tensor and rounding, no relinearization), summed as
  three-polynomial ciphertexts and relinearized once; k' - i subtracts the plaintext constant i
  (Delta i in coefficient 0 of c0, i in every slot); the k factors are multiplied by the tree of
  the plain operator (neighbours paired level by level, an odd last factor carried up,
  relinearized after every Mult); the result is multiplied by the plaintext constant (k!)^-1 mod t.
"""
from __future__ import annotations

import math

import numpy as np

from .core import Key, Oracle


def slot_root(N: int, t: int) -> int:
    psi = pow(3, (t - 1) // (2 * N), t)
    assert pow(psi, N, t) == t - 1, "psi must be a primitive 2N-th root of unity mod t"
    return psi


def slot_points(N: int, t: int) -> np.ndarray:
    psi = slot_root(N, t)
    return np.array([pow(psi, 2 * s + 1, t) for s in range(N)], dtype=np.uint64)


def decode(coeffs: np.ndarray, t: int) -> np.ndarray:
    """Evaluation: slot s = p(w_s) mod t (Horner over the coefficients, all slots at once)."""
    N = len(coeffs)
    w = slot_points(N, t)
    acc = np.zeros(N, dtype=np.uint64)
    for c in range(N - 1, -1, -1):
        acc = (acc * w + np.uint64(int(coeffs[c]) % t)) % np.uint64(t)
    return acc


def encode(slots, N: int, t: int) -> np.ndarray:
    """Interpolation: the polynomial of degree < N with p(w_s) = slots[s]:
    p_c = N^-1 sum_s slots[s] w_s^-c mod t."""
    slots = np.asarray(slots, dtype=np.uint64) % np.uint64(t)
    winv = np.array([pow(int(x), t - 2, t) for x in slot_points(N, t)], dtype=np.uint64)
    ninv = pow(N, t - 2, t)
    out = np.empty(N, dtype=np.uint64)
    term = slots.copy()  # slots[s] w_s^-c, starting at c = 0
    for c in range(N):
        out[c] = int(term.sum() % np.uint64(t)) * ninv % t
        term = (term * winv) % np.uint64(t)
    return out


def sub_constant(orc: Oracle, ct: np.ndarray, v: int) -> np.ndarray:
    """ct - v for the plaintext constant v: c0 - Delta v in coefficient 0."""
    delta = orc.q // orc.t
    out = np.array(ct, dtype=np.uint64, copy=True)
    for j, p in enumerate(orc.primes):
        out[0, j, 0] = (int(out[0, j, 0]) - delta * v) % p
    return out


def constant_plaintext(N: int, v: int) -> np.ndarray:
    pt = np.zeros(N, dtype=np.uint64)
    pt[0] = v
    return pt


def arith_equality(orc: Oracle, key: Key, x: np.ndarray, y: np.ndarray, k: int) -> np.ndarray:
    """Algorithm 2 on ciphertexts x, y [m][2][L][N] -> e [2][L][N]."""
    acc = None
    for xi, yi in zip(x, y):
        prod = orc.mult(xi, yi)
        acc = prod if acc is None else orc.add(acc, prod)
    kp = orc.relin(key, acc)
    factors = np.stack([sub_constant(orc, kp, i) for i in range(k)])
    e = orc.selector(key, factors, np.arange(k, dtype=np.uint32))
    return orc.pm(e, constant_plaintext(orc.N, pow(math.factorial(k), -1, orc.t)))


def plain_equality(xbits: np.ndarray, ybits: np.ndarray, k: int, t: int) -> np.ndarray:
    """Algorithm 2 on plaintext bit vectors [m][slots] (the closed form the ciphertexts must decode to)."""
    kp = (xbits.astype(np.int64) * ybits.astype(np.int64)).sum(axis=0)
    e = np.ones_like(kp)
    for i in range(k):
        e = e * (kp - i) % t
    return e * pow(math.factorial(k), -1, t) % t
