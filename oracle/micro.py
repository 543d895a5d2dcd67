"""Second, independent oracle in pure Python integers for tiny ring degrees (test infrastructure).

Polynomials are lists of Python integers in [0, q); products are schoolbook negacyclic
convolutions over Z; rounding is Python floor division.  It shares nothing with the C++ oracle
except the interface layout ([size][L][N] residues), so agreement between the two pins the
implementation of the FV readings (centred lifts, exact rounding, per-limb digit relinearization).
Only practical for N <= 64.
"""
from __future__ import annotations

import numpy as np

MASK21 = (1 << 21) - 1


def _negacyclic(a, b):
    N = len(a)
    r = [0] * N
    for i, x in enumerate(a):
        if x == 0:
            continue
        for j, y in enumerate(b):
            k = i + j
            if k < N:
                r[k] += x * y
            else:
                r[k - N] -= x * y
    return r


class Micro:
    def __init__(self, N, primes, t=65537):
        self.N, self.t = N, t
        self.primes = [int(p) for p in primes]
        self.L = len(self.primes)
        self.q = 1
        for p in self.primes:
            self.q *= p
        self.delta = self.q // t

    # residues <-> integers mod q
    def to_int(self, res):          # res [L][N] -> list of ints in [0, q)
        out = []
        for i in range(self.N):
            x = 0
            for j, p in enumerate(self.primes):
                Mj = self.q // p
                x += int(res[j][i]) * Mj * pow(Mj, -1, p)
            out.append(x % self.q)
        return out

    def to_res(self, poly):
        return np.array([[x % p for x in poly] for p in self.primes], dtype=np.uint64)

    def centred(self, x):
        x %= self.q
        return x - self.q if x > self.q // 2 else x

    # client
    def encrypt(self, sk, msg, rnd):
        N, L = self.N, self.L
        a_res = np.zeros((L, N), dtype=np.uint64)
        for j, p in enumerate(self.primes):
            for i in range(N):
                idx = (j * N + i) * 2
                a_res[j][i] = ((int(rnd[idx]) << 64) | int(rnd[idx + 1])) % p
        a = self.to_int(a_res)
        e = [bin(int(w) & MASK21).count("1") - bin((int(w) >> 21) & MASK21).count("1")
             for w in rnd[2 * L * N: 2 * L * N + N]]
        s = [int(v) for v in sk]
        a_s = _negacyclic(a, s)
        c0 = [(-a_s[i] + e[i] + self.delta * (int(msg[i]) % self.t)) % self.q for i in range(N)]
        return np.stack([self.to_res(c0), self.to_res(a)])

    def decrypt(self, sk, ct):
        s = [int(v) for v in sk]
        polys = [self.to_int(ct[r]) for r in range(ct.shape[0])]
        x = polys[0][:]
        spow = s
        for r in range(1, len(polys)):
            prod = _negacyclic(polys[r], spow)
            x = [x[i] + prod[i] for i in range(self.N)]
            spow = _negacyclic(spow, s)
        x = [self.centred(v) for v in x]
        return [((2 * self.t * v + self.q) // (2 * self.q)) % self.t for v in x]

    # server
    def mult(self, a, b):
        A = [[self.centred(v) for v in self.to_int(a[r])] for r in range(2)]
        B = [[self.centred(v) for v in self.to_int(b[r])] for r in range(2)]
        X0 = _negacyclic(A[0], B[0])
        X1 = [u + v for u, v in zip(_negacyclic(A[0], B[1]), _negacyclic(A[1], B[0]))]
        X2 = _negacyclic(A[1], B[1])
        out = []
        for X in (X0, X1, X2):
            out.append(self.to_res([((2 * self.t * v + self.q) // (2 * self.q)) % self.q for v in X]))
        return np.stack(out)

    def relin(self, rlk, c3):
        c0, c1 = self.to_int(c3[0]), self.to_int(c3[1])
        for i, qi in enumerate(self.primes):
            D = [int(v) for v in c3[2][i]]          # digit i: [c2]_{q_i} in [0, q_i)
            b, a = self.to_int(rlk[i][0]), self.to_int(rlk[i][1])
            db, da = _negacyclic(D, b), _negacyclic(D, a)
            c0 = [u + v for u, v in zip(c0, db)]
            c1 = [u + v for u, v in zip(c1, da)]
        return np.stack([self.to_res([v % self.q for v in c0]), self.to_res([v % self.q for v in c1])])

    def pm(self, ct, pt):
        P = [int(v) for v in pt]
        return np.stack([self.to_res([v % self.q for v in _negacyclic(self.to_int(ct[r]), P)])
                         for r in range(2)])

    # substitution (query expansion, Algorithm 5): written as polynomial composition over Z
    def compose(self, poly, g):
        """poly(x^g) mod x^N + 1 for an integer polynomial: sum_i poly_i (x^g)^i, with (x^g)^i
        built by repeated negacyclic multiplication by the monomial x^g."""
        N = self.N
        mono = [0] * N
        e = g % (2 * N)
        if e < N:
            mono[e] = 1
        else:
            mono[e - N] = -1
        power = [1] + [0] * (N - 1)
        out = [0] * N
        for c in poly:
            if c:
                out = [u + c * v for u, v in zip(out, power)]
            power = _negacyclic(power, mono)
        return out

    def automorphism(self, ct, g):
        return np.stack([self.to_res([v % self.q for v in self.compose(self.to_int(ct[r]), g)])
                         for r in range(ct.shape[0])])

    def mul_monomial(self, ct, e):
        N = self.N
        mono = [0] * N
        e %= 2 * N
        if e < N:
            mono[e] = 1
        else:
            mono[e - N] = -1
        return np.stack([self.to_res([v % self.q for v in _negacyclic(self.to_int(ct[r]), mono)])
                         for r in range(ct.shape[0])])

    def sub(self, gk, ct, g):
        """Sub_g: (sigma(c0), 0, sigma(c1)) relinearized under the Galois key."""
        sig = self.automorphism(ct, g)
        zero = np.zeros_like(sig[0])
        return self.relin(gk, np.stack([sig[0], zero, sig[1]]))

    # response compression: round(q' x / q) of the centred lift, in Python integers
    def mod_switch(self, ct, keep):
        qk = 1
        for p in self.primes[:keep]:
            qk *= p
        out = []
        for r in range(ct.shape[0]):
            xs = [self.centred(v) for v in self.to_int(ct[r])]
            ys = [(2 * qk * x + self.q) // (2 * self.q) for x in xs]  # floor(q' x / q + 1/2)
            out.append(np.array([[y % p for y in ys] for p in self.primes[:keep]], dtype=np.uint64))
        return np.stack(out)

