// Modular arithmetic on 64-bit words for primes below 2^61, built from the 32-bit integer
// multipliers of CDNA (64-bit products are v_mul_lo_u32 / v_mul_hi_u32 / v_mad_u64_u32 sequences).
//
//  * Shoup multiplication by a fixed operand w with companion w' = floor(w 2^64 / p) (V. Shoup,
//    NTL; see D. Harvey, "Faster arithmetic for number-theoretic transforms", 2014): for any
//    a < 2^64, a w - hi64(a w') p lies in [0, 2p).
//  * Barrett reduction (P. Barrett, 1986) for products of two variables:
//    mu = floor(2^(2s) / p), s = bit length of p; the quotient estimate is at most 2 too small.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "consts.h"

namespace cw {

__device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t p) {
    uint64_t s = a + b;
    return s >= p ? s - p : s;
}
__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t p) {
    return a >= b ? a - b : a + (p - b);
}
// a * w mod p in [0, 2p)
__device__ __forceinline__ uint64_t mul_shoup_lazy(uint64_t a, uint64_t w, uint64_t wq, uint64_t p) {
    uint64_t qh = __umul64hi(a, wq);
    return a * w - qh * p;
}
__device__ __forceinline__ uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wq, uint64_t p) {
    uint64_t r = mul_shoup_lazy(a, w, wq, p);
    return r >= p ? r - p : r;
}
// a mod p for any a < 2^64, with r1 = floor(2^64 / p)
__device__ __forceinline__ uint64_t reduce64(uint64_t a, uint64_t p, uint64_t r1) {
    uint64_t r = a - __umul64hi(a, r1) * p;
    return r >= p ? r - p : r;
}
// a * b mod p for a, b < p < 2^61 (Barrett)
__device__ __forceinline__ uint64_t mul_barrett(uint64_t a, uint64_t b, uint64_t p, uint64_t mu, uint32_t s) {
    uint64_t lo = a * b, hi = __umul64hi(a, b);
    uint64_t z = (hi << (65 - s)) | (lo >> (s - 1));
    uint64_t ph = __umul64hi(z, mu), pl = z * mu;
    uint64_t qh = (ph << (63 - s)) | (pl >> (s + 1));
    uint64_t r = lo - qh * p;
    r = r >= p ? r - p : r;
    return r >= p ? r - p : r;
}

// ---------------------------------------------------------------------------------------------
// Exact centred base conversion
// ---------------------------------------------------------------------------------------------
// v = round(sum_i y_i / p_i) for y_i < p_i.  The 0.64 fixed-point sum of floor(y_i 2^128 / p_i)
// / 2^64 is at most 2 nin units below the true value, so the decision is certain unless the
// fraction lies in a window just below 1/2.  The fast form reports that case through `amb`; the
// caller then hands the coefficient to a fixup kernel that decides it with conv_round_exact.
template <int NI>
__device__ __forceinline__ uint32_t conv_round_fast(const ConvTable& T, const uint64_t* y, uint32_t nin, bool& amb) {
    uint64_t frac = 0;
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        if (i < (int)nin) {
            uint64_t th = y[i] * T.om_hi[i] + __umul64hi(y[i], T.om_lo[i]);
            uint64_t f2 = frac + th;
            c += (f2 < frac);
            frac = f2;
        }
    }
    const uint64_t half = 1ull << 63;
    amb |= (frac < half && frac >= half - 2ull * nin - 2ull);
    return c + (uint32_t)(frac >> 63);
}

// Exact decision (slow path): V = sum_i y_i (P/p_i) as a multiword integer; round(V/P) = c + 1
// iff 2V >= (2c + 1) P, where c = floor of the fixed-point estimate.
__device__ __noinline__ uint32_t conv_round_exact(const ConvTable& T, const uint64_t* y) {
    uint64_t frac = 0;
    uint32_t c = 0;
    for (uint32_t i = 0; i < T.nin; ++i) {
        uint64_t th = y[i] * T.om_hi[i] + __umul64hi(y[i], T.om_lo[i]);
        uint64_t f2 = frac + th;
        c += (f2 < frac);
        frac = f2;
    }
    const uint32_t W = T.W;
    uint64_t V[MAX_W + 2];
    uint64_t R[MAX_W + 2];
    for (uint32_t w = 0; w < W + 2; ++w) V[w] = R[w] = 0;
    for (uint32_t i = 0; i < T.nin; ++i) {
        uint64_t carry = 0;
        for (uint32_t w = 0; w < W; ++w) {
            uint64_t lo = y[i] * T.Phat[i][w], hi = __umul64hi(y[i], T.Phat[i][w]);
            uint64_t s1 = V[w] + lo;
            hi += (s1 < lo);
            uint64_t s2 = s1 + carry;
            hi += (s2 < s1);
            V[w] = s2;
            carry = hi;
        }
        for (uint32_t w = W; w < W + 2; ++w) {
            uint64_t s1 = V[w] + carry;
            carry = (s1 < carry);
            V[w] = s1;
        }
    }
    uint64_t top = 0;  // V <- 2V
    for (uint32_t w = 0; w < W + 2; ++w) {
        uint64_t nt = V[w] >> 63;
        V[w] = (V[w] << 1) | top;
        top = nt;
    }
    uint64_t f = 2ull * c + 1ull, carry = 0;  // R <- (2c + 1) P
    for (uint32_t w = 0; w < W; ++w) {
        uint64_t lo = T.Pw[w] * f, hi = __umul64hi(T.Pw[w], f);
        uint64_t s1 = lo + carry;
        hi += (s1 < lo);
        R[w] = s1;
        carry = hi;
    }
    R[W] = carry;
    for (int w = (int)W + 1; w >= 0; --w)
        if (V[w] != R[w]) return V[w] > R[w] ? c + 1 : c;
    return c + 1;  // 2V = (2c+1)P is impossible for odd P
}

// out_j = sum_i y_i [(P/p_i) mod r_j] - v [P mod r_j]   (mod r_j), for j < T.nout.  A lazy table
// (r_j < 2^59) adds the products in [0, 2 r_j) and r_j - [v P]_{r_j} in (0, r_j], below
// (2 nin + 1) r_j < 2^64, and reduces once; otherwise every product and sum is reduced.
template <int NI>
__device__ __forceinline__ uint64_t conv_out(const ConvTable& T, const uint64_t* y, uint32_t nin, uint32_t v,
                                             uint32_t j) {
    const uint64_t r = T.pout[j];
    if (T.lazy) {
        uint64_t acc = r - mul_shoup((uint64_t)v, T.Pm[j], T.Pmq[j], r);
#pragma unroll
        for (int i = 0; i < NI; ++i)
            if (i < (int)nin) acc += mul_shoup_lazy(y[i], T.M[i][j], T.Mq[i][j], r);
        return reduce64(acc, r, T.r1[j]);
    }
    uint64_t acc = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i)
        if (i < (int)nin) acc = add_mod(acc, mul_shoup(y[i], T.M[i][j], T.Mq[i][j], r), r);
    return sub_mod(acc, mul_shoup((uint64_t)v, T.Pm[j], T.Pmq[j], r), r);
}

}  // namespace cw
