// Constant tables of one parameter set, laid out identically for the host builder and the kernels.
//
// Primes are indexed Q first (the ciphertext primes q_0..q_{L-1}) and then B (the auxiliary primes
// b_0..b_{LB-1}, chosen by the library).  Q*B must hold every exact tensor product X of two centred
// ciphertext polynomials (|X| < N q^2 / 2) and B must hold every rounded result round(t X / q)
// (|y| < t N q / 2 + 1), so B > 4 t N q is required.
#pragma once
#include <stdint.h>

namespace cw {

constexpr int MAX_L = 12;            // ciphertext primes
constexpr int MAX_LB = 13;           // auxiliary primes
constexpr int MAX_LD = 2;            // primes of the deferred key switch's digit sums (after Q and B)
constexpr int MAX_LL = MAX_L + MAX_LB + MAX_LD;  // per-prime tables: Q, then B, then D
constexpr int MAX_CONV = MAX_LB;     // >= max(MAX_L, MAX_LB)
constexpr int MAX_W = 14;            // 64-bit words of a basis product, plus two spare words

// Exact centred conversion from basis P = {p_i} to basis R = {r_j}.  For x with residues x_i:
//   y_i = [x_i (P/p_i)^{-1}]_{p_i} (the caller may fold a factor into this constant),
//   v   = round(sum_i y_i / p_i)   (fraction sum in 0.64 fixed point, exact fallback near 1/2),
//   [x]_centred mod r_j = sum_i y_i [(P/p_i) mod r_j] - v [P mod r_j].
// lazy: every output prime lies below CONV_LAZY_BOUND, so conv_out may add the nin + 1 products of
// [0, 2 r_j) each and reduce the sum once (below (2 nin + 1) 2^59 < 2^64 for nin <= MAX_CONV).
struct ConvTable {
    uint32_t nin, nout, W, lazy;
    uint64_t pin[MAX_CONV];
    uint64_t om_hi[MAX_CONV], om_lo[MAX_CONV];   // floor(2^128 / p_i) = om_hi 2^64 + om_lo
    uint64_t pout[MAX_CONV];
    uint64_t M[MAX_CONV][MAX_CONV];              // (P/p_i) mod r_j
    uint64_t Mq[MAX_CONV][MAX_CONV];             // Shoup companions
    uint64_t Pm[MAX_CONV], Pmq[MAX_CONV];        // P mod r_j
    uint64_t r1[MAX_CONV];                       // floor(2^64 / r_j)
    double Md[MAX_CONV][MAX_CONV];               // (P/p_i) mod r_j as doubles (fp64 path)
    double Pmd[MAX_CONV];                        // P mod r_j as doubles
    uint64_t Pw[MAX_W];                          // P, little-endian words
    uint64_t Phat[MAX_CONV][MAX_W];              // P / p_i
};

constexpr uint64_t CONV_LAZY_BOUND = 1ull << 59;
static_assert((2 * MAX_CONV + 1) * (CONV_LAZY_BOUND >> 32) < (1ull << 32), "lazy conversion sums fit 64 bits");
// The integer path draws its auxiliary primes below CONV_LAZY_BOUND, so its conversions into B are lazy.

// Primes below this bound may use the fp64 transform (see kernels.hip); the exactness argument
// needs every intermediate integer below 2^53.
constexpr uint64_t FP_PRIME_BOUND = 1ull << 50;
constexpr uint64_t FP_LAZY_BOUND = 1ull << 48;  // lazy fp64 forward transforms (no reduction between passes)

struct CtxConst {
    uint32_t N, logN, L, LB, LL, fp;             // fp: transforms run on the fp64 pipe; LL = L + LB (the D
                                                 // primes, when present, follow at LL and LL + 1)
    uint64_t t;
    uint64_t p[MAX_LL];
    uint64_t bar_mu[MAX_LL];                     // floor(2^(2s) / p), s = bit length of p
    uint32_t bar_s[MAX_LL];
    uint64_t r1[MAX_LL];                         // floor(2^64 / p)
    uint64_t ninv[MAX_LL], ninvq[MAX_LL];        // N^{-1} mod p
    double pd[MAX_LL], pinv[MAX_LL];             // p and 1/p as doubles (fp64 transform)
    double ninvd[MAX_LL], ninvdq[MAX_LL];        // N^{-1} mod p and (N^{-1} mod p)/p as doubles
    uint64_t qinv[MAX_L], qinvq[MAX_L];          // [(q/q_i)^{-1}]_{q_i}
    uint64_t delta[MAX_L];                       // Delta = floor(q/t) mod q_i
    uint64_t tqinv[MAX_L], tqinvq[MAX_L];        // [t (q/q_i)^{-1} N^{-1}]_{q_i} (scale input lacks N^{-1})
    uint64_t kb1[MAX_LB], kb1q[MAX_LB];          // [t q^{-1} (B/b_j)^{-1} N^{-1}]_{b_j} (likewise)
    uint64_t kb2[MAX_LB], kb2q[MAX_LB];          // [q^{-1} (B/b_j)^{-1}]_{b_j}
    double tqinvd[MAX_L], kb1d[MAX_LB], kb2d[MAX_LB];  // the same constants as doubles (fp64 path)
    // fp64 path: the tensor products' inverse transform multiplies row k by foldd[k] (tqinv_k for Q,
    // kb1_{k-L} for B, 1 for the digit-sum primes), so the scale kernel reads y_i and kb1_j x_j
    // directly; with the key constant folded into the Q -> B conversion it then forms
    //   z_j = [kb1_j x_j] + sum_i y_i [-kb2_j (q/q_i)]_{b_j} + v [kb2_j q]_{b_j}   (mod b_j),
    // the last constant centred (|fqpd| < b_j / 2), so that v fqpd is an exact double product.
    double foldd[MAX_LL];
    double fqbd[MAX_L][MAX_LB], fqpd[MAX_LB];
    ConvTable qb;                                // q -> B
    ConvTable bq;                                // B -> q
};

// Modulus switching from q = q_0 ... q_{L-1} to q' = q_0 ... q_{keep-1} (response compression):
// r = q / q'.  For x with residues x_i: [x]_r (centred) from the dropped limbs by the exact
// conversion T (dropped -> kept), then x' = (x_j - [x]_r) r^{-1} mod q_j = round(x / r).
struct SwitchConst {
    uint32_t keep, L;
    ConvTable T;                                 // {q_keep..q_{L-1}} -> {q_0..q_{keep-1}}
    uint64_t yc[MAX_L], ycq[MAX_L];              // [(r / q_i)^{-1}]_{q_i} for dropped i (index i - keep)
    uint64_t rinv[MAX_L], rinvq[MAX_L];          // [r^{-1}]_{q_j} for kept j
};

// Exact CRT of the deferred key switch's digit sums from its two primes d0, d1 (context primes LL and
// LL + 1, after Q and B), written b0, b1 below: w = w0 + b0 t, t = (w1 - w0) b0^-1 mod b1, centred
// (w > half stands for w - b0 b1), then reduced mod every q_j.
struct CrtConst {  // passed by value
    uint64_t b0inv, b0invq;            // b0^-1 mod b1 and its Shoup companion
    uint64_t half_hi, half_lo;         // (b0 b1 - 1) / 2 as a 128-bit number
    uint64_t b0q[MAX_L], b0qq[MAX_L];  // b0 mod q_j, Shoup companion
    uint64_t Bq[MAX_L];                // b0 b1 mod q_j
};

// Operand reference of a tree node: a query ciphertext (leaf) or a memoised inner node.
constexpr uint32_t REF_NODE = 0x80000000u;

}  // namespace cw
