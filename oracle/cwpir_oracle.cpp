/*
 * CPU oracle for constant-weight PIR (Mahdavi and Kerschbaum, arXiv 2202.07569) over textbook FV.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference implementation that the GPU library
 * is checked against.  Only the test suite, the package smoke check and the benchmark's CPU-baseline
 * leg may load it; the product path never does.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * What it computes (paper, Sections 2.1, 2.3 and 3):
 *   - FV over R_q = Z_q[x]/(x^N+1) with plaintext ring R_t (Section 2.1.1): encryption with the
 *     secret key, Mult, PM, Add, decryption.
 *   - The plain constant-weight equality operator f_PCW(x, y) = product of x[j] over the one
 *     positions j of y (Section 3.1, equation for the plain constant-weight equality), evaluated on
 *     ciphertexts as a depth-ceil(log2 k) tree (Selection Vector Calculation, Algorithm 6).
 *   - The PIR answer: the baseline inner product of the selection vector with the database
 *     (Section 2.3, Eq. (1)), s inner products of n plaintext multiplications (Section 3.3.3).
 *
 * The paper defers every FV internal to the FV paper and to SEAL.  This file fixes them to the
 * textbook definitions (Fan and Vercauteren, ePrint 2012/144):
 *   - Mult: lift both operands to centred representatives in (-q/2, q/2), multiply exactly over
 *     Z[x]/(x^N+1), then c_i = round(t * X_i / q) mod q.  Ties cannot occur (q odd, gcd(t, q) = 1).
 *   - Relinearization: per-limb RNS digits D_i = [c2]_{q_i} in [0, q_i); rlk_i = (b_i, a_i) with
 *     b_i = [-a_i s + e_i + g_i s^2]_q, g_i = (q/q_i) [(q/q_i)^{-1}]_{q_i}; c0' = c0 + sum D_i b_i,
 *     c1' = c1 + sum D_i a_i (mod q).  Every listed prime is a ciphertext prime.
 *   - PM: the plaintext's coefficients in [0, t) are used as they are (no centring).
 *   - Encryption with the secret key: (c0, c1) = ([-a s + e + Delta m]_q, a), Delta = floor(q/t).
 *
 * Exact polynomial products over Z use a multi-prime negacyclic NTT (ψ-twisted cyclic transform)
 * over an oracle-private set of 62-bit primes whose product exceeds 4 N q^2, followed by CRT
 * reconstruction into big integers.  Products modulo one ciphertext prime use the same transform
 * over that prime.  A schoolbook product is exported beside it as the brute-force check.
 *
 * Big integers: little-endian vectors of 64-bit words; division is binary long division.
 */
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

typedef unsigned __int128 u128;
typedef std::vector<uint64_t> Big;

// ------------------------------------------------------------------------------------------------
// word-level modular arithmetic
// ------------------------------------------------------------------------------------------------
static inline uint64_t addm(uint64_t a, uint64_t b, uint64_t p) {
    uint64_t s = a + b;
    return (s >= p || s < a) ? s - p : s;
}
static inline uint64_t subm(uint64_t a, uint64_t b, uint64_t p) { return a >= b ? a - b : a + (p - b); }
static inline uint64_t mulm(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }
static uint64_t powm(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulm(r, a, p);
        a = mulm(a, a, p);
        e >>= 1;
    }
    return r;
}
static uint64_t invm(uint64_t a, uint64_t p) { return powm(a, p - 2, p); }  // p prime

static bool is_prime_u64(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t sp : small)
        if (n % sp == 0) return n == sp;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t a : small) {  // deterministic for n < 3.3e24
        uint64_t x = powm(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulm(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

// ------------------------------------------------------------------------------------------------
// big unsigned integers
// ------------------------------------------------------------------------------------------------
static void trim(Big& a) { while (!a.empty() && a.back() == 0) a.pop_back(); }
static Big big_u64(uint64_t x) { Big r; if (x) r.push_back(x); return r; }
static int cmp(const Big& a, const Big& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}
static Big add(const Big& a, const Big& b) {
    size_t n = std::max(a.size(), b.size());
    Big r(n + 1);
    u128 c = 0;
    for (size_t i = 0; i < n; ++i) {
        c += (u128)(i < a.size() ? a[i] : 0) + (i < b.size() ? b[i] : 0);
        r[i] = (uint64_t)c;
        c >>= 64;
    }
    r[n] = (uint64_t)c;
    trim(r);
    return r;
}
static void sub_in(Big& a, const Big& b) {  // a -= b, requires a >= b
    uint64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        uint64_t bi = i < b.size() ? b[i] : 0;
        uint64_t d = a[i] - bi;
        uint64_t br = (a[i] < bi) ? 1 : 0;
        uint64_t d2 = d - borrow;
        br |= (d < borrow) ? 1 : 0;
        a[i] = d2;
        borrow = br;
    }
    trim(a);
}
static Big sub(const Big& a, const Big& b) { Big r = a; sub_in(r, b); return r; }
static Big mul_u64(const Big& a, uint64_t m) {
    Big r(a.size() + 1);
    u128 c = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        c += (u128)a[i] * m;
        r[i] = (uint64_t)c;
        c >>= 64;
    }
    r[a.size()] = (uint64_t)c;
    trim(r);
    return r;
}
static Big mul(const Big& a, const Big& b) {
    if (a.empty() || b.empty()) return Big();
    Big r(a.size() + b.size(), 0);
    for (size_t i = 0; i < a.size(); ++i) {
        u128 c = 0;
        for (size_t j = 0; j < b.size(); ++j) {
            c += (u128)a[i] * b[j] + r[i + j];
            r[i + j] = (uint64_t)c;
            c >>= 64;
        }
        r[i + b.size()] = (uint64_t)c;
    }
    trim(r);
    return r;
}
static size_t bitlen(const Big& a) {
    if (a.empty()) return 0;
    return 64 * (a.size() - 1) + (64 - __builtin_clzll(a.back()));
}
static bool testbit(const Big& a, size_t i) {
    size_t w = i / 64;
    return w < a.size() && ((a[w] >> (i % 64)) & 1);
}
static void shl1_or(Big& a, bool low) {
    uint64_t carry = low ? 1 : 0;
    for (auto& w : a) {
        uint64_t nc = w >> 63;
        w = (w << 1) | carry;
        carry = nc;
    }
    if (carry) a.push_back(carry);
}
// Binary long division: num = quo * den + rem, 0 <= rem < den.
static void divmod(const Big& num, const Big& den, Big& quo, Big& rem) {
    quo.assign(num.size() + 1, 0);
    rem.clear();
    for (size_t i = bitlen(num); i-- > 0;) {
        shl1_or(rem, testbit(num, i));
        if (cmp(rem, den) >= 0) {
            sub_in(rem, den);
            quo[i / 64] |= 1ull << (i % 64);
        }
    }
    trim(quo);
}
static uint64_t mod_u64(const Big& a, uint64_t p) {
    u128 r = 0;
    for (size_t i = a.size(); i-- > 0;) r = ((r << 64) | a[i]) % p;
    return (uint64_t)r;
}

struct SInt {  // signed big integer: sign and magnitude
    bool neg = false;
    Big mag;
};
static uint64_t residue(const SInt& v, uint64_t p) {
    uint64_t r = mod_u64(v.mag, p);
    return (v.neg && r) ? p - r : r;
}

// ------------------------------------------------------------------------------------------------
// CRT over a set of primes
// ------------------------------------------------------------------------------------------------
struct Crt {
    std::vector<uint64_t> p;
    Big M, halfM;                 // product, floor(M/2)
    std::vector<Big> Mk;          // M / p_k
    std::vector<uint64_t> inv;    // (M/p_k)^{-1} mod p_k
    void init(const std::vector<uint64_t>& primes) {
        p = primes;
        M = big_u64(1);
        for (uint64_t x : p) M = mul_u64(M, x);
        Mk.resize(p.size());
        inv.resize(p.size());
        for (size_t k = 0; k < p.size(); ++k) {
            Big m = big_u64(1);
            for (size_t j = 0; j < p.size(); ++j)
                if (j != k) m = mul_u64(m, p[j]);
            Mk[k] = m;
            inv[k] = invm(mod_u64(m, p[k]), p[k]);
        }
        Big q, r;
        divmod(M, big_u64(2), halfM, r);
    }
    // value in [0, M) with the given residues x[k * stride]
    Big lift(const uint64_t* x, size_t stride) const {
        Big acc;
        for (size_t k = 0; k < p.size(); ++k) acc = add(acc, mul_u64(Mk[k], mulm(x[k * stride], inv[k], p[k])));
        while (cmp(acc, M) >= 0) sub_in(acc, M);
        return acc;
    }
    // centred representative in (-M/2, M/2)  (M odd)
    SInt lift_centered(const uint64_t* x, size_t stride) const {
        SInt v;
        v.mag = lift(x, stride);
        if (cmp(v.mag, halfM) > 0) {
            v.mag = sub(M, v.mag);
            v.neg = true;
        }
        return v;
    }
};

// ------------------------------------------------------------------------------------------------
// negacyclic NTT modulo one prime: a_i <- a_i psi^i, then a cyclic DFT with omega = psi^2
// (bit-reversal permutation followed by iterative radix-2 butterflies).
// ------------------------------------------------------------------------------------------------
struct Ntt {
    uint64_t p = 0;
    uint32_t N = 0, logN = 0;
    std::vector<uint64_t> psi, psi_inv, w, w_inv;  // psi^i, psi^-i (i<N); omega^i, omega^-i (i<N/2)
    uint64_t n_inv = 0;
    std::vector<uint32_t> rev;
    void init(uint64_t prime, uint32_t n) {
        p = prime;
        N = n;
        logN = 0;
        while ((1u << logN) < N) ++logN;
        uint64_t root = 0;
        for (uint64_t g = 2;; ++g) {
            uint64_t x = powm(g, (p - 1) / (2 * (uint64_t)N), p);
            if (powm(x, N, p) == p - 1) { root = x; break; }
        }
        uint64_t rinv = invm(root, p);
        psi.resize(N); psi_inv.resize(N); w.resize(N / 2); w_inv.resize(N / 2);
        psi[0] = psi_inv[0] = 1;
        for (uint32_t i = 1; i < N; ++i) {
            psi[i] = mulm(psi[i - 1], root, p);
            psi_inv[i] = mulm(psi_inv[i - 1], rinv, p);
        }
        for (uint32_t i = 0; i < N / 2; ++i) {
            w[i] = psi[(2 * i) % N];
            w_inv[i] = psi_inv[(2 * i) % N];
        }
        n_inv = invm(N, p);
        rev.resize(N);
        for (uint32_t i = 0; i < N; ++i) {
            uint32_t r = 0;
            for (uint32_t b = 0; b < logN; ++b)
                if (i & (1u << b)) r |= 1u << (logN - 1 - b);
            rev[i] = r;
        }
    }
    void cyclic(uint64_t* a, const std::vector<uint64_t>& tw) const {
        for (uint32_t i = 0; i < N; ++i)
            if (i < rev[i]) std::swap(a[i], a[rev[i]]);
        for (uint32_t len = 2; len <= N; len <<= 1) {
            uint32_t half = len / 2, step = N / len;
            for (uint32_t i = 0; i < N; i += len)
                for (uint32_t j = 0; j < half; ++j) {
                    uint64_t u = a[i + j];
                    uint64_t v = mulm(a[i + j + half], tw[j * step], p);
                    a[i + j] = addm(u, v, p);
                    a[i + j + half] = subm(u, v, p);
                }
        }
    }
    void forward(uint64_t* a) const {
        for (uint32_t i = 0; i < N; ++i) a[i] = mulm(a[i], psi[i], p);
        cyclic(a, w);
    }
    void inverse(uint64_t* a) const {
        cyclic(a, w_inv);
        for (uint32_t i = 0; i < N; ++i) a[i] = mulm(mulm(a[i], n_inv, p), psi_inv[i], p);
    }
};

// ------------------------------------------------------------------------------------------------
// context
// ------------------------------------------------------------------------------------------------
struct OrcCtx {
    uint32_t N, L;
    uint64_t t;
    std::vector<uint64_t> qp;      // ciphertext primes
    Crt Q;                         // over the ciphertext primes; Q.M = q
    Big Delta;                     // floor(q / t)
    std::vector<uint64_t> delta_r; // Delta mod q_i
    std::vector<Ntt> qntt;         // transform per ciphertext prime
    Crt P;                         // oracle-private product basis, P.M > 4 N q^2
    std::vector<Ntt> pntt;
};

struct OrcKey {  // relinearization key, transformed per ciphertext prime: [i][0=b,1=a][j][N]
    std::vector<uint64_t> hat;
};

static void poly_mul_mod(const OrcCtx* c, uint32_t j, const uint64_t* a, const uint64_t* b, uint64_t* out) {
    const Ntt& T = c->qntt[j];
    std::vector<uint64_t> A(a, a + c->N), B(b, b + c->N);
    T.forward(A.data());
    T.forward(B.data());
    for (uint32_t i = 0; i < c->N; ++i) A[i] = mulm(A[i], B[i], T.p);
    T.inverse(A.data());
    std::memcpy(out, A.data(), sizeof(uint64_t) * c->N);
}

// s in {-1, 0, 1} as a residue polynomial modulo q_j
static void ternary_mod(const int8_t* s, uint32_t N, uint64_t p, uint64_t* out) {
    for (uint32_t i = 0; i < N; ++i) out[i] = s[i] < 0 ? p - 1 : (uint64_t)s[i];
}

// round(t * X / q) for a signed X, as residues mod every ciphertext prime (O5)
static void scale_round(const OrcCtx* c, const SInt& X, uint64_t* out, size_t stride) {
    Big num = mul_u64(X.mag, c->t);
    num = add(add(num, num), c->Q.M);             // 2 t |X| + q
    Big den = add(c->Q.M, c->Q.M);                // 2 q
    Big y, r;
    divmod(num, den, y, r);                       // floor((2t|X| + q) / 2q) = round(t|X|/q)
    for (uint32_t j = 0; j < c->L; ++j) {
        uint64_t v = mod_u64(y, c->qp[j]);
        out[j * stride] = (X.neg && v) ? c->qp[j] - v : v;
    }
}

extern "C" {

OrcCtx* orc_new(uint32_t N, uint32_t L, const uint64_t* q, uint64_t t) {
    OrcCtx* c = new OrcCtx();
    c->N = N;
    c->L = L;
    c->t = t;
    c->qp.assign(q, q + L);
    c->Q.init(c->qp);
    Big r;
    divmod(c->Q.M, big_u64(t), c->Delta, r);
    c->delta_r.resize(L);
    for (uint32_t j = 0; j < L; ++j) c->delta_r[j] = mod_u64(c->Delta, c->qp[j]);
    c->qntt.resize(L);
    for (uint32_t j = 0; j < L; ++j) c->qntt[j].init(c->qp[j], N);
    // product basis: largest primes below 2^62 that are 1 mod 2N, until P > 4 N q^2
    Big bound = mul_u64(mul(c->Q.M, c->Q.M), 4ull * N);
    std::vector<uint64_t> pp;
    Big prod = big_u64(1);
    uint64_t step = 2ull * N;
    uint64_t cand = ((1ull << 62) - 1) / step * step + 1;
    if (cand >= (1ull << 62)) cand -= step;
    while (cmp(prod, bound) <= 0) {
        if (is_prime_u64(cand)) {
            pp.push_back(cand);
            prod = mul_u64(prod, cand);
        }
        cand -= step;
    }
    c->P.init(pp);
    c->pntt.resize(pp.size());
    for (size_t k = 0; k < pp.size(); ++k) c->pntt[k].init(pp[k], N);
    return c;
}

void orc_free(OrcCtx* c) { delete c; }

uint32_t orc_num_product_primes(const OrcCtx* c) { return (uint32_t)c->P.p.size(); }

// ---- pins: transforms and products modulo one prime -------------------------------------------
void orc_negacyclic_mul_ntt(uint32_t N, uint64_t p, const uint64_t* a, const uint64_t* b, uint64_t* out) {
    Ntt T;
    T.init(p, N);
    std::vector<uint64_t> A(a, a + N), B(b, b + N);
    T.forward(A.data());
    T.forward(B.data());
    for (uint32_t i = 0; i < N; ++i) A[i] = mulm(A[i], B[i], p);
    T.inverse(A.data());
    std::memcpy(out, A.data(), sizeof(uint64_t) * N);
}

// brute force: out_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j  (mod p)
void orc_negacyclic_mul_schoolbook(uint32_t N, uint64_t p, const uint64_t* a, const uint64_t* b, uint64_t* out) {
    std::vector<uint64_t> r(N, 0);
    for (uint32_t i = 0; i < N; ++i)
        for (uint32_t j = 0; j < N; ++j) {
            uint64_t v = mulm(a[i], b[j], p);
            uint32_t k = i + j;
            if (k < N) r[k] = addm(r[k], v, p);
            else r[k - N] = subm(r[k - N], v, p);
        }
    std::memcpy(out, r.data(), sizeof(uint64_t) * N);
}

// big-integer long division on word arrays (pinned against Python integers)
void orc_divmod_words(const uint64_t* num, uint32_t nn, const uint64_t* den, uint32_t nd, uint64_t* quo,
                      uint64_t* rem) {
    Big a(num, num + nn), b(den, den + nd), q, r;
    trim(a);
    trim(b);
    divmod(a, b, q, r);
    std::memset(quo, 0, 8 * nn);
    std::memset(rem, 0, 8 * nd);
    for (size_t i = 0; i < q.size(); ++i) quo[i] = q[i];
    for (size_t i = 0; i < r.size(); ++i) rem[i] = r[i];
}

// ---- client side: keys, encryption, decryption ------------------------------------------------
// secret s_i = (w_i mod 3) - 1, one word per coefficient
void orc_keygen(const OrcCtx* c, const uint64_t* rnd, int8_t* sk) {
    for (uint32_t i = 0; i < c->N; ++i) sk[i] = (int8_t)((int)(rnd[i] % 3) - 1);
}

static inline int64_t cbd21(uint64_t w) {
    const uint64_t m = (1ull << 21) - 1;
    return (int64_t)__builtin_popcountll(w & m) - (int64_t)__builtin_popcountll((w >> 21) & m);
}
static inline uint64_t uniform_mod(uint64_t w1, uint64_t w2, uint64_t p) {
    return (uint64_t)((((u128)w1 << 64) | w2) % p);
}
static inline uint64_t signed_mod(int64_t v, uint64_t p) {
    return v >= 0 ? (uint64_t)v % p : (p - ((uint64_t)(-v) % p)) % p;
}

// ct = ([-a s + e + Delta m]_q, a).  rnd_a: 2 L N words (two per residue), rnd_e: N words.
void orc_encrypt(const OrcCtx* c, const int8_t* sk, const uint64_t* msg, const uint64_t* rnd_a,
                 const uint64_t* rnd_e, uint64_t* ct) {
    const uint32_t N = c->N, L = c->L;
    std::vector<uint64_t> s(N), as(N);
    for (uint32_t j = 0; j < L; ++j) {
        uint64_t p = c->qp[j];
        uint64_t* c0 = ct + (size_t)j * N;
        uint64_t* c1 = ct + (size_t)(L + j) * N;
        for (uint32_t i = 0; i < N; ++i) {
            size_t idx = ((size_t)j * N + i) * 2;
            c1[i] = uniform_mod(rnd_a[idx], rnd_a[idx + 1], p);
        }
        ternary_mod(sk, N, p, s.data());
        poly_mul_mod(c, j, c1, s.data(), as.data());
        for (uint32_t i = 0; i < N; ++i) {
            uint64_t e = signed_mod(cbd21(rnd_e[i]), p);
            uint64_t dm = mulm(c->delta_r[j], msg[i] % c->t, p);
            c0[i] = addm(subm(e, as[i], p), dm, p);
        }
    }
}

// rlk [i][0=b,1=a][j][N]; rnd_a: L * 2 L N words, rnd_e: L * N words
void orc_relin_keygen(const OrcCtx* c, const int8_t* sk, const uint64_t* rnd_a, const uint64_t* rnd_e,
                      uint64_t* rlk) {
    const uint32_t N = c->N, L = c->L;
    std::vector<uint64_t> s(N), s2(N), as(N);
    for (uint32_t i = 0; i < L; ++i) {
        // g_i = (q/q_i) * [(q/q_i)^{-1}]_{q_i}
        Big gi = mul_u64(c->Q.Mk[i], c->Q.inv[i]);
        for (uint32_t j = 0; j < L; ++j) {
            uint64_t p = c->qp[j];
            uint64_t* b = rlk + (((size_t)i * 2 + 0) * L + j) * N;
            uint64_t* a = rlk + (((size_t)i * 2 + 1) * L + j) * N;
            for (uint32_t x = 0; x < N; ++x) {
                size_t idx = (((size_t)i * L + j) * N + x) * 2;
                a[x] = uniform_mod(rnd_a[idx], rnd_a[idx + 1], p);
            }
            ternary_mod(sk, N, p, s.data());
            poly_mul_mod(c, j, s.data(), s.data(), s2.data());
            poly_mul_mod(c, j, a, s.data(), as.data());
            uint64_t g = mod_u64(gi, p);
            for (uint32_t x = 0; x < N; ++x) {
                uint64_t e = signed_mod(cbd21(rnd_e[(size_t)i * N + x]), p);
                b[x] = addm(subm(e, as[x], p), mulm(g, s2[x], p), p);
            }
        }
    }
}

// Decrypt a ciphertext of `size` (2 or 3) polynomials: x = [c0 + c1 s (+ c2 s^2)]_q centred,
// m = [round(t x / q)]_t.  Returns the largest log2 |x - Delta m| (centred mod q) over coefficients.
double orc_decrypt(const OrcCtx* c, const int8_t* sk, const uint64_t* ct, uint32_t size, uint64_t* msg) {
    const uint32_t N = c->N, L = c->L;
    std::vector<uint64_t> x((size_t)L * N), s(N), s2(N), tmp(N);
    for (uint32_t j = 0; j < L; ++j) {
        uint64_t p = c->qp[j];
        ternary_mod(sk, N, p, s.data());
        uint64_t* xj = x.data() + (size_t)j * N;
        poly_mul_mod(c, j, ct + (size_t)(L + j) * N, s.data(), xj);
        for (uint32_t i = 0; i < N; ++i) xj[i] = addm(xj[i], ct[(size_t)j * N + i], p);
        if (size == 3) {
            poly_mul_mod(c, j, s.data(), s.data(), s2.data());
            poly_mul_mod(c, j, ct + (size_t)(2 * L + j) * N, s2.data(), tmp.data());
            for (uint32_t i = 0; i < N; ++i) xj[i] = addm(xj[i], tmp[i], p);
        }
    }
    double worst = -1.0;
    Big twoq = add(c->Q.M, c->Q.M);
    for (uint32_t i = 0; i < N; ++i) {
        SInt v = c->Q.lift_centered(x.data() + i, N);
        Big num = add(mul_u64(mul_u64(v.mag, c->t), 2), c->Q.M);
        Big y, r;
        divmod(num, twoq, y, r);                  // round(t |x| / q)
        uint64_t ym = mod_u64(y, c->t);
        uint64_t m = (v.neg && ym) ? c->t - ym : ym;
        msg[i] = m;
        // noise = x - Delta m, reduced to (-q/2, q/2)
        Big dm = mul_u64(c->Delta, m);
        SInt e;
        if (!v.neg) {
            if (cmp(v.mag, dm) >= 0) e.mag = sub(v.mag, dm);
            else { e.mag = sub(dm, v.mag); e.neg = true; }
        } else {
            e.mag = add(v.mag, dm);
            e.neg = true;
        }
        while (cmp(e.mag, c->Q.halfM) > 0) {   // wrap by q towards zero
            if (cmp(e.mag, c->Q.M) >= 0) sub_in(e.mag, c->Q.M);
            else { e.mag = sub(c->Q.M, e.mag); e.neg = !e.neg; }
        }
        double lg = -1.0;
        size_t bl = bitlen(e.mag);
        if (bl) {
            double top = 0;
            size_t sh = bl > 53 ? bl - 53 : 0;
            for (size_t b = bl; b-- > sh;) top = top * 2 + (testbit(e.mag, b) ? 1 : 0);
            lg = std::log2(top) + (double)sh;
        }
        worst = std::max(worst, lg);
    }
    return worst;
}

// ---- server side operations --------------------------------------------------------------------
// Mult without relinearization (textbook FV, see file header): out [3][L][N]
void orc_mult(const OrcCtx* c, const uint64_t* a, const uint64_t* b, uint64_t* out) {
    const uint32_t N = c->N, L = c->L;
    const size_t K = c->P.p.size();
    std::vector<uint64_t> A(2 * K * N), B(2 * K * N), X(3 * K * N);
    for (int poly = 0; poly < 2; ++poly)
        for (uint32_t i = 0; i < N; ++i) {
            SInt va = c->Q.lift_centered(a + (size_t)poly * L * N + i, N);
            SInt vb = c->Q.lift_centered(b + (size_t)poly * L * N + i, N);
            for (size_t k = 0; k < K; ++k) {
                A[((size_t)poly * K + k) * N + i] = residue(va, c->P.p[k]);
                B[((size_t)poly * K + k) * N + i] = residue(vb, c->P.p[k]);
            }
        }
    for (int poly = 0; poly < 2; ++poly)
        for (size_t k = 0; k < K; ++k) {
            c->pntt[k].forward(A.data() + ((size_t)poly * K + k) * N);
            c->pntt[k].forward(B.data() + ((size_t)poly * K + k) * N);
        }
    for (size_t k = 0; k < K; ++k) {
        uint64_t p = c->P.p[k];
        const uint64_t *a0 = A.data() + k * N, *a1 = A.data() + (K + k) * N;
        const uint64_t *b0 = B.data() + k * N, *b1 = B.data() + (K + k) * N;
        uint64_t *x0 = X.data() + k * N, *x1 = X.data() + (K + k) * N, *x2 = X.data() + (2 * K + k) * N;
        for (uint32_t i = 0; i < N; ++i) {
            x0[i] = mulm(a0[i], b0[i], p);
            x1[i] = addm(mulm(a0[i], b1[i], p), mulm(a1[i], b0[i], p), p);
            x2[i] = mulm(a1[i], b1[i], p);
        }
        for (int r = 0; r < 3; ++r) c->pntt[k].inverse(X.data() + ((size_t)r * K + k) * N);
    }
    for (int r = 0; r < 3; ++r)
        for (uint32_t i = 0; i < N; ++i) {
            SInt v = c->P.lift_centered(X.data() + (size_t)r * K * N + i, N);
            scale_round(c, v, out + (size_t)r * L * N + i, N);
        }
}

OrcKey* orc_load_rlk(const OrcCtx* c, const uint64_t* rlk) {
    const uint32_t N = c->N, L = c->L;
    OrcKey* k = new OrcKey();
    k->hat.assign(rlk, rlk + (size_t)L * 2 * L * N);
    for (uint32_t i = 0; i < L; ++i)
        for (int w = 0; w < 2; ++w)
            for (uint32_t j = 0; j < L; ++j) c->qntt[j].forward(k->hat.data() + (((size_t)i * 2 + w) * L + j) * N);
    return k;
}
void orc_key_free(OrcKey* k) { delete k; }

// Relinearization with per-limb digits: [3][L][N] -> [2][L][N]
void orc_relin(const OrcCtx* c, const OrcKey* key, const uint64_t* in, uint64_t* out) {
    const uint32_t N = c->N, L = c->L;
    std::vector<uint64_t> D(N), S0(N), S1(N);
    const uint64_t* c2 = in + (size_t)2 * L * N;
    for (uint32_t j = 0; j < L; ++j) {
        uint64_t p = c->qp[j];
        std::fill(S0.begin(), S0.end(), 0);
        std::fill(S1.begin(), S1.end(), 0);
        for (uint32_t i = 0; i < L; ++i) {
            for (uint32_t x = 0; x < N; ++x) D[x] = c2[(size_t)i * N + x] % p;  // digit i in [0,q_i)
            c->qntt[j].forward(D.data());
            const uint64_t* bh = key->hat.data() + (((size_t)i * 2 + 0) * L + j) * N;
            const uint64_t* ah = key->hat.data() + (((size_t)i * 2 + 1) * L + j) * N;
            for (uint32_t x = 0; x < N; ++x) {
                S0[x] = addm(S0[x], mulm(D[x], bh[x], p), p);
                S1[x] = addm(S1[x], mulm(D[x], ah[x], p), p);
            }
        }
        c->qntt[j].inverse(S0.data());
        c->qntt[j].inverse(S1.data());
        for (uint32_t x = 0; x < N; ++x) {
            out[(size_t)j * N + x] = addm(in[(size_t)j * N + x], S0[x], p);
            out[(size_t)(L + j) * N + x] = addm(in[(size_t)(L + j) * N + x], S1[x], p);
        }
    }
}

// PM: (c0 P, c1 P) with P's coefficients in [0, t) used as they are
void orc_pm(const OrcCtx* c, const uint64_t* ct, const uint64_t* pt, uint64_t* out) {
    const uint32_t N = c->N, L = c->L;
    std::vector<uint64_t> P(N);
    for (uint32_t j = 0; j < L; ++j) {
        for (uint32_t x = 0; x < N; ++x) P[x] = pt[x] % c->qp[j];
        for (int poly = 0; poly < 2; ++poly)
            poly_mul_mod(c, j, ct + ((size_t)poly * L + j) * N, P.data(), out + ((size_t)poly * L + j) * N);
    }
}

void orc_add(const OrcCtx* c, const uint64_t* a, const uint64_t* b, uint32_t size, uint64_t* out) {
    for (uint32_t r = 0; r < size; ++r)
        for (uint32_t j = 0; j < c->L; ++j)
            for (uint32_t x = 0; x < c->N; ++x) {
                size_t i = ((size_t)r * c->L + j) * c->N + x;
                out[i] = addm(a[i], b[i], c->qp[j]);
            }
}

// Selector for one element: product of the query ciphertexts at the codeword's one positions
// (ascending).  Each tree level pairs neighbours (0,1),(2,3),... into Relin(Mult(., .)); an odd
// last node moves up unchanged; k = 1 returns the query ciphertext itself.
void orc_selector(const OrcCtx* c, const OrcKey* key, const uint64_t* query, const uint32_t* pos, uint32_t k,
                  uint64_t* out) {
    const size_t ct = (size_t)2 * c->L * c->N;
    std::vector<std::vector<uint64_t>> level;
    for (uint32_t i = 0; i < k; ++i) level.emplace_back(query + pos[i] * ct, query + (pos[i] + 1) * ct);
    std::vector<uint64_t> c3(3 * c->L * c->N);
    while (level.size() > 1) {
        std::vector<std::vector<uint64_t>> next;
        for (size_t i = 0; i + 1 < level.size(); i += 2) {
            orc_mult(c, level[i].data(), level[i + 1].data(), c3.data());
            std::vector<uint64_t> r(ct);
            orc_relin(c, key, c3.data(), r.data());
            next.push_back(std::move(r));
        }
        if (level.size() % 2) next.push_back(level.back());
        level.swap(next);
    }
    std::memcpy(out, level[0].data(), ct * sizeof(uint64_t));
}

// PIR answer: answer_r = sum_j PM(sel_j, P_{j,r}) mod q over the n elements of the database.
// The modular sum is accumulated per thread in the transformed domain and summed at the end.
void orc_answer(const OrcCtx* c, const OrcKey* key, const uint64_t* query, uint32_t k, uint64_t n, uint32_t s,
                const uint32_t* codewords, const uint16_t* payload, uint64_t* answer, int nthreads) {
    const uint32_t N = c->N, L = c->L;
    const size_t ctsz = (size_t)2 * L * N;
    const size_t accsz = (size_t)s * ctsz;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    std::vector<std::vector<uint64_t>> accs(nthreads, std::vector<uint64_t>(accsz, 0));
#pragma omp parallel num_threads(nthreads)
    {
        std::vector<uint64_t>& acc = accs[omp_get_thread_num()];
        std::vector<uint64_t> sel(ctsz), selh(ctsz), P(N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t e = 0; e < (int64_t)n; ++e) {
            orc_selector(c, key, query, codewords + (size_t)e * k, k, sel.data());
            selh = sel;
            for (int poly = 0; poly < 2; ++poly)
                for (uint32_t j = 0; j < L; ++j) c->qntt[j].forward(selh.data() + ((size_t)poly * L + j) * N);
            for (uint32_t r = 0; r < s; ++r) {
                const uint16_t* pt = payload + ((size_t)e * s + r) * N;
                for (uint32_t j = 0; j < L; ++j) {
                    uint64_t p = c->qp[j];
                    for (uint32_t x = 0; x < N; ++x) P[x] = pt[x] % p;
                    c->qntt[j].forward(P.data());
                    for (int poly = 0; poly < 2; ++poly) {
                        const uint64_t* sh = selh.data() + ((size_t)poly * L + j) * N;
                        uint64_t* a = acc.data() + (size_t)r * ctsz + ((size_t)poly * L + j) * N;
                        for (uint32_t x = 0; x < N; ++x) a[x] = addm(a[x], mulm(sh[x], P[x], p), p);
                    }
                }
            }
        }
    }
    for (size_t i = 0; i < accsz; ++i) {
        uint32_t j = (uint32_t)((i / N) % L);
        uint64_t v = 0;
        for (int th = 0; th < nthreads; ++th) v = addm(v, accs[th][i], c->qp[j]);
        answer[i] = v;
    }
    for (uint32_t r = 0; r < s; ++r)
        for (int poly = 0; poly < 2; ++poly)
            for (uint32_t j = 0; j < L; ++j) c->qntt[j].inverse(answer + (size_t)r * ctsz + ((size_t)poly * L + j) * N);
}

// ---- query expansion (Section 3.3.3 "Query Expansion", Algorithm 5; Algorithm 1) ---------------
// The Galois automorphism x -> x^g (g odd) of R_q: coefficient i of a polynomial moves to position
// i g mod 2N and is negated when that position is N or more (x^N = -1).  Written as the direct
// definition: a scatter over the input coefficients.  in/out: [npoly][L][N], out != in.
void orc_automorphism(const OrcCtx* c, const uint64_t* in, uint32_t npoly, uint32_t g, uint64_t* out) {
    const uint32_t N = c->N, L = c->L;
    for (uint32_t r = 0; r < npoly * L; ++r) {
        const uint64_t p = c->qp[r % L];
        const uint64_t* a = in + (size_t)r * N;
        uint64_t* b = out + (size_t)r * N;
        for (uint32_t i = 0; i < N; ++i) {
            const uint64_t pos = (uint64_t)i * g % (2ull * N);
            if (pos < N) b[pos] = a[i];
            else b[pos - N] = a[i] ? p - a[i] : 0;
        }
    }
}

// Multiplication by the monomial x^e, 0 <= e < 2N: coefficient i moves to (i + e) mod 2N, negated
// past N.  in/out: [npoly][L][N], out != in.
void orc_mul_monomial(const OrcCtx* c, const uint64_t* in, uint32_t npoly, uint32_t e, uint64_t* out) {
    const uint32_t N = c->N, L = c->L;
    for (uint32_t r = 0; r < npoly * L; ++r) {
        const uint64_t p = c->qp[r % L];
        const uint64_t* a = in + (size_t)r * N;
        uint64_t* b = out + (size_t)r * N;
        for (uint32_t i = 0; i < N; ++i) {
            const uint64_t pos = ((uint64_t)i + e) % (2ull * N);
            if (pos < N) b[pos] = a[i];
            else b[pos - N] = a[i] ? p - a[i] : 0;
        }
    }
}

// Galois key for x -> x^g: gk_i = (b_i, a_i), b_i = [-a_i s + e_i + g_i s(x^g)]_q with the digits and
// g_i of the relinearization key.  Randomness layout as orc_relin_keygen.  gk: [L][2][L][N].
void orc_galois_keygen(const OrcCtx* c, const int8_t* sk, uint32_t g, const uint64_t* rnd_a,
                       const uint64_t* rnd_e, uint64_t* gk) {
    const uint32_t N = c->N, L = c->L;
    std::vector<int8_t> sg(N);  // s(x^g): a signed permutation of s, still ternary
    for (uint32_t i = 0; i < N; ++i) {
        const uint64_t pos = (uint64_t)i * g % (2ull * N);
        if (pos < N) sg[pos] = sk[i];
        else sg[pos - N] = (int8_t)-sk[i];
    }
    std::vector<uint64_t> s(N), sgm(N), as(N);
    for (uint32_t i = 0; i < L; ++i) {
        Big gi = mul_u64(c->Q.Mk[i], c->Q.inv[i]);
        for (uint32_t j = 0; j < L; ++j) {
            uint64_t p = c->qp[j];
            uint64_t* b = gk + (((size_t)i * 2 + 0) * L + j) * N;
            uint64_t* a = gk + (((size_t)i * 2 + 1) * L + j) * N;
            for (uint32_t x = 0; x < N; ++x) {
                size_t idx = (((size_t)i * L + j) * N + x) * 2;
                a[x] = uniform_mod(rnd_a[idx], rnd_a[idx + 1], p);
            }
            ternary_mod(sk, N, p, s.data());
            ternary_mod(sg.data(), N, p, sgm.data());
            poly_mul_mod(c, j, a, s.data(), as.data());
            uint64_t gm = mod_u64(gi, p);
            for (uint32_t x = 0; x < N; ++x) {
                uint64_t e = signed_mod(cbd21(rnd_e[(size_t)i * N + x]), p);
                b[x] = addm(subm(e, as[x], p), mulm(gm, sgm[x], p), p);
            }
        }
    }
}

// Substitution Sub_g(ct) (Section 2.1.1): the automorphism on both polynomials, then a key switch of
// the second back to s with the Galois key:
//   (sigma(c0) + sum_i D_i b_i, sum_i D_i a_i),  D_i = [sigma(c1)]_{q_i} in [0, q_i).
// That is the relinearization of the three-polynomial ciphertext (sigma(c0), 0, sigma(c1)) under gk.
void orc_sub(const OrcCtx* c, const OrcKey* gk, const uint64_t* ct, uint32_t g, uint64_t* out) {
    const size_t LN = (size_t)c->L * c->N;
    std::vector<uint64_t> sig(2 * LN), three(3 * LN, 0);
    orc_automorphism(c, ct, 2, g, sig.data());
    std::memcpy(three.data(), sig.data(), LN * 8);
    std::memcpy(three.data() + 2 * LN, sig.data() + LN, LN * 8);
    orc_relin(c, gk, three.data(), out);
}

// ---- response compression (modulus switching; Section 2.2, the SealPIR optimization the paper
// adopts for responses) --------------------------------------------------------------------------
// Every coefficient x of every polynomial, lifted to its centred representative modulo q, becomes
// round(q' x / q) = round(x / r) with q' = q_0 ... q_{keep-1} and r = q / q' (odd, so no ties),
// stored modulo q'.  in: [npoly][L][N]; out: [npoly][keep][N].
void orc_mod_switch(const OrcCtx* c, const uint64_t* in, uint32_t npoly, uint32_t keep, uint64_t* out) {
    const uint32_t N = c->N, L = c->L;
    Big r = big_u64(1);
    for (uint32_t j = keep; j < L; ++j) r = mul_u64(r, c->qp[j]);
    const Big twor = add(r, r);
    for (uint32_t poly = 0; poly < npoly; ++poly)
        for (uint32_t i = 0; i < N; ++i) {
            SInt x = c->Q.lift_centered(in + (size_t)poly * L * N + i, N);
            Big num = add(add(x.mag, x.mag), r);  // round(|x| / r) = floor((2|x| + r) / (2r))
            Big y, rem;
            divmod(num, twor, y, rem);
            for (uint32_t j = 0; j < keep; ++j) {
                uint64_t v = mod_u64(y, c->qp[j]);
                out[((size_t)poly * keep + j) * N + i] = (x.neg && v) ? c->qp[j] - v : v;
            }
        }
}

// ---- folklore PIR (Section 2.4, the plain folklore equality operator) ------------------------------
// 1 - ct: the plaintext constant 1 minus a ciphertext, (Delta - c0, -c1) mod q.  in/out [2][L][N].
void orc_one_minus(const OrcCtx* c, const uint64_t* ct, uint64_t* out) {
    const uint32_t N = c->N, L = c->L;
    for (uint32_t j = 0; j < L; ++j) {
        const uint64_t p = c->qp[j];
        for (uint32_t x = 0; x < N; ++x) {
            const uint64_t c0 = ct[(size_t)j * N + x], c1 = ct[(size_t)(L + j) * N + x];
            out[(size_t)j * N + x] = subm(x == 0 ? c->delta_r[j] : 0, c0, p);
            out[(size_t)(L + j) * N + x] = subm(0, c1, p);
        }
    }
}

}  // extern "C"
