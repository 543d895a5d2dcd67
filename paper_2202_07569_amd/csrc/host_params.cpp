// Host-side number theory for one parameter set: auxiliary primes, transform twiddles, Barrett and
// Shoup constants and the exact base-conversion tables (consts.h).
#include "host_params.h"

#include <algorithm>
#include <cstring>

namespace cw {
namespace host {

typedef unsigned __int128 u128;

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }
uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulmod(r, a, p);
        a = mulmod(a, a, p);
        e >>= 1;
    }
    return r;
}
uint64_t invmod(uint64_t a, uint64_t p) { return powmod(a, p - 2, p); }
uint64_t shoup(uint64_t w, uint64_t p) { return (uint64_t)(((u128)w << 64) / p); }

bool is_prime(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t b : bases)
        if (n % b == 0) return n == b;
    uint64_t d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    for (uint64_t a : bases) {
        uint64_t x = powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool composite = true;
        for (int r = 1; r < s && composite; ++r) {
            x = mulmod(x, x, n);
            if (x == n - 1) composite = false;
        }
        if (composite) return false;
    }
    return true;
}

static uint32_t bitlen64(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

// ---- multiword unsigned integers (little-endian) ----
typedef std::vector<uint64_t> MW;
static void mw_trim(MW& a) { while (!a.empty() && a.back() == 0) a.pop_back(); }
static MW mw_mul(const MW& a, uint64_t m) {
    MW r(a.size() + 1);
    u128 c = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        c += (u128)a[i] * m;
        r[i] = (uint64_t)c;
        c >>= 64;
    }
    r[a.size()] = (uint64_t)c;
    mw_trim(r);
    return r;
}
static uint64_t mw_mod(const MW& a, uint64_t p) {
    u128 r = 0;
    for (size_t i = a.size(); i-- > 0;) r = ((r << 64) | a[i]) % p;
    return (uint64_t)r;
}
static size_t mw_bits(const MW& a) { return a.empty() ? 0 : 64 * (a.size() - 1) + bitlen64(a.back()); }
static int mw_cmp(const MW& a, const MW& b) {
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}
static MW mw_prod(const std::vector<uint64_t>& ps, int skip = -1) {
    MW r{1};
    for (size_t i = 0; i < ps.size(); ++i)
        if ((int)i != skip) r = mw_mul(r, ps[i]);
    return r;
}

uint64_t find_psi(uint64_t p, uint32_t N) {
    for (uint64_t g = 2;; ++g) {
        uint64_t x = powmod(g, (p - 1) / (2ull * N), p);
        if (powmod(x, N, p) == p - 1) return x;
    }
}

std::string validate(uint32_t N, const std::vector<uint64_t>& q, uint64_t t) {
    if (N != 4096 && N != 8192 && N != 16384) return "N must be 4096, 8192 or 16384";
    if (q.empty() || q.size() > (size_t)MAX_L) return "L out of range";
    if (t < 2 || t >= (1ull << 32)) return "t must be in [2, 2^32)";
    for (size_t i = 0; i < q.size(); ++i) {
        uint64_t p = q[i];
        if (p <= (1ull << 30) || p >= (1ull << 61)) return "each q_i must lie in (2^30, 2^61)";
        if (p % (2ull * N) != 1) return "each q_i must be 1 mod 2N";
        if (!is_prime(p)) return "q_i is not prime";
        if (t % p == 0) return "t must be coprime to q";
        for (size_t j = 0; j < i; ++j)
            if (q[j] == p) return "primes must be distinct";
    }
    return "";
}

std::vector<uint64_t> aux_primes(uint32_t N, const std::vector<uint64_t>& q, uint64_t t, uint64_t below) {
    // B > 4 t N q: holds round(t X / q) and, with q, every exact tensor product.
    MW bound = mw_mul(mw_mul(mw_prod(q), t), 4ull * N);
    std::vector<uint64_t> B;
    MW prod{1};
    const uint64_t step = 2ull * N;
    uint64_t c = (below - 1) / step * step + 1;
    if (c >= below) c -= step;
    while (mw_cmp(prod, bound) <= 0) {
        if (is_prime(c) && std::find(q.begin(), q.end(), c) == q.end()) {
            B.push_back(c);
            prod = mw_mul(prod, c);
        }
        c -= step;
    }
    return B;
}

static void build_conv(ConvTable& T, const std::vector<uint64_t>& in, const std::vector<uint64_t>& out) {
    std::memset(&T, 0, sizeof(T));
    T.nin = (uint32_t)in.size();
    T.nout = (uint32_t)out.size();
    MW P = mw_prod(in);
    T.W = (uint32_t)((mw_bits(P) + 63) / 64);
    for (size_t w = 0; w < P.size(); ++w) T.Pw[w] = P[w];
    for (size_t i = 0; i < in.size(); ++i) {
        T.pin[i] = in[i];
        u128 om = (~(u128)0) / in[i];  // floor(2^128 / p) for odd p
        T.om_hi[i] = (uint64_t)(om >> 64);
        T.om_lo[i] = (uint64_t)om;
        MW Ph = mw_prod(in, (int)i);
        for (size_t w = 0; w < Ph.size(); ++w) T.Phat[i][w] = Ph[w];
        for (size_t j = 0; j < out.size(); ++j) {
            T.M[i][j] = mw_mod(Ph, out[j]);
            T.Mq[i][j] = shoup(T.M[i][j], out[j]);
            T.Md[i][j] = (double)T.M[i][j];
        }
    }
    T.lazy = 1;
    for (size_t j = 0; j < out.size(); ++j) {
        T.pout[j] = out[j];
        T.r1[j] = (uint64_t)(((u128)1 << 64) / out[j]);
        if (out[j] >= CONV_LAZY_BOUND) T.lazy = 0;
        T.Pm[j] = mw_mod(P, out[j]);
        T.Pmq[j] = shoup(T.Pm[j], out[j]);
        T.Pmd[j] = (double)T.Pm[j];
    }
}

std::vector<uint64_t> primes_below(uint32_t N, uint64_t below, uint32_t count, const std::vector<uint64_t>& avoid) {
    std::vector<uint64_t> out;
    const uint64_t step = 2ull * N;
    uint64_t c = (below - 1) / step * step + 1;
    if (c >= below) c -= step;
    while (out.size() < count && c > step) {
        if (is_prime(c) && std::find(avoid.begin(), avoid.end(), c) == avoid.end()) out.push_back(c);
        c -= step;
    }
    return out;
}

void build_const(CtxConst& K, uint32_t N, const std::vector<uint64_t>& q, const std::vector<uint64_t>& B,
                 uint64_t t, const std::vector<uint64_t>& D) {
    std::memset(&K, 0, sizeof(K));
    K.N = N;
    K.logN = bitlen64(N) - 1;
    K.L = (uint32_t)q.size();
    K.LB = (uint32_t)B.size();
    K.LL = K.L + K.LB;
    K.t = t;
    std::vector<uint64_t> all(q);
    all.insert(all.end(), B.begin(), B.end());
    all.insert(all.end(), D.begin(), D.end());
    for (uint32_t i = 0; i < (uint32_t)all.size(); ++i) {
        uint64_t p = all[i];
        K.p[i] = p;
        uint32_t s = bitlen64(p);
        K.bar_s[i] = s;
        K.bar_mu[i] = (uint64_t)(((u128)1 << (2 * s)) / p);
        K.r1[i] = (~0ull) / p;
        K.ninv[i] = invmod(N % p, p);
        K.ninvq[i] = shoup(K.ninv[i], p);
        K.pd[i] = (double)p;
        K.pinv[i] = 1.0 / (double)p;
        K.ninvd[i] = (double)K.ninv[i];
        K.ninvdq[i] = (double)K.ninv[i] / (double)p;
    }
    MW Q = mw_prod(q), BB = mw_prod(B);
    {
        MW delta(Q.size(), 0);  // floor(Q / t) by long division in 64-bit digits
        u128 rem = 0;
        for (size_t w = Q.size(); w-- > 0;) {
            const u128 cur = (rem << 64) | Q[w];
            delta[w] = (uint64_t)(cur / t);
            rem = cur % t;
        }
        mw_trim(delta);
        for (uint32_t i = 0; i < K.L; ++i) K.delta[i] = mw_mod(delta, q[i]);
    }
    for (uint32_t i = 0; i < K.L; ++i) {
        uint64_t p = q[i];
        uint64_t qhat = mw_mod(mw_prod(q, (int)i), p);
        K.qinv[i] = invmod(qhat, p);
        K.qinvq[i] = shoup(K.qinv[i], p);
        // the scale kernels read the tensor products without the inverse transform's N^-1 (it is
        // folded here and into kb1): tqinv = t (q/q_i)^-1 N^-1
        K.tqinv[i] = mulmod(mulmod(t % p, K.qinv[i], p), invmod(N % p, p), p);
        K.tqinvq[i] = shoup(K.tqinv[i], p);
        K.tqinvd[i] = (double)K.tqinv[i];
    }
    for (uint32_t j = 0; j < K.LB; ++j) {
        uint64_t b = B[j];
        uint64_t qinv_b = invmod(mw_mod(Q, b), b);
        uint64_t bhat_inv = invmod(mw_mod(mw_prod(B, (int)j), b), b);
        K.kb2[j] = mulmod(qinv_b, bhat_inv, b);
        K.kb2q[j] = shoup(K.kb2[j], b);
        K.kb1[j] = mulmod(mulmod(t % b, K.kb2[j], b), invmod(N % b, b), b);  // with N^-1, like tqinv
        K.kb1q[j] = shoup(K.kb1[j], b);
        K.kb1d[j] = (double)K.kb1[j];
        K.kb2d[j] = (double)K.kb2[j];
    }
    build_conv(K.qb, q, B);
    build_conv(K.bq, B, q);
    for (uint32_t j = 0; j < K.LB; ++j) {
        const uint64_t b = B[j];
        for (uint32_t i = 0; i < K.L; ++i) K.fqbd[i][j] = (double)mulmod(b - K.kb2[j], K.qb.M[i][j], b);
        const uint64_t f = mulmod(K.kb2[j], K.qb.Pm[j], b);
        K.fqpd[j] = f > b / 2 ? -(double)(b - f) : (double)f;  // centred
    }
    for (uint32_t k = 0; k < cw::MAX_LL; ++k) K.foldd[k] = 1.0;
    for (uint32_t i = 0; i < K.L; ++i) K.foldd[i] = K.tqinvd[i];
    for (uint32_t j = 0; j < K.LB; ++j) K.foldd[K.L + j] = K.kb1d[j];
}

void build_switch(SwitchConst& S, const std::vector<uint64_t>& q, uint32_t keep) {
    std::memset(&S, 0, sizeof(S));
    S.keep = keep;
    S.L = (uint32_t)q.size();
    const std::vector<uint64_t> kept(q.begin(), q.begin() + keep), dropped(q.begin() + keep, q.end());
    if (dropped.empty()) return;
    build_conv(S.T, dropped, kept);
    for (size_t i = 0; i < dropped.size(); ++i) {
        S.yc[i] = invmod(mw_mod(mw_prod(dropped, (int)i), dropped[i]), dropped[i]);
        S.ycq[i] = shoup(S.yc[i], dropped[i]);
    }
    const MW r = mw_prod(dropped);
    for (size_t j = 0; j < kept.size(); ++j) {
        S.rinv[j] = invmod(mw_mod(r, kept[j]), kept[j]);
        S.rinvq[j] = shoup(S.rinv[j], kept[j]);
    }
}

void build_crt(CrtConst& cc, const std::vector<uint64_t>& q, uint64_t b0, uint64_t b1) {
    std::memset(&cc, 0, sizeof(cc));
    cc.b0inv = invmod(b0 % b1, b1);
    cc.b0invq = shoup(cc.b0inv, b1);
    const u128 half = ((u128)b0 * b1 - 1) / 2;  // b0 b1 is odd
    cc.half_hi = (uint64_t)(half >> 64);
    cc.half_lo = (uint64_t)half;
    for (size_t j = 0; j < q.size(); ++j) {
        cc.b0q[j] = b0 % q[j];
        cc.b0qq[j] = shoup(cc.b0q[j], q[j]);
        cc.Bq[j] = mulmod(b0 % q[j], b1 % q[j], q[j]);
    }
}

static uint32_t bitrev(uint32_t x, uint32_t logn) {
    uint32_t r = 0;
    for (uint32_t b = 0; b < logn; ++b)
        if (x & (1u << b)) r |= 1u << (logn - 1 - b);
    return r;
}

void build_twiddles_fp(std::vector<double>& twf, const std::vector<uint64_t>& tw, const std::vector<uint64_t>& primes,
                       uint32_t N, const CtxConst& K) {
    twf.assign(tw.size(), 0.0);
    for (size_t k = 0; k < primes.size(); ++k) {
        const uint64_t p = primes[k];
        const uint64_t f = k < K.L ? K.tqinv[k] : k < K.LL ? K.kb1[k - K.L] : 1;  // the fold constant
        const uint64_t* src = tw.data() + k * 4 * (size_t)N;
        double* dst = twf.data() + k * 4 * (size_t)N;
        for (uint32_t i = 0; i < N; ++i) {
            dst[i] = (double)src[i];                          // exact: below 2^53
            dst[N + i] = (double)src[i] / (double)p;          // w / p, correctly rounded
            dst[2 * N + i] = (double)src[2 * N + i];
            dst[3 * N + i] = (double)mulmod(src[2 * N + i], f, p);  // w_inv times the prime's fold constant
        }
    }
}

void build_twiddles(std::vector<uint64_t>& tw, const std::vector<uint64_t>& primes, uint32_t N) {
    uint32_t logn = bitlen64(N) - 1;
    tw.assign(primes.size() * 4 * (size_t)N, 0);
    std::vector<uint64_t> pw(N), pwi(N);
    for (size_t k = 0; k < primes.size(); ++k) {
        uint64_t p = primes[k];
        uint64_t psi = find_psi(p, N), psii = invmod(psi, p);
        pw[0] = pwi[0] = 1;
        for (uint32_t i = 1; i < N; ++i) {
            pw[i] = mulmod(pw[i - 1], psi, p);
            pwi[i] = mulmod(pwi[i - 1], psii, p);
        }
        uint64_t* base = tw.data() + k * 4 * (size_t)N;
        for (uint32_t i = 0; i < N; ++i) {
            uint32_t r = bitrev(i, logn);
            base[i] = pw[r];
            base[N + i] = shoup(pw[r], p);
            base[2 * N + i] = pwi[r];
            base[3 * N + i] = shoup(pwi[r], p);
        }
    }
}

// Saturating binomial table C(a, h) for a < m, h <= k (row-major [a][h]).
std::vector<uint64_t> binom_table(uint32_t m, uint32_t k) {
    std::vector<uint64_t> T((size_t)m * (k + 1), 0);
    for (uint32_t a = 0; a < m; ++a) {
        for (uint32_t h = 0; h <= k; ++h) {
            uint64_t v;
            if (h == 0) v = 1;
            else if (a == 0) v = 0;
            else {
                uint64_t x = T[(size_t)(a - 1) * (k + 1) + h - 1], y = T[(size_t)(a - 1) * (k + 1) + h];
                v = (x > ~0ull - y) ? ~0ull : x + y;
            }
            T[(size_t)a * (k + 1) + h] = v;
        }
    }
    return T;
}

}  // namespace host
}  // namespace cw
