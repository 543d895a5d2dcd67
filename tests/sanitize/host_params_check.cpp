// Host-side parameter construction of the library (auxiliary primes, constant tables, twiddles,
// switch constants, binomial tables) for the workload prime sets and two mixed ones, with checks of
// the lazy conversion flags, floor(2^64 / r), the fold constants, the folded inverse twiddles and
// the scale's centred v-term constant; the test that
// builds this file compiles it with AddressSanitizer and UndefinedBehaviorSanitizer (host code only).
#include <cstdio>
#include <vector>
#include "host_params.h"
using namespace cw;
int main() {
    struct Cfg { uint32_t N; std::vector<uint64_t> q; };
    std::vector<Cfg> cfgs = {
        {4096, {0xffffee001ull, 0xffffc4001ull, 0xffffbe001ull}},
        {8192, {0x7fffffd8001ull, 0x7fffffc8001ull, 0xfffffffc001ull, 0xffffff6c001ull, 0xfffffebc001ull}},
        {16384, {0x3fffffffef8001ull, 0x3fffffffeb8001ull, 0x7fffffffe90001ull, 0x7fffffffd58001ull,
                 0x7fffffffbf0001ull, 0x7fffffffbd0001ull, 0x7fffffffba0001ull, 0x7fffffffb58001ull}},
        {4096, {0x3ffffff84001ull, 0xfffffdc001ull, 0x7ffe6001ull}},
        {4096, {0x1fffffffce001ull, 0x1fffffff96001ull, 0x1ffffffce001ull}},
    };
    for (auto& c : cfgs) {
        std::string why = host::validate(c.N, c.q, 65537);
        if (!why.empty()) { printf("invalid: %s\n", why.c_str()); return 1; }
        for (uint64_t below : {1ull << 50, (unsigned long long)CONV_LAZY_BOUND, 1ull << 61}) {
            auto B = host::aux_primes(c.N, c.q, 65537, below);
            static CtxConst K;
            host::build_const(K, c.N, c.q, B, 65537);
            std::vector<uint64_t> all = c.q;
            all.insert(all.end(), B.begin(), B.end());
            std::vector<uint64_t> tw;
            host::build_twiddles(tw, all, c.N);
            std::vector<double> twf;
            host::build_twiddles_fp(twf, tw, all, c.N, K);
            // conversion tables: lazy exactly when every output prime is below 2^59; floor(2^64 / r)
            bool qlazy = true, blazy = true;
            for (uint64_t b : B) blazy = blazy && b < CONV_LAZY_BOUND;
            for (uint64_t p : c.q) qlazy = qlazy && p < CONV_LAZY_BOUND;
            if (K.qb.lazy != (blazy ? 1u : 0u) || K.bq.lazy != (qlazy ? 1u : 0u)) { printf("lazy flag\n"); return 1; }
            for (const ConvTable* T : {&K.qb, &K.bq})
                for (uint32_t j = 0; j < T->nout; ++j) {
                    const unsigned __int128 r = T->pout[j], lo = (unsigned __int128)T->r1[j] * r;
                    if (lo > ((unsigned __int128)1 << 64) || ((unsigned __int128)1 << 64) - lo >= r) { printf("r1\n"); return 1; }
                }
            // fold constants and the folded inverse twiddle row (fp64 path: every prime below 2^50):
            // [w_inv f]_p times f^-1 gives w_inv back
            const uint32_t L = (uint32_t)c.q.size();
            bool fp = true;
            for (uint64_t p : all) fp = fp && p < FP_PRIME_BOUND;
            for (uint32_t k = 0; fp && k < all.size(); ++k) {
                const uint64_t f = k < L ? K.tqinv[k] : K.kb1[k - L], p = all[k];
                if (K.foldd[k] != (double)f) { printf("foldd\n"); return 1; }
                const uint64_t finv = host::invmod(f, p);
                for (uint32_t i = 0; i < c.N; i += 97) {
                    const uint64_t w3 = (uint64_t)twf[(size_t)k * 4 * c.N + 3 * (size_t)c.N + i];
                    if (host::mulmod(w3, finv, p) != tw[(size_t)k * 4 * c.N + 2 * (size_t)c.N + i]) { printf("row 3\n"); return 1; }
                }
            }
            // the fp64 scale's v-term constant: centred, and [kb2 (q mod b)]_b
            for (uint32_t j = 0; fp && j < B.size(); ++j) {
                const double b = (double)B[j], f = K.fqpd[j];
                if (!(f > -b / 2 && f < b / 2)) { printf("fqpd range\n"); return 1; }
                const uint64_t fr = f < 0 ? B[j] - (uint64_t)(-f) : (uint64_t)f;
                if (fr != host::mulmod(K.kb2[j], K.qb.Pm[j], B[j])) { printf("fqpd value\n"); return 1; }
            }
            for (uint32_t keep = 1; keep <= c.q.size(); ++keep) {
                static SwitchConst S;
                host::build_switch(S, c.q, keep);
            }
            printf("N=%u L=%zu below=2^%d: %zu aux primes, %zu twiddles\n", c.N, c.q.size(),
                   63 - __builtin_clzll(below), B.size(), tw.size());
        }
    }
    for (uint32_t m : {24u, 27u, 569u, 725u})
        for (uint32_t k : {1u, 2u, 4u, 16u}) (void)host::binom_table(m, k);
    printf("ok\n");
    return 0;
}
