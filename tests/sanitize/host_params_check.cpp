// Host-side parameter construction of the library (auxiliary primes, constant tables, twiddles,
// switch constants, binomial tables) for the workload prime sets and two mixed ones; the test that
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
        for (uint64_t below : {1ull << 50, 1ull << 61}) {
            auto B = host::aux_primes(c.N, c.q, 65537, below);
            static CtxConst K;
            host::build_const(K, c.N, c.q, B, 65537);
            std::vector<uint64_t> all = c.q;
            all.insert(all.end(), B.begin(), B.end());
            std::vector<uint64_t> tw;
            host::build_twiddles(tw, all, c.N);
            std::vector<double> twf;
            host::build_twiddles_fp(twf, tw, all, c.N, K);
            for (uint32_t keep = 1; keep <= c.q.size(); ++keep) {
                static SwitchConst S;
                host::build_switch(S, c.q, keep);
            }
            printf("N=%u L=%zu below=2^%d: %zu aux primes, %zu twiddles\n", c.N, c.q.size(),
                   below == (1ull << 50) ? 50 : 61, B.size(), tw.size());
        }
    }
    for (uint32_t m : {24u, 27u, 569u, 725u})
        for (uint32_t k : {1u, 2u, 4u, 16u}) (void)host::binom_table(m, k);
    printf("ok\n");
    return 0;
}
