// Host-side parameter construction (see host_params.cpp).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "consts.h"

namespace cw {
namespace host {

uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p);
uint64_t powmod(uint64_t a, uint64_t e, uint64_t p);
uint64_t invmod(uint64_t a, uint64_t p);
uint64_t shoup(uint64_t w, uint64_t p);
bool is_prime(uint64_t n);
uint64_t find_psi(uint64_t p, uint32_t N);

// "" when (N, q, t) is supported, else the reason.
std::string validate(uint32_t N, const std::vector<uint64_t>& q, uint64_t t);
// Largest primes = 1 mod 2N below `below`, not in q, until their product exceeds 4 t N q.
std::vector<uint64_t> aux_primes(uint32_t N, const std::vector<uint64_t>& q, uint64_t t, uint64_t below);
// D: extra primes whose per-prime constants follow Q and B (no conversion tables).
void build_const(CtxConst& K, uint32_t N, const std::vector<uint64_t>& q, const std::vector<uint64_t>& B,
                 uint64_t t, const std::vector<uint64_t>& D = {});
// `count` largest primes = 1 mod 2N below `below` that are not in `avoid`.
std::vector<uint64_t> primes_below(uint32_t N, uint64_t below, uint32_t count, const std::vector<uint64_t>& avoid);
// [prime][4][N]: psi^bitrev(i), its Shoup companion, psi^-bitrev(i), its Shoup companion.
void build_twiddles(std::vector<uint64_t>& tw, const std::vector<uint64_t>& primes, uint32_t N);
// The same tables as doubles: [prime][4][N] = w, w/p, w_inv, [w_inv f]_p (fp64 transform), where f
// is the prime's fold constant (K.foldd: tqinv for Q, kb1 for B, 1 for the digit-sum primes).
void build_twiddles_fp(std::vector<double>& twf, const std::vector<uint64_t>& tw, const std::vector<uint64_t>& primes,
                       uint32_t N, const CtxConst& K);
std::vector<uint64_t> binom_table(uint32_t m, uint32_t k);
// Constants of the switch from q to its first `keep` primes.
void build_switch(SwitchConst& S, const std::vector<uint64_t>& q, uint32_t keep);
// Constants of the CRT from {b0, b1} to the ciphertext primes q (deferred key switch).
void build_crt(CrtConst& cc, const std::vector<uint64_t>& q, uint64_t b0, uint64_t b1);

}  // namespace host
}  // namespace cw
