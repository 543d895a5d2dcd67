// Seeded query ciphertexts on gfx950: regenerate the uniform second polynomial of secret-key
// ciphertexts from the client's 64-bit seed (the compressed upload of secret-key encryption that
// the paper lists among SealPIR's optimisations, Section 2).
//
// Generator: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) started from state `seed`; word v of
// the sequence is mix(seed + (v + 1) gamma mod 2^64), so every word is computed on its own thread.
// Residue (ciphertext i, limb j, coefficient c), u = (i L + j) N + c, is the two-word draw
//   a = (W(2u) 2^64 + W(2u + 1)) mod q_j.
#include <hip/hip_runtime.h>

#include "arith.h"
#include "kernels.h"

namespace cw {

namespace {

constexpr int SEED_THREADS = 256;
constexpr uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t sm64_word(uint64_t seed, uint64_t v) {
    uint64_t z = seed + (v + 1) * GOLDEN_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// out [count][2][L][N]: out[i][0] = c0[i], out[i][1] = a_i.  One thread per residue; consecutive
// threads take consecutive coefficients of one limb (coalesced loads and stores).
__global__ __launch_bounds__(SEED_THREADS) void k_seeded_query(const CtxConst* __restrict__ K,
                                                              const uint64_t* __restrict__ c0, size_t total,
                                                              uint64_t seed, uint64_t* __restrict__ out) {
    const size_t u = (size_t)blockIdx.x * SEED_THREADS + threadIdx.x;
    if (u >= total) return;
    const size_t LN = (size_t)K->L * K->N;
    const size_t i = u / LN, r = u % LN;
    const uint32_t j = (uint32_t)(r / K->N);
    const uint64_t p = K->p[j], r1 = K->r1[j];
    const uint64_t w1 = sm64_word(seed, 2 * (uint64_t)u), w2 = sm64_word(seed, 2 * (uint64_t)u + 1);
    const uint64_t two64 = 0ull - r1 * p;  // 2^64 - floor(2^64 / p) p = 2^64 mod p
    const uint64_t a = add_mod(mul_barrett(reduce64(w1, p, r1), two64, p, K->bar_mu[j], K->bar_s[j]),
                               reduce64(w2, p, r1), p);
    uint64_t* o = out + i * 2 * LN + r;
    o[0] = c0[u];
    o[LN] = a;
}

}  // namespace

void launch_seeded_query(const Launch& lc, const uint64_t* c0, uint32_t count, uint64_t seed, uint64_t* out) {
    const size_t total = (size_t)count * lc.L * lc.N;
    if (!total) return;
    const unsigned blocks = (unsigned)((total + SEED_THREADS - 1) / SEED_THREADS);
    hipLaunchKernelGGL(k_seeded_query, dim3(blocks), dim3(SEED_THREADS), 0, lc.stream, lc.K, c0, total, seed, out);
}

}  // namespace cw
