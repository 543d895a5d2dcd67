// HIP kernels for gfx950 of the constant-weight PIR server path.
//
// Data layout in HBM (u64 residues, limb-major inside a polynomial, N coefficients per limb):
//   extended ciphertext  [2][LL][N]   over Q then B, transformed (NTT domain)
//   tensor product       [E][3][LL][N]
//   relin staging        [E][L+2][L][N]  rows 0..L-1: digit i reduced mod q_j; rows L, L+1: c0, c1
//   selector             [E][2][L][N]  transformed over Q
//   payload transform    [E][s][L][N]
//   accumulator/answer   [s][2][L][N]
// A "limb-poly" is one row of N residues; its prime is prime_base + (row index mod nl).
#include <hip/hip_runtime.h>

#include "arith.h"
#include "kernels.h"

namespace cw {

constexpr int EW_THREADS = 256;

static inline unsigned blocks_for(size_t n, int t = EW_THREADS) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------------------------
// Negacyclic NTT, one workgroup per limb-poly, the whole limb resident in LDS.
// Forward: Cooley-Tukey with the psi powers merged into the twiddles (psi^bitrev), natural order in,
// bit-reversed order out.  Inverse: Gentleman-Sande with psi^-bitrev, bit-reversed in, natural out,
// scaled by N^-1.  Pointwise products of two forward transforms are negacyclic products.
// ---------------------------------------------------------------------------------------------
template <int LOGN>
__device__ __forceinline__ void ntt_fwd_lds(uint64_t* sm, const uint64_t* __restrict__ psi,
                                            const uint64_t* __restrict__ psiq, uint64_t p) {
    constexpr int N = 1 << LOGN;
#pragma unroll 1
    for (int lt = LOGN - 1, m = 1; lt >= 0; --lt, m <<= 1) {
        const int t = 1 << lt;
        for (int b = threadIdx.x; b < N / 2; b += NTT_THREADS) {
            const int i = b >> lt, j = b & (t - 1);
            const int j1 = (i << (lt + 1)) + j;
            const uint64_t w = psi[m + i], wq = psiq[m + i];
            const uint64_t U = sm[j1];
            const uint64_t V = mul_shoup(sm[j1 + t], w, wq, p);
            sm[j1] = add_mod(U, V, p);
            sm[j1 + t] = sub_mod(U, V, p);
        }
        __syncthreads();
    }
}

template <int LOGN>
__device__ __forceinline__ void ntt_inv_lds(uint64_t* sm, const uint64_t* __restrict__ psi,
                                            const uint64_t* __restrict__ psiq, uint64_t p) {
    constexpr int N = 1 << LOGN;
#pragma unroll 1
    for (int lt = 0, m = N / 2; lt < LOGN; ++lt, m >>= 1) {
        const int t = 1 << lt;
        for (int b = threadIdx.x; b < N / 2; b += NTT_THREADS) {
            const int i = b >> lt, j = b & (t - 1);
            const int j1 = (i << (lt + 1)) + j;
            const uint64_t w = psi[m + i], wq = psiq[m + i];
            const uint64_t U = sm[j1], V = sm[j1 + t];
            sm[j1] = add_mod(U, V, p);
            sm[j1 + t] = mul_shoup(sub_mod(U, V, p), w, wq, p);
        }
        __syncthreads();
    }
}

template <int LOGN>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_fwd(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                         const uint64_t* in, uint64_t* out, uint32_t nl,
                                                         uint32_t pbase) {
    constexpr int N = 1 << LOGN;
    extern __shared__ uint64_t sm[];
    const size_t g = blockIdx.x;
    const uint32_t pi = pbase + (uint32_t)(g % nl);
    const uint64_t p = K->p[pi];
    const uint64_t* psi = tw + (size_t)pi * 4 * N;
    const uint64_t* src = in + g * N;
    for (int i = threadIdx.x; i < N; i += NTT_THREADS) sm[i] = src[i];
    __syncthreads();
    ntt_fwd_lds<LOGN>(sm, psi, psi + N, p);
    uint64_t* dst = out + g * N;
    for (int i = threadIdx.x; i < N; i += NTT_THREADS) dst[i] = sm[i];
}

template <int LOGN>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_inv(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                         const uint64_t* in, uint64_t* out, uint32_t nl,
                                                         uint32_t pbase) {
    constexpr int N = 1 << LOGN;
    extern __shared__ uint64_t sm[];
    const size_t g = blockIdx.x;
    const uint32_t pi = pbase + (uint32_t)(g % nl);
    const uint64_t p = K->p[pi];
    const uint64_t* psi = tw + (size_t)pi * 4 * N + 2 * N;
    const uint64_t* src = in + g * N;
    for (int i = threadIdx.x; i < N; i += NTT_THREADS) sm[i] = src[i];
    __syncthreads();
    ntt_inv_lds<LOGN>(sm, psi, psi + N, p);
    const uint64_t ni = K->ninv[pi], niq = K->ninvq[pi];
    uint64_t* dst = out + g * N;
    for (int i = threadIdx.x; i < N; i += NTT_THREADS) dst[i] = mul_shoup(sm[i], ni, niq, p);
}

// Payload rows: block g = (e s + r) L + j lifts uint16 row (e, r) (values < 2^16 < q_j, so the
// residue is the value itself) and transforms it modulo q_j.
template <int LOGN>
__global__ __launch_bounds__(NTT_THREADS) void k_ntt_payload(const CtxConst* __restrict__ K,
                                                             const uint64_t* __restrict__ tw,
                                                             const uint16_t* __restrict__ pay,
                                                             uint64_t* __restrict__ out) {
    constexpr int N = 1 << LOGN;
    extern __shared__ uint64_t sm[];
    const uint32_t L = K->L;
    const size_t g = blockIdx.x;
    const uint32_t pi = (uint32_t)(g % L);
    const uint64_t p = K->p[pi];
    const uint64_t* psi = tw + (size_t)pi * 4 * N;
    const uint16_t* src = pay + (g / L) * N;
    for (int i = threadIdx.x; i < N; i += NTT_THREADS) sm[i] = src[i];
    __syncthreads();
    ntt_fwd_lds<LOGN>(sm, psi, psi + N, p);
    uint64_t* dst = out + g * N;
    for (int i = threadIdx.x; i < N; i += NTT_THREADS) dst[i] = sm[i];
}

void launch_ntt(const Launch& lc, bool inverse, const uint64_t* in, uint64_t* out, size_t rows, uint32_t nl,
                uint32_t pbase) {
    if (!rows) return;
    const size_t lds = (size_t)lc.N * 8;
    dim3 grid((unsigned)rows), block(NTT_THREADS);
#define CW_NTT_CASE(LG)                                                                                          \
    case LG:                                                                                                     \
        if (inverse)                                                                                             \
            hipLaunchKernelGGL(k_ntt_inv<LG>, grid, block, lds, lc.stream, lc.K, lc.tw, in, out, nl, pbase);   \
        else                                                                                                     \
            hipLaunchKernelGGL(k_ntt_fwd<LG>, grid, block, lds, lc.stream, lc.K, lc.tw, in, out, nl, pbase);   \
        break;
    switch (lc.logN) {
        CW_NTT_CASE(12)
        CW_NTT_CASE(13)
        CW_NTT_CASE(14)
    }
#undef CW_NTT_CASE
}

// Let the transform kernels use the whole limb in dynamic LDS (128 KiB at N = 16384).
hipError_t kernels_init() {
    hipError_t e = hipSuccess;
#define CW_ATTR(K, LG)                                                                                  \
    if (e == hipSuccess)                                                                                \
        e = hipFuncSetAttribute((const void*)K<LG>, hipFuncAttributeMaxDynamicSharedMemorySize, 8 << LG);
    CW_ATTR(k_ntt_fwd, 12) CW_ATTR(k_ntt_fwd, 13) CW_ATTR(k_ntt_fwd, 14)
    CW_ATTR(k_ntt_inv, 12) CW_ATTR(k_ntt_inv, 13) CW_ATTR(k_ntt_inv, 14)
    CW_ATTR(k_ntt_payload, 12) CW_ATTR(k_ntt_payload, 13) CW_ATTR(k_ntt_payload, 14)
#undef CW_ATTR
    return e;
}

void launch_ntt_payload(const Launch& lc, const uint16_t* pay, uint64_t* out, size_t rows_u16) {
    if (!rows_u16) return;
    const size_t lds = (size_t)lc.N * 8;
    dim3 grid((unsigned)(rows_u16 * lc.L)), block(NTT_THREADS);
    switch (lc.logN) {
        case 12: hipLaunchKernelGGL(k_ntt_payload<12>, grid, block, lds, lc.stream, lc.K, lc.tw, pay, out); break;
        case 13: hipLaunchKernelGGL(k_ntt_payload<13>, grid, block, lds, lc.stream, lc.K, lc.tw, pay, out); break;
        case 14: hipLaunchKernelGGL(k_ntt_payload<14>, grid, block, lds, lc.stream, lc.K, lc.tw, pay, out); break;
    }
}

// ---------------------------------------------------------------------------------------------
// Exact centred extension Q -> Q u B of coefficient-form polynomials: in [G][L][N] -> out [G][LL][N]
// ---------------------------------------------------------------------------------------------
template <int NL>
__device__ __forceinline__ bool extend_coeff(const CtxConst* K, const uint64_t* x, size_t xs, uint64_t* o, size_t os,
                                             bool exact) {
    const uint32_t L = K->L, LB = K->LB;
    uint64_t y[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) {
            uint64_t xi = x[i * xs];
            y[i] = mul_shoup(xi, K->qinv[i], K->qinvq[i], K->p[i]);
            o[i * os] = xi;
        }
    bool amb = false;
    uint32_t v = exact ? conv_round_exact(K->qb, y) : conv_round_fast<NL>(K->qb, y, L, amb);
    for (uint32_t j = 0; j < LB; ++j) o[(L + j) * os] = conv_out<NL>(K->qb, y, L, v, j);
    return amb;
}

template <int NL>
__global__ void k_extend(const CtxConst* __restrict__ K, const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                         size_t G, uint64_t* fix, uint32_t* fixcnt) {
    const uint32_t N = K->N, L = K->L, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= G * N) return;
    const size_t g = gid / N, c = gid % N;
    if (extend_coeff<NL>(K, in + g * L * N + c, N, out + g * LL * N + c, N, false)) fix[atomicAdd(fixcnt, 1u)] = gid;
}

template <int NL>
__global__ void k_extend_fix(const CtxConst* __restrict__ K, const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                             uint64_t* fix, uint32_t* fixcnt) {
    const uint32_t N = K->N, L = K->L, LL = K->LL;
    const uint32_t n = *fixcnt;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) {
        const size_t gid = fix[f];
        const size_t g = gid / N, c = gid % N;
        extend_coeff<NL>(K, in + g * L * N + c, N, out + g * LL * N + c, N, true);
    }
    __syncthreads();
    if (threadIdx.x == 0) *fixcnt = 0;
}

void launch_extend(const Launch& lc, const uint64_t* in, uint64_t* out, size_t G) {
    if (!G) return;
    const unsigned nb = blocks_for(G * lc.N);
    if (lc.L <= 4) {
        hipLaunchKernelGGL(k_extend<4>, dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, in, out, G, lc.fix, lc.fixcnt);
        hipLaunchKernelGGL(k_extend_fix<4>, dim3(1), dim3(256), 0, lc.stream, lc.K, in, out, lc.fix, lc.fixcnt);
    } else if (lc.L <= 8) {
        hipLaunchKernelGGL(k_extend<8>, dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, in, out, G, lc.fix, lc.fixcnt);
        hipLaunchKernelGGL(k_extend_fix<8>, dim3(1), dim3(256), 0, lc.stream, lc.K, in, out, lc.fix, lc.fixcnt);
    } else {
        hipLaunchKernelGGL(k_extend<12>, dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, in, out, G, lc.fix, lc.fixcnt);
        hipLaunchKernelGGL(k_extend_fix<12>, dim3(1), dim3(256), 0, lc.stream, lc.K, in, out, lc.fix, lc.fixcnt);
    }
}

// ---------------------------------------------------------------------------------------------
// Tensor product in the transformed domain over Q u B: (a0 b0, a0 b1 + a1 b0, a1 b1)
// ---------------------------------------------------------------------------------------------
__global__ void k_tensor(const CtxConst* __restrict__ K, const uint32_t* __restrict__ refs,
                         const uint64_t* __restrict__ leaves, const uint64_t* __restrict__ nodes,
                         uint64_t* __restrict__ X, uint32_t E) {
    const uint32_t N = K->N, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)E * LL * N) return;
    const size_t c = gid % N, el = gid / N;
    const uint32_t l = (uint32_t)(el % LL);
    const size_t e = el / LL;
    const size_t ct = (size_t)2 * LL * N;
    const uint32_t ra = refs[2 * e], rb = refs[2 * e + 1];
    const uint64_t* A = (ra & REF_NODE) ? nodes + (size_t)(ra & ~REF_NODE) * ct : leaves + (size_t)ra * ct;
    const uint64_t* B = (rb & REF_NODE) ? nodes + (size_t)(rb & ~REF_NODE) * ct : leaves + (size_t)rb * ct;
    const uint64_t p = K->p[l], mu = K->bar_mu[l];
    const uint32_t s = K->bar_s[l];
    const size_t o0 = (size_t)l * N + c, o1 = (size_t)(LL + l) * N + c;
    const uint64_t a0 = A[o0], a1 = A[o1], b0 = B[o0], b1 = B[o1];
    uint64_t* x = X + e * 3 * LL * N + (size_t)l * N + c;
    x[0] = mul_barrett(a0, b0, p, mu, s);
    x[(size_t)LL * N] = add_mod(mul_barrett(a0, b1, p, mu, s), mul_barrett(a1, b0, p, mu, s), p);
    x[(size_t)2 * LL * N] = mul_barrett(a1, b1, p, mu, s);
}

void launch_tensor(const Launch& lc, const uint32_t* refs, const uint64_t* leaves, const uint64_t* nodes, uint64_t* X,
                   uint32_t E) {
    if (!E) return;
    hipLaunchKernelGGL(k_tensor, dim3(blocks_for((size_t)E * lc.LL * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K,
                       refs, leaves, nodes, X, E);
}

// ---------------------------------------------------------------------------------------------
// Exact scale-and-round of a coefficient-form tensor product X over Q u B:
//   r = [t X]_q (centred, exact Q -> B), y = (t X - r) / q in B, c = y (exact centred B -> Q).
// mode SCALE_STAGING writes the relinearization staging layout, SCALE_PLAIN writes [E][3][L][N].
// ---------------------------------------------------------------------------------------------
template <int NL, int NB>
__device__ __forceinline__ bool scale_coeff(const CtxConst* K, const uint64_t* x, size_t xs, uint64_t* cq, bool exact) {
    const uint32_t L = K->L, LB = K->LB;
    uint64_t y[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) y[i] = mul_shoup(x[i * xs], K->tqinv[i], K->tqinvq[i], K->p[i]);
    bool amb = false;
    const uint32_t v = exact ? conv_round_exact(K->qb, y) : conv_round_fast<NL>(K->qb, y, L, amb);
    uint64_t z[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < (int)LB) {
            const uint64_t b = K->p[L + j];
            const uint64_t rb = conv_out<NL>(K->qb, y, L, v, j);
            const uint64_t xb = x[(L + j) * xs];
            z[j] = sub_mod(mul_shoup(xb, K->kb1[j], K->kb1q[j], b), mul_shoup(rb, K->kb2[j], K->kb2q[j], b), b);
        }
    const uint32_t v2 = exact ? conv_round_exact(K->bq, z) : conv_round_fast<NB>(K->bq, z, LB, amb);
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) cq[i] = conv_out<NB>(K->bq, z, LB, v2, i);
    return amb;
}

template <int NL>
__device__ __forceinline__ void scale_store(const CtxConst* K, const uint64_t* cq, uint64_t* out, size_t e, uint32_t r,
                                            size_t c, int mode) {
    const uint32_t N = K->N, L = K->L;
    if (mode == SCALE_PLAIN) {
        uint64_t* o = out + ((e * 3 + r) * L) * N + c;
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if (i < (int)L) o[(size_t)i * N] = cq[i];
        return;
    }
    uint64_t* base = out + e * (L + 2) * L * N + c;
    if (r < 2) {
        uint64_t* o = base + (size_t)(L + r) * L * N;
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if (i < (int)L) o[(size_t)i * N] = cq[i];
    } else {
#pragma unroll
        for (int i = 0; i < NL; ++i)
            if (i < (int)L)
                for (uint32_t j = 0; j < L; ++j)
                    base[((size_t)i * L + j) * N] = (i == (int)j) ? cq[i] : reduce64(cq[i], K->p[j], K->r1[j]);
    }
}

template <int NL, int NB>
__global__ void k_scale(const CtxConst* __restrict__ K, const uint64_t* __restrict__ X, uint64_t* __restrict__ out,
                        uint32_t E, int mode, uint64_t* fix, uint32_t* fixcnt) {
    const uint32_t N = K->N, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)E * 3 * N) return;
    const size_t c = gid % N, er = gid / N;
    const uint32_t r = (uint32_t)(er % 3);
    const size_t e = er / 3;
    uint64_t cq[NL];
    if (scale_coeff<NL, NB>(K, X + er * LL * N + c, N, cq, false)) fix[atomicAdd(fixcnt, 1u)] = gid;
    scale_store<NL>(K, cq, out, e, r, c, mode);
}

template <int NL, int NB>
__global__ void k_scale_fix(const CtxConst* __restrict__ K, const uint64_t* __restrict__ X, uint64_t* __restrict__ out,
                            int mode, uint64_t* fix, uint32_t* fixcnt) {
    const uint32_t N = K->N, LL = K->LL;
    const uint32_t n = *fixcnt;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) {
        const size_t gid = fix[f];
        const size_t c = gid % N, er = gid / N;
        uint64_t cq[NL];
        scale_coeff<NL, NB>(K, X + er * LL * N + c, N, cq, true);
        scale_store<NL>(K, cq, out, er / 3, (uint32_t)(er % 3), c, mode);
    }
    __syncthreads();
    if (threadIdx.x == 0) *fixcnt = 0;
}

void launch_scale(const Launch& lc, const uint64_t* X, uint64_t* out, uint32_t E, int mode) {
    if (!E) return;
    const unsigned nb = blocks_for((size_t)E * 3 * lc.N);
#define CW_SCALE(NLV, NBV)                                                                                    \
    hipLaunchKernelGGL((k_scale<NLV, NBV>), dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, X, out, E, mode, \
                       lc.fix, lc.fixcnt);                                                                    \
    hipLaunchKernelGGL((k_scale_fix<NLV, NBV>), dim3(1), dim3(256), 0, lc.stream, lc.K, X, out, mode, lc.fix, \
                       lc.fixcnt);
    if (lc.L <= 4 && lc.LB <= 5) {
        CW_SCALE(4, 5)
    } else if (lc.L <= 8 && lc.LB <= 9) {
        CW_SCALE(8, 9)
    } else {
        CW_SCALE(12, 13)
    }
#undef CW_SCALE
}

// Relinearization staging from a plain [E][3][L][N] coefficient-form ciphertext.
__global__ void k_relin_stage(const CtxConst* __restrict__ K, const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                              uint32_t E) {
    const uint32_t N = K->N, L = K->L;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)E * N) return;
    const size_t c = gid % N, e = gid / N;
    const uint64_t* src = in + e * 3 * L * N + c;
    uint64_t* base = out + e * (L + 2) * L * N + c;
    for (uint32_t j = 0; j < L; ++j) {
        base[((size_t)L * L + j) * N] = src[(size_t)j * N];
        base[((size_t)(L + 1) * L + j) * N] = src[(size_t)(L + j) * N];
    }
    for (uint32_t i = 0; i < L; ++i) {
        const uint64_t d = src[(size_t)(2 * L + i) * N];
        for (uint32_t j = 0; j < L; ++j) base[((size_t)i * L + j) * N] = (i == j) ? d : reduce64(d, K->p[j], K->r1[j]);
    }
}

void launch_relin_stage(const Launch& lc, const uint64_t* in, uint64_t* out, uint32_t E) {
    if (!E) return;
    hipLaunchKernelGGL(k_relin_stage, dim3(blocks_for((size_t)E * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K, in,
                       out, E);
}

// ---------------------------------------------------------------------------------------------
// Key switching: sel = (c0 + sum_i D_i b_i, c1 + sum_i D_i a_i), transformed over Q.
// rlk: [L][2][L][N] transformed values followed by [L][2][L][N] Shoup companions.
// ---------------------------------------------------------------------------------------------
__global__ void k_relin_mac(const CtxConst* __restrict__ K, const uint64_t* __restrict__ R,
                            const uint64_t* __restrict__ rlk, uint64_t* __restrict__ sel, uint32_t E) {
    const uint32_t N = K->N, L = K->L;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)E * L * N) return;
    const size_t c = gid % N, ej = gid / N;
    const uint32_t j = (uint32_t)(ej % L);
    const size_t e = ej / L;
    const uint64_t p = K->p[j];
    const size_t LN = (size_t)L * N;
    const uint64_t* r = R + e * (L + 2) * LN + (size_t)j * N + c;
    const size_t half = (size_t)L * 2 * LN;
    uint64_t s0 = r[(size_t)L * LN], s1 = r[(size_t)(L + 1) * LN];
    for (uint32_t i = 0; i < L; ++i) {
        const uint64_t d = r[(size_t)i * LN];
        const size_t ob = ((size_t)i * 2 + 0) * LN + (size_t)j * N + c;
        const size_t oa = ((size_t)i * 2 + 1) * LN + (size_t)j * N + c;
        s0 = add_mod(s0, mul_shoup(d, rlk[ob], rlk[half + ob], p), p);
        s1 = add_mod(s1, mul_shoup(d, rlk[oa], rlk[half + oa], p), p);
    }
    uint64_t* o = sel + e * 2 * LN + (size_t)j * N + c;
    o[0] = s0;
    o[LN] = s1;
}

void launch_relin_mac(const Launch& lc, const uint64_t* R, const uint64_t* rlk, uint64_t* sel, uint32_t E) {
    if (!E) return;
    hipLaunchKernelGGL(k_relin_mac, dim3(blocks_for((size_t)E * lc.L * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K,
                       R, rlk, sel, E);
}

// Shoup companions of a transformed key: comp[i] = floor(v[i] 2^64 / p) with p from the limb index.
__global__ void k_shoup_companions(const CtxConst* __restrict__ K, const uint64_t* __restrict__ v, uint64_t* __restrict__ comp,
                                   size_t rows, uint32_t nl) {
    const uint32_t N = K->N;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= rows * N) return;
    const uint64_t p = K->p[(gid / N) % nl];
    // floor(v 2^64 / p) by long division in two 64-bit halves: v < p < 2^61.
    const uint64_t x = v[gid];
    uint64_t q = 0, rem = x;
    for (int b = 63; b >= 0; --b) {
        rem <<= 1;  // rem < p < 2^61 so no overflow
        if (rem >= p) {
            rem -= p;
            q |= 1ull << b;
        }
    }
    comp[gid] = q;
}

void launch_shoup_companions(const Launch& lc, const uint64_t* v, uint64_t* comp, size_t rows, uint32_t nl) {
    if (!rows) return;
    hipLaunchKernelGGL(k_shoup_companions, dim3(blocks_for(rows * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K, v, comp,
                       rows, nl);
}

// ---------------------------------------------------------------------------------------------
// k = 1: the selector is the query ciphertext itself (its Q limbs, transformed).
// ---------------------------------------------------------------------------------------------
__global__ void k_gather_leaf(const CtxConst* __restrict__ K, const uint32_t* __restrict__ refs,
                              const uint64_t* __restrict__ leaves, uint64_t* __restrict__ sel, uint32_t E) {
    const uint32_t N = K->N, L = K->L, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)E * 2 * L * N) return;
    const size_t c = gid % N, rest = gid / N;
    const uint32_t j = (uint32_t)(rest % L);
    const size_t ep = rest / L;
    const uint32_t poly = (uint32_t)(ep % 2);
    const size_t e = ep / 2;
    const uint32_t leaf = refs[2 * e];
    sel[gid] = leaves[((size_t)leaf * 2 * LL + (size_t)poly * LL + j) * N + c];
}

void launch_gather_leaf(const Launch& lc, const uint32_t* refs, const uint64_t* leaves, uint64_t* sel, uint32_t E) {
    if (!E) return;
    hipLaunchKernelGGL(k_gather_leaf, dim3(blocks_for((size_t)E * 2 * lc.L * lc.N)), dim3(EW_THREADS), 0, lc.stream,
                       lc.K, refs, leaves, sel, E);
}

// ---------------------------------------------------------------------------------------------
// Inner product with the database (Eq. (1)): acc_b[r] += sum_e sel_b[e] * P[e][r], transformed
// over Q.  Grid y indexes the B queries that scan the same payload chunk.
// ---------------------------------------------------------------------------------------------
__global__ void k_accumulate(const CtxConst* __restrict__ K, const QueryPtrs qp, const uint64_t* __restrict__ Ph,
                             uint32_t E, uint32_t s) {
    const uint32_t N = K->N, L = K->L;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t LN = (size_t)L * N;
    if (gid >= (size_t)s * 2 * LN) return;
    const size_t cj = gid % LN;  // j * N + c
    const uint32_t j = (uint32_t)(cj / N);
    const size_t rp = gid / LN;
    const uint32_t poly = (uint32_t)(rp % 2), r = (uint32_t)(rp / 2);
    const uint64_t p = K->p[j], mu = K->bar_mu[j];
    const uint32_t sb = K->bar_s[j];
    const uint64_t* sel = qp.sel[blockIdx.y];
    uint64_t* acc = qp.acc[blockIdx.y];
    uint64_t sum = acc[gid];
    for (uint32_t e = 0; e < E; ++e) {
        const uint64_t a = sel[((size_t)e * 2 + poly) * LN + cj];
        const uint64_t b = Ph[((size_t)e * s + r) * LN + cj];
        sum = add_mod(sum, mul_barrett(a, b, p, mu, sb), p);
    }
    acc[gid] = sum;
}

void launch_accumulate(const Launch& lc, const QueryPtrs& qp, const uint64_t* Ph, uint32_t nq, uint32_t E,
                       uint32_t s) {
    if (!E || !nq) return;
    hipLaunchKernelGGL(k_accumulate, dim3(blocks_for((size_t)s * 2 * lc.L * lc.N), nq), dim3(EW_THREADS), 0,
                       lc.stream, lc.K, qp, Ph, E, s);
}

// Pointwise product of a transformed ciphertext [2][L][N] with a transformed plaintext [L][N].
__global__ void k_pointwise_pt(const CtxConst* __restrict__ K, const uint64_t* __restrict__ ct,
                               const uint64_t* __restrict__ pt, uint64_t* __restrict__ out) {
    const uint32_t N = K->N, L = K->L;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)2 * L * N) return;
    const size_t cj = gid % ((size_t)L * N);
    const uint32_t j = (uint32_t)(cj / N);
    out[gid] = mul_barrett(ct[gid], pt[cj], K->p[j], K->bar_mu[j], K->bar_s[j]);
}

void launch_pointwise_pt(const Launch& lc, const uint64_t* ct, const uint64_t* pt, uint64_t* out) {
    hipLaunchKernelGGL(k_pointwise_pt, dim3(blocks_for((size_t)2 * lc.L * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K,
                       ct, pt, out);
}

__global__ void k_fill(uint64_t* __restrict__ p, size_t n, uint64_t v) {
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < n) p[gid] = v;
}

void launch_fill(hipStream_t st, uint64_t* p, size_t n, uint64_t v) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(EW_THREADS), 0, st, p, n, v);
}

// ---------------------------------------------------------------------------------------------
// Codeword tables
// ---------------------------------------------------------------------------------------------
// Algorithm 3 (perfect mapping): scan m' = m-1 .. 0, take m' whenever the remaining rank r is at
// least C(m', h); binom is the saturating table C(a, h), a < m, h <= k.
__global__ void k_map_perfect(const uint64_t* __restrict__ ids, size_t n, uint32_t m, uint32_t k,
                              const uint64_t* __restrict__ binom, uint32_t* __restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    uint64_t r = ids[e];
    uint32_t h = k;
    uint32_t* o = out + e * k;
    for (int mp = (int)m - 1; mp >= 0 && h > 0; --mp) {
        const uint64_t c = binom[(size_t)mp * (k + 1) + h];
        if (r >= c) {
            r -= c;
            o[h - 1] = (uint32_t)mp;  // the h-th one from the top is the h-th smallest position
            --h;
        }
    }
    for (; h > 0; --h) o[h - 1] = 0xFFFFFFFFu;  // rank outside the code (rejected by the caller)
}

void launch_map_perfect(hipStream_t st, const uint64_t* ids, size_t n, uint32_t m, uint32_t k, const uint64_t* binom,
                        uint32_t* out) {
    if (!n) return;
    hipLaunchKernelGGL(k_map_perfect, dim3(blocks_for(n)), dim3(EW_THREADS), 0, st, ids, n, m, k, binom, out);
}

__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Algorithm 8 (lossy mapping): positions H_1(x), H_2(x), ... until k distinct, kept sorted.
__global__ void k_map_lossy(const uint64_t* __restrict__ kw, size_t n, uint32_t m, uint32_t k, uint64_t seed,
                            uint32_t* __restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const uint64_t x = kw[e];
    uint32_t pos[16];
    uint32_t cnt = 0;
    const uint32_t cap = 4096u + 64u * k;  // a bound no uniform hash sequence reaches in practice
    for (uint32_t i = 1; cnt < k && i <= cap; ++i) {
        const uint32_t h = (uint32_t)(splitmix_mix(seed ^ x ^ ((uint64_t)i * 0x9E3779B97F4A7C15ull)) % m);
        uint32_t at = cnt;
        bool dup = false;
        for (uint32_t a = 0; a < cnt; ++a) {
            if (pos[a] == h) dup = true;
            if (pos[a] > h && at == cnt) at = a;
        }
        if (dup) continue;
        for (uint32_t a = cnt; a > at; --a) pos[a] = pos[a - 1];
        pos[at] = h;
        ++cnt;
    }
    for (uint32_t a = 0; a < k; ++a) out[e * k + a] = a < cnt ? pos[a] : 0xFFFFFFFFu;
}

void launch_map_lossy(hipStream_t st, const uint64_t* kw, size_t n, uint32_t m, uint32_t k, uint64_t seed,
                      uint32_t* out) {
    if (!n) return;
    hipLaunchKernelGGL(k_map_lossy, dim3(blocks_for(n)), dim3(EW_THREADS), 0, st, kw, n, m, k, seed, out);
}

}  // namespace cw
