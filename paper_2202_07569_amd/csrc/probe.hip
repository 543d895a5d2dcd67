// Issue-rate probes of the VALU instructions the transforms are built from (diagnostics): the fp64
// instructions of the fp64 path and the 32-bit integer multiplies and 64-bit adds of the integer path.
// Each thread runs PROBE_CHAINS independent chains of `iters` steps of one operation, so the
// scheduler always has independent work; out[gid] receives the chains' sum (keeps them live).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cw {

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_CHAINS = 8;

template <int OP>
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_fp64(double* __restrict__ out, uint32_t iters, double a,
                                                               double b) {
    double v[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) v[c] = (double)(threadIdx.x + c) * 0.5;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) {
            if constexpr (OP == 0) v[c] = __builtin_fma(v[c], a, b);
            else if constexpr (OP == 1) v[c] = v[c] * a;
            else if constexpr (OP == 2) v[c] = v[c] + b;
            else v[c] = __builtin_rint(v[c]) + b;  // v_rndne_f64 and v_add_f64
        }
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += v[c];
    out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

// Integer operations of the integer-path transforms (64-bit words built from 32-bit pieces):
//   OP 0  v_mul_lo_u32     x = x * a
//   OP 1  v_mul_hi_u32     x = hi32(x * a), a = 2^32 - 1 (x - 1 for x >= 1: the chain stays live)
//   OP 2  v_mad_u64_u32    y = lo32(y) * a + y   (64-bit result)
//   OP 3  v_lshl_add_u64   y = y + b   (gfx950 adds 64-bit words in one instruction)
template <int OP>
__global__ __launch_bounds__(PROBE_THREADS) void k_probe_int(uint64_t* __restrict__ out, uint32_t iters, uint32_t a,
                                                              uint64_t b) {
    uint32_t x[PROBE_CHAINS];
    uint64_t y[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) {
        x[c] = 0x80000000u + threadIdx.x * 8u + (uint32_t)c;
        y[c] = ((uint64_t)threadIdx.x << 32) + (uint64_t)c * 977u + 1u;
    }
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) {
            if constexpr (OP == 0) x[c] = x[c] * a;
            else if constexpr (OP == 1) x[c] = __umulhi(x[c], a);
            else if constexpr (OP == 2) y[c] = (uint64_t)(uint32_t)y[c] * a + y[c];
            else y[c] = y[c] + b;
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += (OP <= 1) ? (uint64_t)x[c] : y[c];
    out[(size_t)blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

}  // namespace

uint32_t probe_threads() { return PROBE_THREADS; }

// Wave-instructions of the timed operation per launch: waves * iters * chains.
double launch_probe_int(hipStream_t st, int op, uint32_t blocks, uint32_t iters, uint64_t* out) {
    const uint32_t a = op == 1 ? 0xFFFFFFFFu : 0x9E3779B9u;
    const uint64_t b = 0x9E3779B97F4A7C15ull;
    switch (op) {
        case 0: hipLaunchKernelGGL(k_probe_int<0>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
        case 1: hipLaunchKernelGGL(k_probe_int<1>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
        case 2: hipLaunchKernelGGL(k_probe_int<2>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
        default: hipLaunchKernelGGL(k_probe_int<3>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
    }
    const double waves = (double)blocks * (PROBE_THREADS / 64);
    return waves * iters * PROBE_CHAINS;
}

// Wave-instructions of the timed operation per launch: waves * iters * chains * (2 for op 3).
double launch_probe_fp64(hipStream_t st, int op, uint32_t blocks, uint32_t iters, double* out) {
    const double a = 1.0000001, b = 0.25;
    switch (op) {
        case 0: hipLaunchKernelGGL(k_probe_fp64<0>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
        case 1: hipLaunchKernelGGL(k_probe_fp64<1>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
        case 2: hipLaunchKernelGGL(k_probe_fp64<2>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
        default: hipLaunchKernelGGL(k_probe_fp64<3>, dim3(blocks), dim3(PROBE_THREADS), 0, st, out, iters, a, b); break;
    }
    const double waves = (double)blocks * (PROBE_THREADS / 64);
    return waves * iters * PROBE_CHAINS * (op == 3 ? 2.0 : 1.0);
}

}  // namespace cw
