// Issue-rate probe of the fp64 VALU instructions the transforms are built from (diagnostics).
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

}  // namespace

uint32_t probe_threads() { return PROBE_THREADS; }

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
