// HIP kernels for gfx950 of the constant-weight PIR server path.
//
// Data layout in HBM (u64 residues, limb-major inside a polynomial, N coefficients per limb):
//   extended ciphertext  [2][LL][N]   over Q then B, transformed (NTT domain)
//   tensor product       [E][3][LL][N]
//   product after scale  [E][3][L][N]  coefficient form over Q
//   relin staging        [E][L+2][L][N]  transformed; rows 0..L-1: digit i mod q_j; rows L, L+1: c0, c1
//   selector             [E][2][L][N]  transformed over Q
//   payload transform    [E][s][L][N]
//   accumulator/answer   [s][2][L][N]
// A "limb-poly" is one row of N residues; its prime is prime_base + (row index mod nl).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "arith.h"
#include "kernels.h"

namespace cw {

constexpr int EW_THREADS = 256;

static inline unsigned blocks_for(size_t n, int t = EW_THREADS) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------------------------
// Negacyclic NTT: one workgroup per limb-poly, register-resident radix-2^r passes.
//
// Forward: Cooley-Tukey butterflies with the psi powers merged into the twiddles (table index
// m + i holds psi^bitrev(m + i)), stage s pairing the indices that differ in bit LOGN-1-s.  Inverse:
// Gentleman-Sande butterflies with psi^-bitrev, the stages in reverse order, then N^-1.  Lazy
// reduction (D. Harvey 2014): forward values stay in [0, 4p), inverse values in [0, 2p), with the
// final reduction to [0, p) at the store (p < 2^61, so 4p < 2^63).
//
// The LOGN stages are cut into three passes of r_p stages.  In pass p a thread holds EPT = 2^R
// elements: the 2^r_p combinations of the pass's index bits times 2^(R - r_p) "extra" bits, so
// every butterfly of the pass is between two of its registers.  Between passes the values go
// through LDS.  The first forward pass reads natural order (coalesced); the last forward pass
// writes element u of thread t to position u*T + t (coalesced).  That permuted order is the
// library's transformed layout: every transformed array comes from this kernel, products in that
// domain are pointwise, and the inverse reads the same layout back.
// ---------------------------------------------------------------------------------------------
// A transform shape: 2^R elements per thread (T = N / 2^R threads) and NP passes of r(p) stages.
template <int LOGN_, int R_, int NP_, int R0, int R1 = 0, int R2 = 0, int R3 = 0, int R4 = 0>
struct Shape {
    static constexpr int LOGN = LOGN_, R = R_, NP = NP_;
    static constexpr int N = 1 << LOGN, EPT = 1 << R, T = 1 << (LOGN - R);
    static constexpr int LDS_WORDS = N + N / 16;
    __host__ __device__ static constexpr int r(int p) {
        return p == 0 ? R0 : p == 1 ? R1 : p == 2 ? R2 : p == 3 ? R3 : R4;
    }
    __host__ __device__ static constexpr int S0(int p) {
        int s = 0;
        for (int q = 0; q < p; ++q) s += r(q);
        return s;
    }
    static_assert(R0 == R, "the first pass reads whole coalesced rows");
    static_assert(R0 + R1 + R2 + R3 + R4 == LOGN, "passes must cover every stage");
};

// The shapes per ring degree that the kernels may use.  Every kernel that writes or reads the
// transformed layout must agree on that layout (position u*T + tid holds natural index
// elem_index<Sh, NP-1>(tid, u)), which depends only on R and on the last pass: the stages run in
// the same order whatever their grouping, so the array they leave is the same.  The variants of
// one degree therefore share R and the last pass and differ in how the middle stages are grouped
// into passes (which exchanges stay inside a wavefront, how many stages share the registers
// between two exchanges); the autotuner picks one per context.  Eight elements per thread leave
// room for the key-switching accumulators (k_relin).
template <int LOGN, int V>
struct ShapeVar;
template <>
struct ShapeVar<12, 0> {
    using type = Shape<12, 3, 4, 3, 3, 3, 3>;
};
template <>
struct ShapeVar<13, 0> {
    using type = Shape<13, 3, 5, 3, 3, 3, 2, 2>;
};
template <>
struct ShapeVar<13, 1> {
    using type = Shape<13, 3, 5, 3, 3, 2, 3, 2>;
};
template <>
struct ShapeVar<13, 2> {
    using type = Shape<13, 3, 5, 3, 2, 3, 3, 2>;
};
template <>
struct ShapeVar<14, 0> {
    using type = Shape<14, 4, 4, 4, 4, 3, 3>;
};
template <>
struct ShapeVar<14, 1> {
    using type = Shape<14, 4, 4, 4, 3, 4, 3>;
};
__host__ __device__ constexpr uint32_t shape_key(uint32_t logN, uint32_t v) { return logN * 4 + v; }

// Calls f(Sh{}) with the shape variant v of degree 2^logN (nothing for an unknown pair; the host
// checks the variant against ntt_shape_count first).
template <class F>
void with_shape(uint32_t logN, uint32_t v, F&& f) {
    switch (shape_key(logN, v)) {
        case shape_key(12, 0): f(ShapeVar<12, 0>::type{}); break;
        case shape_key(13, 0): f(ShapeVar<13, 0>::type{}); break;
        case shape_key(13, 1): f(ShapeVar<13, 1>::type{}); break;
        case shape_key(13, 2): f(ShapeVar<13, 2>::type{}); break;
        case shape_key(14, 0): f(ShapeVar<14, 0>::type{}); break;
        case shape_key(14, 1): f(ShapeVar<14, 1>::type{}); break;
        default: break;
    }
}

uint32_t ntt_shape_count(uint32_t logN) { return logN == 13 ? 3 : logN == 14 ? 2 : logN == 12 ? 1 : 0; }

uint32_t ntt_shape_stages(uint32_t logN, uint32_t v, uint32_t* stages) {
    uint32_t np = 0;
    with_shape(logN, v, [&](auto tag) {
        using Sh = decltype(tag);
        np = Sh::NP;
        for (int q = 0; q < Sh::NP; ++q) stages[q] = (uint32_t)Sh::r(q);
    });
    return np;
}

template <class A, class B>
constexpr bool same_layout() {
    return A::LOGN == B::LOGN && A::R == B::R && A::r(A::NP - 1) == B::r(B::NP - 1);
}
static_assert(same_layout<ShapeVar<13, 0>::type, ShapeVar<13, 1>::type>() &&
                  same_layout<ShapeVar<13, 0>::type, ShapeVar<13, 2>::type>() &&
                  same_layout<ShapeVar<14, 0>::type, ShapeVar<14, 1>::type>(),
              "shape variants of one degree must leave the same transformed layout");

template <class Sh, int P>
struct PassGeo {
    static constexpr int R = Sh::R;
    static constexpr int rp = Sh::r(P);
    static constexpr int S0 = Sh::S0(P);                // stages before this pass
    static constexpr int plo = Sh::LOGN - S0 - rp;      // lowest pass bit
    static constexpr int x = R - rp;                    // extra bits
    static_assert(plo == 0 || plo >= x, "extra bits must sit below a middle pass");
};

// Natural index of element u of thread tid in pass P.
template <class Sh, int P>
__device__ __forceinline__ uint32_t elem_index(uint32_t tid, uint32_t u) {
    using G = PassGeo<Sh, P>;
    constexpr int x = G::x, rp = G::rp, plo = G::plo;
    if constexpr (plo == 0) {  // last pass: the extra bits sit just above the pass bits
        return (u >> x) | ((u & ((1u << x) - 1u)) << rp) | (tid << G::R);
    } else {  // extra bits lowest, then tid low part, pass bits, tid high part
        const uint32_t ev = u & ((1u << x) - 1u), pv = u >> x;
        const uint32_t tl = tid & ((1u << (plo - x)) - 1u), th = tid >> (plo - x);
        return ev | (tl << x) | (pv << plo) | (th << (plo + rp));
    }
}

__host__ __device__ constexpr uint32_t lds_pad(uint32_t idx) { return idx + (idx >> 4); }

// elem_index splits into a thread part and an element part with disjoint bits:
//   elem_index(tid, u) = elem_index(tid, 0) | elem_index(0, u).
// Shifts and the LDS padding distribute over such a split: for disjoint a and b,
// (a | b) >> k = (a >> k) + (b >> k) and lds_pad(a | b) = lds_pad(a) + lds_pad(b).  The transforms
// therefore form each address as a per-thread base (once per pass or stage) plus a compile-time
// offset, which the memory instructions take as an immediate.

template <class Sh, int P>
__device__ __forceinline__ void fwd_pass(uint64_t* a, uint32_t tid, const uint64_t* __restrict__ psi,
                                         const uint64_t* __restrict__ psiq, uint64_t p) {
    using G = PassGeo<Sh, P>;
    const uint64_t p2 = 2 * p;
#pragma unroll
    for (int sp = 0; sp < G::rp; ++sp) {
        const int s = G::S0 + sp;
        const int pb = G::x + G::rp - 1 - sp;
        const uint32_t tb = (1u << s) + (elem_index<Sh, P>(tid, 0u) >> (Sh::LOGN - s));
        const uint64_t* __restrict__ ps = psi + tb;
        const uint64_t* __restrict__ pq = psiq + tb;
#pragma unroll
        for (int u0 = 0; u0 < Sh::EPT; ++u0) {
            if (u0 & (1 << pb)) continue;
            const int u1 = u0 | (1 << pb);
            const uint32_t c = elem_index<Sh, P>(0u, (uint32_t)u0) >> (Sh::LOGN - s);
            const uint64_t w = ps[c], wq = pq[c];
            uint64_t X = a[u0];
            X = X >= p2 ? X - p2 : X;
            const uint64_t T = mul_shoup_lazy(a[u1], w, wq, p);
            a[u0] = X + T;
            a[u1] = X - T + p2;
        }
    }
}

template <class Sh, int P>
__device__ __forceinline__ void inv_pass(uint64_t* a, uint32_t tid, const uint64_t* __restrict__ psi,
                                         const uint64_t* __restrict__ psiq, uint64_t p) {
    using G = PassGeo<Sh, P>;
    const uint64_t p2 = 2 * p;
#pragma unroll
    for (int sp = G::rp - 1; sp >= 0; --sp) {
        const int s = G::S0 + sp;
        const int pb = G::x + G::rp - 1 - sp;
        const uint32_t tb = (1u << s) + (elem_index<Sh, P>(tid, 0u) >> (Sh::LOGN - s));
        const uint64_t* __restrict__ ps = psi + tb;
        const uint64_t* __restrict__ pq = psiq + tb;
#pragma unroll
        for (int u0 = 0; u0 < Sh::EPT; ++u0) {
            if (u0 & (1 << pb)) continue;
            const int u1 = u0 | (1 << pb);
            const uint32_t c = elem_index<Sh, P>(0u, (uint32_t)u0) >> (Sh::LOGN - s);
            const uint64_t w = ps[c], wq = pq[c];
            const uint64_t X = a[u0], Y = a[u1];
            const uint64_t Sm = X + Y;
            a[u0] = Sm >= p2 ? Sm - p2 : Sm;
            a[u1] = mul_shoup_lazy(X - Y + p2, w, wq, p);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// fp64 arithmetic for primes below 2^50 (CtxConst::fp).  Residues are integer-valued doubles in a
// signed lazy range.  For |y| < 2^53 and a twiddle w < p:
//   h = fl(y w), l = fma(y, w, -h) = y w - h exactly, q = rint(h fl(1/p)),
//   T = fma(-q, p, h) + l = y w - q p exactly,
// because h - q p and T are integers below 2^52 in magnitude.  The quotient estimate satisfies
// |q - y w / p| <= 1/2 + 3 |y| 2^-53, so |T| <= (1/2 + 3 |y| 2^-53) p; for p < 2^50 that is at most
// (1/2 + 0.375 |y| / p) p.  fred(x) = x - rint(x / p) p leaves |x| <= p/2 (plus 2^-52 |x|).
// Forward: a pass of at most three stages starting from |x| <= p ends below 4.8p; inverse: from
// |x| <= p/2 below 4p; the final N^-1 product stays below 2p.  Every value stays below 2^53, so
// every operation above is exact.
// Lazy forward transform (primes below 2^48): with |y| = b p the product satisfies
// |T| <= (1/2 + 3 b 2^-5) p, so a stage maps a bound b to b (1 + 3/32) + 1/2; from b = 1 the 13
// stages of N = 8192 end below 15 p < 2^52, and no reduction is needed before the final one.
// ---------------------------------------------------------------------------------------------
#pragma clang fp contract(off)
__device__ __forceinline__ double fmulmod(double y, double w, double p, double pinv) {
    const double h = y * w;
    const double l = __builtin_fma(y, w, -h);
    const double q = __builtin_rint(h * pinv);
    return __builtin_fma(-q, p, h) + l;
}
__device__ __forceinline__ double fred(double x, double p, double pinv) {
    return __builtin_fma(-__builtin_rint(x * pinv), p, x);
}

// TWPAD: the twiddle table is an LDS copy stored with the exchange buffer's padding (lds_pad), which
// keeps the last stages' per-lane twiddle reads free of bank conflicts.
template <class Sh, int P, bool LAZY = false, bool TWPAD = false>
__device__ __forceinline__ void fwd_pass_fp(double* a, uint32_t tid, const double* __restrict__ tw, double p,
                                            double pinv) {
    using G = PassGeo<Sh, P>;
    static_assert(G::rp <= 3, "the fp64 bound needs passes of at most three stages");
    if constexpr (P > 0 && !LAZY) {
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) a[u] = fred(a[u], p, pinv);
    }
#pragma unroll
    for (int sp = 0; sp < G::rp; ++sp) {
        const int s = G::S0 + sp;
        const int pb = G::x + G::rp - 1 - sp;
        const uint32_t tb = (1u << s) + (elem_index<Sh, P>(tid, 0u) >> (Sh::LOGN - s));
        const double* __restrict__ ts = tw + (TWPAD ? lds_pad(tb) : tb);
#pragma unroll
        for (int u0 = 0; u0 < Sh::EPT; ++u0) {
            if (u0 & (1 << pb)) continue;
            const int u1 = u0 | (1 << pb);
            const uint32_t c = elem_index<Sh, P>(0u, (uint32_t)u0) >> (Sh::LOGN - s);
            const double T = fmulmod(a[u1], ts[TWPAD ? lds_pad(c) : c], p, pinv);
            const double X = a[u0];
            a[u0] = X + T;
            a[u1] = X - T;
        }
    }
}

// Inverse transforms with bounds tracked at compile time (LZ > 0).  In a pass the pair of a
// butterfly has one bound b (in units of p), set by the pass bits its registers share; the sum
// leaves below 2b and the product below m(2b) = 1/2 + c 2b, where c = 3 p_max 2^-53 (the fmulmod
// bound above).  So every register's bound at the end of a pass is a function of its register
// index alone, given the pass's entry bound; registers above `thr` are reduced there (to 1/2 +
// 2^-40), and the next pass starts from the largest bound left.  Every value stays below the
// all-sum chain's entry bound 2^rp, which is checked against cap = 2^53 / p_max.
// LZ = 1: any prime below 2^50 (c = 3/8, cap 8), thr 0.6 (every register reduced between passes,
//         none before the first: the inputs are tensor products, below 1.4 p);
// LZ = 2: primes below 2^44 (c = 3/512, cap 512), thr 32 (one or two registers reduced in a whole
//         transform, depending on the shape).
struct InvLazy {
    double c, cap, thr, a0;
};
__host__ __device__ constexpr InvLazy inv_lazy(int LZ) {
    return LZ == 2 ? InvLazy{3.0 / 512, 512.0, 32.0, 1.4} : InvLazy{3.0 / 8, 8.0, 0.6, 1.4};
}
template <class Sh>
__host__ __device__ constexpr double inv_reg_bound(int P, int u, double a, double c) {
    const int rp = Sh::r(P), x = Sh::R - rp;
    double b = a;
    for (int sp = rp - 1; sp >= 0; --sp) {
        const int pb = x + rp - 1 - sp;
        b = ((u >> pb) & 1) ? 0.5 + c * 2 * b : 2 * b;
    }
    return b;
}
// entry bound of inverse pass P (the passes run from NP - 1 down to 0)
template <class Sh>
__host__ __device__ constexpr double inv_pass_in(int P, int LZ) {
    const InvLazy z = inv_lazy(LZ);
    double a = z.a0;
    for (int q = Sh::NP - 1; q > P; --q) {
        double m = 0.5 + 0x1p-40;
        for (int u = 0; u < Sh::EPT; ++u) {
            const double b = inv_reg_bound<Sh>(q, u, a, z.c);
            if (b <= z.thr && b > m) m = b;
        }
        a = m;
    }
    return a;
}
// registers reduced at the end of pass P (bit u), none after the last (the caller reduces all)
template <class Sh>
__host__ __device__ constexpr uint32_t inv_fred_mask(int P, int LZ) {
    uint32_t mask = 0;
    if (P == 0) return 0;
    const double a = inv_pass_in<Sh>(P, LZ);
    for (int u = 0; u < Sh::EPT; ++u)
        if (inv_reg_bound<Sh>(P, u, a, inv_lazy(LZ).c) > inv_lazy(LZ).thr) mask |= 1u << u;
    return mask;
}
template <class Sh>
__host__ __device__ constexpr bool inv_lazy_exact(int LZ) {
    for (int P = Sh::NP - 1; P >= 0; --P)
        if (inv_pass_in<Sh>(P, LZ) * (double)(1 << Sh::r(P)) >= inv_lazy(LZ).cap) return false;
    return true;
}

// FOLD (first pass only): the transform's first stage also multiplies by the constant f, the upper
// output as fmulmod(X + Y, f) and the lower one through the twiddle row [w_inv f]_p that follows the
// inverse twiddles (tw + N); by linearity the whole transform then returns f times its result.
// Both products stay within the bounds the lazy schedules assume for X + Y and (X - Y) w.
template <class Sh, int P, int LZ = 0, bool FOLD = false>
__device__ __forceinline__ void inv_pass_fp(double* a, uint32_t tid, const double* __restrict__ tw, double p,
                                            double pinv, double f = 1.0) {
    using G = PassGeo<Sh, P>;
    static_assert(G::rp <= 3, "the fp64 bound needs passes of at most three stages");
    static_assert(LZ == 0 || inv_lazy_exact<Sh>(LZ), "the lazy inverse transform would leave the exact range");
    static_assert(!FOLD || P == Sh::NP - 1, "the fold belongs to the first stage");
    if constexpr (LZ == 0) {
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) a[u] = fred(a[u], p, pinv);
    }
#pragma unroll
    for (int sp = G::rp - 1; sp >= 0; --sp) {
        const bool fold = FOLD && sp == G::rp - 1;
        const int s = G::S0 + sp;
        const int pb = G::x + G::rp - 1 - sp;
        const uint32_t tb = (1u << s) + (elem_index<Sh, P>(tid, 0u) >> (Sh::LOGN - s));
        const double* __restrict__ ts = tw + (fold ? Sh::N : 0) + tb;
#pragma unroll
        for (int u0 = 0; u0 < Sh::EPT; ++u0) {
            if (u0 & (1 << pb)) continue;
            const int u1 = u0 | (1 << pb);
            const uint32_t c = elem_index<Sh, P>(0u, (uint32_t)u0) >> (Sh::LOGN - s);
            const double X = a[u0], Y = a[u1];
            a[u0] = fold ? fmulmod(X + Y, f, p, pinv) : X + Y;
            a[u1] = fmulmod(X - Y, ts[c], p, pinv);
        }
    }
    if constexpr (LZ > 0) {
        constexpr uint32_t mask = inv_fred_mask<Sh>(P, LZ);
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u)
            if ((mask >> u) & 1u) a[u] = fred(a[u], p, pinv);
    }
}
#pragma clang fp contract(on)

// x < 2^52 -> the double x, exactly: 2^52 + x has the bits 0x433 (exponent) and x (mantissa).
__device__ __forceinline__ double u52_to_double(uint64_t x) {
    return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 4503599627370496.0;
}

// integer-valued double in (-p, p) -> residue in [0, p) (p < 2^52): the mantissa of 2^52 + x.
__device__ __forceinline__ uint64_t fp_to_residue(double x, double p) {
    x = x < 0.0 ? x + p : x;
    return (uint64_t)__double_as_longlong(x + 4503599627370496.0) & 0xFFFFFFFFFFFFFull;
}

// Index bit that bit b of the thread index occupies in pass P (see elem_index).
template <class Sh, int P>
__host__ __device__ constexpr int tid_bit_pos(int b) {
    using G = PassGeo<Sh, P>;
    if constexpr (G::plo == 0) return b + Sh::R;
    else return b < G::plo - G::x ? G::x + b : b + G::x + G::rp;
}
// An exchange between passes PA and PB stays inside each wavefront when every thread-index bit
// above the lane bits occupies the same index bit in both passes: a wavefront then reads back
// exactly the LDS words it wrote.
template <class Sh, int PA, int PB>
__host__ __device__ constexpr bool wave_local() {
    constexpr int TB = Sh::LOGN - Sh::R;
    for (int b = 6; b < TB; ++b)
        if (tid_bit_pos<Sh, PA>(b) != tid_bit_pos<Sh, PB>(b)) return false;
    return true;
}
// Whether the exchange that fed pass PA (from the pass before it, in the direction PA -> PB) was
// wavefront-local.
template <class Sh, int PA, int PB, bool FIRST>
__host__ __device__ constexpr bool prev_wave_local() {
    if constexpr (FIRST) return false;
    else if constexpr (PA < PB) return wave_local<Sh, PA - 1, PA>();
    else return wave_local<Sh, PA + 1, PA>();
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// registers of pass PA -> LDS -> registers of pass PB.  FIRST: the first exchange of a transform.
// A workgroup-wide exchange starts with a barrier (earlier reads of the buffer by other waves must
// be done before it is overwritten) and has a second one between its writes and reads.  A
// wavefront-local exchange needs only wavefront ordering, plus a leading barrier when it follows a
// workgroup-wide exchange or starts the transform, whose readers may still be reading this
// wavefront's words.  The transform therefore leaves the buffer with reads possibly pending, and
// every later user starts with a barrier.
template <class Sh, int PA, int PB, bool FIRST, class V>
__device__ __forceinline__ void exchange(V* a, V* sm, uint32_t tid) {
    constexpr bool WL = wave_local<Sh, PA, PB>();
    constexpr bool prev_wl = prev_wave_local<Sh, PA, PB, FIRST>();
    if constexpr (!(WL && prev_wl)) __syncthreads();
    V* wa = sm + lds_pad(elem_index<Sh, PA>(tid, 0u));
    V* ra = sm + lds_pad(elem_index<Sh, PB>(tid, 0u));
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) wa[lds_pad(elem_index<Sh, PA>(0u, u))] = a[u];
    if constexpr (WL) wave_sync();
    else __syncthreads();
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) a[u] = ra[lds_pad(elem_index<Sh, PB>(0u, u))];
    if constexpr (WL) wave_sync();
}

// Twiddle tables of one prime: integer form [4][N] (w, w', w_inv, w_inv') and double form
// [4][N] (w, w/p, w_inv, w_inv/p; the fp64 passes read only w and w_inv).
struct TwRow {
    const uint64_t* i;
    const double* f;
};

template <class Sh, bool FP, int P, bool LAZY = false, bool TWPAD = false>
__device__ __forceinline__ void fwd_passes(void* av, void* smv, uint32_t tid, TwRow tw, const CtxConst* K,
                                           uint32_t pi) {
    if constexpr (FP) {
        double* a = (double*)av;
        fwd_pass_fp<Sh, P, LAZY, TWPAD>(a, tid, tw.f, K->pd[pi], K->pinv[pi]);
        if constexpr (P + 1 < Sh::NP) {
            exchange<Sh, P, P + 1, P == 0>(a, (double*)smv, tid);
            fwd_passes<Sh, FP, P + 1, LAZY, TWPAD>(av, smv, tid, tw, K, pi);
        }
    } else {
        uint64_t* a = (uint64_t*)av;
        fwd_pass<Sh, P>(a, tid, tw.i, tw.i + Sh::N, K->p[pi]);
        if constexpr (P + 1 < Sh::NP) {
            exchange<Sh, P, P + 1, P == 0>(a, (uint64_t*)smv, tid);
            fwd_passes<Sh, FP, P + 1>(av, smv, tid, tw, K, pi);
        }
    }
}

template <class Sh, bool FP, int P, int LZ = 0, bool FOLD = false>
__device__ __forceinline__ void inv_passes(void* av, void* smv, uint32_t tid, TwRow tw, const CtxConst* K,
                                           uint32_t pi) {
    if constexpr (FP) {
        double* a = (double*)av;
        constexpr bool F = FOLD && P == Sh::NP - 1;
        inv_pass_fp<Sh, P, LZ, F>(a, tid, tw.f + 2 * Sh::N, K->pd[pi], K->pinv[pi], F ? K->foldd[pi] : 1.0);
        if constexpr (P > 0) {
            exchange<Sh, P, P - 1, P == Sh::NP - 1>(a, (double*)smv, tid);
            inv_passes<Sh, FP, P - 1, LZ, FOLD>(av, smv, tid, tw, K, pi);
        }
    } else {
        uint64_t* a = (uint64_t*)av;
        inv_pass<Sh, P>(a, tid, tw.i + 2 * Sh::N, tw.i + 3 * Sh::N, K->p[pi]);
        if constexpr (P > 0) {
            exchange<Sh, P, P - 1, P == Sh::NP - 1>(a, (uint64_t*)smv, tid);
            inv_passes<Sh, FP, P - 1>(av, smv, tid, tw, K, pi);
        }
    }
}

// fp64 transforms of integer-valued doubles v[] (first-pass pattern in, |v| <= p for the forward
// transform; any |v| < 2^53 for the inverse, whose passes start by reducing).  On return v[] holds
// the outputs reduced to [-p/2, p/2]: the forward transform in the transformed layout, the inverse
// (including N^-1) in the first pass's natural-order pattern.
// REDUCE = false (lazy transforms only) leaves the outputs unreduced, below (b (35/32)^13 + 11.8) p
// for inputs below b p; the caller reduces them later.
template <class Sh, bool LAZY = false, bool TWPAD = false, bool REDUCE = true>
__device__ __forceinline__ void ntt_fwd_f(double* v, uint64_t* sm, uint32_t tid, TwRow tw, const CtxConst* K,
                                          uint32_t pi) {
    static_assert(!LAZY || Sh::LOGN <= 13, "the lazy bound covers at most 13 stages");
    static_assert(REDUCE || LAZY, "only the lazy transform may skip its final reduction");
    fwd_passes<Sh, true, 0, LAZY, TWPAD>(v, sm, tid, tw, K, pi);
    if constexpr (REDUCE) {
        const double p = K->pd[pi], pinv = K->pinv[pi];
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) v[u] = fred(v[u], p, pinv);
    }
}
// NINV = false leaves out the factor N^-1 (the caller folds it into a later constant).  LZ > 0:
// the lazy schedules of inv_pass_fp (inputs below 1.4 p; LZ = 2 only for primes below 2^44).
// FOLD: the result is multiplied by the prime's fold constant K->foldd[pi] (see inv_pass_fp).
template <class Sh, bool NINV = true, int LZ = 0, bool FOLD = false>
__device__ __forceinline__ void ntt_inv_f(double* v, uint64_t* sm, uint32_t tid, TwRow tw, const CtxConst* K,
                                          uint32_t pi) {
    inv_passes<Sh, true, Sh::NP - 1, LZ, FOLD>(v, sm, tid, tw, K, pi);
    const double p = K->pd[pi], pinv = K->pinv[pi], ni = K->ninvd[pi];
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) v[u] = NINV ? fred(fmulmod(v[u], ni, p, pinv), p, pinv) : fred(v[u], p, pinv);
}

// Forward transform of the EPT values a[] (residues in [0, p), first-pass pattern) of thread tid;
// on return a[] holds the thread's outputs (transformed layout) reduced to [0, p).
template <class Sh, bool FP>
__device__ __forceinline__ void ntt_fwd_regs(uint64_t* a, uint64_t* sm, uint32_t tid, TwRow tw, const CtxConst* K,
                                             uint32_t pi) {
    if constexpr (FP) {
        double v[Sh::EPT];
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) v[u] = u52_to_double(a[u]);
        ntt_fwd_f<Sh>(v, sm, tid, tw, K, pi);
        const double p = K->pd[pi];
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) a[u] = fp_to_residue(v[u], p);
    } else {
        fwd_passes<Sh, false, 0>(a, sm, tid, tw, K, pi);
        const uint64_t p = K->p[pi], p2 = 2 * p;
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) {
            uint64_t x = a[u];
            x = x >= p2 ? x - p2 : x;
            a[u] = x >= p ? x - p : x;
        }
    }
}

// Inverse transform (including N^-1) of a[] (transformed layout); returns residues in [0, p) in
// the first pass's natural-order pattern.
template <class Sh, bool FP, bool NINV = true>
__device__ __forceinline__ void ntt_inv_regs(uint64_t* a, uint64_t* sm, uint32_t tid, TwRow tw, const CtxConst* K,
                                             uint32_t pi) {
    if constexpr (FP) {
        double v[Sh::EPT];
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) v[u] = u52_to_double(a[u]);
        ntt_inv_f<Sh, NINV>(v, sm, tid, tw, K, pi);
        const double p = K->pd[pi];
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) a[u] = fp_to_residue(v[u], p);
    } else {
        inv_passes<Sh, false, Sh::NP - 1>(a, sm, tid, tw, K, pi);
        const uint64_t p = K->p[pi], ni = K->ninv[pi], niq = K->ninvq[pi];
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) {
            if constexpr (NINV) {
                const uint64_t x = mul_shoup_lazy(a[u], ni, niq, p);
                a[u] = x >= p ? x - p : x;
            } else {  // inverse outputs lie in [0, 2p)
                const uint64_t x = a[u];
                a[u] = x >= p ? x - p : x;
            }
        }
    }
}

__device__ __forceinline__ TwRow tw_row(const uint64_t* tw, const double* twf, uint32_t pi, uint32_t N) {
    return TwRow{tw + (size_t)pi * 4 * N, twf ? twf + (size_t)pi * 4 * N : nullptr};
}

// ---------------------------------------------------------------------------------------------
// XCD-aware workgroup numbering.  MI355X deals workgroups to its 8 XCDs round-robin (workgroup b
// runs on XCD b mod 8), and each XCD has its own L2.  Workgroups that read the same data are
// numbered 8 apart so that they share an XCD and run close together: for a grid of `groups`
// groups of `per` workgroups, workgroup b belongs to group (b / (8 per)) * 8 + b mod 8 and is
// member (b / 8) mod per of it.  The grid is rounded up to whole sets of 8 groups; workgroups past
// the last group return at once.
// ---------------------------------------------------------------------------------------------
constexpr uint32_t XCDS = 8;
__host__ __device__ __forceinline__ size_t xcd_grid(size_t groups, uint32_t per) {
    return (groups + XCDS - 1) / XCDS * XCDS * per;
}
__device__ __forceinline__ void xcd_split(size_t b, uint32_t per, size_t& group, uint32_t& member) {
    const size_t slot = b / XCDS;
    group = slot / per * XCDS + b % XCDS;
    member = (uint32_t)(slot % per);
}

// Key-switch workgroup b -> (element-query eq, output limb j).  G = 0: xcd_split, the L limbs of an
// element on one XCD (they read the same digit rows).  G > 0: blocks of G element-queries, limb-major
// inside a block, so that workgroups running together read the same key limb.
__host__ __device__ __forceinline__ size_t relin_grid(size_t nEQ, uint32_t L, uint32_t G) {
    return G ? (nEQ + G - 1) / G * G * L : xcd_grid(nEQ, L);
}
__device__ __forceinline__ void relin_split(size_t b, uint32_t L, uint32_t G, size_t& eq, uint32_t& j) {
    if (G == 0) {
        xcd_split(b, L, eq, j);
        return;
    }
    const size_t blk = b / ((size_t)G * L), r = b % ((size_t)G * L);
    j = (uint32_t)(r / G);
    eq = blk * G + r % G;
}

// ---------------------------------------------------------------------------------------------
// Row drivers: one workgroup per row.  A row policy supplies prime(g), load(g, tid, a) (the EPT
// inputs of thread tid in the first pass's pattern: natural order for the forward transform, the
// transformed layout for the inverse) and store(g, tid, u, v) for one reduced output.
// ---------------------------------------------------------------------------------------------
template <class Sh, bool FP, class Row>
__device__ __forceinline__ void ntt_fwd_row(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                            const double* __restrict__ twf, const Row& row) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    const uint32_t tid = threadIdx.x;
    const size_t g = blockIdx.x;
    uint64_t a[Sh::EPT];
    row.load(g, tid, a);
    const uint32_t pi = row.prime(g);
    ntt_fwd_regs<Sh, FP>(a, sm, tid, tw_row(tw, twf, pi, Sh::N), K, pi);
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) row.store(g, tid, u, a[u]);
}

template <class Sh, bool FP, class Row>
__device__ __forceinline__ void ntt_inv_row(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                            const double* __restrict__ twf, const Row& row) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    const uint32_t tid = threadIdx.x;
    const size_t g = blockIdx.x;
    uint64_t a[Sh::EPT];
    row.load(g, tid, a);
    const uint32_t pi = row.prime(g);
    ntt_inv_regs<Sh, FP>(a, sm, tid, tw_row(tw, twf, pi, Sh::N), K, pi);
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) row.store(g, tid, u, a[u]);
}

// Forward outputs go to the transformed layout (u*T + tid); inverse outputs to natural order.
template <class Sh>
__device__ __forceinline__ size_t transformed_pos(size_t g, uint32_t tid, int u) {
    return g * Sh::N + (size_t)u * Sh::T + tid;
}
template <class Sh>
__device__ __forceinline__ size_t natural_pos(size_t g, uint32_t tid, int u) {
    return g * Sh::N + elem_index<Sh, 0>(tid, u);
}

// Plain rows of a [rows][N] array, prime = pbase + row mod nl.  With skip > 0 the array is blocks
// of nl rows of which the first `skip` are left as they are: transform g is row skip + g mod
// (nl - skip) of block g / (nl - skip).
template <class Sh>
struct RowsFwdU64 {
    const uint64_t* in;
    uint64_t* out;
    uint32_t nl, pbase, skip;
    __device__ size_t row(size_t g) const {
        const uint32_t w = nl - skip;
        return (g / w) * nl + skip + g % w;
    }
    __device__ uint32_t prime(size_t g) const { return pbase + (uint32_t)(row(g) % nl); }
    __device__ void load(size_t g, uint32_t tid, uint64_t* a) const {
        const size_t r = row(g);
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) a[u] = in[natural_pos<Sh>(r, tid, u)];
    }
    __device__ void store(size_t g, uint32_t tid, int u, uint64_t v) const {
        out[transformed_pos<Sh>(row(g), tid, u)] = v;
    }
};

template <class Sh>
struct RowsInvU64 {
    const uint64_t* in;
    uint64_t* out;
    uint32_t nl, pbase;
    __device__ uint32_t prime(size_t g) const { return pbase + (uint32_t)(g % nl); }
    __device__ void load(size_t g, uint32_t tid, uint64_t* a) const {
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) a[u] = in[transformed_pos<Sh>(g, tid, u)];
    }
    __device__ void store(size_t g, uint32_t tid, int u, uint64_t v) const { out[natural_pos<Sh>(g, tid, u)] = v; }
};

// Payload rows: row g = (e s + r) nl + j lifts uint16 row (e, r) (values < 2^16 < every prime, so
// the residue is the value itself) and transforms it modulo prime j of the context (the L ciphertext
// primes, then, for nl > L, the first auxiliary primes).
template <class Sh>
struct RowsPayload {
    const uint16_t* pay;
    uint64_t* out;
    uint32_t L;  // rows per uint16 row (nl)
    uint32_t q, dbase;  // rows j >= q use context prime dbase + j - q
    __device__ uint32_t prime(size_t g) const {
        const uint32_t j = (uint32_t)(g % L);
        return j < q ? j : dbase + j - q;
    }
    __device__ void load(size_t g, uint32_t tid, uint64_t* a) const {
        const uint16_t* src = pay + (g / L) * Sh::N;
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) a[u] = src[elem_index<Sh, 0>(tid, u)];
    }
    __device__ void store(size_t g, uint32_t tid, int u, uint64_t v) const { out[transformed_pos<Sh>(g, tid, u)] = v; }
};

// Relinearization staging rows: row (e, i, j) of [E][L+2][L][N] is digit i (row 2L+i of the
// coefficient-form product [E][3][L][N]) reduced mod q_j for i < L, and c0 / c1 limb j for
// i = L, L+1; the reduction is done while loading.
template <class Sh>
struct RowsDigits {
    const uint64_t* c3;
    uint64_t* out;
    const CtxConst* K;
    uint32_t L;
    __device__ uint32_t prime(size_t g) const { return (uint32_t)(g % L); }
    __device__ void load(size_t g, uint32_t tid, uint64_t* a) const {
        const uint32_t j = (uint32_t)(g % L);
        const size_t ei = g / L;
        const uint32_t i = (uint32_t)(ei % (L + 2));
        const size_t e = ei / (L + 2);
        const uint64_t* base = c3 + e * 3 * L * Sh::N;
        const uint64_t* src = i < L ? base + ((size_t)2 * L + i) * Sh::N : base + ((size_t)(i - L) * L + j) * Sh::N;
        if (i < L && i != j) {
            const uint64_t p = K->p[j], r1 = K->r1[j];
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u) a[u] = reduce64(src[elem_index<Sh, 0>(tid, u)], p, r1);
        } else {
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u) a[u] = src[elem_index<Sh, 0>(tid, u)];
        }
    }
    __device__ void store(size_t g, uint32_t tid, int u, uint64_t v) const { out[transformed_pos<Sh>(g, tid, u)] = v; }
};

// Tensor product rows fused into the inverse transform: row g = (e 3 + r) LL + l of X is
// (a0 b0, a0 b1 + a1 b0, a1 b1)[r] in limb l of element e's operands, formed while loading.  The
// three rows of one (e, l) read the same four operand rows; the kernel numbers its workgroups so
// that they run on one XCD (see xcd_split).
template <class Sh>
struct RowsTensor {
    const uint32_t* refs;
    const uint64_t* leaves;
    const uint64_t* nodes;
    uint64_t* out;
    const CtxConst* K;
    uint32_t LL;
    size_t eshift;  // rows of earlier queries in a batched launch: refs index = element - eshift
    size_t gshift;  // output row of row g is g - gshift (a launch over part of the batch)
    __device__ uint32_t prime(size_t g) const { return (uint32_t)(g % LL); }
    __device__ void load(size_t g, uint32_t tid, uint64_t* a) const {
        constexpr int N = Sh::N, T = Sh::T;
        const uint32_t l = (uint32_t)(g % LL);
        const size_t er = g / LL;
        const uint32_t r = (uint32_t)(er % 3);
        const size_t e = er / 3;
        const size_t ct = (size_t)2 * LL * N;
        const uint32_t ra = refs[2 * (e - eshift)], rb = refs[2 * (e - eshift) + 1];
        const uint64_t* A = (ra & REF_NODE) ? nodes + (size_t)(ra & ~REF_NODE) * ct : leaves + (size_t)ra * ct;
        const uint64_t* B = (rb & REF_NODE) ? nodes + (size_t)(rb & ~REF_NODE) * ct : leaves + (size_t)rb * ct;
        const uint64_t p = K->p[l], mu = K->bar_mu[l];
        const uint32_t s = K->bar_s[l];
        const size_t o0 = (size_t)l * N + tid, o1 = (size_t)(LL + l) * N + tid;
        if (r == 0) {
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u) a[u] = mul_barrett(A[o0 + u * T], B[o0 + u * T], p, mu, s);
        } else if (r == 2) {
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u) a[u] = mul_barrett(A[o1 + u * T], B[o1 + u * T], p, mu, s);
        } else {
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u)
                a[u] = add_mod(mul_barrett(A[o0 + u * T], B[o1 + u * T], p, mu, s),
                               mul_barrett(A[o1 + u * T], B[o0 + u * T], p, mu, s), p);
        }
    }
    // fp64 operand format: the operands are integer-valued doubles in [-p/2, p/2]; each product
    // is below 0.7 p in magnitude (fmulmod's bound), X1 below 1.4 p.
    __device__ void load_f(size_t g, uint32_t tid, double* a) const {
        constexpr int N = Sh::N, T = Sh::T;
        const uint32_t l = (uint32_t)(g % LL);
        const size_t er = g / LL;
        const uint32_t r = (uint32_t)(er % 3);
        const size_t e = er / 3;
        const size_t ct = (size_t)2 * LL * N;
        const uint32_t ra = refs[2 * (e - eshift)], rb = refs[2 * (e - eshift) + 1];
        const double* lv = (const double*)leaves;
        const double* nd = (const double*)nodes;
        const double* A = (ra & REF_NODE) ? nd + (size_t)(ra & ~REF_NODE) * ct : lv + (size_t)ra * ct;
        const double* B = (rb & REF_NODE) ? nd + (size_t)(rb & ~REF_NODE) * ct : lv + (size_t)rb * ct;
        const double p = K->pd[l], pinv = K->pinv[l];
        const size_t o0 = (size_t)l * N + tid, o1 = (size_t)(LL + l) * N + tid;
        if (r == 0) {
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u) a[u] = fmulmod(A[o0 + u * T], B[o0 + u * T], p, pinv);
        } else if (r == 2) {
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u) a[u] = fmulmod(A[o1 + u * T], B[o1 + u * T], p, pinv);
        } else {
#pragma unroll
            for (int u = 0; u < Sh::EPT; ++u)
                a[u] = fmulmod(A[o0 + u * T], B[o1 + u * T], p, pinv) + fmulmod(A[o1 + u * T], B[o0 + u * T], p, pinv);
        }
    }
    __device__ void store(size_t g, uint32_t tid, int u, uint64_t v) const {
        out[natural_pos<Sh>(g - gshift, tid, u)] = v;
    }
};

// Forward transform of coefficient-form rows (u64 residues in [0, p)) into the fp64 operand
// format: integer-valued doubles in [-p/2, p/2], transformed layout.
// skip: as in RowsFwdU64 (the first `skip` rows of every block of nl stay as they are).
template <class Sh>
__global__ __launch_bounds__(Sh::T) void k_ntt_fwd_operand(const CtxConst* __restrict__ K,
                                                           const uint64_t* __restrict__ tw,
                                                           const double* __restrict__ twf, const uint64_t* in,
                                                           double* out, uint32_t nl, uint32_t pbase, uint32_t skip) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    const uint32_t tid = threadIdx.x;
    const uint32_t w = nl - skip;
    const size_t g = (size_t)(blockIdx.x / w) * nl + skip + blockIdx.x % w;
    const uint32_t pi = pbase + (uint32_t)(g % nl);
    double v[Sh::EPT];
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) v[u] = u52_to_double(in[natural_pos<Sh>(g, tid, u)]);
    ntt_fwd_f<Sh>(v, sm, tid, tw_row(tw, twf, pi, Sh::N), K, pi);
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) out[transformed_pos<Sh>(g, tid, u)] = v[u];
}

template <class Sh, bool FP>
__global__ __launch_bounds__(Sh::T) void k_ntt_fwd(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                   const double* __restrict__ twf, const uint64_t* in, uint64_t* out,
                                                   uint32_t nl, uint32_t pbase, uint32_t skip) {
    ntt_fwd_row<Sh, FP>(K, tw, twf, RowsFwdU64<Sh>{in, out, nl, pbase, skip});
}
template <class Sh, bool FP>
__global__ __launch_bounds__(Sh::T) void k_ntt_inv(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                   const double* __restrict__ twf, const uint64_t* in, uint64_t* out,
                                                   uint32_t nl, uint32_t pbase) {
    ntt_inv_row<Sh, FP>(K, tw, twf, RowsInvU64<Sh>{in, out, nl, pbase});
}
template <class Sh, bool FP>
__global__ __launch_bounds__(Sh::T) void k_ntt_payload(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                       const double* __restrict__ twf, const uint16_t* __restrict__ pay,
                                                       uint64_t* __restrict__ out, uint32_t nl, uint32_t dbase) {
    ntt_fwd_row<Sh, FP>(K, tw, twf, RowsPayload<Sh>{pay, out, nl, K->L, dbase});
}
// Staged digit transforms: row g = (e, i, j) of [E][L+2][L][N].  The L workgroups of one (e, i)
// read the same digit row (reduced modulo each q_j while loading); xcd_split puts them on one XCD,
// so the row comes from HBM once and from that XCD's L2 for the others.
template <class Sh, bool FP>
__global__ __launch_bounds__(Sh::T) void k_ntt_digits(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                      const double* __restrict__ twf, const uint64_t* __restrict__ c3,
                                                      uint64_t* __restrict__ out, size_t groups) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    const uint32_t L = K->L, tid = threadIdx.x;
    size_t grp;
    uint32_t j;
    xcd_split(blockIdx.x, L, grp, j);
    if (grp >= groups) return;
    const size_t g = grp * L + j;
    const RowsDigits<Sh> row{c3, out, K, L};
    uint64_t a[Sh::EPT];
    row.load(g, tid, a);
    ntt_fwd_regs<Sh, FP>(a, sm, tid, tw_row(tw, twf, j, Sh::N), K, j);
#pragma unroll
    for (int u = 0; u < Sh::EPT; ++u) row.store(g, tid, u, a[u]);
}
template <class Sh, bool FP>
__global__ __launch_bounds__(Sh::T, Sh::LOGN == 13 ? 8 : 1) void k_ntt_inv_tensor(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                          const double* __restrict__ twf,
                                                          const uint32_t* __restrict__ refs, const Batch bt,
                                                          uint64_t* __restrict__ X, size_t groups, size_t eq0) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    size_t el;
    uint32_t r;
    xcd_split(blockIdx.x, 3, el, r);
    if (el >= groups) return;
    const uint32_t LL = K->LL;
    const size_t eq = eq0 + el / LL;      // row of the batch: query q, element e; X holds rows from eq0 on
    const uint32_t q = (uint32_t)(eq / bt.E);
    const size_t g = (eq * 3 + r) * LL + el % LL;
    const RowsTensor<Sh> row{refs, bt.leaves[q], bt.nodes[q], X, K, LL, (size_t)q * bt.E, eq0 * 3 * LL};
    const uint32_t tid = threadIdx.x;
    const uint32_t pi = row.prime(g);
    // X leaves without the transform's factor N^-1: the scale kernels, its only readers, take it
    // with their first constants (tqinv, kb1), which the fp64 transform multiplies in at its first
    // stage (X row k holds [f_k x]_{p_k}, f = K->foldd, as centred doubles).  The tensor products
    // enter below 1.4 p, so the inverse transform takes a lazy schedule (rows modulo primes below
    // 2^44 almost unreduced).
    if constexpr (FP) {
        double v[Sh::EPT];
        row.load_f(g, tid, v);
        constexpr int LZB = inv_lazy_exact<Sh>(1) ? 1 : 0;    // a first pass of three stages from 1.4 p
        constexpr int LZQ = inv_lazy_exact<Sh>(2) ? 2 : LZB;  // would reach 11.2 p, beyond 8 p below 2^50
        if (K->pd[pi] < 0x1p44) ntt_inv_f<Sh, false, LZQ, true>(v, sm, tid, tw_row(tw, twf, pi, Sh::N), K, pi);
        else ntt_inv_f<Sh, false, LZB, true>(v, sm, tid, tw_row(tw, twf, pi, Sh::N), K, pi);
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) row.store(g, tid, u, (uint64_t)__double_as_longlong(v[u]));  // centred
    } else {
        uint64_t a[Sh::EPT];
        row.load(g, tid, a);
        ntt_inv_regs<Sh, FP, false>(a, sm, tid, tw_row(tw, twf, pi, Sh::N), K, pi);
#pragma unroll
        for (int u = 0; u < Sh::EPT; ++u) row.store(g, tid, u, a[u]);
    }
}

// ---------------------------------------------------------------------------------------------
// Key switching fused with the digit transforms: workgroup (e, j) transforms, one after the other,
// the L digits [c2_i]_{q_i} reduced mod q_j and the rows c0_j, c1_j, and accumulates
//   sel0 = c0^ + sum_i D_i^ b_ij^,  sel1 = c1^ + sum_i D_i^ a_ij^   (mod q_j)
// in registers, so the transformed digits never leave the chip.  rlk: [L][2][L][N] transformed
// values followed by [L][2][L][N] Shoup companions; out: sel [E][2][L][N] (transformed).
// ---------------------------------------------------------------------------------------------


template <class Sh>
__global__ __launch_bounds__(Sh::T) void k_relin(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                 const double* __restrict__ twf, const uint64_t* __restrict__ c3,
                                                 const Batch bt, uint32_t G) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    constexpr int N = Sh::N, T = Sh::T, EPT = Sh::EPT;
    const uint32_t L = K->L, tid = threadIdx.x;
    size_t eq;
    uint32_t j;
    relin_split(blockIdx.x, L, G, eq, j);
    if (eq >= (size_t)bt.nq * bt.E) return;
    const uint32_t q = (uint32_t)(eq / bt.E);
    const size_t e = eq % bt.E;
    uint64_t* __restrict__ sel = bt.sel[q];
    const TwRow twr = tw_row(tw, twf, j, N);
    const uint64_t* base = c3 + eq * 3 * L * N;
    const size_t LN = (size_t)L * N;
    uint64_t* o0 = sel + e * 2 * LN + (size_t)j * N + tid;
    {
        const uint64_t* __restrict__ rlk = bt.rlk[q];
        const uint64_t p = K->p[j], r1 = K->r1[j];
        const size_t half = (size_t)L * 2 * LN;
        uint64_t acc0[EPT], acc1[EPT], a[EPT];
        for (uint32_t i = 0; i < L + 2; ++i) {
            uint32_t t = tid;
            TwRow tr = twr;
            asm volatile("" : "+v"(t), "+v"(tr.i), "+v"(tr.f));
            const uint64_t* src = i < L ? base + ((size_t)2 * L + i) * N : base + ((size_t)(i - L) * L + j) * N;
            if (i < L && i != j) {
#pragma unroll
                for (int u = 0; u < EPT; ++u) a[u] = reduce64(src[elem_index<Sh, 0>(t, u)], p, r1);
            } else {
#pragma unroll
                for (int u = 0; u < EPT; ++u) a[u] = src[elem_index<Sh, 0>(t, u)];
            }
            ntt_fwd_regs<Sh, false>(a, sm, t, tr, K, j);
            asm volatile("" ::: "memory");
            if (i < L) {
                const uint64_t* bh = rlk + ((size_t)i * 2 + 0) * LN + (size_t)j * N + t;
                const uint64_t* ah = rlk + ((size_t)i * 2 + 1) * LN + (size_t)j * N + t;
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const size_t o = (size_t)u * T;
                    const uint64_t tb = mul_shoup(a[u], bh[o], bh[half + o], p);
                    const uint64_t ta = mul_shoup(a[u], ah[o], ah[half + o], p);
                    acc0[u] = i == 0 ? tb : add_mod(acc0[u], tb, p);
                    acc1[u] = i == 0 ? ta : add_mod(acc1[u], ta, p);
                }
            } else {
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    if (i == L) acc0[u] = add_mod(acc0[u], a[u], p);
                    else acc1[u] = add_mod(acc1[u], a[u], p);
                }
            }
            asm volatile("" ::: "memory");
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            o0[(size_t)u * T] = acc0[u];
            o0[LN + (size_t)u * T] = acc1[u];
        }
    }
}

// N = 16384 does not fit 16 elements plus two accumulators per thread in the 128 registers that a
// 1024-thread workgroup allows; there the digits are transformed to `staging` [E][L+2][L][N] and
// multiplied-accumulated by a second kernel.
// fp64 key switch (every prime below 2^50).  The key is in the fp64 operand format (entries in
// [-p/2, p/2]); the digits D_i < q_i are exact doubles.  Without LAZY every digit is reduced mod q_j
// by fred and every transform output to [-p/2, p/2], so each product is below 0.7 p and each
// accumulator below (0.7 L + 0.5) p < 2^53.  LAZY (every ciphertext prime below 2^48, and
// (2.4 L + 16) max q_i < 2^53, checked by the host): a digit with q_i <= 2.5 q_j enters the
// transform as it is (else it is reduced first) and no transform output is reduced.  Outputs stay
// below 19.8 q_j (the stage bound below, from 2.5 q_j), each product below (1/2 + 3 * 19.8 / 32) q_j
// < 2.4 q_j, the c0 and c1 transforms below 15 q_j, so each accumulator stays below (2.4 L + 15) q_j:
// every sum is exact, and the final fred brings it to [-p/2, p/2].
// All L + 2 transforms of the workgroup use prime q_j: its forward twiddles are staged in LDS once,
// which leaves global memory to the operand rows.  The next operand row is loaded while the
// current one is transformed (no global load inside the transform waits behind it).
template <class Sh, bool LAZY>
__global__ __launch_bounds__(Sh::T) void k_relin_f(const CtxConst* __restrict__ K, const double* __restrict__ twf,
                                                   const uint64_t* __restrict__ c3, const Batch bt, uint32_t G) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    __shared__ double twl[Sh::LDS_WORDS];  // padded like the exchange buffer
    constexpr int N = Sh::N, T = Sh::T, EPT = Sh::EPT;
    const uint32_t L = K->L, tid = threadIdx.x;
    size_t eq;
    uint32_t j;
    relin_split(blockIdx.x, L, G, eq, j);
    if (eq >= (size_t)bt.nq * bt.E) return;
    const uint32_t q = (uint32_t)(eq / bt.E);
    const size_t e = eq % bt.E;
    {
        const double* __restrict__ g = twf + (size_t)j * 4 * N;  // forward twiddles of q_j
#pragma unroll
        for (int u = 0; u < EPT; ++u) twl[lds_pad(u * T + tid)] = g[u * T + tid];
    }
    const double* __restrict__ rlk = (const double*)bt.rlk[q];
    uint64_t* __restrict__ sel = bt.sel[q];
    const uint64_t* base = c3 + eq * 3 * L * N;
    const size_t LN = (size_t)L * N;
    const double p = K->pd[j], pinv = K->pinv[j];
    auto src_row = [&](uint32_t i) {
        return i < L ? base + ((size_t)2 * L + i) * N : base + ((size_t)(i - L) * L + j) * N;
    };
    uint64_t nx[EPT];
    {
        const uint64_t* src = src_row(0);
#pragma unroll
        for (int u = 0; u < EPT; ++u) nx[u] = src[elem_index<Sh, 0>(tid, u)];
    }
    __syncthreads();  // twiddles staged
    double acc0[EPT], acc1[EPT], v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) acc0[u] = acc1[u] = 0.0;
    for (uint32_t i = 0; i < L + 2; ++i) {
        // The transform's index arithmetic does not depend on i; an opaque copy of the thread index
        // per iteration keeps the compiler from hoisting all of it out of the loop into registers.
        uint32_t t = tid;
        asm volatile("" : "+v"(t));
        // Lazy transforms start from the digit as it is when q_i <= 2.5 q_j (the outputs then stay
        // below 19.8 q_j); otherwise the digit is first reduced mod q_j.
        const bool reduce = !LAZY || (i < L && i != j && K->pd[i] > 2.5 * p);
        if (reduce) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) v[u] = fred(u52_to_double(nx[u]), p, pinv);
        } else {
#pragma unroll
            for (int u = 0; u < EPT; ++u) v[u] = u52_to_double(nx[u]);
        }
        if (i + 1 < L + 2) {
            const uint64_t* src = src_row(i + 1);
#pragma unroll
            for (int u = 0; u < EPT; ++u) nx[u] = src[elem_index<Sh, 0>(t, u)];
        }
        ntt_fwd_f<Sh, LAZY, true, !LAZY>(v, sm, t, TwRow{nullptr, twl}, K, j);
        asm volatile("" ::: "memory");  // keep the key loads below the transform
        if (i < L) {
            const double* bh = rlk + ((size_t)i * 2 + 0) * LN + (size_t)j * N + t;
            const double* ah = rlk + ((size_t)i * 2 + 1) * LN + (size_t)j * N + t;
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const size_t o = (size_t)u * T;
                acc0[u] += fmulmod(v[u], bh[o], p, pinv);
                acc1[u] += fmulmod(v[u], ah[o], p, pinv);
            }
        } else {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                if (i == L) acc0[u] = acc0[u] + v[u];
                else acc1[u] = acc1[u] + v[u];
            }
        }
        asm volatile("" ::: "memory");
    }
    uint64_t* o0 = sel + e * 2 * LN + (size_t)j * N + tid;
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        o0[(size_t)u * T] = fp_to_residue(fred(acc0[u], p, pinv), p);
        o0[LN + (size_t)u * T] = fp_to_residue(fred(acc1[u], p, pinv), p);
    }
}

void launch_relin(const Launch& lc, const uint64_t* c3, const Batch& bt, uint64_t* staging) {
    if (!bt.E || !bt.nq) return;
    const unsigned blocks = (unsigned)relin_grid((size_t)bt.nq * bt.E, lc.L, lc.relin_group);
    const uint32_t G = lc.relin_group;
    if (relin_needs_staging(lc.logN)) {
        launch_ntt_digits(lc, c3, staging, bt.nq * bt.E);
        launch_relin_mac(lc, staging, bt);
        return;
    }
    with_shape(lc.logN, lc.shape, [&](auto tag) {
        using Sh = decltype(tag);
        if constexpr (Sh::LOGN <= 13) {
            if (lc.fp && lc.q_lazy)
                hipLaunchKernelGGL((k_relin_f<Sh, true>), dim3(blocks), dim3(Sh::T), 0, lc.stream, lc.K, lc.twf, c3,
                                   bt, G);
            else if (lc.fp)
                hipLaunchKernelGGL((k_relin_f<Sh, false>), dim3(blocks), dim3(Sh::T), 0, lc.stream, lc.K, lc.twf, c3,
                                   bt, G);
            else
                hipLaunchKernelGGL((k_relin<Sh>), dim3(blocks), dim3(Sh::T), 0, lc.stream, lc.K, lc.tw, lc.twf, c3,
                                   bt, G);
        }
    });
}

bool relin_needs_staging(uint32_t logN) { return logN >= 14; }

// ---------------------------------------------------------------------------------------------
// Root products with the key switch deferred past the inner product.
//
// The answer is linear in every selector.  With element e's root product c = (c0, c1, c2) and its
// relinearization digits D_i = [c2]_{q_i} (integers in [0, q_i)),
//   sel_e = (c0 + sum_i D_i b_i, c1 + sum_i D_i a_i)   and so
//   answer_r = (sum_e c0 P_er + sum_i b_i W_ir,  sum_e c1 P_er + sum_i a_i W_ir),   W_ir = sum_e D_ei P_er
// in R_q: the same residues as relinearizing every element first.  W_ir is a sum of negacyclic
// products of small non-negative integer polynomials, so its coefficients are integers below
// n N max q_i 2^16 in magnitude; two auxiliary primes with b0 b1 above twice that bound hold it
// exactly (the host checks the bound per database), and W_ir mod q_j follows by CRT once per
// answer.  Per element that is 2L transforms modulo the q_j (c0, c1) and 2L modulo b0, b1 (the
// digits), against L^2 + 2L and 2 L^2 N key products for relinearizing it; the key multiplies the
// L digit sums once per answer.
//
// k_root_pm_f: workgroup (slice, query, unit) transforms the unit's one or two rows of every element
// of its slice (all modulo one prime, whose forward twiddles are staged in LDS once), multiplies
// each by the element's transformed payload rows modulo that prime and sums them in registers; the
// sums leave as residues in [0, p) into part[slice][q][r][row][N].  Workgroups of one slice share
// an XCD (xcd_split), with the units of one prime side by side (they read the same payload rows).
// Bounds: without LAZY a transform output is in [-p/2, p/2] and each product below (1/2 + 2^-5) p,
// so eight products keep a sum below 4.3 p + p/2 < 2^53 before it is reduced again.  LAZY (every
// prime of the launch below 2^48; the two digit-sum primes always are): inputs below p, no
// reduction between passes or of the outputs, which stay below 15 p (the lazy stage bound); each
// product is then below (1/2 + 3 * 15 / 32) p < 2 p and eight of them, with the reduced sum, below
// 16.5 p < 2^53.
// ---------------------------------------------------------------------------------------------
template <class Sh, int S, bool TWO, bool LAZY>
__global__ __launch_bounds__(Sh::T) void k_root_pm_f(const CtxConst* __restrict__ K, const double* __restrict__ twf,
                                                     const uint64_t* __restrict__ C, const uint64_t* __restrict__ Ph,
                                                     uint64_t* __restrict__ part, const RootPlan rp) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    __shared__ double twl[Sh::LDS_WORDS];  // padded like the exchange buffer
    constexpr int N = Sh::N, T = Sh::T, EPT = Sh::EPT;
    const uint32_t L = K->L, tid = threadIdx.x;
    size_t sl;
    uint32_t mem;
    xcd_split(blockIdx.x, rp.nq * rp.U, sl, mem);
    if (sl >= rp.nslices) return;
    const uint32_t q = mem % rp.nq;
    const RootUnit un = rp.u[mem / rp.nq];
    const uint32_t pr = un.prime;
    {
        const double* __restrict__ g = twf + (size_t)pr * 4 * N;  // forward twiddles of the unit's prime
#pragma unroll
        for (int u = 0; u < EPT; ++u) twl[lds_pad(u * T + tid)] = g[u * T + tid];
    }
    const double p = K->pd[pr], pinv = K->pinv[pr];
    // a digit (rows 2L..3L-1 of the product) may exceed the unit's prime: reduce it first
    const bool red0 = un.src0 >= 2 * L && K->pd[un.src0 - 2 * L] > p;
    const bool two = TWO && un.two;
    const bool red1 = two && un.src1 >= 2 * L && K->pd[un.src1 - 2 * L] > p;
    const uint32_t e0 = (uint32_t)sl * rp.slice;
    const uint32_t e1 = min(rp.E, e0 + rp.slice);
    double acc0[S][EPT], acc1[TWO ? S : 1][EPT], v[EPT];
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
        for (int u = 0; u < EPT; ++u) acc0[r][u] = 0.0;
    if constexpr (TWO) {
#pragma unroll
        for (int r = 0; r < S; ++r)
#pragma unroll
            for (int u = 0; u < EPT; ++u) acc1[r][u] = 0.0;
    }
    // steps i = (element, row): the next step's row is loaded while the current one is transformed
    const uint32_t per = two ? 2u : 1u, steps = (e1 - e0) * per;
    auto src_of = [&](uint32_t i) {
        const uint32_t e = e0 + i / per;
        return C + ((size_t)q * rp.E + e) * 3 * L * N + (size_t)((i % per) ? un.src1 : un.src0) * N;
    };
    uint64_t nx[EPT];
    {
        const uint64_t* src = src_of(0);
#pragma unroll
        for (int u = 0; u < EPT; ++u) nx[u] = src[elem_index<Sh, 0>(tid, u)];
    }
    // One payload row per element (S = 1, every unit has nr = 1 and r0 = 0): the row of the next
    // element is loaded once its predecessor's last product is taken, so that it arrives during the
    // next transform instead of after it.
    constexpr bool PF = S == 1;
    auto prow_of = [&](uint32_t e) {
        return Ph + ((size_t)e * rp.s + un.r0) * rp.LP * N + (size_t)un.prow * N;
    };
    uint64_t pw[PF ? EPT : 1];
    if constexpr (PF) {
        const uint64_t* s0 = prow_of(e0) + tid;
#pragma unroll
        for (int u = 0; u < EPT; ++u) pw[u] = s0[(size_t)u * T];
    }
    __syncthreads();  // twiddles staged
    for (uint32_t i = 0; i < steps; ++i) {
        uint32_t t = tid;
        asm volatile("" : "+v"(t));  // keep the per-row index arithmetic out of registers across rows
        const uint32_t e = e0 + i / per, k = i % per;
        const bool red = k ? red1 : red0;
#pragma unroll
        for (int u = 0; u < EPT; ++u) v[u] = u52_to_double(nx[u]);
        if (red) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) v[u] = fred(v[u], p, pinv);
        }
        if (i + 1 < steps) {
            const uint64_t* src = src_of(i + 1);
#pragma unroll
            for (int u = 0; u < EPT; ++u) nx[u] = src[elem_index<Sh, 0>(t, u)];
        }
        ntt_fwd_f<Sh, LAZY, true, !LAZY>(v, sm, t, TwRow{nullptr, twl}, K, pr);
        asm volatile("" ::: "memory");  // keep the payload loads below the transform
        if constexpr (PF) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const double w = u52_to_double(pw[u]);
                if constexpr (TWO) {
                    if (k) acc1[0][u] += fmulmod(v[u], w, p, pinv);
                    else acc0[0][u] += fmulmod(v[u], w, p, pinv);
                } else {
                    acc0[0][u] += fmulmod(v[u], w, p, pinv);
                }
            }
            if (k + 1 == per && e + 1 < e1) {
                const uint64_t* sn = prow_of(e + 1) + t;
#pragma unroll
                for (int u = 0; u < EPT; ++u) pw[u] = sn[(size_t)u * T];
            }
        }
        const uint64_t* ph = prow_of(e);
#pragma unroll
        for (int r = 0; r < (PF ? 0 : S); ++r) {
            if (r < (int)un.nr) {
                const uint64_t* pr_row = ph + (size_t)r * rp.LP * N + t;
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const double w = u52_to_double(pr_row[(size_t)u * T]);
                    if constexpr (TWO) {
                        if (k) acc1[r][u] += fmulmod(v[u], w, p, pinv);
                        else acc0[r][u] += fmulmod(v[u], w, p, pinv);
                    } else {
                        acc0[r][u] += fmulmod(v[u], w, p, pinv);
                    }
                }
            }
        }
        asm volatile("" ::: "memory");
        if (k + 1 == per && ((e - e0) & 7u) == 7u) {
#pragma unroll
            for (int r = 0; r < S; ++r)
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    acc0[r][u] = fred(acc0[r][u], p, pinv);
                    if constexpr (TWO) acc1[r][u] = fred(acc1[r][u], p, pinv);
                }
        }
    }
    const size_t LPS = (size_t)rp.RR * N;  // one r block of part
    uint64_t* out = part + ((sl * rp.nq + q) * rp.s) * LPS + tid;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        if (r < (int)un.nr) {
            uint64_t* o0 = out + (size_t)(un.r0 + r) * LPS + (size_t)un.row0 * N;
            uint64_t* o1 = out + (size_t)(un.r0 + r) * LPS + (size_t)un.row1 * N;
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                o0[(size_t)u * T] = fp_to_residue(fred(acc0[r][u], p, pinv), p);
                if constexpr (TWO)
                    if (two) o1[(size_t)u * T] = fp_to_residue(fred(acc1[r][u], p, pinv), p);
            }
        }
    }
}

// Integer form of k_root_pm_f (some prime at or above 2^50, or N = 16384): the same units and
// sums with the integer transform, whose twiddles (value and Shoup companion) come from global
// memory (at N = 16384 the exchange buffer leaves no room for them in LDS), and Barrett products of
// the transformed row with the payload rows, added into accumulators kept in [0, p).  The next
// row is loaded during the current transform where eight elements per thread leave the registers
// for it (N <= 8192).
template <class Sh, int S, bool TWO>
__global__ __launch_bounds__(Sh::T) void k_root_pm_i(const CtxConst* __restrict__ K, const uint64_t* __restrict__ tw,
                                                     const uint64_t* __restrict__ C, const uint64_t* __restrict__ Ph,
                                                     uint64_t* __restrict__ part, const RootPlan rp) {
    __shared__ uint64_t sm[Sh::LDS_WORDS];
    constexpr int N = Sh::N, T = Sh::T, EPT = Sh::EPT;
    constexpr bool PF = EPT <= 8;
    const uint32_t L = K->L, tid = threadIdx.x;
    size_t sl;
    uint32_t mem;
    xcd_split(blockIdx.x, rp.nq * rp.U, sl, mem);
    if (sl >= rp.nslices) return;
    const uint32_t q = mem % rp.nq;
    const RootUnit un = rp.u[mem / rp.nq];
    const uint32_t pr = un.prime;
    const uint64_t p = K->p[pr], r1 = K->r1[pr], mu = K->bar_mu[pr];
    const uint32_t sb = K->bar_s[pr];
    const TwRow twr = tw_row(tw, nullptr, pr, N);
    // a digit (rows 2L..3L-1 of the product) may exceed the unit's prime: reduce it first
    const bool red0 = un.src0 >= 2 * L && K->p[un.src0 - 2 * L] > p;
    const bool two = TWO && un.two;
    const bool red1 = two && un.src1 >= 2 * L && K->p[un.src1 - 2 * L] > p;
    const uint32_t e0 = (uint32_t)sl * rp.slice;
    const uint32_t e1 = min(rp.E, e0 + rp.slice);
    uint64_t acc0[S][EPT], acc1[TWO ? S : 1][EPT], a[EPT];
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
        for (int u = 0; u < EPT; ++u) acc0[r][u] = 0;
    if constexpr (TWO) {
#pragma unroll
        for (int r = 0; r < S; ++r)
#pragma unroll
            for (int u = 0; u < EPT; ++u) acc1[r][u] = 0;
    }
    const uint32_t per = two ? 2u : 1u, steps = (e1 - e0) * per;
    auto src_of = [&](uint32_t i) {
        const uint32_t e = e0 + i / per;
        return C + ((size_t)q * rp.E + e) * 3 * L * N + (size_t)((i % per) ? un.src1 : un.src0) * N;
    };
    uint64_t nx[PF ? EPT : 1];
    if constexpr (PF) {
        const uint64_t* src = src_of(0);
#pragma unroll
        for (int u = 0; u < EPT; ++u) nx[u] = src[elem_index<Sh, 0>(tid, u)];
    }
    for (uint32_t i = 0; i < steps; ++i) {
        uint32_t t = tid;
        asm volatile("" : "+v"(t));  // keep the per-row index arithmetic out of registers across rows
        const uint32_t e = e0 + i / per, k = i % per;
        const bool red = k ? red1 : red0;
        if constexpr (PF) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) a[u] = nx[u];
            if (i + 1 < steps) {
                const uint64_t* src = src_of(i + 1);
#pragma unroll
                for (int u = 0; u < EPT; ++u) nx[u] = src[elem_index<Sh, 0>(t, u)];
            }
        } else {
            const uint64_t* src = src_of(i);
#pragma unroll
            for (int u = 0; u < EPT; ++u) a[u] = src[elem_index<Sh, 0>(t, u)];
        }
        if (red) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) a[u] = reduce64(a[u], p, r1);
        }
        ntt_fwd_regs<Sh, false>(a, sm, t, twr, K, pr);
        asm volatile("" ::: "memory");  // keep the payload loads below the transform
        const uint64_t* ph = Ph + ((size_t)e * rp.s + un.r0) * rp.LP * N + (size_t)un.prow * N;
#pragma unroll
        for (int r = 0; r < S; ++r) {
            if (r < (int)un.nr) {
                const uint64_t* pr_row = ph + (size_t)r * rp.LP * N + t;
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const uint64_t x = mul_barrett(a[u], pr_row[(size_t)u * T], p, mu, sb);
                    if constexpr (TWO) {
                        if (k) acc1[r][u] = add_mod(acc1[r][u], x, p);
                        else acc0[r][u] = add_mod(acc0[r][u], x, p);
                    } else {
                        acc0[r][u] = add_mod(acc0[r][u], x, p);
                    }
                }
            }
        }
        asm volatile("" ::: "memory");
    }
    const size_t LPS = (size_t)rp.RR * N;  // one r block of part
    uint64_t* out = part + ((sl * rp.nq + q) * rp.s) * LPS + tid;
#pragma unroll
    for (int r = 0; r < S; ++r) {
        if (r < (int)un.nr) {
            uint64_t* o0 = out + (size_t)(un.r0 + r) * LPS + (size_t)un.row0 * N;
            uint64_t* o1 = out + (size_t)(un.r0 + r) * LPS + (size_t)un.row1 * N;
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                o0[(size_t)u * T] = acc0[r][u];
                if constexpr (TWO)
                    if (two) o1[(size_t)u * T] = acc1[r][u];
            }
        }
    }
}

void launch_root_pm(const Launch& lc, const uint64_t* C, const uint64_t* Ph, const RootPlan& plan, uint64_t* part) {
    if (!plan.E || !plan.nq) return;
    const unsigned blocks = (unsigned)xcd_grid(plan.nslices, plan.nq * plan.U);
    // one payload row per element: units are row pairs; otherwise single rows with up to two
    // payload rows (the accumulators stay at 2 EPT doubles per thread either way)
    const bool pairs = plan.s == 1;
    with_shape(lc.logN, lc.shape, [&](auto tag) {
        using Sh = decltype(tag);
        if (!lc.fp) {
            if (pairs)
                hipLaunchKernelGGL((k_root_pm_i<Sh, 1, true>), dim3(blocks), dim3(Sh::T), 0, lc.stream, lc.K, lc.tw, C,
                                   Ph, part, plan);
            else
                hipLaunchKernelGGL((k_root_pm_i<Sh, 2, false>), dim3(blocks), dim3(Sh::T), 0, lc.stream, lc.K, lc.tw,
                                   C, Ph, part, plan);
            return;
        }
        if constexpr (Sh::LOGN <= 13) {
#define CW_ROOT(SS, TW, LZ)                                                                                  \
    hipLaunchKernelGGL((k_root_pm_f<Sh, SS, TW, LZ>), dim3(blocks), dim3(Sh::T), 0, lc.stream, lc.K, lc.twf, C, Ph, \
                       part, plan)
            if (pairs) {
                if (plan.lazy) CW_ROOT(1, true, true);
                else CW_ROOT(1, true, false);
            } else {
                if (plan.lazy) CW_ROOT(2, false, true);
                else CW_ROOT(2, false, false);
            }
#undef CW_ROOT
        }
    });
}

// racc_q[r][row][c] += sum over slices of part[slice][q][r][row][c] (mod the row's prime).
__global__ void k_root_reduce(const CtxConst* __restrict__ K, const uint64_t* __restrict__ part, const RootPlan rp,
                              const QueryPtrs qp) {
    const uint32_t N = K->N, L = K->L;
    const size_t per = (size_t)rp.s * rp.RR * N;  // one query's accumulators
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= per * rp.nq) return;
    const uint32_t q = (uint32_t)(gid / per);
    const size_t x = gid % per;
    const uint32_t row = (uint32_t)((x >> K->logN) % rp.RR);  // N is a power of two
    const uint32_t pi = row < 2 * L ? row % L : K->LL + (row - 2 * L) % rp.A;
    const uint64_t p = K->p[pi];
    uint64_t a = qp.acc[q][x];
    for (uint32_t sl = 0; sl < rp.nslices; ++sl) a = add_mod(a, part[((size_t)sl * rp.nq + q) * per + x], p);
    qp.acc[q][x] = a;
}

void launch_root_reduce(const Launch& lc, const uint64_t* part, const RootPlan& plan, const QueryPtrs& qp) {
    const size_t n = (size_t)plan.nq * plan.s * plan.RR * lc.N;
    if (!n) return;
    hipLaunchKernelGGL(k_root_reduce, dim3(blocks_for(n)), dim3(EW_THREADS), 0, lc.stream, lc.K, part, plan, qp);
}

// Wc [s][L][2][N] -> WQ [s][L][L][N] (see launch_root_crt).
__global__ void k_root_crt(const CtxConst* __restrict__ K, const CrtConst cc, const uint64_t* __restrict__ Wc,
                           uint32_t s, uint64_t* __restrict__ WQ) {
    const uint32_t N = K->N, L = K->L;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)s * L * N) return;
    const size_t c = gid & (N - 1), ri = gid >> K->logN;  // ri = r L + i (N is a power of two)
    const uint64_t b0 = K->p[K->LL], b1 = K->p[K->LL + 1];
    const uint64_t w0 = Wc[(ri * 2 + 0) * N + c], w1 = Wc[(ri * 2 + 1) * N + c];
    // t = (w1 - w0) b0^-1 mod b1; w0 < b0 < 2 b1
    const uint64_t w0b = w0 >= b1 ? w0 - b1 : w0;
    const uint64_t t = mul_shoup(sub_mod(w1, w0b, b1), cc.b0inv, cc.b0invq, b1);
    // w = w0 + b0 t in [0, b0 b1); centred: subtract b0 b1 when w > (b0 b1 - 1) / 2
    const uint64_t lo = b0 * t, hi = __umul64hi(b0, t);
    const uint64_t wlo = lo + w0, whi = hi + (wlo < lo ? 1u : 0u);
    const bool neg = whi > cc.half_hi || (whi == cc.half_hi && wlo > cc.half_lo);
    uint64_t* o = WQ + ri * L * N + c;
    for (uint32_t j = 0; j < L; ++j) {
        const uint64_t p = K->p[j], r1 = K->r1[j];
        uint64_t x = add_mod(reduce64(w0, p, r1), mul_shoup(reduce64(t, p, r1), cc.b0q[j], cc.b0qq[j], p), p);
        if (neg) x = sub_mod(x, cc.Bq[j], p);
        o[(size_t)j * N] = x;
    }
}

void launch_root_crt(const Launch& lc, const CrtConst& cc, const uint64_t* Wc, uint32_t s, uint64_t* WQ) {
    const size_t n = (size_t)s * lc.L * lc.N;
    if (!n) return;
    hipLaunchKernelGGL(k_root_crt, dim3(blocks_for(n)), dim3(EW_THREADS), 0, lc.stream, lc.K, cc, Wc, s, WQ);
}

// answer[r][poly][j][c] = racc[r][poly L + j][c] + sum_i WQ^[r][i][j][c] key[i][poly][j][c] mod q_j.
__global__ void k_root_combine(const CtxConst* __restrict__ K, const uint64_t* __restrict__ racc,
                               const uint64_t* __restrict__ WQ, const uint64_t* __restrict__ rlk, uint32_t s,
                               uint32_t RR, uint64_t* __restrict__ answer) {
    const uint32_t N = K->N, L = K->L;
    const size_t LN = (size_t)L * N;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)s * 2 * LN) return;
    const size_t c = gid & (N - 1);
    const uint32_t j = (uint32_t)((gid >> K->logN) % L);
    const uint32_t poly = (uint32_t)((gid / LN) % 2);
    const uint32_t r = (uint32_t)(gid / (2 * LN));
    const uint64_t p = K->p[j], mu = K->bar_mu[j];
    const uint32_t sb = K->bar_s[j];
    uint64_t a = racc[((size_t)r * RR + poly * L + j) * N + c];
    const size_t half = (size_t)L * 2 * LN;  // integer keys: companions follow the values
    for (uint32_t i = 0; i < L; ++i) {
        const uint64_t w = WQ[(((size_t)r * L + i) * L + j) * N + c];
        const size_t ko = ((size_t)i * 2 + poly) * LN + (size_t)j * N + c;
        uint64_t kv;
        if (K->fp) {
            kv = fp_to_residue(((const double*)rlk)[ko], K->pd[j]);
            a = add_mod(a, mul_barrett(w, kv, p, mu, sb), p);
        } else {
            a = add_mod(a, mul_shoup(w, rlk[ko], rlk[half + ko], p), p);
        }
    }
    answer[gid] = a;
}

void launch_root_combine(const Launch& lc, const uint64_t* racc, const uint64_t* WQ, const uint64_t* rlk, uint32_t s,
                         uint32_t RR, uint64_t* answer) {
    const size_t n = (size_t)s * 2 * lc.L * lc.N;
    if (!n) return;
    hipLaunchKernelGGL(k_root_combine, dim3(blocks_for(n)), dim3(EW_THREADS), 0, lc.stream, lc.K, racc, WQ, rlk, s, RR,
                       answer);
}

// Static LDS of the transform kernels stays below the 160 KiB per workgroup of gfx950; nothing to
// raise at run time.
hipError_t kernels_init() { return hipSuccess; }

// Dispatch on the ring degree and on the transform arithmetic (fp64 only for N <= 8192: the
// N = 16384 shape has four-stage passes, outside the fp64 bound).
#define CW_FP_SPLIT(LC, KERN, GRID, ...)                                                                      \
    if ((LC).fp) hipLaunchKernelGGL((KERN<Sh, true>), GRID, dim3(Sh::T), 0, (LC).stream, __VA_ARGS__);          \
    else hipLaunchKernelGGL((KERN<Sh, false>), GRID, dim3(Sh::T), 0, (LC).stream, __VA_ARGS__);
#define CW_NTT_DISPATCH(LC, KERN, GRID, ...)                                                                 \
    switch (shape_key((LC).logN, (LC).shape)) {                                                             \
        case shape_key(12, 0): {                                                                            \
            using Sh = ShapeVar<12, 0>::type;                                                               \
            CW_FP_SPLIT(LC, KERN, GRID, __VA_ARGS__)                                                        \
        } break;                                                                                            \
        case shape_key(13, 0): {                                                                            \
            using Sh = ShapeVar<13, 0>::type;                                                               \
            CW_FP_SPLIT(LC, KERN, GRID, __VA_ARGS__)                                                        \
        } break;                                                                                            \
        case shape_key(13, 1): {                                                                            \
            using Sh = ShapeVar<13, 1>::type;                                                               \
            CW_FP_SPLIT(LC, KERN, GRID, __VA_ARGS__)                                                        \
        } break;                                                                                            \
        case shape_key(13, 2): {                                                                            \
            using Sh = ShapeVar<13, 2>::type;                                                               \
            CW_FP_SPLIT(LC, KERN, GRID, __VA_ARGS__)                                                        \
        } break;                                                                                            \
        case shape_key(14, 0): {                                                                            \
            using Sh = ShapeVar<14, 0>::type;                                                               \
            hipLaunchKernelGGL((KERN<Sh, false>), GRID, dim3(Sh::T), 0, (LC).stream, __VA_ARGS__);             \
        } break;                                                                                            \
        case shape_key(14, 1): {                                                                            \
            using Sh = ShapeVar<14, 1>::type;                                                               \
            hipLaunchKernelGGL((KERN<Sh, false>), GRID, dim3(Sh::T), 0, (LC).stream, __VA_ARGS__);             \
        } break;                                                                                            \
    }

void launch_ntt(const Launch& lc, bool inverse, const uint64_t* in, uint64_t* out, size_t rows, uint32_t nl,
                uint32_t pbase) {
    if (!rows) return;
    if (inverse) {
        CW_NTT_DISPATCH(lc, k_ntt_inv, dim3((unsigned)rows), lc.K, lc.tw, lc.twf, in, out, nl, pbase)
    } else {
        CW_NTT_DISPATCH(lc, k_ntt_fwd, dim3((unsigned)rows), lc.K, lc.tw, lc.twf, in, out, nl, pbase, 0u)
    }
}

void launch_ntt_operand(const Launch& lc, const uint64_t* in, uint64_t* out, size_t rows, uint32_t nl,
                        uint32_t pbase, uint32_t skip) {
    if (!rows) return;
    if (!lc.fp) {
        CW_NTT_DISPATCH(lc, k_ntt_fwd, dim3((unsigned)rows), lc.K, lc.tw, lc.twf, in, out, nl, pbase, skip)
        return;
    }
    with_shape(lc.logN, lc.shape, [&](auto tag) {
        using Sh = decltype(tag);
        if constexpr (Sh::LOGN <= 13)
            hipLaunchKernelGGL(k_ntt_fwd_operand<Sh>, dim3((unsigned)rows), dim3(Sh::T), 0, lc.stream, lc.K, lc.tw,
                               lc.twf, in, (double*)out, nl, pbase, skip);
    });
}

void launch_ntt_digits(const Launch& lc, const uint64_t* c3, uint64_t* out, uint32_t E) {
    if (!E) return;
    const size_t groups = (size_t)E * (lc.L + 2);
    CW_NTT_DISPATCH(lc, k_ntt_digits, dim3((unsigned)xcd_grid(groups, lc.L)), lc.K, lc.tw, lc.twf, c3, out, groups)
}

void launch_ntt_inv_tensor(const Launch& lc, const uint32_t* refs, const Batch& bt, uint64_t* X, size_t eq0,
                           size_t count) {
    if (!bt.E || !bt.nq) return;
    const size_t total = (size_t)bt.nq * bt.E;
    if (count == 0 || eq0 + count > total) count = total - eq0;
    const size_t groups = count * lc.LL;
    CW_NTT_DISPATCH(lc, k_ntt_inv_tensor, dim3((unsigned)xcd_grid(groups, 3)), lc.K, lc.tw, lc.twf, refs, bt, X,
                    groups, eq0)
}

void launch_ntt_payload(const Launch& lc, const uint16_t* pay, uint64_t* out, size_t rows_u16, uint32_t nl,
                        uint32_t dbase) {
    if (!rows_u16) return;
    if (!nl) nl = lc.L;
    const size_t rows = rows_u16 * nl;
    CW_NTT_DISPATCH(lc, k_ntt_payload, dim3((unsigned)rows), lc.K, lc.tw, lc.twf, pay, out, nl, dbase)
}

// ---------------------------------------------------------------------------------------------
// Exact centred extension Q -> Q u B of coefficient-form polynomials: in [G][L][N] -> out [G][LL][N]
// ---------------------------------------------------------------------------------------------
template <int NL>
__device__ __forceinline__ bool extend_coeff(const CtxConst* K, const uint64_t* x, size_t xs, uint64_t* o, size_t os,
                                             bool exact, bool write_q) {
    const uint32_t L = K->L, LB = K->LB;
    uint64_t y[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) {
            uint64_t xi = x[i * xs];
            y[i] = mul_shoup(xi, K->qinv[i], K->qinvq[i], K->p[i]);
            if (write_q) o[i * os] = xi;
        }
    bool amb = false;
    uint32_t v = exact ? conv_round_exact(K->qb, y) : conv_round_fast<NL>(K->qb, y, L, amb);
    for (uint32_t j = 0; j < LB; ++j) o[(L + j) * os] = conv_out<NL>(K->qb, y, L, v, j);
    return amb;
}

template <int NL>
__global__ void k_extend(const CtxConst* __restrict__ K, const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                         size_t G, uint64_t* fix, uint32_t* fixcnt, uint32_t write_q) {
    const uint32_t N = K->N, L = K->L, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= G * N) return;
    const size_t g = gid >> K->logN, c = gid & (N - 1);  // N is a power of two
    if (extend_coeff<NL>(K, in + g * L * N + c, N, out + g * LL * N + c, N, false, write_q != 0))
        fix[atomicAdd(fixcnt, 1u)] = gid;
}

template <int NL>
__global__ void k_extend_fix(const CtxConst* __restrict__ K, const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                             uint64_t* fix, uint32_t* fixcnt, uint32_t write_q) {
    const uint32_t N = K->N, L = K->L, LL = K->LL;
    const uint32_t n = *fixcnt;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) {
        const size_t gid = fix[f];
        const size_t g = gid >> K->logN, c = gid & (N - 1);
        extend_coeff<NL>(K, in + g * L * N + c, N, out + g * LL * N + c, N, true, write_q != 0);
    }
    __syncthreads();
    if (threadIdx.x == 0) *fixcnt = 0;
}

void launch_extend(const Launch& lc, const uint64_t* in, uint64_t* out, size_t G, bool write_q) {
    if (!G) return;
    const unsigned nb = blocks_for(G * lc.N);
    const uint32_t wq = write_q ? 1u : 0u;
#define CW_EXT(NL)                                                                                            \
    hipLaunchKernelGGL(k_extend<NL>, dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, in, out, G, lc.fix, lc.fixcnt, wq); \
    hipLaunchKernelGGL(k_extend_fix<NL>, dim3(1), dim3(256), 0, lc.stream, lc.K, in, out, lc.fix, lc.fixcnt, wq);
    if (lc.L <= 4) {
        CW_EXT(4)
    } else if (lc.L <= 8) {
        CW_EXT(8)
    } else {
        CW_EXT(12)
    }
#undef CW_EXT
}

// Rows j < L of out [G][LL][N] (transformed operands) from in [G][L][N] (transformed residues in
// [0, p)): the same values, as centred doubles on the fp64 path (what k_ntt_fwd_operand leaves).
__global__ void k_operand_q_rows(const CtxConst* __restrict__ K, const uint64_t* __restrict__ in,
                                 uint64_t* __restrict__ out, size_t G) {
    const uint32_t N = K->N, L = K->L, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= G * L * N) return;
    const size_t c = gid & (N - 1), gj = gid >> K->logN;  // N is a power of two
    const uint32_t j = (uint32_t)(gj % L);
    const size_t g = gj / L;
    const uint64_t x = in[gid];
    uint64_t o = x;
    if (K->fp) {
        const uint64_t p = K->p[j];
        const double d = x > (p - 1) / 2 ? (double)x - K->pd[j] : (double)x;
        o = (uint64_t)__double_as_longlong(d);
    }
    out[(g * LL + j) * N + c] = o;
}

void launch_operand_q_rows(const Launch& lc, const uint64_t* in, uint64_t* out, size_t G) {
    const size_t n = G * lc.L * lc.N;
    if (!n) return;
    hipLaunchKernelGGL(k_operand_q_rows, dim3(blocks_for(n)), dim3(EW_THREADS), 0, lc.stream, lc.K, in, out, G);
}

// ---------------------------------------------------------------------------------------------
// Exact scale-and-round of a coefficient-form tensor product X over Q u B:
//   r = [t X]_q (centred, exact Q -> B), y = (t X - r) / q in B, c = y (exact centred B -> Q).
// Output: coefficient form [E][3][L][N].  PRE: X as the fp64 tensor transform leaves it: row k holds
// [f_k X]_{p_k} with the first constants f (tqinv for Q, kb1 for B), as centred doubles.
// ---------------------------------------------------------------------------------------------
template <int NL, int NB, bool PRE>
__device__ __forceinline__ bool scale_coeff(const CtxConst* K, const uint64_t* x, size_t xs, uint64_t* cq, bool exact) {
    const uint32_t L = K->L, LB = K->LB;
    uint64_t y[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L)
            y[i] = PRE ? fp_to_residue(__longlong_as_double((long long)x[i * xs]), K->pd[i])
                       : mul_shoup(x[i * xs], K->tqinv[i], K->tqinvq[i], K->p[i]);
    bool amb = false;
    const uint32_t v = exact ? conv_round_exact(K->qb, y) : conv_round_fast<NL>(K->qb, y, L, amb);
    uint64_t z[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < (int)LB) {
            const uint64_t b = K->p[L + j];
            const uint64_t rb = conv_out<NL>(K->qb, y, L, v, j);
            const uint64_t xb = PRE ? fp_to_residue(__longlong_as_double((long long)x[(L + j) * xs]), K->pd[L + j])
                                    : mul_shoup(x[(L + j) * xs], K->kb1[j], K->kb1q[j], b);
            z[j] = sub_mod(xb, mul_shoup(rb, K->kb2[j], K->kb2q[j], b), b);
        }
    const uint32_t v2 = exact ? conv_round_exact(K->bq, z) : conv_round_fast<NB>(K->bq, z, LB, amb);
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) cq[i] = conv_out<NB>(K->bq, z, LB, v2, i);
    return amb;
}

// fp64 form (every prime below 2^50; X as the fp64 tensor transform leaves it, PRE above): the same
// conversions on doubles.  |y_i| <= q_i / 2 (plus 2^-52 of it), so |S| = |sum y_i / q_i| <= L/2 and
// |v| <= (L + 1)/2.  The rounding decisions v, v2 come from double sums whose error is below 2^-45;
// a sum within 2^-40 of a half is reported as ambiguous and the exact integer form redoes the
// coefficient.  The key constant kb2 is folded into the Q -> B products (fqbd, fqpd), so z_j is the
// input [kb1 x_j] (|.| <= b/2), L products (each below (1/2 + 3 |y_i| 2^-53) b <= 0.69 b in
// magnitude) and v fqpd, an exact product (|fqpd| < b/2): for L <= 5 the sum stays below 6 b < 2^53
// (b < 2^50) and is reduced once.  The outputs take -v2 [B]_{q_i}, exact as well
// (|v2| <= (LB + 1)/2, B mod q_i below q_i), and LB products below 0.69 q_i (|z_j| <= b/2 < 2^49):
// for LB <= 6 below 8 q_i.  The general form (EX = false) reduces the two exact products and every
// few sums.
#pragma clang fp contract(off)
template <int NL, int NB, bool EX>
__device__ __forceinline__ bool scale_coeff_fp(const CtxConst* K, const uint64_t* x, size_t xs, uint64_t* cq) {
    const uint32_t L = EX ? NL : K->L, LB = EX ? NB : K->LB;
    static_assert(!EX || (NL <= 5 && NB <= 6), "the single-reduction bounds");
    double y[NL];
    double S = 0.0;
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) {
            y[i] = __longlong_as_double((long long)x[i * xs]);
            S += y[i] * K->pinv[i];
        }
    const double v = __builtin_rint(S);
    bool amb = __builtin_fabs(S - v) > 0.5 - 0x1p-40;
    double z[NB];
    double S2 = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if (j < (int)LB) {
            const uint32_t jj = L + j;
            const double b = K->pd[jj], binv = K->pinv[jj];
            const double vf = v * K->fqpd[j];  // exact: |v| <= 7, |fqpd| < 2^49
            double acc = __longlong_as_double((long long)x[jj * xs]) + (EX ? vf : fred(vf, b, binv));
#pragma unroll
            for (int i = 0; i < NL; ++i)
                if (i < (int)L) {
                    acc += fmulmod(y[i], K->fqbd[i][j], b, binv);
                    if (!EX && (i % 5) == 4) acc = fred(acc, b, binv);
                }
            z[j] = fred(acc, b, binv);
            S2 += z[j] * binv;
        }
    const double v2 = __builtin_rint(S2);
    amb |= __builtin_fabs(S2 - v2) > 0.5 - 0x1p-40;
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) {
            const double p = K->pd[i], pinv = K->pinv[i];
            const double vp = v2 * K->bq.Pmd[i];  // exact: |v2| <= 7, B mod q_i < 2^50
            double c = EX ? -vp : -fred(vp, p, pinv);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (j < (int)LB) {
                    c += fmulmod(z[j], K->bq.Md[j][i], p, pinv);
                    if (!EX && (j % 6) == 5) c = fred(c, p, pinv);
                }
            cq[i] = fp_to_residue(fred(c, p, pinv), p);
        }
    return amb;
}
#pragma clang fp contract(on)

template <int NL>
__device__ __forceinline__ void scale_store(const CtxConst* K, const uint64_t* cq, uint64_t* out, size_t er, size_t c) {
    const uint32_t N = K->N, L = K->L;
    uint64_t* o = out + er * L * N + c;
#pragma unroll
    for (int i = 0; i < NL; ++i)
        if (i < (int)L) o[(size_t)i * N] = cq[i];
}

template <int NL, int NB, bool FP, bool EX = false>
__global__ void k_scale(const CtxConst* __restrict__ K, const uint64_t* __restrict__ X, uint64_t* __restrict__ out,
                        uint32_t E, uint64_t* fix, uint32_t* fixcnt) {
    const uint32_t N = K->N, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)E * 3 * N) return;
    const size_t c = gid & (N - 1), er = gid >> K->logN;  // N is a power of two
    uint64_t cq[NL];
    bool amb;
    if constexpr (FP) amb = scale_coeff_fp<NL, NB, EX>(K, X + er * LL * N + c, N, cq);
    else amb = scale_coeff<NL, NB, false>(K, X + er * LL * N + c, N, cq, false);
    if (amb) fix[atomicAdd(fixcnt, 1u)] = gid;
    scale_store<NL>(K, cq, out, er, c);
}

// PRE: X as the fp64 tensor transform leaves it (rows multiplied by their first constants, centred doubles).
template <int NL, int NB, bool PRE>
__global__ void k_scale_fix(const CtxConst* __restrict__ K, const uint64_t* __restrict__ X, uint64_t* __restrict__ out,
                            uint64_t* fix, uint32_t* fixcnt) {
    const uint32_t N = K->N, LL = K->LL;
    const uint32_t n = *fixcnt;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) {
        const size_t gid = fix[f];
        const size_t c = gid & (N - 1), er = gid >> K->logN;
        uint64_t cq[NL];
        scale_coeff<NL, NB, PRE>(K, X + er * LL * N + c, N, cq, true);
        scale_store<NL>(K, cq, out, er, c);
    }
    __syncthreads();
    if (threadIdx.x == 0) *fixcnt = 0;
}

void launch_scale(const Launch& lc, const uint64_t* X, uint64_t* out, uint32_t E) {
    if (!E) return;
    const unsigned nb = blocks_for((size_t)E * 3 * lc.N);
#define CW_SCALE(NLV, NBV)                                                                                    \
    if (lc.fp)                                                                                                \
        hipLaunchKernelGGL((k_scale<NLV, NBV, true>), dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, X, out, E, \
                           lc.fix, lc.fixcnt);                                                                \
    else                                                                                                      \
        hipLaunchKernelGGL((k_scale<NLV, NBV, false>), dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, X, out, E, \
                           lc.fix, lc.fixcnt);                                                                \
    if (lc.fp)                                                                                                \
        hipLaunchKernelGGL((k_scale_fix<NLV, NBV, true>), dim3(1), dim3(256), 0, lc.stream, lc.K, X, out, lc.fix, \
                           lc.fixcnt);                                                                        \
    else                                                                                                      \
        hipLaunchKernelGGL((k_scale_fix<NLV, NBV, false>), dim3(1), dim3(256), 0, lc.stream, lc.K, X, out, lc.fix, \
                           lc.fixcnt);
    if (lc.fp && lc.L == 5 && lc.LB == 5) {  // the N = 8192 parameter sets
        hipLaunchKernelGGL((k_scale<5, 5, true, true>), dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, X, out, E,
                           lc.fix, lc.fixcnt);
        hipLaunchKernelGGL((k_scale_fix<8, 9, true>), dim3(1), dim3(256), 0, lc.stream, lc.K, X, out, lc.fix, lc.fixcnt);
    } else if (lc.fp && lc.L == 3 && lc.LB == 3) {  // N = 4096, three 36-bit primes
        hipLaunchKernelGGL((k_scale<3, 3, true, true>), dim3(nb), dim3(EW_THREADS), 0, lc.stream, lc.K, X, out, E,
                           lc.fix, lc.fixcnt);
        hipLaunchKernelGGL((k_scale_fix<4, 5, true>), dim3(1), dim3(256), 0, lc.stream, lc.K, X, out, lc.fix, lc.fixcnt);
    } else if (lc.L <= 4 && lc.LB <= 5) {
        CW_SCALE(4, 5)
    } else if (lc.L <= 8 && lc.LB <= 9) {
        CW_SCALE(8, 9)
    } else {
        CW_SCALE(12, 13)
    }
#undef CW_SCALE
}

// ---------------------------------------------------------------------------------------------
// Key switching: sel = (c0 + sum_i D_i b_i, c1 + sum_i D_i a_i), transformed over Q.
// rlk: [L][2][L][N] transformed values followed by [L][2][L][N] Shoup companions.
// ---------------------------------------------------------------------------------------------
// Workgroup b covers EW_THREADS coefficients of limb j of element-query eq, with eq varying fastest:
// the workgroups running together (and those of one XCD, b mod 8) read the same slice of the key
// limb (2L values and their companions per coefficient, 32 MB for the whole key at N = 16384),
// which then comes from L2, and stream different staged digit rows.
__global__ void k_relin_mac(const CtxConst* __restrict__ K, const uint64_t* __restrict__ R, const Batch bt) {
    const uint32_t N = K->N, L = K->L;
    const size_t EQ = (size_t)bt.nq * bt.E, b = blockIdx.x;
    const size_t eq = b % EQ, rest = b / EQ;
    const uint32_t j = (uint32_t)(rest % L);
    const size_t c = (rest / L) * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const uint32_t q = (uint32_t)(eq / bt.E);
    const size_t e = eq % bt.E;
    const uint64_t* __restrict__ rlk = bt.rlk[q];
    const uint64_t p = K->p[j];
    const size_t LN = (size_t)L * N;
    const uint64_t* r = R + eq * (L + 2) * LN + (size_t)j * N + c;
    const size_t half = (size_t)L * 2 * LN;
    uint64_t s0 = r[(size_t)L * LN], s1 = r[(size_t)(L + 1) * LN];
    for (uint32_t i = 0; i < L; ++i) {
        const uint64_t d = r[(size_t)i * LN];
        const size_t ob = ((size_t)i * 2 + 0) * LN + (size_t)j * N + c;
        const size_t oa = ((size_t)i * 2 + 1) * LN + (size_t)j * N + c;
        s0 = add_mod(s0, mul_shoup(d, rlk[ob], rlk[half + ob], p), p);
        s1 = add_mod(s1, mul_shoup(d, rlk[oa], rlk[half + oa], p), p);
    }
    uint64_t* o = bt.sel[q] + e * 2 * LN + (size_t)j * N + c;
    o[0] = s0;
    o[LN] = s1;
}

void launch_relin_mac(const Launch& lc, const uint64_t* R, const Batch& bt) {
    if (!bt.E || !bt.nq) return;
    const size_t blocks = (size_t)bt.nq * bt.E * lc.L * ((lc.N + EW_THREADS - 1) / EW_THREADS);
    hipLaunchKernelGGL(k_relin_mac, dim3((unsigned)blocks), dim3(EW_THREADS), 0, lc.stream, lc.K, R, bt);
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
__global__ void k_gather_leaf(const CtxConst* __restrict__ K, const uint32_t* __restrict__ refs, const Batch bt) {
    const uint32_t N = K->N, L = K->L, LL = K->LL;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)bt.E * 2 * L * N;
    if (gid >= (size_t)bt.nq * per) return;
    const uint32_t q = (uint32_t)(gid / per);
    const size_t gq = gid % per;
    const size_t c = gq & (N - 1), rest = gq >> K->logN;  // N is a power of two
    const uint32_t j = (uint32_t)(rest % L);
    const size_t ep = rest / L;
    const uint32_t poly = (uint32_t)(ep % 2);
    const size_t e = ep / 2;
    const uint32_t leaf = refs[2 * e];
    const size_t src = ((size_t)leaf * 2 * LL + (size_t)poly * LL + j) * N + c;
    bt.sel[q][gq] = K->fp ? fp_to_residue(((const double*)bt.leaves[q])[src], K->pd[j]) : bt.leaves[q][src];
}

void launch_gather_leaf(const Launch& lc, const uint32_t* refs, const Batch& bt) {
    if (!bt.E || !bt.nq) return;
    hipLaunchKernelGGL(k_gather_leaf, dim3(blocks_for((size_t)bt.nq * bt.E * 2 * lc.L * lc.N)), dim3(EW_THREADS), 0,
                       lc.stream, lc.K, refs, bt);
}

// ---------------------------------------------------------------------------------------------
// Inner product with the database (Eq. (1)): acc_b[r] += sum_e sel_b[e] * P[e][r], transformed
// over Q.  Grid y indexes groups of the B queries that scan the same payload chunk.
// ---------------------------------------------------------------------------------------------
// acc_q[r][poly] += sum_e sel_q[e][poly] * Ph[e][r] (mod q_j) for a group of up to QG queries.
// A workgroup is ACC_SLICES wavefronts over the same 64 coefficients: wavefront w takes the w-th
// contiguous slice of the E elements, and the slices are summed through LDS at the end, so that
// enough waves are in flight to cover HBM latency (the loop is a stream of loads with a Barrett
// product each).  Each thread keeps both polynomials of its coefficient for every query of the
// group, so a transformed payload row is read once per group rather than once per query and
// polynomial.  Modular sums do not depend on the order of their terms.
constexpr int ACC_SLICES = 8;
template <int QG>
__global__ __launch_bounds__(64 * ACC_SLICES) void k_accumulate(const CtxConst* __restrict__ K,
                                                                const QueryPtrs qp, const uint64_t* __restrict__ Ph,
                                                                uint32_t nq, uint32_t E, uint32_t s) {
    __shared__ uint64_t red[ACC_SLICES - 1][2 * QG][64];
    const uint32_t N = K->N, L = K->L;
    const size_t LN = (size_t)L * N;
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const size_t gid = (size_t)blockIdx.x * 64 + lane;  // (r, j, c) over s L N
    const bool valid = gid < (size_t)s * LN;
    const size_t cj = gid % LN;
    const uint32_t r = (uint32_t)(gid / LN);
    const uint32_t j = (uint32_t)(cj / N);
    const uint64_t p = K->p[j], mu = K->bar_mu[j];
    const uint32_t sb = K->bar_s[j];
    const uint32_t q0 = blockIdx.y * QG;
    const uint32_t nqg = nq - q0 < (uint32_t)QG ? nq - q0 : (uint32_t)QG;
    uint64_t s0[QG], s1[QG];
#pragma unroll
    for (int q = 0; q < QG; ++q) s0[q] = s1[q] = 0;
    const uint32_t e_lo = (uint32_t)((uint64_t)E * w / ACC_SLICES);
    const uint32_t e_hi = (uint32_t)((uint64_t)E * (w + 1) / ACC_SLICES);
    if (valid) {
#pragma unroll 2
        for (uint32_t e = e_lo; e < e_hi; ++e) {
            const uint64_t b = Ph[((size_t)e * s + r) * LN + cj];
            const size_t o = (size_t)e * 2 * LN + cj;
#pragma unroll
            for (int q = 0; q < QG; ++q) {
                if ((uint32_t)q < nqg) {
                    const uint64_t* sel = qp.sel[q0 + q];
                    s0[q] = add_mod(s0[q], mul_barrett(sel[o], b, p, mu, sb), p);
                    s1[q] = add_mod(s1[q], mul_barrett(sel[o + LN], b, p, mu, sb), p);
                }
            }
        }
    }
    if (w > 0) {
#pragma unroll
        for (int q = 0; q < QG; ++q) {
            red[w - 1][2 * q][lane] = s0[q];
            red[w - 1][2 * q + 1][lane] = s1[q];
        }
    }
    __syncthreads();
    if (w == 0 && valid) {
#pragma unroll
        for (int q = 0; q < QG; ++q) {
            if ((uint32_t)q < nqg) {
                uint64_t a0 = s0[q], a1 = s1[q];
#pragma unroll
                for (int v = 0; v < ACC_SLICES - 1; ++v) {
                    a0 = add_mod(a0, red[v][2 * q][lane], p);
                    a1 = add_mod(a1, red[v][2 * q + 1][lane], p);
                }
                uint64_t* acc = qp.acc[q0 + q] + (size_t)r * 2 * LN + cj;
                acc[0] = add_mod(acc[0], a0, p);
                acc[LN] = add_mod(acc[LN], a1, p);
            }
        }
    }
}

void launch_accumulate(const Launch& lc, const QueryPtrs& qp, const uint64_t* Ph, uint32_t nq, uint32_t E,
                       uint32_t s) {
    if (!E || !nq) return;
    const unsigned bx = (unsigned)(((size_t)s * lc.L * lc.N + 63) / 64);
#define CW_ACC(QG)                                                                                          \
    hipLaunchKernelGGL(k_accumulate<QG>, dim3(bx, (nq + QG - 1) / QG), dim3(64 * ACC_SLICES), 0, lc.stream, \
                       lc.K, qp, Ph, nq, E, s)
    if (nq == 1) CW_ACC(1);
    else if (nq == 2) CW_ACC(2);
    else CW_ACC(4);
#undef CW_ACC
}

// ---------------------------------------------------------------------------------------------
// Query expansion (Algorithm 5).  One thread per coefficient of one polynomial limb of one item.
// The automorphism is written as a gather: output coefficient o of sigma_g(a) is a_i for
// i = o g^-1 mod 2N when that is below N, else -a_(i - N) (x^N = -1).  The monomial x^(-e) moves
// coefficient i to i - e, negated when it wraps (x^(-e) = -x^(N - e)).
// ---------------------------------------------------------------------------------------------
__global__ void k_expand_stage(const CtxConst* __restrict__ K, const uint64_t* __restrict__ cts, uint32_t c,
                               uint32_t a, size_t E, uint32_t ginv, uint64_t* __restrict__ staging) {
    const uint32_t N = K->N, L = K->L;
    const size_t LN = (size_t)L * N;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= E * 2 * LN) return;
    const uint32_t o = (uint32_t)(gid % N);
    const uint32_t l = (uint32_t)((gid / N) % L);
    const uint32_t poly = (uint32_t)((gid / LN) % 2);
    const size_t e = gid / (2 * LN);
    const size_t j = e >> a, b = e & ((1u << a) - 1u);
    const uint64_t* src = cts + (((j << c) + b) * 2 + poly) * LN + (size_t)l * N;
    const uint64_t p = K->p[l];
    const uint32_t i = (uint32_t)((uint64_t)o * ginv % (2ull * N));
    const uint64_t v = i < N ? src[i] : (src[i - N] ? p - src[i - N] : 0);
    uint64_t* dst = staging + e * 3 * LN + (size_t)l * N + o;
    if (poly == 0) {
        dst[0] = v;
        dst[LN] = 0;
    } else {
        dst[2 * LN] = v;
    }
}

__global__ void k_expand_combine(const CtxConst* __restrict__ K, const uint64_t* __restrict__ src,
                                 const uint64_t* __restrict__ sub, uint32_t c, uint32_t a, size_t E,
                                 uint64_t* __restrict__ dst) {
    const uint32_t N = K->N, L = K->L;
    const size_t LN = (size_t)L * N;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= E * 2 * LN) return;
    const uint32_t o = (uint32_t)(gid % N);
    const size_t row = gid / N;  // (e, poly, l)
    const uint32_t l = (uint32_t)(row % L);
    const size_t e = gid / (2 * LN);
    const size_t pl = row % (2 * (size_t)L);  // poly * L + l
    const size_t j = e >> a, b = e & ((1u << a) - 1u);
    const uint64_t p = K->p[l];
    const uint64_t* x = src + (((j << c) + b) * 2) * LN + pl * N;
    const uint64_t* y = sub + row * N;
    dst[(((j << c) + b) * 2) * LN + pl * N + o] = add_mod(x[o], y[o], p);
    const uint32_t sh = 1u << a;
    const uint32_t i = o + sh;
    const uint64_t d = i < N ? sub_mod(x[i], y[i], p) : sub_mod(y[i - N], x[i - N], p);
    dst[(((j << c) + b + sh) * 2) * LN + pl * N + o] = d;
}

void launch_expand_stage(const Launch& lc, const uint64_t* cts, uint32_t c, uint32_t a, uint32_t h, uint32_t ginv,
                         uint64_t* staging) {
    const size_t E = (size_t)h << a;
    if (!E) return;
    hipLaunchKernelGGL(k_expand_stage, dim3(blocks_for(E * 2 * lc.L * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K,
                       cts, c, a, E, ginv, staging);
}

void launch_expand_combine(const Launch& lc, const uint64_t* src, const uint64_t* sub, uint32_t c, uint32_t a,
                           uint32_t h, uint64_t* dst) {
    const size_t E = (size_t)h << a;
    if (!E) return;
    hipLaunchKernelGGL(k_expand_combine, dim3(blocks_for(E * 2 * lc.L * lc.N)), dim3(EW_THREADS), 0, lc.stream,
                       lc.K, src, sub, c, a, E, dst);
}

// ---------------------------------------------------------------------------------------------
// Modulus switching (response compression): one thread per coefficient.  [x]_r centred comes from
// the dropped limbs by the exact conversion (fast rounding decision, exact fallback in the fixup
// kernel), then x' = (x_j - [x]_r) r^{-1} mod q_j for every kept limb.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ bool switch_coeff(const CtxConst* K, const SwitchConst* S, const uint64_t* x,
                                             uint64_t* y, bool exact, uint64_t* out, size_t os) {
    const uint32_t N = K->N, keep = S->keep, nd = S->L - keep;
    for (uint32_t i = 0; i < nd; ++i) {
        const uint64_t p = K->p[keep + i];
        y[i] = mul_shoup(x[(size_t)(keep + i) * N], S->yc[i], S->ycq[i], p);
    }
    bool amb = false;
    const uint32_t v = exact ? conv_round_exact(S->T, y) : conv_round_fast<MAX_L>(S->T, y, nd, amb);
    for (uint32_t j = 0; j < keep; ++j) {
        const uint64_t p = K->p[j];
        const uint64_t xr = conv_out<MAX_L>(S->T, y, nd, v, j);  // [x]_r mod q_j
        out[(size_t)j * os] = mul_shoup(sub_mod(x[(size_t)j * N], xr, p), S->rinv[j], S->rinvq[j], p);
    }
    return amb;
}

__global__ void k_mod_switch(const CtxConst* __restrict__ K, const SwitchConst* __restrict__ S,
                             const uint64_t* __restrict__ in, size_t polys, uint64_t* __restrict__ out,
                             uint64_t* fix, uint32_t* fixcnt) {
    const uint32_t N = K->N, L = K->L, keep = S->keep;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= polys * N) return;
    const size_t poly = gid / N, c = gid % N;
    uint64_t y[MAX_L];
    if (switch_coeff(K, S, in + poly * L * N + c, y, false, out + poly * keep * N + c, N))
        fix[atomicAdd(fixcnt, 1u)] = gid;
}

__global__ void k_mod_switch_fix(const CtxConst* __restrict__ K, const SwitchConst* __restrict__ S,
                                 const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t* fix,
                                 uint32_t* fixcnt) {
    const uint32_t N = K->N, L = K->L, keep = S->keep;
    const uint32_t n = *fixcnt;
    for (uint32_t f = threadIdx.x; f < n; f += blockDim.x) {
        const size_t gid = fix[f];
        const size_t poly = gid / N, c = gid % N;
        uint64_t y[MAX_L];
        switch_coeff(K, S, in + poly * L * N + c, y, true, out + poly * keep * N + c, N);
    }
    __syncthreads();
    if (threadIdx.x == 0) *fixcnt = 0;
}

__global__ void k_copy_limbs(const uint64_t* __restrict__ in, size_t polys, uint32_t L, uint32_t keep, uint32_t N,
                             uint64_t* __restrict__ out) {
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= polys * keep * N) return;
    const size_t poly = gid / ((size_t)keep * N), r = gid % ((size_t)keep * N);
    out[gid] = in[poly * L * N + r];
}

void launch_mod_switch(const Launch& lc, const SwitchConst* S, uint32_t keep, const uint64_t* in, size_t polys,
                       uint64_t* out) {
    if (!polys) return;
    if (keep == lc.L) {  // nothing dropped: the identity
        hipLaunchKernelGGL(k_copy_limbs, dim3(blocks_for(polys * keep * lc.N)), dim3(EW_THREADS), 0, lc.stream, in,
                           polys, lc.L, keep, lc.N, out);
        return;
    }
    hipLaunchKernelGGL(k_mod_switch, dim3(blocks_for(polys * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K, S, in, polys,
                       out, lc.fix, lc.fixcnt);
    hipLaunchKernelGGL(k_mod_switch_fix, dim3(1), dim3(256), 0, lc.stream, lc.K, S, in, out, lc.fix, lc.fixcnt);
}

// ---------------------------------------------------------------------------------------------
// Arithmetic equality helpers (element-wise, one thread per coefficient).
// ---------------------------------------------------------------------------------------------
__global__ void k_pair_refs(uint32_t* refs, uint32_t n, uint32_t a0, uint32_t b0) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    refs[2 * i] = a0 + i;
    refs[2 * i + 1] = b0 + i;
}

__global__ void k_sum_rows(const CtxConst* __restrict__ K, const uint64_t* __restrict__ C, uint32_t cnt,
                           uint32_t rows, bool first, uint64_t* __restrict__ S) {
    const uint32_t N = K->N, L = K->L;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)rows * N;
    if (gid >= per) return;
    const uint64_t p = K->p[(gid / N) % L];
    uint64_t acc = first ? 0 : S[gid];
    for (uint32_t e = 0; e < cnt; ++e) acc = add_mod(acc, C[(size_t)e * per + gid], p);
    S[gid] = acc;
}

__global__ void k_sub_consts(const CtxConst* __restrict__ K, const uint64_t* __restrict__ ct, uint32_t k,
                             uint64_t* __restrict__ F) {
    const uint32_t N = K->N, L = K->L;
    const size_t c2 = (size_t)2 * L * N;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)k * c2) return;
    const uint32_t i = (uint32_t)(gid / c2);
    const size_t w = gid % c2;  // (poly * L + j) * N + c
    const uint32_t c = (uint32_t)(w % N), j = (uint32_t)((w / N) % L);
    const uint64_t p = K->p[j];
    uint64_t v = ct[w];
    if (w < (size_t)L * N && c == 0) v = sub_mod(v, mul_barrett(K->delta[j], i, p, K->bar_mu[j], K->bar_s[j]), p);
    F[gid] = v;
}

__global__ void k_scalar_mul(const CtxConst* __restrict__ K, const uint64_t* __restrict__ ct, size_t total,
                             uint64_t c, uint64_t* __restrict__ out) {
    const uint32_t N = K->N, L = K->L;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const uint32_t j = (uint32_t)((gid / N) % L);
    out[gid] = mul_barrett(ct[gid], c, K->p[j], K->bar_mu[j], K->bar_s[j]);
}

void launch_pair_refs(hipStream_t st, uint32_t* refs, uint32_t n, uint32_t a0, uint32_t b0) {
    if (!n) return;
    hipLaunchKernelGGL(k_pair_refs, dim3(blocks_for(n)), dim3(EW_THREADS), 0, st, refs, n, a0, b0);
}
void launch_sum_rows(const Launch& lc, const uint64_t* C, uint32_t cnt, uint32_t rows, bool first, uint64_t* S) {
    hipLaunchKernelGGL(k_sum_rows, dim3(blocks_for((size_t)rows * lc.N)), dim3(EW_THREADS), 0, lc.stream, lc.K, C,
                       cnt, rows, first, S);
}
void launch_sub_consts(const Launch& lc, const uint64_t* ct, uint32_t k, uint64_t* F) {
    if (!k) return;
    hipLaunchKernelGGL(k_sub_consts, dim3(blocks_for((size_t)k * 2 * lc.L * lc.N)), dim3(EW_THREADS), 0, lc.stream,
                       lc.K, ct, k, F);
}
void launch_scalar_mul(const Launch& lc, const uint64_t* ct, uint32_t count, uint64_t c, uint64_t* out) {
    const size_t total = (size_t)count * lc.L * lc.N;
    if (!total) return;
    hipLaunchKernelGGL(k_scalar_mul, dim3(blocks_for(total)), dim3(EW_THREADS), 0, lc.stream, lc.K, ct, total, c,
                       out);
}

// Folklore leaves: leaf 2i = 1 - x_i = (Delta - c0, -c1) (Delta in coefficient 0 only), leaf 2i + 1 = x_i.
__global__ void k_folklore_leaves(const CtxConst* __restrict__ K, const uint64_t* __restrict__ query, uint32_t ell,
                                  uint64_t* __restrict__ out) {
    const uint32_t N = K->N, L = K->L;
    const size_t ct = (size_t)2 * L * N;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (size_t)ell * ct) return;
    const size_t i = gid / ct, w = gid % ct;  // w = (poly * L + j) * N + c
    const uint32_t c = (uint32_t)(w % N), j = (uint32_t)((w / N) % L), poly = (uint32_t)(w / ((size_t)L * N));
    const uint64_t p = K->p[j], x = query[gid];
    const uint64_t d = (poly == 0 && c == 0) ? K->delta[j] : 0;
    out[(2 * i) * ct + w] = sub_mod(d, x, p);
    out[(2 * i + 1) * ct + w] = x;
}

void launch_folklore_leaves(const Launch& lc, const uint64_t* query, uint32_t ell, uint64_t* out) {
    if (!ell) return;
    hipLaunchKernelGGL(k_folklore_leaves, dim3(blocks_for((size_t)ell * 2 * lc.L * lc.N)), dim3(EW_THREADS), 0,
                       lc.stream, lc.K, query, ell, out);
}

// dst row e = src row order[e], rows of `row` uint16 (a multiple of 8), copied in 16-byte words.
__global__ void k_gather_rows(const uint16_t* __restrict__ src, const uint64_t* __restrict__ order, uint64_t n,
                              size_t row, uint16_t* __restrict__ dst) {
    const size_t words = row / 8;  // 16-byte words per row
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n * words) return;
    const size_t e = gid / words, w = gid % words;
    ((uint4*)dst)[e * words + w] = ((const uint4*)src)[order[e] * words + w];
}

void launch_gather_rows(hipStream_t st, const uint16_t* src, const uint64_t* order, uint64_t n, size_t row,
                        uint16_t* dst) {
    if (!n) return;
    hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(n * (row / 8))), dim3(EW_THREADS), 0, st, src, order, n, row,
                       dst);
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

// Range check of `polys` polynomials [polys][L][N] (residue c of limb j must be below q_j): any
// residue out of range sets *flag to 1 (grid-stride loop, one residue per thread and step).
__global__ void k_check_residues(const CtxConst* __restrict__ K, const uint64_t* __restrict__ x, size_t polys,
                                 uint32_t* __restrict__ flag) {
    const uint32_t N = K->N, L = K->L;
    const size_t words = polys * L * N;
    bool bad = false;
    for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (size_t)gridDim.x * blockDim.x)
        bad = bad || x[w] >= K->p[(w / N) % L];
    if (bad) atomicOr(flag, 1u);
}

void launch_check_residues(const Launch& lc, const uint64_t* x, size_t polys, uint32_t* flag) {
    if (!polys) return;
    const size_t words = polys * lc.L * lc.N;
    const size_t blocks = std::min<size_t>(blocks_for(words), (size_t)lc.cus * 16);
    hipLaunchKernelGGL(k_check_residues, dim3(std::max<size_t>(1, blocks)), dim3(EW_THREADS), 0, lc.stream, lc.K, x,
                       polys, flag);
}

// ---------------------------------------------------------------------------------------------
// Codeword tables
// ---------------------------------------------------------------------------------------------
// Algorithm 3 (perfect mapping), computed as the inverse of the colex rank that Algorithm 7 defines,
// x = sum_h C(p_h, h) over the ascending positions p_1 < ... < p_k: for h = k, ..., 1 the position
// p_h is the largest p below p_{h+1} (below m for h = k) with C(p, h) <= r, the remaining rank, and
// r then drops by C(p_h, h).  Each p_h is a binary search over the saturating table C(a, h), a < m
// (k searches of log2 m steps instead of a scan over m).  A rank outside the code leaves r > 0 and
// marks the whole codeword 0xFFFFFFFF (rejected by the caller).
__global__ void k_map_perfect(const uint64_t* __restrict__ ids, size_t n, uint32_t m, uint32_t k,
                              const uint64_t* __restrict__ binom, uint32_t* __restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    uint64_t r = ids[e];
    uint32_t* o = out + e * k;
    int hi = (int)m - 1;
    bool ok = true;
    for (uint32_t h = k; h >= 1 && ok; --h) {
        int lo = (int)h - 1;  // C(h - 1, h) = 0 <= r: the smallest candidate always qualifies
        ok = lo <= hi;
        while (ok && lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (binom[(size_t)mid * (k + 1) + h] <= r)
                lo = mid;
            else
                hi = mid - 1;
        }
        if (!ok) break;
        o[h - 1] = (uint32_t)lo;  // the h-th one from the top is the h-th smallest position
        r -= binom[(size_t)lo * (k + 1) + h];
        hi = lo - 1;
    }
    if (!ok || r != 0)
        for (uint32_t h = 0; h < k; ++h) o[h] = 0xFFFFFFFFu;
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
