// Launch wrappers of the gfx950 kernels (kernels.hip).  Every wrapper enqueues on lc.stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "consts.h"

namespace cw {

constexpr int MAX_BATCH = 32;  // queries per accumulate launch

struct QueryPtrs {  // passed by value as a kernel argument
    const uint64_t* sel[MAX_BATCH];
    uint64_t* acc[MAX_BATCH];
};

// Up to MAX_QB queries whose selectors are computed in one launch per stage.  They process the
// same E elements (the operand references are shared); element e of query q is row q*E + e of the
// launch's work buffers.  Passed by value as a kernel argument.
constexpr int MAX_QB = 8;
// Operand format of transformed extended operands and keys: with the fp64 transforms (Launch::fp)
// the 8-byte words hold integer-valued doubles in [-p/2, p/2]; otherwise u64 residues in [0, p)
// (keys followed by their Shoup companions).
struct Batch {
    uint32_t nq, E;
    const uint64_t* leaves[MAX_QB];  // resident query [m][2][LL][N], operand format
    const uint64_t* nodes[MAX_QB];   // memoised tree nodes [pairs][2][LL][N] (or null), operand format
    const uint64_t* rlk[MAX_QB];     // transformed key [L][2][L][N], operand format
    uint64_t* sel[MAX_QB];           // selectors out [E][2][L][N], u64 residues
};

struct Launch {
    hipStream_t stream;
    const CtxConst* K;    // device copy of the constants
    const uint64_t* tw;   // device twiddles [LL][4][N]
    const double* twf;    // the same as doubles (fp64 transform), or null
    bool fp;              // transforms run on the fp64 pipe (every prime below 2^50, N <= 8192)
    bool q_lazy;          // fp, every ciphertext prime below 2^48 and (2.4 L + 16) max q_i < 2^53: the
                          // key switch's transforms modulo q_j need no reduction between passes or
                          // of their outputs
    uint32_t N, logN, L, LB, LL;
    uint32_t cus;         // compute units of the device
    uint32_t relin_group; // key-switch workgroup order: 0 = the L limbs of an element side by side on
                          // one XCD; G > 0 = blocks of G elements, limb-major inside a block
    uint32_t shape;       // transform shape variant of this degree (< ntt_shape_count(logN))
    uint64_t* fix;        // fixup list for ambiguous conversions (capacity >= coefficients per launch)
    uint32_t* fixcnt;     // its counter; zero between launches
};

// Root products with the key switch deferred past the inner product (see kernels.hip).  A unit is
// the work of one workgroup per element: one or two rows of the coefficient-form root products
// C [nq E][3][L][N] (row src = poly * L + limb), transformed modulo context prime `prime`, each
// multiplied by payload rows r0 .. r0 + nr - 1 of the element and summed into accumulator row
// `row` of the query's [s][RR][N] accumulators (rows 0 .. 2L-1: c0 and c1 limbs modulo q_j;
// row 2L + i A + a: digit i modulo the deferred switch's prime a, context prime LL + a).
constexpr int ROOT_MAX_UNITS = 112;
struct RootUnit {
    uint16_t src0, src1, row0, row1;
    uint8_t prime, prow, r0, nr, two;  // prow: the prime's row among an element's payload rows
};
struct RootPlan {  // passed by value
    uint32_t nq, E, slice, nslices, s, LP, RR, U, A, lazy;
    RootUnit u[ROOT_MAX_UNITS];
};
hipError_t kernels_init();
// Transform shape variants of degree 2^logN (all leave the same transformed layout), and the stage
// counts of variant v's passes in order (returns the number of passes; stages holds up to 8).
uint32_t ntt_shape_count(uint32_t logN);
uint32_t ntt_shape_stages(uint32_t logN, uint32_t v, uint32_t* stages);
void launch_ntt(const Launch& lc, bool inverse, const uint64_t* in, uint64_t* out, size_t rows, uint32_t nl,
                uint32_t pbase);
// Forward transform of coefficient-form rows (u64 in [0, p)) into the operand format (in place
// allowed).  skip > 0: the rows form blocks of nl of which the first `skip` are left as they are;
// rows counts the transformed ones (blocks * (nl - skip)).
void launch_ntt_operand(const Launch& lc, const uint64_t* in, uint64_t* out, size_t rows, uint32_t nl,
                        uint32_t pbase, uint32_t skip = 0);
// Lift and transform uint16 rows: out [rows_u16][nl][N], row j modulo context prime j for j < L and
// prime dbase + j - L above (nl = 0: L).
void launch_ntt_payload(const Launch& lc, const uint16_t* pay, uint64_t* out, size_t rows_u16, uint32_t nl = 0,
                        uint32_t dbase = 0);
// Transformed relinearization staging [E][L+2][L][N] straight from a coefficient-form [E][3][L][N].
void launch_ntt_digits(const Launch& lc, const uint64_t* c3, uint64_t* out, uint32_t E);
// Exact centred extension of coefficient-form [G][L][N] to [G][LL][N] (Q rows copied unless
// write_q is false, then only the B rows are written).
void launch_extend(const Launch& lc, const uint64_t* in, uint64_t* out, size_t G, bool write_q = true);
// Rows j < L of out [G][LL][N] in the operand format from transformed residues in [G][L][N].
void launch_operand_q_rows(const Launch& lc, const uint64_t* in, uint64_t* out, size_t G);
// Tensor product (a0 b0, a0 b1 + a1 b0, a1 b1) of E operand pairs over Q u B, formed while loading
// and inverse-transformed: X [E][3][LL][N] in coefficient form.
// Only rows eq0 .. eq0 + count - 1 of the batch (row eq = q E + e; count = 0: to the end), stored from
// X on (X [count][3][LL][N]).
void launch_ntt_inv_tensor(const Launch& lc, const uint32_t* refs, const Batch& bt, uint64_t* X, size_t eq0 = 0,
                           size_t count = 0);
void launch_scale(const Launch& lc, const uint64_t* X, uint64_t* out, uint32_t E);
void launch_relin_mac(const Launch& lc, const uint64_t* R, const Batch& bt);
// Key switching of E coefficient-form products [E][3][L][N] into transformed selectors [E][2][L][N]
// (digit reduction, digit transforms and the multiply-accumulate with the key in one kernel).
void launch_relin(const Launch& lc, const uint64_t* c3, const Batch& bt, uint64_t* staging);
// Whether launch_relin needs its staging buffer [E][L+2][L][N] at this ring degree.
bool relin_needs_staging(uint32_t logN);
// Deferred root key switch (fp64 or integer transforms): part [nslices][nq][s][RR][N] receives each
// slice's sums of transformed rows times payload rows Ph [E][s][LP][N] (residues).
void launch_root_pm(const Launch& lc, const uint64_t* C, const uint64_t* Ph, const RootPlan& plan, uint64_t* part);
// racc_q [s][RR][N] += sum over slices of part[.][q] (mod each row's prime), q < nq.
void launch_root_reduce(const Launch& lc, const uint64_t* part, const RootPlan& plan, const QueryPtrs& qp);
// Wc [s][L][2][N] (coefficient form, digit i modulo d0 and d1) -> WQ [s][L][L][N]: the centred
// integer digit sum modulo every q_j.
void launch_root_crt(const Launch& lc, const CrtConst& cc, const uint64_t* Wc, uint32_t s, uint64_t* WQ);
// answer [s][2][L][N] (transformed) = racc c rows + sum_i WQ^[r][i][j] key[i][poly][j] mod q_j, WQ^
// transformed; key in the path's operand format.
void launch_root_combine(const Launch& lc, const uint64_t* racc, const uint64_t* WQ, const uint64_t* rlk, uint32_t s,
                         uint32_t RR, uint64_t* answer);
void launch_shoup_companions(const Launch& lc, const uint64_t* v, uint64_t* comp, size_t rows, uint32_t nl);
void launch_gather_leaf(const Launch& lc, const uint32_t* refs, const Batch& bt);
void launch_accumulate(const Launch& lc, const QueryPtrs& qp, const uint64_t* Ph, uint32_t nq, uint32_t E,
                       uint32_t s);
void launch_pointwise_pt(const Launch& lc, const uint64_t* ct, const uint64_t* pt, uint64_t* out);
// Query expansion, level a of c, over E = h 2^a items (packed ciphertext j, slot b), ciphertexts
// [h 2^c][2][L][N] in coefficient form with slot b of packed ciphertext j at j 2^c + b.
//   stage:   staging [E][3][L][N] = (sigma_g(c0), 0, sigma_g(c1)) of cts[j 2^c + b], where
//            sigma_g is x -> x^g and ginv = g^-1 mod 2N
//   combine: dst[j 2^c + b] = src[..] + sub[e], dst[j 2^c + b + 2^a] = x^(-2^a) (src[..] - sub[e]),
//            sub [E][2][L][N] in coefficient form; dst != src
void launch_expand_stage(const Launch& lc, const uint64_t* cts, uint32_t c, uint32_t a, uint32_t h, uint32_t ginv,
                         uint64_t* staging);
void launch_expand_combine(const Launch& lc, const uint64_t* src, const uint64_t* sub, uint32_t c, uint32_t a,
                           uint32_t h, uint64_t* dst);
// Modulus switching of `polys` polynomials [polys][L][N] -> [polys][keep][N] (coefficient form),
// x' = round(x q' / q) on centred representatives; S is a device copy of the switch constants.
void launch_mod_switch(const Launch& lc, const SwitchConst* S, uint32_t keep, const uint64_t* in, size_t polys,
                       uint64_t* out);
// Arithmetic equality helpers.
//   pair_refs:  refs[2i] = a0 + i, refs[2i + 1] = b0 + i for i < n
//   sum_rows:   S [rows][N] (+)= sum over e < cnt of C[e][rows][N] (mod the row's prime, row r uses
//               prime r mod L); overwrites S when `first`
//   sub_consts: F[i] = ct - i (the plaintext constant i: Delta i off coefficient 0 of c0), i < k
//   scalar_mul: out = ct * c (mod q_j), ct [count][L][N], c < every q_j
void launch_pair_refs(hipStream_t st, uint32_t* refs, uint32_t n, uint32_t a0, uint32_t b0);
void launch_sum_rows(const Launch& lc, const uint64_t* C, uint32_t cnt, uint32_t rows, bool first, uint64_t* S);
void launch_sub_consts(const Launch& lc, const uint64_t* ct, uint32_t k, uint64_t* F);
void launch_scalar_mul(const Launch& lc, const uint64_t* ct, uint32_t count, uint64_t c, uint64_t* out);
// Folklore leaves: out [2 ell][2][L][N] = (1 - x_i, x_i) for the query bits x_i [ell][2][L][N].
void launch_folklore_leaves(const Launch& lc, const uint64_t* query, uint32_t ell, uint64_t* out);
// Seeded query ciphertexts (seeded.hip): out [count][2][L][N] with out[i][0] = c0[i] ([count][L][N])
// and out[i][1] the uniform polynomial regenerated from `seed`.
void launch_seeded_query(const Launch& lc, const uint64_t* c0, uint32_t count, uint64_t seed, uint64_t* out);
// fp64 issue-rate probe (probe.hip): `blocks` workgroups of probe_threads() threads run `iters`
// steps of operation op (0 fma, 1 mul, 2 add, 3 rint + add) on 8 independent chains each, writing
// one double per thread to out; returns the wave-instructions of the timed operation(s).
uint32_t probe_threads();
double launch_probe_fp64(hipStream_t st, int op, uint32_t blocks, uint32_t iters, double* out);
// Integer issue-rate probe (probe.hip): op 0 v_mul_lo_u32, 1 v_mul_hi_u32, 2 v_mad_u64_u32,
// 3 v_lshl_add_u64 (64-bit add), on 8 independent chains; one u64 per thread to out.
double launch_probe_int(hipStream_t st, int op, uint32_t blocks, uint32_t iters, uint64_t* out);
// Row gather: dst row e = src row order[e] for e < n, rows of `row` uint16 (a multiple of 8).
void launch_gather_rows(hipStream_t st, const uint16_t* src, const uint64_t* order, uint64_t n, size_t row,
                        uint16_t* dst);
void launch_fill(hipStream_t st, uint64_t* p, size_t n, uint64_t v);
// Residue range check of `polys` polynomials [polys][L][N]: sets *flag (device) to 1 if any residue
// of limb j is >= q_j; the flag is left as it is otherwise.
void launch_check_residues(const Launch& lc, const uint64_t* x, size_t polys, uint32_t* flag);
void launch_map_perfect(hipStream_t st, const uint64_t* ids, size_t n, uint32_t m, uint32_t k, const uint64_t* binom,
                        uint32_t* out);
void launch_map_lossy(hipStream_t st, const uint64_t* kw, size_t n, uint32_t m, uint32_t k, uint64_t seed,
                      uint32_t* out);

}  // namespace cw
