/*
 * cwpir.h — C ABI of the MI355X (gfx950) server path of constant-weight PIR
 * (Mahdavi and Kerschbaum, "Constant-weight PIR: Single-round Keyword PIR via Constant-weight
 * Equality Operators", arXiv 2202.07569).
 *
 * The calls follow the protocol's stages (Section 3.3, table "Stages of PIR using constant-weight
 * codewords"): Setup (pir_setup, pir_load_key, pir_encode_db: choose parameters and put the
 * database in plaintext form with its precomputed codewords) and Process (pir_answer,
 * pir_answer_batch: selection vector by the plain constant-weight equality operator, Section 3.1
 * and Algorithm 6, followed by the inner product with the database, Section 2.3 Eq. (1) and the
 * "Inner Product" step of Section 3.3.3).  Query construction, key generation and decryption
 * are client-side and are not in this library.
 *
 * Arithmetic.  FV over R_q = Z_q[x]/(x^N+1), q = q_0 ... q_{L-1} (every listed prime is a
 * ciphertext prime), plaintext modulus t (Section 2.1.1).  All results are exact integers and are
 * bit-identical to the textbook definitions:
 *   Mult   c_r = round(t * X_r / q) mod q, X = centred lifts multiplied over Z[x]/(x^N+1);
 *   Relin  per-limb digits D_i = [c2]_{q_i} in [0, q_i):  (c0 + sum_i D_i b_i, c1 + sum_i D_i a_i);
 *   PM     plaintext coefficients in [0, t) taken as they are;
 *   selector of element j: product of the query ciphertexts at j's ascending one positions
 *          p_1 < ... < p_k, as the tree that pairs neighbours level by level ((p1 p2)(p3 p4)...),
 *          carries an odd last factor up and relinearizes after every Mult; k = 1 gives the query
 *          ciphertext itself;
 *   answer_r = sum_j PM(sel_j, P_{j,r}) mod q  for r in [s].
 *
 * Layouts (all little-endian uint64 residues in [0, q_i) unless stated):
 *   polynomial limb   N residues in coefficient order
 *   ciphertext        [2][L][N]              (c0 limbs, then c1 limbs)
 *   query             [m][2][L][N]           one ciphertext per codeword bit (compression c = 0)
 *   relin key         [L digits][2][L][N]    digit i holds (b_i, a_i)
 *   payload           uint16 [n][s][N]       coefficients in [0, 2^16) (< t = 65537)
 *   codewords         uint32 [n][k]          strictly ascending positions in [0, m)
 *   answer            [s][2][L][N]
 *
 * Ownership.  The caller owns every buffer it passes.  "dev" pointers are device memory of the
 * context's device (allocated by the caller, e.g. through PyTorch); "host" pointers are host
 * memory.  The library owns its internal copies (encoded database, transformed keys, work buffers)
 * and releases them in the matching *_free call.  Asynchronous calls enqueue work on the given HIP
 * stream (NULL = the default stream) and return before it runs: their inputs must stay alive and
 * unmodified, and their outputs unread, until the stream has completed the work.
 *
 * Errors.  Every int-returning call returns PIR_OK (0) or a negative code; pir_last_error()
 * returns a message for the calling thread's last failure.  No C++ exception crosses the ABI.
 * A HIP error inside a call returns PIR_E_DEVICE and poisons the context: later calls on it
 * return PIR_E_DEVICE.
 *
 * Concurrency.  Calls on one context are serialised by a lock; the context's work buffers are
 * shared, so two answers in flight on different streams of the same context are ordered by the
 * library (it waits for the previous call's stream before reusing them).
 */
#ifndef CWPIR_H
#define CWPIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIR_OK 0
#define PIR_E_INVALID (-1)     /* bad shape or parameter, residue >= q_i, bad codeword          */
#define PIR_E_NOMEM (-2)       /* allocation failed or the HBM budget is exceeded               */
#define PIR_E_DEVICE (-3)      /* HIP runtime error; the context is poisoned                    */
#define PIR_E_BUSY (-4)        /* the server is not idle (pir_serve_set_policy)                 */
#define PIR_E_UNSUPPORTED (-5) /* N not in {4096, 8192, 16384}, L or k out of range             */

#define PIR_MAX_L 12           /* ciphertext primes */
#define PIR_MAX_K 16           /* Hamming weight of the codewords (tree depth <= 4) */

typedef struct pir_ctx pir_ctx;
typedef struct pir_key pir_key;
typedef struct pir_db pir_db;
typedef struct pir_server pir_server;

typedef struct {
    uint32_t N;                /* ring degree: 4096, 8192 or 16384                                */
    uint32_t L;                /* number of ciphertext primes, 1..PIR_MAX_L                       */
    const uint64_t* q;         /* host [L]: distinct primes, each = 1 mod 2N and < 2^61           */
    uint64_t t;                /* plaintext modulus, 2 <= t < 2^32, coprime to q                  */
    uint64_t hbm_budget_bytes; /* cap on the library's own device allocations; 0 = no cap         */
    int32_t device;            /* HIP device ordinal                                              */
    uint32_t chunk_elems;      /* elements per processing chunk, 1..4096; 0 = default by N        */
    uint64_t memo_bytes;       /* cap on HBM for inner tree nodes shared by a whole database
                                  (k >= 3); above it they are shared within a chunk only;
                                  0 = default (a quarter of the budget, else 8 GiB)               */
} pir_params;

/* Setup (Section 3.3.1): validate the parameters and build the per-prime transform tables and the
 * exact base-conversion constants on `device`.  *out receives the context.  Synchronous. */
int pir_setup(const pir_params* params, pir_ctx** out);

/* Setup: load a relinearization key rlk (host or dev [L][2][L][N], coefficient form; see
 * "Relin" above) into the library's transformed representation.  Synchronous. */
int pir_load_key(pir_ctx* ctx, const uint64_t* rlk, pir_key** out);

/* Setup (Section 3.3.1, "Put DB in plaintext format"; codewords precomputed there as well):
 * copy n elements of s plaintexts each, with their weight-k codewords of length m, into the
 * library's device memory and precompute the selection-vector schedule (shared inner tree nodes
 * for k >= 3).  codewords: host [n][k]; payload: host or dev uint16 [n][s][N].  Synchronous. */
int pir_encode_db(pir_ctx* ctx, uint64_t n, uint32_t s, uint32_t m, uint32_t k, const uint32_t* codewords,
                  const uint16_t* payload, pir_db** out);

/* Process (Section 3.3.3: selection vector, Algorithm 6, then s inner products with the
 * database, Eq. (1)): answer = [s][2][L][N] for the query [m][2][L][N].  query and answer are dev
 * pointers; asynchronous on `stream` (a hipStream_t).  The query residues are not range-checked
 * here (that would need a wait on the device): a residue >= q_i gives an undefined answer.
 * Callers that cannot vouch for their queries check them first with pir_check_query. */
int pir_answer(pir_ctx* ctx, const pir_key* key, const pir_db* db, const uint64_t* query, uint64_t* answer,
               void* stream);

/* Range check of `count` ciphertexts (dev [count][2][L][N], e.g. a query with count = m): PIR_OK when
 * every residue of limb j is below q_j, PIR_E_INVALID (the context stays usable) otherwise.  One
 * read of the ciphertexts on `stream`; waits for the result (synchronous). */
int pir_check_query(pir_ctx* ctx, const uint64_t* query, uint32_t count, void* stream);

/* Process B queries in one call: the query ciphertexts' selection trees run side by side and
 * queries on the same database share one scan of its payload.  keys[b], dbs[b], queries[b],
 * answers[b] are as in pir_answer.  Every answer is bit-identical to pir_answer's.  Asynchronous. */
int pir_answer_batch(pir_ctx* ctx, uint32_t B, const pir_key* const* keys, const pir_db* const* dbs,
                     const uint64_t* const* queries, uint64_t* const* answers, void* stream);

/* Serving with continuous batching (Section 3.3.3 "Process", applied to a stream of queries on
 * several resident databases).  A server queues submitted queries and, at every pir_serve_step,
 * admits waiting queries into free slots and then advances each database that has active queries
 * by one chunk of elements: all its active queries compute their selectors for that chunk side by
 * side (as in pir_answer_batch) and share one transform of the chunk's payload.  A database's chunk
 * cursor rotates, so a query admitted mid-scan starts at the current chunk and completes after
 * one full cycle.  The answer is a sum over all elements and is bit-identical to pir_answer's.
 *
 *   pir_serve_open    server with max_slots (1..1024) concurrent queries and its own HIP stream
 *                     (default priority).  Synchronous.
 *   pir_serve_submit  queue one query; *ticket receives its id.  key/db from this context; query
 *                     (dev [m][2][L][N]) must be ready on the device when submitted and stay
 *                     unmodified, and answer (dev [s][2][L][N]) stays unread, until the ticket
 *                     completes.  The query's residues are range-checked first (pir_check_query,
 *                     on a stream of the server's own, waited for; it does not wait for the
 *                     queued rounds): PIR_E_INVALID for a residue >= q_i, and nothing is queued.
 *   pir_serve_step    admit (in submission order, while each query's buffers fit the context's
 *                     HBM budget) and run one round; returns the number of queries queued or active
 *                     (>= 0), or an error.  A query that does not fit waits for running queries to
 *                     finish; before that, the buffers idle slots keep for reuse and the context's
 *                     cached work buffers of other calls are released and the allocation retried.
 *                     PIR_E_NOMEM when no query is active and the oldest waiting one still does not
 *                     fit (it stays queued; the server and context stay usable).  Keeps at most two
 *                     rounds queued on the device.  Ordered after the context's other asynchronous
 *                     calls.
 *   pir_serve_poll    1 when the ticket's answer is complete in device memory (the ticket is then
 *                     released), 0 while it is queued or running, PIR_E_INVALID for an unknown or
 *                     released ticket.
 *   pir_serve_stats   counters: rounds run, queries admitted, tickets released; slots in use and
 *                     queries waiting now.  Any output pointer may be NULL.
 *   pir_serve_set_policy  which databases a round advances: PIR_SERVE_ROUND_ROBIN (default) every
 *                     database with active queries by one chunk, so queries share the GPU (short
 *                     queries finish early); PIR_SERVE_OLDEST_FIRST only the database of the oldest
 *                     active query, whose later queries ride along (first come, first served, with
 *                     batching); PIR_SERVE_SIZE_AGED only the active query with the smallest
 *                     priority submit time + aging * (elements of its database), one chunk per
 *                     round and no ride-along (a size-aware ordering that keeps the tail of first
 *                     come, first served; see pir_serve_set_aging).  Answers do not depend on the
 *                     policy.  Only an idle server (nothing queued or active) changes its policy:
 *                     PIR_E_BUSY otherwise.
 *   pir_serve_set_aging  the weight of PIR_SERVE_SIZE_AGED, in nanoseconds per database element
 *                     (>= 0, finite; default 0, which orders by submission).  Applies to queries
 *                     admitted afterwards.
 *   pir_serve_close   wait for the server's queued work and release its slots and stream.
 * A server belongs to one context; calls on it are serialised with that context's other calls. */
int pir_serve_open(pir_ctx* ctx, uint32_t max_slots, pir_server** out);
int pir_serve_submit(pir_server* srv, const pir_key* key, const pir_db* db, const uint64_t* query,
                     uint64_t* answer, uint64_t* ticket);
int pir_serve_step(pir_server* srv);
int pir_serve_poll(pir_server* srv, uint64_t ticket);
#define PIR_SERVE_ROUND_ROBIN 0
#define PIR_SERVE_OLDEST_FIRST 1
#define PIR_SERVE_SIZE_AGED 2
int pir_serve_set_policy(pir_server* srv, int policy);
int pir_serve_set_aging(pir_server* srv, double ns_per_element);
int pir_serve_stats(pir_server* srv, uint64_t* rounds, uint64_t* admitted, uint64_t* completed,
                    uint32_t* active, uint32_t* pending);
void pir_serve_close(pir_server* srv);

/* Query expansion (Section 3.3.3 "Query Expansion", Algorithm 5), for queries packed by the client
 * with compression factor c (Algorithm 4: h = ceil(m / 2^c) ciphertexts, ciphertext j encrypting
 * sum_i 2^-c E_q[j 2^c + i] x^i).
 *   pir_load_galois_key  load a key switching from s(x^g) to s, layout as the relinearization key
 *                        ([L digits][2][L][N], digit i holds b_i = -a_i s + e_i + g_i s(x^g), a_i);
 *                        g odd in (1, 2N).  Synchronous.
 *   pir_expand           packed (dev [h][2][L][N]) -> query (dev [m][2][L][N]): the first m of the
 *                        h 2^c ciphertexts of Algorithm 5, ciphertext j 2^c + b being slot b of
 *                        packed ciphertext j.  gkeys[a] (a < c) is the Galois key of
 *                        g = N / 2^a + 1.  Sub_g is the automorphism x -> x^g followed by the key
 *                        switch with per-limb digits [.]_{q_i} of the relinearization path.  The
 *                        output is a c = 0 query for pir_answer.  Asynchronous. */
int pir_load_galois_key(pir_ctx* ctx, uint32_t galois_elt, const uint64_t* gk, pir_key** out);
int pir_expand(pir_ctx* ctx, const pir_key* const* gkeys, uint32_t c, const uint64_t* packed, uint32_t h, uint32_t m,
               uint64_t* query, void* stream);

/* Folklore PIR (Section 2.4, the plain folklore equality operator f_PF): the client sends the
 * l = ceil(log2 n) bits of the target index, one ciphertext per bit (query dev [l][2][L][N]); the
 * server forms the 2l leaves (out dev [2l][2][L][N]): leaf 2i = 1 - x_i = (Delta - c0, -c1),
 * Delta = floor(q/t), and leaf 2i + 1 = x_i.  With element j's codeword {2i + bit_i(j)} (weight l,
 * length 2l) pir_answer then evaluates f_PF as the product tree above.  Asynchronous. */
int pir_folklore_leaves(pir_ctx* ctx, const uint64_t* query, uint32_t ell, uint64_t* out, void* stream);

/* Arithmetic constant-weight equality (Section 3.1, Algorithm 2) between two encrypted codewords of
 * CW(m, k): x, y dev [m][2][L][N], bit i of the codeword in ciphertext i (batch-encoded: every slot
 * holds its own comparison).  out (dev [2][L][N]) encrypts e = (1/k!) prod_{i < k} (k' - i) with
 * k' = sum_i x_i y_i: the m products (Mult, exact rounding) are summed and relinearized once, the
 * factors k' - i (the plaintext constant i subtracted) are multiplied by the product tree above,
 * and the result is multiplied by the plaintext constant (k!)^-1 mod t (k! invertible mod t).
 * Returns after the result is computed (synchronous). */
int pir_arith_equality(pir_ctx* ctx, const pir_key* key, const uint64_t* x, const uint64_t* y, uint32_t m, uint32_t k,
                       uint64_t* out, void* stream);

/* Response compression (the modulus switching of responses that the paper takes over from SealPIR,
 * Section 2.2): `count` polynomials in (dev [count][L][N], e.g. an answer [s][2][L][N] as 2s
 * polynomials) are switched from q to q' = q_0 ... q_{keep-1}: every coefficient's centred
 * representative x becomes round(q' x / q) (q / q' is odd, so there are no ties), written to out
 * (dev [count][keep][N]).  The client decrypts with q'.  1 <= keep <= L; in and out must not overlap.
 * Asynchronous. */
int pir_mod_switch(pir_ctx* ctx, const uint64_t* in, uint32_t count, uint32_t keep, uint64_t* out, void* stream);

/* Response compression for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same switch as
 * pir_mod_switch, bit for bit, with arguments, layouts and overlap rule as there.  It allocates
 * nothing and does not synchronise: its only scratch (the counter and list of coefficients whose
 * rounding takes the exact fallback) lives in a fixed array of 4 MiB + 256 bytes per GPU, which the
 * library holds from the first pir_setup on that GPU until the process ends.  Limit: count * N <=
 * 2^19 coefficients per call (e.g. 32 polynomials at N = 16384, 128 at N = 4096); larger requests
 * return PIR_E_INVALID and enqueue nothing, so split them into several calls.  Every call on one GPU
 * shares that GPU's array (across contexts too): calls whose work overlaps on the device race, so
 * order them on one stream or with events.  Asynchronous. */
int pir_mod_switch_noalloc(pir_ctx* ctx, const uint64_t* in, uint32_t count, uint32_t keep, uint64_t* out,
                           void* stream);

/* Seeded query ciphertexts (the compressed upload of secret-key encryption that the paper lists
 * among SealPIR's optimisations, Section 2; the upload column of the communication-cost table).
 * A secret-key ciphertext ([-a s + e + Delta m]_q, a) has a uniform a that the client need not
 * send: it sends c0 and a 64-bit seed.  The server rebuilds the full ciphertexts:
 *   c0   dev [count][L][N], residues in [0, q_j) (copied as they are)
 *   out  dev [count][2][L][N]: out[i][0] = c0[i], out[i][1][j][c] = (W(2u) 2^64 + W(2u + 1)) mod q_j
 *        with u = (i L + j) N + c and W(v) = SplitMix64 output number v + 1 from state `seed`,
 *        i.e. mix(seed + (v + 1) 0x9E3779B97F4A7C15 mod 2^64) (Steele, Lea and Flood 2014).
 * The result is a c = 0 query for pir_answer, or packed ciphertexts for pir_expand.  c0 and out
 * must not overlap; count * L * N must stay below 2^38.  count = 0 does nothing.  Asynchronous. */
int pir_seeded_query(pir_ctx* ctx, const uint64_t* c0, uint32_t count, uint64_t seed, uint64_t* out, void* stream);

/* Captured answers (HIP graphs), for callers that answer many queries of the same shape, e.g. a
 * serving loop with fixed query and answer slots.  pir_graph_capture runs pir_answer_batch once
 * for the given arguments (the answers for the queries' current contents are written) and records
 * its whole launch sequence into a HIP graph with work buffers of its own.  pir_graph_launch
 * replays it on `stream`, answering whatever the query buffers hold when the replay runs; it is
 * ordered after the context's other asynchronous calls like pir_answer.  Keys, databases, query
 * and answer buffers named at capture must outlive the graph; free graphs before their context.
 * While a graph exists the context's schedule is fixed.  pir_graph_capture is synchronous. */
typedef struct pir_graph pir_graph;
int pir_graph_capture(pir_ctx* ctx, uint32_t B, const pir_key* const* keys, const pir_db* const* dbs,
                      const uint64_t* const* queries, uint64_t* const* answers, pir_graph** out);
int pir_graph_launch(pir_graph* graph, void* stream);
void pir_graph_free(pir_graph* graph);

/* FV operations on single ciphertexts (Section 2.1.1: Multiplication, Plain multiplication), the
 * building blocks of the path, exposed for checking.  All pointers dev; asynchronous.
 *   pir_mult      a, b [2][L][N] -> out [3][L][N]    (textbook Mult, no relinearization)
 *   pir_relin     in [3][L][N]   -> out [2][L][N]
 *   pir_pm        ct [2][L][N], uint16 pt [N] -> out [2][L][N]                                */
int pir_mult(pir_ctx* ctx, const uint64_t* a, const uint64_t* b, uint64_t* out, void* stream);
int pir_relin(pir_ctx* ctx, const pir_key* key, const uint64_t* in, uint64_t* out, void* stream);
int pir_pm(pir_ctx* ctx, const uint64_t* ct, const uint16_t* pt, uint64_t* out, void* stream);

/* Selectors of chosen elements (Algorithm 6 for a subset of identifiers): out [count][2][L][N]
 * holds sel_j for j = elems[0..count) (host uint64 indices < n), coefficient form.  dev query/out;
 * synchronous (returns after the selectors are written). */
int pir_selectors(pir_ctx* ctx, const pir_key* key, const pir_db* db, const uint64_t* query,
                  const uint64_t* elems, uint32_t count, uint64_t* out, void* stream);

/* Codeword tables (Section 3.2 and the appendix on mappings), computed on the device.
 *   pir_map_perfect  Algorithm 3: ids (dev uint64 [n], each < C(m,k)) -> dev uint32 [n][k]
 *   pir_map_lossy    Algorithm 8 with H_i(x) = SplitMix64-mix(seed ^ x ^ i*0x9E3779B97F4A7C15)
 *                    mod m, i = 1, 2, ...: keywords (dev uint64 [n]) -> dev uint32 [n][k]
 * Positions are written ascending.  Asynchronous; m <= 65535, 1 <= k <= 16. */
int pir_map_perfect(pir_ctx* ctx, const uint64_t* ids, uint64_t n, uint32_t m, uint32_t k, uint32_t* out,
                    void* stream);
int pir_map_lossy(pir_ctx* ctx, const uint64_t* keywords, uint64_t n, uint32_t m, uint32_t k, uint64_t seed,
                  uint32_t* out, void* stream);

/* Launch schedule and its autotuner.  A schedule fixes how the path is cut into launches, never
 * what it computes (every schedule gives bit-identical answers):
 *   chunk_elems  elements per chunk (selector launches and payload transform), 1..4096
 *   query_group  queries whose selectors share one launch per stage, 1..8
 *   relin_group  order of the key-switching workgroups: 0 = the L output limbs of an element
 *                side by side on one XCD (they read the same digit rows); G > 0 = blocks of G
 *                elements, limb-major inside a block (workgroups running together read the same
 *                key limb).  N = 16384 stages its key switch and ignores it.
 *   ntt_shape    transform shape variant, below pir_ntt_shape_count: how the stages of every
 *                transform are grouped into passes between LDS exchanges.  All variants of a
 *                ring degree leave the same transformed layout, so the choice never changes a
 *                result.
 *   ns_per_elem  measured time per element and query (output of the tuner; ignored on input)
 * The schedule is per context and can change only while no database is encoded (PIR_E_INVALID
 * otherwise).
 *   pir_get_schedule  current schedule.
 *   pir_set_schedule  apply a schedule (e.g. one tuned earlier for the same N, L, batch and k).
 *   pir_autotune      time candidate schedules for `batch` queries per call on one database of
 *                     weight-k codewords and s plaintexts per element, on synthetic inputs of the
 *                     context's parameters (a grid over chunk and query group, then the
 *                     key-switch order at the best pair, then the transform shape at the best
 *                     schedule); apply the fastest and write it to *best (may be NULL).
 *                     records[0..max_records) receive the measured candidates in order (may be
 *                     NULL).  Candidates that do not fit the HBM budget are skipped.  Returns the
 *                     number of candidates measured, or an error.  Synchronous; the library's work
 *                     buffers are released afterwards. */
/* Where the relinearization of each element's root product happens (Section 3.3.3: the answer is
 * the inner product of the selection vector with the database, Eq. (1), and it is linear in every
 * selector).  Deferred: for trees with a multiplication and databases whose digit sums fit the
 * CRT of two dedicated primes (below 2^48 on the fp64 path, below 2^61 on the integer path), the root
 * products are multiplied into the payload before relinearization, their relinearization digits
 * summed separately, and the key multiplies those sums once per answer.  mode 0: never (every
 * selector is relinearized); 1 (the default): where allowed and the database is large enough to
 * repay the per-answer work (n (L^2 - 2L) >= 2048); 2: wherever allowed.  The answers are
 * bit-identical in every mode.  Changes only while no database is encoded (PIR_E_INVALID
 * otherwise).  pir_get_defer_relin returns the mode. */
int pir_set_defer_relin(pir_ctx* ctx, int mode);
int pir_get_defer_relin(pir_ctx* ctx);

typedef struct {
    uint32_t chunk_elems;
    uint32_t query_group;
    uint32_t relin_group;
    uint32_t ntt_shape;
    double ns_per_elem;
} pir_schedule;
int pir_get_schedule(pir_ctx* ctx, pir_schedule* out);
int pir_set_schedule(pir_ctx* ctx, const pir_schedule* schedule);
int pir_autotune(pir_ctx* ctx, uint32_t batch, uint32_t k, uint32_t s, pir_schedule* records, uint32_t max_records,
                 pir_schedule* best);

/* Introspection.  pir_ctx_aux_primes: the auxiliary basis B of the exact scale-and-round (the
 * largest primes = 1 mod 2N below 2^50 on the fp64 path, below 2^59 on the integer path (below 2^61
 * when 2^59 would take more than 13), until prod B > 4 t N q); returns their count and, when
 * out_primes is not NULL, writes them there. */
uint32_t pir_ctx_aux_primes(const pir_ctx* ctx, uint64_t* out_primes /* may be NULL */);
uint64_t pir_ctx_device_bytes(const pir_ctx* ctx);       /* bytes the library holds on the device */
uint64_t pir_db_pair_count(const pir_db* db);            /* distinct inner tree nodes (k >= 3)    */
/* 1 when answers on this database relinearize the root products after the inner product
 * (pir_set_defer_relin: the mode at encoding, the digit-sum bound and k >= 2), else 0 (also for a
 * null database). */
int pir_db_root_deferred(const pir_db* db);
/* Transform shape variants of the context's ring degree (pir_schedule.ntt_shape), and the number
 * of stages of each pass of variant `shape` in order (stages: room for 8; returns the number of
 * passes, 0 for an unknown variant or a null argument).  Each pass runs its stages in registers;
 * consecutive passes exchange through LDS. */
uint32_t pir_ntt_shape_count(const pir_ctx* ctx);
uint32_t pir_ntt_shape_stages(const pir_ctx* ctx, uint32_t shape, uint32_t* stages);

/* Kernel timing with HIP events on the launching stream.  When enabled, every kernel family's
 * launch is bracketed by events; pir_profile_read synchronises on them and returns, per family,
 * the summed milliseconds, the number of bracketed launches and the algorithmic work done
 * (butterflies for transforms, coefficients for the element-wise kernels).  Names stay valid
 * until the library is unloaded.  Any output pointer may be NULL.  Returns the number of
 * families (or a negative error code). */
int pir_profile_enable(pir_ctx* ctx, int on);
int pir_profile_read(pir_ctx* ctx, uint32_t max, const char** names, double* total_ms, uint64_t* launches,
                     double* work, int reset);

/* Diagnostics: issue rate of the fp64 instructions the transforms are built from.  Runs `blocks`
 * workgroups of 256 threads, each thread `iters` steps of one operation on 8 independent chains
 * (op 0 v_fma_f64, 1 v_mul_f64, 2 v_add_f64, 3 v_rndne_f64 followed by v_add_f64), once to warm up
 * and once timed with HIP events on `stream`; *ms receives the timed launch's duration and
 * *wave_instr the wave-instructions it issued of the timed operation(s).  1 <= blocks <= 2^20,
 * 1 <= iters <= 2^20.  Synchronous.  The rate (wave_instr / time) per CU and clock is the
 * reference for what the kernels' SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES counters can reach. */
int pir_probe_fp64(pir_ctx* ctx, int op, uint32_t blocks, uint32_t iters, double* ms, double* wave_instr,
                   void* stream);

/* Diagnostics: the same for the 32-bit integer instructions the integer-path transforms (N = 16384,
 * or primes at or above 2^50) are built from: op 0 v_mul_lo_u32, 1 v_mul_hi_u32, 2 v_mad_u64_u32,
 * 3 v_lshl_add_u64 (gfx950's one-instruction 64-bit add).  Arguments, timing and *wave_instr as for
 * pir_probe_fp64 (one wave-instruction per chain and step).  Synchronous. */
int pir_probe_int(pir_ctx* ctx, int op, uint32_t blocks, uint32_t iters, double* ms, double* wave_instr,
                  void* stream);

void pir_db_free(pir_db* db);
void pir_key_free(pir_key* key);
void pir_free(pir_ctx* ctx);
const char* pir_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CWPIR_H */
