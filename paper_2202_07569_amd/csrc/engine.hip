// Host engine and C ABI (include/cwpir.h) of the constant-weight PIR server path on gfx950.
//
// One answer (Section 3.3.3) runs as:
//   1. query residency: every query ciphertext is extended exactly from Q to Q u B and
//      transformed (once per query);
//   2. per group of elements: the distinct inner nodes of the elements' product trees (k >= 3) are
//      computed once, depth by depth — Mult + Relin, then extended and transformed again — and
//      kept in HBM;
//   3. per chunk of E elements: the root Mult + Relin of each element's tree gives its selector
//      (transformed over Q); the chunk's payload rows are lifted and transformed once and
//      multiplied into the accumulators of every query scanning this database;
//   4. the accumulators are transformed back into the answer ciphertexts.
// Everything is enqueued on the caller's stream; work buffers are owned by the context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/cwpir.h"
#include "host_params.h"
#include "kernels.h"

using cw::CtxConst;
using cw::Launch;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct ProfRec {
    const char* name;
    hipEvent_t a, b;
    double work;
};

struct pir_ctx {
    int device = 0;
    uint32_t N = 0, logN = 0, L = 0, LB = 0, LL = 0;
    uint64_t t = 0;
    std::vector<uint64_t> primes;  // Q then B
    CtxConst K;
    CtxConst* dK = nullptr;
    uint64_t* dtw = nullptr;
    double* dtwf = nullptr;
    bool fp = false;
    uint64_t budget = 0, held = 0;
    bool poisoned = false;
    std::recursive_mutex mu;
    uint64_t* dfix = nullptr;
    uint32_t* dfixcnt = nullptr;
    uint32_t* dflag = nullptr;  // result word of the residue range check (256-byte allocation)
    size_t fix_cap = 0;
    uint32_t chunk = 0;  // elements per chunk
    uint32_t qb = cw::MAX_QB;     // queries per selector launch
    uint32_t relin_group = 0;     // key-switch workgroup order (Launch::relin_group)
    uint32_t shape = 0;           // transform shape variant (Launch::shape)
    uint32_t live_dbs = 0;        // encoded databases not yet freed
    uint32_t live_graphs = 0;     // captured answers not yet freed
    uint32_t cus = 0;    // compute units
    uint64_t memo_cap = 0;
    std::map<std::string, DevBuf> ws;
    hipEvent_t done = nullptr;
    bool prof = false;
    std::vector<ProfRec> recs;
    struct ProfAcc {
        double ms = 0, work = 0;
        uint64_t launches = 0;
    };
    std::map<std::string, ProfAcc> prof_acc;
    std::map<std::pair<uint32_t, uint32_t>, uint64_t*> binom;  // (m, k) -> device table
    std::map<uint32_t, cw::SwitchConst*> switches;            // keep -> device switch constants
    uint32_t xslab = 0;       // most element-queries per tensor + scale launch (bounds the X buffer)
    int defer_mode = 1;       // root key switch after the inner product: 0 never, 1 where it pays, 2 where allowed
    bool crt_ok = false;      // the two primes of the deferred key switch exist
    cw::CrtConst crt{};
    void* scratch = nullptr;  // this device's copy of the no-allocation scratch array (device address)
    std::string scratch_err;  // why it is missing, if it is
};

struct pir_key {
    pir_ctx* ctx = nullptr;
    uint32_t galois = 0;    // 0: relinearization key; g: key switching from s(x^g) to s
    uint64_t* d = nullptr;  // [L][2][L][N] transformed, then [L][2][L][N] Shoup companions
    size_t bytes = 0;
};

struct Group {
    uint64_t e0 = 0, ne = 0;   // element range
    uint32_t p0 = 0, np = 0;   // node range in the node table
    std::vector<uint32_t> level_end;  // end of each depth's nodes, relative to p0
};

struct pir_db {
    pir_ctx* ctx = nullptr;
    uint64_t n = 0;
    uint32_t s = 0, m = 0, k = 0;
    uint16_t* dpay = nullptr;
    std::vector<uint32_t> cw;    // host codewords [n][k]
    std::vector<Group> groups;
    uint32_t* dpairs = nullptr;  // [pairs][2] leaf positions
    uint32_t* drefs = nullptr;   // [n][2] root operands
    uint32_t max_pairs = 0;
    uint64_t total_pairs = 0;
    size_t pay_bytes = 0, pairs_bytes = 0, refs_bytes = 0;
    bool live = false;           // counted in ctx->live_dbs
    bool defer_ok = false;       // the digit sums of this database fit the CRT of two auxiliary primes
    bool defer_worth = false;    // n (L^2 - 2L) >= 2048: deferring saves more than it adds per answer
};

// ------------------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------------------
// Deferred key switch of the root products (kernels.hip, "Root products with the key switch
// deferred past the inner product"): used when the database's digit sums fit the CRT of two
// auxiliary primes, for trees with at least one multiplication.
constexpr uint32_t ROOT_A = 2;  // auxiliary primes holding the digit sums
// Mode 2 defers wherever the bound allows; mode 1 (the default) also asks that the database be
// large enough to repay the per-answer work (the digit sums' CRT and key products, about L^2 + 3L
// transforms and a dozen launches) with the L^2 - 2L transforms saved per element.
static bool deferred(const pir_ctx* ctx, const pir_db* db) {
    return ctx->defer_mode == 2 ? db->defer_ok : ctx->defer_mode == 1 && db->defer_ok && db->defer_worth;
}
static uint32_t root_rows(const pir_ctx* ctx) { return 2 * ctx->L + ROOT_A * ctx->L; }  // RR

static uint32_t root_units(const pir_ctx* ctx, uint32_t s) {
    const uint32_t L = ctx->L;
    return s == 1 ? L + ROOT_A * ((L + 1) / 2) : root_rows(ctx) * ((s + 1) / 2);
}


#define CW_HIP(ctx, expr)                                                                                \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) {                                                                          \
            (ctx)->poisoned = true;                                                                      \
            return fail(PIR_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_));         \
        }                                                                                                \
    } while (0)

#define CW_TRY(expr)                \
    do {                            \
        int rc_ = (expr);           \
        if (rc_ != PIR_OK) return rc_; \
    } while (0)

static int dev_alloc(pir_ctx* ctx, void** p, size_t bytes) {
    *p = nullptr;
    if (!bytes) return PIR_OK;
    if (ctx->budget && ctx->held + bytes > ctx->budget)
        return fail(PIR_E_NOMEM, "HBM budget exceeded (" + std::to_string(ctx->held + bytes) + " > " +
                                     std::to_string(ctx->budget) + " bytes)");
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(PIR_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    ctx->held += bytes;
    return PIR_OK;
}

static void dev_free(pir_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    ctx->held -= bytes;
}

// Work buffer `name` of at least `bytes`; growing waits for all queued work first.
static int ws_get(pir_ctx* ctx, const std::string& name, size_t bytes, void** out) {
    DevBuf& b = ctx->ws[name];
    if (b.bytes >= bytes && b.p) {
        *out = b.p;
        return PIR_OK;
    }
    if (b.p) {
        CW_HIP(ctx, hipDeviceSynchronize());
        dev_free(ctx, b.p, b.bytes);
        b.p = nullptr;
        b.bytes = 0;
    }
    CW_TRY(dev_alloc(ctx, &b.p, bytes));
    b.bytes = bytes;
    *out = b.p;
    return PIR_OK;
}

template <typename T>
static int ws_get_t(pir_ctx* ctx, const std::string& name, size_t count, T** out) {
    void* p = nullptr;
    CW_TRY(ws_get(ctx, name, count * sizeof(T), &p));
    *out = (T*)p;
    return PIR_OK;
}

// Release cached work buffers other than the per-chunk ones every answer path uses (X, C, R, Ph, P);
// the caller has made sure that no queued work still reads them.
static void trim_work_buffers(pir_ctx* ctx) {
    for (auto it = ctx->ws.begin(); it != ctx->ws.end();) {
        const std::string& n = it->first;
        if (n == "X" || n == "C" || n == "R" || n == "Ph" || n == "P") {
            ++it;
            continue;
        }
        dev_free(ctx, it->second.p, it->second.bytes);
        it = ctx->ws.erase(it);
    }
}

static Launch make_launch(pir_ctx* ctx, hipStream_t st) {
    Launch lc;
    lc.stream = st;
    lc.K = ctx->dK;
    lc.tw = ctx->dtw;
    lc.twf = ctx->dtwf;
    lc.fp = ctx->fp;
    // the lazy key switch needs every ciphertext prime below 2^48 and its accumulators, below
    // (2.4 L + 15) max q_i, below 2^53
    double maxq = 0.0;
    lc.q_lazy = ctx->fp;
    for (uint32_t i = 0; i < ctx->L; ++i) {
        lc.q_lazy = lc.q_lazy && ctx->primes[i] < cw::FP_LAZY_BOUND;
        maxq = std::max(maxq, (double)ctx->primes[i]);
    }
    lc.q_lazy = lc.q_lazy && (2.4 * ctx->L + 16.0) * maxq < 9007199254740992.0;
    lc.N = ctx->N;
    lc.logN = ctx->logN;
    lc.L = ctx->L;
    lc.LB = ctx->LB;
    lc.LL = ctx->LL;
    lc.cus = ctx->cus;
    lc.relin_group = ctx->relin_group;
    lc.shape = ctx->shape;
    lc.fix = ctx->dfix;
    lc.fixcnt = ctx->dfixcnt;
    return lc;
}

// Profiling bracket: events on the launching stream around one kernel family's launch(es), with
// the algorithmic work they do (butterflies for transforms, coefficients for the others).
struct Prof {
    pir_ctx* ctx;
    const char* name;
    hipStream_t st;
    double work;
    hipEvent_t a = nullptr;
    Prof(pir_ctx* c, const char* n, hipStream_t s, double w = 0) : ctx(c), name(n), st(s), work(w) {
        if (ctx->prof && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, st);
    }
    ~Prof() {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, st) == hipSuccess)
            ctx->recs.push_back({name, a, b, work});
    }
};

static double bfly(const pir_ctx* ctx, size_t rows) { return (double)rows * (ctx->N / 2) * ctx->logN; }

static int check_launch(pir_ctx* ctx) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(PIR_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorName(e) + ": " +
                                      hipGetErrorString(e));
    }
    return PIR_OK;
}

// Order this call after the context's previous asynchronous call (possibly on another stream).
static int begin_async(pir_ctx* ctx, hipStream_t st) {
    CW_HIP(ctx, hipSetDevice(ctx->device));
    CW_HIP(ctx, hipStreamWaitEvent(st, ctx->done, 0));
    return PIR_OK;
}
static int end_async(pir_ctx* ctx, hipStream_t st) {
    CW_TRY(check_launch(ctx));
    CW_HIP(ctx, hipEventRecord(ctx->done, st));
    return PIR_OK;
}

// ------------------------------------------------------------------------------------------------
// no-allocation scratch
//
// pir_mod_switch_noalloc keeps its fixup counter and fixup list in this file-scope array instead of
// the context's buffers: bytes [0, 256) hold the counter, the rest the list (one 64-bit coefficient
// index per entry, NOALLOC_MAX_COEFFS entries).  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name is a host-side stand-in; kernels get the
// device address, looked up once per device (pir_setup, with the device current) and kept below.
// ------------------------------------------------------------------------------------------------
constexpr size_t NOALLOC_MAX_COEFFS = size_t(1) << 19;
constexpr size_t NOALLOC_SCRATCH_BYTES = 256 + NOALLOC_MAX_COEFFS * 8;
// External linkage on purpose: the HIP runtime resolves a registered device variable through the
// code object's dynamic symbol table, which holds global symbols only (a `static` array stays a
// local symbol there, and looking it up is fatal).
__device__ __align__(256) uint64_t cwpir_noalloc_scratch[NOALLOC_SCRATCH_BYTES / 8];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];        // device address of the array, per device ordinal
static std::string g_scratch_err[NOALLOC_MAX_DEVICES];  // why the lookup failed, if it did

// Called with `device` current.  A failed lookup leaves *out null: only pir_mod_switch_noalloc
// depends on it, and it then reports the lookup's error.
static void scratch_address(int device, void** out, std::string* why) {
    *out = nullptr;
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
        *why = "device ordinal beyond the scratch table";
        return;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_err[device].empty()) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(cwpir_noalloc_scratch));
        if (e == hipSuccess && p) {
            g_scratch_ptr[device] = p;
        } else {
            (void)hipGetLastError();
            g_scratch_err[device] =
                std::string("hipGetSymbolAddress(cwpir_noalloc_scratch) failed: ") + hipGetErrorString(e);
        }
    }
    *out = g_scratch_ptr[device];
    *why = g_scratch_err[device];
}

// Device constants of the modulus switch to q_0 ... q_{keep-1} (built once per keep).
static int switch_const(pir_ctx* ctx, uint32_t keep, cw::SwitchConst** out) {
    cw::SwitchConst*& dS = ctx->switches[keep];
    if (!dS) {
        cw::SwitchConst S;
        cw::host::build_switch(S, std::vector<uint64_t>(ctx->primes.begin(), ctx->primes.begin() + ctx->L), keep);
        CW_TRY(dev_alloc(ctx, (void**)&dS, sizeof(S)));
        CW_HIP(ctx, hipMemcpy(dS, &S, sizeof(S), hipMemcpyHostToDevice));
    }
    *out = dS;
    return PIR_OK;
}

// ------------------------------------------------------------------------------------------------
// setup
// ------------------------------------------------------------------------------------------------
extern "C" int pir_setup(const pir_params* params, pir_ctx** out) {
    if (!params || !out || !params->q) return fail(PIR_E_INVALID, "null argument");
    *out = nullptr;
    std::vector<uint64_t> q(params->q, params->q + params->L);
    if (params->L == 0 || params->L > PIR_MAX_L) return fail(PIR_E_UNSUPPORTED, "L out of range");
    if (params->N != 4096 && params->N != 8192 && params->N != 16384)
        return fail(PIR_E_UNSUPPORTED, "N must be 4096, 8192 or 16384");
    std::string why = cw::host::validate(params->N, q, params->t);
    if (!why.empty()) return fail(PIR_E_INVALID, why);
    // fp64 transforms need every prime below 2^50; then the auxiliary primes are chosen below 2^50
    bool fp = params->N <= 8192;
    for (uint64_t x : q) fp = fp && x < cw::FP_PRIME_BOUND;
    // (on the integer path below 2^59, where the conversions into B reduce lazily, unless that takes
    // more than MAX_LB primes; then below 2^61)
    std::vector<uint64_t> B = cw::host::aux_primes(params->N, q, params->t, fp ? cw::FP_PRIME_BOUND : cw::CONV_LAZY_BOUND);
    if (!fp && B.size() > (size_t)cw::MAX_LB) B = cw::host::aux_primes(params->N, q, params->t, 1ull << 61);
    if (B.size() > (size_t)cw::MAX_LB) return fail(PIR_E_UNSUPPORTED, "auxiliary basis too large");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(PIR_E_DEVICE, "no HIP device");
    if (params->device < 0 || params->device >= ndev) return fail(PIR_E_INVALID, "bad device ordinal");

    auto cleanup_early = [](int rc, pir_ctx* c) {
        delete c;
        return rc;
    };
    pir_ctx* ctx = new pir_ctx();
    ctx->device = params->device;
    ctx->N = params->N;
    ctx->logN = params->N == 4096 ? 12 : params->N == 8192 ? 13 : 14;
    ctx->L = params->L;
    ctx->LB = (uint32_t)B.size();
    ctx->LL = ctx->L + ctx->LB;
    ctx->t = params->t;
    ctx->budget = params->hbm_budget_bytes;
    ctx->primes = q;
    ctx->primes.insert(ctx->primes.end(), B.begin(), B.end());
    ctx->fp = fp;
    // two more primes for the deferred key switch's digit sums, after Q and B in every per-prime
    // table: below 2^48 on the fp64 path (their lazy transforms need no reduction between passes),
    // below 2^61 on the integer path (the lazy integer transform keeps values below 4p < 2^64)
    std::vector<uint64_t> D = cw::host::primes_below(ctx->N, fp ? cw::FP_LAZY_BOUND : (1ull << 61), 2, ctx->primes);
    if (D.size() == 2) ctx->primes.insert(ctx->primes.end(), D.begin(), D.end());
    else D.clear();
    cw::host::build_const(ctx->K, ctx->N, q, B, ctx->t, D);
    ctx->K.fp = fp ? 1 : 0;
    if (params->chunk_elems > 4096) return cleanup_early(fail(PIR_E_INVALID, "chunk_elems must be <= 4096"), ctx);
    ctx->chunk = params->chunk_elems ? params->chunk_elems : (ctx->N >= 16384 ? 128 : 256);
    ctx->memo_cap = params->memo_bytes ? params->memo_bytes : (ctx->budget ? ctx->budget / 4 : (8ull << 30));
    auto cleanup = [&](int rc) {
        pir_free(ctx);
        return rc;
    };
    if (hipSetDevice(ctx->device) != hipSuccess) return cleanup(fail(PIR_E_DEVICE, "hipSetDevice failed"));
    (void)hipGetLastError();  // a pending error of earlier runtime calls on this thread is not ours
    if (cw::kernels_init() != hipSuccess) return cleanup(fail(PIR_E_DEVICE, "kernel attribute setup failed"));
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess)
            return cleanup(fail(PIR_E_DEVICE, "hipGetDeviceProperties failed"));
        ctx->cus = (uint32_t)std::max(1, prop.multiProcessorCount);
    }
    std::vector<uint64_t> tw;
    std::vector<double> twf;
    cw::host::build_twiddles(tw, ctx->primes, ctx->N);
    if (fp) cw::host::build_twiddles_fp(twf, tw, ctx->primes, ctx->N, ctx->K);
    int rc;
    if ((rc = dev_alloc(ctx, (void**)&ctx->dK, sizeof(CtxConst))) != PIR_OK) return cleanup(rc);
    if ((rc = dev_alloc(ctx, (void**)&ctx->dtw, tw.size() * 8)) != PIR_OK) return cleanup(rc);
    if (fp && (rc = dev_alloc(ctx, (void**)&ctx->dtwf, twf.size() * 8)) != PIR_OK) return cleanup(rc);
    if (fp && hipMemcpy(ctx->dtwf, twf.data(), twf.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(PIR_E_DEVICE, "twiddle upload failed"));
    ctx->fix_cap = (size_t)3 * ctx->chunk * ctx->N * cw::MAX_QB;  // coefficients of one batched launch
    if ((rc = dev_alloc(ctx, (void**)&ctx->dfix, ctx->fix_cap * 8)) != PIR_OK) return cleanup(rc);
    if ((rc = dev_alloc(ctx, (void**)&ctx->dfixcnt, 256)) != PIR_OK) return cleanup(rc);
    if ((rc = dev_alloc(ctx, (void**)&ctx->dflag, 256)) != PIR_OK) return cleanup(rc);
    if (hipMemcpy(ctx->dK, &ctx->K, sizeof(CtxConst), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->dtw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(ctx->dfixcnt, 0, 256) != hipSuccess || hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return cleanup(fail(PIR_E_DEVICE, "device initialisation failed"));
    // tensor slabs of at most 1 GiB of X (slabs of 64 element-queries, 126 MB at N = 8192, which
    // stay in the Infinity Cache, measured 9 % slower for the tensor kernel and no faster for the
    // scale kernel), and at least four workgroups per compute unit per launch
    {
        const uint64_t per_eq = (uint64_t)3 * ctx->LL * ctx->N * 8;
        const uint64_t by_cache = std::max<uint64_t>(1, (1024ull << 20) / per_eq);
        const uint64_t by_grid = (4ull * ctx->cus + 3 * ctx->LL - 1) / (3 * ctx->LL);
        ctx->xslab = (uint32_t)std::max(by_cache, by_grid);
    }
    if (D.size() == 2) {
        cw::host::build_crt(ctx->crt, q, D[0], D[1]);
        ctx->crt_ok = true;
    }
    // switch constants for every keep, so that response compression never allocates later
    for (uint32_t keep = 1; keep <= ctx->L; ++keep) {
        cw::SwitchConst* dS = nullptr;
        if ((rc = switch_const(ctx, keep, &dS)) != PIR_OK) return cleanup(rc);
    }
    scratch_address(ctx->device, &ctx->scratch, &ctx->scratch_err);
    *out = ctx;
    return PIR_OK;
}

extern "C" void pir_free(pir_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& r : ctx->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto& kv : ctx->ws) dev_free(ctx, kv.second.p, kv.second.bytes);
    for (auto& kv : ctx->binom) (void)hipFree(kv.second);
    for (auto& kv : ctx->switches) dev_free(ctx, kv.second, sizeof(cw::SwitchConst));
    dev_free(ctx, ctx->dK, sizeof(CtxConst));
    dev_free(ctx, ctx->dtw, ctx->primes.size() * 4 * ctx->N * 8);
    if (ctx->dtwf) dev_free(ctx, ctx->dtwf, ctx->primes.size() * 4 * ctx->N * 8);
    dev_free(ctx, ctx->dfix, ctx->fix_cap * 8);
    dev_free(ctx, ctx->dfixcnt, 256);
    dev_free(ctx, ctx->dflag, 256);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    delete ctx;
}

extern "C" uint32_t pir_ctx_aux_primes(const pir_ctx* ctx, uint64_t* out) {
    if (!ctx) return 0;
    if (out)
        for (uint32_t j = 0; j < ctx->LB; ++j) out[j] = ctx->primes[ctx->L + j];
    return ctx->LB;
}

extern "C" uint64_t pir_ctx_device_bytes(const pir_ctx* ctx) { return ctx ? ctx->held : 0; }

extern "C" uint32_t pir_ntt_shape_count(const pir_ctx* ctx) { return ctx ? cw::ntt_shape_count(ctx->logN) : 0; }

extern "C" uint32_t pir_ntt_shape_stages(const pir_ctx* ctx, uint32_t shape, uint32_t* stages) {
    if (!ctx || !stages || shape >= cw::ntt_shape_count(ctx->logN)) return 0;
    return cw::ntt_shape_stages(ctx->logN, shape, stages);
}

extern "C" const char* pir_last_error(void) { return g_err.c_str(); }

// Every entry point takes the context's lock and clears the thread's last HIP error: a launch of
// this library is checked (check_launch) by the call that makes it, so a pending error at entry
// belongs to earlier, unrelated runtime calls on this thread and must not be taken for ours.
#define CW_ENTER(ctx)                                                               \
    if (!(ctx)) return fail(PIR_E_INVALID, "null context");                         \
    std::lock_guard<std::recursive_mutex> lock_((ctx)->mu);                         \
    if ((ctx)->poisoned) return fail(PIR_E_DEVICE, "context poisoned by an earlier device error"); \
    (void)hipGetLastError();

// ------------------------------------------------------------------------------------------------
// keys
// ------------------------------------------------------------------------------------------------
extern "C" int pir_load_key(pir_ctx* ctx, const uint64_t* rlk, pir_key** out) {
    CW_ENTER(ctx);
    if (!rlk || !out) return fail(PIR_E_INVALID, "null argument");
    *out = nullptr;
    CW_HIP(ctx, hipSetDevice(ctx->device));
    const uint32_t N = ctx->N, L = ctx->L;
    const size_t rows = (size_t)L * 2 * L, half = rows * N;
    std::vector<uint64_t> host(half);
    CW_HIP(ctx, hipMemcpy(host.data(), rlk, half * 8, hipMemcpyDefault));
    for (size_t r = 0; r < rows; ++r) {
        const uint64_t p = ctx->primes[r % L];
        for (uint32_t c = 0; c < N; ++c)
            if (host[r * N + c] >= p) return fail(PIR_E_INVALID, "relinearization key residue >= q_j");
    }
    pir_key* key = new pir_key();
    key->ctx = ctx;
    key->bytes = (ctx->fp ? 1 : 2) * half * 8;  // the integer operand format adds Shoup companions
    int rc = dev_alloc(ctx, (void**)&key->d, key->bytes);
    if (rc != PIR_OK) {
        delete key;
        return rc;
    }
    hipStream_t st = nullptr;
    Launch lc = make_launch(ctx, st);
    if (hipMemcpy(key->d, host.data(), half * 8, hipMemcpyHostToDevice) != hipSuccess) {
        pir_key_free(key);
        ctx->poisoned = true;
        return fail(PIR_E_DEVICE, "key upload failed");
    }
    cw::launch_ntt_operand(lc, key->d, key->d, rows, L, 0);
    if (!ctx->fp) cw::launch_shoup_companions(lc, key->d, key->d + half, rows, L);
    const hipError_t es = hipDeviceSynchronize(), el = hipGetLastError();
    if (es != hipSuccess || el != hipSuccess) {
        pir_key_free(key);
        ctx->poisoned = true;
        return fail(PIR_E_DEVICE, std::string("key transform failed: ") + hipGetErrorName(es) + " / " +
                                      hipGetErrorName(el));
    }
    *out = key;
    return PIR_OK;
}

extern "C" void pir_key_free(pir_key* key) {
    if (!key) return;
    std::lock_guard<std::recursive_mutex> lock(key->ctx->mu);
    (void)hipSetDevice(key->ctx->device);
    (void)hipDeviceSynchronize();
    dev_free(key->ctx, key->d, key->bytes);
    delete key;
}

// ------------------------------------------------------------------------------------------------
// database
// ------------------------------------------------------------------------------------------------
// Product tree of one element (leaves = its ascending positions): each level pairs neighbours
// (0,1), (2,3), ... into Mult+Relin nodes and carries an odd last operand up unchanged, until two
// operands remain, the root's (k = 1: the leaf itself).  k=2 (p1 p2); k=3 ((p1 p2) p3);
// k=4 ((p1 p2)(p3 p4)); k=5 (((p1 p2)(p3 p4)) p5); ...  A non-root node depends only on its two
// operands, so equal nodes are computed once per group.  Nodes are listed by depth (a node's
// operands are leaves or nodes of smaller depth), and level_end marks where each depth ends.
struct PlanBuild {
    std::vector<uint32_t> pairs;      // [np][2] operand refs (leaf position, or REF_NODE | node)
    std::vector<uint32_t> level_end;  // end of each depth's nodes in `pairs`
    std::vector<uint32_t> refs;       // [ne][2] root operands
};

static void plan_elements(const uint32_t* cw, uint64_t e0, uint64_t ne, uint32_t k, PlanBuild& pb) {
    std::unordered_map<uint64_t, uint32_t> ids;
    std::vector<uint32_t> ops, depth, roots;
    auto dep = [&](uint32_t r) -> uint32_t { return (r & cw::REF_NODE) ? depth[r & ~cw::REF_NODE] : 0u; };
    auto node = [&](uint32_t a, uint32_t b) -> uint32_t {
        const uint64_t key = ((uint64_t)a << 32) | b;
        auto it = ids.find(key);
        if (it != ids.end()) return it->second | cw::REF_NODE;
        const uint32_t id = (uint32_t)depth.size();
        ops.push_back(a);
        ops.push_back(b);
        depth.push_back(std::max(dep(a), dep(b)) + 1);
        ids.emplace(key, id);
        return id | cw::REF_NODE;
    };
    std::vector<uint32_t> lvl, nxt;
    roots.reserve(2 * ne);
    for (uint64_t e = e0; e < e0 + ne; ++e) {
        lvl.assign(cw + e * k, cw + e * k + k);
        while (lvl.size() > 2) {
            nxt.clear();
            for (size_t i = 0; i + 1 < lvl.size(); i += 2) nxt.push_back(node(lvl[i], lvl[i + 1]));
            if (lvl.size() % 2) nxt.push_back(lvl.back());
            lvl.swap(nxt);
        }
        roots.push_back(lvl[0]);
        roots.push_back(lvl.size() == 2 ? lvl[1] : 0u);
    }
    // list the nodes by depth and renumber
    const uint32_t nn = (uint32_t)depth.size();
    std::vector<uint32_t> order(nn), newid(nn);
    for (uint32_t i = 0; i < nn; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return depth[x] < depth[y]; });
    for (uint32_t r = 0; r < nn; ++r) newid[order[r]] = r;
    auto remap = [&](uint32_t r) { return (r & cw::REF_NODE) ? (newid[r & ~cw::REF_NODE] | cw::REF_NODE) : r; };
    pb.pairs.reserve(2 * (size_t)nn);
    for (uint32_t r = 0; r < nn; ++r) {
        pb.pairs.push_back(remap(ops[2 * (size_t)order[r]]));
        pb.pairs.push_back(remap(ops[2 * (size_t)order[r] + 1]));
        if (r + 1 == nn || depth[order[r + 1]] != depth[order[r]]) pb.level_end.push_back(r + 1);
    }
    for (uint32_t r : roots) pb.refs.push_back(remap(r));
}

static size_t node_bytes(const pir_ctx* ctx) { return (size_t)2 * ctx->LL * ctx->N * 8; }

// Payload rows [n][s][N] in the internal order: dst row e = src row order[e].  A device source is
// gathered by a kernel; a host source through a bounded host staging buffer.
static int upload_payload(pir_ctx* ctx, const uint16_t* src, const std::vector<uint64_t>& order, uint32_t s,
                          uint16_t* dst) {
    const uint64_t n = order.size();
    const size_t row = (size_t)s * ctx->N;  // uint16 per element
    hipPointerAttribute_t attr{};
    const bool on_device = hipPointerGetAttributes(&attr, src) == hipSuccess && attr.type == hipMemoryTypeDevice;
    (void)hipGetLastError();
    if (on_device) {
        uint64_t* dorder = nullptr;
        CW_TRY(dev_alloc(ctx, (void**)&dorder, n * 8));
        hipError_t e = hipMemcpy(dorder, order.data(), n * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            cw::launch_gather_rows(nullptr, src, dorder, n, row, dst);
            e = hipDeviceSynchronize();
            if (e == hipSuccess) e = hipGetLastError();
        }
        dev_free(ctx, dorder, n * 8);
        if (e != hipSuccess) {
            ctx->poisoned = true;
            return fail(PIR_E_DEVICE, std::string("payload upload failed: ") + hipGetErrorString(e));
        }
        return PIR_OK;
    }
    const uint64_t per = std::max<uint64_t>(1, (64ull << 20) / (row * 2));  // rows per 64 MiB staging
    std::vector<uint16_t> stage(std::min<uint64_t>(per, n) * row);
    for (uint64_t e0 = 0; e0 < n; e0 += per) {
        const uint64_t cnt = std::min(per, n - e0);
        for (uint64_t i = 0; i < cnt; ++i) std::memcpy(&stage[i * row], src + order[e0 + i] * row, row * 2);
        CW_HIP(ctx, hipMemcpy(dst + e0 * row, stage.data(), cnt * row * 2, hipMemcpyHostToDevice));
    }
    return PIR_OK;
}

extern "C" int pir_encode_db(pir_ctx* ctx, uint64_t n, uint32_t s, uint32_t m, uint32_t k, const uint32_t* codewords,
                             const uint16_t* payload, pir_db** out) {
    CW_ENTER(ctx);
    if (!out) return fail(PIR_E_INVALID, "null argument");
    *out = nullptr;
    if (k < 1 || k > PIR_MAX_K) return fail(PIR_E_UNSUPPORTED, "k must be in [1, 16]");
    if (s < 1 || m < k || m >= 0x7fffffffu) return fail(PIR_E_INVALID, "bad s or m");
    if (n && (!codewords || !payload)) return fail(PIR_E_INVALID, "null argument");
    if (n > (1ull << 40)) return fail(PIR_E_INVALID, "n too large");
    for (uint64_t e = 0; e < n; ++e) {
        const uint32_t* p = codewords + e * k;
        for (uint32_t a = 0; a < k; ++a) {
            if (p[a] >= m) return fail(PIR_E_INVALID, "codeword position >= m at element " + std::to_string(e));
            if (a && p[a] <= p[a - 1])
                return fail(PIR_E_INVALID, "codeword positions not strictly ascending at element " + std::to_string(e));
        }
    }
    CW_HIP(ctx, hipSetDevice(ctx->device));
    pir_db* db = new pir_db();
    db->ctx = ctx;
    db->n = n;
    db->s = s;
    db->m = m;
    db->k = k;
    db->cw.assign(codewords, codewords + n * k);
    // Internal element order: ascending codewords.  The answer is a sum over all elements, so the
    // order does not change it; sorted, consecutive elements share their first operand (a query
    // ciphertext for k = 2, a tree node for k >= 3), which then stays in cache, and a chunk
    // touches fewer distinct tree nodes.
    std::vector<uint64_t> order(n);
    for (uint64_t e = 0; e < n; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
        return std::lexicographical_compare(codewords + a * k, codewords + a * k + k, codewords + b * k,
                                            codewords + b * k + k);
    });
    std::vector<uint32_t> scw(n * k);
    for (uint64_t e = 0; e < n; ++e) std::memcpy(&scw[e * k], codewords + order[e] * k, (size_t)k * 4);
    // schedule: one group sharing all tree nodes when they fit the memo budget, else one
    // group per chunk of elements
    const uint32_t E = ctx->chunk;
    PlanBuild all;
    plan_elements(scw.data(), 0, n, k, all);
    const uint64_t memo_cap = ctx->memo_cap;
    const uint64_t np_all = all.pairs.size() / 2;
    PlanBuild pb;
    if (k < 3 || np_all * node_bytes(ctx) <= memo_cap) {
        Group g;
        g.e0 = 0;
        g.ne = n;
        g.p0 = 0;
        g.np = (uint32_t)np_all;
        g.level_end = all.level_end;
        db->groups.push_back(g);
        pb = std::move(all);
    } else {
        for (uint64_t e0 = 0; e0 < n; e0 += E) {
            Group g;
            g.e0 = e0;
            g.ne = std::min<uint64_t>(E, n - e0);
            g.p0 = (uint32_t)(pb.pairs.size() / 2);
            PlanBuild local;
            plan_elements(scw.data(), e0, g.ne, k, local);
            g.np = (uint32_t)(local.pairs.size() / 2);
            g.level_end = local.level_end;
            pb.pairs.insert(pb.pairs.end(), local.pairs.begin(), local.pairs.end());
            pb.refs.insert(pb.refs.end(), local.refs.begin(), local.refs.end());
            db->groups.push_back(g);
        }
    }
    for (auto& g : db->groups) db->max_pairs = std::max(db->max_pairs, g.np);
    db->total_pairs = pb.pairs.size() / 2;
    // deferred key switch: every coefficient of a digit sum sum_e D_e P_e lies below
    // n N max q_i (2^16 - 1) in magnitude, which the CRT of its two primes must hold with its sign
    if (ctx->crt_ok && k >= 2) {
        typedef unsigned __int128 u128;
        uint64_t maxq = 0;
        for (uint32_t i = 0; i < ctx->L; ++i) maxq = std::max(maxq, ctx->primes[i]);
        const u128 bound = (u128)std::max<uint64_t>(n, 1) * ctx->N * maxq;  // n < 2^40, N <= 2^14, q < 2^62
        const u128 prod = (u128)ctx->primes[ctx->LL] * ctx->primes[ctx->LL + 1];
        db->defer_ok = bound < (prod >> 17) && root_units(ctx, s) <= (uint32_t)cw::ROOT_MAX_UNITS;  // 2 bound 2^16 < b0 b1
        const uint64_t L = ctx->L;
        db->defer_worth = L >= 3 && n * (L * L - 2 * L) >= 2048;
    }
    const size_t pay_bytes = (size_t)n * s * ctx->N * 2;
    int rc = dev_alloc(ctx, (void**)&db->dpay, pay_bytes);
    if (rc == PIR_OK) db->pay_bytes = pay_bytes;
    if (rc == PIR_OK) rc = dev_alloc(ctx, (void**)&db->dpairs, std::max<size_t>(8, pb.pairs.size() * 4));
    if (rc == PIR_OK) db->pairs_bytes = std::max<size_t>(8, pb.pairs.size() * 4);
    if (rc == PIR_OK) rc = dev_alloc(ctx, (void**)&db->drefs, std::max<size_t>(8, pb.refs.size() * 4));
    if (rc == PIR_OK) db->refs_bytes = std::max<size_t>(8, pb.refs.size() * 4);
    if (rc != PIR_OK) {
        pir_db_free(db);
        return rc;
    }
    if (pay_bytes && (rc = upload_payload(ctx, payload, order, s, db->dpay)) != PIR_OK) {
        pir_db_free(db);
        return rc;
    }
    if ((!pb.pairs.empty() && hipMemcpy(db->dpairs, pb.pairs.data(), pb.pairs.size() * 4, hipMemcpyHostToDevice) != hipSuccess) ||
        (!pb.refs.empty() && hipMemcpy(db->drefs, pb.refs.data(), pb.refs.size() * 4, hipMemcpyHostToDevice) != hipSuccess) ||
        hipDeviceSynchronize() != hipSuccess) {
        pir_db_free(db);
        ctx->poisoned = true;
        return fail(PIR_E_DEVICE, "database upload failed");
    }
    db->live = true;
    ++ctx->live_dbs;
    *out = db;
    return PIR_OK;
}

extern "C" void pir_db_free(pir_db* db) {
    if (!db) return;
    pir_ctx* ctx = db->ctx;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    dev_free(ctx, db->dpay, db->pay_bytes);
    dev_free(ctx, db->dpairs, db->pairs_bytes);
    dev_free(ctx, db->drefs, db->refs_bytes);
    if (db->live) --ctx->live_dbs;
    delete db;
}

extern "C" uint64_t pir_db_pair_count(const pir_db* db) { return db ? db->total_pairs : 0; }

extern "C" int pir_db_root_deferred(const pir_db* db) {
    return db && db->ctx && deferred(db->ctx, db) && db->k >= 2 ? 1 : 0;
}

// ------------------------------------------------------------------------------------------------
// the path
// ------------------------------------------------------------------------------------------------
struct Bufs {
    uint64_t* X = nullptr;   // [QB E][3][LL][N]  tensor products over Q u B
    uint64_t* C = nullptr;   // [QB E][3][L][N]   after scale-and-round, coefficient form
    uint64_t* R = nullptr;   // [QB E][L+2][L][N] transformed digits (only where key switching is staged)
    uint64_t* Ph = nullptr;  // [E][s][L (+ ROOT_A)][N] transformed payload rows
    uint64_t* P = nullptr;   // deferred key switch: per-slice partial sums [slices][QB][s][RR][N]
};

// Elements per workgroup of the deferred key switch: enough workgroups for four per compute unit,
// and slices of at most 64 elements.
// A root workgroup runs alone on its compute unit (its exchange buffer and twiddle copy fill the
// LDS; at N = 4096 two fit), so a launch takes ceil(workgroups / resident) rounds of one
// workgroup's time, which grows with the slice (plus about one element's worth of set-up: the
// twiddle copy, the first row, the sums written out).  The slice minimises that product; among
// equal costs the longer slice writes fewer partial sums.  The workgroups of slice g run on XCD
// g mod 8 (xcd_split), so on the integer path the rounds are those of the busiest XCD, which holds
// ceil(slices / 8) slices on an eighth of the compute units (at the keyword parameters this took
// the root products from 6.3 to 3.2 ms per launch: slice 32 instead of 64, whose four slices left
// half of the XCDs idle).  The fp64 kernel counts all compute units together: on the one-query
// launches of the mid parameters (1024 elements, 11 units, about 4 TB/s) that choice (slice 45)
// measured 41.7 ms per answer against 41.9, 46.1 and 47.4 ms for slices 23, 64 and 32, and 42.4 ms
// for the busiest-XCD choice (16).
static uint32_t root_slice(const pir_ctx* ctx, uint32_t E, uint32_t nq, uint32_t units) {
    const uint64_t resident = (uint64_t)std::max<uint32_t>(ctx->cus, 1) * (ctx->fp && ctx->N == 4096 ? 2 : 1);
    const uint64_t per = (uint64_t)nq * units;
    const bool by_xcd = !ctx->fp;
    const uint64_t slots = by_xcd ? std::max<uint64_t>(1, resident / 8) : resident;
    uint64_t best = 1, best_cost = ~0ull;
    for (uint64_t slice = 1; slice <= 64; ++slice) {
        const uint64_t slices = ((uint64_t)std::max<uint32_t>(E, 1) + slice - 1) / slice;
        const uint64_t groups = (by_xcd ? (slices + 7) / 8 : slices) * per;
        const uint64_t cost = (groups + slots - 1) / slots * (slice + 1);
        if (cost <= best_cost) {
            best_cost = cost;
            best = slice;
        }
    }
    return (uint32_t)best;
}

// Work buffers for launches over up to `nq` queries of E elements each.
static int get_bufs(pir_ctx* ctx, uint32_t E, uint32_t nq, uint32_t s, Bufs& b, bool defer = false) {
    const size_t N = ctx->N, L = ctx->L, LL = ctx->LL, EQ = (size_t)E * nq;
    CW_TRY(ws_get_t(ctx, "X", std::min<size_t>(EQ, std::max<size_t>(1, ctx->xslab)) * 3 * LL * N, &b.X));
    CW_TRY(ws_get_t(ctx, "C", EQ * 3 * L * N, &b.C));
    if (cw::relin_needs_staging(ctx->logN)) CW_TRY(ws_get_t(ctx, "R", EQ * (L + 2) * L * N, &b.R));
    if (s) CW_TRY(ws_get_t(ctx, "Ph", (size_t)E * s * (L + (ctx->crt_ok ? ROOT_A : 0)) * N, &b.Ph));
    if (s && defer) {  // the most partial rows of any launch: up to nq queries, up to s payload rows
        size_t most = 0;
        for (uint32_t n = 1; n <= nq; ++n)
            for (uint32_t sp = 1; sp <= s; ++sp) {
                const uint32_t sl = root_slice(ctx, E, n, root_units(ctx, sp));
                most = std::max<size_t>(most, (size_t)((E + sl - 1) / sl) * n * sp);
            }
        CW_TRY(ws_get_t(ctx, "P", most * root_rows(ctx) * N, &b.P));
    }
    return PIR_OK;
}

// Per-query state of one answer in progress.
struct QState {
    const pir_key* key = nullptr;
    const uint64_t* query = nullptr;  // caller's [m][2][L][N]
    uint64_t* answer = nullptr;       // caller's [s][2][L][N]; accumulates in the transformed domain
    uint64_t* QX = nullptr;           // resident query [m][2][LL][N]
    uint64_t* nodes = nullptr;        // memoised tree nodes [max_pairs][2][LL][N] (k >= 3)
    uint64_t* sel = nullptr;          // selectors [E][2][L][N] (deferred: scratch of the tree nodes only)
    uint64_t* racc = nullptr;         // deferred key switch: accumulators [s][RR][N], transformed
};

static size_t qx_words(const pir_ctx* ctx, const pir_db* db) { return (size_t)db->m * 2 * ctx->LL * ctx->N; }
static size_t node_words(const pir_ctx* ctx, const pir_db* db) {
    return db->k >= 3 ? (size_t)std::max<uint32_t>(db->max_pairs, 1) * 2 * ctx->LL * ctx->N : 0;
}
// Selectors of a chunk; with the deferred key switch only the inner tree nodes (k >= 3) need them.
static size_t sel_words(const pir_ctx* ctx, const pir_db* db) {
    if (deferred(ctx, db) && db->k < 3) return 0;
    return (size_t)ctx->chunk * 2 * ctx->L * ctx->N;
}
static size_t racc_words(const pir_ctx* ctx, const pir_db* db) {
    return deferred(ctx, db) ? (size_t)db->s * root_rows(ctx) * ctx->N : 0;
}
static uint32_t num_chunks(const pir_ctx* ctx, const pir_db* db) {
    return (uint32_t)((db->n + ctx->chunk - 1) / ctx->chunk);
}

// Query residency: extend [m][2][L][N] to Q u B and transform.
static int make_leaves(pir_ctx* ctx, const Launch& lc, const uint64_t* query, uint32_t m, uint64_t* QX) {
    const size_t N = ctx->N, L = ctx->L, LL = ctx->LL;
    const size_t G = (size_t)2 * m, gmax = std::max<size_t>(1, ctx->fix_cap / N);
    {
        Prof pr(ctx, "extend", lc.stream, (double)G * N);
        for (size_t g0 = 0; g0 < G; g0 += gmax) {
            size_t g = std::min(gmax, G - g0);
            cw::launch_extend(lc, query + g0 * L * N, QX + g0 * LL * N, g);
        }
    }
    Prof pr(ctx, "ntt_fwd", lc.stream, bfly(ctx, G * LL));
    cw::launch_ntt_operand(lc, QX, QX, G * LL, (uint32_t)LL, 0);
    return check_launch(ctx);
}

// Mult + Relin of bt.E operand pairs (refs into leaves/nodes) for each query of the batch; the
// results, transformed over Q, go to bt.sel[q].
// Mult of bt.E operand pairs for each query of the batch: the tensor products, inverse-transformed,
// scaled and rounded into b.C [nq E][3][L][N] (coefficient form).
// The tensor products go through X in slabs of at most ctx->xslab rows (element-queries), each
// scaled into C right after it is written: X is bounded by the slab, not by the launch.  The slabs
// of a launch are of equal size (to one row), so that no launch is a small tail.
static void mult_only(pir_ctx* ctx, const Launch& lc, const Bufs& b, const uint32_t* refs, const cw::Batch& bt) {
    const size_t rows = (size_t)bt.nq * bt.E, most = std::max<size_t>(1, ctx->xslab);
    const size_t nslab = (rows + most - 1) / most, slab = std::max<size_t>(1, (rows + nslab - 1) / nslab);
    for (size_t eq0 = 0; eq0 < rows; eq0 += slab) {
        const size_t cnt = std::min(slab, rows - eq0);
        {
            Prof pr(ctx, "ntt_inv_tensor", lc.stream, bfly(ctx, cnt * 3 * ctx->LL));
            cw::launch_ntt_inv_tensor(lc, refs, bt, b.X, eq0, cnt);
        }
        Prof pr(ctx, "scale", lc.stream, (double)cnt * 3 * ctx->N);
        cw::launch_scale(lc, b.X, b.C + eq0 * 3 * ctx->L * ctx->N, (uint32_t)cnt);
    }
}

static void mult_relin(pir_ctx* ctx, const Launch& lc, const Bufs& b, const uint32_t* refs, const cw::Batch& bt) {
    mult_only(ctx, lc, b, refs, bt);
    const size_t rows = (size_t)bt.nq * bt.E;
    Prof pr(ctx, "relin", lc.stream, bfly(ctx, rows * (ctx->L + 2) * ctx->L));
    cw::launch_relin(lc, b.C, bt, b.R);
}

// Units of the deferred key switch (see cw::RootUnit): with one payload row per element, the pairs
// (c0_j, c1_j) modulo q_j and the digit pairs (D_i, D_i+1) modulo each auxiliary prime; otherwise
// every row alone, with up to two payload rows per unit.
static cw::RootPlan root_plan(const pir_ctx* ctx, uint32_t s, uint32_t nq, uint32_t E, uint32_t cnt) {
    cw::RootPlan rp{};
    const uint32_t L = ctx->L;
    rp.nq = nq;
    rp.E = cnt;
    rp.s = s;
    rp.LP = L + ROOT_A;
    rp.RR = root_rows(ctx);
    rp.A = ROOT_A;
    auto add = [&](uint32_t src0, uint32_t row0, uint32_t src1, uint32_t row1, bool two, uint32_t prime, uint32_t r0,
                   uint32_t nr) {
        cw::RootUnit& u = rp.u[rp.U++];
        u.src0 = (uint16_t)src0;
        u.row0 = (uint16_t)row0;
        u.src1 = (uint16_t)src1;
        u.row1 = (uint16_t)row1;
        u.two = two ? 1 : 0;
        u.prime = (uint8_t)prime;
        u.prow = (uint8_t)(prime < L ? prime : L + (prime - ctx->LL));
        u.r0 = (uint8_t)r0;
        u.nr = (uint8_t)nr;
    };
    // rows of C per element: c0 limb j = j, c1 limb j = L + j, digit i = 2L + i; accumulator rows:
    // c0 / c1 limb j = j / L + j, digit i modulo deferred-switch prime a = 2L + i A + a (context
    // prime LL + a)
    const uint32_t LL = ctx->LL;
    // the units of one digit (or digit pair) modulo the two primes are adjacent: their workgroups
    // run side by side on one XCD (xcd_split) and read the digit rows once from HBM
    if (s == 1) {
        for (uint32_t j = 0; j < L; ++j) add(j, j, L + j, L + j, true, j, 0, 1);
        for (uint32_t i = 0; i < L; i += 2)
            for (uint32_t a = 0; a < ROOT_A; ++a)
                add(2 * L + i, 2 * L + i * ROOT_A + a, 2 * L + i + 1, 2 * L + (i + 1) * ROOT_A + a, i + 1 < L, LL + a, 0, 1);
    } else {
        for (uint32_t r0 = 0; r0 < s; r0 += 2) {
            const uint32_t nr = std::min<uint32_t>(2, s - r0);
            for (uint32_t j = 0; j < 2 * L; ++j) add(j, j, 0, 0, false, j % L, r0, nr);
            for (uint32_t i = 0; i < L; ++i)
                for (uint32_t a = 0; a < ROOT_A; ++a) add(2 * L + i, 2 * L + i * ROOT_A + a, 0, 0, false, LL + a, r0, nr);
        }
    }
    rp.lazy = 1;  // lazy transforms when every ciphertext prime is below 2^48 (the D primes are)
    for (uint32_t j = 0; j < L; ++j) rp.lazy = rp.lazy && ctx->primes[j] < cw::FP_LAZY_BOUND;
    rp.slice = root_slice(ctx, E, nq, rp.U);
    rp.nslices = (cnt + rp.slice - 1) / rp.slice;
    return rp;
}

static cw::Batch one_query(uint32_t E, const uint64_t* leaves, const uint64_t* nodes, const pir_key* key, uint64_t* sel) {
    cw::Batch bt{};
    bt.nq = 1;
    bt.E = E;
    bt.leaves[0] = leaves;
    bt.nodes[0] = nodes;
    bt.rlk[0] = key->d;
    bt.sel[0] = sel;
    return bt;
}

// Memoised tree nodes pairs[0..np) into nodes (extended, transformed), depth by depth (a node reads
// nodes of smaller depth only), in chunks of E; `tmp` holds E selectors.
static void make_nodes(pir_ctx* ctx, const Launch& lc, const Bufs& b, const uint32_t* pairs,
                       const std::vector<uint32_t>& level_end, const uint64_t* leaves, const pir_key* key,
                       uint64_t* tmp, uint64_t* nodes, uint32_t E) {
    const size_t N = ctx->N, L = ctx->L, LL = ctx->LL;
    uint32_t start = 0;
    for (uint32_t end : level_end) {
        for (uint32_t p0 = start; p0 < end; p0 += E) {
            const uint32_t cnt = std::min(E, end - p0);
            mult_relin(ctx, lc, b, pairs + 2 * (size_t)p0, one_query(cnt, leaves, nodes, key, tmp));
            // the node's rows modulo the q_j are the key switch's output, already transformed: they
            // are taken as they are; only the auxiliary rows go through coefficients and back
            uint64_t* dst = nodes + (size_t)p0 * 2 * LL * N;
            {
                Prof pr(ctx, "extend", lc.stream, (double)2 * cnt * N);
                cw::launch_operand_q_rows(lc, tmp, dst, (size_t)2 * cnt);
            }
            {
                Prof pr(ctx, "ntt_inv", lc.stream, bfly(ctx, (size_t)cnt * 2 * L));
                cw::launch_ntt(lc, true, tmp, tmp, (size_t)cnt * 2 * L, L, 0);
            }
            {
                Prof pr(ctx, "extend", lc.stream, (double)2 * cnt * N);
                cw::launch_extend(lc, tmp, dst, (size_t)2 * cnt, false);
            }
            Prof pr(ctx, "ntt_fwd", lc.stream, bfly(ctx, (size_t)cnt * 2 * (LL - L)));
            cw::launch_ntt_operand(lc, dst, dst, (size_t)cnt * 2 * (LL - L), LL, 0, L);
        }
        start = end;
    }
}

static void roots(pir_ctx* ctx, const Launch& lc, const Bufs& b, uint32_t k, const uint32_t* refs,
                  const cw::Batch& bt) {
    if (k == 1) {
        Prof pr(ctx, "gather", lc.stream);
        cw::launch_gather_leaf(lc, refs, bt);
        return;
    }
    mult_relin(ctx, lc, b, refs, bt);
}

// Start an answer: resident query, zeroed accumulator and, when the database shares its tree
// products across all elements, those products.
static int prepare_query(pir_ctx* ctx, const Launch& lc, const Bufs& b, const pir_db* db, QState& qs) {
    CW_TRY(make_leaves(ctx, lc, qs.query, db->m, qs.QX));
    {
        Prof pr(ctx, "fill", lc.stream);
        if (deferred(ctx, db) && db->k >= 2) cw::launch_fill(lc.stream, qs.racc, racc_words(ctx, db), 0);
        else cw::launch_fill(lc.stream, qs.answer, (size_t)db->s * 2 * ctx->L * ctx->N, 0);
    }
    if (db->groups.size() == 1 && db->groups[0].np)
        make_nodes(ctx, lc, b, db->dpairs, db->groups[0].level_end, qs.QX, qs.key, qs.sel, qs.nodes, ctx->chunk);
    return check_launch(ctx);
}

// One chunk of the database for a set of queries: their selectors (one launch per stage for up to
// MAX_QB queries), one transform of the chunk's payload rows, and one multiply-accumulate launch
// for up to MAX_BATCH queries.
static int chunk_step(pir_ctx* ctx, const Launch& lc, const Bufs& b, const pir_db* db, uint32_t c, QState* const* qs,
                      uint32_t nq) {
    const size_t N = ctx->N, L = ctx->L;
    const uint32_t E = ctx->chunk, s = db->s, k = db->k;
    const uint64_t e0 = (uint64_t)c * E;
    const uint32_t cnt = (uint32_t)std::min<uint64_t>(E, db->n - e0);
    if (db->groups.size() > 1 && db->groups[c].np)  // tree nodes shared within this chunk only
        for (uint32_t q = 0; q < nq; ++q)
            make_nodes(ctx, lc, b, db->dpairs + 2 * (size_t)db->groups[c].p0, db->groups[c].level_end, qs[q]->QX, qs[q]->key,
                       qs[q]->sel, qs[q]->nodes, E);
    const uint32_t* refs = db->drefs + 2 * e0;
    if (deferred(ctx, db) && k >= 2) {
        // the chunk's payload modulo the q_j and the auxiliary primes, then per group of queries:
        // root products, their transforms times the payload summed per slice, slices into the
        // query's accumulators (the key switch waits for finalize_query)
        {
            Prof pr(ctx, "payload_ntt", lc.stream, bfly(ctx, (size_t)cnt * s * (L + ROOT_A)));
            cw::launch_ntt_payload(lc, db->dpay + e0 * s * N, b.Ph, (size_t)cnt * s, (uint32_t)L + ROOT_A, ctx->LL);
        }
        for (uint32_t q0 = 0; q0 < nq; q0 += ctx->qb) {
            cw::Batch bt{};
            bt.nq = std::min<uint32_t>(ctx->qb, nq - q0);
            bt.E = cnt;
            cw::QueryPtrs qp{};
            for (uint32_t q = 0; q < bt.nq; ++q) {
                const QState* x = qs[q0 + q];
                bt.leaves[q] = x->QX;
                bt.nodes[q] = x->nodes;
                bt.rlk[q] = x->key->d;
                qp.acc[q] = x->racc;
            }
            mult_only(ctx, lc, b, refs, bt);
            const cw::RootPlan rp = root_plan(ctx, s, bt.nq, E, cnt);
            {
                Prof pr(ctx, "root_pm", lc.stream,
                        bfly(ctx, (size_t)bt.nq * cnt * root_rows(ctx) * (s == 1 ? 1 : (s + 1) / 2)));
                cw::launch_root_pm(lc, b.C, b.Ph, rp, b.P);
            }
            Prof pr(ctx, "root_reduce", lc.stream, (double)rp.nslices * bt.nq * s * rp.RR * N);
            cw::launch_root_reduce(lc, b.P, rp, qp);
        }
        return check_launch(ctx);
    }
    for (uint32_t q0 = 0; q0 < nq; q0 += ctx->qb) {
        cw::Batch bt{};
        bt.nq = std::min<uint32_t>(ctx->qb, nq - q0);
        bt.E = cnt;
        for (uint32_t q = 0; q < bt.nq; ++q) {
            const QState* x = qs[q0 + q];
            bt.leaves[q] = x->QX;
            bt.nodes[q] = x->nodes;
            bt.rlk[q] = x->key->d;
            bt.sel[q] = x->sel;
        }
        roots(ctx, lc, b, k, refs, bt);
    }
    {
        Prof pr(ctx, "payload_ntt", lc.stream, bfly(ctx, (size_t)cnt * s * L));
        cw::launch_ntt_payload(lc, db->dpay + e0 * s * N, b.Ph, (size_t)cnt * s);
    }
    Prof pr(ctx, "accumulate", lc.stream, (double)nq * cnt * s * 2 * L * N);
    for (uint32_t q0 = 0; q0 < nq; q0 += cw::MAX_BATCH) {
        cw::QueryPtrs qp;
        const uint32_t n = std::min<uint32_t>(cw::MAX_BATCH, nq - q0);
        for (uint32_t q = 0; q < n; ++q) {
            qp.sel[q] = qs[q0 + q]->sel;
            qp.acc[q] = qs[q0 + q]->answer;
        }
        cw::launch_accumulate(lc, qp, b.Ph, n, cnt, s);
    }
    return check_launch(ctx);
}

static int finalize_query(pir_ctx* ctx, const Launch& lc, const pir_db* db, QState& qs) {
    const uint32_t L = ctx->L, s = db->s, RR = root_rows(ctx);
    const size_t N = ctx->N;
    if (deferred(ctx, db) && db->k >= 2) {
        // the deferred key switch: digit sums back to coefficients modulo b0 and b1, CRT to the
        // q_j, transformed again, multiplied by the key and added to the c0 / c1 sums
        uint64_t *Wc, *WQ;
        CW_TRY(ws_get_t(ctx, "root_wc", (size_t)s * L * ROOT_A * N, &Wc));
        CW_TRY(ws_get_t(ctx, "root_wq", (size_t)s * L * L * N, &WQ));
        Prof pr(ctx, "root_finalize", lc.stream, bfly(ctx, (size_t)s * (L * ROOT_A + L * L)));
        for (uint32_t r = 0; r < s; ++r)
            cw::launch_ntt(lc, true, qs.racc + ((size_t)r * RR + 2 * L) * N, Wc + (size_t)r * L * ROOT_A * N,
                           (size_t)L * ROOT_A, ROOT_A, ctx->LL);
        cw::launch_root_crt(lc, ctx->crt, Wc, s, WQ);
        cw::launch_ntt(lc, false, WQ, WQ, (size_t)s * L * L, L, 0);
        cw::launch_root_combine(lc, qs.racc, WQ, qs.key->d, s, RR, qs.answer);
    }
    Prof pr(ctx, "ntt_inv", lc.stream, bfly(ctx, (size_t)s * 2 * L));
    cw::launch_ntt(lc, true, qs.answer, qs.answer, (size_t)s * 2 * L, L, 0);
    return check_launch(ctx);
}

// B queries against one database.
static int answer_same_db(pir_ctx* ctx, hipStream_t st, const pir_db* db, uint32_t B, const pir_key* const* keys,
                          const uint64_t* const* queries, uint64_t* const* answers) {
    const uint32_t E = ctx->chunk;
    Launch lc = make_launch(ctx, st);
    Bufs b;
    CW_TRY(get_bufs(ctx, E, std::min<uint32_t>(B, ctx->qb), db->s, b, deferred(ctx, db)));
    uint64_t *QX, *nodes = nullptr, *sel = nullptr, *racc = nullptr;
    const size_t qx_one = qx_words(ctx, db), node_one = node_words(ctx, db), sel_one = sel_words(ctx, db);
    const size_t racc_one = racc_words(ctx, db);
    CW_TRY(ws_get_t(ctx, "QX", qx_one * B, &QX));
    if (node_one) CW_TRY(ws_get_t(ctx, "nodes", node_one * B, &nodes));
    if (sel_one) CW_TRY(ws_get_t(ctx, "sel", sel_one * B, &sel));
    if (racc_one) CW_TRY(ws_get_t(ctx, "racc", racc_one * B, &racc));
    std::vector<QState> st_q(B);
    std::vector<QState*> ptrs(B);
    for (uint32_t q = 0; q < B; ++q) {
        QState& x = st_q[q];
        x.key = keys[q];
        x.query = queries[q];
        x.answer = answers[q];
        x.QX = QX + q * qx_one;
        x.nodes = node_one ? nodes + q * node_one : nullptr;
        x.sel = sel_one ? sel + q * sel_one : nullptr;
        x.racc = racc_one ? racc + q * racc_one : nullptr;
        ptrs[q] = &x;
        CW_TRY(prepare_query(ctx, lc, b, db, x));
    }
    const uint32_t nc = num_chunks(ctx, db);
    for (uint32_t c = 0; c < nc; ++c) CW_TRY(chunk_step(ctx, lc, b, db, c, ptrs.data(), B));
    for (uint32_t q = 0; q < B; ++q) CW_TRY(finalize_query(ctx, lc, db, st_q[q]));
    return PIR_OK;
}

static int answer_dbs(pir_ctx* ctx, hipStream_t st, uint32_t B, const pir_key* const* keys, const pir_db* const* dbs,
                      const uint64_t* const* queries, uint64_t* const* answers);

static int check_batch(pir_ctx* ctx, uint32_t B, const pir_key* const* keys, const pir_db* const* dbs,
                       const uint64_t* const* queries, uint64_t* const* answers) {
    if (!keys || !dbs || !queries || !answers) return fail(PIR_E_INVALID, "null argument");
    for (uint32_t q = 0; q < B; ++q) {
        if (!keys[q] || !dbs[q] || !queries[q] || !answers[q]) return fail(PIR_E_INVALID, "null argument");
        if (keys[q]->ctx != ctx || dbs[q]->ctx != ctx) return fail(PIR_E_INVALID, "handle from another context");
        if (keys[q]->galois) return fail(PIR_E_INVALID, "a Galois key is not a relinearization key");
    }
    return PIR_OK;
}

extern "C" int pir_answer_batch(pir_ctx* ctx, uint32_t B, const pir_key* const* keys, const pir_db* const* dbs,
                                const uint64_t* const* queries, uint64_t* const* answers, void* stream) {
    CW_ENTER(ctx);
    if (B == 0) return PIR_OK;
    CW_TRY(check_batch(ctx, B, keys, dbs, queries, answers));
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    CW_TRY(answer_dbs(ctx, st, B, keys, dbs, queries, answers));
    return end_async(ctx, st);
}

// B queries: queries on the same database share its payload scan; databases run in first-seen
// order.  Enqueues only (no host synchronisation), so it can be captured into a graph.
static int answer_dbs(pir_ctx* ctx, hipStream_t st, uint32_t B, const pir_key* const* keys, const pir_db* const* dbs,
                      const uint64_t* const* queries, uint64_t* const* answers) {
    std::vector<const pir_db*> order;
    for (uint32_t q = 0; q < B; ++q)
        if (std::find(order.begin(), order.end(), dbs[q]) == order.end()) order.push_back(dbs[q]);
    for (const pir_db* db : order) {
        std::vector<const pir_key*> ks;
        std::vector<const uint64_t*> qs;
        std::vector<uint64_t*> as;
        for (uint32_t q = 0; q < B; ++q)
            if (dbs[q] == db) {
                ks.push_back(keys[q]);
                qs.push_back(queries[q]);
                as.push_back(answers[q]);
            }
        CW_TRY(answer_same_db(ctx, st, db, (uint32_t)ks.size(), ks.data(), qs.data(), as.data()));
    }
    return PIR_OK;
}

extern "C" int pir_answer(pir_ctx* ctx, const pir_key* key, const pir_db* db, const uint64_t* query, uint64_t* answer,
                          void* stream) {
    return pir_answer_batch(ctx, 1, &key, &db, &query, &answer, stream);
}

extern "C" int pir_selectors(pir_ctx* ctx, const pir_key* key, const pir_db* db, const uint64_t* query,
                             const uint64_t* elems, uint32_t count, uint64_t* out, void* stream) {
    CW_ENTER(ctx);
    if (!key || !db || !query || (count && (!elems || !out))) return fail(PIR_E_INVALID, "null argument");
    for (uint32_t i = 0; i < count; ++i)
        if (elems[i] >= db->n) return fail(PIR_E_INVALID, "element index out of range");
    if (!count) return PIR_OK;
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    const size_t N = ctx->N, L = ctx->L, LL = ctx->LL;
    const uint32_t E = ctx->chunk, k = db->k;
    Launch lc = make_launch(ctx, st);
    Bufs b;
    CW_TRY(get_bufs(ctx, E, 1, 0, b));
    uint64_t *QX, *sel, *nodes = nullptr;
    CW_TRY(ws_get_t(ctx, "QX", (size_t)db->m * 2 * LL * N, &QX));
    CW_TRY(ws_get_t(ctx, "sel", (size_t)E * 2 * L * N, &sel));
    CW_TRY(make_leaves(ctx, lc, query, db->m, QX));
    for (uint32_t c0 = 0; c0 < count; c0 += E) {
        const uint32_t cnt = std::min(E, count - c0);
        std::vector<uint32_t> cw((size_t)cnt * k);
        for (uint32_t i = 0; i < cnt; ++i)
            std::memcpy(&cw[(size_t)i * k], &db->cw[elems[c0 + i] * k], k * 4);
        PlanBuild pb;
        plan_elements(cw.data(), 0, cnt, k, pb);
        uint32_t *dpairs, *drefs;
        CW_TRY(ws_get_t(ctx, "sel_pairs", std::max<size_t>(2, pb.pairs.size()), &dpairs));
        CW_TRY(ws_get_t(ctx, "sel_refs", pb.refs.size(), &drefs));
        if (!pb.pairs.empty())
            CW_HIP(ctx, hipMemcpyAsync(dpairs, pb.pairs.data(), pb.pairs.size() * 4, hipMemcpyHostToDevice, st));
        CW_HIP(ctx, hipMemcpyAsync(drefs, pb.refs.data(), pb.refs.size() * 4, hipMemcpyHostToDevice, st));
        const uint32_t np = (uint32_t)(pb.pairs.size() / 2);
        if (np) {
            CW_TRY(ws_get_t(ctx, "sel_nodes", (size_t)np * 2 * LL * N, &nodes));
            make_nodes(ctx, lc, b, dpairs, pb.level_end, QX, key, sel, nodes, E);
        }
        roots(ctx, lc, b, k, drefs, one_query(cnt, QX, nodes, key, sel));
        cw::launch_ntt(lc, true, sel, out + (size_t)c0 * 2 * L * N, (size_t)cnt * 2 * L, L, 0);
        CW_HIP(ctx, hipStreamSynchronize(st));  // the plan lives in pageable host memory
    }
    return end_async(ctx, st);
}

// Range check of `polys` polynomials [polys][L][N] on stream st; waits for the result.
static int check_residues(pir_ctx* ctx, hipStream_t st, const uint64_t* x, size_t polys) {
    if (!polys) return PIR_OK;
    CW_HIP(ctx, hipSetDevice(ctx->device));
    Launch lc = make_launch(ctx, st);
    cw::launch_fill(st, (uint64_t*)ctx->dflag, 1, 0);
    cw::launch_check_residues(lc, x, polys, ctx->dflag);
    CW_TRY(check_launch(ctx));
    uint32_t h = 0;
    CW_HIP(ctx, hipMemcpyAsync(&h, ctx->dflag, 4, hipMemcpyDeviceToHost, st));
    CW_HIP(ctx, hipStreamSynchronize(st));
    if (h) return fail(PIR_E_INVALID, "a query residue is not below its prime (residue >= q_i)");
    return PIR_OK;
}

extern "C" int pir_check_query(pir_ctx* ctx, const uint64_t* query, uint32_t count, void* stream) {
    CW_ENTER(ctx);
    if (count && !query) return fail(PIR_E_INVALID, "null argument");
    return check_residues(ctx, (hipStream_t)stream, query, (size_t)count * 2);
}

// ------------------------------------------------------------------------------------------------
// serving: continuous batching
//
// A server owns a stream and up to max_slots query slots.  Each call of pir_serve_step admits
// waiting requests into free slots (when their buffers fit the HBM budget) and then runs one round:
// every database with active queries advances by one chunk, and all its active queries process
// that same chunk together (one selector launch per stage for up to MAX_QB queries, one payload
// transform, one multiply-accumulate).  A database's chunk cursor keeps rotating, so a query that
// joins mid-scan starts at the current chunk and leaves after one full cycle: the answer is a sum
// over all chunks and does not depend on their order.  Under the size-aged policy a round instead
// advances the one active query with the smallest priority along its own cursor.  At most two
// rounds are in flight.
// ------------------------------------------------------------------------------------------------
struct ServeReq {
    const pir_key* key;
    const pir_db* db;
    const uint64_t* query;
    uint64_t* answer;
    uint64_t ticket;
    uint64_t submit_ns;  // host steady clock at submission
};

struct ServeSlot {
    bool used = false;
    const pir_db* db = nullptr;
    uint64_t ticket = 0;
    uint32_t chunks_left = 0;
    uint32_t next = 0;   // PIR_SERVE_SIZE_AGED: the query's own next chunk
    double key = 0.0;    // PIR_SERVE_SIZE_AGED: priority (smaller first)
    QState qs;
    uint64_t* buf = nullptr;  // QX, nodes and sel of this slot
    size_t buf_words = 0;
};

struct pir_server {
    pir_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t check_stream = nullptr;  // residue checks of submitted queries
    std::vector<ServeSlot> slots;
    std::deque<ServeReq> pending;
    std::map<const pir_db*, uint32_t> cursor;
    std::unordered_map<uint64_t, hipEvent_t> done;   // ticket -> completion event
    std::set<uint64_t> in_flight;                    // tickets submitted and not yet completed
    std::deque<hipEvent_t> rounds;
    uint64_t next_ticket = 1;
    uint64_t n_rounds = 0, n_admitted = 0, n_completed = 0;
    int policy = PIR_SERVE_ROUND_ROBIN;
    double aging_ns = 0.0;  // PIR_SERVE_SIZE_AGED weight per database element
};

extern "C" int pir_serve_open(pir_ctx* ctx, uint32_t max_slots, pir_server** out) {
    CW_ENTER(ctx);
    if (!out || max_slots == 0 || max_slots > 1024) return fail(PIR_E_INVALID, "max_slots must be in [1, 1024]");
    *out = nullptr;
    CW_HIP(ctx, hipSetDevice(ctx->device));
    pir_server* srv = new pir_server();
    srv->ctx = ctx;
    srv->slots.resize(max_slots);
    if (hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess) {
        delete srv;
        return fail(PIR_E_DEVICE, "stream creation failed");
    }
    if (hipStreamCreateWithFlags(&srv->check_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(srv->stream);
        delete srv;
        return fail(PIR_E_DEVICE, "stream creation failed");
    }
    *out = srv;
    return PIR_OK;
}

extern "C" int pir_serve_submit(pir_server* srv, const pir_key* key, const pir_db* db, const uint64_t* query,
                                uint64_t* answer, uint64_t* ticket) {
    if (!srv) return fail(PIR_E_INVALID, "null server");
    pir_ctx* ctx = srv->ctx;
    CW_ENTER(ctx);
    if (!key || !db || !query || !answer || !ticket) return fail(PIR_E_INVALID, "null argument");
    if (key->ctx != ctx || db->ctx != ctx) return fail(PIR_E_INVALID, "handle from another context");
    if (key->galois) return fail(PIR_E_INVALID, "a Galois key is not a relinearization key");
    CW_TRY(check_residues(ctx, srv->check_stream, query, (size_t)2 * db->m));
    *ticket = srv->next_ticket++;
    const uint64_t now = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                             std::chrono::steady_clock::now().time_since_epoch())
                             .count();
    srv->pending.push_back({key, db, query, answer, *ticket, now});
    srv->in_flight.insert(*ticket);
    return PIR_OK;
}

static int serve_admit(pir_server* srv, const Launch& lc, const Bufs& b) {
    pir_ctx* ctx = srv->ctx;
    for (ServeSlot& sl : srv->slots) {
        if (srv->pending.empty()) break;
        if (sl.used) continue;
        const ServeReq r = srv->pending.front();
        const size_t qxw = qx_words(ctx, r.db), nw = node_words(ctx, r.db), sw = sel_words(ctx, r.db);
        const size_t rw = racc_words(ctx, r.db);
        const size_t need = qxw + nw + sw + rw;
        if (sl.buf_words < need) {
            if (sl.buf) {
                CW_HIP(ctx, hipStreamSynchronize(srv->stream));
                dev_free(ctx, sl.buf, sl.buf_words * 8);
                sl.buf = nullptr;
                sl.buf_words = 0;
            }
            if (dev_alloc(ctx, (void**)&sl.buf, need * 8) != PIR_OK) {
                // idle slots keep their buffers for reuse: release them (once their queued work has
                // run) and the context's cached work buffers that serving does not use, then retry
                CW_HIP(ctx, hipStreamSynchronize(srv->stream));
                for (ServeSlot& o : srv->slots)
                    if (!o.used && o.buf) {
                        dev_free(ctx, o.buf, o.buf_words * 8);
                        o.buf = nullptr;
                        o.buf_words = 0;
                    }
                trim_work_buffers(ctx);
                if (dev_alloc(ctx, (void**)&sl.buf, need * 8) != PIR_OK) {
                    bool any = false;
                    for (const ServeSlot& o : srv->slots) any = any || o.used;
                    if (!any) return PIR_E_NOMEM;  // nothing running will free memory: report it
                    g_err.clear();                 // the request waits for a running query to finish
                    return PIR_OK;
                }
            }
            sl.buf_words = need;
        }
        sl.used = true;
        sl.db = r.db;
        sl.ticket = r.ticket;
        sl.chunks_left = num_chunks(ctx, r.db);
        sl.next = 0;
        sl.key = (double)r.submit_ns + srv->aging_ns * (double)r.db->n;
        sl.qs = QState{};
        sl.qs.key = r.key;
        sl.qs.query = r.query;
        sl.qs.answer = r.answer;
        sl.qs.QX = sl.buf;
        sl.qs.nodes = nw ? sl.buf + qxw : nullptr;
        sl.qs.sel = sw ? sl.buf + qxw + nw : nullptr;
        sl.qs.racc = rw ? sl.buf + qxw + nw + sw : nullptr;
        srv->pending.pop_front();
        ++srv->n_admitted;
        CW_TRY(prepare_query(ctx, lc, b, r.db, sl.qs));
    }
    return PIR_OK;
}

static int serve_finish(pir_server* srv, const Launch& lc, ServeSlot& sl) {
    pir_ctx* ctx = srv->ctx;
    CW_TRY(finalize_query(ctx, lc, sl.db, sl.qs));
    hipEvent_t ev;
    CW_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    CW_HIP(ctx, hipEventRecord(ev, srv->stream));
    srv->done[sl.ticket] = ev;
    sl.used = false;  // stream order keeps the slot's buffers until the queued work has run
    return PIR_OK;
}

extern "C" int pir_serve_step(pir_server* srv) {
    if (!srv) return fail(PIR_E_INVALID, "null server");
    pir_ctx* ctx = srv->ctx;
    CW_ENTER(ctx);
    CW_TRY(begin_async(ctx, srv->stream));  // work buffers are shared with the context's other calls
    while (srv->rounds.size() >= 2) {  // bound the queued work
        CW_HIP(ctx, hipEventSynchronize(srv->rounds.front()));
        (void)hipEventDestroy(srv->rounds.front());
        srv->rounds.pop_front();
    }
    Launch lc = make_launch(ctx, srv->stream);
    uint32_t max_s = 1;
    bool defer = false;
    for (const ServeSlot& sl : srv->slots)
        if (sl.used) {
            max_s = std::max(max_s, sl.db->s);
            defer = defer || deferred(ctx, sl.db);
        }
    for (const ServeReq& r : srv->pending) {
        max_s = std::max(max_s, r.db->s);
        defer = defer || deferred(ctx, r.db);
    }
    Bufs b;
    CW_TRY(get_bufs(ctx, ctx->chunk, ctx->qb, max_s, b, defer));
    CW_TRY(serve_admit(srv, lc, b));
    if (srv->policy == PIR_SERVE_SIZE_AGED) {  // one chunk of the query with the smallest priority
        ServeSlot* best = nullptr;
        for (ServeSlot& sl : srv->slots)
            if (sl.used && (!best || sl.key < best->key || (sl.key == best->key && sl.ticket < best->ticket)))
                best = &sl;
        if (best) {
            const uint32_t nc = num_chunks(ctx, best->db);
            if (nc) {
                QState* q = &best->qs;
                CW_TRY(chunk_step(ctx, lc, b, best->db, best->next, &q, 1));
                best->next = (best->next + 1) % nc;
            }
            if (best->chunks_left) --best->chunks_left;
            if (!best->chunks_left) CW_TRY(serve_finish(srv, lc, *best));
        }
    }
    // otherwise one round: every database with active queries advances by one chunk (round robin),
    // or only the database of the oldest active query (oldest first)
    std::vector<const pir_db*> dbs;
    if (srv->policy == PIR_SERVE_OLDEST_FIRST) {
        const ServeSlot* oldest = nullptr;
        for (const ServeSlot& sl : srv->slots)
            if (sl.used && (!oldest || sl.ticket < oldest->ticket)) oldest = &sl;
        if (oldest) dbs.push_back(oldest->db);
    } else if (srv->policy == PIR_SERVE_ROUND_ROBIN) {
        for (const ServeSlot& sl : srv->slots)
            if (sl.used && std::find(dbs.begin(), dbs.end(), sl.db) == dbs.end()) dbs.push_back(sl.db);
    }
    for (const pir_db* db : dbs) {
        std::vector<ServeSlot*> active;
        std::vector<QState*> qs;
        for (ServeSlot& sl : srv->slots)
            if (sl.used && sl.db == db) {
                active.push_back(&sl);
                qs.push_back(&sl.qs);
            }
        const uint32_t nc = num_chunks(ctx, db);
        if (nc) {
            uint32_t& c = srv->cursor[db];
            c %= nc;
            CW_TRY(chunk_step(ctx, lc, b, db, c, qs.data(), (uint32_t)qs.size()));
            c = (c + 1) % nc;
        }
        for (ServeSlot* sl : active) {
            if (sl->chunks_left) --sl->chunks_left;
            if (!sl->chunks_left) CW_TRY(serve_finish(srv, lc, *sl));
        }
    }
    CW_TRY(end_async(ctx, srv->stream));
    hipEvent_t ev;
    CW_HIP(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    CW_HIP(ctx, hipEventRecord(ev, srv->stream));
    srv->rounds.push_back(ev);
    ++srv->n_rounds;
    uint32_t busy = (uint32_t)srv->pending.size();
    for (const ServeSlot& sl : srv->slots) busy += sl.used ? 1 : 0;
    return (int)busy;
}

extern "C" int pir_serve_set_policy(pir_server* srv, int policy) {
    if (!srv) return fail(PIR_E_INVALID, "null server");
    CW_ENTER(srv->ctx);
    if (policy != PIR_SERVE_ROUND_ROBIN && policy != PIR_SERVE_OLDEST_FIRST && policy != PIR_SERVE_SIZE_AGED)
        return fail(PIR_E_INVALID, "unknown serving policy");
    bool busy = !srv->pending.empty();
    for (const ServeSlot& sl : srv->slots) busy = busy || sl.used;
    if (busy && policy != srv->policy) return fail(PIR_E_BUSY, "the policy changes only on an idle server");
    srv->policy = policy;
    return PIR_OK;
}

extern "C" int pir_serve_set_aging(pir_server* srv, double ns_per_element) {
    if (!srv) return fail(PIR_E_INVALID, "null server");
    CW_ENTER(srv->ctx);
    if (!(ns_per_element >= 0.0) || !std::isfinite(ns_per_element))
        return fail(PIR_E_INVALID, "aging must be finite and non-negative");
    srv->aging_ns = ns_per_element;
    return PIR_OK;
}

extern "C" int pir_serve_poll(pir_server* srv, uint64_t ticket) {
    if (!srv) return fail(PIR_E_INVALID, "null server");
    pir_ctx* ctx = srv->ctx;
    CW_ENTER(ctx);
    auto it = srv->done.find(ticket);
    if (it == srv->done.end()) {
        if (srv->in_flight.count(ticket)) return 0;
        return fail(PIR_E_INVALID, "unknown or already collected ticket");
    }
    hipError_t e = hipEventQuery(it->second);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(PIR_E_DEVICE, std::string("hipEventQuery failed: ") + hipGetErrorString(e));
    }
    (void)hipEventDestroy(it->second);
    srv->done.erase(it);
    srv->in_flight.erase(ticket);
    ++srv->n_completed;
    return 1;
}

extern "C" int pir_serve_stats(pir_server* srv, uint64_t* rounds, uint64_t* admitted, uint64_t* completed,
                               uint32_t* active, uint32_t* pending) {
    if (!srv) return fail(PIR_E_INVALID, "null server");
    CW_ENTER(srv->ctx);
    if (rounds) *rounds = srv->n_rounds;
    if (admitted) *admitted = srv->n_admitted;
    if (completed) *completed = srv->n_completed;
    uint32_t a = 0;
    for (const ServeSlot& sl : srv->slots) a += sl.used ? 1 : 0;
    if (active) *active = a;
    if (pending) *pending = (uint32_t)srv->pending.size();
    return PIR_OK;
}

extern "C" void pir_serve_close(pir_server* srv) {
    if (!srv) return;
    pir_ctx* ctx = srv->ctx;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(srv->stream);
    for (ServeSlot& sl : srv->slots) dev_free(ctx, sl.buf, sl.buf_words * 8);
    for (auto& kv : srv->done) (void)hipEventDestroy(kv.second);
    for (hipEvent_t e : srv->rounds) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(srv->stream);
    (void)hipStreamDestroy(srv->check_stream);
    delete srv;
}

// ------------------------------------------------------------------------------------------------
// single FV operations
// ------------------------------------------------------------------------------------------------
extern "C" int pir_mult(pir_ctx* ctx, const uint64_t* a, const uint64_t* b_, uint64_t* out, void* stream) {
    CW_ENTER(ctx);
    if (!a || !b_ || !out) return fail(PIR_E_INVALID, "null argument");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    const size_t N = ctx->N, L = ctx->L, LL = ctx->LL;
    Launch lc = make_launch(ctx, st);
    Bufs b;
    CW_TRY(get_bufs(ctx, 1, 1, 0, b));
    uint64_t* QX;
    uint32_t* refs;
    CW_TRY(ws_get_t(ctx, "op_leaves", (size_t)2 * 2 * LL * N, &QX));
    CW_TRY(ws_get_t(ctx, "op_refs", 2, &refs));
    static const uint32_t h_refs[2] = {0, 1};
    CW_HIP(ctx, hipMemcpyAsync(refs, h_refs, 8, hipMemcpyHostToDevice, st));
    cw::launch_extend(lc, a, QX, 2);
    cw::launch_extend(lc, b_, QX + 2 * LL * N, 2);
    cw::launch_ntt_operand(lc, QX, QX, 4 * LL, LL, 0);
    cw::Batch bt{};
    bt.nq = 1;
    bt.E = 1;
    bt.leaves[0] = QX;
    cw::launch_ntt_inv_tensor(lc, refs, bt, b.X);
    cw::launch_scale(lc, b.X, out, 1);
    (void)L;
    return end_async(ctx, st);
}

extern "C" int pir_relin(pir_ctx* ctx, const pir_key* key, const uint64_t* in, uint64_t* out, void* stream) {
    CW_ENTER(ctx);
    if (!key || !in || !out) return fail(PIR_E_INVALID, "null argument");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    const uint32_t L = ctx->L;
    Launch lc = make_launch(ctx, st);
    Bufs b;
    CW_TRY(get_bufs(ctx, 1, 1, 0, b));
    cw::launch_relin(lc, in, one_query(1, nullptr, nullptr, key, out), b.R);
    cw::launch_ntt(lc, true, out, out, (size_t)2 * L, L, 0);
    return end_async(ctx, st);
}

extern "C" int pir_pm(pir_ctx* ctx, const uint64_t* ct, const uint16_t* pt, uint64_t* out, void* stream) {
    CW_ENTER(ctx);
    if (!ct || !pt || !out) return fail(PIR_E_INVALID, "null argument");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    const size_t N = ctx->N, L = ctx->L;
    Launch lc = make_launch(ctx, st);
    uint64_t *tct, *tpt;
    CW_TRY(ws_get_t(ctx, "op_ct", 2 * L * N, &tct));
    CW_TRY(ws_get_t(ctx, "op_pt", L * N, &tpt));
    cw::launch_ntt(lc, false, ct, tct, 2 * L, (uint32_t)L, 0);
    cw::launch_ntt_payload(lc, pt, tpt, 1);
    cw::launch_pointwise_pt(lc, tct, tpt, tct);
    cw::launch_ntt(lc, true, tct, out, 2 * L, (uint32_t)L, 0);
    return end_async(ctx, st);
}

// ------------------------------------------------------------------------------------------------
// codeword tables
// ------------------------------------------------------------------------------------------------
extern "C" int pir_map_perfect(pir_ctx* ctx, const uint64_t* ids, uint64_t n, uint32_t m, uint32_t k, uint32_t* out,
                               void* stream) {
    CW_ENTER(ctx);
    if (n && (!ids || !out)) return fail(PIR_E_INVALID, "null argument");
    if (k < 1 || k > 16 || m < k || m > 65535) return fail(PIR_E_INVALID, "need 1 <= k <= 16, k <= m <= 65535");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    auto key = std::make_pair(m, k);
    uint64_t* tab = nullptr;
    auto it = ctx->binom.find(key);
    if (it == ctx->binom.end()) {
        std::vector<uint64_t> T = cw::host::binom_table(m, k);
        CW_HIP(ctx, hipMalloc((void**)&tab, T.size() * 8));
        CW_HIP(ctx, hipMemcpy(tab, T.data(), T.size() * 8, hipMemcpyHostToDevice));
        ctx->binom[key] = tab;
    } else {
        tab = it->second;
    }
    cw::launch_map_perfect(st, ids, n, m, k, tab, out);
    return end_async(ctx, st);
}

extern "C" int pir_map_lossy(pir_ctx* ctx, const uint64_t* keywords, uint64_t n, uint32_t m, uint32_t k, uint64_t seed,
                             uint32_t* out, void* stream) {
    CW_ENTER(ctx);
    if (n && (!keywords || !out)) return fail(PIR_E_INVALID, "null argument");
    if (k < 1 || k > 16 || m < k || m > 65535) return fail(PIR_E_INVALID, "need 1 <= k <= 16, k <= m <= 65535");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    cw::launch_map_lossy(st, keywords, n, m, k, seed, out);
    return end_async(ctx, st);
}

// ------------------------------------------------------------------------------------------------
// profiling
// ------------------------------------------------------------------------------------------------
// Warm-up launch, then one launch timed with HIP events on `st`; `launch` enqueues the probe into
// the 8-byte-per-thread buffer `out` and returns its wave-instruction count.
template <class F>
static int run_probe(pir_ctx* ctx, hipStream_t st, uint32_t blocks, double* ms, double* wave_instr, F launch) {
    CW_TRY(begin_async(ctx, st));
    uint64_t* out;
    CW_TRY(ws_get_t(ctx, "probe", (size_t)blocks * cw::probe_threads(), &out));
    hipEvent_t e0, e1;
    CW_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(PIR_E_DEVICE, "event creation failed");
    }
    launch(out);  // warm-up
    (void)hipEventRecord(e0, st);
    const double wi = launch(out);
    (void)hipEventRecord(e1, st);
    float t = 0.f;
    const bool ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok) return fail(PIR_E_DEVICE, "probe timing failed");
    *ms = t;
    *wave_instr = wi;
    return end_async(ctx, st);
}

static int check_probe(double* ms, double* wave_instr, int op, uint32_t blocks, uint32_t iters) {
    if (!ms || !wave_instr) return fail(PIR_E_INVALID, "null argument");
    if (op < 0 || op > 3) return fail(PIR_E_INVALID, "op must lie in [0, 3]");
    if (blocks < 1 || blocks > (1u << 20) || iters < 1 || iters > (1u << 20))
        return fail(PIR_E_INVALID, "blocks and iters must lie in [1, 2^20]");
    return PIR_OK;
}

extern "C" int pir_probe_fp64(pir_ctx* ctx, int op, uint32_t blocks, uint32_t iters, double* ms,
                              double* wave_instr, void* stream) {
    CW_ENTER(ctx);
    CW_TRY(check_probe(ms, wave_instr, op, blocks, iters));
    hipStream_t st = (hipStream_t)stream;
    return run_probe(ctx, st, blocks, ms, wave_instr,
                     [&](uint64_t* out) { return cw::launch_probe_fp64(st, op, blocks, iters, (double*)out); });
}

extern "C" int pir_probe_int(pir_ctx* ctx, int op, uint32_t blocks, uint32_t iters, double* ms, double* wave_instr,
                             void* stream) {
    CW_ENTER(ctx);
    CW_TRY(check_probe(ms, wave_instr, op, blocks, iters));
    hipStream_t st = (hipStream_t)stream;
    return run_probe(ctx, st, blocks, ms, wave_instr,
                     [&](uint64_t* out) { return cw::launch_probe_int(st, op, blocks, iters, out); });
}

extern "C" int pir_profile_enable(pir_ctx* ctx, int on) {
    CW_ENTER(ctx);
    ctx->prof = on != 0;
    return PIR_OK;
}

extern "C" int pir_profile_read(pir_ctx* ctx, uint32_t max, const char** names, double* total_ms, uint64_t* launches,
                                double* work, int reset) {
    CW_ENTER(ctx);
    for (auto& r : ctx->recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto& acc = ctx->prof_acc[r.name];
            acc.ms += ms;
            acc.work += r.work;
            acc.launches += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->recs.clear();
    uint32_t i = 0;
    static std::set<std::string> keep;  // node-based: returned pointers stay valid
    for (auto& kv : ctx->prof_acc) {
        if (i < max) {
            if (names) names[i] = keep.insert(kv.first).first->c_str();
            if (total_ms) total_ms[i] = kv.second.ms;
            if (launches) launches[i] = kv.second.launches;
            if (work) work[i] = kv.second.work;
        }
        ++i;
    }
    if (reset) ctx->prof_acc.clear();
    return (int)i;
}

// ------------------------------------------------------------------------------------------------
// schedule autotuner
//
// The schedule decides how the work is cut into launches, never what is computed: elements per
// chunk, queries per selector launch, and the order of the key-switch workgroups.  pir_autotune
// times candidate schedules on synthetic inputs of the context's own parameters (uniform residues,
// uniform uint16 payload, the first n weight-k subsets in lexicographic order) and keeps the
// fastest: a grid over (chunk, query group), then the workgroup order at the best pair.
// ------------------------------------------------------------------------------------------------
namespace {
struct TuneMix {  // SplitMix64 (Steele, Lea and Flood 2014) for the tuner's synthetic inputs
    uint64_t z;
    uint64_t next() {
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        return x ^ (x >> 31);
    }
};

uint64_t binom_u64(uint32_t m, uint32_t k) {
    if (k > m) return 0;
    unsigned __int128 r = 1;
    for (uint32_t i = 1; i <= k; ++i) r = r * (m - k + i) / i;
    return r > ~0ull ? ~0ull : (uint64_t)r;
}

// rows [rows][L][N] of uniform residues mod q_j (row r uses prime r mod L)
void uniform_rows(TuneMix& g, const std::vector<uint64_t>& q, size_t rows, uint32_t N, std::vector<uint64_t>& out) {
    const size_t L = q.size();
    out.resize(rows * L * N);
    for (size_t r = 0; r < rows * L; ++r)
        for (uint32_t c = 0; c < N; ++c) out[r * N + c] = g.next() % q[r % L];
}
}  // namespace

static void schedule_of(const pir_ctx* ctx, pir_schedule* s, double ns) {
    s->chunk_elems = ctx->chunk;
    s->query_group = ctx->qb;
    s->relin_group = ctx->relin_group;
    s->ntt_shape = ctx->shape;
    s->ns_per_elem = ns;
}

// Fixup-list capacity for launches of the current schedule.
static int ensure_fix(pir_ctx* ctx) {
    const size_t need = (size_t)3 * ctx->chunk * ctx->N * ctx->qb;
    if (ctx->fix_cap >= need) return PIR_OK;
    CW_HIP(ctx, hipDeviceSynchronize());
    dev_free(ctx, ctx->dfix, ctx->fix_cap * 8);
    ctx->dfix = nullptr;
    ctx->fix_cap = 0;
    CW_TRY(dev_alloc(ctx, (void**)&ctx->dfix, need * 8));
    ctx->fix_cap = need;
    return PIR_OK;
}

static int check_schedule(const pir_ctx* ctx, const pir_schedule* s) {
    if (s->chunk_elems < 1 || s->chunk_elems > 4096) return fail(PIR_E_INVALID, "chunk_elems must be in [1, 4096]");
    if (s->query_group < 1 || s->query_group > (uint32_t)cw::MAX_QB)
        return fail(PIR_E_INVALID, "query_group must be in [1, 8]");
    if (s->relin_group > 4096) return fail(PIR_E_INVALID, "relin_group must be <= 4096");
    if (s->ntt_shape >= cw::ntt_shape_count(ctx->logN))
        return fail(PIR_E_INVALID, "ntt_shape must be below pir_ntt_shape_count");
    if (ctx->live_dbs || ctx->live_graphs)
        return fail(PIR_E_INVALID, "the schedule is fixed once a database is encoded");
    return PIR_OK;
}

extern "C" int pir_set_defer_relin(pir_ctx* ctx, int mode) {
    CW_ENTER(ctx);
    if (mode < 0 || mode > 2) return fail(PIR_E_INVALID, "mode must be 0, 1 or 2");
    if (ctx->live_dbs || ctx->live_graphs)
        return fail(PIR_E_INVALID, "the root key switch mode changes only while no database is encoded");
    ctx->defer_mode = mode;
    return PIR_OK;
}

extern "C" int pir_get_defer_relin(pir_ctx* ctx) {
    CW_ENTER(ctx);
    return ctx->defer_mode;
}

extern "C" int pir_get_schedule(pir_ctx* ctx, pir_schedule* out) {
    CW_ENTER(ctx);
    if (!out) return fail(PIR_E_INVALID, "null argument");
    schedule_of(ctx, out, 0.0);
    return PIR_OK;
}

extern "C" int pir_set_schedule(pir_ctx* ctx, const pir_schedule* s) {
    CW_ENTER(ctx);
    if (!s) return fail(PIR_E_INVALID, "null argument");
    CW_TRY(check_schedule(ctx, s));
    ctx->chunk = s->chunk_elems;
    ctx->qb = s->query_group;
    ctx->relin_group = s->relin_group;
    ctx->shape = s->ntt_shape;
    return ensure_fix(ctx);
}

extern "C" int pir_autotune(pir_ctx* ctx, uint32_t batch, uint32_t k, uint32_t s, pir_schedule* records,
                            uint32_t max_records, pir_schedule* best) {
    CW_ENTER(ctx);
    if (batch < 1 || batch > 64) return fail(PIR_E_INVALID, "batch must be in [1, 64]");
    if (k < 1 || k > PIR_MAX_K) return fail(PIR_E_INVALID, "k must be in [1, 4]");
    if (s < 1 || s > 8) return fail(PIR_E_INVALID, "s must be in [1, 8]");
    if (ctx->live_dbs || ctx->live_graphs) return fail(PIR_E_INVALID, "autotune runs before any database is encoded");
    CW_HIP(ctx, hipSetDevice(ctx->device));
    const uint32_t N = ctx->N, L = ctx->L;
    const std::vector<uint64_t> q(ctx->primes.begin(), ctx->primes.begin() + L);
    // the deferred key switch sums partial products per slice of a chunk, so fewer, longer chunks
    // save partial-sum traffic: it also tries 1024 and 2048 elements
    const bool can_defer = ctx->defer_mode && ctx->crt_ok && k >= 2;
    const std::vector<uint32_t> chunks = N >= 16384 ? std::vector<uint32_t>{32, 64, 128, 256}
                                         : can_defer ? std::vector<uint32_t>{64, 128, 256, 512, 1024, 2048}
                                                     : std::vector<uint32_t>{64, 128, 256, 512};
    // synthetic database: n elements, the first n weight-k subsets of the smallest m that has them
    const uint64_t n = k == 1 ? 256 : (uint64_t)chunks.back() * 4;
    uint32_t m = k;
    while (binom_u64(m, k) < n) ++m;
    std::vector<uint32_t> cw((size_t)n * k);
    {
        std::vector<uint32_t> c(k);
        for (uint32_t i = 0; i < k; ++i) c[i] = i;
        for (uint64_t e = 0; e < n; ++e) {
            std::memcpy(&cw[(size_t)e * k], c.data(), (size_t)k * 4);
            int i = (int)k - 1;  // next subset in lexicographic order
            while (i >= 0 && c[i] == m - k + (uint32_t)i) --i;
            if (i < 0) break;
            ++c[i];
            for (uint32_t j = (uint32_t)i + 1; j < k; ++j) c[j] = c[j - 1] + 1;
        }
    }
    TuneMix g{0x5EEDull ^ ((uint64_t)N << 32) ^ L};
    std::vector<uint16_t> pay((size_t)n * s * N);
    for (auto& x : pay) x = (uint16_t)g.next();
    std::vector<uint64_t> host;
    uniform_rows(g, q, (size_t)L * 2, N, host);
    pir_key* key = nullptr;
    CW_TRY(pir_load_key(ctx, host.data(), &key));
    const size_t qw = (size_t)m * 2 * L * N, aw = (size_t)s * 2 * L * N;
    uint64_t *dq = nullptr, *da = nullptr;
    int rc = dev_alloc(ctx, (void**)&dq, qw * 8 * batch);
    if (rc == PIR_OK) rc = dev_alloc(ctx, (void**)&da, aw * 8 * batch);
    for (uint32_t b = 0; rc == PIR_OK && b < batch; ++b) {
        uniform_rows(g, q, (size_t)m * 2, N, host);
        if (hipMemcpy(dq + b * qw, host.data(), qw * 8, hipMemcpyHostToDevice) != hipSuccess) {
            ctx->poisoned = true;
            rc = fail(PIR_E_DEVICE, "tuning input upload failed");
        }
    }
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == PIR_OK && (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                         hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
        ctx->poisoned = true;
        rc = fail(PIR_E_DEVICE, "tuning stream setup failed");
    }
    std::vector<const pir_key*> keys(batch, key);
    std::vector<const uint64_t*> qs(batch);
    std::vector<uint64_t*> as(batch);
    for (uint32_t b = 0; b < batch; ++b) {
        qs[b] = dq + b * qw;
        as[b] = da + b * aw;
    }
    const pir_schedule start{ctx->chunk, ctx->qb, ctx->relin_group, ctx->shape, 0.0};
    pir_schedule cur{ctx->chunk, 1, 0, ctx->shape, 0.0};
    pir_schedule top{0, 0, 0, 0, 0.0};
    uint32_t nrec = 0;
    pir_db* db = nullptr;
    uint32_t db_chunk = 0;
    // ns per element-query of schedule x (1 warm-up, then the better of 2 timed runs)
    auto measure = [&](const pir_schedule& x, double& ns) -> int {
        ctx->chunk = x.chunk_elems;
        ctx->qb = x.query_group;
        ctx->relin_group = x.relin_group;
        ctx->shape = x.ntt_shape;
        CW_TRY(ensure_fix(ctx));
        if (!db || db_chunk != x.chunk_elems) {  // the element plan depends on the chunk
            if (db) pir_db_free(db);
            db = nullptr;
            CW_TRY(pir_encode_db(ctx, n, s, m, k, cw.data(), pay.data(), &db));
            db_chunk = x.chunk_elems;
        }
        double bestms = 1e30;
        for (int r = 0; r < 3; ++r) {
            CW_HIP(ctx, hipEventRecord(e0, st));
            CW_TRY(answer_same_db(ctx, st, db, batch, keys.data(), qs.data(), as.data()));
            CW_HIP(ctx, hipEventRecord(e1, st));
            CW_HIP(ctx, hipEventSynchronize(e1));
            float ms = 0.f;
            CW_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
            if (r > 0) bestms = std::min(bestms, (double)ms);
        }
        ns = bestms * 1e6 / ((double)n * batch);
        return PIR_OK;
    };
    auto consider = [&](const pir_schedule& x) -> int {
        double ns = 0.0;
        const int r = measure(x, ns);
        if (r == PIR_E_NOMEM) {  // does not fit the budget: skipped
            g_err.clear();
            return PIR_OK;
        }
        CW_TRY(r);
        pir_schedule rec = x;
        rec.ns_per_elem = ns;
        if (records && nrec < max_records) records[nrec] = rec;
        ++nrec;
        if (top.chunk_elems == 0 || ns < top.ns_per_elem) top = rec;
        return PIR_OK;
    };
    // the chunk and the query group trade off (both set the rows per launch): a joint grid, then
    // the key-switch order at the best pair
    if (rc == PIR_OK) {
        for (uint32_t c : chunks) {
            for (uint32_t w : {1u, 2u, 4u, 8u}) {
                if (w > batch) continue;
                cur.chunk_elems = c;
                cur.query_group = w;
                cur.relin_group = 0;
                if ((rc = consider(cur)) != PIR_OK) break;
            }
            if (rc != PIR_OK) break;
        }
    }
    if (rc == PIR_OK && top.chunk_elems && !cw::relin_needs_staging(ctx->logN)) {
        cur = top;
        for (uint32_t G : {8u, 32u, 128u}) {  // the incumbent has G = 0
            cur.relin_group = G;
            if ((rc = consider(cur)) != PIR_OK) break;
        }
    }
    // then the transform shape at the best schedule so far (the incumbent has the starting shape)
    if (rc == PIR_OK && top.chunk_elems) {
        cur = top;
        const uint32_t incumbent = top.ntt_shape;
        for (uint32_t v = 0; v < cw::ntt_shape_count(ctx->logN); ++v) {
            if (v == incumbent) continue;
            cur.ntt_shape = v;
            if ((rc = consider(cur)) != PIR_OK) break;
        }
    }
    if (st) (void)hipStreamSynchronize(st);
    if (db) pir_db_free(db);
    pir_key_free(key);
    dev_free(ctx, dq, qw * 8 * batch);
    dev_free(ctx, da, aw * 8 * batch);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    for (auto& kv : ctx->ws) dev_free(ctx, kv.second.p, kv.second.bytes);  // sized for the largest trial
    ctx->ws.clear();
    const pir_schedule& use = (rc == PIR_OK && top.chunk_elems) ? top : start;
    ctx->chunk = use.chunk_elems;
    ctx->qb = use.query_group;
    ctx->relin_group = use.relin_group;
    ctx->shape = use.ntt_shape;
    if (rc != PIR_OK) return rc;
    if (!top.chunk_elems) return fail(PIR_E_NOMEM, "no candidate schedule fits the HBM budget");
    CW_TRY(ensure_fix(ctx));
    if (best) *best = top;
    return (int)nrec;
}

// ------------------------------------------------------------------------------------------------
// captured answers (HIP graphs)
//
// pir_graph_capture records the whole launch sequence of one pir_answer_batch call into a HIP graph
// with its own work buffers; pir_graph_launch replays it.  Every launch reads its inputs from
// device memory at run time, so a replay answers whatever the query buffers hold then.  The path
// clears its counters and accumulators with kernels, never with memset nodes.
// ------------------------------------------------------------------------------------------------
struct pir_graph {
    pir_ctx* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::map<std::string, DevBuf> ws;  // the graph's own work buffers
};

extern "C" void pir_graph_free(pir_graph* g) {
    if (!g) return;
    pir_ctx* ctx = g->ctx;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (auto& kv : g->ws) dev_free(ctx, kv.second.p, kv.second.bytes);
    --ctx->live_graphs;
    delete g;
}

extern "C" int pir_graph_capture(pir_ctx* ctx, uint32_t B, const pir_key* const* keys, const pir_db* const* dbs,
                                 const uint64_t* const* queries, uint64_t* const* answers, pir_graph** out) {
    CW_ENTER(ctx);
    if (!out || B == 0) return fail(PIR_E_INVALID, "need an output handle and B >= 1");
    *out = nullptr;
    CW_TRY(check_batch(ctx, B, keys, dbs, queries, answers));
    CW_HIP(ctx, hipSetDevice(ctx->device));
    CW_HIP(ctx, hipDeviceSynchronize());
    pir_graph* g = new pir_graph();
    g->ctx = ctx;
    ++ctx->live_graphs;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        pir_graph_free(g);
        ctx->poisoned = true;
        return fail(PIR_E_DEVICE, "stream creation failed");
    }
    const bool prof = ctx->prof;
    ctx->prof = false;
    std::swap(ctx->ws, g->ws);
    // an eager run sizes the graph's work buffers (nothing may be allocated while capturing) and
    // leaves the current queries' answers in place
    int rc = answer_dbs(ctx, st, B, keys, dbs, queries, answers);
    if (rc == PIR_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(PIR_E_DEVICE, "warm-up run failed");
    if (rc == PIR_OK) {
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(PIR_E_DEVICE, "hipStreamBeginCapture failed");
        } else {
            rc = answer_dbs(ctx, st, B, keys, dbs, queries, answers);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(st, &graph);
            g->graph = graph;
            if (rc == PIR_OK && e != hipSuccess) rc = fail(PIR_E_DEVICE, "hipStreamEndCapture failed");
            if (rc == PIR_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
                rc = fail(PIR_E_DEVICE, "hipGraphInstantiate failed");
        }
    }
    std::swap(ctx->ws, g->ws);
    ctx->prof = prof;
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (rc != PIR_OK) {
        const std::string msg = g_err;
        if (rc == PIR_E_DEVICE) ctx->poisoned = true;
        pir_graph_free(g);
        return fail(rc, msg);
    }
    *out = g;
    return PIR_OK;
}

extern "C" int pir_graph_launch(pir_graph* g, void* stream) {
    if (!g) return fail(PIR_E_INVALID, "null graph");
    pir_ctx* ctx = g->ctx;
    CW_ENTER(ctx);
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    CW_HIP(ctx, hipGraphLaunch(g->exec, st));
    return end_async(ctx, st);
}

// ------------------------------------------------------------------------------------------------
// query expansion (Section 3.3.3 "Query Expansion", Algorithm 5)
//
// Level a of c turns slots b < 2^a of every packed ciphertext into slots b and b + 2^a:
//   c0 = Sub_g(cts[b]) with g = N / 2^a + 1;  cts[b] += c0;  cts[b + 2^a] = x^(-2^a) (cts[b] - c0)
// (the same value as x^(-2^a) cts[b] - x^(-2^a) c0).  Sub_g is the automorphism followed by the key
// switch of the relinearization path: the three-polynomial input (sigma(c0), 0, sigma(c1)) under
// the Galois key, transformed back to coefficient form.  All h 2^a substitutions of a level run in
// one launch per stage.  Ciphertexts live in two ping-pong buffers.
// ------------------------------------------------------------------------------------------------
extern "C" int pir_load_galois_key(pir_ctx* ctx, uint32_t galois_elt, const uint64_t* gk, pir_key** out) {
    CW_ENTER(ctx);
    if (!out) return fail(PIR_E_INVALID, "null argument");
    *out = nullptr;
    if (galois_elt % 2 == 0 || galois_elt >= 2 * ctx->N || galois_elt == 1)
        return fail(PIR_E_INVALID, "the Galois element must be odd, in (1, 2N)");
    pir_key* key = nullptr;
    CW_TRY(pir_load_key(ctx, gk, &key));
    key->galois = galois_elt;
    *out = key;
    return PIR_OK;
}

static uint32_t inv_mod_2n(uint32_t g, uint32_t twoN) {  // g odd: g^-1 mod 2N by brute force
    for (uint32_t x = 1; x < twoN; x += 2)
        if ((uint64_t)g * x % twoN == 1) return x;
    return 0;
}

extern "C" int pir_expand(pir_ctx* ctx, const pir_key* const* gkeys, uint32_t c, const uint64_t* packed, uint32_t h,
                          uint32_t m, uint64_t* query, void* stream) {
    CW_ENTER(ctx);
    const uint32_t N = ctx->N, L = ctx->L;
    if (!packed || !query || (c && !gkeys)) return fail(PIR_E_INVALID, "null argument");
    if (c > ctx->logN) return fail(PIR_E_INVALID, "c must be at most log2 N");
    if (m == 0 || h != (m + (1u << c) - 1) >> c) return fail(PIR_E_INVALID, "need m >= 1 and h = ceil(m / 2^c)");
    for (uint32_t a = 0; a < c; ++a) {
        if (!gkeys[a] || gkeys[a]->ctx != ctx) return fail(PIR_E_INVALID, "missing Galois key or another context");
        if (gkeys[a]->galois != N / (1u << a) + 1)
            return fail(PIR_E_INVALID, "gkeys[a] must switch from x -> x^(N/2^a + 1)");
    }
    hipStream_t st = (hipStream_t)stream;
    const size_t LN = (size_t)L * N, ct = 2 * LN;
    CW_TRY(begin_async(ctx, st));
    if (c == 0) {
        CW_HIP(ctx, hipMemcpyAsync(query, packed, (size_t)m * ct * 8, hipMemcpyDeviceToDevice, st));
        return end_async(ctx, st);
    }
    const size_t slots = (size_t)h << c, Emax = (size_t)h << (c - 1);
    uint64_t *A, *B, *stage, *sub, *R = nullptr;
    CW_TRY(ws_get_t(ctx, "exp_a", slots * ct, &A));
    CW_TRY(ws_get_t(ctx, "exp_b", slots * ct, &B));
    CW_TRY(ws_get_t(ctx, "exp_stage", Emax * 3 * LN, &stage));
    CW_TRY(ws_get_t(ctx, "exp_sub", Emax * ct, &sub));
    if (cw::relin_needs_staging(ctx->logN)) CW_TRY(ws_get_t(ctx, "exp_R", Emax * (L + 2) * LN, &R));
    Launch lc = make_launch(ctx, st);
    for (uint32_t j = 0; j < h; ++j)
        CW_HIP(ctx, hipMemcpyAsync(A + ((size_t)j << c) * ct, packed + (size_t)j * ct, ct * 8, hipMemcpyDeviceToDevice, st));
    for (uint32_t a = 0; a < c; ++a) {
        const uint32_t E = h << a, g = N / (1u << a) + 1;
        {
            Prof pr(ctx, "expand", st, (double)E * 2 * LN);
            cw::launch_expand_stage(lc, A, c, a, h, inv_mod_2n(g, 2 * N), stage);
        }
        cw::Batch bt{};
        bt.nq = 1;
        bt.E = E;
        bt.rlk[0] = gkeys[a]->d;
        bt.sel[0] = sub;
        {
            Prof pr(ctx, "relin", st, bfly(ctx, (size_t)E * (L + 2) * L));
            cw::launch_relin(lc, stage, bt, R);
        }
        {
            Prof pr(ctx, "ntt_inv", st, bfly(ctx, (size_t)E * 2 * L));
            cw::launch_ntt(lc, true, sub, sub, (size_t)E * 2 * L, L, 0);
        }
        {
            Prof pr(ctx, "expand", st, (double)E * 2 * LN);
            cw::launch_expand_combine(lc, A, sub, c, a, h, B);
        }
        std::swap(A, B);
    }
    CW_HIP(ctx, hipMemcpyAsync(query, A, (size_t)m * ct * 8, hipMemcpyDeviceToDevice, st));
    return end_async(ctx, st);
}

// ------------------------------------------------------------------------------------------------
// response compression (modulus switching)
// ------------------------------------------------------------------------------------------------
static bool switch_overlap(const pir_ctx* ctx, const uint64_t* in, uint32_t count, uint32_t keep, const uint64_t* out) {
    const uintptr_t a0 = (uintptr_t)in, a1 = a0 + (size_t)count * ctx->L * ctx->N * 8;
    const uintptr_t b0 = (uintptr_t)out, b1 = b0 + (size_t)count * keep * ctx->N * 8;
    return count && a0 < b1 && b0 < a1;
}

extern "C" int pir_mod_switch(pir_ctx* ctx, const uint64_t* in, uint32_t count, uint32_t keep, uint64_t* out,
                              void* stream) {
    CW_ENTER(ctx);
    if (count && (!in || !out)) return fail(PIR_E_INVALID, "null argument");
    if (keep < 1 || keep > ctx->L) return fail(PIR_E_INVALID, "keep must be in [1, L]");
    if (switch_overlap(ctx, in, count, keep, out)) return fail(PIR_E_INVALID, "in and out must not overlap");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    cw::SwitchConst* dS = nullptr;
    CW_TRY(switch_const(ctx, keep, &dS));
    Launch lc = make_launch(ctx, st);
    const size_t N = ctx->N, per = std::max<size_t>(1, ctx->fix_cap / N);  // polynomials per launch
    Prof pr(ctx, "mod_switch", st, (double)count * N);
    for (size_t p0 = 0; p0 < count; p0 += per) {
        const size_t n = std::min<size_t>(per, count - p0);
        cw::launch_mod_switch(lc, dS, keep, in + p0 * ctx->L * N, n, out + p0 * keep * N);
    }
    return end_async(ctx, st);
}

// The same switch with the fixup counter and list in the per-device scratch array: no allocation,
// no host synchronisation, one fill kernel (the counter starts at zero) and the two switch kernels.
extern "C" int pir_mod_switch_noalloc(pir_ctx* ctx, const uint64_t* in, uint32_t count, uint32_t keep, uint64_t* out,
                                      void* stream) {
    CW_ENTER(ctx);
    if (count && (!in || !out)) return fail(PIR_E_INVALID, "null argument");
    if (keep < 1 || keep > ctx->L) return fail(PIR_E_INVALID, "keep must be in [1, L]");
    if ((uint64_t)count * ctx->N > NOALLOC_MAX_COEFFS)
        return fail(PIR_E_INVALID, "count * N exceeds the no-allocation limit of 2^19 coefficients per call");
    if (switch_overlap(ctx, in, count, keep, out)) return fail(PIR_E_INVALID, "in and out must not overlap");
    if (!count) return PIR_OK;
    if (!ctx->scratch) return fail(PIR_E_DEVICE, "no scratch array on this device: " + ctx->scratch_err);
    auto it = ctx->switches.find(keep);
    if (it == ctx->switches.end() || !it->second) return fail(PIR_E_DEVICE, "switch constants missing");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    Launch lc = make_launch(ctx, st);
    lc.fixcnt = (uint32_t*)ctx->scratch;
    lc.fix = (uint64_t*)((char*)ctx->scratch + 256);
    cw::launch_fill(st, (uint64_t*)ctx->scratch, 1, 0);  // the last call on this device may have left anything
    cw::launch_mod_switch(lc, it->second, keep, in, count, out);
    return end_async(ctx, st);
}

// ------------------------------------------------------------------------------------------------
// seeded query ciphertexts (Section 2, secret-key encryption compresses the upload)
// ------------------------------------------------------------------------------------------------
extern "C" int pir_seeded_query(pir_ctx* ctx, const uint64_t* c0, uint32_t count, uint64_t seed, uint64_t* out,
                                void* stream) {
    CW_ENTER(ctx);
    if (!count) return PIR_OK;
    if (!c0 || !out) return fail(PIR_E_INVALID, "null argument");
    const size_t total = (size_t)count * ctx->L * ctx->N;
    if (total >= (1ull << 38)) return fail(PIR_E_INVALID, "count * L * N must stay below 2^38");
    const uintptr_t a0 = (uintptr_t)c0, a1 = a0 + total * 8, b0 = (uintptr_t)out, b1 = b0 + 2 * total * 8;
    if (a0 < b1 && b0 < a1) return fail(PIR_E_INVALID, "c0 and out must not overlap");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    Prof pr(ctx, "seeded_query", st, (double)total);
    cw::launch_seeded_query(make_launch(ctx, st), c0, count, seed, out);
    return end_async(ctx, st);
}

// ------------------------------------------------------------------------------------------------
// folklore PIR leaves (Section 2.4, plain folklore operator)
// ------------------------------------------------------------------------------------------------
extern "C" int pir_folklore_leaves(pir_ctx* ctx, const uint64_t* query, uint32_t ell, uint64_t* out, void* stream) {
    CW_ENTER(ctx);
    if (ell && (!query || !out)) return fail(PIR_E_INVALID, "null argument");
    if (ell > 64) return fail(PIR_E_INVALID, "ell must be at most 64");
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    cw::launch_folklore_leaves(make_launch(ctx, st), query, ell, out);
    return end_async(ctx, st);
}

// ------------------------------------------------------------------------------------------------
// arithmetic constant-weight equality (Section 3.1, Algorithm 2), on batch-encoded ciphertexts
//
// k' = Relin(sum_i Mult(x_i, y_i)): the m products (tensor and exact rounding, in chunks) are summed
// as three-polynomial ciphertexts and key-switched once; the factors k' - i (i < k) then go through
// the product tree of the plain operator (memoised nodes, one root); the result is multiplied by
// the plaintext constant (k!)^-1 mod t.
// ------------------------------------------------------------------------------------------------
extern "C" int pir_arith_equality(pir_ctx* ctx, const pir_key* key, const uint64_t* x, const uint64_t* y, uint32_t m,
                                  uint32_t k, uint64_t* out, void* stream) {
    CW_ENTER(ctx);
    if (!key || !x || !y || !out) return fail(PIR_E_INVALID, "null argument");
    if (key->ctx != ctx || key->galois) return fail(PIR_E_INVALID, "need a relinearization key of this context");
    if (m < 1 || k < 1 || k > PIR_MAX_K || k > m) return fail(PIR_E_INVALID, "need 1 <= k <= min(m, 16)");
    uint64_t fact = 1;  // k! mod t, which must be invertible
    for (uint32_t i = 2; i <= k; ++i) fact = fact * i % ctx->t;
    if (fact == 0) return fail(PIR_E_INVALID, "k! is not invertible mod t");
    const uint64_t finv = cw::host::powmod(fact, ctx->t - 2, ctx->t);  // t prime
    hipStream_t st = (hipStream_t)stream;
    CW_TRY(begin_async(ctx, st));
    const size_t N = ctx->N, L = ctx->L, LL = ctx->LL;
    const uint32_t E = std::min<uint32_t>(m, ctx->chunk);
    Launch lc = make_launch(ctx, st);
    Bufs b;
    CW_TRY(get_bufs(ctx, E, 1, 0, b));
    uint64_t *QX, *S, *kp, *F, *FX, *sel, *nodes = nullptr;
    uint32_t* refs;
    CW_TRY(ws_get_t(ctx, "ae_qx", (size_t)2 * m * 2 * LL * N, &QX));
    CW_TRY(ws_get_t(ctx, "ae_refs", (size_t)2 * std::max<uint32_t>(E, 1), &refs));
    CW_TRY(ws_get_t(ctx, "ae_sum", 3 * L * N, &S));
    CW_TRY(ws_get_t(ctx, "ae_kp", 2 * L * N, &kp));
    CW_TRY(ws_get_t(ctx, "ae_f", (size_t)k * 2 * L * N, &F));
    CW_TRY(ws_get_t(ctx, "ae_fx", (size_t)k * 2 * LL * N, &FX));
    CW_TRY(ws_get_t(ctx, "ae_sel", (size_t)std::max<uint32_t>(E, 1) * 2 * L * N, &sel));
    // operands: x then y, extended and transformed
    CW_TRY(make_leaves(ctx, lc, x, m, QX));
    CW_TRY(make_leaves(ctx, lc, y, m, QX + (size_t)m * 2 * LL * N));
    // k' = Relin(sum of the m products)
    for (uint32_t i0 = 0; i0 < m; i0 += E) {
        const uint32_t cnt = std::min(E, m - i0);
        cw::launch_pair_refs(st, refs, cnt, i0, m + i0);
        cw::Batch bt = one_query(cnt, QX, nullptr, key, sel);
        mult_only(ctx, lc, b, refs, bt);
        cw::launch_sum_rows(lc, b.C, cnt, (uint32_t)(3 * L), i0 == 0, S);
    }
    {
        Prof pr(ctx, "relin", st, bfly(ctx, (L + 2) * L));
        cw::launch_relin(lc, S, one_query(1, QX, nullptr, key, kp), b.R);
    }
    cw::launch_ntt(lc, true, kp, kp, 2 * L, (uint32_t)L, 0);
    // prod_{i < k} (k' - i) by the plain operator's tree
    cw::launch_sub_consts(lc, kp, k, F);
    CW_TRY(make_leaves(ctx, lc, F, k, FX));
    std::vector<uint32_t> pos(k);
    for (uint32_t i = 0; i < k; ++i) pos[i] = i;
    PlanBuild pb;
    plan_elements(pos.data(), 0, 1, k, pb);
    const uint32_t np = (uint32_t)(pb.pairs.size() / 2);
    uint32_t *dpairs, *droot;
    CW_TRY(ws_get_t(ctx, "ae_pairs", std::max<size_t>(2, pb.pairs.size()), &dpairs));
    CW_TRY(ws_get_t(ctx, "ae_root", 2, &droot));
    if (np) {
        CW_TRY(ws_get_t(ctx, "ae_nodes", (size_t)np * 2 * LL * N, &nodes));
        CW_HIP(ctx, hipMemcpyAsync(dpairs, pb.pairs.data(), pb.pairs.size() * 4, hipMemcpyHostToDevice, st));
    }
    CW_HIP(ctx, hipMemcpyAsync(droot, pb.refs.data(), 8, hipMemcpyHostToDevice, st));
    if (np) make_nodes(ctx, lc, b, dpairs, pb.level_end, FX, key, sel, nodes, E);
    roots(ctx, lc, b, k, droot, one_query(1, FX, nodes, key, sel));
    cw::launch_ntt(lc, true, sel, sel, 2 * L, (uint32_t)L, 0);
    // times the plaintext constant (k!)^-1
    cw::launch_scalar_mul(lc, sel, 2, finv, out);
    CW_TRY(end_async(ctx, st));
    CW_HIP(ctx, hipStreamSynchronize(st));  // the tree plan was copied from pageable host memory
    return PIR_OK;
}
