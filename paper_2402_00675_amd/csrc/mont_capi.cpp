// C ABI: per-modulus setup, argument checking and launches of the streaming,
// exponentiation and range kernels.  See include/mont.h for the contract.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <chrono>
#include <mutex>
#include <string>

#include "../../include/mont.h"
#include "mont_common.hpp"
#ifdef MONT_DEBUG
#include "mont_debug.hpp"
#endif
#include "mont_kernels.hpp"

namespace mont {

// ------------------------------------------------------------ error text

static thread_local std::string g_err;

mont_status_t fail(mont_status_t code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    log_msg(1, "error %d: %s", (int)code, buf);
    return code;
}

int log_level()
{
    const char *v = std::getenv("MONT_LOG");
    if (!v || !*v)
        return 0;
    if (!std::strcmp(v, "error"))
        return 1;
    if (!std::strcmp(v, "info"))
        return 2;
    if (!std::strcmp(v, "debug"))
        return 3;
    return std::atoi(v);
}

void log_msg(int level, const char *fmt, ...)
{
    if (log_level() < level)
        return;
    char buf[640];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[mont %s] %s\n", level <= 1 ? "error" : level == 2 ? "info" : "debug", buf);
}

int tune_override()
{
    const char *v = std::getenv("MONT_TUNE");
    if (!v || !*v)
        return -1;
    return std::atoi(v) != 0 ? 1 : 0;
}

mont_status_t hip_fail(hipError_t e, const char *what)
{
    return fail(MONT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int device_cus()
{
    static std::atomic<int> cus[64];  // per device, 0 until first asked (static storage: zero-initialised)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 256;
    int v = cus[dev].load(std::memory_order_relaxed);
    if (!v) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

KCtx to_kctx(const mont_ctx_t &c)
{
    KCtx k;
    k.N = c.N;
    k.nprime = c.nprime;
    k.ninv = c.ninv;
    k.n2lo = c.ninv2_lo;
    k.n2hi = c.ninv2_hi;
    k.r2 = c.r2_mod_n;
    k.rmodn = c.r_mod_n;
    k.alpha = c.alpha;
    k.w = c.w;
    return k;
}

int width_class(uint32_t w) { return w == 16 ? 0 : w == 32 ? 1 : w == 64 ? 2 : -1; }

// ------------------------------------------------------- launch shapes

static std::mutex g_launch_mu;
static Launch g_launch[3][3][NVARIANT];  // [op][width class][variant]
static bool g_launch_init = false;

static void launch_defaults()
{
    if (g_launch_init)
        return;
    for (auto &a : g_launch)
        for (auto &b : a)
            for (auto &l : b)
                l = Launch{};
    // exponentiation (op 2) keeps the default of one element per lane: with
    // 4-bit window tables in LDS (16 entries per element) more workgroups
    // then fit on a CU, and on MI355X (2^22 elements, clocks at steady state)
    // one element per lane measured 7 % faster than two at 64 bits and 1 %
    // at 32 bits; four were 11-30 % slower
    g_launch_init = true;
}

Launch get_launch(int op, int wc, int variant)
{
    std::lock_guard<std::mutex> g(g_launch_mu);
    launch_defaults();
    return g_launch[op][wc][variant];
}

void set_launch(int op, int wc, int variant, const Launch &l)
{
    std::lock_guard<std::mutex> g(g_launch_mu);
    launch_defaults();
    g_launch[op][wc][variant] = l;
}

// -------------------------------------------------------------- checks

mont_status_t check_ctx(const mont_ctx_t *ctx)
{
    if (!ctx)
        return fail(MONT_E_INVAL, "null context");
    if (width_class(ctx->w) < 0 || ctx->N < 3 || !(ctx->N & 1u) || (ctx->w < 64 && (ctx->N >> ctx->w)))
        return fail(MONT_E_INVAL, "context not initialised by mont_setup");
    return MONT_OK;
}

mont_status_t check_variant(const mont_ctx_t *ctx, int variant)
{
    if (variant < 0 || variant >= NVARIANT)
        return fail(MONT_E_INVAL, "unknown variant %d", variant);
    if (!(ctx->valid & (1u << variant)))
        return fail(MONT_E_DOMAIN, "variant %d is not valid for N=%llu at w=%u", variant,
                    (unsigned long long)ctx->N, ctx->w);
    if (variant == SIGNED_PLANTARD_ALPHA && ctx->alpha < 1)
        return fail(MONT_E_DOMAIN, "Algorithm 4 needs alpha >= 1");
    return MONT_OK;
}

}  // namespace mont

using namespace mont;

// ===================================================================== ABI

extern "C" {

const char *mont_last_error(void) { return g_err.c_str(); }

uint32_t mont_version(void) { return (1u << 16) | 3u; }

mont_status_t mont_setup(uint64_t N, uint32_t log2R, mont_ctx_t *ctx) { return setup_ctx(N, log2R, ctx); }

mont_status_t mont_set_alpha(mont_ctx_t *ctx, uint32_t alpha)
{
    mont_status_t rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (alpha < 1)
        return fail(MONT_E_DOMAIN, "alpha = 0 makes Algorithm 4 incorrect (Example 3.1)");
    if (alpha + 2 > ctx->w || (ctx->N >> (ctx->w - alpha - 1)) != 0)
        return fail(MONT_E_DOMAIN, "Algorithm 4 needs N < 2^(w - alpha - 1)");
    ctx->alpha = alpha;
    ctx->valid |= 1u << SIGNED_PLANTARD_ALPHA;
    return MONT_OK;
}

static mont_status_t run_map(int op, const mont_ctx_t *ctxs, uint32_t rows, const void *in0, const void *in1,
                             void *out, size_t n, size_t ld, mont_variant_t variant, void *stream,
                             const KConst *kc = nullptr)
{
    for (uint32_t r = 0; r < rows; ++r) {
        mont_status_t rc = check_ctx(&ctxs[r]);
        if (rc)
            return rc;
        if (ctxs[r].w != ctxs[0].w)
            return fail(MONT_E_INVAL, "all residue rows must share one word size");
        rc = check_variant(&ctxs[r], variant);
        if (rc)
            return rc;
    }
    if (n == 0)
        return MONT_OK;
    if (!in0 || !out || (op == 0 && !in1))
        return fail(MONT_E_INVAL, "null data pointer");
    const int op_launch = op == 2 ? 0 : op;  // the fixed-operand product shares the product's launch shape
    KCtx k[MAX_ROWS];
    for (uint32_t r = 0; r < rows; ++r)
        k[r] = to_kctx(ctxs[r]);
    MapArgs a;
    a.op = op;
    a.variant = variant;
    a.rows = (int)rows;
    a.ctx = k;
    a.in0 = in0;
    a.in1 = in1;
    a.out = out;
    a.n = n;
    a.ld = ld;
    if (kc)
        a.kc = *kc;
    const int wc = width_class(ctxs[0].w);
    const Launch L = get_launch(op_launch, wc, variant);
    hipStream_t s = (hipStream_t)stream;
#ifdef MONT_DEBUG
    {
        const uint32_t w = ctxs[0].w;
        const size_t es = w / 8;
        const uint64_t mask = w == 64 ? ~0ull : (1ull << w) - 1;
        for (uint32_t r = 0; r < rows; ++r) {
            const char *p0 = (const char *)in0 + (size_t)r * ld * es * (op == 1 ? 2 : 1);
            const char *p1 = in1 ? (const char *)in1 + (size_t)r * ld * es : nullptr;
            const int kind = op == 0 ? DBG_PRODUCT : op == 1 ? DBG_T : DBG_CONST;
            const hipError_t de = debug_check(kind, ctxs[r], variant, p0, p1, kc ? kc->b & mask : 0, n, s);
            if (de != hipSuccess)
                return hip_fail(de, "precondition check");
        }
    }
#endif
    hipError_t e = wc == 0 ? launch_map<16>(a, L, s) : wc == 1 ? launch_map<32>(a, L, s) : launch_map<64>(a, L, s);
    if (e != hipSuccess)
        return hip_fail(e, op == 1 ? "mont_redc launch" : "mont_mul launch");
    return MONT_OK;
}

mont_status_t mont_redc(const mont_ctx_t *ctx, const void *T, void *out, size_t n, mont_variant_t variant,
                        void *stream)
{
    return run_map(1, ctx, 1, T, nullptr, out, n, n, variant, stream);
}

mont_status_t mont_mul(const mont_ctx_t *ctx, const void *a, const void *b, void *out, size_t n,
                       mont_variant_t variant, void *stream)
{
    return run_map(0, ctx, 1, a, b, out, n, n, variant, stream);
}

mont_status_t mont_mul_const(const mont_ctx_t *ctx, const void *a, uint64_t b, void *out, size_t n,
                             mont_variant_t variant, void *stream)
{
    mont_status_t rc = check_ctx(ctx);
    if (rc)
        return rc;
    rc = check_variant(ctx, variant);
    if (rc)
        return rc;
    typedef unsigned __int128 u128;
    const uint32_t w = ctx->w;
    const u128 one = 1;
    const uint64_t maskw = w == 64 ? ~0ull : (1ull << w) - 1;
    const bool sgn = variant == MONT_SIGNED || variant == MONT_SIGNED_PLANTARD || variant == MONT_SIGNED_PLANTARD_ALPHA;
    // b as a w-bit value: [0, N) for the unsigned variants, |b| < N (two's complement) for the signed ones
    const uint64_t bw = b & maskw;
    int64_t bs = (int64_t)bw;
    if (sgn && w < 64 && (bw >> (w - 1)))
        bs = (int64_t)(bw | ~maskw);
    if (sgn ? (bs < 0 ? (uint64_t)(-bs) : (uint64_t)bs) >= ctx->N : bw >= ctx->N)
        return fail(MONT_E_DOMAIN, "fixed operand outside the variant's operand range");
    KConst k;
    k.b = sgn ? (uint64_t)bs : bw;
    if (variant == MONT_CLASSIC) {
        k.b1 = (uint64_t)(((u128)bw * ctx->nprime) & maskw);
        k.b2 = 0;
    } else if (variant == MONT_SIGNED) {
        k.b1 = (uint64_t)(((u128)bw * ctx->ninv) & maskw);
        k.b2 = 0;
    } else {
        // b' = b N^{-1} mod 2^(2w), b sign-extended to 2w bits for the signed forms
        const u128 bx = sgn ? (u128)(__int128)bs : (u128)bw;
        const u128 ninv2 = ((u128)ctx->ninv2_hi << 64) | ctx->ninv2_lo;
        u128 bp = bx * ninv2;
        if (w < 64)
            bp &= (one << (2 * w)) - 1;
        k.b1 = (uint64_t)bp;  // the whole 2w-bit value for w <= 32, its low word for w = 64
        k.b2 = w == 64 ? (uint64_t)(bp >> 64) : 0;
    }
    return run_map(2, ctx, 1, a, nullptr, out, n, n, variant, stream, &k);
}

mont_status_t mont_mul_rns(const mont_ctx_t *ctxs, uint32_t k, const void *a, const void *b, void *out, size_t n,
                           size_t ld, mont_variant_t variant, void *stream)
{
    if (!ctxs || k < 1 || k > MONT_RNS_MAX)
        return fail(MONT_E_INVAL, "need 1 <= k <= %d contexts", MONT_RNS_MAX);
    if (n > ld)
        return fail(MONT_E_INVAL, "n > ld");
    return run_map(0, ctxs, k, a, b, out, n, ld, variant, stream);
}

mont_status_t mont_pow(const mont_ctx_t *ctx, const void *x, const uint64_t *e, void *out, size_t n, void *stream)
{
    mont_status_t rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (n == 0)
        return MONT_OK;
    if (!x || !e || !out)
        return fail(MONT_E_INVAL, "null data pointer");
    const KCtx k = to_kctx(*ctx);
    const int wc = width_class(ctx->w);
    const Launch L = get_launch(2, wc, CLASSIC);
    hipStream_t s = (hipStream_t)stream;
#ifdef MONT_DEBUG
    if (const hipError_t de = debug_check(DBG_BELOW_N, *ctx, CLASSIC, x, nullptr, 0, n, s))
        return hip_fail(de, "precondition check");
#endif
    hipError_t err = wc == 0   ? launch_pow<16>(k, x, e, out, n, L.unroll, L.blocks_per_cu, s)
                     : wc == 1 ? launch_pow<32>(k, x, e, out, n, L.unroll, L.blocks_per_cu, s)
                               : launch_pow<64>(k, x, e, out, n, L.unroll, L.blocks_per_cu, s);
    if (err != hipSuccess)
        return hip_fail(err, "mont_pow launch");
    return MONT_OK;
}

mont_status_t mont_redc_range(const mont_ctx_t *ctx, uint64_t T0, void *out, size_t n, mont_variant_t variant,
                              void *stream)
{
    mont_status_t rc = check_ctx(ctx);
    if (rc)
        return rc;
    rc = check_variant(ctx, variant);
    if (rc)
        return rc;
    if (variant != MONT_CLASSIC && variant != MONT_PLANTARD)
        return fail(MONT_E_UNSUPPORTED, "mont_redc_range covers the unsigned variants");
    if (ctx->w == 64)
        return fail(MONT_E_UNSUPPORTED, "mont_redc_range covers w = 16 and 32");
    if (n == 0)
        return MONT_OK;
    // the last T must stay in the Require range: T < R N (classic), T <= N^2 (Plantard)
    const unsigned __int128 last = (unsigned __int128)T0 + n - 1;
    const unsigned __int128 lim = variant == MONT_CLASSIC ? ((unsigned __int128)ctx->N << ctx->w) - 1
                                                          : (unsigned __int128)ctx->N * ctx->N;
    if (last > lim)
        return fail(MONT_E_DOMAIN, "range leaves the variant's input range");
    if (!out)
        return fail(MONT_E_INVAL, "null output");
    const KCtx k = to_kctx(*ctx);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = ctx->w == 16 ? launch_range<16>(k, variant, T0, out, n, s)
                                : launch_range<32>(k, variant, T0, out, n, s);
    if (e != hipSuccess)
        return hip_fail(e, "mont_redc_range launch");
    return MONT_OK;
}

mont_status_t mont_set_launch(uint32_t op, uint32_t w, mont_variant_t variant, const mont_launch_t *l)
{
    const int wc = width_class(w);
    if (op > 2 || wc < 0 || (int)variant < 0 || (int)variant >= NVARIANT || !l)
        return fail(MONT_E_INVAL, "bad launch key");
    if (l->unroll != 1 && l->unroll != 2 && l->unroll != 4)
        return fail(MONT_E_INVAL, "unroll must be 1, 2 or 4");
    if (l->block != 64 && l->block != 256)
        return fail(MONT_E_INVAL, "block must be 64 or 256");
    Launch L;
    L.unroll = (int)l->unroll;
    L.nontemporal = l->nontemporal ? 1 : 0;
    L.blocks_per_cu = (int)l->blocks_per_cu;
    L.block = (int)l->block;
    set_launch((int)op, wc, (int)variant, L);
    return MONT_OK;
}

mont_status_t mont_get_launch(uint32_t op, uint32_t w, mont_variant_t variant, mont_launch_t *l)
{
    const int wc = width_class(w);
    if (op > 2 || wc < 0 || (int)variant < 0 || (int)variant >= NVARIANT || !l)
        return fail(MONT_E_INVAL, "bad launch key");
    const Launch L = get_launch((int)op, wc, (int)variant);
    l->unroll = (uint32_t)L.unroll;
    l->nontemporal = (uint32_t)L.nontemporal;
    l->blocks_per_cu = (uint32_t)L.blocks_per_cu;
    l->block = (uint32_t)L.block;
    return MONT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuning

namespace mont {

static std::string mul_tune_key(uint32_t w, int variant, size_t n)
{
    int lg = 0;
    while ((n >> lg) > 1)
        ++lg;
    char k[96];
    snprintf(k, sizeof k, "mul:w%u:v%d:log2n%d", w, variant, lg);
    return tune_key_prefix() + k;
}

}  // namespace mont

extern "C" mont_status_t mont_tune_mul(const mont_ctx_t *ctx, const void *a, const void *b, void *out, size_t n,
                                       mont_variant_t variant, mont_launch_t *best, void *stream)
{
    mont_status_t rc = check_ctx(ctx);
    if (rc)
        return rc;
    rc = check_variant(ctx, variant);
    if (rc)
        return rc;
    if (n == 0 || !a || !b || !out)
        return fail(MONT_E_INVAL, "tuning needs non-empty device buffers");
    hipStream_t s = (hipStream_t)stream;
    const int wc = width_class(ctx->w);
    const std::string key = mul_tune_key(ctx->w, variant, n);
    const Launch saved = get_launch(0, wc, variant);
    Launch bestL = saved;
    TuneRecord rec;
    if (tune_override() == 0) {
        // tuning switched off: the current shape computes the product
        log_msg(2, "mul tune: %s: MONT_TUNE=0, current shape kept", key.c_str());
    } else if (tune_lookup(key, rec) && rec.count("unroll") && rec.count("nontemporal") && rec.count("blocks_per_cu")) {
        // a shape tuned earlier for this device, library version, width, variant and size class
        bestL.unroll = (int)rec["unroll"];
        bestL.nontemporal = (int)rec["nontemporal"];
        bestL.blocks_per_cu = (int)rec["blocks_per_cu"];
        bestL.block = rec.count("block") ? (int)rec["block"] : BLOCK;
        if ((bestL.unroll != 1 && bestL.unroll != 2 && bestL.unroll != 4) || (bestL.block != 64 && bestL.block != 256))
            bestL = saved;
        set_launch(0, wc, variant, bestL);
        log_msg(2, "mul tune: %s: cached shape unroll %d, nt %d, %d workgroups/CU, block %d", key.c_str(),
                bestL.unroll, bestL.nontemporal, bestL.blocks_per_cu, bestL.block);
    } else {
        // Candidates write a library-owned buffer: a and b are only read, so an
        // in-place call (out == a or out == b) is exact.
        void *scratch = nullptr;
        if (hipMalloc(&scratch, n * (ctx->w / 8)) != hipSuccess)
            return fail(MONT_E_NOMEM, "tuning output of %zu elements", n);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0)
                (void)hipEventDestroy(e0);
            (void)hipFree(scratch);
            return fail(MONT_E_DEVICE, "event create");
        }
        float best_ms = 1e30f;
        const int unrolls[] = {1, 2, 4};
        const int bpcs[] = {0, 4, 8, 16};
        const int blocks[] = {64, 256};
        // clocks to their loaded state first (about 25 ms of the current shape)
        {
            const auto t0 = std::chrono::steady_clock::now();
            do {
                for (int r = 0; r < 4 && !rc; ++r)
                    rc = mont_mul(ctx, a, b, scratch, n, variant, stream);
                if (!rc && hipStreamSynchronize(s) != hipSuccess)
                    rc = fail(MONT_E_DEVICE, "tuning warm-up failed");
            } while (!rc && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(25));
        }
        // every candidate shape: workgroup size x unroll x non-temporal x workgroups per CU; the first
        // failure ends the sweep
        for (int c = 0; c < 2 * 3 * 2 * 4 && !rc; ++c) {
            Launch L;
            L.block = blocks[c / 24];
            L.unroll = unrolls[(c / 8) % 3];
            L.nontemporal = (c / 4) % 2;
            L.blocks_per_cu = bpcs[c % 4];
            set_launch(0, wc, variant, L);
            rc = mont_mul(ctx, a, b, scratch, n, variant, stream);  // warm
            if (!rc && hipEventRecord(e0, s) != hipSuccess)
                rc = fail(MONT_E_DEVICE, "event record");
            for (int r = 0; r < 5 && !rc; ++r)
                rc = mont_mul(ctx, a, b, scratch, n, variant, stream);
            if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = fail(MONT_E_DEVICE, "tuning run failed");
            if (rc)
                break;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) {
                best_ms = ms;
                bestL = L;
            }
        }
        if (hipStreamSynchronize(s) != hipSuccess && !rc)
            rc = fail(MONT_E_DEVICE, "tuning runs failed");
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipFree(scratch);
        set_launch(0, wc, variant, rc ? saved : bestL);
        if (rc)
            return rc;
        log_msg(2, "mul tune: %s: unroll %d, nt %d, %d workgroups/CU, block %d (%.4f ms per call)", key.c_str(),
                bestL.unroll, bestL.nontemporal, bestL.blocks_per_cu, bestL.block, best_ms / 5);
        tune_store(key, {{"unroll", (double)bestL.unroll},
                         {"nontemporal", (double)bestL.nontemporal},
                         {"blocks_per_cu", (double)bestL.blocks_per_cu},
                         {"block", (double)bestL.block},
                         {"ms", best_ms / 5}});
    }
    if (best) {
        best->unroll = (uint32_t)bestL.unroll;
        best->nontemporal = (uint32_t)bestL.nontemporal;
        best->blocks_per_cu = (uint32_t)bestL.blocks_per_cu;
        best->block = (uint32_t)bestL.block;
    }
    // the caller's out receives one product with the chosen shape
    return mont_mul(ctx, a, b, out, n, variant, stream);
}

#ifndef MONT_DEBUG
// The release library keeps no precondition counters (mont_debug.hip, built
// into the MONT_DEBUG library only, does).
extern "C" mont_status_t mont_debug_violations(uint64_t *count, int reset)
{
    (void)reset;
    if (count)
        *count = 0;
    return fail(MONT_E_UNSUPPORTED, "library built without MONT_DEBUG: load libmont_debug.so to count violations");
}
#endif
