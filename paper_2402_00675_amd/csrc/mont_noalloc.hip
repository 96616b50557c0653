// mont_batch_run_noalloc: a ragged batch (mont_batch_create + mont_batch_run
// in one call) that allocates no device memory.  The batch's constant and
// tile tables live in a fixed file-scope device array instead of
// library-owned allocations; the kernel is the ragged batch kernel, one pass
// over the tiles (one workgroup per tile, static order), the default shape of
// a batch.
//
// Host code never uses the array's name as an address: each device's copy of
// it is located once with hipGetSymbolAddress (the first call on that
// device, with the device current) and that address is what the copy and the
// kernel receive.  The tables are assembled in a static host array (no heap
// allocation either) under a mutex, copied to the device array on the
// caller's stream, and the call waits for that copy before releasing the host
// array.  Every call on one device shares its device array: calls that
// overlap on one device (other streams, other threads) race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "mont_common.hpp"
#ifdef MONT_DEBUG
#include "mont_debug.hpp"
#endif
#include "mont_ragged.hpp"

namespace mont {

// [0, 64): zero words (the ragged kernel's counter argument; unused by the
// static schedule); then nctx per-modulus constant records (64 bytes each)
// and the tile table (32 bytes per tile) from the next 16-byte boundary.  The
// host array of the same size holds these and, after them, the validated
// segments (32 bytes each), which the kernel does not read.
static __device__ __align__(256) unsigned char scratch[MONT_NOALLOC_SCRATCH_BYTES];

constexpr size_t NA_HEAD = 64;
constexpr int NA_MAX_DEV = 64;

static std::mutex g_na_mu;
static void *g_na_dev[NA_MAX_DEV];  // device address of each device's scratch copy
alignas(256) static unsigned char g_na_host[MONT_NOALLOC_SCRATCH_BYTES];

// The device address of scratch on the current device (g_na_mu held).
static mont_status_t scratch_address(void **p)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "current device");
    if (dev < 0 || dev >= NA_MAX_DEV)
        return fail(MONT_E_UNSUPPORTED, "device %d: at most %d devices", dev, NA_MAX_DEV);
    if (!g_na_dev[dev]) {
        void *q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol address");
        g_na_dev[dev] = q;
    }
    *p = g_na_dev[dev];
    return MONT_OK;
}

static size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

}  // namespace mont

using namespace mont;

extern "C" mont_status_t mont_batch_run_noalloc(const mont_ctx_t *ctxs, uint32_t nctx, const mont_seg_t *segs,
                                                uint32_t nseg, const mont_pools_t *pools, uint32_t tile_elems,
                                                void *stream)
{
    if ((nctx && !ctxs) || (nseg && !segs) || !pools)
        return fail(MONT_E_INVAL, "null table or pools");
    const uint32_t tb = tile_elems ? tile_elems : 4096;
    if (tb < 256 || tb > (1u << 20) || (tb & (tb - 1)))
        return fail(MONT_E_INVAL, "tile_elems must be 0 or a power of two in [256, 2^20]");
    const uint32_t pow_tile = 1024;
    for (uint32_t i = 0; i < nctx; ++i)
        if (mont_status_t rc = check_ctx(&ctxs[i]))
            return fail(rc, "context %u: %s", i, mont_last_error());
    // sizes first, before any device use: everything must fit the scratch array
    uint64_t ntiles = 0;
    for (uint32_t i = 0; i < nseg; ++i) {
        const mont_seg_t &sg = segs[i];
        if (sg.ctx >= nctx || sg.op > MONT_OP_POW)
            return fail(MONT_E_INVAL, "segment %u: context index or op out of range", i);
        const int wc = width_class(ctxs[sg.ctx].w);
        const uint64_t te = seg_tile_elems(tb, pow_tile, (uint32_t)wc, sg.op);
        if (sg.n >= (1ull << 40))
            return fail(MONT_E_INVAL, "segment %u: size too large", i);
        ntiles += (sg.n + te - 1) / te;
    }
    // device tables [0, need): head, constants, tiles; the validated segments
    // follow them in the host array only
    const size_t o_ctx = NA_HEAD;
    const size_t o_tile = align16(o_ctx + (size_t)nctx * sizeof(KCtx));
    const uint64_t need = o_tile + ntiles * sizeof(DTile);
    const uint64_t o_seg = align16(need);
    if (o_seg + (uint64_t)nseg * sizeof(DSeg) > MONT_NOALLOC_SCRATCH_BYTES)
        return fail(MONT_E_INVAL,
                    "batch tables need %llu bytes (%u contexts, %u segments, %llu tiles of %u elements): more than "
                    "the %u-byte scratch array; use a larger tile_elems or mont_batch_create",
                    (unsigned long long)(o_seg + (uint64_t)nseg * sizeof(DSeg)), nctx, nseg,
                    (unsigned long long)ntiles, tb,
                    (unsigned)MONT_NOALLOC_SCRATCH_BYTES);
    if (ntiles == 0)
        return MONT_OK;
    hipStream_t s = (hipStream_t)stream;

    std::lock_guard<std::mutex> g(g_na_mu);
    std::memset(g_na_host, 0, NA_HEAD);
    KCtx *hc = reinterpret_cast<KCtx *>(g_na_host + o_ctx);
    for (uint32_t i = 0; i < nctx; ++i)
        hc[i] = to_kctx(ctxs[i]);
    DSeg *hs = reinterpret_cast<DSeg *>(g_na_host + o_seg);
    for (uint32_t i = 0; i < nseg; ++i) {
        if (mont_status_t rc = make_dseg(ctxs, nctx, segs[i], i, hs[i]))
            return rc;
    }
    // pool checks, as mont_batch_run makes them
    for (uint32_t i = 0; i < nseg; ++i) {
        const uint32_t wc = hs[i].wc;
        if (segs[i].n && (!pools->in0[wc] || !pools->out[wc] || (segs[i].op != MONT_OP_REDC && !pools->in1[wc])))
            return fail(MONT_E_INVAL, "segment %u: pool for width class %u is NULL", i, wc);
    }
    for (int wc = 0; wc < 3; ++wc)
        if (((uintptr_t)pools->in0[wc] | (uintptr_t)pools->in1[wc] | (uintptr_t)pools->out[wc]) & 15u)
            return fail(MONT_E_INVAL, "pool pointers must be 16-byte aligned");
    // Tile table in the order a batch uses: exponentiation tiles first, then the
    // streaming tiles grouped by (width class, operation, variant), segment order
    // inside a group; with a tile count that is a multiple of 8, logical tile
    // 8p + x is stored at x (ntiles / 8) + p (the XCD-renumbered one-pass grid
    // then visits the logical order).
    DTile *ht = reinterpret_cast<DTile *>(g_na_host + o_tile);
    const bool perm = ntiles % 8 == 0;
    const uint64_t c8 = ntiles / 8;
    uint64_t L = 0;
    auto put = [&](uint32_t seg, uint64_t start, uint32_t cnt) {
        const uint64_t pos = perm ? (L % 8) * c8 + L / 8 : L;
        ht[pos] = make_tile(hs[seg], start, cnt);
        ++L;
    };
    auto cut = [&](uint32_t i) {
        const uint64_t te = seg_tile_elems(tb, pow_tile, hs[i].wc, segs[i].op);
        for (uint64_t st = 0; st < segs[i].n; st += te)
            put(i, st, (uint32_t)std::min<uint64_t>(te, segs[i].n - st));
    };
    for (uint32_t i = 0; i < nseg; ++i)
        if (segs[i].op == MONT_OP_POW)
            cut(i);
    for (uint32_t wc = 0; wc < 3; ++wc)
        for (uint32_t op = 0; op < 2; ++op)
            for (uint32_t v = 0; v < (uint32_t)NVARIANT; ++v)
                for (uint32_t i = 0; i < nseg; ++i)
                    if (hs[i].wc == wc && segs[i].op == op && segs[i].variant == v)
                        cut(i);
    if (L != ntiles)
        return fail(MONT_E_INVAL, "internal: tile count %llu != %llu", (unsigned long long)L,
                    (unsigned long long)ntiles);
#ifdef MONT_DEBUG
    for (uint32_t i = 0; i < nseg; ++i) {
        const mont_seg_t &sg = segs[i];
        const mont_ctx_t &c = ctxs[sg.ctx];
        const size_t es = c.w / 8;
        const uint32_t wc = hs[i].wc;
        const char *i0 = (const char *)pools->in0[wc], *i1 = (const char *)pools->in1[wc];
        hipError_t de;
        if (sg.op == MONT_OP_MUL)
            de = debug_check(DBG_PRODUCT, c, sg.variant, i0 + sg.off * es, i1 + sg.off1 * es, 0, sg.n, s);
        else if (sg.op == MONT_OP_REDC)
            de = debug_check(DBG_T, c, sg.variant, i0 + sg.off * 2 * es, nullptr, 0, sg.n, s);
        else
            de = debug_check(DBG_BELOW_N, c, CLASSIC, i0 + sg.off * es, nullptr, 0, sg.n, s);
        if (de != hipSuccess)
            return hip_fail(de, "precondition check");
    }
#endif
    void *base = nullptr;
    if (mont_status_t rc = scratch_address(&base))
        return rc;
    hipError_t e = hipMemcpyAsync(base, g_na_host, (size_t)need, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // the host tables are reused by the next call
    if (e != hipSuccess)
        return hip_fail(e, "scratch table upload");
    DPools P;
    for (int i = 0; i < 3; ++i) {
        P.in0[i] = pools->in0[i];
        P.in1[i] = pools->in1[i];
        P.out[i] = pools->out[i];
    }
    unsigned char *d = static_cast<unsigned char *>(base);
    e = launch_ragged(reinterpret_cast<const KCtx *>(d + o_ctx), reinterpret_cast<const DTile *>(d + o_tile),
                      (uint32_t)ntiles, P, reinterpret_cast<uint32_t *>(d), 0u, (uint32_t)ntiles, true, s);
    return e == hipSuccess ? MONT_OK : hip_fail(e, "ragged launch");
}
