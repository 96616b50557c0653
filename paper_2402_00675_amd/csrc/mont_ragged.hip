// Ragged batches: thousands of independent vectors, each with its own
// modulus, word size, length and operation, in ONE persistent launch.
//
// Host side: every segment is cut into tiles (equal output bytes for the
// streaming ops, a fixed element count for exponentiation); a table of
// per-modulus constants and a tile table {pool offsets, count, constants
// index, op, variant, width} are uploaded once.  Device side: one workgroup
// per tile (one pass), or a persistent grid (a multiple of the CU count) that
// walks the tile table round-robin (static) or through atomic tile counters
// (dynamic: one counter, or one per XCD; the last workgroup to finish resets
// them, so a replay needs no memset), fetching the next tile's record (or claiming it) while
// the current one runs.  The tile's record is wave-uniform, so it is fetched
// with scalar loads and its constants stay in SGPRs; the op / word size /
// variant switch is a uniform branch.
//
// Launches can be replayed from a hipGraph whose kernel node is updated in
// place when the caller's pool pointers change.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "mont_common.hpp"
#ifdef MONT_DEBUG
#include "mont_debug.hpp"
#endif
#include "mont_ragged.hpp"

namespace mont {

constexpr int RAGGED_U = 4;  // 16-byte chunks in flight per lane

template <int W>
struct WC {
    static constexpr int v = W == 16 ? 0 : W == 32 ? 1 : 2;
};

template <int W, int V, int OP, bool NT, int BS>
__device__ __forceinline__ void tile_map(const KCtx &c, const DPools &P, uint64_t g0, uint64_t g1, uint32_t cnt)
{
    using R = Red<W, V>;
    using El = typename R::E;
    using TT = typename R::TT;
    constexpr int E = 16 / (int)sizeof(El);
    constexpr int wc = WC<W>::v;
    const R red(c);
    const El *pa = (const El *)P.in0[wc];
    // indexed by g like pa; (g1 - g0) is a multiple of E so 16-byte chunks stay aligned
    const El *pb = (const El *)P.in1[wc] + (int64_t)(g1 - g0);
    const TT *pt = (const TT *)P.in0[wc];
    El *po = (El *)P.out[wc];

    // Element-wise head: up to the next 128-byte line of out when every
    // operand reaches a line boundary at the same element (pools at one
    // phase), so no 16-byte chunk of the body straddles two lines; else up to
    // the next 16-byte chunk.  Wave-uniform scalar arithmetic.
    uint32_t h = (E - g0 % E) % E;
    {
        constexpr uint32_t s0 = OP == 0 ? sizeof(El) : sizeof(TT);
        const uintptr_t ao = (uintptr_t)(po + g0);
        const uint32_t hl = (uint32_t)(((128 - (ao & 127)) & 127) / sizeof(El));
        const bool in_line = OP == 0 ? ((uintptr_t)(pa + g0) + hl * s0) % 128 == 0 &&
                                           ((uintptr_t)(pb + g0) + hl * sizeof(El)) % 128 == 0
                                     : ((uintptr_t)(pt + g0) + hl * s0) % 128 == 0;
        if (in_line)
            h = hl;
    }
    const uint32_t head = std::min(cnt, h);
    if (threadIdx.x < head) {
        const uint64_t g = g0 + threadIdx.x;
        if constexpr (OP == 0)
            po[g] = red.mul(pa[g], pb[g]);
        else
            po[g] = red.redc(pt[g]);
    }
    const uint64_t gv = g0 + head;  // multiple of E: 16-byte aligned for aligned pools
    const uint32_t rest = cnt - head;
    const uint32_t nv = rest / E;
    for (uint32_t c0 = threadIdx.x; c0 < nv; c0 += BS * RAGGED_U) {
        El a[RAGGED_U][E], b[RAGGED_U][E];
        TT t[RAGGED_U][E];
#pragma unroll
        for (int u = 0; u < RAGGED_U; ++u) {
            const uint32_t ci = c0 + u * BS;
            if (ci < nv) {
                const uint64_t g = gv + (uint64_t)ci * E;
                if constexpr (OP == 0) {
                    load_chunk<El, E, NT>(pa + g, a[u]);
                    load_chunk<El, E, NT>(pb + g, b[u]);
                } else {
                    load_chunk<TT, E, NT>(pt + g, t[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < RAGGED_U; ++u) {
            const uint32_t ci = c0 + u * BS;
            if (ci < nv) {
                El o[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if constexpr (OP == 0)
                        o[e] = red.mul(a[u][e], b[u][e]);
                    else
                        o[e] = red.redc(t[u][e]);
                }
                store_chunk<El, E, NT>(po + gv + (uint64_t)ci * E, o);
            }
        }
    }
    const uint32_t tail = rest - nv * E;
    if (threadIdx.x < tail) {
        const uint64_t g = gv + (uint64_t)nv * E + threadIdx.x;
        if constexpr (OP == 0)
            po[g] = red.mul(pa[g], pb[g]);
        else
            po[g] = red.redc(pt[g]);
    }
}

template <int W, int BS>
__device__ __forceinline__ void tile_pow(const KCtx &c, const DPools &P, uint64_t g0, uint64_t g1, uint32_t cnt)
{
    using R = Red<W, CLASSIC>;
    using El = typename R::E;
    constexpr int wc = WC<W>::v;
    const R red(c);
    const El r2 = (El)c.r2, one = (El)c.rmodn;
    const El *px = (const El *)P.in0[wc];
    const uint64_t *pe = (const uint64_t *)P.in1[wc] + (int64_t)(g1 - g0);
    El *po = (El *)P.out[wc];
    __shared__ El tab[4 * BS];
    El *const mine = tab + threadIdx.x;
    const int mode = ladder_mode<W>(c.N);  // wave-uniform
    for (uint32_t i = threadIdx.x; i < cnt; i += BS) {
        const uint64_t g = g0 + i;
        const El x[1] = {px[g]};
        const uint64_t k[1] = {pe[g]};
        El y[1];
        if (W == 32 && mode == 3) {
            pow_lanes<R, W == 32 ? 3 : 0, 1>(red, x, k, r2, one, mine, BS, y);
            po[g] = Ladder<R, W == 32 ? 3 : 0>::out(red, y[0]);
        } else if (W == 64 && mode == 1) {
            pow_lanes<R, W == 64 ? 1 : 0, 1>(red, x, k, r2, one, mine, BS, y);
            po[g] = Ladder<R, W == 64 ? 1 : 0>::out(red, y[0]);
        } else {
            pow_lanes<R, 0, 1>(red, x, k, r2, one, mine, BS, y);
            po[g] = Ladder<R, 0>::out(red, y[0]);
        }
    }
}

template <int W, int OP, bool NT, int BS>
__device__ __forceinline__ void tile_variant(uint32_t variant, const KCtx &c, const DPools &P, uint64_t g0,
                                             uint64_t g1, uint32_t cnt)
{
    switch (variant) {
    case CLASSIC:
        tile_map<W, CLASSIC, OP, NT, BS>(c, P, g0, g1, cnt);
        break;
    case SIGNED:
        tile_map<W, SIGNED, OP, NT, BS>(c, P, g0, g1, cnt);
        break;
    case PLANTARD:
        tile_map<W, PLANTARD, OP, NT, BS>(c, P, g0, g1, cnt);
        break;
    case SIGNED_PLANTARD:
        tile_map<W, SIGNED_PLANTARD, OP, NT, BS>(c, P, g0, g1, cnt);
        break;
    default:
        tile_map<W, SIGNED_PLANTARD_ALPHA, OP, NT, BS>(c, P, g0, g1, cnt);
        break;
    }
}

template <int W, bool NT, int BS>
__device__ __forceinline__ void tile_width(uint32_t op, uint32_t variant, const KCtx &c, const DPools &P,
                                           uint64_t g0, uint64_t g1, uint32_t cnt)
{
    if (op == MONT_OP_MUL)
        tile_variant<W, 0, NT, BS>(variant, c, P, g0, g1, cnt);
    else if (op == MONT_OP_REDC)
        tile_variant<W, 1, NT, BS>(variant, c, P, g0, g1, cnt);
    else
        tile_pow<W, BS>(c, P, g0, g1, cnt);
}

template <bool NT, int BS>
__global__ void __launch_bounds__(BS)
    k_ragged(const KCtx *__restrict__ ctab, const DTile *__restrict__ tiles, uint32_t ntiles, DPools P,
             uint32_t *__restrict__ ctr, uint32_t dynamic)
{
    // dynamic: 0 static, 1 one tile counter, 8 one counter per XCD.
    // Eight counters: with a grid that is a multiple of 8 (else one counter is
    // used), workgroup b (dispatched to XCD b mod 8) claims from counter
    // x = b mod 8 the tiles of the x-th eighth of the table in order (one
    // counter on one address serializes its atomics: one claim every ~11 ns
    // measured, so 1.5 x 10^6 tiles of 512 elements took 17 ms); each counter
    // has its own 128-byte line.  A workgroup whose eighth is used up moves on
    // to the next one, so XCDs that run faster than others take over their
    // remaining tiles.
    const uint32_t nx = dynamic == 8 && gridDim.x % 8u == 0 ? 8u : 1u;
    uint32_t sh = blockIdx.x % nx;  // lane 0's current shard
    uint32_t left = nx;             // shards lane 0 has not yet found used up
    const uint32_t lg = nx == 8 ? 3 : 0;
    auto shard_lo = [&](uint32_t x) { return (uint32_t)(((uint64_t)ntiles * x) >> lg); };  // ntiles x / nx
    // lane 0: the tile for `claim` of shard sh, or the next tile of a later
    // shard that still has one (ntiles once every shard is used up)
    auto next_tile = [&](uint32_t claim) {
        uint32_t t = shard_lo(sh) + claim;
        while (t >= shard_lo(sh + 1)) {
            if (!--left)
                return ntiles;
            sh = sh + 1 == nx ? 0 : sh + 1;
            t = shard_lo(sh) + atomicAdd(&ctr[CTR_STRIDE * sh], 1u);
        }
        return t;
    };
    __shared__ uint32_t s_next[2];
    uint32_t t;
    int buf = 0;
    if (dynamic) {
        if (threadIdx.x == 0)
            s_next[0] = next_tile(atomicAdd(&ctr[CTR_STRIDE * sh], 1u));
        __syncthreads();
        t = s_next[0];
    } else {
        t = xcd_block(blockIdx.x, gridDim.x);
    }
    t = __builtin_amdgcn_readfirstlane(t);
    DTile td{};
    if (t < ntiles)
        td = tiles[t];
    while (t < ntiles) {
        // The next tile is fetched while this one runs: its index from the counter
        // (the claim's result is first needed after the tile), or, statically, its
        // record.
        uint32_t claim = 0;
        if (dynamic && threadIdx.x == 0)
            claim = atomicAdd(&ctr[CTR_STRIDE * sh], 1u);
        const uint32_t tn = t + gridDim.x;
        DTile nd{};
        if (!dynamic && tn < ntiles)
            nd = tiles[tn];
        const KCtx &kc = ctab[td.ctx];
        const uint32_t wc = td.vw >> 8, variant = td.vw & 0xffu;
        if (wc == 0)
            tile_width<16, NT, BS>(td.op, variant, kc, P, td.g0, td.g1, td.cnt);
        else if (wc == 1)
            tile_width<32, NT, BS>(td.op, variant, kc, P, td.g0, td.g1, td.cnt);
        else
            tile_width<64, NT, BS>(td.op, variant, kc, P, td.g0, td.g1, td.cnt);
        if (dynamic) {
            if (threadIdx.x == 0)
                s_next[buf ^ 1] = next_tile(claim);
            __syncthreads();  // s_next[buf^1] written; everyone done with s_next[buf]
            buf ^= 1;
            t = __builtin_amdgcn_readfirstlane(s_next[buf]);
            if (t < ntiles)
                td = tiles[t];
        } else {
            t = tn;
            td = nd;
        }
    }
    if (dynamic) {
        // Every workgroup has made its last counter increment before it gets
        // here; the last one to arrive resets every counter for the next run.
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            const uint32_t d = atomicAdd(&ctr[CTR_STRIDE * 8], 1u);
            if (d == gridDim.x - 1) {
                for (uint32_t x = 0; x < nx; ++x)
                    atomicExch(&ctr[CTR_STRIDE * x], 0u);
                atomicExch(&ctr[CTR_STRIDE * 8], 0u);
            }
        }
    }
}

}  // namespace mont

using namespace mont;

// ------------------------------------------------------------------ host

struct mont_batch {
    int dev = 0;
    std::vector<mont_ctx_t> ctxs;
    std::vector<mont_seg_t> segs;
    std::vector<DSeg> hsegs;     // validated segments (host only: tiles carry what the kernel needs)
    KCtx *dctx = nullptr;        // the batch's per-modulus constants, indexed by the tiles
    DTile *dtiles = nullptr;
    uint32_t *dctr = nullptr;
    size_t tiles_cap = 0;
    uint32_t ntiles = 0;
    uint64_t elements = 0;
    uint32_t tile_base = 4096;   // 32-bit streaming tile (elements)
    uint32_t pow_tile = 1024;
    uint32_t blocks_per_cu = 0;  // 0: one workgroup per tile (one pass), else a persistent grid
    uint32_t grid = 0;
    uint32_t flags = 0;
    uint32_t op_mask = 0;
    bool tuned = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;
    bool nt = true;              // non-temporal loads/stores
    DPools last{};
    uint32_t last_grid = 0, last_dyn = 0, last_ntiles = 0;
    bool last_nt = true;
    DTile *last_tiles = nullptr;
    uint32_t block = BLOCK;      // lanes per workgroup: 64 or 256
    uint32_t counters = 8;       // tile counters of the dynamic schedule: 1, or 8 (one per XCD)
    uint32_t last_block = BLOCK;
};

namespace mont {

mont_status_t make_dseg(const mont_ctx_t *ctxs, uint32_t nctx, const mont_seg_t &sg, uint32_t i, DSeg &d)
{
    mont_status_t rc = MONT_OK;
    if (sg.ctx >= nctx)
        rc = fail(MONT_E_INVAL, "segment %u: context index %u out of range", i, sg.ctx);
    else if (sg.op > MONT_OP_POW)
        rc = fail(MONT_E_INVAL, "segment %u: unknown op %u", i, (unsigned)sg.op);
    else if (sg.op == MONT_OP_POW && sg.variant != MONT_CLASSIC)
        rc = fail(MONT_E_UNSUPPORTED, "segment %u: exponentiation uses the classic variant", i);
    else if (sg.n >= (1ull << 40) || sg.off >= (1ull << 48) || sg.off1 >= (1ull << 48))
        rc = fail(MONT_E_INVAL, "segment %u: size or offset too large", i);
    else if (sg.op == MONT_OP_MUL && ((sg.off1 - sg.off) & (uint64_t)(128 / ctxs[sg.ctx].w - 1)) != 0)
        rc = fail(MONT_E_INVAL, "segment %u: off1 - off must be a multiple of %u", i, 128 / ctxs[sg.ctx].w);
    else {
        rc = check_variant(&ctxs[sg.ctx], sg.variant);
        if (rc)
            rc = fail(rc, "segment %u: %s", i, mont_last_error());
    }
    if (rc)
        return rc;
    std::memset(&d, 0, sizeof d);
    d.ctx = sg.ctx;
    d.off = sg.off;
    d.off1 = sg.off1;
    d.op = sg.op;
    d.variant = sg.variant;
    d.wc = (uint32_t)width_class(ctxs[sg.ctx].w);
    return MONT_OK;
}

uint32_t seg_tile_elems(uint32_t tile_base, uint32_t pow_tile, uint32_t wc, uint32_t op)
{
    if (op == MONT_OP_POW)
        return pow_tile;
    // equal output bytes per tile: 16-bit tiles have twice the elements of 32-bit ones
    return wc == 0 ? tile_base * 2 : wc == 1 ? tile_base : tile_base / 2;
}

static uint32_t tile_elems(const mont_batch &b, uint32_t wc, uint32_t op)
{
    return seg_tile_elems(b.tile_base, b.pow_tile, wc, op);
}

static mont_status_t build_tiles(mont_batch &b, hipStream_t s)
{
    std::vector<DTile> pow_tiles, map_tiles;
    for (uint32_t i = 0; i < b.segs.size(); ++i) {
        const mont_seg_t &sg = b.segs[i];
        const uint32_t wc = b.hsegs[i].wc;
        const uint64_t te = tile_elems(b, wc, sg.op);
        for (uint64_t st = 0; st < sg.n; st += te)
            (sg.op == MONT_OP_POW ? pow_tiles : map_tiles)
                .push_back(make_tile(b.hsegs[i], st, (uint32_t)std::min<uint64_t>(te, sg.n - st)));
    }
    // Streaming tiles grouped by (width class, operation, variant), segment
    // order kept inside a group: at any moment the workgroups then run one code
    // path over one set of pools (on MI355X, 31- and 62-bit segments
    // interleaved in segment order ran 9 % slower than the two classes one
    // after the other).
    auto key = [](const DTile &t) { return ((t.vw >> 8) << 16) | (t.op << 8) | (t.vw & 0xffu); };
    std::stable_sort(map_tiles.begin(), map_tiles.end(),
                     [&](const DTile &x, const DTile &y) { return key(x) < key(y); });
    // the heaviest tiles (exponentiation) first, so a dynamic schedule ends level
    std::vector<DTile> all;
    all.reserve(pow_tiles.size() + map_tiles.size());
    all.insert(all.end(), pow_tiles.begin(), pow_tiles.end());
    all.insert(all.end(), map_tiles.begin(), map_tiles.end());
    if (all.size() >= 0xffffffffull)
        return fail(MONT_E_INVAL, "too many tiles");
    // A one-pass grid (one workgroup per tile) renumbers workgroups so that
    // XCD x walks the x-th eighth of the table (xcd_block, when the tile count
    // is a multiple of 8): store logical tile 8p + x at x * (n/8) + p, so that
    // the XCDs, advancing together, visit the logical order above.
    if (!b.blocks_per_cu && !(b.flags & MONT_BATCH_DYNAMIC) && all.size() % 8 == 0 && !all.empty()) {
        const size_t c = all.size() / 8;
        std::vector<DTile> perm(all.size());
        for (size_t p = 0; p < c; ++p)
            for (size_t x = 0; x < 8; ++x)
                perm[x * c + p] = all[8 * p + x];
        all.swap(perm);
    }
    if (all.size() > b.tiles_cap) {
        if (b.dtiles)
            (void)hipFree(b.dtiles);
        b.dtiles = nullptr;
        const size_t cap = std::max<size_t>(all.size(), 1);
        if (hipMalloc(&b.dtiles, cap * sizeof(DTile)) != hipSuccess)
            return fail(MONT_E_NOMEM, "tile table of %zu entries", cap);
        b.tiles_cap = cap;
    }
    b.ntiles = (uint32_t)all.size();
    if (!all.empty()) {
        hipError_t e = hipMemcpyAsync(b.dtiles, all.data(), all.size() * sizeof(DTile), hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return hip_fail(e, "tile table upload");
        e = hipStreamSynchronize(s);  // the host vector dies here
        if (e != hipSuccess)
            return hip_fail(e, "tile table upload");
    }
    const uint64_t g = b.blocks_per_cu ? (uint64_t)device_cus() * b.blocks_per_cu : (uint64_t)b.ntiles;
    b.grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, b.ntiles));
    return MONT_OK;
}

static DPools to_dpools(const mont_pools_t &p)
{
    DPools d;
    for (int i = 0; i < 3; ++i) {
        d.in0[i] = p.in0[i];
        d.in1[i] = p.in1[i];
        d.out[i] = p.out[i];
    }
    return d;
}

static mont_status_t check_pools(const mont_batch &b, const mont_pools_t *p)
{
    if (!p)
        return fail(MONT_E_INVAL, "null pools");
    for (size_t i = 0; i < b.segs.size(); ++i) {
        const mont_seg_t &sg = b.segs[i];
        if (!sg.n)
            continue;
        const uint32_t wc = b.hsegs[i].wc;
        if (!p->in0[wc] || !p->out[wc] || (sg.op != MONT_OP_REDC && !p->in1[wc]))
            return fail(MONT_E_INVAL, "segment %zu: pool for width class %u is NULL", i, wc);
    }
    for (int wc = 0; wc < 3; ++wc) {
        const uintptr_t a = (uintptr_t)p->in0[wc] | (uintptr_t)p->in1[wc] | (uintptr_t)p->out[wc];
        if (a & 15u)
            return fail(MONT_E_INVAL, "pool pointers must be 16-byte aligned");
    }
    return MONT_OK;
}

void *ragged_kernel_ptr(bool nt, uint32_t block)
{
    if (block == 64)
        return nt ? (void *)k_ragged<true, 64> : (void *)k_ragged<false, 64>;
    return nt ? (void *)k_ragged<true, BLOCK> : (void *)k_ragged<false, BLOCK>;
}

hipError_t launch_ragged(const KCtx *ctab, const DTile *tiles, uint32_t ntiles, const DPools &P, uint32_t *ctr,
                         uint32_t dyn, uint32_t grid, bool nt, hipStream_t s, uint32_t block)
{
    const uint32_t bs = block == 64 ? 64 : BLOCK;
    void *args[] = {&ctab, &tiles, &ntiles, const_cast<DPools *>(&P), &ctr, &dyn};
    return hipLaunchKernel(ragged_kernel_ptr(nt, bs), dim3(grid), dim3(bs), args, 0, s);
}

static mont_status_t launch_direct(mont_batch &b, const DPools &P, hipStream_t s, uint32_t dyn)
{
    const hipError_t e = launch_ragged(b.dctx, b.dtiles, b.ntiles, P, b.dctr, dyn, b.grid, b.nt, s, b.block);
    return e == hipSuccess ? MONT_OK : hip_fail(e, "ragged launch");
}

static mont_status_t launch_graph(mont_batch &b, const DPools &P, hipStream_t s, uint32_t dyn)
{
    DPools Pc = P;
    KCtx *ctab = b.dctx;
    DTile *tiles = b.dtiles;
    uint32_t nt = b.ntiles;
    uint32_t *ctr = b.dctr;
    void *args[] = {&ctab, &tiles, &nt, &Pc, &ctr, &dyn};
    hipKernelNodeParams kp{};
    kp.func = ragged_kernel_ptr(b.nt, b.block);
    kp.gridDim = dim3(b.grid);
    kp.blockDim = dim3(b.block);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipError_t e;
    if (b.exec && (b.last_nt != b.nt || b.last_block != b.block)) {
        // another kernel (non-temporal hint or workgroup size): an executable graph's
        // kernel node cannot change its function, so the graph is built again (after
        // the batch's earlier runs, on this stream)
        log_msg(2, "ragged graph rebuilt: kernel changed (workgroup %u, nt %d)", b.block, (int)b.nt);
        e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return hip_fail(e, "ragged graph rebuild");
        (void)hipGraphExecDestroy(b.exec);
        (void)hipGraphDestroy(b.graph);
        b.exec = nullptr;
        b.graph = nullptr;
    }
    if (!b.exec) {
        e = hipGraphCreate(&b.graph, 0);
        if (e == hipSuccess)
            e = hipGraphAddKernelNode(&b.node, b.graph, nullptr, 0, &kp);
        if (e == hipSuccess)
            e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
        if (e != hipSuccess)
            return hip_fail(e, "ragged graph build");
    } else if (std::memcmp(&b.last, &P, sizeof P) != 0 || b.last_grid != b.grid || b.last_dyn != dyn ||
               b.last_ntiles != b.ntiles || b.last_tiles != b.dtiles) {
        e = hipGraphExecKernelNodeSetParams(b.exec, b.node, &kp);
        if (e != hipSuccess)
            return hip_fail(e, "ragged graph update");
    }
    b.last = P;
    b.last_grid = b.grid;
    b.last_dyn = dyn;
    b.last_nt = b.nt;
    b.last_ntiles = b.ntiles;
    b.last_tiles = b.dtiles;
    b.last_block = b.block;
    e = hipGraphLaunch(b.exec, s);
    return e == hipSuccess ? MONT_OK : hip_fail(e, "ragged graph launch");
}

static mont_status_t run_once(mont_batch &b, const DPools &P, hipStream_t s)
{
    if (b.ntiles == 0)
        return MONT_OK;
    const uint32_t dyn = (b.flags & MONT_BATCH_DYNAMIC) ? b.counters : 0u;
    return (b.flags & MONT_BATCH_GRAPH) ? launch_graph(b, P, s, dyn) : launch_direct(b, P, s, dyn);
}

// Tuning: tile size x workgroups per CU x schedule, timed with HIP events.
struct RaggedTune {
    uint32_t tile_base, blocks_per_cu, dynamic, nt, block;
};

static std::string tune_key(const mont_batch &b)
{
    uint64_t ops[3] = {0, 0, 0};
    for (const auto &sg : b.segs)
        ops[sg.op] += sg.n;
    char k[160];
    int lg = 0;
    while ((b.elements >> lg) > 1)
        ++lg;
    snprintf(k, sizeof k, "ragged:nseg=%zu:log2n=%d:mul=%d:redc=%d:pow=%d", b.segs.size() >= 1024 ? 1024 : b.segs.size(),
             lg, ops[0] > 0, ops[1] > 0, ops[2] > 0);
    return tune_key_prefix() + k;
}

// Library-owned output pools of the batch's extent per width class: the tuner
// writes its candidate runs there, so the caller's buffers are only read
// (a batch whose outputs overwrite its inputs stays correct).
struct ScratchOut {
    void *p[3] = {nullptr, nullptr, nullptr};
    ~ScratchOut()
    {
        for (void *q : p)
            if (q)
                (void)hipFree(q);
    }
};

static mont_status_t scratch_outputs(const mont_batch &b, const DPools &P, ScratchOut &so, DPools &Pt)
{
    static const size_t esz[3] = {2, 4, 8};
    uint64_t ext[3] = {0, 0, 0};
    for (size_t i = 0; i < b.segs.size(); ++i) {
        const mont_seg_t &sg = b.segs[i];
        if (sg.n)
            ext[b.hsegs[i].wc] = std::max<uint64_t>(ext[b.hsegs[i].wc], sg.off + sg.n);
    }
    Pt = P;
    for (int wc = 0; wc < 3; ++wc) {
        if (!ext[wc])
            continue;
        if (hipMalloc(&so.p[wc], ext[wc] * esz[wc]) != hipSuccess)
            return fail(MONT_E_NOMEM, "tuning output pool of %llu bytes", (unsigned long long)(ext[wc] * esz[wc]));
        Pt.out[wc] = so.p[wc];
    }
    return MONT_OK;
}

static mont_status_t tune(mont_batch &b, const DPools &Pcaller, hipStream_t s)
{
    const std::string key = tune_key(b);
    {
        // a shape tuned earlier (this process, or $MONT_TUNE_CACHE) for this device,
        // library version and batch class
        TuneRecord r;
        if (tune_lookup(key, r) && r.count("tile_elems") && r.count("blocks_per_cu") && r.count("dynamic") &&
            r.count("nontemporal")) {
            const uint32_t t = (uint32_t)r["tile_elems"], bpc = (uint32_t)r["blocks_per_cu"];
            const uint32_t bs = r.count("block") ? (uint32_t)r["block"] : BLOCK;
            const uint32_t dyn = (uint32_t)r["dynamic"];
            if (t >= 256 && t <= (1u << 20) && !(t & (t - 1)) && bpc <= 64 && (bs == 64 || bs == 256) &&
                (dyn == 0 || dyn == 1 || dyn == 8)) {
                b.tile_base = t;
                b.blocks_per_cu = bpc;
                b.block = bs;
                b.nt = r["nontemporal"] != 0;
                b.flags = (b.flags & ~MONT_BATCH_DYNAMIC) | (dyn ? MONT_BATCH_DYNAMIC : 0u);
                if (dyn)
                    b.counters = dyn;
                log_msg(2, "ragged tune: %s: cached shape tile %u, %u workgroups/CU, counters %u, nt %d", key.c_str(),
                        t, bpc, dyn, (int)b.nt);
                return build_tiles(b, s);
            }
        }
    }
    ScratchOut so;
    DPools P;
    if (mont_status_t rs = scratch_outputs(b, Pcaller, so, P))
        return rs;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return fail(MONT_E_DEVICE, "event create");
    }
    const uint32_t tiles[] = {1024, 2048, 4096, 8192, 16384};
    const uint32_t bpcs[] = {0, 2, 4, 8};
    const uint32_t kinds[] = {0, 1, 8};
    // 64-lane workgroups stay available through mont_batch_set_shape but are not
    // swept: on the ragged kernel they never won (the per-tile descriptor and
    // constant loads are amortized over 4x fewer lanes).
    float best = 1e30f;
    RaggedTune bt{b.tile_base, b.blocks_per_cu, (b.flags & MONT_BATCH_DYNAMIC) ? b.counters : 0u, b.nt ? 1u : 0u,
                  b.block};
    const uint32_t saved_flags = b.flags;
    b.flags &= ~MONT_BATCH_GRAPH;  // time direct launches
    mont_status_t rc = MONT_OK;
    // bring the clocks to their loaded state first (about 25 ms of the starting
    // shape), so the first candidates are not timed on an idle GPU
    if ((rc = build_tiles(b, s)))
        goto done;
    {
        const auto t0 = std::chrono::steady_clock::now();
        do {
            for (int r = 0; r < 4 && !rc; ++r)
                rc = run_once(b, P, s);
            if (!rc && hipStreamSynchronize(s) != hipSuccess)
                rc = fail(MONT_E_DEVICE, "tuning warm-up failed");
        } while (!rc && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(25));
        if (rc)
            goto done;
    }
    for (uint32_t tb : tiles) {
        b.tile_base = tb;
        b.pow_tile = 1024;
        for (uint32_t bpc : bpcs) {
            b.blocks_per_cu = bpc;
            if ((rc = build_tiles(b, s)))
                goto done;
            // schedules: static, one tile counter, eight (one per XCD); either access
            for (uint32_t v = 0; v < 6; ++v) {
                const uint32_t dyn = kinds[v % 3], nt = v / 3, bs = BLOCK;
                if (dyn && !bpc)
                    continue;  // one workgroup per tile: nothing to balance
                b.flags = (b.flags & ~MONT_BATCH_DYNAMIC) | (dyn ? MONT_BATCH_DYNAMIC : 0u);
                if (dyn)
                    b.counters = dyn;
                b.nt = nt != 0;
                b.block = bs;
                if ((rc = run_once(b, P, s)))  // warm
                    goto done;
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < 5; ++r)
                    if ((rc = run_once(b, P, s)))
                        goto done;
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) {
                    rc = fail(MONT_E_DEVICE, "tuning run failed");
                    goto done;
                }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    bt = {tb, bpc, dyn, nt, bs};
                }
            }
        }
    }
done:
    // the scratch pools are freed on return; nothing of the sweep may still run then
    if (hipStreamSynchronize(s) != hipSuccess && !rc)
        rc = fail(MONT_E_DEVICE, "tuning runs failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the best shape so far (the starting one if none was timed), also after a failure
    b.flags = (saved_flags & ~MONT_BATCH_DYNAMIC) | (bt.dynamic ? MONT_BATCH_DYNAMIC : 0u);
    if (bt.dynamic)
        b.counters = bt.dynamic;
    b.tile_base = bt.tile_base;
    b.blocks_per_cu = bt.blocks_per_cu;
    b.nt = bt.nt != 0;
    b.block = bt.block;
    if (rc) {
        (void)build_tiles(b, s);
        return rc;
    }
    log_msg(2, "ragged tune: %s: tile %u, %u workgroups/CU, counters %u, nt %u (%.4f ms per run)", key.c_str(),
            bt.tile_base, bt.blocks_per_cu, bt.dynamic, bt.nt, best / 5);
    tune_store(key, {{"tile_elems", (double)bt.tile_base},
                     {"blocks_per_cu", (double)bt.blocks_per_cu},
                     {"dynamic", (double)bt.dynamic},
                     {"nontemporal", (double)bt.nt},
                     {"block", (double)bt.block},
                     {"ms", best / 5}});
    return build_tiles(b, s);
}

}  // namespace mont

extern "C" {

mont_status_t mont_batch_create(const mont_ctx_t *ctxs, uint32_t nctx, const mont_seg_t *segs, uint32_t nseg,
                                uint32_t flags, mont_batch_t **out, void *stream)
{
    if (!out)
        return fail(MONT_E_INVAL, "null output handle");
    *out = nullptr;
    if ((nctx && !ctxs) || (nseg && !segs))
        return fail(MONT_E_INVAL, "null table");
    for (uint32_t i = 0; i < nctx; ++i) {
        mont_status_t rc = check_ctx(&ctxs[i]);
        if (rc)
            return fail(rc, "context %u: %s", i, mont_last_error());
    }
    mont_batch *b = new (std::nothrow) mont_batch;
    if (!b)
        return fail(MONT_E_NOMEM, "batch");
    b->ctxs.assign(ctxs, ctxs + nctx);
    b->segs.assign(segs, segs + nseg);
    b->flags = flags;
    b->hsegs.resize(nseg);
    for (uint32_t i = 0; i < nseg; ++i) {
        const mont_seg_t &sg = segs[i];
        if (mont_status_t rc = make_dseg(ctxs, nctx, sg, i, b->hsegs[i])) {
            delete b;
            return rc;
        }
        b->elements += sg.n;
        b->op_mask |= 1u << sg.op;
    }
    (void)hipGetDevice(&b->dev);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMalloc(&b->dctx, std::max<size_t>(nctx, 1) * sizeof(KCtx));
    if (e == hipSuccess)
        e = hipMalloc(&b->dctr, CTR_BYTES);
    if (e != hipSuccess) {
        mont_batch_destroy(b);
        return fail(MONT_E_NOMEM, "batch tables");
    }
    std::vector<KCtx> kctx(nctx);
    for (uint32_t i = 0; i < nctx; ++i)
        kctx[i] = to_kctx(ctxs[i]);
    if (e == hipSuccess && nctx)
        e = hipMemcpyAsync(b->dctx, kctx.data(), nctx * sizeof(KCtx), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // the host tables die here
    if (e == hipSuccess)
        e = hipMemsetAsync(b->dctr, 0, CTR_BYTES, s);
    if (e != hipSuccess) {
        mont_batch_destroy(b);
        return hip_fail(e, "batch upload");
    }
    mont_status_t rc = build_tiles(*b, s);
    if (rc) {
        mont_batch_destroy(b);
        return rc;
    }
    *out = b;
    return MONT_OK;
}

mont_status_t mont_batch_run(mont_batch_t *b, const mont_pools_t *pools, void *stream)
{
    if (!b)
        return fail(MONT_E_INVAL, "null batch");
    mont_status_t rc = check_pools(*b, pools);
    if (rc)
        return rc;
    const DPools P = to_dpools(*pools);
    hipStream_t s = (hipStream_t)stream;
#ifdef MONT_DEBUG
    for (size_t i = 0; i < b->segs.size(); ++i) {
        const mont_seg_t &sg = b->segs[i];
        const mont_ctx_t &c = b->ctxs[sg.ctx];
        const size_t es = c.w / 8;
        const uint32_t wc = b->hsegs[i].wc;
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
    const int tov = tune_override();
    if ((tov == 1 || (tov != 0 && (b->flags & MONT_BATCH_TUNE))) && !b->tuned) {
        rc = tune(*b, P, s);
        if (rc)
            return rc;
        b->tuned = true;
    }
    if (log_level() >= 3)
        log_msg(3, "ragged run: %llu tiles, grid %u x %u lanes, tile %u, counters %u, nt %d, graph %d",
                (unsigned long long)b->ntiles, b->grid, b->block, b->tile_base,
                (b->flags & MONT_BATCH_DYNAMIC) ? b->counters : 0u, (int)b->nt, (b->flags & MONT_BATCH_GRAPH) ? 1 : 0);
    return run_once(*b, P, s);
}

static mont_status_t run_only(mont_batch_t *b, const mont_pools_t *pools, void *stream, uint32_t op)
{
    if (!b)
        return fail(MONT_E_INVAL, "null batch");
    if (b->op_mask & ~(1u << op))
        return fail(MONT_E_INVAL, "batch holds segments of another operation");
    return mont_batch_run(b, pools, stream);
}

mont_status_t mont_mul_ragged(mont_batch_t *b, const mont_pools_t *p, void *s) { return run_only(b, p, s, MONT_OP_MUL); }
mont_status_t mont_redc_ragged(mont_batch_t *b, const mont_pools_t *p, void *s) { return run_only(b, p, s, MONT_OP_REDC); }
mont_status_t mont_pow_ragged(mont_batch_t *b, const mont_pools_t *p, void *s) { return run_only(b, p, s, MONT_OP_POW); }

mont_status_t mont_batch_run_pervector(mont_batch_t *b, const mont_pools_t *pools, void *stream)
{
    if (!b)
        return fail(MONT_E_INVAL, "null batch");
    mont_status_t rc = check_pools(*b, pools);
    if (rc)
        return rc;
    static const size_t esz[3] = {2, 4, 8};
    for (size_t i = 0; i < b->segs.size(); ++i) {
        const mont_seg_t &sg = b->segs[i];
        if (!sg.n)
            continue;
        const mont_ctx_t *c = &b->ctxs[sg.ctx];
        const uint32_t wc = b->hsegs[i].wc;
        const size_t es = esz[wc];
        const char *i0 = (const char *)pools->in0[wc];
        const char *i1 = (const char *)pools->in1[wc];
        char *o = (char *)pools->out[wc];
        if (sg.op == MONT_OP_MUL)
            rc = mont_mul(c, i0 + sg.off * es, i1 + sg.off1 * es, o + sg.off * es, sg.n,
                          (mont_variant_t)sg.variant, stream);
        else if (sg.op == MONT_OP_REDC)
            rc = mont_redc(c, i0 + sg.off * 2 * es, o + sg.off * es, sg.n, (mont_variant_t)sg.variant, stream);
        else
            rc = mont_pow(c, i0 + sg.off * es, (const uint64_t *)i1 + sg.off1, o + sg.off * es, sg.n, stream);
        if (rc)
            return rc;
    }
    return MONT_OK;
}

mont_status_t mont_batch_info(const mont_batch_t *b, mont_batch_info_t *info)
{
    if (!b || !info)
        return fail(MONT_E_INVAL, "null argument");
    info->ntiles = b->ntiles;
    info->elements = b->elements;
    info->tile_elems = b->tile_base;
    info->grid = b->grid;
    info->block = b->block;
    info->flags = b->flags | (b->nt ? MONT_BATCH_NONTEMPORAL : 0u);
    info->blocks_per_cu = b->blocks_per_cu;
    info->pow_tile = b->pow_tile;
    info->counters = (b->flags & MONT_BATCH_DYNAMIC) ? b->counters : 0u;
    return MONT_OK;
}

mont_status_t mont_batch_set_shape(mont_batch_t *b, const mont_batch_shape_t *sh, void *stream)
{
    if (!b || !sh)
        return fail(MONT_E_INVAL, "null argument");
    const uint32_t t = sh->tile_elems;
    if (t < 256 || t > (1u << 20) || (t & (t - 1)))
        return fail(MONT_E_INVAL, "tile_elems must be a power of two in [256, 2^20]");
    if (sh->blocks_per_cu > 64)
        return fail(MONT_E_INVAL, "blocks_per_cu must be at most 64");
    if ((sh->dynamic != 0 && sh->dynamic != 1 && sh->dynamic != 8) || sh->nontemporal > 1)
        return fail(MONT_E_INVAL, "dynamic is 0, 1 or 8 and nontemporal 0 or 1");
    if (sh->block != 0 && sh->block != 64 && sh->block != 256)
        return fail(MONT_E_INVAL, "block must be 0 (256), 64 or 256");
    b->block = sh->block == 64 ? 64 : BLOCK;
    b->tile_base = t;
    b->blocks_per_cu = sh->blocks_per_cu;
    b->nt = sh->nontemporal != 0;
    b->flags = (b->flags & ~MONT_BATCH_DYNAMIC) | (sh->dynamic ? MONT_BATCH_DYNAMIC : 0u);
    if (sh->dynamic)
        b->counters = sh->dynamic;
    b->tuned = true;  // an explicit shape replaces tuning
    return build_tiles(*b, (hipStream_t)stream);
}

void mont_batch_destroy(mont_batch_t *b)
{
    if (!b)
        return;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->dctx)
        (void)hipFree(b->dctx);
    if (b->dtiles)
        (void)hipFree(b->dtiles);
    if (b->dctr)
        (void)hipFree(b->dctr);
    delete b;
}

}  // extern "C"
