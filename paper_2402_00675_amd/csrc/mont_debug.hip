// MONT_DEBUG builds only: the counting kernel behind the precondition checks
// (ranges in mont_debug.hpp) and mont_debug_violations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "mont_debug.hpp"

namespace mont {

__device__ unsigned long long g_dbg_violations;  // per device; zero at load
static std::atomic<uint64_t> g_dbg_host{0};      // counts made on the host (serving jobs)

struct DbgArgs {
    uint64_t N, b;
    uint32_t w, alpha;
    int32_t kind, variant;
};

// Element i of a w-bit (or, for T, 2w-bit) array as an unsigned 64-bit pattern
// (lo) and, for 128-bit T, its high word.
template <int W>
__device__ __forceinline__ uint64_t ld_w(const void *p, uint64_t i)
{
    if constexpr (W == 16)
        return ((const uint16_t *)p)[i];
    else if constexpr (W == 32)
        return ((const uint32_t *)p)[i];
    else
        return ((const uint64_t *)p)[i];
}

template <int W>
__device__ bool dbg_bad(const DbgArgs &a, const void *in0, const void *in1, uint64_t i)
{
    bool neg = false;
    dbg_u128 mag = 0;
    if (a.kind == DBG_BELOW_N)
        return ld_w<W>(in0, i) >= a.N;
    if (a.kind == DBG_PRODUCT || a.kind == DBG_CONST) {
        dbg_product(a.variant, W, ld_w<W>(in0, i), a.kind == DBG_CONST ? a.b : ld_w<W>(in1, i), &neg, &mag);
    } else {
        const bool sgn = a.variant == SIGNED || a.variant == SIGNED_PLANTARD || a.variant == SIGNED_PLANTARD_ALPHA;
        dbg_u128 t;
        if constexpr (W == 64) {
            const uint64_t *q = (const uint64_t *)in0 + 2 * i;
            t = ((dbg_u128)q[1] << 64) | q[0];
        } else {
            t = ld_w<2 * W>(in0, i);
        }
        const dbg_u128 top = (dbg_u128)1 << (2 * W - 1);
        if (sgn && (t & top)) {
            neg = true;
            const dbg_u128 mask = W == 64 ? ~(dbg_u128)0 : (((dbg_u128)1 << (2 * W)) - 1);
            mag = (~t + 1) & mask;
        } else {
            mag = t;
        }
    }
    return !dbg_t_in_range(a.variant, W, a.N, a.alpha, neg, mag);
}

// Every lane of a wave runs the same number of passes (the block's base index
// is uniform), so the ballot sees the whole wave; lane 0 adds its count with
// one vector atomic.
template <int W>
__global__ void __launch_bounds__(BLOCK) k_dbg(DbgArgs a, const void *in0, const void *in1, uint64_t n)
{
    for (uint64_t base = (uint64_t)blockIdx.x * BLOCK; base < n; base += (uint64_t)gridDim.x * BLOCK) {
        const uint64_t i = base + threadIdx.x;
        const bool bad = i < n && dbg_bad<W>(a, in0, in1, i);
        const unsigned long long m = __ballot(bad);
        if ((threadIdx.x & 63u) == 0 && m)
            atomicAdd(&g_dbg_violations, (unsigned long long)__popcll(m));
    }
}

hipError_t debug_check(int kind, const mont_ctx_t &c, int variant, const void *in0, const void *in1, uint64_t b,
                       uint64_t n, hipStream_t s)
{
    if (!n)
        return hipSuccess;
    DbgArgs a;
    a.N = c.N;
    a.b = b;
    a.w = c.w;
    a.alpha = c.alpha;
    a.kind = kind;
    a.variant = variant;
    const uint64_t blocks = std::min<uint64_t>((n + BLOCK - 1) / BLOCK, (uint64_t)device_cus() * 8);
    const dim3 grid((unsigned)blocks), blk(BLOCK);
    if (c.w == 16)
        hipLaunchKernelGGL(k_dbg<16>, grid, blk, 0, s, a, in0, in1, n);
    else if (c.w == 32)
        hipLaunchKernelGGL(k_dbg<32>, grid, blk, 0, s, a, in0, in1, n);
    else
        hipLaunchKernelGGL(k_dbg<64>, grid, blk, 0, s, a, in0, in1, n);
    return hipGetLastError();
}

void debug_count_host(uint64_t k) { g_dbg_host.fetch_add(k, std::memory_order_relaxed); }

}  // namespace mont

using namespace mont;

extern "C" mont_status_t mont_debug_violations(uint64_t *count, int reset)
{
    hipError_t e = hipDeviceSynchronize();
    unsigned long long dev = 0;
    if (e == hipSuccess)
        e = hipMemcpyFromSymbol(&dev, HIP_SYMBOL(g_dbg_violations), sizeof dev, 0, hipMemcpyDeviceToHost);
    if (e == hipSuccess && reset) {
        const unsigned long long zero = 0;
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_dbg_violations), &zero, sizeof zero, 0, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess)
        return hip_fail(e, "mont_debug_violations");
    const uint64_t host = reset ? g_dbg_host.exchange(0) : g_dbg_host.load();
    if (count)
        *count = (uint64_t)dev + host;
    return MONT_OK;
}
