// Reference streaming kernel for roofline measurements: out = a XOR b over
// 16-byte chunks, with exactly the access pattern and launch shape of the
// Montgomery product kernels (one chunk per lane, non-temporal loads and
// stores, one pass, XCD-contiguous workgroup order) and no arithmetic.  Its
// bandwidth is the practical ceiling the product kernels are compared with.
#include <hip/hip_runtime.h>

#include "mont_common.hpp"

namespace mont {

__global__ void __launch_bounds__(BLOCK)
    k_xor_ref(const u32x4 *__restrict__ a, const u32x4 *__restrict__ b, u32x4 *__restrict__ o, uint64_t n16)
{
    const uint64_t i = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (i < n16) {
        const u32x4 x = __builtin_nontemporal_load(a + i);
        const u32x4 y = __builtin_nontemporal_load(b + i);
        __builtin_nontemporal_store(x ^ y, o + i);
    }
}

}  // namespace mont

using namespace mont;

extern "C" mont_status_t mont_stream_ref(const void *a, const void *b, void *out, size_t bytes, void *stream)
{
    if (bytes == 0)
        return MONT_OK;
    if (!a || !b || !out || (((uintptr_t)a | (uintptr_t)b | (uintptr_t)out | bytes) & 15u))
        return fail(MONT_E_INVAL, "mont_stream_ref needs 16-byte aligned buffers and a multiple of 16 bytes");
    const uint64_t n16 = bytes / 16;
    const uint64_t grid = (n16 + BLOCK - 1) / BLOCK;
    if (grid > 0x7fffffffu)
        return fail(MONT_E_INVAL, "buffer too large");
    hipLaunchKernelGGL(k_xor_ref, dim3((unsigned)grid), dim3(BLOCK), 0, (hipStream_t)stream, (const u32x4 *)a,
                       (const u32x4 *)b, (u32x4 *)out, n16);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MONT_OK : hip_fail(e, "mont_stream_ref launch");
}
