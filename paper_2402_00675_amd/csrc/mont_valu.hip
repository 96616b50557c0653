// VALU issue-rate reference kernels (measurement aid): long runs of one
// integer instruction kind, eight independent dependency chains per lane so
// that issue rate, not latency, bounds them.  Used to state the measured
// peak of the instructions the reduction kernels are made of.
#include <hip/hip_runtime.h>

#include "mont_common.hpp"

namespace mont {

template <int KIND>
__global__ void __launch_bounds__(BLOCK) k_valu(uint32_t iters, uint32_t seed, uint64_t *__restrict__ out)
{
    const uint32_t t = blockIdx.x * BLOCK + threadIdx.x;
    uint32_t x[8];
    uint64_t y[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        x[c] = t * 2654435761u + seed + 97u * c;
        y[c] = ((uint64_t)x[c] << 17) ^ c;
    }
    const uint32_t m = seed | 1u;
    const uint64_t m64 = ((uint64_t)seed << 32) | m;
    uint64_t cy[8] = {};  // kind 15: per-chain carry masks (scalar register pairs)
    // Exact instruction streams: a self-referential multiply-add for
    // v_mad_u64_u32, register-only ALU inline assembly for the others (the
    // compiler would otherwise fold repeated products algebraically).  Kinds 7
    // (compares writing the condition mask VCC, which nothing reads), 11
    // (moves), 14 (carry-out adds, VCC written and never read), 15 (carry
    // chains, one scalar register pair per chain), 20 (compares) and 21 (signed
    // multiply-adds, VCC written) put a round's eight
    // instructions in one statement: the compiler adds a wait state after
    // every separate statement of those forms.
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if constexpr (KIND == 7) {
                    if (c == 0)
                        asm volatile("v_cmp_le_u64_e32 vcc, %0, %8\n\tv_cmp_le_u64_e32 vcc, %1, %8\n\t"
                                     "v_cmp_le_u64_e32 vcc, %2, %8\n\tv_cmp_le_u64_e32 vcc, %3, %8\n\t"
                                     "v_cmp_le_u64_e32 vcc, %4, %8\n\tv_cmp_le_u64_e32 vcc, %5, %8\n\t"
                                     "v_cmp_le_u64_e32 vcc, %6, %8\n\tv_cmp_le_u64_e32 vcc, %7, %8"
                                     :
                                     : "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(y[3]), "v"(y[4]), "v"(y[5]), "v"(y[6]),
                                       "v"(y[7]), "v"(m64)
                                     : "vcc");
                } else if constexpr (KIND == 0) {
                    // y = hi(y) * m + y: one v_mad_u64_u32, not foldable (the factor is y's own high word)
                    y[c] = (uint64_t)(uint32_t)(y[c] >> 32) * m + y[c];
                } else if constexpr (KIND == 1) {
                    asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 2) {
                    asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 3) {
                    asm volatile("v_mul_u32_u24 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 4) {
                    asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 5) {
                    asm volatile("v_lshl_add_u64 %0, %0, 1, %1" : "+v"(y[c]) : "v"(m64));
                } else if constexpr (KIND == 6) {
                    asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(x[c]) : "v"(m), "s"(m64));
                } else if constexpr (KIND == 8) {
                    asm volatile("v_lshrrev_b64 %0, 1, %0" : "+v"(y[c]));
                } else if constexpr (KIND == 9) {
                    asm volatile("v_sub_u32 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 10) {
                    asm volatile("v_min_u32 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 11) {
                    if (c == 0)
                        asm volatile("v_mov_b32 %0, %8\n\tv_mov_b32 %1, %8\n\tv_mov_b32 %2, %8\n\tv_mov_b32 %3, %8\n\t"
                                     "v_mov_b32 %4, %8\n\tv_mov_b32 %5, %8\n\tv_mov_b32 %6, %8\n\tv_mov_b32 %7, %8"
                                     : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                                       "+v"(x[6]), "+v"(x[7])
                                     : "v"(m));
                } else if constexpr (KIND == 12) {
                    asm volatile("v_and_or_b32 %0, %0, %1, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 13) {
                    asm volatile("v_add3_u32 %0, %0, %1, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 16) {
                    asm volatile("v_or_b32 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 17) {
                    asm volatile("v_and_b32 %0, %0, %1" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 18) {
                    asm volatile("v_lshlrev_b32 %0, 1, %0" : "+v"(x[c]));
                } else if constexpr (KIND == 19) {
                    asm volatile("v_alignbit_b32 %0, %0, %1, 31" : "+v"(x[c]) : "v"(m));
                } else if constexpr (KIND == 20) {
                    if (c == 0)
                        asm volatile("v_cmp_ne_u32_e32 vcc, 0, %0\n\tv_cmp_ne_u32_e32 vcc, 0, %1\n\t"
                                     "v_cmp_ne_u32_e32 vcc, 0, %2\n\tv_cmp_ne_u32_e32 vcc, 0, %3\n\t"
                                     "v_cmp_ne_u32_e32 vcc, 0, %4\n\tv_cmp_ne_u32_e32 vcc, 0, %5\n\t"
                                     "v_cmp_ne_u32_e32 vcc, 0, %6\n\tv_cmp_ne_u32_e32 vcc, 0, %7"
                                     :
                                     : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(x[4]), "v"(x[5]), "v"(x[6]),
                                       "v"(x[7])
                                     : "vcc");
                } else if constexpr (KIND == 21) {
                    // signed y = x * m + y (the exponentiation ladder's product form), VCC written, never read
                    if (c == 0)
                        asm volatile("v_mad_i64_i32 %0, vcc, %8, %16, %0\n\tv_mad_i64_i32 %1, vcc, %9, %16, %1\n\t"
                                     "v_mad_i64_i32 %2, vcc, %10, %16, %2\n\tv_mad_i64_i32 %3, vcc, %11, %16, %3\n\t"
                                     "v_mad_i64_i32 %4, vcc, %12, %16, %4\n\tv_mad_i64_i32 %5, vcc, %13, %16, %5\n\t"
                                     "v_mad_i64_i32 %6, vcc, %14, %16, %6\n\tv_mad_i64_i32 %7, vcc, %15, %16, %7"
                                     : "+v"(y[0]), "+v"(y[1]), "+v"(y[2]), "+v"(y[3]), "+v"(y[4]), "+v"(y[5]),
                                       "+v"(y[6]), "+v"(y[7])
                                     : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(x[4]), "v"(x[5]), "v"(x[6]),
                                       "v"(x[7]), "v"(m)
                                     : "vcc");
                } else if constexpr (KIND == 14) {
                    if (c == 0)
                        asm volatile("v_add_co_u32 %0, vcc, %0, %8\n\tv_add_co_u32 %1, vcc, %1, %8\n\t"
                                     "v_add_co_u32 %2, vcc, %2, %8\n\tv_add_co_u32 %3, vcc, %3, %8\n\t"
                                     "v_add_co_u32 %4, vcc, %4, %8\n\tv_add_co_u32 %5, vcc, %5, %8\n\t"
                                     "v_add_co_u32 %6, vcc, %6, %8\n\tv_add_co_u32 %7, vcc, %7, %8"
                                     : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                                       "+v"(x[6]), "+v"(x[7])
                                     : "v"(m)
                                     : "vcc");
                } else {
                    // carry in and out through one scalar register pair per chain
                    if (c == 0)
                        asm volatile("v_addc_co_u32_e64 %0, %8, %0, %16, %8\n\tv_addc_co_u32_e64 %1, %9, %1, %16, %9\n\t"
                                     "v_addc_co_u32_e64 %2, %10, %2, %16, %10\n\tv_addc_co_u32_e64 %3, %11, %3, %16, %11\n\t"
                                     "v_addc_co_u32_e64 %4, %12, %4, %16, %12\n\tv_addc_co_u32_e64 %5, %13, %5, %16, %13\n\t"
                                     "v_addc_co_u32_e64 %6, %14, %6, %16, %14\n\tv_addc_co_u32_e64 %7, %15, %7, %16, %15"
                                     : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]),
                                       "+v"(x[6]), "+v"(x[7]), "+s"(cy[0]), "+s"(cy[1]), "+s"(cy[2]), "+s"(cy[3]),
                                       "+s"(cy[4]), "+s"(cy[5]), "+s"(cy[6]), "+s"(cy[7])
                                     : "v"(m));
                }
            }
        }
    }
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        acc ^= y[c] ^ x[c] ^ cy[c];
    out[t] = acc;
}

}  // namespace mont

using namespace mont;

extern "C" mont_status_t mont_valu_ref(uint32_t kind, uint32_t iters, uint32_t blocks, void *out, void *stream)
{
    if (kind > 21 || !out || !blocks || blocks > (1u << 20))
        return fail(MONT_E_INVAL, "kind 0..21, 1 <= blocks <= 2^20, output of blocks * 256 uint64");
    hipStream_t s = (hipStream_t)stream;
    uint64_t *o = (uint64_t *)out;
    typedef void (*kfn)(uint32_t, uint32_t, uint64_t *);
    static const kfn kinds[22] = {k_valu<0>,  k_valu<1>,  k_valu<2>,  k_valu<3>,  k_valu<4>,  k_valu<5>,
                                  k_valu<6>,  k_valu<7>,  k_valu<8>,  k_valu<9>,  k_valu<10>, k_valu<11>,
                                  k_valu<12>, k_valu<13>, k_valu<14>, k_valu<15>, k_valu<16>, k_valu<17>,
                                  k_valu<18>, k_valu<19>, k_valu<20>, k_valu<21>};
    hipLaunchKernelGGL(kinds[kind], dim3(blocks), dim3(BLOCK), 0, s, iters, 12345u, o);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MONT_OK : hip_fail(e, "mont_valu_ref launch");
}
