// Precondition checks of MONT_DEBUG builds.  Each algorithm states the range
// of inputs it is defined on (its Require line; Section 1 for classic REDC):
//   classic REDC            0 <= T < N R                 (R = 2^w)
//   Algorithm 1 (signed)    -N R/2 < T < N R/2
//   Algorithm 2 (Plantard)  0 <= T <= N^2
//   Algorithm 3             |T| <= 2^(2n-2)              (n = w)
//   Algorithm 4             |T| <= 2^(2 alpha) N^2
// A product a b is an input T of its variant; exponentiation, NTT and CRT
// operands must be residues below their modulus.  Debug builds count the
// elements that break these ranges (the release library never checks them:
// there the output for such elements is unspecified).
#pragma once

#include "mont_common.hpp"

namespace mont {

typedef unsigned __int128 dbg_u128;

// |T| = mag with sign neg: inside the variant's Require range?
__host__ __device__ inline bool dbg_t_in_range(int variant, uint32_t w, uint64_t N, uint32_t alpha, bool neg,
                                               dbg_u128 mag)
{
    const dbg_u128 n2 = (dbg_u128)N * N;  // Algorithms 2-4 need N < 2^(w-1), so no overflow there
    switch (variant) {
    case CLASSIC:
        return (!neg || mag == 0) && mag < ((dbg_u128)N << w);
    case SIGNED:
        return mag < ((dbg_u128)N << (w - 1));
    case PLANTARD:
        return (!neg || mag == 0) && mag <= n2;
    case SIGNED_PLANTARD:
        return mag <= ((dbg_u128)1 << (2 * w - 2));
    default:
        return mag <= (n2 << (2 * alpha));
    }
}

// The product a b of two w-bit operands (two's complement for the signed
// variants) as sign and magnitude.
__host__ __device__ inline void dbg_product(int variant, uint32_t w, uint64_t a, uint64_t b, bool *neg, dbg_u128 *mag)
{
    const bool sgn = variant == SIGNED || variant == SIGNED_PLANTARD || variant == SIGNED_PLANTARD_ALPHA;
    uint64_t ua = a, ub = b;
    bool na = false, nb = false;
    if (sgn) {
        const uint64_t top = 1ull << (w - 1), mask = w == 64 ? ~0ull : (1ull << w) - 1;
        if (a & top) {
            na = true;
            ua = (~a + 1) & mask;  // |a| of a negative w-bit value (2^(w-1) stays 2^(w-1))
        }
        if (b & top) {
            nb = true;
            ub = (~b + 1) & mask;
        }
    }
    *neg = na != nb;
    *mag = (dbg_u128)ua * ub;
}

enum DbgKind {
    DBG_PRODUCT = 0,  // in0[i] in1[i] (w-bit operands)
    DBG_CONST = 1,    // in0[i] b (b passed as a value)
    DBG_T = 2,        // in0[i], a 2w-bit T
    DBG_BELOW_N = 3,  // in0[i] < N (w-bit residues)
};

// Counts (into the device counter read by mont_debug_violations) the
// elements of one call that break their range; enqueued on `s` ahead of the
// call's own kernel.
hipError_t debug_check(int kind, const mont_ctx_t &c, int variant, const void *in0, const void *in1, uint64_t b,
                       uint64_t n, hipStream_t s);

// Host-side count for operands that live in host memory (serving jobs).
void debug_count_host(uint64_t k);

}  // namespace mont
