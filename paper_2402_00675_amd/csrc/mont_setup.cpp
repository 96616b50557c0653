// Per-modulus constants (host).  Section 1 defines N' = R - (N^{-1} mod R);
// Algorithms 1-4 use N^{-1} mods R and N^{-1} mod 2^(2w).
//
// N^{-1} modulo 2^128 comes from Newton-Hensel lifting x <- x (2 - N x),
// which doubles the number of correct low bits each step (an odd N is its own
// inverse modulo 8, so six steps give 3 * 2^6 = 192 >= 128 bits).  The result
// is checked against Qin's identity (Theorem 2.1) in the form of its proof:
// N^{-1} N = 1 + l R with l < N, and (N - l) R = 1 (mod N).
#include <cstring>

#include "mont_common.hpp"

namespace mont {

typedef unsigned __int128 u128;

mont_status_t setup_ctx(uint64_t N, uint32_t w, mont_ctx_t *ctx)
{
    if (!ctx)
        return fail(MONT_E_INVAL, "null context");
    if (w != 16 && w != 32 && w != 64)
        return fail(MONT_E_INVAL, "log2R must be 16, 32 or 64 (got %u)", w);
    if (N < 3 || !(N & 1u) || (w < 64 && (N >> w)))
        return fail(MONT_E_INVAL, "N must be odd with 3 <= N < 2^%u", w);
    std::memset(ctx, 0, sizeof *ctx);

    u128 x = N;
    for (int i = 0; i < 6; ++i)
        x = x * (2 - (u128)N * x);
    const u128 one = 1;
    const u128 maskw = w == 64 ? ~(u128)0 >> 64 : (one << w) - 1;
    const uint64_t ninv = (uint64_t)(x & maskw);
    const u128 inv2 = w == 64 ? x : (x & ((one << (2 * w)) - 1));

    const uint64_t r_mod_n = (uint64_t)((one << w) % N);
    const uint64_t r2_mod_n = (uint64_t)(((u128)r_mod_n * r_mod_n) % N);

    // Theorem 2.1 (Qin's identity) in its proof's form
    const u128 prod = (u128)ninv * N;  // = 1 + l R
    if ((prod & maskw) != 1)
        return fail(MONT_E_INVAL, "internal: N^{-1} mod R failed for N=%llu", (unsigned long long)N);
    const u128 l = (prod - 1) >> w;
    if (!(l < N) || (((u128)(N - (uint64_t)l) * r_mod_n) % N) != 1)
        return fail(MONT_E_INVAL, "internal: Qin's identity failed for N=%llu", (unsigned long long)N);

    ctx->N = N;
    ctx->w = w;
    ctx->ninv = ninv;
    ctx->nprime = (uint64_t)(((one << w) - ninv) & maskw);
    ctx->ninv2_lo = (uint64_t)inv2;
    ctx->ninv2_hi = w == 64 ? (uint64_t)(inv2 >> 64) : 0;
    ctx->r_mod_n = r_mod_n;
    ctx->r2_mod_n = r2_mod_n;

    uint32_t valid = 1u << CLASSIC;
    const u128 half = one << (w - 1);
    if ((u128)N < half) {
        valid |= 1u << SIGNED;          // 2N < R (Algorithm 1)
        valid |= 1u << SIGNED_PLANTARD; // N < 2^(w-1) (Algorithm 3)
    }
    // Algorithm 2: N < 2^w / phi  <=>  N^2 < (2^w - N) 2^w
    if ((u128)N * N < (((one << w) - N) << w))
        valid |= 1u << PLANTARD;
    // Algorithm 4 with alpha = 1: N < 2^(w-2)
    if ((u128)N < (one << (w - 2))) {
        valid |= 1u << SIGNED_PLANTARD_ALPHA;
        ctx->alpha = 1;
    }
    ctx->valid = valid;
    return MONT_OK;
}

}  // namespace mont
