// Device integer arithmetic for Montgomery-type reductions on gfx950.
//
// One reduction struct per (word size w, variant).  Each exposes
//   E    -- the w-bit residue type (signed for the signed variants)
//   TT   -- the 2w-bit input type of REDC
//   redc(T)   -- the reduction of a 2w-bit T
//   mul(a, b) -- redc(a * b), the Montgomery product
// and is built from the per-modulus constants in KCtx (held in scalar
// registers: every lane of a wave uses the same modulus).
//
// All reductions compute the paper's CRT quotient (T - mN)/R, or its negation
// (mN - T)/R for the Plantard family (Section 2, eq. qin4), with R a power of
// two so that "mod R" is a truncation and "/R" is taking a high word:
//
//   classic   (Section 1)       m = (T mod R) N' mod R,  t = (T + mN)/R,
//                               t >= N ? t - N : t.
//                               (T + mN)/R = hi(T) + hi(mN) + [lo(T) != 0],
//                               because lo(T) + lo(mN) is 0 or exactly R.
//   signed    (Algorithm 1)     m0 = a0 N^{-1} mods R (the low word of the
//                               product read as two's complement, which is the
//                               [-R/2, R/2) range of mods), t = floor(m0 N / R)
//                               = signed high word, r = a1 - t.
//   Plantard  (Algorithm 2)     R = 2^(2w): m = T N^{-1} mod R; only its high
//                               word is needed: q = floor(m / 2^w) + 1,
//                               r = floor(q N / 2^w) = high word of q N.  The
//                               r = N branch is dead (Remark in Section 3.2).
//   signed Plantard (Alg. 3)    m = T N^{-1} mods R; q = round(m / 2^w) =
//                               hi_s(m) + bit(w-1) of lo(m);
//                               r = round(q N / 2^w) = hi_s(qN) + bit(w-1) of lo(qN).
//   Algorithm 4 (alpha >= 1)    q = floor(m / 2^w) + 2^alpha, r = floor(q N / 2^w),
//                               evaluated as floor((hi_s(m) N + N 2^alpha) / 2^w)
//                               so the sum never leaves the wide type.
//
// Products wider than 32 bits are assembled from 32x32->64 partial products
// (v_mad_u64_u32) with explicit carry propagation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mont {

enum Variant { CLASSIC = 0, SIGNED = 1, PLANTARD = 2, SIGNED_PLANTARD = 3, SIGNED_PLANTARD_ALPHA = 4 };
constexpr int NVARIANT = 5;

// Per-modulus constants as the kernels see them (64 bytes, passed by value).
struct KCtx {
    uint64_t N;
    uint64_t nprime;  // 2^w - N^{-1} mod 2^w
    uint64_t ninv;    // N^{-1} mod 2^w
    uint64_t n2lo;    // N^{-1} mod 2^(2w), low 64 bits
    uint64_t n2hi;    // high 64 bits (w = 64)
    uint64_t r2;      // 2^(2w) mod N
    uint64_t rmodn;   // 2^w mod N
    uint32_t alpha;
    uint32_t w;
};

// Precomputed constants of a product by a fixed operand b (mont_mul_const).
// classic: b1 = b N' mod 2^w; signed: b1 = b N^{-1} mod 2^w; Plantard family:
// (b1, b2) = b N^{-1} mod 2^(2w) as (low, high) 64-bit words, b taken as a
// 2w-bit two's complement for the signed forms.  With them the quotient
// digit m = T N^{-1} mod R = a (b N^{-1}) mod R is formed from a alone.
struct KConst {
    uint64_t b;
    uint64_t b1;
    uint64_t b2;
};

struct u128v {
    uint64_t lo, hi;
};

// ---------------------------------------------------------------- 64-bit

// Full 64x64 -> 128 product from four 32x32 -> 64 partial products.
__device__ __forceinline__ u128v mul_64x64(uint64_t a, uint64_t b)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t t1 = (uint64_t)a1 * b0 + (p00 >> 32);          // < 2^64
    const uint64_t t2 = (uint64_t)a0 * b1 + (uint32_t)t1;         // < 2^64
    const uint64_t hi = (uint64_t)a1 * b1 + (t1 >> 32) + (t2 >> 32);
    return {(t2 << 32) | (uint32_t)p00, hi};
}

// a^2 with the cross product computed once.
__device__ __forceinline__ u128v sqr_64(uint64_t a)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint64_t p00 = (uint64_t)a0 * a0;
    const uint64_t p01 = (uint64_t)a0 * a1;
    const uint64_t p11 = (uint64_t)a1 * a1;
    // a^2 = p11 2^64 + 2 p01 2^32 + p00
    const uint64_t t1 = (p01 << 1) + (p00 >> 32);                 // may carry out of 64 bits
    const uint64_t c1 = ((p01 >> 63) & 1u) + (uint64_t)(t1 < (p01 << 1));
    const uint64_t hi = p11 + (t1 >> 32) + (c1 << 32);
    return {(t1 << 32) | (uint32_t)p00, hi};
}

__device__ __forceinline__ uint64_t mulhi_64(uint64_t a, uint64_t b) { return mul_64x64(a, b).hi; }

// 64 x 64 -> 128 for operands below 2^63 (a1, b1 < 2^31): the middle column
// a0 b1 + a1 b0 + hi(a0 b0) stays below 2^64, so no carry word is needed.
__device__ __forceinline__ u128v mul_63(uint64_t a, uint64_t b)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t mid = (uint64_t)a0 * b1 + ((uint64_t)a1 * b0 + (p00 >> 32));
    const uint64_t hi = (uint64_t)a1 * b1 + (mid >> 32);
    return {(mid << 32) | (uint32_t)p00, hi};
}

// a^2 for a below 2^63: 2 a1 fits in 32 bits and 2 a0 a1 + hi(a0^2) < 2^64.
__device__ __forceinline__ u128v sqr_63(uint64_t a)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint64_t p00 = (uint64_t)a0 * a0;
    const uint64_t mid = (uint64_t)a0 * (a1 << 1) + (p00 >> 32);
    const uint64_t hi = (uint64_t)a1 * a1 + (mid >> 32);
    return {(mid << 32) | (uint32_t)p00, hi};
}

// Signed product of two int64 as a 128-bit two's complement (lo, hi).
__device__ __forceinline__ u128v mul_s64(int64_t a, int64_t b)
{
    u128v p = mul_64x64((uint64_t)a, (uint64_t)b);
    p.hi -= (a < 0 ? (uint64_t)b : 0) + (b < 0 ? (uint64_t)a : 0);
    return p;
}

// Signed x (int64) times unsigned-but-below-2^63 N: 128-bit two's complement.
__device__ __forceinline__ u128v mul_s64_u63(int64_t x, uint64_t N)
{
    u128v p = mul_64x64((uint64_t)x, N);
    p.hi -= (x < 0 ? N : 0);
    return p;
}

// ----------------------------------------------------- reduction structs

template <int W, int V>
struct Red;

// ---------------------------------------------------------- w = 16

template <>
struct Red<16, CLASSIC> {
    using E = uint16_t;
    using TT = uint32_t;
    uint32_t N, np;
    uint16_t np16, N16;  // the same constants as 16-bit values (for 16-bit multiplies)
    __device__ __forceinline__ explicit Red(const KCtx &c)
        : N((uint32_t)c.N), np((uint32_t)c.nprime & 0xffffu), np16((uint16_t)c.nprime), N16((uint16_t)c.N)
    {
    }
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t tl = T & 0xffffu;
        const uint32_t m = (tl * np) & 0xffffu;
        const uint32_t t = (T >> 16) + ((m * N) >> 16) + (tl != 0u);  // < 2N
        return (E)(t >= N ? t - N : t);
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((uint32_t)a * (uint32_t)b); }
    __device__ __forceinline__ E sqr(E a) const { return mul(a, a); }
    // (T + mN)/R without the final subtraction, for N < 2^14 and a b < 4N^2:
    // T + mN < 2^30 + 2^30 fits a 32-bit word and the result is below
    // 4N^2/R + N <= 2N.  m is formed by a 16-bit multiply (only T mod R
    // matters), so T, m and T + mN take three instructions.
    __device__ __forceinline__ E mul_lazy(E a, E b) const
    {
        const uint32_t T = (uint32_t)a * (uint32_t)b;
        const uint16_t m = (uint16_t)((uint16_t)T * np16);
        return (E)(((uint32_t)m * (uint32_t)N16 + T) >> 16);
    }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint32_t T = (uint32_t)a * (uint32_t)k.b;
        const uint32_t m = ((uint32_t)a * (uint32_t)k.b1) & 0xffffu;   // (T mod R) N' mod R
        const uint32_t t = (T >> 16) + ((m * N) >> 16) + ((T & 0xffffu) != 0u);
        return (E)(t >= N ? t - N : t);
    }
};

template <>
struct Red<16, SIGNED> {
    using E = int16_t;
    using TT = int32_t;
    int32_t N;
    uint32_t ninv;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N((int32_t)c.N), ninv((uint32_t)c.ninv & 0xffffu) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t a0 = (uint32_t)T & 0xffffu;
        const int32_t a1 = T >> 16;                                   // floor(T / R)
        const int32_t m0 = (int32_t)(int16_t)(uint16_t)(a0 * ninv);   // a0 N^{-1} mods R
        const int32_t t = (m0 * N) >> 16;                             // floor(m0 N / R)
        return (E)(a1 - t);
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((int32_t)a * (int32_t)b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const int32_t T = (int32_t)a * (int32_t)(int16_t)k.b;
        const int32_t m0 = (int32_t)(int16_t)(uint16_t)((uint32_t)(int32_t)a * (uint32_t)k.b1);
        return (E)((T >> 16) - ((m0 * N) >> 16));
    }
};

template <>
struct Red<16, PLANTARD> {
    using E = uint16_t;
    using TT = uint32_t;
    uint32_t N, n2;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N((uint32_t)c.N), n2((uint32_t)c.n2lo) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t m = T * n2;              // T N^{-1} mod 2^32
        const uint32_t q = (m >> 16) + 1u;      // < 2^16 on the input range
        return (E)((q * N) >> 16);
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((uint32_t)a * (uint32_t)b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint32_t m = (uint32_t)a * (uint32_t)k.b1;   // a (b N^{-1}) mod 2^32: no product a b
        return (E)((((m >> 16) + 1u) * N) >> 16);
    }
};

template <>
struct Red<16, SIGNED_PLANTARD> {
    using E = int16_t;
    using TT = int32_t;
    int32_t N;
    uint32_t n2;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N((int32_t)c.N), n2((uint32_t)c.n2lo) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const int32_t m = (int32_t)((uint32_t)T * n2);        // T N^{-1} mods 2^32
        const int32_t q = (m >> 16) + ((m >> 15) & 1);        // round(m / 2^16), half up
        const int32_t p = q * N;
        return (E)((p >> 16) + ((p >> 15) & 1));              // round(q N / 2^16)
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((int32_t)a * (int32_t)b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const int32_t m = (int32_t)((uint32_t)(int32_t)a * (uint32_t)k.b1);
        const int32_t q = (m >> 16) + ((m >> 15) & 1);
        const int32_t p = q * N;
        return (E)((p >> 16) + ((p >> 15) & 1));
    }
};

template <>
struct Red<16, SIGNED_PLANTARD_ALPHA> {
    using E = int16_t;
    using TT = int32_t;
    int32_t N;
    uint32_t n2, alpha;
    __device__ __forceinline__ explicit Red(const KCtx &c)
        : N((int32_t)c.N), n2((uint32_t)c.n2lo), alpha(c.alpha) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const int32_t m = (int32_t)((uint32_t)T * n2);
        const int32_t p = (m >> 16) * N + (N << alpha);       // (floor(m/2^16) + 2^alpha) N
        return (E)(p >> 16);
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((int32_t)a * (int32_t)b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const int32_t m = (int32_t)((uint32_t)(int32_t)a * (uint32_t)k.b1);
        return (E)(((m >> 16) * N + (N << alpha)) >> 16);
    }
};

// ---------------------------------------------------------- w = 32

template <>
struct Red<32, CLASSIC> {
    using E = uint32_t;
    using TT = uint64_t;
    uint32_t N, np;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N((uint32_t)c.N), np((uint32_t)c.nprime) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t tl = (uint32_t)T, th = (uint32_t)(T >> 32);
        const uint32_t m = tl * np;
        const uint64_t t = (uint64_t)th + __umulhi(m, N) + (tl != 0u);   // < 2N
        return t >= N ? (uint32_t)(t - N) : (uint32_t)t;
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((uint64_t)a * b); }
    // Products of values in (-N, N) held as two's-complement words, N < 2^31:
    // with m = T N' mod 2^32 read as a signed word, T + m N is divisible by
    // 2^32 and |T + m N| < N^2 + 2^31 N < 2^32 N, so the quotient lies in
    // (-N, N) again and needs no correction (Algorithm 1's signed reduction,
    // with -N^{-1} in place of N^{-1}): three instructions per product.
    __device__ __forceinline__ E mul_signed(E a, E b) const
    {
        // Empty statements that hide the origins of T and m from the compiler:
        // without them it widens m's 32-bit multiply to a 64-bit one or forms
        // T's low word with an extra multiply (one to three more instructions).
        int64_t T = (int64_t)(int32_t)a * (int64_t)(int32_t)b;
        asm("" : "+v"(T));
        uint32_t m = (uint32_t)T * np;
        asm("" : "+v"(m));
        return (E)(uint32_t)(((int64_t)(int32_t)m * (int64_t)(int32_t)N + T) >> 32);
    }
    __device__ __forceinline__ E sqr(E a) const { return mul(a, a); }
    // Products for N < 2^31 and inputs below N: T + mN < 2^32 N + N^2 < 2^64,
    // so one multiply-add forms the whole sum, its high word t = (T + mN)/R is
    // below 2N < 2^32, and the unsigned min(t, t - N) is the reduced value
    // (t - N wraps above t when t < N).
    __device__ __forceinline__ E mul_fast(E a, E b) const
    {
        const uint64_t T = (uint64_t)a * b;
        const uint32_t m = (uint32_t)T * np;
        const uint32_t t = (uint32_t)(((uint64_t)m * N + T) >> 32);
        return min(t, t - N);
    }
    // (T + mN)/R without the final subtraction, for N < 2^30 and a b < 4N^2
    // (say a < 4N and b < N, or both below 2N): T + mN < 4N^2 + 2^32 N < 2^63
    // and the result is below 4N^2/R + N <= 2N.
    __device__ __forceinline__ E mul_lazy(E a, E b) const
    {
        const uint64_t T = (uint64_t)a * b;
        const uint32_t m = (uint32_t)T * np;
        return (uint32_t)(((uint64_t)m * N + T) >> 32);
    }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint64_t T = (uint64_t)a * (uint32_t)k.b;
        const uint32_t tl = (uint32_t)T, th = (uint32_t)(T >> 32);
        const uint32_t m = a * (uint32_t)k.b1;
        const uint64_t t = (uint64_t)th + __umulhi(m, N) + (tl != 0u);
        return t >= N ? (uint32_t)(t - N) : (uint32_t)t;
    }
};

template <>
struct Red<32, SIGNED> {
    using E = int32_t;
    using TT = int64_t;
    int32_t N;
    uint32_t ninv;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N((int32_t)c.N), ninv((uint32_t)c.ninv) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t a0 = (uint32_t)T;
        const int32_t a1 = (int32_t)(T >> 32);
        const int32_t m0 = (int32_t)(a0 * ninv);
        return a1 - __mulhi(m0, N);
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((int64_t)a * b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const int64_t T = (int64_t)a * (int32_t)(uint32_t)k.b;
        const int32_t m0 = (int32_t)((uint32_t)a * (uint32_t)k.b1);
        return (int32_t)(T >> 32) - __mulhi(m0, N);
    }
};

template <>
struct Red<32, PLANTARD> {
    using E = uint32_t;
    using TT = uint64_t;
    uint32_t N, nl, nh;
    __device__ __forceinline__ explicit Red(const KCtx &c)
        : N((uint32_t)c.N), nl((uint32_t)c.n2lo), nh((uint32_t)(c.n2lo >> 32)) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t tl = (uint32_t)T, th = (uint32_t)(T >> 32);
        const uint32_t mh = __umulhi(tl, nl) + tl * nh + th * nl;   // floor((T N^{-1} mod 2^64) / 2^32)
        return __umulhi(mh + 1u, N);
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((uint64_t)a * b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint32_t bl = (uint32_t)k.b1, bh = (uint32_t)(k.b1 >> 32);
        const uint32_t mh = __umulhi(a, bl) + a * bh;   // floor((a (b N^{-1}) mod 2^64) / 2^32)
        return __umulhi(mh + 1u, N);
    }
};

template <>
struct Red<32, SIGNED_PLANTARD> {
    using E = int32_t;
    using TT = int64_t;
    int32_t N;
    uint32_t nl, nh;
    __device__ __forceinline__ explicit Red(const KCtx &c)
        : N((int32_t)c.N), nl((uint32_t)c.n2lo), nh((uint32_t)(c.n2lo >> 32)) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t tl = (uint32_t)T, th = (uint32_t)((uint64_t)T >> 32);
        const uint32_t ml = tl * nl;
        const uint32_t mh = __umulhi(tl, nl) + tl * nh + th * nl;
        const int32_t q = (int32_t)mh + (int32_t)(ml >> 31);        // round(m / 2^32)
        const int64_t p = (int64_t)q * N;
        return (int32_t)(p >> 32) + (int32_t)((uint32_t)p >> 31);   // round(q N / 2^32)
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((int64_t)a * b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint64_t m = (uint64_t)(int64_t)a * k.b1;  // a (b N^{-1}) mod 2^64, two's complement
        const int32_t q = (int32_t)(uint32_t)(m >> 32) + (int32_t)((uint32_t)m >> 31);
        const int64_t p = (int64_t)q * N;
        return (int32_t)(p >> 32) + (int32_t)((uint32_t)p >> 31);
    }
};

template <>
struct Red<32, SIGNED_PLANTARD_ALPHA> {
    using E = int32_t;
    using TT = int64_t;
    int32_t N;
    uint32_t nl, nh, alpha;
    __device__ __forceinline__ explicit Red(const KCtx &c)
        : N((int32_t)c.N), nl((uint32_t)c.n2lo), nh((uint32_t)(c.n2lo >> 32)), alpha(c.alpha) {}
    __device__ __forceinline__ E redc(TT T) const
    {
        const uint32_t tl = (uint32_t)T, th = (uint32_t)((uint64_t)T >> 32);
        const uint32_t mh = __umulhi(tl, nl) + tl * nh + th * nl;
        const int64_t p = (int64_t)(int32_t)mh * N + ((int64_t)N << alpha);
        return (int32_t)(p >> 32);
    }
    __device__ __forceinline__ E mul(E a, E b) const { return redc((int64_t)a * b); }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint64_t m = (uint64_t)(int64_t)a * k.b1;
        const int64_t p = (int64_t)(int32_t)(uint32_t)(m >> 32) * N + ((int64_t)N << alpha);
        return (int32_t)(p >> 32);
    }
};

// ---------------------------------------------------------- w = 64

struct T128 {
    uint64_t lo, hi;
};

template <>
struct Red<64, CLASSIC> {
    using E = uint64_t;
    using TT = T128;
    uint64_t N, np;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N(c.N), np(c.nprime) {}
    __device__ __forceinline__ E reduce(uint64_t tl, uint64_t th) const
    {
        const uint64_t m = tl * np;
        const uint64_t mh = mulhi_64(m, N);
        // t = th + mh + [tl != 0] < 2N, which may need 65 bits when N > 2^63
        const uint64_t s = th + mh;
        const uint64_t t = s + (tl != 0u);
        const bool carry = (s < th) | (t < s);
        return (carry | (t >= N)) ? t - N : t;
    }
    __device__ __forceinline__ E redc(TT T) const { return reduce(T.lo, T.hi); }
    __device__ __forceinline__ E mul(E a, E b) const
    {
        const u128v p = mul_64x64(a, b);
        return reduce(p.lo, p.hi);
    }
    __device__ __forceinline__ E sqr(E a) const
    {
        const u128v p = sqr_64(a);
        return reduce(p.lo, p.hi);
    }
    // (T + mN)/R without the final subtraction: for N < 2^62 and inputs below
    // 2N the result is below 2N (the sum T + mN < 2RN never leaves 128 bits).
    // With n1 = hi(N) < 2^30, floor(mN/R) = m1 n1 + hi(y) + hi(z) for
    // x = m0 n0, y = m1 n0 + hi(x) < 2^64 and z = m0 n1 + lo(y) < 2^62 + 2^32,
    // and th < 2^62, so every partial sum fits in 64 bits.
    __device__ __forceinline__ E reduce_lazy(uint64_t tl, uint64_t th) const
    {
        const uint64_t m = tl * np;
        const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
        const uint32_t n0 = (uint32_t)N, n1 = (uint32_t)(N >> 32);
        const uint64_t x = (uint64_t)m0 * n0;
        const uint64_t y = (uint64_t)m1 * n0 + (x >> 32);
        const uint64_t z = (uint64_t)m0 * n1 + (uint32_t)y;
        const uint64_t w = (uint64_t)m1 * n1 + (th + (y >> 32));
        // w + hi(z) + [tl != 0] as one 32-bit carry chain
        unsigned int c;
        const uint32_t lo = __builtin_addc((uint32_t)w, (uint32_t)(z >> 32), (unsigned int)(tl != 0u), &c);
        return ((uint64_t)((uint32_t)(w >> 32) + c) << 32) | lo;
    }
    __device__ __forceinline__ E mul_fast(E a, E b) const
    {
        const u128v p = mul_63(a, b);
        return reduce_lazy(p.lo, p.hi);
    }
    __device__ __forceinline__ E sqr_fast(E a) const
    {
        const u128v p = sqr_63(a);
        return reduce_lazy(p.lo, p.hi);
    }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const u128v p = mul_64x64(a, k.b);
        const uint64_t m = a * k.b1;
        const uint64_t s = p.hi + mulhi_64(m, N);
        const uint64_t t = s + (p.lo != 0u);
        const bool carry = (s < p.hi) | (t < s);
        return (carry | (t >= N)) ? t - N : t;
    }
};

template <>
struct Red<64, SIGNED> {
    using E = int64_t;
    using TT = T128;
    uint64_t N, ninv;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N(c.N), ninv(c.ninv) {}
    __device__ __forceinline__ E reduce(uint64_t tl, uint64_t th) const
    {
        const int64_t m0 = (int64_t)(tl * ninv);                 // a0 N^{-1} mods 2^64
        const int64_t t = (int64_t)mul_s64_u63(m0, N).hi;        // floor(m0 N / 2^64)
        return (int64_t)(th - (uint64_t)t);                      // a1 - t
    }
    __device__ __forceinline__ E redc(TT T) const { return reduce(T.lo, T.hi); }
    __device__ __forceinline__ E mul(E a, E b) const
    {
        const u128v p = mul_s64(a, b);
        return reduce(p.lo, p.hi);
    }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const u128v p = mul_s64(a, (int64_t)k.b);
        const int64_t m0 = (int64_t)((uint64_t)a * k.b1);
        return (int64_t)(p.hi - mul_s64_u63(m0, N).hi);
    }
};

template <>
struct Red<64, PLANTARD> {
    using E = uint64_t;
    using TT = T128;
    uint64_t N, nl, nh;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N(c.N), nl(c.n2lo), nh(c.n2hi) {}
    __device__ __forceinline__ E reduce(uint64_t tl, uint64_t th) const
    {
        const uint64_t mh = mulhi_64(tl, nl) + tl * nh + th * nl;  // floor((T N^{-1} mod 2^128) / 2^64)
        return mulhi_64(mh + 1u, N);
    }
    __device__ __forceinline__ E redc(TT T) const { return reduce(T.lo, T.hi); }
    __device__ __forceinline__ E mul(E a, E b) const
    {
        const u128v p = mul_64x64(a, b);
        return reduce(p.lo, p.hi);
    }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint64_t mh = mulhi_64(a, k.b1) + a * k.b2;   // floor((a (b N^{-1}) mod 2^128) / 2^64)
        return mulhi_64(mh + 1u, N);
    }
};

template <>
struct Red<64, SIGNED_PLANTARD> {
    using E = int64_t;
    using TT = T128;
    uint64_t N, nl, nh;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N(c.N), nl(c.n2lo), nh(c.n2hi) {}
    __device__ __forceinline__ E reduce(uint64_t tl, uint64_t th) const
    {
        const u128v ml = mul_64x64(tl, nl);
        const uint64_t mh = ml.hi + tl * nh + th * nl;
        const int64_t q = (int64_t)mh + (int64_t)(ml.lo >> 63);  // round(m / 2^64)
        const u128v p = mul_s64_u63(q, N);
        return (int64_t)(p.hi + (p.lo >> 63));                   // round(q N / 2^64)
    }
    __device__ __forceinline__ E redc(TT T) const { return reduce(T.lo, T.hi); }
    __device__ __forceinline__ E mul(E a, E b) const
    {
        const u128v p = mul_s64(a, b);
        return reduce(p.lo, p.hi);
    }
    // a as a 128-bit two's complement: (a_lo, a < 0 ? 2^64 - 1 : 0)
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const u128v ml = mul_64x64((uint64_t)a, k.b1);
        const uint64_t mh = ml.hi + (uint64_t)a * k.b2 - (a < 0 ? k.b1 : 0);
        const int64_t q = (int64_t)mh + (int64_t)(ml.lo >> 63);
        const u128v p = mul_s64_u63(q, N);
        return (int64_t)(p.hi + (p.lo >> 63));
    }
};

template <>
struct Red<64, SIGNED_PLANTARD_ALPHA> {
    using E = int64_t;
    using TT = T128;
    uint64_t N, nl, nh;
    uint32_t alpha;
    __device__ __forceinline__ explicit Red(const KCtx &c) : N(c.N), nl(c.n2lo), nh(c.n2hi), alpha(c.alpha) {}
    __device__ __forceinline__ E reduce(uint64_t tl, uint64_t th) const
    {
        const uint64_t mh = mulhi_64(tl, nl) + tl * nh + th * nl;
        u128v p = mul_s64_u63((int64_t)mh, N);                   // floor(m / 2^64) N
        const uint64_t add = N << alpha;                          // < 2^63
        const uint64_t lo = p.lo + add;
        p.hi += (lo < add);
        return (int64_t)p.hi;                                     // floor(. / 2^64)
    }
    __device__ __forceinline__ E redc(TT T) const { return reduce(T.lo, T.hi); }
    __device__ __forceinline__ E mul(E a, E b) const
    {
        const u128v p = mul_s64(a, b);
        return reduce(p.lo, p.hi);
    }
    __device__ __forceinline__ E mul_const(E a, const KConst &k) const
    {
        const uint64_t mh = mulhi_64((uint64_t)a, k.b1) + (uint64_t)a * k.b2 - (a < 0 ? k.b1 : 0);
        u128v p = mul_s64_u63((int64_t)mh, N);
        const uint64_t add = N << alpha;
        const uint64_t lo = p.lo + add;
        p.hi += (lo < add);
        return (int64_t)p.hi;
    }
};

}  // namespace mont
