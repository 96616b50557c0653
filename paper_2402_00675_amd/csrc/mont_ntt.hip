// Batched number-theoretic transforms whose butterflies use the library's
// reductions (the application that motivates Montgomery-type algorithms in
// Sections 1 and 3).
//
// Forward:  X_k = sum_j x_j w^(j k) mod N,  inverse: x_j = n^{-1} sum_k X_k w^(-j k) mod N,
// for a root w with w^(n/2) = -1 (mod N), n = 2^log2n <= 4096, on `batch`
// polynomials of n residues in [0, N) stored contiguously (natural order in
// and out, in place).
//
// Lengths 2 to 1024 (k_nttw): one wavefront per max(n, 256) coefficients,
// loaded from HBM straight into registers in bit-reversed order and exchanged
// between radix-4 steps through a conflict-free LDS layout.  Lengths 2048 and
// 4096 (k_nttm): one workgroup of four wavefronts per polynomial, each taking
// a quarter of the 256-position blocks through the same steps, then trading
// through LDS so that the stages across blocks run in registers.  The
// twiddle product is a product by a fixed operand:
//   classic  -- Montgomery product with w^k R mod N;
//   Plantard -- Plantard product with b = -w^k 2^(2w) mod N through the
//               precomputed b N^{-1} mod 2^(2w) (mont_mul_const), so the
//               product never forms a b (Section 3.2's operand saving).
// Twiddles are computed once per (N, w, root, n, variant, direction) on the
// host and kept in library-owned device memory.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "mont_common.hpp"
#ifdef MONT_DEBUG
#include "mont_debug.hpp"
#endif

namespace mont {

// FAST: N < 2^(w-1), so sums of two residues fit a word (branch-free modular
// add and subtract below); with classic twiddles it also means N < 2^31 at
// w = 32 or N < 2^62 at w = 64, the ladder's smaller-modulus products (the
// 64-bit one is lazy, below 2N, so one conditional subtraction follows), and
// at w = 16 the three-instruction lazy product and one subtraction.
template <class R, int V, bool FAST>
__device__ __forceinline__ typename R::E tw_mul(const R &red, typename R::E a, const KConst &w)
{
    using El = typename R::E;
    if constexpr (V == CLASSIC && FAST && sizeof(El) == 8) {
        const El u = red.mul_fast(a, (El)w.b);
        return u >= red.N ? u - red.N : u;
    } else if constexpr (V == CLASSIC && FAST && sizeof(El) == 4) {
        return red.mul_fast(a, (El)w.b);
    } else if constexpr (V == CLASSIC && FAST && sizeof(El) == 2) {
        // N < 2^15, a, b < N: T + mN < 2^30 + 2^31 fits 32 bits and the quotient is below 2N
        const El t = red.mul_lazy(a, (El)w.b), d = (El)(t - (El)red.N);
        return d < t ? d : t;
    } else if constexpr (V == CLASSIC) {
        return red.mul(a, (El)w.b);
    } else {
        return red.mul_const(a, w);
    }
}

template <class El, bool FAST>
__device__ __forceinline__ El add_mod(El u, El t, El N)
{
    const El s = (El)(u + t);
    if constexpr (FAST) {
        const El d = (El)(s - N);  // s < 2N <= 2^w: s - N wraps above s exactly when s < N
        return d < s ? d : s;
    } else {
        return (s < u || s >= N) ? (El)(s - N) : s;  // s < u: the sum wrapped (N > 2^(w-1))
    }
}

template <class El, bool FAST>
__device__ __forceinline__ El sub_mod(El u, El t, El N)
{
    if constexpr (FAST) {
        const El d = (El)(u - t), e = (El)(d + N);  // u < t: d wrapped and d + N < d
        return e < d ? e : d;
    } else {
        return u >= t ? (El)(u - t) : (El)(u + (N - t));
    }
}

// Twiddle as kept in device memory and LDS: what tw_mul needs of a KConst,
// nothing more (8 bytes, 16 for the 64-bit Plantard form).
template <int W, int V>
struct TwL {
    uint64_t b;  // classic: w^k R mod N; Plantard (w <= 32): b N^{-1} mod 2^(2w)
    static TwL from(const KConst &k) { return {V == CLASSIC ? k.b : k.b1}; }
    __device__ __forceinline__ KConst get() const
    {
        KConst k{};
        if constexpr (V == CLASSIC)
            k.b = b;
        else
            k.b1 = b;
        return k;
    }
};
template <>
struct TwL<64, PLANTARD> {
    uint64_t b1, b2;
    static TwL from(const KConst &k) { return {k.b1, k.b2}; }
    __device__ __forceinline__ KConst get() const
    {
        KConst k{};
        k.b1 = b1;
        k.b2 = b2;
        return k;
    }
};

// The kernels' LAZY argument picks the butterfly.  LAZY = 0: every sum and
// difference reduced modulo N.
//
// LAZY = 1 (classic twiddles, 4N <= 2^w: N < 2^14 at w = 16, N < 2^30 at
// w = 32, N < 2^61 at w = 64, the latter so that operands stay below 2^63):
// coefficients live in [0, 4N) between stages.  The twiddle product without
// its final subtraction is below 4N^2/R + N <= 2N; u is brought below 2N by
// one conditional subtraction; then u + t and u - t + 2N both lie in [0, 4N)
// with no further correction (the lazy butterfly of Harvey's NTT).  Results
// are reduced to [0, N) once, when they are written out.
//
// LAZY = 2 (the same products, for moduli far below the word): u is not
// reduced at all.  With t < 2N, u + t and u - t + 2N lie in (0, B + 2N) when
// u lies in [0, B), so each stage raises the bound by 2N: inputs below N,
// below 3N after stage 0 (no products), 5N after stage 1 (its products see
// operands below 3N) and (2L + 1) N after L >= 2 stages.  Taken when that
// final bound fits the word (and stays below 2^63 at w = 64, the product's
// operand limit); the product then still ends below 2N (a b < R N), and the
// results are reduced by one product with 1 or n^{-1} in Montgomery form.
//
// LAZY = 3 (Plantard twiddles, N <= 2^(w-1)): the product by a fixed operand
// (m = a (b N^{-1}) mod 2^(2w), r = floor((floor(m / 2^w) + 1) N / 2^w)) is
// exact for every w-bit a, not only below N.  With k = (m N - T) / 2^(2w),
// T = a b, k is an integer in [0, N), congruent to -T 2^(-2w), and
// (floor(m / 2^w) + 1) N / 2^w lies in (k + T/2^(2w), k + T/2^(2w) + N/2^w],
// inside (k, k + 1) when T < 2^w (2^w - N), which a < 2^w and b < N <= 2^(w-1)
// guarantee: r = k.  So t is in [0, N), u + t and u - t + N need no
// reduction, and each stage raises the bound by N (below 3N after stage 0,
// 4N after stage 1, (L + 2) N after L stages).  Taken when that fits the word;
// the outputs are reduced by the same product with 1 or n^{-1}.
template <class R>
__device__ __forceinline__ typename R::E lazy_mul(const R &red, typename R::E a, typename R::E b)
{
    return red.mul_lazy(a, b);
}
template <>
__device__ __forceinline__ uint64_t lazy_mul(const Red<64, CLASSIC> &red, uint64_t a, uint64_t b)
{
    return red.mul_fast(a, b);  // the 64-bit ladder product is already lazy
}

template <class El>
__device__ __forceinline__ El below(El x, El m)  // x < 2m  ->  x mod m
{
    const El d = (El)(x - m);
    return d < x ? d : x;
}

template <class R, int V, bool FAST, int LAZY, class T>
__device__ __forceinline__ void butterfly(const R &red, typename R::E &u, typename R::E &v, const T &w,
                                          typename R::E N)
{
    using El = typename R::E;
    if constexpr (LAZY == 3) {
        const El t = tw_mul<R, V, FAST>(red, v, w.get());
        const El x = u;
        u = (El)(x + t);
        v = (El)((El)(x + N) - t);
    } else if constexpr (LAZY) {
        const El t = lazy_mul(red, v, (El)w.get().b);
        const El x = LAZY == 2 ? u : below<El>(u, (El)(2 * N));
        u = (El)(x + t);
        v = (El)((El)(x + 2 * N) - t);
    } else {
        const El t = tw_mul<R, V, FAST>(red, v, w.get());
        const El x = u;
        u = add_mod<El, FAST>(x, t, N);
        v = sub_mod<El, FAST>(x, t, N);
    }
}

// Workgroups per CU launched for the one-wave-per-unit kernel (its waves loop
// over the batch, the next unit's loads in flight).  Measured on MI355X over
// 2^26 coefficients: up to length 256 (one block of 256 positions per unit)
// 32 per CU beat 8 by 3-12 % at every width (more than the CU holds at once,
// so the dispatcher refills CUs as workgroups finish; 64 was no better and one
// unit per wave, with nothing prefetched, up to 2.4x slower); at 512 and 1024
// (two and four blocks per unit) 8 stayed best or within 1 %.
__host__ __device__ constexpr int nttw_bpc(uint32_t log2n) { return log2n <= 8 ? 32 : 8; }

// Butterfly by the unit twiddle (the first two stages of a bit-reversed
// decimation-in-time transform multiply by 1 or by w^(n/4) only).  LAZY:
// u, v < 2N give u + v < 4N and u - v + 2N in (0, 4N).
template <class El, bool FAST, int LAZY>
__device__ __forceinline__ void butterfly1(El &u, El &v, El N)
{
    const El x = u;
    if constexpr (LAZY) {
        u = (El)(x + v);
        v = (El)((El)(x + 2 * N) - v);
    } else {
        u = add_mod<El, FAST>(x, v, N);
        v = sub_mod<El, FAST>(x, v, N);
    }
}

// Four coefficients of one lane into its 4 consecutive LDS slots, one LDS
// write (two for 64-bit words).
template <class El>
__device__ __forceinline__ void lds_put4(El *p, const El (&a)[4])
{
    if constexpr (sizeof(El) == 2) {
        uint2 v;
        v.x = (uint32_t)a[0] | ((uint32_t)a[1] << 16);
        v.y = (uint32_t)a[2] | ((uint32_t)a[3] << 16);
        *(uint2 *)p = v;
    } else if constexpr (sizeof(El) == 4) {
        *(uint4 *)p = make_uint4(a[0], a[1], a[2], a[3]);
    } else {
        *(ulonglong2 *)p = make_ulonglong2(a[0], a[1]);
        *(ulonglong2 *)(p + 2) = make_ulonglong2(a[2], a[3]);
    }
}

// Between exchange steps the lanes of one wavefront read LDS words other lanes
// of the same wavefront wrote: a release fence, the wavefront barrier and an
// acquire fence, all at wavefront scope, order those writes before the reads
// under the memory model (a wave's LDS accesses complete in order, so this
// costs no wait; it keeps the compiler from moving the accesses across it).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The four radix-4 steps (stages 0..7, those below L) of NB blocks of 256
// positions held by one wavefront, four positions per lane in each (lane maps
// and LDS layout at k_nttw); block b goes through the 256 LDS words at
// sb + 256 b, and the blocks' steps interleave.  tw9: the lane's twiddles of
// stages 1..7 in the order t01, t10, t11, t12, t20, t21, t22, t30, t31, t32
// (stage 0 and half of stage 1 multiply by 1).  On return a[b][k] holds
// position lane + 64 k of block b.
template <class R, int V, bool FAST, int LAZY, int NB, int L, class T>
__device__ __forceinline__ void block_steps(const R &red, typename R::E (&a)[NB][4], typename R::E *sb,
                                            uint32_t lane, uint32_t base1, uint32_t base2, uint32_t base3,
                                            const T (&tw9)[10], typename R::E N)
{
    using El = typename R::E;
    constexpr bool H1 = L > 1, H2 = L > 2, H3 = L > 3, H4 = L > 4, H5 = L > 5, H6 = L > 6, H7 = L > 7;  // stage st exists
    // step 0: stage 0 (unit twiddles), stage 1 (1 and w^(n/4))
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        butterfly1<El, FAST, LAZY>(a[b][0], a[b][1], N);
        butterfly1<El, FAST, LAZY>(a[b][2], a[b][3], N);
        if constexpr (H1) {
            butterfly1<El, FAST, LAZY>(a[b][0], a[b][2], N);
            butterfly<R, V, FAST, LAZY>(red, a[b][1], a[b][3], tw9[0], N);
        }
        lds_put4<El>(sb + 256 * b + 4 * lane, a[b]);
    }
    wave_lds_sync();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const El *q = sb + 256 * b;
        a[b][0] = q[base1];
        a[b][1] = q[base1 + 128];
        a[b][2] = q[base1 + 64];
        a[b][3] = q[base1 + 192];
    }
    wave_lds_sync();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if constexpr (H2) {
            butterfly<R, V, FAST, LAZY>(red, a[b][0], a[b][1], tw9[1], N);
            butterfly<R, V, FAST, LAZY>(red, a[b][2], a[b][3], tw9[1], N);
        }
        if constexpr (H3) {
            butterfly<R, V, FAST, LAZY>(red, a[b][0], a[b][2], tw9[2], N);
            butterfly<R, V, FAST, LAZY>(red, a[b][1], a[b][3], tw9[3], N);
        }
        lds_put4<El>(sb + 256 * b + 4 * lane, a[b]);
    }
    wave_lds_sync();
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            a[b][k] = sb[256 * b + base2 + 64 * k];
    wave_lds_sync();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if constexpr (H4) {
            butterfly<R, V, FAST, LAZY>(red, a[b][0], a[b][1], tw9[4], N);
            butterfly<R, V, FAST, LAZY>(red, a[b][2], a[b][3], tw9[4], N);
        }
        if constexpr (H5) {
            butterfly<R, V, FAST, LAZY>(red, a[b][0], a[b][2], tw9[5], N);
            butterfly<R, V, FAST, LAZY>(red, a[b][1], a[b][3], tw9[6], N);
        }
        lds_put4<El>(sb + 256 * b + 4 * lane, a[b]);
    }
    wave_lds_sync();
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < 4; ++k)
            a[b][k] = sb[256 * b + base3 + 64 * k];
    wave_lds_sync();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if constexpr (H6) {
            butterfly<R, V, FAST, LAZY>(red, a[b][0], a[b][1], tw9[7], N);
            butterfly<R, V, FAST, LAZY>(red, a[b][2], a[b][3], tw9[7], N);
        }
        if constexpr (H7) {
            butterfly<R, V, FAST, LAZY>(red, a[b][0], a[b][2], tw9[8], N);
            butterfly<R, V, FAST, LAZY>(red, a[b][1], a[b][3], tw9[9], N);
        }
    }
}

// Lengths n = 2^L, 1 <= L <= 10: one wavefront per unit of max(n, 256)
// consecutive coefficients, no workgroup barriers.
//
// A unit is one polynomial when n >= 256 and 256/n polynomials side by side
// when n < 256; below, "positions" are those of the unit's bit-reversed array
// (each polynomial reversed within itself).  In a decimation-in-time transform
// stage st pairs positions that differ in bit st, with the twiddle
// w^(j n / 2^(st+1)) = tw[j << (L - 1 - st)] at position j mod 2^st.  Stages
// L..7 do not exist when n < 256 and are skipped (the polynomials of a unit
// never mix).  When n = 256 G, G = 2 or 4, the first eight stages act on G
// separate blocks of 256 positions; block b holds the coefficients
// x[brev(b) + G m], m = 0..255 (brev over log2 G bits), so the G values a
// lane needs for one slot of all blocks are G consecutive words; after those
// stages the remaining log2 G stages pair positions that differ only in the
// block index, and a lane already holds every member of its groups: they run
// in registers.
//
// Within a block of 256, positions P split into four 2-bit fields F0..F3
// (F_s = bits 2s, 2s+1); radix-4 step s runs stages 2s and 2s+1 on the groups
// of four positions that differ only in F_s.  A lane owns one group per step:
//   step 0  lane = brev6(F1 + 4 F2 + 16 F3); slot k (F0 = k) is position
//           4 brev6(lane) + k: coefficient lane + 64 brev2(k) when n >= 256
//           (each load reads 64 consecutive words or G-word chunks), runs of
//           16 or more consecutive words when n < 256
//   step 1  lane = F0 + 4 F3 + 16 F2       (slot F1)
//   step 2  lane = F0 + 4 F1 + 16 F3       (slot F2)
//   step 3  lane = F0 + 4 F1 + 16 F2       (slot F3): position lane + 64 k,
//           written to x[256 b + lane + 64 k] of the unit after the last stage
//           (64 consecutive words per store)
// Between steps each lane writes its four slots to 16 consecutive bytes of the
// block's LDS buffer at 16 lane (conflict-free: 16 lanes fill the 64 four-byte
// banks) and reads the next group at base_s + 64 k (immediate offsets), where
// the bases of the 64 lanes are 64 distinct banks:
//   base_1 = F0 + 4 brev2(F3) + 16 brev2(F2)   (slot k at base_1 + 64 brev2(k))
//   base_2 = F1 + 4 F0 + 16 F3
//   base_3 = F2 + 4 F0 + 16 F1
// Stage 0 and half of stage 1 multiply by 1 and skip the product.  A lane's
// twiddles are the same for every unit and stay in registers; waves loop over
// units (the next one's loads in flight).  `nelem` (the batch's coefficient
// count) bounds the last unit when n < 256.
template <int W, int V, bool FAST, int LAZY, int L, class S>
__global__ void __launch_bounds__(BLOCK)
    k_nttw(KCtx c, void *__restrict__ data, uint64_t units, uint64_t nelem, const TwL<W, V> *__restrict__ tw,
           KConst scale, uint32_t do_scale, uint32_t vec)
{
    using R = Red<W, V>;
    using El = typename R::E;  // arithmetic; S: the coefficients' storage type (as wide or narrower)
    using T = TwL<W, V>;
    static_assert(L >= 1 && L <= 10, "lengths 2 to 1024");
    constexpr int G = L > 8 ? 1 << (L - 8) : 1;
    constexpr uint32_t UNIT = 256u * G;
    constexpr int WAVES = BLOCK / 64;
    __shared__ __align__(16) El lds[WAVES][G][256];
    const R red(c);
    const El N = (El)c.N;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    auto br2 = [](uint32_t f) { return ((f & 1u) << 1) | (f >> 1); };
    const uint32_t f0 = lane & 3u, f1 = (lane >> 2) & 3u, f2 = lane >> 4;
    const uint32_t base1 = f0 + 4 * br2(f1) + 16 * br2(f2);  // step-1 lane: F0 = f0, F3 = f1, F2 = f2
    const uint32_t base2 = f1 + 4 * f0 + 16 * f2;            // step-2 lane: F0 = f0, F1 = f1, F3 = f2
    const uint32_t base3 = f2 + 4 * f0 + 16 * f1;            // step-3 lane: F0 = f0, F1 = f1, F2 = f2
    const uint32_t j2 = f0 + 4 * f1;
    auto twi = [&](int st, uint32_t j) -> T { return tw[j << (L - 1 - st)]; };
    T tw9[10]{};  // t01, t10, t11, t12, t20, t21, t22, t30, t31, t32 (stages that exist)
    if constexpr (L > 1)
        tw9[0] = twi(1, 1);
    if constexpr (L > 2)
        tw9[1] = twi(2, f0);
    if constexpr (L > 3) {
        tw9[2] = twi(3, f0);
        tw9[3] = twi(3, f0 + 4);
    }
    if constexpr (L > 4)
        tw9[4] = twi(4, j2);
    if constexpr (L > 5) {
        tw9[5] = twi(5, j2);
        tw9[6] = twi(5, j2 + 16);
    }
    if constexpr (L > 6)
        tw9[7] = twi(6, lane);
    if constexpr (L > 7) {
        tw9[8] = twi(7, lane);
        tw9[9] = twi(7, lane + 64);
    }
    // stages across blocks (G > 1), at position j = lane + 64 k of the block: stage 8 uses
    // tw[j << (L - 9)], stage 9 (G = 4) tw[j] and tw[j + 256]
    T u0[4], u1[4], u2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t j = lane + 64u * (uint32_t)k;
        if constexpr (G == 2) {
            u0[k] = tw[j];
        } else if constexpr (G == 4) {
            u0[k] = tw[2 * j];
            u1[k] = tw[j];
            u2[k] = tw[j + 256];
        }
    }
    // G = 1: the unit offset of slot k's coefficient (position 4 brev6(lane) + k)
    uint32_t off[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t P = 4 * (__brev(lane) >> 26) + (uint32_t)k;
        const uint32_t p = P & ((1u << L) - 1);
        off[k] = (P - p) + (__brev(p) >> (32 - L));
    }
    auto outv = [&](El y) -> El {
        if constexpr (LAZY == 3)  // scale: the product by 1 or n^{-1}
            return tw_mul<R, V, FAST>(red, y, scale);
        else if constexpr (LAZY == 2)  // scale: 1 or n^{-1}, times R mod N
            return below<El>(lazy_mul(red, y, (El)scale.b), N);
        else if constexpr (LAZY)
            return do_scale ? below<El>(lazy_mul(red, y, (El)scale.b), N) : below<El>(below<El>(y, (El)(2 * N)), N);
        else
            return do_scale ? tw_mul<R, V, FAST>(red, y, scale) : y;
    };
    const uint64_t stride = (uint64_t)gridDim.x * WAVES;
    uint64_t t = (uint64_t)blockIdx.x * WAVES + wv;
    El nx[G][4];
    auto fetch = [&](uint64_t p) {
        if constexpr (G == 1) {
            const S *x = (const S *)data + p * UNIT;
            if (L >= 8 || (p + 1) * UNIT <= nelem) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    nx[0][k] = (El)x[off[k]];
            } else {  // the batch's last, partial unit: whole polynomials in or out
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    nx[0][k] = p * UNIT + off[k] < nelem ? (El)x[off[k]] : (El)0;
            }
        } else {
            // block b, slot k: x[brev(b) + G (lane + 64 brev2(k))]; chunk element e is block brev(e)
            const S *x = (const S *)data + p * UNIT + (uint64_t)G * lane;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const S *q = x + 64 * G * br2((uint32_t)k);
                S v[G];
                if (vec) {
                    load_chunk<S, G, false>(q, v);
                } else {
#pragma unroll
                    for (int e = 0; e < G; ++e)
                        v[e] = q[e];
                }
#pragma unroll
                for (int e = 0; e < G; ++e)
                    nx[G == 1 ? 0 : (int)(__brev((uint32_t)e) >> (32 - __builtin_ctz(G)))][k] = (El)v[e];
            }
        }
    };
    if (t < units)
        fetch(t);
    for (; t < units; t += stride) {
        El a[G][4];
#pragma unroll
        for (int b = 0; b < G; ++b)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                a[b][k] = nx[b][k];
        if (t + stride < units)
            fetch(t + stride);
        block_steps<R, V, FAST, LAZY, G, L>(red, a, &lds[wv][0][0], lane, base1, base2, base3, tw9, N);
        // the stages across blocks: position lane + 64 k of every block, in registers
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if constexpr (G == 2) {
                butterfly<R, V, FAST, LAZY>(red, a[0][k], a[1][k], u0[k], N);
            } else if constexpr (G == 4) {
                butterfly<R, V, FAST, LAZY>(red, a[0][k], a[1][k], u0[k], N);
                butterfly<R, V, FAST, LAZY>(red, a[2][k], a[3][k], u0[k], N);
                butterfly<R, V, FAST, LAZY>(red, a[0][k], a[2][k], u1[k], N);
                butterfly<R, V, FAST, LAZY>(red, a[1][k], a[3][k], u2[k], N);
            }
        }
        S *y = (S *)data + t * UNIT + lane;
        if (L >= 8 || (t + 1) * UNIT <= nelem) {
#pragma unroll
            for (int b = 0; b < G; ++b)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    y[256 * b + 64 * k] = (S)outv(a[b][k]);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (t * UNIT + lane + 64 * k < nelem)
                    y[64 * k] = (S)outv(a[0][k]);
        }
    }
}

// Lengths 2048 and 4096 (L = 11, 12): one workgroup of four wavefronts per
// polynomial, workgroups looping over the batch.
//
// Positions, blocks and the radix-4 steps within a block are those of k_nttw:
// G = 2^(L-8) blocks of 256 positions, block b holding x[brev(b) + G m].  Wave
// v takes the G/4 blocks b with brev(b) = v G/4 + e, e < G/4, so for each slot
// a lane loads G/4 consecutive words, and runs stages 0..7 on them, block e
// through the 256 LDS words at 256 (v G/4 + e).  The waves then trade through
// those same n words: each writes position lane + 64 k of its blocks in place,
// and after a barrier lane l of wave v reads position 64 v + l of every block,
// so the L - 8 stages across blocks run in its registers, with the G - 1
// twiddles they take at that position held for the whole run.  Results leave
// as 64 consecutive words per store.  A second barrier, before the next
// polynomial's first LDS write, waits for every wave's reads.
template <int W, int V, bool FAST, int LAZY, int L, class S>
__global__ void __launch_bounds__(BLOCK)
    k_nttm(KCtx c, void *__restrict__ data, uint64_t batch, const TwL<W, V> *__restrict__ tw, KConst scale,
           uint32_t do_scale, uint32_t vec)
{
    using R = Red<W, V>;
    using El = typename R::E;  // arithmetic; S: the coefficients' storage type (as wide or narrower)
    using T = TwL<W, V>;
    static_assert(L == 11 || L == 12, "lengths 2048 and 4096");
    static_assert(BLOCK == 256, "four wavefronts per workgroup");
    constexpr int LG = L - 8, G = 1 << LG, GW = G / 4;
    constexpr uint32_t n = 1u << L;
    __shared__ __align__(16) El sx[n];
    const R red(c);
    const El N = (El)c.N;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    auto br2 = [](uint32_t f) { return ((f & 1u) << 1) | (f >> 1); };
    const uint32_t f0 = lane & 3u, f1 = (lane >> 2) & 3u, f2 = lane >> 4;
    const uint32_t base1 = f0 + 4 * br2(f1) + 16 * br2(f2);
    const uint32_t base2 = f1 + 4 * f0 + 16 * f2;
    const uint32_t base3 = f2 + 4 * f0 + 16 * f1;
    const uint32_t j2 = f0 + 4 * f1;
    auto twi = [&](int st, uint32_t j) -> T { return tw[j << (L - 1 - st)]; };
    const T tw9[10] = {twi(1, 1), twi(2, f0),   twi(3, f0),   twi(3, f0 + 4), twi(4, j2),
                       twi(5, j2), twi(5, j2 + 16), twi(6, lane), twi(7, lane), twi(7, lane + 64)};
    // stage 8 + h pairs blocks b and b + 2^h at position P = 64 v + l: twiddle
    // tw[(P + 256 r) << (L - 9 - h)], r = b mod 2^h, kept at cx[2^h - 1 + r]
    const uint32_t P = 64u * wv + lane;
    T cx[G - 1];
#pragma unroll
    for (int h = 0; h < LG; ++h)
#pragma unroll
        for (int r = 0; r < (1 << h); ++r)
            cx[(1 << h) - 1 + r] = tw[(P + 256u * (uint32_t)r) << (L - 9 - h)];
    auto outv = [&](El y) -> El {
        if constexpr (LAZY == 3)  // scale: the product by 1 or n^{-1}
            return tw_mul<R, V, FAST>(red, y, scale);
        else if constexpr (LAZY == 2)  // scale: 1 or n^{-1}, times R mod N
            return below<El>(lazy_mul(red, y, (El)scale.b), N);
        else if constexpr (LAZY)
            return do_scale ? below<El>(lazy_mul(red, y, (El)scale.b), N) : below<El>(below<El>(y, (El)(2 * N)), N);
        else
            return do_scale ? tw_mul<R, V, FAST>(red, y, scale) : y;
    };
    El nx[GW][4];
    auto fetch = [&](uint64_t p) {
        // block brev(v G/4 + e), slot k: x[v G/4 + e + G (lane + 64 brev2(k))]
        const S *x = (const S *)data + p * n + (uint64_t)(G * lane + GW * wv);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const S *q = x + 64 * G * br2((uint32_t)k);
            S v[GW];
            if (vec) {
                load_chunk<S, GW, false>(q, v);
            } else {
#pragma unroll
                for (int e = 0; e < GW; ++e)
                    v[e] = q[e];
            }
#pragma unroll
            for (int e = 0; e < GW; ++e)
                nx[e][k] = (El)v[e];
        }
    };
    El *sw = sx + 256u * GW * wv;  // this wave's blocks
    uint64_t p = blockIdx.x;
    if (p < batch)
        fetch(p);
    for (; p < batch; p += gridDim.x) {  // uniform over the workgroup: the barriers are safe
        El a[GW][4];
#pragma unroll
        for (int e = 0; e < GW; ++e)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                a[e][k] = nx[e][k];
        if (p + gridDim.x < batch)
            fetch(p + gridDim.x);
        __syncthreads();  // the previous polynomial's exchange reads are done
        block_steps<R, V, FAST, LAZY, GW, L>(red, a, sw, lane, base1, base2, base3, tw9, N);
#pragma unroll
        for (int e = 0; e < GW; ++e)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                sw[256 * e + 64 * k + lane] = a[e][k];
        __syncthreads();
        El z[G];
#pragma unroll
        for (int b = 0; b < G; ++b)
            z[b] = sx[256u * (__brev((uint32_t)b) >> (32 - LG)) + P];
#pragma unroll
        for (int h = 0; h < LG; ++h)
#pragma unroll
            for (int b = 0; b < G; ++b)
                if (!(b & (1 << h)))
                    butterfly<R, V, FAST, LAZY>(red, z[b], z[b + (1 << h)], cx[(1 << h) - 1 + (b & ((1 << h) - 1))],
                                                N);
        S *y = (S *)data + p * n + P;
#pragma unroll
        for (int b = 0; b < G; ++b)
            y[256 * b] = (S)outv(z[b]);
    }
}

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t N) { return (uint64_t)(((u128)a * b) % N); }

static uint64_t powmod(uint64_t a, uint64_t e, uint64_t N)
{
    uint64_t r = 1 % N;
    a %= N;
    while (e) {
        if (e & 1)
            r = mulmod(r, a, N);
        a = mulmod(a, a, N);
        e >>= 1;
    }
    return r;
}

// The fixed-operand constants that make tw_mul(a, .) = a v mod N.
static KConst twiddle_const(const mont_ctx_t &c, int variant, uint64_t v)
{
    KConst k{};
    const uint32_t w = c.w;
    if (variant == CLASSIC) {
        k.b = mulmod(v, c.r_mod_n, c.N);  // v R mod N: REDC(a (v R)) = a v
        return k;
    }
    // Plantard returns -a b 2^(-2w): take b = -v 2^(2w) mod N
    const uint64_t r2w = c.r2_mod_n;  // 2^(2w) mod N
    const uint64_t bv = mulmod(v, r2w, c.N);
    const uint64_t b = bv ? c.N - bv : 0;
    const u128 ninv2 = ((u128)c.ninv2_hi << 64) | c.ninv2_lo;
    u128 bp = (u128)b * ninv2;
    if (w < 64)
        bp &= ((u128)1 << (2 * w)) - 1;
    k.b = b;
    k.b1 = (uint64_t)bp;
    k.b2 = w == 64 ? (uint64_t)(bp >> 64) : 0;
    return k;
}

struct TwKey {
    uint64_t N, root;
    uint32_t w, log2n;
    int variant, inverse;
    bool operator<(const TwKey &o) const
    {
        return std::tie(N, root, w, log2n, variant, inverse) < std::tie(o.N, o.root, o.w, o.log2n, o.variant, o.inverse);
    }
};

struct TwEntry {
    void *dev = nullptr;  // n/2 compact twiddles (TwL of the width and variant)
    KConst scale{};       // the product by n^{-1}
    KConst one{};         // the product by 1
};

static std::mutex g_tw_mu;
static std::map<std::pair<int, TwKey>, TwEntry> g_tw;  // (device, key)

static mont_status_t twiddles(const mont_ctx_t &c, int variant, uint64_t root, uint32_t log2n, int inverse,
                              TwEntry *out)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    const TwKey key{c.N, root, c.w, log2n, variant, inverse};
    std::lock_guard<std::mutex> g(g_tw_mu);
    auto it = g_tw.find({dev, key});
    if (it != g_tw.end()) {
        *out = it->second;
        return MONT_OK;
    }
    const uint32_t n = 1u << log2n;
    const uint64_t w = inverse ? powmod(root, n - 1, c.N) : root % c.N;  // root^{-1} = root^(n-1)
    std::vector<KConst> h(n / 2);
    uint64_t p = 1 % c.N;
    for (uint32_t k = 0; k < n / 2; ++k) {
        h[k] = twiddle_const(c, variant, p);
        p = mulmod(p, w, c.N);
    }
    TwEntry e;
    // n^{-1} mod N: N odd, so (N + 1)/2 is 2^{-1}
    const uint64_t half = (uint64_t)(((u128)c.N + 1) / 2);
    e.scale = twiddle_const(c, variant, powmod(half, log2n, c.N));
    e.one = twiddle_const(c, variant, 1);
    // compact device form: b (classic), b N^{-1} mod 2^(2w) (Plantard, w <= 32), its two words (w = 64)
    const bool two = variant != CLASSIC && c.w == 64;
    std::vector<uint64_t> hc;
    hc.reserve(h.size() * (two ? 2 : 1));
    for (const KConst &q : h) {
        if (variant == CLASSIC) {
            hc.push_back(q.b);
        } else {
            hc.push_back(q.b1);
            if (two)
                hc.push_back(q.b2);
        }
    }
    if (hipMalloc(&e.dev, hc.size() * sizeof(uint64_t)) != hipSuccess)
        return fail(MONT_E_NOMEM, "twiddle table");
    const hipError_t err = hipMemcpy(e.dev, hc.data(), hc.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(e.dev);
        return hip_fail(err, "twiddle upload");
    }
    g_tw[{dev, key}] = e;
    *out = e;
    return MONT_OK;
}

// Workgroups of kernel K that one CU holds at once (registers and LDS), asked once.
template <auto K>
static unsigned resident_per_cu()
{
    static const unsigned v = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void *>(K), BLOCK, 0) !=
                hipSuccess ||
            b < 1) {
            (void)hipGetLastError();
            b = 1;
        }
        return (unsigned)b;
    }();
    return v;
}

// W: the arithmetic's word; S: the coefficients' storage type (16-bit data
// are transformed with 32-bit words: see mont_ntt below).
template <int W, class S>
static hipError_t go_ntt(const KCtx &k, int variant, void *data, size_t batch, uint32_t log2n, const TwEntry &t,
                         int inverse, hipStream_t s)
{
    using El = S;  // alignment of the chunk loads is that of the stored words
    const uint32_t n = 1u << log2n;
    const uint32_t inv = (uint32_t)inverse;
    // FAST needs N < 2^(w-1); classic twiddles at w >= 32 also the ladder's smaller-modulus bound;
    // LAZY (classic twiddles) needs 4N <= 2^w, with operands below 2^63 at w = 64
    const bool small = k.N < (1ull << (W - 1));
    const bool fast = variant == CLASSIC && W != 16 ? fast_ladder<W>(k.N) : small;
    const bool lazy = variant == CLASSIC && ((W == 16 && k.N < (1ull << 14)) || (W == 32 && k.N < (1ull << 30)) ||
                                             (W == 64 && k.N < (1ull << 61)));
    // no reduction between stages when the final bound (2 log2n + 1) N fits the word (below 2^63 at w = 64)
    const u128 bound2 = (u128)(2 * log2n + 1) * k.N;
    const bool lazy2 = lazy && bound2 <= (W == 64 ? (u128)1 << 63 : (u128)1 << W);
    // Plantard twiddles: no reduction between stages when (log2n + 2) N fits the word
    const bool lazy3 = variant == PLANTARD && small && (u128)(log2n + 2) * k.N <= (u128)1 << W;
    const KConst sc2 = inverse ? t.scale : t.one;  // the output product of the lazy2 and lazy3 forms
    const auto *twc = (const TwL<W, CLASSIC> *)t.dev;
    const auto *twp = (const TwL<W, PLANTARD> *)t.dev;
    const dim3 b(BLOCK);
    if (log2n <= 10) {
        // one wavefront per unit of max(n, 256) coefficients, waves looping over the units
        constexpr uint64_t WAVES = BLOCK / 64;
        const uint64_t nelem = (uint64_t)batch << log2n;
        const uint64_t units = log2n >= 8 ? (uint64_t)batch : (nelem + 255) / 256;
        const uint64_t blocks = std::min<uint64_t>((units + WAVES - 1) / WAVES, (uint64_t)device_cus() * nttw_bpc(log2n));
        const dim3 g((unsigned)blocks);
        // chunk loads (n / 256 words per lane and slot) when the polynomials are aligned to them
        const size_t chunk = std::min<size_t>(16, std::max<size_t>(1, (size_t)n / 256) * sizeof(El));
        const uint32_t cv = (uintptr_t)data % chunk == 0 ? 1u : 0u;
        auto go = [&](auto lc) {
            constexpr int LL = decltype(lc)::value;
            if (lazy2)
                hipLaunchKernelGGL((k_nttw<W, CLASSIC, true, 2, LL, S>), g, b, 0, s, k, data, units, nelem, twc, sc2,
                                   inv, cv);
            else if (lazy)
                hipLaunchKernelGGL((k_nttw<W, CLASSIC, true, 1, LL, S>), g, b, 0, s, k, data, units, nelem, twc,
                                   t.scale, inv, cv);
            else if (variant == CLASSIC && fast)
                hipLaunchKernelGGL((k_nttw<W, CLASSIC, true, 0, LL, S>), g, b, 0, s, k, data, units, nelem, twc,
                                   t.scale, inv, cv);
            else if (variant == CLASSIC)
                hipLaunchKernelGGL((k_nttw<W, CLASSIC, false, 0, LL, S>), g, b, 0, s, k, data, units, nelem, twc,
                                   t.scale, inv, cv);
            else if (lazy3)
                hipLaunchKernelGGL((k_nttw<W, PLANTARD, true, 3, LL, S>), g, b, 0, s, k, data, units, nelem, twp, sc2,
                                   inv, cv);
            else if (fast)
                hipLaunchKernelGGL((k_nttw<W, PLANTARD, true, 0, LL, S>), g, b, 0, s, k, data, units, nelem, twp,
                                   t.scale, inv, cv);
            else
                hipLaunchKernelGGL((k_nttw<W, PLANTARD, false, 0, LL, S>), g, b, 0, s, k, data, units, nelem, twp,
                                   t.scale, inv, cv);
        };
        switch (log2n) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        case 4: go(std::integral_constant<int, 4>{}); break;
        case 5: go(std::integral_constant<int, 5>{}); break;
        case 6: go(std::integral_constant<int, 6>{}); break;
        case 7: go(std::integral_constant<int, 7>{}); break;
        case 8: go(std::integral_constant<int, 8>{}); break;
        case 9: go(std::integral_constant<int, 9>{}); break;
        default: go(std::integral_constant<int, 10>{}); break;
        }
        return hipGetLastError();
    }
    // one workgroup per polynomial, workgroups looping over the batch: twice as many as the CUs hold
    // at once (registers decide: 64-bit words fit two per CU, narrower words four or more); against
    // exactly as many, twice measured 1-5 % faster on MI355X at every width, four times mixed
    // chunk loads (n / 1024 words per lane and slot) when the polynomials are aligned to them
    const size_t chunk = std::min<size_t>(16, (size_t)n / 1024 * sizeof(El));
    const uint32_t cv = (uintptr_t)data % chunk == 0 ? 1u : 0u;
    const uint64_t nb = batch;
    auto grid = [&](unsigned per_cu) { return dim3((unsigned)std::min<uint64_t>(nb, (uint64_t)device_cus() * per_cu * 2)); };
#define MONT_NTTM(VV, F, Z, TWP, SC)                                                                               \
    hipLaunchKernelGGL((k_nttm<W, VV, F, Z, LL, S>), grid(resident_per_cu<k_nttm<W, VV, F, Z, LL, S>>()), b, 0,  \
                       s, k, data, nb, TWP, SC, inv, cv)
    auto go = [&](auto lc) {
        constexpr int LL = decltype(lc)::value;
        if (lazy2)
            MONT_NTTM(CLASSIC, true, 2, twc, sc2);
        else if (lazy)
            MONT_NTTM(CLASSIC, true, 1, twc, t.scale);
        else if (variant == CLASSIC && fast)
            MONT_NTTM(CLASSIC, true, 0, twc, t.scale);
        else if (variant == CLASSIC)
            MONT_NTTM(CLASSIC, false, 0, twc, t.scale);
        else if (lazy3)
            MONT_NTTM(PLANTARD, true, 3, twp, sc2);
        else if (fast)
            MONT_NTTM(PLANTARD, true, 0, twp, t.scale);
        else
            MONT_NTTM(PLANTARD, false, 0, twp, t.scale);
    };
#undef MONT_NTTM
    if (log2n == 11)
        go(std::integral_constant<int, 11>{});
    else
        go(std::integral_constant<int, 12>{});
    return hipGetLastError();
}

}  // namespace mont

using namespace mont;

extern "C" mont_status_t mont_ntt(const mont_ctx_t *ctx, void *data, size_t batch, uint32_t log2n, uint64_t root,
                                  int inverse, mont_variant_t variant, void *stream)
{
    mont_status_t rc = check_ctx(ctx);
    if (rc)
        return rc;
    if (variant != MONT_CLASSIC && variant != MONT_PLANTARD)
        return fail(MONT_E_UNSUPPORTED, "mont_ntt uses the classic or the Plantard twiddle product");
    rc = check_variant(ctx, variant);
    if (rc)
        return rc;
    if (log2n < 1 || log2n > 12)
        return fail(MONT_E_INVAL, "transform length 2^log2n with 1 <= log2n <= 12");
    const uint64_t N = ctx->N;
    if (root % N == 0 || powmod(root, 1ull << (log2n - 1), N) != N - 1)
        return fail(MONT_E_DOMAIN, "root^(n/2) must be -1 mod N");
    if (batch == 0)
        return MONT_OK;
    if (!data)
        return fail(MONT_E_INVAL, "null data");
    if (batch > 0x7fffffffull)
        return fail(MONT_E_INVAL, "batch too large");
    // 16-bit coefficients whose 16-bit butterflies would need reductions
    // between stages ((2 log2n + 1) N, or (log2n + 2) N for Plantard
    // twiddles, beyond the word) are transformed with 32-bit words when the
    // transform is 16 long or longer: loaded and stored as 16 bits, computed
    // with the 32-bit reductions of the same modulus.  The twiddle products
    // return a v whatever R is, so the results are those of the 16-bit forms,
    // and the unreduced butterflies then apply (5-10 % faster at N = 12289
    // from length 256 on, 18-20 % at N = 18433 and 25-39 % at N = 40961 from
    // length 64 on; at lengths 2 and 4 the 16-bit forms measured faster, and
    // moduli such as 3329, whose 16-bit butterflies stay unreduced, keep them).
    bool wide16 = false;
    if (ctx->w == 16) {
        const bool unreduced16 = variant == MONT_CLASSIC
                                     ? N < (1u << 14) && (2 * log2n + 1) * N <= (1u << 16)
                                     : N < (1u << 15) && (log2n + 2) * N <= (1u << 16);
        wide16 = !unreduced16 && log2n >= 4;
    }
    mont_ctx_t c32;
    const mont_ctx_t *cw = ctx;
    if (wide16) {
        rc = setup_ctx(N, 32, &c32);
        if (rc)
            return rc;
        cw = &c32;
    }
    TwEntry t;
    rc = twiddles(*cw, variant, root, log2n, inverse ? 1 : 0, &t);
    if (rc)
        return rc;
    const KCtx k = to_kctx(*cw);
    hipStream_t s = (hipStream_t)stream;
#ifdef MONT_DEBUG
    if (const hipError_t de = debug_check(DBG_BELOW_N, *ctx, CLASSIC, data, nullptr, 0, (uint64_t)batch << log2n, s))
        return hip_fail(de, "precondition check");
#endif
    const int iv = inverse ? 1 : 0;
    const hipError_t e = wide16         ? go_ntt<32, uint16_t>(k, variant, data, batch, log2n, t, iv, s)
                         : ctx->w == 16 ? go_ntt<16, uint16_t>(k, variant, data, batch, log2n, t, iv, s)
                         : ctx->w == 32 ? go_ntt<32, uint32_t>(k, variant, data, batch, log2n, t, iv, s)
                                        : go_ntt<64, uint64_t>(k, variant, data, batch, log2n, t, iv, s);
    return e == hipSuccess ? MONT_OK : hip_fail(e, "mont_ntt launch");
}
