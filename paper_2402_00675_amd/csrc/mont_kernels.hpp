// Streaming, exponentiation and exhaustive-range kernels for gfx950.
//
// Streaming kernels (mont_mul, mont_redc) are HBM-bound: each lane moves
// 16-byte chunks (8 x u16, 4 x u32 or 2 x u64 residues) with optional
// non-temporal hints, U chunks in flight per lane, a grid-stride loop whose
// grid is either one pass over the data or a multiple of the CU count, and a
// scalar tail.  Per-modulus constants are kernel arguments (wave-uniform, so
// they live in SGPRs); a residue-number-system call indexes a by-value table
// of contexts with the row number blockIdx.y.
#pragma once

#include "mont_arith.hpp"

namespace mont {

constexpr int BLOCK = 256;
constexpr int MAX_ROWS = 32;

template <int NR>
struct KTab {
    KCtx c[NR];
};

// Launch shape of the streaming kernels.  The default (one 16-byte chunk per
// lane, non-temporal loads and stores, one pass over the data) was the
// fastest measured on MI355X for the 2-read/1-write pattern at HBM-resident
// sizes; grid-stride loops over a CU-multiple grid were 10-20% slower.
// Workgroups of one wavefront streamed 1.5-2 % faster than 256-lane ones
// (finer-grained dispatch across the CUs, shorter tail).
struct Launch {
    int unroll = 1;        // 1, 2, 4
    int nontemporal = 1;   // 0 / 1
    int blocks_per_cu = 0; // 0: one pass
    int block = 64;        // lanes per workgroup of the 16-byte path: 64 or 256
};

struct MapArgs {
    int op;        // 0 mul, 1 redc, 2 mul by the fixed operand in kc
    int variant;
    int rows;      // >= 1
    const KCtx *ctx;  // rows entries (host)
    const void *in0, *in1;
    void *out;
    uint64_t n, ld;   // per row: n elements, row stride ld elements
    KConst kc{};      // op 2 only
    uint32_t head = 0;  // elements before in0 / in1 / out (below 128 / element size), computed element-wise
};

// ------------------------------------------------------------ memory helpers

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int B>
struct Raw;
template <>
struct Raw<16> {
    using type = u32x4;
};
template <>
struct Raw<8> {
    using type = u32x2;
};
template <>
struct Raw<4> {
    using type = uint32_t;
};
template <>
struct Raw<2> {
    using type = uint16_t;
};

template <int B, bool NT>
__device__ __forceinline__ typename Raw<B>::type ld_raw(const void *p)
{
    using R = typename Raw<B>::type;
    if constexpr (NT)
        return __builtin_nontemporal_load((const R *)p);
    else
        return *(const R *)p;
}

template <int B, bool NT>
__device__ __forceinline__ void st_raw(void *p, typename Raw<B>::type v)
{
    using R = typename Raw<B>::type;
    if constexpr (NT)
        __builtin_nontemporal_store(v, (R *)p);
    else
        *(R *)p = v;
}

// E consecutive X's, loaded with 16-byte (or narrower) accesses.
template <class X, int E, bool NT>
__device__ __forceinline__ void load_chunk(const X *p, X (&v)[E])
{
    constexpr int B = E * (int)sizeof(X);
    if constexpr (B <= 16) {
        auto r = ld_raw<B, NT>(p);
        __builtin_memcpy(&v[0], &r, B);
    } else {
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            auto r = ld_raw<16, NT>((const char *)p + 16 * k);
            __builtin_memcpy((char *)&v[0] + 16 * k, &r, 16);
        }
    }
}

template <class X, int E, bool NT>
__device__ __forceinline__ void store_chunk(X *p, const X (&v)[E])
{
    constexpr int B = E * (int)sizeof(X);
    static_assert(B <= 16, "stores are at most 16 bytes");
    typename Raw<B>::type r;
    __builtin_memcpy(&r, &v[0], B);
    st_raw<B, NT>(p, r);
}

// ------------------------------------------------------------------ kernels

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on
// XCD i mod 8).  Renumbering them so that each XCD walks one contiguous eighth
// of the index space keeps each XCD's traffic in a compact address window;
// it is a bijection whenever the grid is a multiple of 8 (else the identity).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t g)
{
    if (g % 8u)
        return b;
    return (b % 8u) * (g / 8u) + b / 8u;
}

// out[i] = red.mul(a[i], b[i]) (OP 0), red.redc(T[i]) (OP 1) or
// red.mul_const(a[i], kc) (OP 2), per row, in workgroups of BS lanes.  out
// may be in0 or in1 (in-place calls): every element is read and written by
// the same lane, reads first, so the pointers carry no __restrict__.  The
// `head` elements just before the (16-byte aligned) pointers, at indices
// -head .. -1, are computed element-wise by workgroup 0, like the tail.
template <int W, int V, int OP, int E, int U, bool NT, int NR, int BS>
__global__ void __launch_bounds__(BS)
    k_map(KTab<NR> tab, const void *in0, const void *in1, void *out, uint64_t n, uint64_t ld, KConst kc,
          uint32_t head)
{
    using R = Red<W, V>;
    using El = typename R::E;
    using TT = typename R::TT;
    const R red(tab.c[NR == 1 ? 0 : blockIdx.y]);
    const uint64_t row = (uint64_t)blockIdx.y * ld;
    const El *pa = (const El *)in0 + row;
    const El *pb = (const El *)in1 + row;
    const TT *pt = (const TT *)in0 + row;
    El *po = (El *)out + row;

    const uint64_t nchunk = n / E;
    const uint64_t step = (uint64_t)gridDim.x * (BS * U);
    const uint32_t bx = xcd_block(blockIdx.x, gridDim.x);
    // A do-while rather than a for loop: with one chunk per lane, the for form
    // compiled its non-temporal stores as ordinary ones (5 % slower at the
    // 6 GiB RNS product); every store of this form keeps its hint.
    uint64_t base = (uint64_t)bx * (BS * U) + threadIdx.x;
    do {
        El a[U][E], b[U][E];
        TT t[U][E];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + (uint64_t)u * BS;
            if (i < nchunk) {
                if constexpr (OP == 0) {
                    load_chunk<El, E, NT>(pa + i * E, a[u]);
                    load_chunk<El, E, NT>(pb + i * E, b[u]);
                } else if constexpr (OP == 2) {
                    load_chunk<El, E, NT>(pa + i * E, a[u]);
                } else {
                    load_chunk<TT, E, NT>(pt + i * E, t[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + (uint64_t)u * BS;
            if (i < nchunk) {
                El o[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if constexpr (OP == 0)
                        o[e] = red.mul(a[u][e], b[u][e]);
                    else if constexpr (OP == 2)
                        o[e] = red.mul_const(a[u][e], kc);
                    else
                        o[e] = red.redc(t[u][e]);
                }
                store_chunk<El, E, NT>(po + i * E, o);
            }
        }
        base += step;
    } while (base < nchunk);
    if constexpr (E > 1) {
        // the last n mod E elements of the row, and the head before it
        if (bx == 0) {
            auto one = [&](int64_t i) {
                if constexpr (OP == 0)
                    po[i] = red.mul(pa[i], pb[i]);
                else if constexpr (OP == 2)
                    po[i] = red.mul_const(pa[i], kc);
                else
                    po[i] = red.redc(pt[i]);
            };
            if (threadIdx.x < (unsigned)E && nchunk * E + threadIdx.x < n)
                one((int64_t)(nchunk * E + threadIdx.x));
            for (uint32_t j = threadIdx.x; j < head; j += BS)
                one((int64_t)j - (int64_t)head);
        }
    }
}

template <int W>
struct WideT;
template <>
struct WideT<16> {
    __device__ static uint32_t of(uint16_t y) { return y; }
};
template <>
struct WideT<32> {
    __device__ static uint64_t of(uint32_t y) { return y; }
};
template <>
struct WideT<64> {
    __device__ static T128 of(uint64_t y) { return {y, 0}; }
};


// Ladder products by mode.  0: the general classic product.  1 (w = 64,
// N < 2^62): the final subtraction is dropped ("lazy": for 4N <= R and inputs
// below 2N, (T + mN)/R < 4N^2/R + N <= 2N, so every result stays below 2N and
// is a valid input again).  3 (w = 32, N < 2^31): signed products, values in
// (-N, N) as two's-complement words, three instructions per product and no
// correction (Red<32, CLASSIC>::mul_signed).
template <int W>
__host__ __device__ __forceinline__ bool fast_ladder(uint64_t N)
{
    return (W == 64 && N < (1ull << 62)) || (W == 32 && N < (1ull << 31));
}

template <int W>
__host__ __device__ __forceinline__ int ladder_mode(uint64_t N)
{
    return !fast_ladder<W>(N) ? 0 : W == 32 ? 3 : 1;
}

template <class R, int MODE>
struct Ladder {
    __device__ __forceinline__ static typename R::E mul(const R &r, typename R::E a, typename R::E b)
    {
        if constexpr (MODE == 3)
            return r.mul_signed(a, b);
        else if constexpr (MODE == 1)
            return r.mul_fast(a, b);
        else
            return r.mul(a, b);
    }
    __device__ __forceinline__ static typename R::E sqr(const R &r, typename R::E a)
    {
        if constexpr (MODE == 3)
            return r.mul_signed(a, a);
        else if constexpr (MODE == 1)
            return r.sqr_fast(a);
        else
            return r.sqr(a);
    }
    // Montgomery form (in the mode's range) to the residue in [0, N)
    __device__ __forceinline__ static typename R::E out(const R &r, typename R::E y)
    {
        using El = typename R::E;
        if constexpr (MODE == 3)
            y = (int32_t)y < 0 ? (El)(y + r.N) : y;
        return r.redc(WideT<8 * (int)sizeof(El)>::of(y));
    }
};

// x^e mod N for U elements of one lane, in lockstep (U independent product
// chains per wave): Montgomery form x R = REDC(x * (R^2 mod N)), a
// left-to-right WB-bit fixed-window ladder of Montgomery products (every lane
// runs the same 64/WB windows: no divergence); the caller converts back with
// one REDC (Ladder::out).  The returned Montgomery-form values are below 2N
// (mode 1), in (-N, N) (mode 3) or below N.  Element u's 2^WB window entries
// (x^j in Montgomery form, j = 0 .. 2^WB - 1) live in LDS at
// tab[u * BLOCK + j * stride]: one LDS read per window instead of a register
// select.  Lanes of a wave use adjacent words of each entry row, so the reads
// are free of bank conflicts.  Per element: 2^WB - 2 products for the table,
// (64/WB - 1) (WB squarings + 1 product) for the windows (the top one is a
// table read) and one product into the Montgomery form: 96 products at WB = 2,
// 90 at WB = 4 (which also halves the window-index arithmetic), plus the
// caller's REDC back.
template <class R, int MODE, int U, int WB = 2>
__device__ __forceinline__ void pow_lanes(const R &red, const typename R::E (&x)[U], const uint64_t (&k)[U],
                                          typename R::E r2, typename R::E one, typename R::E *tab, uint32_t stride,
                                          typename R::E (&y)[U])
{
    using El = typename R::E;
    using L = Ladder<R, MODE>;
    static_assert(WB == 2 || WB == 4, "2- or 4-bit windows");
    constexpr int NE = 1 << WB;
    constexpr uint32_t MASK = NE - 1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        El e[NE];
        e[0] = one;
        e[1] = L::mul(red, x[u], r2);
#pragma unroll
        for (int j = 2; j < NE; ++j)
            e[j] = (j & 1) ? L::mul(red, e[j - 1], e[1]) : L::sqr(red, e[j / 2]);
        El *t = tab + u * BLOCK;
#pragma unroll
        for (int j = 0; j < NE; ++j)
            t[j * stride] = e[j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        y[u] = tab[u * BLOCK + (uint32_t)(k[u] >> (64 - WB)) * stride];
#pragma unroll 4
    for (int s = 64 - 2 * WB; s >= 0; s -= WB) {
        El t[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            t[u] = tab[u * BLOCK + ((uint32_t)(k[u] >> s) & MASK) * stride];
#pragma unroll
        for (int q = 0; q < WB; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u)
                y[u] = L::sqr(red, y[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            y[u] = L::mul(red, y[u], t[u]);
    }
}

// Window width of the standalone exponentiation kernel: 4 bits for every
// ladder (16-entry tables of 2, 4 or 8 bytes per element in LDS, one element
// per lane by default): 91 products per element instead of 97, measured 6-12 %
// faster than 2-bit windows for the general forms (16-bit words, and moduli
// above 2^31 or 2^62) and 2-3 % for the lazy 64-bit ladder.
template <int MODE>
constexpr int pow_window() { return 4; }

template <int W, int U, int MODE>
__global__ void __launch_bounds__(BLOCK)
    k_pow(KCtx c, const void *xin, const uint64_t *ein, void *out, uint64_t n)  // out may be xin (in place)
{
    using R = Red<W, CLASSIC>;
    using El = typename R::E;
    constexpr int WB = pow_window<MODE>();
    __shared__ El tab[(1 << WB) * BLOCK * U];
    const R red(c);
    const El r2 = (El)c.r2, one = (El)c.rmodn;
    const El *px = (const El *)xin;
    El *po = (El *)out;
    const uint64_t step = (uint64_t)gridDim.x * (BLOCK * U);
    for (uint64_t base = (uint64_t)blockIdx.x * (BLOCK * U) + threadIdx.x; base < n; base += step) {
        El x[U];
        uint64_t k[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + (uint64_t)u * BLOCK;
            x[u] = i < n ? px[i] : (El)0;
            k[u] = i < n ? ein[i] : 0;
        }
        El y[U];
        pow_lanes<R, MODE, U, WB>(red, x, k, r2, one, tab + threadIdx.x, BLOCK * U, y);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = base + (uint64_t)u * BLOCK;
            if (i < n)
                po[i] = Ladder<R, MODE>::out(red, y[u]);
        }
    }
}

// out[i] = REDC(T0 + i): exhaustive sweeps with no input traffic.
template <int W, int V, int E>
__global__ void __launch_bounds__(BLOCK) k_range(KCtx c, uint64_t T0, void *__restrict__ out, uint64_t n)
{
    using R = Red<W, V>;
    using El = typename R::E;
    using TT = typename R::TT;
    const R red(c);
    El *po = (El *)out;
    const uint64_t nchunk = n / E;
    const uint64_t step = (uint64_t)gridDim.x * BLOCK;
    for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; i < nchunk; i += step) {
        El o[E];
        const TT t0 = (TT)(T0 + i * E);
#pragma unroll
        for (int e = 0; e < E; ++e)
            o[e] = red.redc((TT)(t0 + (TT)e));
        store_chunk<El, E, true>(po + i * E, o);
    }
    if constexpr (E > 1) {
        if (blockIdx.x == 0 && threadIdx.x < (unsigned)E) {
            const uint64_t i = nchunk * E + threadIdx.x;
            if (i < n)
                po[i] = red.redc((TT)(T0 + i));
        }
    }
}

// ----------------------------------------------------------- host launchers

int device_cus();

template <int W>
hipError_t launch_map(const MapArgs &a, const Launch &L, hipStream_t s);
template <int W>
hipError_t launch_pow(const KCtx &c, const void *x, const uint64_t *e, void *out, uint64_t n, int unroll,
                      int blocks_per_cu, hipStream_t s);
template <int W>
hipError_t launch_range(const KCtx &c, int variant, uint64_t T0, void *out, uint64_t n, hipStream_t s);

}  // namespace mont
