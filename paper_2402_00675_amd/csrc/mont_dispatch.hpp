// Host-side launch templates for the streaming, exponentiation and range
// kernels.  Each word size is instantiated in its own translation unit
// (mont_k16.hip, mont_k32.hip, mont_k64.hip) so the builds run in parallel.
#pragma once

#include <algorithm>
#include <type_traits>

#include "mont_kernels.hpp"

namespace mont {

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

template <int W, int V, int OP, int E, int U, bool NT, int BS = BLOCK>
hipError_t go_map(const MapArgs &a, dim3 grid, hipStream_t s)
{
    if (a.rows == 1) {
        KTab<1> t;
        t.c[0] = a.ctx[0];
        hipLaunchKernelGGL((k_map<W, V, OP, E, U, NT, 1, BS>), grid, dim3(BS), 0, s, t, a.in0, a.in1, a.out, a.n,
                           a.ld, a.kc, a.head);
    } else if constexpr (OP == 0) {
        KTab<MAX_ROWS> t{};
        for (int r = 0; r < a.rows; ++r)
            t.c[r] = a.ctx[r];
        hipLaunchKernelGGL((k_map<W, V, OP, E, U, NT, MAX_ROWS, BS>), grid, dim3(BS), 0, s, t, a.in0, a.in1,
                           a.out, a.n, a.ld, a.kc, a.head);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

inline uint64_t grid_x(uint64_t nchunk, int per_thread, int rows, const Launch &L, int bs = BLOCK)
{
    const uint64_t per_block = (uint64_t)bs * per_thread;
    uint64_t gx = (nchunk + per_block - 1) / per_block;
    if (L.blocks_per_cu > 0) {
        const uint64_t cap = std::max<uint64_t>(1, (uint64_t)device_cus() * L.blocks_per_cu / rows);
        gx = std::min(gx, cap);
    }
    return std::min<uint64_t>(std::max<uint64_t>(gx, 1), 0x7fffffffu);
}

template <int W, int V, int OP>
hipError_t launch_map_v(const MapArgs &a, const Launch &L, hipStream_t s)
{
    using R = Red<W, V>;
    using El = typename R::E;
    constexpr int E = 16 / (int)sizeof(El);
    const bool rows_ok = a.rows == 1 || (a.ld * sizeof(El)) % 16 == 0;
    const bool vec = aligned16(a.in0) && (OP != 0 || aligned16(a.in1)) && aligned16(a.out) && rows_ok;
    // Operands that all become aligned after the same first h elements (equal
    // offsets, the usual case for slices of aligned arrays): the 16-byte body
    // starts at element h, and the kernel's first workgroup computes the h
    // elements before it along with the tail.  h aligns the body to 128 bytes
    // (a cache line) when every operand allows it, else to 16 bytes.
    const size_t s0 = OP == 1 ? 2 * sizeof(El) : sizeof(El);  // REDC reads 2w-bit T
    auto head_for = [&](uintptr_t al) -> uint64_t {
        const uint64_t h = ((al - ((uintptr_t)a.out & (al - 1))) & (al - 1)) / sizeof(El);
        const bool ok = ((uintptr_t)a.in0 + h * s0) % al == 0 &&
                        (OP != 0 || ((uintptr_t)a.in1 + h * sizeof(El)) % al == 0) &&
                        (a.rows == 1 || (a.ld * sizeof(El)) % al == 0);
        return ok ? h : ~0ull;
    };
    uint64_t h = head_for(128);
    if (h == ~0ull)
        h = head_for(16);
    if (!vec && rows_ok && E > 1 && a.head == 0 && (uintptr_t)a.out % sizeof(El) == 0 && h != ~0ull && h > 0 &&
        h < a.n) {
        MapArgs bd = a;
        bd.n = a.n - h;
        bd.in0 = (const char *)a.in0 + h * s0;
        if (OP == 0)
            bd.in1 = (const char *)a.in1 + h * sizeof(El);
        bd.out = (char *)a.out + h * sizeof(El);
        bd.head = (uint32_t)h;
        return launch_map_v<W, V, OP>(bd, L, s);
    }
    if (!vec) {
        dim3 grid((unsigned)grid_x(a.n, 1, a.rows, L), (unsigned)a.rows);
        return go_map<W, V, OP, 1, 1, false>(a, grid, s);
    }
    const int U = (L.unroll == 4 || L.unroll == 1) ? L.unroll : 2;
    const int bs = L.block == 64 ? 64 : BLOCK;
    dim3 grid((unsigned)grid_x(a.n / E, U, a.rows, L, bs), (unsigned)a.rows);
    auto go = [&](auto bs_c) {
        constexpr int B = decltype(bs_c)::value;
        if (L.nontemporal) {
            if (U == 1)
                return go_map<W, V, OP, E, 1, true, B>(a, grid, s);
            if (U == 2)
                return go_map<W, V, OP, E, 2, true, B>(a, grid, s);
            return go_map<W, V, OP, E, 4, true, B>(a, grid, s);
        }
        if (U == 1)
            return go_map<W, V, OP, E, 1, false, B>(a, grid, s);
        if (U == 2)
            return go_map<W, V, OP, E, 2, false, B>(a, grid, s);
        return go_map<W, V, OP, E, 4, false, B>(a, grid, s);
    };
    return bs == 64 ? go(std::integral_constant<int, 64>{}) : go(std::integral_constant<int, BLOCK>{});
}

template <int W, int OP>
hipError_t launch_map_op(const MapArgs &a, const Launch &L, hipStream_t s)
{
    switch (a.variant) {
    case CLASSIC:
        return launch_map_v<W, CLASSIC, OP>(a, L, s);
    case SIGNED:
        return launch_map_v<W, SIGNED, OP>(a, L, s);
    case PLANTARD:
        return launch_map_v<W, PLANTARD, OP>(a, L, s);
    case SIGNED_PLANTARD:
        return launch_map_v<W, SIGNED_PLANTARD, OP>(a, L, s);
    case SIGNED_PLANTARD_ALPHA:
        return launch_map_v<W, SIGNED_PLANTARD_ALPHA, OP>(a, L, s);
    default:
        return hipErrorInvalidValue;
    }
}

template <int W>
hipError_t launch_map(const MapArgs &a, const Launch &L, hipStream_t s)
{
    return a.op == 0 ? launch_map_op<W, 0>(a, L, s) : a.op == 1 ? launch_map_op<W, 1>(a, L, s)
                                                              : launch_map_op<W, 2>(a, L, s);
}

template <int W>
hipError_t launch_pow(const KCtx &c, const void *x, const uint64_t *e, void *out, uint64_t n, int unroll,
                      int blocks_per_cu, hipStream_t s)
{
    Launch L;
    L.blocks_per_cu = blocks_per_cu;
    const int U = (unroll == 2 || unroll == 4) ? unroll : 1;
    dim3 grid((unsigned)grid_x(n, U, 1, L));
    // ladder mode by modulus (see ladder_mode): lazy products for w = 64, N < 2^62;
    // signed three-instruction products for w = 32, N < 2^31
    const int mode = ladder_mode<W>(c.N);
    auto go = [&](auto mode_c) {
        constexpr int M = decltype(mode_c)::value;
        if (U == 4)
            hipLaunchKernelGGL((k_pow<W, 4, M>), grid, dim3(BLOCK), 0, s, c, x, e, out, n);
        else if (U == 2)
            hipLaunchKernelGGL((k_pow<W, 2, M>), grid, dim3(BLOCK), 0, s, c, x, e, out, n);
        else
            hipLaunchKernelGGL((k_pow<W, 1, M>), grid, dim3(BLOCK), 0, s, c, x, e, out, n);
    };
    if constexpr (W == 32) {
        if (mode == 3)
            go(std::integral_constant<int, 3>{});
        else
            go(std::integral_constant<int, 0>{});
    } else if constexpr (W == 64) {
        if (mode == 1)
            go(std::integral_constant<int, 1>{});
        else
            go(std::integral_constant<int, 0>{});
    } else {
        go(std::integral_constant<int, 0>{});
    }
    return hipGetLastError();
}

template <int W>
hipError_t launch_range(const KCtx &c, int variant, uint64_t T0, void *out, uint64_t n, hipStream_t s)
{
    if constexpr (W == 64) {
        return hipErrorInvalidValue;
    } else {
        using El = typename Red<W, CLASSIC>::E;
        constexpr int E = 16 / (int)sizeof(El);
        Launch L;
        const bool vec = aligned16(out);
        dim3 grid((unsigned)grid_x(vec ? n / E : n, 1, 1, L));
        if (variant == CLASSIC) {
            if (vec)
                hipLaunchKernelGGL((k_range<W, CLASSIC, E>), grid, dim3(BLOCK), 0, s, c, T0, out, n);
            else
                hipLaunchKernelGGL((k_range<W, CLASSIC, 1>), grid, dim3(BLOCK), 0, s, c, T0, out, n);
        } else if (variant == PLANTARD) {
            if (vec)
                hipLaunchKernelGGL((k_range<W, PLANTARD, E>), grid, dim3(BLOCK), 0, s, c, T0, out, n);
            else
                hipLaunchKernelGGL((k_range<W, PLANTARD, 1>), grid, dim3(BLOCK), 0, s, c, T0, out, n);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
}

}  // namespace mont

#define MONT_INSTANTIATE_WIDTH(W)                                                                             \
    namespace mont {                                                                                          \
    template hipError_t launch_map<W>(const MapArgs &, const Launch &, hipStream_t);                          \
    template hipError_t launch_pow<W>(const KCtx &, const void *, const uint64_t *, void *, uint64_t, int, int, \
                                      hipStream_t);                                                           \
    template hipError_t launch_range<W>(const KCtx &, int, uint64_t, void *, uint64_t, hipStream_t);          \
    }
