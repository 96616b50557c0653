// Reconstruction of integers from residue-number-system rows (the
// multi-modulus Chinese Remainder Theorem; Section 2 derives the two-modulus
// case from Qin's identity and points to the general one).
//
// For pairwise coprime odd moduli N_0..N_{k-1} (64-bit words) and residues
// x_i, the unique X in [0, N_0 ... N_{k-1}) with X = x_i (mod N_i) is formed by
// Garner's mixed-radix conversion
//     v_0 = x_0,  v_i = ((x_i - v_0) c_{0,i} - v_1) c_{1,i} ... - v_{i-1}) c_{i-1,i}  mod N_i,
//     c_{j,i} = N_j^{-1} mod N_i,
//     X = v_0 + N_0 (v_1 + N_1 (v_2 + ... + N_{k-2} v_{k-1})),
// where each modular product is a product by a constant.  In general it is a
// Montgomery product against c_{j,i} R mod N_i: REDC(t (c R)) = t c (mod N_i).
// A v_j that is not yet reduced modulo N_i is multiplied the same way
// (v_j (cR) < R N_i is inside REDC's range), so (t - v_j) c =
// REDC(t cR) - REDC(v_j cR) needs no separate reduction; when every modulus is
// below twice every other one, a single conditional subtraction reduces v_j
// instead (one product per step).  When moreover every modulus is below 2^62
// the steps take Shoup's fixed-operand product on unreduced values (see
// FORM 2 below).  The mixed-radix digits are then folded into k little-endian
// 64-bit words by Horner's rule with 64x64->128 multiply-adds.  Constants are
// kernel arguments (read with scalar loads); residues are limb-major [k][ld],
// the result element-major [n][k] words, written through LDS.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mont_common.hpp"
#ifdef MONT_DEBUG
#include "mont_debug.hpp"
#endif

namespace mont {

constexpr int CRT_MAX = 16;

constexpr int CRT_PAIRS = CRT_MAX * (CRT_MAX - 1) / 2;

// The constant of step (j, i), j < i, sits at pair index i (i - 1)/2 + j.
struct CrtTab {
    uint64_t N[CRT_MAX];
    uint64_t np[CRT_MAX];
    uint64_t c[CRT_PAIRS];   // forms 0, 1: (N_j^{-1} mod N_i) R mod N_i;  forms 2, 3: N_j^{-1} mod N_i
    uint64_t cq[CRT_PAIRS];  // forms 2, 3: floor(c 2^64 / N_i)
};

__host__ __device__ constexpr int crt_pair(int j, int i) { return i * (i - 1) / 2 + j; }

// Shoup's product by a fixed c < N with the precomputed quotient factor
// cq = floor(c 2^64 / N): for any 64-bit d, q = floor(d cq / 2^64) is at
// least floor(d c / N) - 1 and at most d c / N, so d c - q N (computed modulo
// 2^64) is d c mod N or that plus N: a value below 2N, whatever d is.
__device__ __forceinline__ uint64_t shoup_mul(uint64_t d, uint64_t c, uint64_t cq, uint64_t N)
{
    const uint64_t q = mulhi_64(d, cq);
    return d * c - q * N;
}

// Shoup's product with the quotient from three of the four 32 x 32 partial
// products of d cq (the low x low one is dropped): with d = d1 2^32 + d0 and
// cq = k1 2^32 + k0, q = d1 k1 + hi(d1 k0) + hi(d0 k1) misses from the exact
// floor(d cq / 2^64) only the carries of lo(d1 k0) + lo(d0 k1) + hi(d0 k0)
// into bit 64, at most 2.  So q is between floor(d c / N) - 3 and d c / N, and
// d c - q N is d c mod N plus 0, N, 2N or 3N: a value below 4N.
__device__ __forceinline__ uint64_t shoup_mul3(uint64_t d, uint64_t c, uint64_t cq, uint64_t N)
{
    const uint32_t d0 = (uint32_t)d, d1 = (uint32_t)(d >> 32);
    const uint32_t k0 = (uint32_t)cq, k1 = (uint32_t)(cq >> 32);
    const uint64_t q = (uint64_t)d1 * k1 + ((uint64_t)__umulhi(d1, k0) + __umulhi(d0, k1));
    return d * c - q * N;
}

// t - m when t >= m, else t: the borrow of the subtraction picks the result.
__device__ __forceinline__ uint64_t sub_if_ge(uint64_t t, uint64_t m)
{
    unsigned b0, b1;
    const uint32_t dl = __builtin_subc((uint32_t)t, (uint32_t)m, 0u, &b0);
    const uint32_t dh = __builtin_subc((uint32_t)(t >> 32), (uint32_t)(m >> 32), b0, &b1);
    return b1 ? t : ((uint64_t)dh << 32 | dl);
}

// a N + c for N < 2^62 (n1 < 2^30) and any 64-bit a, c; the sum is below
// 2^127.  Partial sums: a0 n0 + lo(c) < 2^64, t1 = a0 n1 + hi(p00) < 2^62 +
// 2^32, mid = a1 n0 + lo(t1) + hi(c) < 2^64, hi = a1 n1 + hi(t1) + hi(mid)
// < 2^63: no carry word anywhere.
__device__ __forceinline__ u128v mul_add_62(uint64_t a, uint64_t N, uint64_t c)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t n0 = (uint32_t)N, n1 = (uint32_t)(N >> 32);
    const uint64_t p00 = (uint64_t)a0 * n0 + (uint32_t)c;
    const uint64_t t1 = (uint64_t)a0 * n1 + (p00 >> 32);
    const uint64_t mid = (uint64_t)a1 * n0 + ((uint64_t)(uint32_t)t1 + (c >> 32));
    const uint64_t hi = (uint64_t)a1 * n1 + ((t1 >> 32) + (mid >> 32));
    return {(mid << 32) | (uint32_t)p00, hi};
}

// FORM 0: any coprime odd moduli (Montgomery products, two per step).
// FORM 1 (NARROW): every modulus below twice every other one, so v_j needs one
// conditional subtraction and each step is one Montgomery product.  FORM 2:
// NARROW and every modulus below 2^62: Shoup steps on unreduced values,
// t <- shoup(t + 2N_i - v_j) with t < 2N_i and v_j < N_j < 2N_i, so the
// operand stays below 4N_i < 2^64 and each step is one fixed-operand product
// with no reduction before or after it (the digit is reduced once at the
// end), and carry-free Horner steps.  FORM 3: FORM 2 with every modulus below
// 2^61 and the three-product quotient: t < 4N_i, the operand t + 2N_i - v_j
// stays below 6N_i < 2^64, and the digit is reduced by subtracting 2N_i and
// N_i at the end.
template <int K, int FORM>
__global__ void __launch_bounds__(BLOCK)
    k_crt(CrtTab tab, const uint64_t *__restrict__ res, uint64_t ld, uint64_t n, uint64_t *__restrict__ out)
{
    const uint64_t base = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * BLOCK;  // the block's first element
    const uint64_t e = base + threadIdx.x;
    // the lanes past n still take part in the block's output pass: they read
    // the last element (their results are not written)
    const uint64_t *p = res + (e < n ? e : n - 1);
    uint64_t x[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        x[i] = __builtin_nontemporal_load(p);
        if (i + 1 < K)
            p += ld;  // never past the last row
    }
    uint64_t v[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        KCtx c{};
        c.N = tab.N[i];
        c.nprime = tab.np[i];
        const Red<64, CLASSIC> red(c);
        uint64_t t = x[i];
#pragma unroll
        for (int j = 0; j < i; ++j) {
            const uint64_t cb = tab.c[crt_pair(j, i)];
            if constexpr (FORM == 3) {
                t = shoup_mul3(t + 2 * c.N - v[j], cb, tab.cq[crt_pair(j, i)], c.N);
            } else if constexpr (FORM == 2) {
                t = shoup_mul(t + 2 * c.N - v[j], cb, tab.cq[crt_pair(j, i)], c.N);
            } else if constexpr (FORM == 1) {
                const uint64_t vj = v[j] >= c.N ? v[j] - c.N : v[j];
                const uint64_t d = t >= vj ? t - vj : t + (c.N - vj);
                t = red.mul(d, cb);
            } else {
                const uint64_t a = red.mul(t, cb);
                const uint64_t b = red.mul(v[j], cb);
                t = a >= b ? a - b : a + (c.N - b);
            }
        }
        if constexpr (FORM == 3)
            t = sub_if_ge(t, 2 * c.N);
        if constexpr (FORM >= 2)
            t = sub_if_ge(t, c.N);
        v[i] = t;
    }
    uint64_t acc[K];
    acc[0] = v[K - 1];
#pragma unroll
    for (int w = 1; w < K; ++w)
        acc[w] = 0;
#pragma unroll
    for (int i = K - 2; i >= 0; --i) {
        const uint64_t Ni = tab.N[i];
        uint64_t carry = v[i];
        // acc holds K - 1 - i words; acc * N_i + v_i fills K - i words
#pragma unroll
        for (int w = 0; w < K - 1 - i; ++w) {
            if constexpr (FORM >= 2) {
                const u128v p = mul_add_62(acc[w], Ni, carry);
                acc[w] = p.lo;
                carry = p.hi;
            } else {
                const u128v p = mul_64x64(acc[w], Ni);
                const uint64_t lo = p.lo + carry;
                carry = p.hi + (lo < carry);
                acc[w] = lo;
            }
        }
        acc[K - 1 - i] = carry;
    }
    // The block's results leave through LDS: element-major output written
    // straight from the lanes would put 16-byte stores 8k bytes apart, every
    // wave writing parts of many cache lines at once (the access pattern
    // alone, without arithmetic, runs at a quarter of the rate of the same
    // bytes written as below).  Here consecutive lanes write consecutive
    // 16-byte chunks of the block's contiguous output.  Rows of K + 1 words
    // spread each lane's LDS writes over the banks.
    constexpr uint32_t SR = K + 1;
    __shared__ uint64_t st[BLOCK * SR];
#pragma unroll
    for (int w = 0; w < K; ++w)
        st[threadIdx.x * SR + w] = acc[w];
    __syncthreads();
    const uint32_t words = (uint32_t)(min((uint64_t)BLOCK, n - base) * K);
    uint64_t *ob = out + base * K;  // 16-byte aligned: out is, and base is a multiple of BLOCK
    for (uint32_t q = threadIdx.x; 2 * q < words; q += BLOCK) {
        const uint32_t w0 = 2 * q, w1 = w0 + 1;
        const uint64_t a0 = st[(w0 / K) * SR + w0 % K];
        if (w1 < words) {
            const uint64_t a1 = st[(w1 / K) * SR + w1 % K];
            u32x4 v;
            v.x = (uint32_t)a0;
            v.y = (uint32_t)(a0 >> 32);
            v.z = (uint32_t)a1;
            v.w = (uint32_t)(a1 >> 32);
            __builtin_nontemporal_store(v, (u32x4 *)(ob + w0));
        } else {
            ob[w0] = a0;
        }
    }
}

template <int K>
static void go_crt(const CrtTab &t, int form, const uint64_t *res, uint64_t ld, uint64_t n, uint64_t *out,
                   hipStream_t s)
{
    const unsigned grid = (unsigned)((n + BLOCK - 1) / BLOCK);
    if (form == 3)
        hipLaunchKernelGGL((k_crt<K, 3>), dim3(grid), dim3(BLOCK), 0, s, t, res, ld, n, out);
    else if (form == 2)
        hipLaunchKernelGGL((k_crt<K, 2>), dim3(grid), dim3(BLOCK), 0, s, t, res, ld, n, out);
    else if (form == 1)
        hipLaunchKernelGGL((k_crt<K, 1>), dim3(grid), dim3(BLOCK), 0, s, t, res, ld, n, out);
    else
        hipLaunchKernelGGL((k_crt<K, 0>), dim3(grid), dim3(BLOCK), 0, s, t, res, ld, n, out);
}

typedef unsigned __int128 u128;

// a^{-1} mod m (m odd, gcd 1) by the extended Euclidean algorithm; 0 if none.
static uint64_t inv_mod(uint64_t a, uint64_t m)
{
    __int128 r0 = m, r1 = a % m, s0 = 0, s1 = 1;
    while (r1) {
        const __int128 q = r0 / r1, r2 = r0 - q * r1, s2 = s0 - q * s1;
        r0 = r1;
        r1 = r2;
        s0 = s1;
        s1 = s2;
    }
    if (r0 != 1)
        return 0;
    return (uint64_t)(s0 < 0 ? s0 + m : s0);
}

}  // namespace mont

using namespace mont;

extern "C" mont_status_t mont_crt(const mont_ctx_t *ctxs, uint32_t k, const void *res, size_t n, size_t ld,
                                  void *out, void *stream)
{
    if (!ctxs || k < 1 || k > CRT_MAX)
        return fail(MONT_E_INVAL, "need 1 <= k <= %d moduli", CRT_MAX);
    for (uint32_t i = 0; i < k; ++i) {
        mont_status_t rc = check_ctx(&ctxs[i]);
        if (rc)
            return rc;
        if (ctxs[i].w != 64)
            return fail(MONT_E_UNSUPPORTED, "mont_crt takes 64-bit word contexts");
    }
    if (n > ld)
        return fail(MONT_E_INVAL, "n > ld");
    CrtTab t{};
    uint64_t lo = ~0ull, hi = 0;
    for (uint32_t i = 0; i < k; ++i) {
        t.N[i] = ctxs[i].N;
        t.np[i] = ctxs[i].nprime;
        lo = std::min(lo, ctxs[i].N);
        hi = std::max(hi, ctxs[i].N);
    }
    const bool narrow = (u128)hi < 2 * (u128)lo;  // every v_j < 2 N_i: one conditional subtraction reduces it
    const int form = narrow ? (hi < (1ull << 61) ? 3 : hi < (1ull << 62) ? 2 : 1) : 0;
    for (uint32_t i = 1; i < k; ++i) {
        const uint64_t Ni = ctxs[i].N;
        for (uint32_t j = 0; j < i; ++j) {
            const uint64_t c = inv_mod(ctxs[j].N % Ni, Ni);
            if (!c)
                return fail(MONT_E_DOMAIN, "moduli %u and %u are not coprime", j, i);
            const int p = crt_pair((int)j, (int)i);
            if (form >= 2) {
                t.c[p] = c;
                t.cq[p] = (uint64_t)(((u128)c << 64) / Ni);  // below 2^64: c < N_i
            } else {
                t.c[p] = (uint64_t)(((u128)c * ctxs[i].r_mod_n) % Ni);  // c R mod N_i
            }
        }
    }
    if (n == 0)
        return MONT_OK;
    if (!res || !out || ((uintptr_t)out & 15u))
        return fail(MONT_E_INVAL, "null residues or output not 16-byte aligned");
    if ((n + BLOCK - 1) / BLOCK > 0x7fffffffull)
        return fail(MONT_E_INVAL, "too many elements");
    hipStream_t s = (hipStream_t)stream;
    const uint64_t *r = (const uint64_t *)res;
    uint64_t *o = (uint64_t *)out;
#ifdef MONT_DEBUG
    for (uint32_t i = 0; i < k; ++i)
        if (const hipError_t de = debug_check(DBG_BELOW_N, ctxs[i], CLASSIC, r + (size_t)i * ld, nullptr, 0, n, s))
            return hip_fail(de, "precondition check");
#endif
    switch (k) {
#define C(K)                                \
    case K:                                 \
        go_crt<K>(t, form, r, ld, n, o, s);   \
        break;
        C(1) C(2) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16)
#undef C
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MONT_OK : hip_fail(e, "mont_crt launch");
}
