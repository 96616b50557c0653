/*
 * CPU oracle for Montgomery-type reduction, multiplication and
 * exponentiation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library calls, links or loads
 * this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or constant with
 * the GPU path.
 *
 * Every result is computed from its plain number-theoretic definition with
 * ordinary 128-bit integer division ('%'), never with Montgomery arithmetic:
 *
 *   c(T) = (T mod N) * (R^{-1} mod N) mod N,  R^{-1} by extended Euclid,
 *
 * which is the value the paper's CRT framework (Section 2, eq. qin3/qin4)
 * says every Montgomery-type reduction returns up to the choice of
 * representative.  Each variant then picks the representative its
 * algorithm is proved to return:
 *
 *   classic REDC (Section 1)            c                    in [0, N)
 *   signed Montgomery (Section 3.1,
 *     Algorithm 1)                      the r = c (mod N) with
 *                                       T/R - N/2 < r <= T/R + N/2
 *   Plantard (Section 3.2, Alg. 2)      (-c) mod N           in [0, N)
 *   signed Plantard (Section 3.2,
 *     Algorithm 3)                      (-c) mods N
 *   Huang's signed Plantard with a
 *     parameter alpha >= 1 (Section 3.3,
 *     Algorithm 4)                      (-c) mods N
 *
 * "mods" is the least absolute remainder in [-N/2, N/2) (Section 2).  For
 * odd N this is [-(N-1)/2, (N-1)/2].
 *
 * The signed-Montgomery window follows from the algorithm's choice of the
 * quotient digit m = T N^{-1} mods R, i.e. m in [-R/2, R/2): with
 * r = (T - mN)/R, m >= -R/2 <=> r <= T/R + N/2 and m < R/2 <=>
 * r > T/R - N/2.  The window is a half-open interval of length N, so it
 * holds exactly one integer of each residue class.
 *
 * Input ranges follow the Require lines of the algorithms (inclusive bounds
 * where the Require line is inclusive).  An input outside its variant's
 * range is reported as an error rather than given a value, because there
 * the algorithms are not defined.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

/* Variant codes of the oracle's own interface. */
enum {
    ORC_CLASSIC = 0,
    ORC_SIGNED = 1,
    ORC_PLANTARD = 2,
    ORC_SIGNED_PLANTARD = 3,
    ORC_SIGNED_PLANTARD_ALPHA = 4
};

enum { ORC_OK = 0, ORC_EARG = -1, ORC_EDOMAIN = -2 };

static __thread int64_t orc_bad_index = -1;

int64_t orc_last_bad_index(void) { return orc_bad_index; }

/* 2^k mod N by k modular doublings. */
static uint64_t pow2_mod(unsigned k, uint64_t N)
{
    u128 r = 1 % N;
    for (unsigned i = 0; i < k; ++i)
        r = (r * 2u) % N;
    return (uint64_t)r;
}

/* a^{-1} mod N by the extended Euclidean algorithm; 0 when gcd(a, N) != 1. */
uint64_t orc_inv_mod(uint64_t a, uint64_t N)
{
    if (N < 2)
        return 0;
    i128 r0 = (i128)N, r1 = (i128)(a % N);
    i128 s0 = 0, s1 = 1;
    while (r1 != 0) {
        i128 q = r0 / r1;
        i128 t = r0 - q * r1;
        r0 = r1;
        r1 = t;
        t = s0 - q * s1;
        s0 = s1;
        s1 = t;
    }
    if (r0 != 1)
        return 0;
    if (s0 < 0)
        s0 += (i128)N;
    return (uint64_t)s0;
}

/* Non-negative remainder of a signed 128-bit integer. */
static uint64_t mod_signed(i128 T, uint64_t N)
{
    i128 r = T % (i128)N;
    if (r < 0)
        r += (i128)N;
    return (uint64_t)r;
}

/* x in [0, N) mapped to the least absolute remainder, N odd. */
static int64_t mods_of(uint64_t x, uint64_t N)
{
    return x <= (N - 1) / 2 ? (int64_t)x : (int64_t)((i128)x - (i128)N);
}

/* Parameters of one reduction, fixed per call. */
typedef struct {
    int variant;
    unsigned w;     /* machine word: R = 2^w (classic, signed), 2^(2w) (Plantard family) */
    unsigned alpha; /* Algorithm 4 parameter */
    uint64_t N;
    uint64_t rinv;  /* R^{-1} mod N for the variant's own R */
} orc_par;

static int par_init(orc_par *p, int variant, unsigned w, unsigned alpha, uint64_t N)
{
    if (w < 2 || w > 64 || N < 3 || (N & 1u) == 0)
        return ORC_EARG;
    if (w < 64 && N >> w)
        return ORC_EARG; /* N must be below the word */
    p->variant = variant;
    p->w = w;
    p->alpha = alpha;
    p->N = N;
    unsigned logR;
    switch (variant) {
    case ORC_CLASSIC:
        logR = w;
        break;
    case ORC_SIGNED:
        /* Algorithm 1: 2N < R */
        if (N >= ((u128)1 << (w - 1)))
            return ORC_EDOMAIN;
        logR = w;
        break;
    case ORC_PLANTARD: {
        /* Algorithm 2: N < 2^w / phi  <=>  N^2 < (2^w - N) 2^w  (phi^2 = phi + 1) */
        u128 lhs = (u128)N * N;
        u128 rhs = (((u128)1 << w) - N) << w;
        if (!(lhs < rhs))
            return ORC_EDOMAIN;
        logR = 2 * w;
        break;
    }
    case ORC_SIGNED_PLANTARD:
        /* Algorithm 3: N < 2^(w-1) */
        if (N >= ((u128)1 << (w - 1)))
            return ORC_EDOMAIN;
        logR = 2 * w;
        break;
    case ORC_SIGNED_PLANTARD_ALPHA:
        /* Algorithm 4 is proved only for alpha >= 1; N < 2^(w - alpha - 1) */
        if (alpha < 1 || alpha + 2 > w)
            return ORC_EDOMAIN;
        if (N >= ((u128)1 << (w - alpha - 1)))
            return ORC_EDOMAIN;
        logR = 2 * w;
        break;
    default:
        return ORC_EARG;
    }
    p->rinv = orc_inv_mod(pow2_mod(logR, N), N);
    return p->rinv ? ORC_OK : ORC_EARG;
}

/* Reduction of an unsigned 128-bit T (classic, Plantard). */
static int reduce_u(const orc_par *p, u128 T, uint64_t *out)
{
    const uint64_t N = p->N;
    if (p->variant == ORC_CLASSIC) {
        u128 RN = (u128)N << p->w; /* R N < 2^128 since N < 2^w <= 2^64 */
        if (!(T < RN))
            return ORC_EDOMAIN;
    } else { /* ORC_PLANTARD: 0 <= T <= N^2 */
        if (T > (u128)N * N)
            return ORC_EDOMAIN;
    }
    uint64_t c = (uint64_t)(((u128)(uint64_t)(T % N) * p->rinv) % N);
    *out = p->variant == ORC_CLASSIC ? c : (c == 0 ? 0 : N - c);
    return ORC_OK;
}

/* Reduction of a signed 128-bit T (signed, signed Plantard, Algorithm 4). */
static int reduce_s(const orc_par *p, i128 T, int64_t *out)
{
    const uint64_t N = p->N;
    const unsigned w = p->w;
    i128 aT = T < 0 ? -T : T;
    if (p->variant == ORC_SIGNED) {
        /* |T| < N R / 2  <=>  |T| < N 2^(w-1) */
        if (!(aT < ((i128)N << (w - 1))))
            return ORC_EDOMAIN;
    } else if (p->variant == ORC_SIGNED_PLANTARD) {
        if (aT > ((i128)1 << (2 * w - 2)))
            return ORC_EDOMAIN;
    } else { /* ORC_SIGNED_PLANTARD_ALPHA: |T| <= 2^(2 alpha) N^2 */
        if (aT > (((i128)N * (i128)N) << (2 * p->alpha)))
            return ORC_EDOMAIN;
    }
    uint64_t c = (uint64_t)(((u128)mod_signed(T, N) * p->rinv) % N);
    if (p->variant == ORC_SIGNED) {
        /* T = a1 R + a0 with 0 <= a0 < R */
        i128 a1 = T >> w; /* arithmetic shift = floor division */
        i128 a0 = T - (a1 << w);
        uint64_t d0 = mod_signed((i128)c - a1, N);
        i128 hi = (a0 < ((i128)1 << (w - 1))) ? (i128)((N - 1) / 2) : (i128)((N + 1) / 2);
        i128 d = (i128)d0 <= hi ? (i128)d0 : (i128)d0 - (i128)N;
        *out = (int64_t)(a1 + d);
    } else {
        uint64_t neg = c == 0 ? 0 : N - c;
        *out = mods_of(neg, N);
    }
    return ORC_OK;
}

static int is_signed_variant(int v)
{
    return v == ORC_SIGNED || v == ORC_SIGNED_PLANTARD || v == ORC_SIGNED_PLANTARD_ALPHA;
}

/* ---- container access: elements are w/8 bytes, T is 2w/8 bytes ---------- */

static i128 load_elem(const void *p, size_t i, unsigned cw, int sgn)
{
    switch (cw) {
    case 16:
        return sgn ? (i128)((const int16_t *)p)[i] : (i128)((const uint16_t *)p)[i];
    case 32:
        return sgn ? (i128)((const int32_t *)p)[i] : (i128)((const uint32_t *)p)[i];
    default:
        return sgn ? (i128)((const int64_t *)p)[i] : (i128)((const uint64_t *)p)[i];
    }
}

static u128 load_T_u(const void *p, size_t i, unsigned cw)
{
    switch (cw) {
    case 16:
        return ((const uint32_t *)p)[i];
    case 32:
        return ((const uint64_t *)p)[i];
    default: {
        const uint64_t *q = (const uint64_t *)p + 2 * i;
        return ((u128)q[1] << 64) | q[0];
    }
    }
}

static i128 load_T_s(const void *p, size_t i, unsigned cw)
{
    switch (cw) {
    case 16:
        return ((const int32_t *)p)[i];
    case 32:
        return ((const int64_t *)p)[i];
    default:
        return (i128)load_T_u(p, i, cw);
    }
}

static void store_elem(void *p, size_t i, unsigned cw, uint64_t v)
{
    switch (cw) {
    case 16:
        ((uint16_t *)p)[i] = (uint16_t)v;
        break;
    case 32:
        ((uint32_t *)p)[i] = (uint32_t)v;
        break;
    default:
        ((uint64_t *)p)[i] = v;
        break;
    }
}

static int reduce_any(const orc_par *p, int sgn, i128 Ts, u128 Tu, uint64_t *bits)
{
    if (sgn) {
        int64_t r;
        int rc = reduce_s(p, Ts, &r);
        *bits = (uint64_t)r;
        return rc;
    }
    return reduce_u(p, Tu, bits);
}

/*
 * out[i] = REDC_variant(T[i]) for container width cw in {16, 32, 64}
 * (w = cw).  T elements are 2w bits: uint32/int32, uint64/int64, or
 * little-endian (lo, hi) uint64 pairs for w = 64.
 */
int orc_redc(int variant, unsigned cw, unsigned alpha, uint64_t N, const void *T, void *out, size_t n)
{
    if (cw != 16 && cw != 32 && cw != 64)
        return ORC_EARG;
    orc_par p;
    int rc = par_init(&p, variant, cw, alpha, N);
    if (rc)
        return rc;
    const int sgn = is_signed_variant(variant);
    orc_bad_index = -1;
    for (size_t i = 0; i < n; ++i) {
        uint64_t bits;
        rc = sgn ? reduce_any(&p, 1, load_T_s(T, i, cw), 0, &bits)
                 : reduce_any(&p, 0, 0, load_T_u(T, i, cw), &bits);
        if (rc) {
            orc_bad_index = (int64_t)i;
            return rc;
        }
        store_elem(out, i, cw, bits);
    }
    return ORC_OK;
}

/* out[i] = REDC_variant(a[i] * b[i]); a, b, out are w-bit containers. */
int orc_mul(int variant, unsigned cw, unsigned alpha, uint64_t N, const void *a, const void *b, void *out,
            size_t n)
{
    if (cw != 16 && cw != 32 && cw != 64)
        return ORC_EARG;
    orc_par p;
    int rc = par_init(&p, variant, cw, alpha, N);
    if (rc)
        return rc;
    const int sgn = is_signed_variant(variant);
    orc_bad_index = -1;
    for (size_t i = 0; i < n; ++i) {
        uint64_t bits;
        if (sgn) {
            i128 T = load_elem(a, i, cw, 1) * load_elem(b, i, cw, 1);
            rc = reduce_any(&p, 1, T, 0, &bits);
        } else {
            u128 T = (u128)load_elem(a, i, cw, 0) * (u128)load_elem(b, i, cw, 0);
            rc = reduce_any(&p, 0, 0, T, &bits);
        }
        if (rc) {
            orc_bad_index = (int64_t)i;
            return rc;
        }
        store_elem(out, i, cw, bits);
    }
    return ORC_OK;
}

/*
 * Any word size w in [2, 64] with T held in int64 (used for small words and
 * hand-checked examples): T must fit in 64 bits.  out holds the result's
 * bit pattern (two's complement for the signed variants).
 */
int orc_redc_i64(int variant, unsigned w, unsigned alpha, uint64_t N, const int64_t *T, int64_t *out, size_t n)
{
    orc_par p;
    int rc = par_init(&p, variant, w, alpha, N);
    if (rc)
        return rc;
    const int sgn = is_signed_variant(variant);
    orc_bad_index = -1;
    for (size_t i = 0; i < n; ++i) {
        uint64_t bits;
        if (!sgn && T[i] < 0) {
            orc_bad_index = (int64_t)i;
            return ORC_EDOMAIN;
        }
        rc = reduce_any(&p, sgn, (i128)T[i], (u128)(uint64_t)T[i], &bits);
        if (rc) {
            orc_bad_index = (int64_t)i;
            return rc;
        }
        out[i] = (int64_t)bits;
    }
    return ORC_OK;
}

/* out[i] = x[i]^e[i] mod N by square-and-multiply with '%'; x^0 = 1. */
int orc_pow(unsigned cw, uint64_t N, const void *x, const uint64_t *e, void *out, size_t n)
{
    if ((cw != 16 && cw != 32 && cw != 64) || N < 3 || (N & 1u) == 0)
        return ORC_EARG;
    if (cw < 64 && N >> cw)
        return ORC_EARG;
    orc_bad_index = -1;
    for (size_t i = 0; i < n; ++i) {
        uint64_t base = (uint64_t)load_elem(x, i, cw, 0);
        if (base >= N) {
            orc_bad_index = (int64_t)i;
            return ORC_EDOMAIN;
        }
        uint64_t k = e[i];
        u128 acc = 1;
        u128 b = base;
        while (k) {
            if (k & 1u)
                acc = (acc * b) % N;
            b = (b * b) % N;
            k >>= 1;
        }
        store_elem(out, i, cw, (uint64_t)(acc % N));
    }
    return ORC_OK;
}

/*
 * Discrete Fourier transform over Z_N by its definition (O(n^2)):
 * forward X_k = sum_j x_j w^(j k) mod N; inverse x_j = n^{-1} sum_k X_k w^(-j k)
 * mod N with w^{-1} = w^(n-1) when w^n = 1.  x and out are n residues of
 * container width cw (unsigned).  Returns ORC_EARG when n^{-1} or w^{-1}
 * does not exist.
 */
int orc_dft(unsigned cw, uint64_t N, const void *x, uint64_t w, unsigned log2n, int inverse, void *out)
{
    if ((cw != 16 && cw != 32 && cw != 64) || N < 3 || log2n > 20)
        return ORC_EARG;
    const uint64_t n = 1ull << log2n;
    uint64_t wi = w % N;
    if (inverse) {
        wi = orc_inv_mod(wi, N);
        if (!wi)
            return ORC_EARG;
    }
    /* powers w^m for m < n */
    uint64_t *powers = (uint64_t *)malloc(n * sizeof(uint64_t));
    if (!powers)
        return ORC_EARG;
    powers[0] = 1 % N;
    for (uint64_t m = 1; m < n; ++m)
        powers[m] = (uint64_t)(((u128)powers[m - 1] * wi) % N);
    uint64_t ninv = 1;
    if (inverse) {
        ninv = orc_inv_mod(n % N, N);
        if (!ninv) {
            free(powers);
            return ORC_EARG;
        }
    }
    for (uint64_t k = 0; k < n; ++k) {
        u128 acc = 0;
        for (uint64_t j = 0; j < n; ++j) {
            const uint64_t xj = (uint64_t)load_elem(x, j, cw, 0);
            acc = (acc + (u128)xj * powers[(j * k) & (n - 1)]) % N;
        }
        store_elem(out, k, cw, (uint64_t)((acc * ninv) % N));
    }
    free(powers);
    return ORC_OK;
}
