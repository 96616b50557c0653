"""Ranges of the products by a fixed operand that the transforms rely on when
they leave coefficients unreduced between stages.

Plantard's product by a fixed operand (Section 3.2's form: b' = b N^{-1} mod
2^(2w) precomputed, m = a b' mod 2^(2w), r = floor((floor(m / 2^w) + 1) N / 2^w))
returns a b (-2^(-2w)) mod N, already reduced, for every w-bit a once
N <= 2^(w-1): the quotient estimate stays inside (k, k + 1) for
k = (m N - a b) / 2^(2w) while a b < 2^w (2^w - N).  Above that bound it fails
for some inputs.

Montgomery's product without its final subtraction, (T + mN) / R with
m = -T N^{-1} mod R, stays below 2N for every a < R when b < N (T < R N).

Both are checked here with Python integers: exhaustively over every 16-bit a,
by sampling at 32 and 64 bits (with the largest inputs always included).

Shoup's product by a fixed c with a quotient from three of the four partial
products (the CRT reconstruction's steps for moduli below 2^61) is checked the
same way: its result stays below 4N for every 64-bit input.
"""
import random

import pytest


def plantard_const(w, N, v):
    """The fixed operand for a product by v: b = -v 2^(2w) mod N, as b N^{-1} mod 2^(2w)."""
    b = (-v * pow(2, 2 * w, N)) % N
    return b * pow(N, -1, 1 << (2 * w)) % (1 << (2 * w))


def plantard_fixed(w, N, a, bp):
    m = a * bp % (1 << (2 * w))
    return ((m >> w) + 1) * N >> w


def montgomery_lazy(w, N, a, b):
    R = 1 << w
    T = a * b
    m = (-T * pow(N, -1, R)) % R
    assert (T + m * N) % R == 0
    return (T + m * N) // R


@pytest.mark.parametrize("N", [3329, 12289, 32749])
def test_plantard_fixed_exhaustive_w16(N):
    for v in (0, 1, 2, N - 1, 1234 % N, 4321 % N):
        bp = plantard_const(16, N, v)
        for a in range(1 << 16):
            assert plantard_fixed(16, N, a, bp) == a * v % N, (N, v, a)


@pytest.mark.parametrize("N", [36097, 40961])
def test_plantard_fixed_needs_the_bound(N):
    """N > 2^15: some 16-bit inputs come out wrong, so the transforms keep reducing."""
    wrong = 0
    for v in (1, 2, 12345, N - 1):
        bp = plantard_const(16, N, v)
        wrong += sum(plantard_fixed(16, N, a, bp) != a * v % N for a in range(1 << 16))
    assert wrong > 0


@pytest.mark.parametrize("w,N", [(32, 8380417), (32, 1073692673), (32, (1 << 31) - 1),
                                 (64, 1125899906826241), (64, 4611686018326724609), (64, (1 << 63) - 25)])
def test_plantard_fixed_sampled(w, N):
    g = random.Random(w * 1000003 + N % 1000)
    for _ in range(3000):
        v = g.randrange(N)
        bp = plantard_const(w, N, v)
        for a in (g.randrange(1 << w), (1 << w) - 1, (1 << w) - 1 - g.randrange(1 << 20), g.randrange(N)):
            assert plantard_fixed(w, N, a, bp) == a * v % N, (w, N, v, a)


@pytest.mark.parametrize("w,N", [(16, 3329), (16, 12289), (32, 8380417), (32, 1073692673),
                                 (64, 1125899906826241), (64, (1 << 61) - 1)])
def test_montgomery_lazy_below_2n(w, N):
    g = random.Random(w + N)
    R = 1 << w
    for _ in range(3000):
        b = g.randrange(N)
        for a in (g.randrange(R), R - 1, g.randrange(25 * N) % R):
            r = montgomery_lazy(w, N, a, b)
            assert r < 2 * N and r % N == a * b * pow(R, -1, N) % N, (w, N, a, b)


def shoup3(d, c, cq, N):
    """The CRT kernel's Shoup product with a three-partial-product quotient (the
    low x low product of d and cq dropped), modulo 2^64 as the kernel computes it."""
    M32 = (1 << 32) - 1
    d0, d1, k0, k1 = d & M32, d >> 32, cq & M32, cq >> 32
    q = d1 * k1 + ((d1 * k0) >> 32) + ((d0 * k1) >> 32)
    return (d * c - q * N) % (1 << 64), q


@pytest.mark.parametrize("bits", [40, 59, 60, 61])
def test_shoup_three_product_quotient(bits):
    """For N < 2^61, c < N, cq = floor(c 2^64 / N) and any 64-bit d: the result is
    d c mod N plus at most 3N (below 4N), and the quotient is at most 2 below the
    exact floor(d cq / 2^64).  With t < 4N and a digit v below 2N, the next
    operand t + 2N - v stays below 6N < 2^64."""
    rnd = random.Random(bits)
    for _ in range(300):
        N = rnd.randrange(1 << (bits - 1), 1 << bits) | 1
        for c in [1, 2, N - 1, N - 2, N // 2] + [rnd.randrange(1, N) for _ in range(10)]:
            cq = (c << 64) // N
            ds = [0, 1, (1 << 64) - 1, (1 << 64) - 2, 6 * N - 1, 4 * N - 1] + \
                 [rnd.randrange(1 << 64) for _ in range(20)]
            for d in ds:
                r, q = shoup3(d, c, cq, N)
                exact = (d * cq) >> 64
                assert exact - 2 <= q <= exact
                assert r < 4 * N and r % N == d * c % N, (N, c, d)
    assert 6 * ((1 << 61) - 1) < 1 << 64
