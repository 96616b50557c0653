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
