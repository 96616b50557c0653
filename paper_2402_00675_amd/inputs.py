"""Seeded synthetic inputs for the Montgomery-type workloads.

This module only draws random numbers; it holds none of the reduction
arithmetic.  The tests feed the same arrays to the CPU oracle and to the GPU
library, and the benchmark uses the same recipes.

The paper has no datasets or benchmark suites: its setting is word-size
moduli for NTT-based lattice cryptography (Sections 1 and 3).  Every workload
here is synthetic, with the shapes below:

* ``WORKLOAD_R16``  -- N = 3329, R = 2^16: two uint16 vectors of 2^20
  residues uniform in [0, N), plus every T in [0, R N).
* ``WORKLOAD_R32``  -- N = 8380417, R = 2^32 (Plantard family: R = 2^64):
  2^26 residues, uint32 uniform in [0, N) for the unsigned forms and int32
  uniform in [-(N-1)/2, (N-1)/2] for the signed forms.
* ``WORKLOAD_RNS64`` -- eight distinct random 60-bit primes, R = 2^64,
  uint64 arrays of shape [8][2^25] (limb-major), row i uniform in [0, N_i).
* ``WORKLOAD_RAGGED`` -- 4096 vectors, lengths floor(exp(U(ln 2^8, ln 2^20))),
  each with its own odd modulus: 31-bit (uint32, R = 2^32) or 62-bit
  (uint64, R = 2^64) with probability 1/2 each.
* ``WORKLOAD_SERVE`` -- 100,000 jobs with Poisson arrivals: 60% products,
  40% exponentiations with a uniform 64-bit exponent; lengths log-uniform in
  [2^8, 2^18]; modulus odd 31- or 62-bit.

Seeds: numpy PCG64 with seed ``SEED_BASE + workload index (+ repeat)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 240200675

# workload indices (used to derive seeds)
W_R16, W_R32, W_RNS64, W_RAGGED, W_SERVE = range(5)


def rng(index: int, rep: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index + 1000 * rep))


def uniform_residues(g: np.random.Generator, N: int, n: int, dtype) -> np.ndarray:
    """n integers uniform in [0, N), stored as dtype."""
    return g.integers(0, N, size=n, dtype=np.uint64).astype(dtype)


def centered_residues(g: np.random.Generator, N: int, n: int, dtype) -> np.ndarray:
    """n integers uniform in [-(N-1)/2, (N-1)/2] (N odd), stored as dtype."""
    h = (N - 1) // 2
    return (g.integers(0, N, size=n, dtype=np.int64) - h).astype(dtype)


def u64_uniform(g: np.random.Generator, n: int) -> np.ndarray:
    """n integers uniform in [0, 2^64)."""
    return g.integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)


def odd_modulus(g: np.random.Generator, bits: int) -> int:
    """Uniform odd integer with exactly `bits` bits: in [2^(bits-1), 2^bits)."""
    lo = 1 << (bits - 1)
    v = int(g.integers(lo >> 1, (1 << bits) >> 1, dtype=np.uint64))
    return 2 * v + 1


# The first twelve primes as Miller-Rabin bases: no strong pseudoprime to all of
# them exists below 3.18e23 (Sorenson and Webster, 2015), far above 2^64.
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 2^64 (the first twelve primes as bases)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def random_primes(g: np.random.Generator, bits: int, k: int) -> list:
    """k distinct primes uniform among odd `bits`-bit integers."""
    out = []
    while len(out) < k:
        c = odd_modulus(g, bits)
        if c not in out and is_prime(c):
            out.append(c)
    return out


def log_uniform_lengths(g: np.random.Generator, lo: int, hi: int, k: int) -> np.ndarray:
    """k lengths floor(exp(U(ln lo, ln hi))), clipped to [lo, hi]."""
    v = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), size=k))).astype(np.int64)
    return np.clip(v, lo, hi)


# ---------------------------------------------------------------------------
# workload descriptions

@dataclass
class R16Workload:
    N: int = 3329
    w: int = 16
    n: int = 1 << 20

    def operands(self, rep: int = 0):
        g = rng(W_R16, rep)
        return (uniform_residues(g, self.N, self.n, np.uint16),
                uniform_residues(g, self.N, self.n, np.uint16))


@dataclass
class R32Workload:
    N: int = 8380417
    w: int = 32
    n: int = 1 << 26

    def operands(self, signed: bool, rep: int = 0, n: int | None = None):
        g = rng(W_R32, rep + (500 if signed else 0))
        n = self.n if n is None else n
        if signed:
            return (centered_residues(g, self.N, n, np.int32), centered_residues(g, self.N, n, np.int32))
        return (uniform_residues(g, self.N, n, np.uint32), uniform_residues(g, self.N, n, np.uint32))


@dataclass
class RNS64Workload:
    k: int = 8
    bits: int = 60
    n: int = 1 << 25
    moduli: list = field(default_factory=list)

    def __post_init__(self):
        if not self.moduli:
            self.moduli = random_primes(rng(W_RNS64), self.bits, self.k)

    def operands(self, rep: int = 0, n: int | None = None):
        """a, b of shape [k][n], row i uniform in [0, N_i)."""
        g = rng(W_RNS64, rep + 1)
        n = self.n if n is None else n
        a = np.empty((self.k, n), dtype=np.uint64)
        b = np.empty((self.k, n), dtype=np.uint64)
        for i, N in enumerate(self.moduli):
            a[i] = g.integers(0, N, size=n, dtype=np.uint64)
            b[i] = g.integers(0, N, size=n, dtype=np.uint64)
        return a, b


@dataclass
class RaggedWorkload:
    nseg: int = 4096
    lo: int = 1 << 8
    hi: int = 1 << 20

    def segments(self, rep: int = 0, nseg: int | None = None, hi: int | None = None):
        """Per segment: (length, modulus bits, modulus)."""
        g = rng(W_RAGGED, rep)
        nseg = self.nseg if nseg is None else nseg
        lens = log_uniform_lengths(g, self.lo, self.hi if hi is None else hi, nseg)
        wide = g.integers(0, 2, size=nseg).astype(bool)
        mods = [odd_modulus(g, 62 if wd else 31) for wd in wide]
        return lens, wide, mods

    def operands(self, lens, wide, mods, rep: int = 0):
        """Operands packed into one uint32 pool and one uint64 pool, in segment
        order, each vector starting on a 16-byte boundary (so a per-vector
        launch can use 16-byte accesses too)."""
        g = rng(W_RAGGED, rep + 1)
        pad32 = [(int(n) + 3) // 4 * 4 for n, wd in zip(lens, wide) if not wd]
        pad64 = [(int(n) + 1) // 2 * 2 for n, wd in zip(lens, wide) if wd]
        n32 = int(sum(pad32))
        n64 = int(sum(pad64))
        a32 = np.zeros(n32, np.uint32)
        b32 = np.zeros(n32, np.uint32)
        a64 = np.zeros(n64, np.uint64)
        b64 = np.zeros(n64, np.uint64)
        offs = []
        o32 = o64 = 0
        for n, wd, N in zip(lens, wide, mods):
            n = int(n)
            if wd:
                a64[o64:o64 + n] = g.integers(0, N, size=n, dtype=np.uint64)
                b64[o64:o64 + n] = g.integers(0, N, size=n, dtype=np.uint64)
                offs.append(o64)
                o64 += (n + 1) // 2 * 2
            else:
                a32[o32:o32 + n] = g.integers(0, N, size=n, dtype=np.uint64).astype(np.uint32)
                b32[o32:o32 + n] = g.integers(0, N, size=n, dtype=np.uint64).astype(np.uint32)
                offs.append(o32)
                o32 += (n + 3) // 4 * 4
        return np.array(offs, np.int64), (a32, b32), (a64, b64)


@dataclass
class ServeWorkload:
    njobs: int = 100_000
    p_mul: float = 0.6
    lo: int = 1 << 8
    hi: int = 1 << 18

    def jobs(self, rate_per_s: float, rep: int = 0, njobs: int | None = None):
        """Job list: arrival time (s), op ('mul' | 'pow'), length, modulus, seed."""
        g = rng(W_SERVE, rep)
        njobs = self.njobs if njobs is None else njobs
        gaps = g.exponential(1.0 / rate_per_s, size=njobs)
        t = np.cumsum(gaps) - gaps[0]
        ops = np.where(g.uniform(size=njobs) < self.p_mul, 0, 1)
        lens = log_uniform_lengths(g, self.lo, self.hi, njobs)
        wide = g.integers(0, 2, size=njobs).astype(bool)
        mods = [odd_modulus(g, 62 if wd else 31) for wd in wide]
        seeds = g.integers(0, 2**63 - 1, size=njobs, dtype=np.int64)
        return t, ops, lens, wide, mods, seeds
