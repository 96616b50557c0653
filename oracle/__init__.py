"""CPU oracle for Montgomery-type reductions (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The library never does, and this package
imports nothing from the library: the two share no code, constants or
tables.

Results are computed from plain definitions (see ``orc.c``): the value
``T * R^{-1} mod N`` is found with ordinary 128-bit division and an
extended-Euclid inverse, then each variant's proved representative is picked
(classic REDC, Section 1; signed Montgomery, Algorithm 1; Plantard,
Algorithm 2; signed Plantard, Algorithm 3; Huang's signed Plantard for
alpha >= 1, Algorithm 4).

Two pieces are pure Python because they are per-modulus or per-example:

* :func:`constants` -- the per-modulus constants of each algorithm
  (``N^{-1} mod R``, ``N' = R - N^{-1}`` from REDC's definition in Section 1,
  ``N^{-1} mods R`` for the signed forms, ``R mod N``, ``R^2 mod N``), from an
  extended-Euclid inverse;
* :func:`sigpredc2_steps` -- Algorithm 4 evaluated step by step, which for
  alpha = 0 is *not* a correct reduction (Example 3.1); it exists only so the
  tests can reproduce the paper's counter-example.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

VARIANTS = {
    "classic": 0,
    "signed": 1,
    "plantard": 2,
    "signed_plantard": 3,
    "signed_plantard_alpha": 4,
}
SIGNED = {"signed", "signed_plantard", "signed_plantard_alpha"}


class OracleDomainError(ValueError):
    """An input lies outside the Require range of its algorithm."""


def build(force: bool = False) -> str:
    """Compile ``orc.c`` with gcc into ``liborc.so`` next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        vp, u64, u32, i32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint, ctypes.c_int, ctypes.c_size_t
        lib.orc_redc.argtypes = [i32, u32, u32, u64, vp, vp, sz]
        lib.orc_mul.argtypes = [i32, u32, u32, u64, vp, vp, vp, sz]
        lib.orc_redc_i64.argtypes = [i32, u32, u32, u64, vp, vp, sz]
        lib.orc_pow.argtypes = [u32, u64, vp, vp, vp, sz]
        lib.orc_dft.argtypes = [u32, u64, vp, u64, u32, i32, vp]
        lib.orc_dft.restype = i32
        lib.orc_inv_mod.argtypes = [u64, u64]
        lib.orc_inv_mod.restype = u64
        lib.orc_last_bad_index.restype = ctypes.c_int64
        for f in (lib.orc_redc, lib.orc_mul, lib.orc_redc_i64, lib.orc_pow):
            f.restype = i32
        _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc == 0:
        return
    if rc == -2:
        raise OracleDomainError("%s: input outside the algorithm's range (first bad index %d)"
                                % (what, _load().orc_last_bad_index()))
    raise ValueError("%s: bad arguments (rc=%d)" % (what, rc))


def elem_dtype(variant: str, w: int):
    s = variant in SIGNED
    return {16: np.int16 if s else np.uint16, 32: np.int32 if s else np.uint32,
            64: np.int64 if s else np.uint64}[w]


def T_dtype(variant: str, w: int):
    """Container of a 2w-bit input T (w = 64 uses (lo, hi) uint64 pairs)."""
    s = variant in SIGNED
    return {16: np.int32 if s else np.uint32, 32: np.int64 if s else np.uint64, 64: np.uint64}[w]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def redc(variant: str, w: int, N: int, T: np.ndarray, alpha: int = 0) -> np.ndarray:
    """REDC of every T[i] (2w-bit container) for word size w in {16, 32, 64}."""
    T = np.ascontiguousarray(T)
    n = T.shape[0]
    out = np.empty(n, dtype=elem_dtype(variant, w))
    _check(_load().orc_redc(VARIANTS[variant], w, alpha, N, _ptr(T), _ptr(out), n), "redc")
    return out


def mul(variant: str, w: int, N: int, a: np.ndarray, b: np.ndarray, alpha: int = 0) -> np.ndarray:
    """REDC(a[i] * b[i]) for word size w in {16, 32, 64}."""
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    assert a.shape == b.shape and a.ndim == 1
    out = np.empty(a.shape[0], dtype=elem_dtype(variant, w))
    _check(_load().orc_mul(VARIANTS[variant], w, alpha, N, _ptr(a), _ptr(b), _ptr(out), a.shape[0]), "mul")
    return out


def redc_small(variant: str, w: int, N: int, T, alpha: int = 0) -> np.ndarray:
    """REDC for any word size 2 <= w <= 64 with T given as int64 values."""
    T = np.ascontiguousarray(np.asarray(T, dtype=np.int64))
    out = np.empty(T.shape[0], dtype=np.int64)
    _check(_load().orc_redc_i64(VARIANTS[variant], w, alpha, N, _ptr(T), _ptr(out), T.shape[0]), "redc_small")
    if variant not in SIGNED:
        out = out.view(np.uint64)
    return out


def pow(w: int, N: int, x: np.ndarray, e: np.ndarray) -> np.ndarray:  # noqa: A001
    """x[i] ** e[i] mod N (ordinary residues in and out, x^0 = 1)."""
    x = np.ascontiguousarray(x)
    e = np.ascontiguousarray(e, dtype=np.uint64)
    assert x.shape == e.shape
    out = np.empty_like(x)
    _check(_load().orc_pow(w, N, _ptr(x), _ptr(e), _ptr(out), x.shape[0]), "pow")
    return out


def dft(w: int, N: int, x: np.ndarray, root: int, inverse: bool = False) -> np.ndarray:
    """Transform of one vector by the definition: X_k = sum_j x_j root^(j k) mod N (forward), or
    x_j = n^{-1} sum_k X_k root^(-j k) mod N (inverse); len(x) a power of two."""
    x = np.ascontiguousarray(x)
    n = x.shape[0]
    log2n = n.bit_length() - 1
    assert 1 << log2n == n
    out = np.empty_like(x)
    _check(_load().orc_dft(w, N, _ptr(x), root, log2n, 1 if inverse else 0, _ptr(out)), "dft")
    return out


def inv_mod(a: int, N: int) -> int:
    """a^{-1} mod N (N < 2^64) by the C extended-Euclid routine; 0 if none."""
    return int(_load().orc_inv_mod(a, N))


# --------------------------------------------------------------------------
# pure-Python pieces

def _egcd_inverse(a: int, m: int) -> int:
    """Inverse of a modulo m by the extended Euclidean algorithm (Python ints)."""
    r0, r1, s0, s1 = m, a % m, 0, 1
    while r1:
        q = r0 // r1
        r0, r1 = r1, r0 - q * r1
        s0, s1 = s1, s0 - q * s1
    if r0 != 1:
        raise ValueError("%d is not invertible modulo %d" % (a, m))
    return s0 % m


def mods(x: int, n: int) -> int:
    """Least absolute remainder of x modulo n, in [-n/2, n/2) (Section 2)."""
    r = x % n
    return r - n if 2 * r >= n else r


def constants(N: int, w: int) -> dict:
    """Per-modulus constants for word size w (Python ints).

    R = 2^w for classic and signed Montgomery; R2 = 2^(2w) for the Plantard
    family.  ``nprime`` is N' = R - (N^{-1} mod R) of REDC (Section 1).
    ``ninv_mods`` is N^{-1} mods R (Algorithm 1) and ``ninv2_mods`` is
    N^{-1} mods 2^(2w) (Algorithms 3, 4).  ``valid`` lists the variants whose
    precondition on N holds.
    """
    if N < 3 or N % 2 == 0 or N >= 1 << w:
        raise ValueError("need an odd N with 3 <= N < 2^w")
    R, R2 = 1 << w, 1 << (2 * w)
    ninv = _egcd_inverse(N, R)
    ninv2 = _egcd_inverse(N, R2)
    valid = {"classic"}
    if 2 * N < R:
        valid.add("signed")
    if N * N + N * R < R2:          # N < 2^w / phi
        valid.add("plantard")
    if N < 1 << (w - 1):
        valid.add("signed_plantard")
    return {
        "N": N, "w": w,
        "ninv": ninv,
        "nprime": R - ninv,
        "ninv_mods": mods(ninv, R),
        "ninv2": ninv2,
        "ninv2_mods": mods(ninv2, R2),
        "r_mod_n": R % N,
        "r2_mod_n": R * R % N,
        "rinv_mod_n": _egcd_inverse(R % N, N),
        "r2inv_mod_n": _egcd_inverse(R2 % N, N),
        "valid": valid,
    }


def sigpredc2_steps(T: int, N: int, n: int, alpha: int) -> dict:
    """Algorithm 4 (Section 3.3) evaluated step by step with Python integers.

    R = 2^(2n), N~^{-1} = N^{-1} mods R, m = T N~^{-1} mods R,
    r = floor((floor(m / 2^n) + 2^alpha) N / 2^n).  Returns the intermediate
    values and the true value (mN - T)/R that the algorithm is meant to
    produce.  For alpha = 0 the two can differ (Example 3.1).
    """
    R = 1 << (2 * n)
    ninv_t = mods(_egcd_inverse(N, R), R)
    m = mods(T * ninv_t, R)
    q = (m >> n) + (1 << alpha)           # floor(m / 2^n) + 2^alpha
    r = (q * N) >> n                      # floor(q N / 2^n)
    exact, rem = divmod(m * N - T, R)     # R divides mN - T (Section 3.3)
    assert rem == 0
    return {"R": R, "ninv_mods": ninv_t, "m": m, "r": r, "exact": exact,
            "mN_minus_T_over_2n": (m * N - T) >> n,
            "q_alpha0_times_N": ((m >> n) + 1) * N}


def crt(residues, moduli):
    """The integers X in [0, prod N_j) with X = r_j (mod N_j), from the CRT formula
    X = sum_j r_j M_j (M_j^{-1} mod N_j) mod M, M = prod N_j, M_j = M / N_j
    (for two moduli this is eq. (qin1): T = r1 R^{-1} R + r2 N^{-1} N mod NR).
    residues: k sequences of equal length (Python ints); returns a list."""
    M = 1
    for N in moduli:
        M *= N
    coef = []
    for N in moduli:
        Mj = M // N
        coef.append(Mj * _egcd_inverse(Mj % N, N))
    k = len(moduli)
    n = len(residues[0])
    return [sum(int(residues[j][i]) * coef[j] for j in range(k)) % M for i in range(n)]
