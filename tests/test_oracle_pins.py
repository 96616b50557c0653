"""Pins of the CPU oracle to the paper and to plain mathematics.

None of these checks re-types the oracle's own formula.  They use:
* the worked example the paper prints (Section 3.3, Example 3.1);
* Qin's identity (Section 2, Theorem 2.1) and the defining property of an
  inverse, checked by multiplication;
* brute force over all inputs at tiny word sizes, both as a search for the
  unique residue with the required congruence and range and as the step by
  step evaluation of each algorithm (Section 1 REDC; Algorithms 1-4);
* exhaustive checking of the 16-bit workload (N = 3329, R = 2^16) against
  the congruence r R = T (mod N);
* Python's built-in big-integer pow/inverse on random wide inputs.
"""
import json
import os

import numpy as np
import pytest

import oracle as orc

HERE = os.path.dirname(os.path.abspath(__file__))


def odd_moduli(lo, hi):
    return [N for N in range(max(lo, 3), hi) if N % 2 == 1]


# ----------------------------------------------------------------- example


def test_example_3_1_counterexample():
    ex = json.load(open(os.path.join(HERE, "golden", "example_3_1.json")))
    n, N, alpha, T = ex["n"], ex["N"], ex["alpha"], ex["T"]
    assert 1 << (2 * n) == ex["R"]
    c = orc.constants(N, n)
    assert c["ninv2_mods"] == ex["ninv_mods_R"]
    st = orc.sigpredc2_steps(T, N, n, alpha)
    assert st["ninv_mods"] == ex["ninv_mods_R"]
    assert st["m"] == ex["m"]
    assert st["mN_minus_T_over_2n"] == ex["mN_minus_T_over_2n"] == -15 * 64
    assert st["q_alpha0_times_N"] == ex["floor_m_over_2n_plus_1_times_N"]
    assert st["r"] == ex["algorithm_4_output"]
    lo, hi = ex["required_interval"]
    assert not (lo <= st["r"] <= hi)
    # The correct value -T R~^{-1} mods N is (mN - T)/R = -960/64 = -15; the
    # signed-Plantard oracle (Algorithm 3 has the same target and is proved
    # correct on this input range) must return it.
    assert st["exact"] == -15
    got = int(orc.redc_small("signed_plantard", n, N, [T])[0])
    assert got == -15
    assert (got - st["r"]) % N != 0          # -16 is not even congruent
    assert (got * ex["R"] + T) % N == 0       # r R = -T (mod N)


# --------------------------------------------------------- constants / Qin


@pytest.mark.parametrize("w", [8, 16, 32, 64])
def test_qin_identity_and_constants(w):
    g = np.random.default_rng(11)
    R = 1 << w
    Ns = {3, R - 1 if w < 64 else (1 << 64) - 59}
    Ns |= {int(x) | 1 for x in g.integers(3, min(R, 2**63), size=40, dtype=np.uint64)}
    for N in sorted(Ns):
        if N < 3:
            continue
        c = orc.constants(N, w)
        ninv, rinv = c["ninv"], c["rinv_mod_n"]
        assert (N * ninv) % R == 1 and 1 <= ninv < R
        assert (R * rinv) % N == 1 and 0 < rinv < N
        # Theorem 2.1: R^{-1} R + N^{-1} N = 1 + N R
        assert rinv * R + ninv * N == 1 + N * R
        # its proof: N^{-1} N = 1 + l R with l < N and R^{-1} = N - l
        l_, rem = divmod(ninv * N - 1, R)
        assert rem == 0 and l_ < N and rinv == N - l_
        assert c["nprime"] == R - ninv and (N * c["nprime"]) % R == R - 1
        assert c["ninv"] == pow(N, -1, R)
        assert c["ninv2"] == pow(N, -1, R * R) and (N * c["ninv2"]) % (R * R) == 1
        assert -R // 2 <= c["ninv_mods"] < R // 2 and (c["ninv_mods"] - ninv) % R == 0
        assert c["r2_mod_n"] == pow(2, 2 * w, N)
        assert orc.inv_mod(R % N, N) == rinv


def test_inv_mod_c_against_builtin():
    g = np.random.default_rng(5)
    for _ in range(300):
        N = int(g.integers(3, 2**63, dtype=np.uint64)) * 2 + 1
        a = int(g.integers(1, 2**63, dtype=np.uint64))
        from math import gcd
        want = pow(a, -1, N) if gcd(a, N) == 1 else 0
        assert orc.inv_mod(a, N) == want


# --------------------------------------------------- classic REDC (Section 1)


@pytest.mark.parametrize("w", [4, 6, 8])
def test_classic_brute_force(w):
    R = 1 << w
    for N in odd_moduli(3, R):
        T = np.arange(R * N, dtype=np.int64)
        got = orc.redc_small("classic", w, N, T).astype(np.int64)
        # brute-force search: the unique r in [0, N) with r R = T (mod N)
        table = np.empty(N, np.int64)
        table[(np.arange(N) * R) % N] = np.arange(N)
        assert np.array_equal(got, table[T % N])
        # REDC as printed in Section 1 (m, t, conditional subtract)
        nprime = R - pow(N, -1, R)
        m = ((T % R) * nprime) % R
        t = (T + m * N) // R
        assert np.all((T + m * N) % R == 0) and np.all(t < 2 * N)
        assert np.array_equal(got, np.where(t >= N, t - N, t))


def test_classic_exhaustive_r16_n3329():
    """All T in [0, R N) for N = 3329, R = 2^16 (the 16-bit workload)."""
    N, R = 3329, 1 << 16
    total = R * N
    step = 1 << 24
    for s in range(0, total, step):
        T = np.arange(s, min(s + step, total), dtype=np.uint32)
        r = orc.redc("classic", 16, N, T).astype(np.int64)
        assert r.max() < N
        assert not np.any((r * R - T.astype(np.int64)) % N)
    # sampled comparison with Python integers
    rinv = pow(R, -1, N)
    for T in [0, 1, R - 1, R, R * N - 1, N - 1, N, 12345678, 5 * R]:
        assert int(orc.redc("classic", 16, N, np.array([T], np.uint32))[0]) == T * rinv % N


def test_classic_edge_values_wide():
    for w, N in [(32, 8380417), (32, (1 << 32) - 5), (64, (1 << 62) - 57), (64, (1 << 64) - 59)]:
        R = 1 << w
        rinv = pow(R, -1, N)
        Ts = [0, 1, R - 1, R, R * N - 1, N - 1, N, 7 * R, (N - 1) * R, R * N // 2]
        if w == 32:
            arr = np.array(Ts, dtype=np.uint64)
        else:
            arr = np.array([[t & (2**64 - 1), t >> 64] for t in Ts], dtype=np.uint64)
        got = orc.redc("classic", w, N, arr)
        for t, r in zip(Ts, got):
            assert int(r) == t * rinv % N
        # T = k R reduces to k mod N
        assert int(got[Ts.index(7 * R)]) == 7 % N


# ------------------------------------------------ signed Montgomery (Alg. 1)


@pytest.mark.parametrize("w", [4, 6, 8])
def test_signed_montgomery_brute_force(w):
    R = 1 << w
    for N in odd_moduli(3, R // 2):        # 2N < R
        H = N * R // 2
        T = np.arange(-H + 1, H, dtype=np.int64)      # |T| < N R / 2
        got = orc.redc_small("signed", w, N, T)
        # Algorithm 1 step by step
        ninv = pow(N, -1, R)
        a1 = T >> w
        a0 = T & (R - 1)
        m0 = (a0 * ninv) % R
        m0 = np.where(m0 >= R // 2, m0 - R, m0)        # mods R in [-R/2, R/2)
        t = (m0 * N) >> w                               # floor(m0 N / R)
        assert np.array_equal(got, a1 - t)
        # Ensure line: r = T R^{-1} (mod N), -N < r < N
        assert np.all(np.abs(got) < N)
        assert not np.any((got * R - T) % N)


def test_mods_range_is_section_2s():
    """The least absolute remainder of Section 2 lies in [-n/2, n/2): for even n
    the tie value n/2 is taken as -n/2.  Checked as the congruence and the range
    for every x in a window, not by re-typing the formula."""
    for n in (7, 8, 9, 16, 256, 3329):
        for x in range(-3 * n, 3 * n):
            r = orc.mods(x, n)
            assert (r - x) % n == 0 and -n <= 2 * r < n, (x, n, r)
    assert orc.mods(4, 8) == -4 and orc.mods(128, 256) == -128 and orc.mods(3, 7) == 3 and orc.mods(4, 7) == -3


def test_signed_montgomery_tie_rule():
    """m0 = -R/2 is taken when a0 N^{-1} = R/2 (mods is [-R/2, R/2))."""
    w, N = 8, 101
    R = 1 << w
    ninv = pow(N, -1, R)
    a0 = (R // 2) * pow(ninv, -1, R) % R          # a0 N^{-1} = R/2 (mod R)
    T = 3 * R + a0
    r = int(orc.redc_small("signed", w, N, [T])[0])
    assert r == 3 - ((-(R // 2)) * N >> w)
    assert r != 3 - (((R // 2) * N) >> w)


# ------------------------------------------------------- Plantard (Alg. 2)


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_plantard_brute_force(n):
    R = 1 << (2 * n)
    for N in odd_moduli(3, 1 << n):
        if not N * N + N * (1 << n) < R:           # N < 2^n / phi
            continue
        T = np.arange(0, N * N + 1, dtype=np.int64)   # 0 <= T <= N^2
        got = orc.redc_small("plantard", n, N, T).astype(np.int64)
        ninv = pow(N, -1, R)
        m = (T * ninv) % R
        q = (m >> n) + 1
        assert q.max() < (1 << n)                   # fits an n-bit word
        r = (q * N) >> n
        assert not np.any(r == N)                  # the branch is dead (Remark)
        assert np.array_equal(got, r)
        assert np.all((got >= 0) & (got < N))
        assert not np.any((got * R + T) % N)       # r = -T R^{-1} (mod N)


# ------------------------------------------------ signed Plantard (Alg. 3)


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_signed_plantard_brute_force(n):
    R = 1 << (2 * n)
    B = 1 << (2 * n - 2)
    T = np.arange(-B, B + 1, dtype=np.int64)           # |T| <= 2^(2n-2)
    for N in odd_moduli(3, 1 << (n - 1)):            # N < 2^(n-1)
        got = orc.redc_small("signed_plantard", n, N, T)
        ninv = orc.mods(pow(N, -1, R), R)
        m = (T * ninv) % R
        m = np.where(m >= R // 2, m - R, m)           # mods R
        q = (m + (1 << (n - 1))) >> n                 # round half up
        assert np.all(np.abs(q) < (1 << (n - 1)) + 1)
        r = (q * N + (1 << (n - 1))) >> n
        assert np.array_equal(got, r)
        h = (N - 1) // 2
        assert np.all((got >= -h) & (got <= h))
        assert not np.any((got * R + T) % N)


# ---------------------------------------------- Huang's variant (Alg. 4)


@pytest.mark.parametrize("n", [5, 6, 7])
@pytest.mark.parametrize("alpha", [1, 2])
def test_alg4_alpha_ge_1_brute_force(n, alpha):
    R = 1 << (2 * n)
    for N in odd_moduli(3, 1 << (n - alpha - 1)):
        B = (N * N) << (2 * alpha)
        T = np.arange(-B, B + 1, dtype=np.int64)
        got = orc.redc_small("signed_plantard_alpha", n, N, T, alpha=alpha)
        ninv = orc.mods(pow(N, -1, R), R)
        m = (T * ninv) % R
        m = np.where(m >= R // 2, m - R, m)
        r = (((m >> n) + (1 << alpha)) * N) >> n
        assert np.array_equal(got, r)


# failures of Algorithm 4 with alpha = 0 over all odd N in [3, 2^(n-1)) and
# all |T| <= N^2: (failures, total, first failing (N, T))
ALG4_ALPHA0 = {5: (91, 1365, (7, -46)), 6: (861, 10925, (9, -73)), 7: (7535, 87389, (13, -167))}


@pytest.mark.parametrize("n", [5, 6, 7])
def test_alg4_alpha0_fails(n):
    R = 1 << (2 * n)
    fails = total = 0
    first = None
    for N in odd_moduli(3, 1 << (n - 1)):
        T = np.arange(-N * N, N * N + 1, dtype=np.int64)
        want = orc.redc_small("signed_plantard", n, N, T)
        ninv = orc.mods(pow(N, -1, R), R)
        m = (T * ninv) % R
        m = np.where(m >= R // 2, m - R, m)
        r = (((m >> n) + 1) * N) >> n
        bad = r != want
        if first is None and bad.any():
            first = (N, int(T[np.argmax(bad)]))
        fails += int(bad.sum())
        total += T.size
    assert (fails, total, first) == ALG4_ALPHA0[n]
    with pytest.raises(orc.OracleDomainError):
        orc.redc_small("signed_plantard_alpha", n, 7, [0], alpha=0)


# ----------------------------------------------------- wide words, samples


@pytest.mark.parametrize("w", [16, 32, 64])
def test_mul_against_python_integers(w):
    g = np.random.default_rng(w)
    R = 1 << w
    R2 = R * R
    n = 500
    for N in [int(g.integers(3, R // 4)) | 1 for _ in range(3)] + [R // 2 - 1 if w < 64 else (1 << 62) - 57]:
        N = N | 1
        dt = {16: np.uint16, 32: np.uint32, 64: np.uint64}[w]
        sdt = {16: np.int16, 32: np.int32, 64: np.int64}[w]
        a = g.integers(0, N, size=n, dtype=np.uint64).astype(dt)
        b = g.integers(0, N, size=n, dtype=np.uint64).astype(dt)
        got = orc.mul("classic", w, N, a, b)
        ri = pow(R, -1, N)
        assert [int(x) for x in got] == [int(x) * int(y) * ri % N for x, y in zip(a, b)]
        if N * N + N * R < R2:
            got = orc.mul("plantard", w, N, a, b)
            r2i = pow(R2, -1, N)
            assert [int(x) for x in got] == [(-int(x) * int(y) * r2i) % N for x, y in zip(a, b)]
        h = (N - 1) // 2
        sa = (g.integers(0, N, size=n, dtype=np.uint64).astype(np.int64) - h).astype(sdt)
        sb = (g.integers(0, N, size=n, dtype=np.uint64).astype(np.int64) - h).astype(sdt)
        got = orc.mul("signed", w, N, sa, sb)
        for x, y, r in zip(sa, sb, got):
            T = int(x) * int(y)
            r = int(r)
            assert (r * R - T) % N == 0 and abs(r) < N
            assert T / R - N / 2 < r <= T / R + N / 2
        got = orc.mul("signed_plantard", w, N, sa, sb)
        r2i = pow(R2, -1, N)
        assert [int(r) for r in got] == [orc.mods(-int(x) * int(y) * r2i, N) for x, y in zip(sa, sb)]


@pytest.mark.parametrize("w", [16, 32, 64])
def test_pow_against_builtin(w):
    g = np.random.default_rng(100 + w)
    R = 1 << w
    dt = {16: np.uint16, 32: np.uint32, 64: np.uint64}[w]
    for N in [3, R - 1 if w < 64 else (1 << 64) - 59, int(g.integers(3, min(R, 2**63))) | 1]:
        x = g.integers(0, N, size=300, dtype=np.uint64).astype(dt)
        e = g.integers(0, 2**64 - 1, size=300, dtype=np.uint64, endpoint=True)
        e[:4] = [0, 1, 2, 2**64 - 1]
        x[0] = 0
        got = orc.pow(w, N, x, e)
        assert [int(v) for v in got] == [pow(int(a), int(k), N) for a, k in zip(x, e)]
        assert int(got[0]) == 1                      # 0^0 = 1


def test_pow_fermat():
    for N, w in [(8380417, 32), (3329, 16), ((1 << 61) - 1, 64)]:
        x = np.arange(1, 200, dtype={16: np.uint16, 32: np.uint32, 64: np.uint64}[w])
        e = np.full(x.shape, N - 1, np.uint64)
        assert np.all(orc.pow(w, N, x, e) == 1)


# ------------------------------------------------------- domain rejection


def test_domain_rejections():
    with pytest.raises(orc.OracleDomainError):
        orc.redc_small("classic", 8, 101, [256 * 101])          # T = R N
    with pytest.raises(orc.OracleDomainError):
        orc.redc_small("signed", 8, 101, [101 * 128])           # |T| = N R / 2
    with pytest.raises(orc.OracleDomainError):
        orc.redc_small("signed", 8, 129, [0])                   # 2N >= R
    with pytest.raises(orc.OracleDomainError):
        orc.redc_small("plantard", 6, 31, [31 * 31 + 1])         # T > N^2
    with pytest.raises(orc.OracleDomainError):
        orc.redc_small("plantard", 6, 41, [0])                  # N >= 2^n / phi
    with pytest.raises(orc.OracleDomainError):
        orc.redc_small("signed_plantard", 6, 31, [(1 << 10) + 1])  # |T| > 2^(2n-2)
    # inclusive Require bounds are accepted
    orc.redc_small("plantard", 6, 39, [39 * 39])
    orc.redc_small("signed_plantard", 6, 31, [-(1 << 10), 1 << 10])
    with pytest.raises(ValueError):
        orc.redc_small("classic", 8, 100, [0])                  # even N


# --------------------------------------------------------------- CRT


def test_crt_two_moduli_is_qin_form():
    """For moduli (N, R), the oracle's CRT is eq. (qin1)'s T = r1 R^{-1} R + r2 N^{-1} N (mod NR)."""
    g = np.random.default_rng(21)
    for w in (8, 16, 32):
        R = 1 << w
        for N in [3, 101, R - 1] + [int(x) | 1 for x in g.integers(3, R, size=5)]:
            c = orc.constants(N, w)
            r1 = [int(x) for x in g.integers(0, N, size=50)]
            r2 = [int(x) for x in g.integers(0, R, size=50)]
            got = orc.crt([r1, r2], [N, R])
            want = [(a * c["rinv_mod_n"] * R + b * c["ninv"] * N) % (N * R) for a, b in zip(r1, r2)]
            assert got == want


def test_crt_brute_force_and_properties():
    # tiny pairwise coprime moduli: search every X in [0, M)
    mods = [3, 5, 7, 11]
    M = 3 * 5 * 7 * 11
    table = {tuple(X % m for m in mods): X for X in range(M)}
    g = np.random.default_rng(22)
    res = [[int(x) for x in g.integers(0, m, size=200)] for m in mods]
    got = orc.crt(res, mods)
    assert got == [table[tuple(r[i] for r in res)] for i in range(200)]
    # wide moduli: the defining congruences and range
    mods = [(1 << 61) - 1, (1 << 62) - 57, 1000000007, 998244353, (1 << 64) - 59]
    res = [[int(x) % m for x in g.integers(0, 2**63, size=100, dtype=np.uint64)] for m in mods]
    P = 1
    for m in mods:
        P *= m
    for i, X in enumerate(orc.crt(res, mods)):
        assert 0 <= X < P and all(X % m == r[i] for m, r in zip(mods, res))


# --------------------------------------------------------------- DFT


def _root(N, n):
    for g in range(2, 10000):
        w = pow(g, (N - 1) // n, N)
        if pow(w, n // 2, N) == N - 1:
            return w
    raise ValueError("no root")


def test_dft_closed_forms_and_inverse():
    for N, log2n in [(17, 4), (12289, 6), (8380417, 8), ((1 << 64) - (1 << 32) + 1, 5)]:
        n = 1 << log2n
        w = _root(N, n)
        delta = np.zeros(n, np.uint64)
        delta[1] = 1                                   # x = X^1  ->  X_k = w^k
        assert [int(v) for v in orc.dft(64, N, delta, w)] == [pow(w, k, N) for k in range(n)]
        ones = np.ones(n, np.uint64)                   # sum_j w^(jk) = n [k = 0]
        assert [int(v) for v in orc.dft(64, N, ones, w)] == [n % N] + [0] * (n - 1)
        g = np.random.default_rng(log2n)
        x = g.integers(0, N, size=n, dtype=np.uint64)
        X = orc.dft(64, N, x, w)
        assert np.array_equal(orc.dft(64, N, X, w, inverse=True), x)


def test_dft_convolution_theorem():
    """DFT(a) . DFT(b) = DFT(a * b) for the cyclic convolution (brute force)."""
    N, n = 12289, 32
    w = _root(N, n)
    g = np.random.default_rng(3)
    a = [int(v) for v in g.integers(0, N, size=n)]
    b = [int(v) for v in g.integers(0, N, size=n)]
    conv = [sum(a[j] * b[(k - j) % n] for j in range(n)) % N for k in range(n)]
    A = orc.dft(32, N, np.array(a, np.uint32), w)
    B = orc.dft(32, N, np.array(b, np.uint32), w)
    C = orc.dft(32, N, np.array(conv, np.uint32), w)
    assert [int(x) * int(y) % N for x, y in zip(A, B)] == [int(c) for c in C]


# ------------------------------------------- algorithms step by step, wide words


def _steps(variant, w, N, T, alpha=1):
    """Each algorithm's steps with Python integers (Section 1 REDC, Algorithms 1-4)."""
    if variant == "classic":
        R = 1 << w
        m = (T % R) * (R - pow(N, -1, R)) % R
        t = (T + m * N) // R
        return t - N if t >= N else t
    if variant == "signed":
        R = 1 << w
        a1, a0 = T >> w, T & (R - 1)
        m0 = orc.mods(a0 * pow(N, -1, R), R)
        return a1 - ((m0 * N) >> w)
    R = 1 << (2 * w)
    if variant == "plantard":
        m = T * pow(N, -1, R) % R
        r = (((m >> w) + 1) * N) >> w
        return 0 if r == N else r
    m = orc.mods(T * orc.mods(pow(N, -1, R), R), R)
    if variant == "signed_plantard":
        q = (m + (1 << (w - 1))) >> w                  # round half up
        return (q * N + (1 << (w - 1))) >> w
    return (((m >> w) + (1 << alpha)) * N) >> w        # Algorithm 4


@pytest.mark.parametrize("w", [16, 32, 64])
def test_algorithm_steps_match_oracle_wide(w):
    import random
    rnd = random.Random(w)
    for _ in range(40):
        top = rnd.choice([w - 3, w - 1, w])
        N = rnd.randrange(3, 1 << top) | 1
        for variant in ["classic", "signed", "plantard", "signed_plantard", "signed_plantard_alpha"]:
            c = orc.constants(N, w)
            if variant == "signed_plantard_alpha":
                if not N < 1 << (w - 2):
                    continue
            elif variant not in c["valid"]:
                continue
            R = 1 << w
            lo, hi = {"classic": (0, R * N - 1), "signed": (-(N * R // 2) + 1, N * R // 2 - 1),
                      "plantard": (0, N * N), "signed_plantard": (-(1 << (2 * w - 2)), 1 << (2 * w - 2)),
                      "signed_plantard_alpha": (-4 * N * N, 4 * N * N)}[variant]
            Ts = [lo, hi, 0] + [rnd.randint(lo, hi) for _ in range(60)]
            if w < 64:
                dt = {16: np.int32, 32: np.int64}[w] if variant.startswith("signed") else \
                     {16: np.uint32, 32: np.uint64}[w]
                arr = np.array(Ts, dtype=dt)
            else:
                arr = np.array([[t & (2**64 - 1), (t >> 64) & (2**64 - 1)] for t in Ts], dtype=np.uint64)
            got = orc.redc(variant, w, N, arr, alpha=1)
            want = [_steps(variant, w, N, T) for T in Ts]
            assert [int(x) for x in got] == want, (variant, w, N)
