"""Bit-exact parity of the HIP library against the CPU oracle (needs a GPU).

Every case runs the library through its C ABI on seeded inputs and compares
each output element with the oracle.  Sizes span many 16-byte chunks and
workgroups and end in a ragged tail; edge values of each variant's input
range are always included.
"""
import concurrent.futures as cf
import os
import random

import numpy as np
import pytest

import oracle as orc
import paper_2402_00675_amd as mg
from paper_2402_00675_amd import inputs as inp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIGNED = {"signed", "signed_plantard", "signed_plantard_alpha"}
ALL_VARIANTS = ["classic", "signed", "plantard", "signed_plantard", "signed_plantard_alpha"]
MODULI = {
    16: [3, 5, 3329, 7681, 12289, 32767, 40503, 65521, 65535],
    32: [3, 8380417, (1 << 30) + 3, 2147483647, 2654435761, 4294967291],
    64: [3, (1 << 61) - 1, (1 << 62) - 57, (1 << 63) - 25, (1 << 64) - 59],
}
NP_E = {16: (np.uint16, np.int16), 32: (np.uint32, np.int32), 64: (np.uint64, np.int64)}
WORKERS = min(8, len(os.sched_getaffinity(0)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def sync():
    torch.cuda.synchronize()


def elem_np(variant, w):
    return NP_E[w][1] if variant in SIGNED else NP_E[w][0]


def operands(variant, w, N, n, g):
    """Two operand vectors whose product meets the variant's input range."""
    dt = elem_np(variant, w)
    if variant in SIGNED:
        h = (N - 1) // 2
        # signed variants need N < 2^(w-1), so N - 1 fits in int64 for every w
        a = g.integers(0, N, size=n, dtype=np.uint64).astype(np.int64) - h
        b = g.integers(0, N, size=n, dtype=np.uint64).astype(np.int64) - h
        edges = [0, 1, -1, h, -h, h - 1]
    else:
        a = g.integers(0, N, size=n, dtype=np.uint64)
        b = g.integers(0, N, size=n, dtype=np.uint64)
        edges = [0, 1, N - 1, N // 2, N - 2]
    k = min(len(edges), n)
    a[:k] = edges[:k]
    b[:k] = edges[::-1][:k]
    if n > 2 * k:
        a[-k:] = edges[:k]
        b[-k:] = edges[:k]
    return a.astype(dt), b.astype(dt)


def t_bounds(variant, w, N, alpha=1):
    """Inclusive [lo, hi] of T for the variant (Require lines of Algorithms 1-4)."""
    R = 1 << w
    if variant == "classic":
        return 0, R * N - 1
    if variant == "signed":
        return -(N * R // 2) + 1, N * R // 2 - (1 if (N * R) % 2 == 0 else 0)
    if variant == "plantard":
        return 0, N * N
    if variant == "signed_plantard":
        B = 1 << (2 * w - 2)
        return -B, B
    B = (N * N) << (2 * alpha)
    return -B, B


def t_values(variant, w, N, n, seed, alpha=1):
    lo, hi = t_bounds(variant, w, N, alpha)
    if variant == "signed":
        hi = min(hi, N * (1 << w) // 2 - 1)
    rnd = random.Random(seed)
    vals = [lo, hi, 0, 1, min(hi, 1 << w), min(hi, (1 << w) - 1), min(hi, N), min(hi, N - 1),
            max(lo, -1), max(lo, -(1 << w)), min(hi, (1 << (w - 1))), min(hi, 3 << (w - 1))]
    vals = [v for v in vals if lo <= v <= hi][:n]
    vals += [rnd.randint(lo, hi) for _ in range(n - len(vals))]
    return vals


def pack_T(vals, variant, w):
    if w < 64:
        dt = {16: np.int32, 32: np.int64}[w] if variant in SIGNED else {16: np.uint32, 32: np.uint64}[w]
        return np.array(vals, dtype=dt)
    m = (1 << 64) - 1
    return np.array([[v & m, (v >> 64) & m] for v in vals], dtype=np.uint64)


def valid_cases():
    for w, Ns in MODULI.items():
        for N in Ns:
            c = mg.setup(N, w)
            for v in ALL_VARIANTS:
                if c.valid(v):
                    yield w, N, v


CASES = list(valid_cases())


@pytest.mark.parametrize("w,N,variant", CASES, ids=["w%d-N%d-%s" % c for c in CASES])
def test_mul_parity(w, N, variant):
    g = inp.rng(99, w * 7 + N % 1000)
    n = 100_003 if w < 64 else 40_009
    a, b = operands(variant, w, N, n, g)
    c = mg.setup(N, w)
    got = host(mg.mul(c, dev(a), dev(b), variant=variant))
    want = orc.mul(variant, w, N, a, b, alpha=c.s.alpha)
    assert got.dtype == want.dtype
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "first mismatch at %d: a=%d b=%d got %d want %d" % (
        bad[0], a[bad[0]], b[bad[0]], got[bad[0]], want[bad[0]])


@pytest.mark.parametrize("w,N,variant", CASES, ids=["w%d-N%d-%s" % c for c in CASES])
def test_redc_parity(w, N, variant):
    n = 30_011 if w < 64 else 8_009
    c = mg.setup(N, w)
    vals = t_values(variant, w, N, n, seed=w * 1000 + N % 997, alpha=c.s.alpha)
    T = pack_T(vals, variant, w)
    got = host(mg.redc(c, dev(T), n=n, variant=variant))
    want = orc.redc(variant, w, N, T, alpha=c.s.alpha)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "first mismatch at %d: T=%d got %d want %d" % (bad[0], vals[bad[0]], got[bad[0]],
                                                                           want[bad[0]])


def edge_T(variant, w, N, seed, alpha=1):
    """T values at the corners of each algorithm's intermediate quantities, from closed forms.

    Classic and signed (R = 2^w, T = a1 R + a0): low words a0 = 0, 1, R/2, R - 1 (for Algorithm 1
    a0 = R/2 gives the mods tie m0 = a0 N^{-1} mods R = -R/2, since (R/2) N = R/2 mod R), high words
    at both ends of the range, T = N j (t = (T + mN)/R is exactly N before the correction: m = R - j),
    and the largest |T|.  Plantard family (R = 2^(2n), m = T N^{-1} mod R or mods R, q = floor(m/2^n)):
    T = N j (m = j), the largest reachable q for T <= N^2 (T = 2^(2n) - N D with
    D = ceil((2^(2n) - N^2)/N): q = 2^n - ceil(D/2^n), which reaches 2^n - 2 for N close to 2^n/phi
    and never 2^n - 1, the dead branch of Algorithm 2's remark), low halves of m at 0, 2^(n-1)
    (the round-half-up tie of Algorithm 3's first rounding) and 2^n - 1, q at both ends of its
    signed range (Algorithms 3 and 4), and the largest |T|.  Values outside the Require range
    are dropped.
    """
    rnd = random.Random(seed)
    lo, hi = t_bounds(variant, w, N, alpha)
    out = []

    def add(t):
        if lo <= t <= hi and (variant != "signed" or abs(t) < N * (1 << w) // 2):
            out.append(t)

    if variant in ("classic", "signed"):
        R = 1 << w
        h = (N - 1) // 2
        a1s = [0, 1, 2, N - 1, N - 2, h, h - 1] if variant == "classic" else [0, 1, -1, h - 1, h - 2, -h, -h - 1]
        a1s += [rnd.randint(-h if variant == "signed" else 0, N - 1 if variant == "classic" else h - 1)
                for _ in range(8)]
        for a1 in a1s:
            for a0 in (0, 1, R // 2, R // 2 - 1, R // 2 + 1, R - 1):
                add(a1 * R + a0)
        for j in [1, 2, R - 1, R - 2, R // 2] + [rnd.randrange(1, R) for _ in range(8)]:
            add(N * j)
            add(-N * j)
        add(hi)
        add(lo)
        return out
    n = w
    R2 = 1 << (2 * n)
    sgn = variant != "plantard"

    def from_m(m):
        t = (m % R2) * N % R2
        if sgn and t >= R2 // 2:
            t -= R2
        return t

    for j in [0, 1, 2, 3, N - 1, N] + [rnd.randrange(N) for _ in range(6)]:
        add(N * j)
        add(-N * j)
    if not sgn:
        D = -(-(R2 - N * N) // N)
        for k in range(8):
            add(R2 - N * (D + k))
        add(N * N)
        add(N * N - 1)
    qs = ([(1 << n) - 1, (1 << n) - 2, 0, 1] if not sgn else
          [(1 << (n - 1)) - 1, (1 << (n - 1)) - 2, -(1 << (n - 1)), -(1 << (n - 1)) + 1, 0, -1])
    for l in (0, 1 << (n - 1), (1 << n) - 1):
        for _ in range(300):
            q = rnd.randrange(1 << n) if not sgn else rnd.randrange(-(1 << (n - 1)), 1 << (n - 1))
            add(from_m(q * (1 << n) + l))
    for q in qs:
        for _ in range(300):
            add(from_m(q * (1 << n) + rnd.randrange(1 << n)))
    add(hi)
    add(lo)
    return out


# the largest odd moduli below 2^w / phi (Algorithm 2's bound): the quotient q reaches 2^n - 2
PHI_EDGE = [(32, 2654435769, "plantard"), (64, 11400714819323198485, "plantard")]
EDGE_CASES = [c for c in CASES if c[0] > 16] + PHI_EDGE


@pytest.mark.parametrize("w,N,variant", EDGE_CASES, ids=["w%d-N%d-%s" % c for c in EDGE_CASES])
def test_redc_edge_vectors(w, N, variant):
    """The closed-form edge values of edge_T at 32 and 64 bits, element by element."""
    c = mg.setup(N, w)
    assert c.valid(variant)
    vals = edge_T(variant, w, N, seed=w + N % 991, alpha=c.s.alpha)
    assert len(vals) > 15
    T = pack_T(vals, variant, w)
    got = host(mg.redc(c, dev(T), n=len(vals), variant=variant))
    want = orc.redc(variant, w, N, T, alpha=c.s.alpha)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "first mismatch at %d: T=%d got %d want %d" % (bad[0], vals[bad[0]], got[bad[0]],
                                                                           want[bad[0]])


@pytest.mark.parametrize("w,N,variant", CASES, ids=["w%d-N%d-%s" % c for c in CASES])
def test_mul_const_parity(w, N, variant):
    """Fixed-operand product equals the product with b broadcast, for edge and random b."""
    g = inp.rng(95, w * 7 + N % 1000)
    n = 30_011
    a, bs = operands(variant, w, N, n, g)
    c = mg.setup(N, w)
    da = dev(a)
    h = (N - 1) // 2
    picks = [int(bs[7]), int(bs[n // 2])] + ([0, 1, -1, h, -h] if variant in SIGNED else [0, 1, N - 1, N // 2])
    for b in picks:
        got = host(mg.mul_const(c, da, b, variant=variant))
        want = orc.mul(variant, w, N, a, np.full(n, b, dtype=a.dtype), alpha=c.s.alpha)
        assert np.array_equal(got, want), (b, np.nonzero(got != want)[0][:5])
    with pytest.raises(mg.MontError) as e:
        mg.mul_const(c, da, N if variant not in SIGNED else -N, variant=variant)
    assert e.value.code == -2


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 9, 15, 16, 17, 255, 256, 257, 1023, 4097])
@pytest.mark.parametrize("w", [16, 32, 64])
def test_small_and_misaligned(w, n):
    """Tails shorter than a chunk, and element-aligned but not 16-byte aligned pointers."""
    N = {16: 3329, 32: 8380417, 64: (1 << 62) - 57}[w]
    c = mg.setup(N, w)
    g = inp.rng(98, n + w)
    for variant in ["classic", "signed", "plantard", "signed_plantard"]:
        a, b = operands(variant, w, N, n + 1, g)
        da, db = dev(a), dev(b)
        want = orc.mul(variant, w, N, a[1:], b[1:])
        out = torch.empty(n + 1, dtype=da.dtype, device="cuda")
        mg.mul(c, da[1:], db[1:], out=out[1:], variant=variant)       # head + 16-byte body
        assert np.array_equal(host(out)[1:], want)
        got = host(mg.mul(c, da[1:].clone(), db[1:].clone(), variant=variant))  # aligned path
        assert np.array_equal(got, want)
        out2 = torch.zeros(n + 2, dtype=da.dtype, device="cuda")
        mg.mul(c, da[1:], db[1:], out=out2[2:], variant=variant)      # offsets differ: element-wise path
        assert np.array_equal(host(out2)[2:], want)


def _offset_views(x, k, n):
    """n elements of a fresh device copy of x, starting k elements past a 16-byte aligned address."""
    buf = torch.zeros(n + k + 8, dtype=x.dtype, device="cuda")
    assert buf.data_ptr() % 16 == 0
    buf[k:k + n] = x[:n]
    return buf, buf[k:k + n]


@pytest.mark.parametrize("w", [16, 32, 64])
def test_equal_offset_heads(w):
    """Pointers at one offset k within a 16-byte chunk (a head of 16/size - k elements, then the
    16-byte body), for every k, products, fixed-operand products, reductions, RNS rows and
    in-place calls; lengths shorter than the head, equal to it and spanning many chunks."""
    N = {16: 3329, 32: 8380417, 64: (1 << 62) - 57}[w]
    c = mg.setup(N, w)
    E = 128 // w
    g = inp.rng(99, w)
    for variant in ["classic", "signed_plantard"]:
        for k in range(E):
            for n in sorted({1, E - k, E - k + 1, 3 * E + 1, 100_003}):
                a, b = operands(variant, w, N, n, g)
                want = orc.mul(variant, w, N, a, b)
                ba, va = _offset_views(dev(a), k, n)
                bb, vb = _offset_views(dev(b), k, n)
                bo, vo = _offset_views(torch.zeros(n, dtype=va.dtype, device="cuda"), k, n)
                mg.mul(c, va, vb, out=vo, variant=variant)
                assert np.array_equal(host(vo), want), (variant, k, n)
                assert not host(bo)[:k].any() and not host(bo)[k + n:].any()   # nothing outside
                # b one 16-byte chunk further: the body can reach 16-byte but not 128-byte alignment
                _, vb16 = _offset_views(dev(b), k + E, n)
                vo.zero_()
                mg.mul(c, va, vb16, out=vo, variant=variant)
                assert np.array_equal(host(vo), want), ("16-byte head", variant, k, n)
                kb = int(b[0])
                mg.mul_const(c, va, kb, out=vo, variant=variant)
                assert np.array_equal(host(vo), orc.mul(variant, w, N, a, np.full(n, kb, dtype=a.dtype))), (k, n)
                mg.mul(c, va, vb, out=va, variant=variant)                      # in place
                assert np.array_equal(host(va), want), ("in place", variant, k, n)
                vals = t_values(variant, w, N, n, seed=k + n)
                T = pack_T(vals, variant, w)
                T2 = T.reshape(n, -1)        # one row per T (two words at w = 64)
                tbuf = torch.zeros((n + k + 8) * T2.shape[1], dtype=dev(T2).dtype, device="cuda").view(n + k + 8, -1)
                tbuf[k:k + n] = dev(T2)
                mg.redc(c, tbuf[k:k + n], n=n, out=vo, variant=variant)
                assert np.array_equal(host(vo), orc.redc(variant, w, N, T)), ("redc", variant, k, n)


@pytest.mark.parametrize("pad", [0, 2])
def test_rns_rows_at_an_offset(pad):
    """RNS rows whose first element sits one word past a 16-byte boundary: a row stride that is a
    multiple of 128 bytes (every row's body starts on a line) and one that is a multiple of 16
    bytes only (bodies start on 16-byte chunks)."""
    wl = inp.RNS64Workload(n=20_000)
    a0, b0 = wl.operands(n=wl.n)
    k = a0.shape[0]
    ld = wl.n + pad
    a = np.zeros((k, ld), np.uint64)
    b = np.zeros((k, ld), np.uint64)
    a[:, :wl.n] = a0
    b[:, :wl.n] = b0
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    flat = {}
    for name, x in (("a", a), ("b", b), ("o", np.zeros_like(a))):
        buf = torch.zeros(k * ld + 2, dtype=torch.uint64, device="cuda")
        buf[1:1 + k * ld] = dev(x.reshape(-1))
        flat[name] = buf[1:1 + k * ld].view(k, ld)
    n = wl.n - 3
    mg.mul_rns(ctxs, flat["a"], flat["b"], out=flat["o"], n=n)
    got = host(flat["o"])
    for i, N in enumerate(wl.moduli):
        assert np.array_equal(got[i, :n], orc.mul("classic", 64, N, a[i, :n], b[i, :n])), i
        assert not got[i, n:].any()


LAUNCHES = [(u, nt, bpc, bs) for u in (1, 2, 4) for nt in (0, 1) for bpc in (0, 4) for bs in (64, 256)]


@pytest.mark.parametrize("u,nt,bpc,bs", LAUNCHES)
def test_launch_shapes(u, nt, bpc, bs):
    """Every unroll / non-temporal / grid shape gives the same results."""
    saved = {(op, w, v): mg.get_launch(op, w, v) for op in (mg.OP_MUL, mg.OP_REDC) for w in (16, 32, 64)
             for v in ["classic", "signed_plantard"]}
    try:
        for w, N in [(16, 3329), (32, 8380417), (64, (1 << 60) - 93)]:
            c = mg.setup(N, w)
            for variant in ["classic", "signed_plantard"]:
                mg.set_launch(mg.OP_MUL, w, variant, u, nt, bpc, bs)
                mg.set_launch(mg.OP_REDC, w, variant, u, nt, bpc, bs)
                a, b = operands(variant, w, N, 300_007, inp.rng(97, u * 10 + nt + bpc))
                got = host(mg.mul(c, dev(a), dev(b), variant=variant))
                assert np.array_equal(got, orc.mul(variant, w, N, a, b))
                vals = t_values(variant, w, N, 5000, seed=u + 7 * nt + bpc)
                T = pack_T(vals, variant, w)
                assert np.array_equal(host(mg.redc(c, dev(T), n=5000, variant=variant)),
                                      orc.redc(variant, w, N, T))
    finally:
        for (op, w, variant), L in saved.items():
            mg.set_launch(op, w, variant, **L)


def test_alg4_alpha_values():
    """Algorithm 4 with alpha = 1..4 at w = 16/32 (inputs up to 2^(2 alpha) N^2)."""
    for w, N in [(16, 331), (16, 1001), (32, 8380417), (32, 100003)]:
        for alpha in range(1, 5):
            c = mg.setup(N, w)
            if N >= 1 << (w - alpha - 1):
                continue
            c.set_alpha(alpha)
            vals = t_values("signed_plantard_alpha", w, N, 20_000, seed=alpha, alpha=alpha)
            T = pack_T(vals, "signed_plantard_alpha", w)
            got = host(mg.redc(c, dev(T), n=len(vals), variant="signed_plantard_alpha"))
            assert np.array_equal(got, orc.redc("signed_plantard_alpha", w, N, T, alpha=alpha))


# --------------------------------------------------------------- exhaustive


def _oracle_chunks(fn, starts, size):
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        return list(ex.map(lambda s: fn(s, size), starts))


def test_exhaustive_classic_r16_n3329():
    """All 218,169,344 T in [0, R N) for N = 3329, R = 2^16."""
    N, R = 3329, 1 << 16
    c = mg.setup(N, 16)
    total = R * N
    out = host(mg.redc_range(c, 0, total))
    step = 1 << 24

    def chk(s, size):
        e = min(s + size, total)
        want = orc.redc("classic", 16, N, np.arange(s, e, dtype=np.uint32))
        return int(np.count_nonzero(out[s:e] != want))

    assert sum(_oracle_chunks(chk, range(0, total, step), step)) == 0


def test_exhaustive_plantard_r16_n3329():
    """All T in [0, N^2] for Plantard with n = 16 (R = 2^32)."""
    N = 3329
    c = mg.setup(N, 16)
    total = N * N + 1
    out = host(mg.redc_range(c, 0, total, variant="plantard"))
    want = orc.redc("plantard", 16, N, np.arange(0, total, dtype=np.uint32))
    assert np.array_equal(out, want)


def _exhaustive_signed(variant, lo, hi, step=1 << 26, alpha=1):
    N = 3329
    c = mg.setup(N, 16)
    if variant == "signed_plantard_alpha":
        c.set_alpha(alpha)
    bad = 0
    for s in range(lo, hi + 1, step):
        e = min(s + step, hi + 1)
        T = torch.arange(s, e, dtype=torch.int32, device="cuda")
        got = host(mg.redc(c, T, variant=variant))
        del T

        def chk(s2, size, got=got, s=s, e=e):
            e2 = min(s2 + size, e)
            want = orc.redc(variant, 16, N, np.arange(s2, e2, dtype=np.int32), alpha=alpha)
            return int(np.count_nonzero(got[s2 - s:e2 - s] != want))

        bad += sum(_oracle_chunks(chk, range(s, e, 1 << 22), 1 << 22))
    return bad


def test_exhaustive_signed_r16_n3329():
    """Algorithm 1 over every |T| < N R / 2 (R = 2^16)."""
    H = 3329 * (1 << 15)
    assert _exhaustive_signed("signed", -H + 1, H - 1) == 0


def test_exhaustive_signed_plantard_r16_n3329():
    """Algorithm 3 over every |T| <= 2^30 (n = 16)."""
    B = 1 << 30
    assert _exhaustive_signed("signed_plantard", -B, B, step=1 << 27) == 0


def test_exhaustive_alg4_r16_n3329():
    """Algorithm 4 (alpha = 1, 2) over every |T| <= 2^(2 alpha) N^2."""
    for alpha in (1, 2):
        B = (3329 * 3329) << (2 * alpha)
        assert _exhaustive_signed("signed_plantard_alpha", -B, B, alpha=alpha) == 0


def test_range_top_of_classic_w32():
    N = 8380417
    c = mg.setup(N, 32)
    n = 1_000_003
    T0 = N * (1 << 32) - n
    got = host(mg.redc_range(c, T0, n))
    want = orc.redc("classic", 32, N, np.arange(T0, T0 + n, dtype=np.uint64))
    assert np.array_equal(got, want)


# -------------------------------------------------------------------- pow


@pytest.mark.parametrize("w", [16, 32, 64])
def test_pow_parity(w):
    dt = NP_E[w][0]
    g = inp.rng(96, w)
    # both sides of the smaller-modulus ladder forms: signed products for N < 2^31 (w = 32), lazy ones
    # for N < 2^62 (w = 64)
    Ns = {16: [3, 3329, 65521, 65535],
          32: [3, 8380417, (1 << 30) - 35, (1 << 30) + 3, (1 << 31) - 1, (1 << 31) + 1, 4294967291],
          64: [3, (1 << 61) - 1, (1 << 62) - 57, (1 << 62) - 1, (1 << 62) + 1, (1 << 64) - 59]}[w]
    for N in Ns:
        n = 20_011
        x = g.integers(0, N, size=n, dtype=np.uint64).astype(dt)
        e = inp.u64_uniform(g, n)
        x[:6] = [0, 0, 1, N - 1, N - 1, 2 % N]
        e[:6] = [0, 5, 2**64 - 1, 1, 2, 2**64 - 1]
        e[6:10] = [0, 1, 2, 3]
        c = mg.setup(N, w)
        got = host(mg.pow(c, dev(x), dev(e)))
        want = orc.pow(w, N, x, e)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (N, bad[:5], x[bad[:5]], e[bad[:5]])


@pytest.mark.parametrize("unroll", [1, 2, 4])
def test_pow_launch_shapes(unroll):
    """Every lockstep width of the ladder (elements per lane) gives the same results."""
    g = inp.rng(96, 100 + unroll)
    for w, N in ((32, 8380417), (32, (1 << 31) - 1), (32, 4294967291), (64, (1 << 62) - 57), (64, (1 << 64) - 59)):
        saved = mg.get_launch(mg.OP_POW, w, "classic")
        try:
            mg.set_launch(mg.OP_POW, w, "classic", unroll=unroll)
            n = 5003
            x = g.integers(0, N, size=n, dtype=np.uint64).astype(NP_E[w][0])
            e = inp.u64_uniform(g, n)
            got = host(mg.pow(mg.setup(N, w), dev(x), dev(e)))
            assert np.array_equal(got, orc.pow(w, N, x, e)), (w, N, unroll)
        finally:
            mg.set_launch(mg.OP_POW, w, "classic", **saved)


# -------------------------------------------------------------------- RNS


@pytest.mark.parametrize("ld_extra", [0, 5])
def test_rns_parity(ld_extra):
    wl = inp.RNS64Workload(n=100_003)
    n = wl.n
    ld = 100_008 + ld_extra
    a0, b0 = wl.operands(n=n)
    a = np.zeros((wl.k, ld), np.uint64)
    b = np.zeros((wl.k, ld), np.uint64)
    a[:, :n] = a0
    b[:, :n] = b0
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    out = torch.zeros((wl.k, ld), dtype=torch.uint64, device="cuda")
    mg.mul_rns(ctxs, dev(a), dev(b), out=out, n=n)
    got = host(out)
    for i, N in enumerate(wl.moduli):
        assert np.array_equal(got[i, :n], orc.mul("classic", 64, N, a0[i], b0[i])), i
        assert not got[i, n:].any()  # untouched padding


# ----------------------------------------------------------------- ragged


def ragged_case(seed, nseg, maxlen, ops, widths=(16, 32, 64)):
    """Segments with random width, op, variant and length, packed into pools."""
    g = np.random.default_rng(seed)
    ctxs, segs, meta = [], [], []
    cur0 = {16: 0, 32: 0, 64: 0}
    cur1 = {16: 0, 32: 0, 64: 0}   # byte cursor in in1
    for i in range(nseg):
        w = int(g.choice(widths))
        N = int(g.integers(3, 1 << (w - 3), dtype=np.uint64)) | 1 if g.uniform() < 0.8 else \
            int(g.integers(1 << (w - 1), (1 << w) - 1, dtype=np.uint64)) | 1
        c = mg.setup(N, w)
        op = int(g.choice(ops))
        if op == mg.OP_POW:
            variant = "classic"
        else:
            vs = [v for v in ALL_VARIANTS if c.valid(v)]
            variant = vs[int(g.integers(0, len(vs)))]
        n = int(np.exp(g.uniform(0, np.log(maxlen)))) if g.uniform() < 0.95 else 0
        es = w // 8
        E = 16 // es
        off = cur0[w] + int(g.integers(0, 5))
        cur0[w] = off + n + 3
        if op == mg.OP_MUL:
            # b at a byte offset congruent to off (mod 16)
            b0 = (cur1[w] + 15) // 16 * 16 + (off % E) * es
            off1 = b0 // es
            cur1[w] = b0 + n * es + 8
        elif op == mg.OP_POW:
            b0 = (cur1[w] + 7) // 8 * 8
            off1 = b0 // 8
            cur1[w] = b0 + 8 * n + 8
        else:
            off1 = off
        ctxs.append(c)
        segs.append((i, op, variant, n, off, off1))
        meta.append((w, N, op, variant, n, off, off1))
    return ctxs, segs, meta, cur0, cur1


def ragged_buffers(meta, cur0, cur1, seed):
    g = np.random.default_rng(seed + 1)
    in0 = {w: np.zeros(2 * cur0[w] + 16, dtype=NP_E[w][0]) for w in (16, 32, 64)}   # room for 2w-bit T
    in1 = {w: np.zeros(cur1[w] + 16, dtype=np.uint8) for w in (16, 32, 64)}
    inputs = []
    for (w, N, op, variant, n, off, off1) in meta:
        if op == mg.OP_MUL:
            a, b = operands(variant, w, N, n, g)
            in0[w][off:off + n] = a.view(NP_E[w][0])
            in1[w][off1 * (w // 8):(off1 + n) * (w // 8)] = b.view(np.uint8)
            inputs.append((a, b))
        elif op == mg.OP_POW:
            x = g.integers(0, N, size=n, dtype=np.uint64).astype(NP_E[w][0])
            e = inp.u64_uniform(g, n)
            in0[w][off:off + n] = x
            in1[w][off1 * 8:(off1 + n) * 8] = e.view(np.uint8)
            inputs.append((x, e))
        else:
            T = pack_T(t_values(variant, w, N, n, seed=off, alpha=1), variant, w) if n else \
                pack_T([], variant, w)
            raw = T.view(NP_E[w][0]).reshape(-1)
            k = 2 if w < 64 else 2          # a 2w-bit T spans two w-bit slots
            in0[w][off * k:(off + n) * k] = raw[:n * k]
            inputs.append((T, None))
    return in0, in1, inputs


def check_ragged(meta, inputs, out):
    for (w, N, op, variant, n, off, off1), (x, y) in zip(meta, inputs):
        got = out[w][off:off + n]
        # contexts keep mont_setup's default alpha = 1 for Algorithm 4
        if op == mg.OP_MUL:
            want = orc.mul(variant, w, N, x, y, alpha=1).view(NP_E[w][0])
        elif op == mg.OP_POW:
            want = orc.pow(w, N, x, y)
        else:
            want = orc.redc(variant, w, N, x, alpha=1).view(NP_E[w][0])
        assert np.array_equal(got, want), (w, N, op, variant, n, off)


def run_ragged(meta, segs, ctxs, in0, in1, cur0, flags, reps=1, pervector=False):
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    d1 = {w: dev(in1[w]) for w in (16, 32, 64)}
    do = {w: torch.zeros(cur0[w] + 16, dtype=d0[w].dtype, device="cuda") for w in (16, 32, 64)}
    P = mg.pools([d0[16], d0[32], d0[64]], [d1[16], d1[32], d1[64]], [do[16], do[32], do[64]])
    b = mg.Batch(ctxs, segs, flags=flags)
    outs = []
    for _ in range(reps):
        for w in do:
            do[w].zero_()
        if pervector:
            b.run_pervector(P)
        else:
            b.run(P)
        sync()
        outs.append({w: host(do[w]) for w in do})
    info = b.info()
    b.close()
    return outs, info


@pytest.mark.parametrize("flags", [0, mg.BATCH_DYNAMIC, mg.BATCH_GRAPH, mg.BATCH_GRAPH | mg.BATCH_DYNAMIC])
def test_ragged_mul_pow_mixed(flags):
    ctxs, segs, meta, cur0, cur1 = ragged_case(11, 300, 20_000, [mg.OP_MUL, mg.OP_MUL, mg.OP_POW])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, 11)
    outs, info = run_ragged(meta, segs, ctxs, in0, in1, cur0, flags, reps=3)
    assert info["ntiles"] > 300
    for o in outs:                       # every replay (the tile counter resets itself)
        check_ragged(meta, inputs, o)


def test_ragged_redc_all_variants():
    ctxs, segs, meta, cur0, cur1 = ragged_case(12, 200, 10_000, [mg.OP_REDC])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, 12)
    outs, _ = run_ragged(meta, segs, ctxs, in0, in1, cur0, mg.BATCH_GRAPH | mg.BATCH_DYNAMIC, reps=2)
    for o in outs:
        check_ragged(meta, inputs, o)


def test_ragged_pervector_and_tuned_agree():
    ctxs, segs, meta, cur0, cur1 = ragged_case(13, 120, 50_000, [mg.OP_MUL, mg.OP_POW])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, 13)
    pv, _ = run_ragged(meta, segs, ctxs, in0, in1, cur0, 0, pervector=True)
    tu, info = run_ragged(meta, segs, ctxs, in0, in1, cur0, mg.BATCH_TUNE | mg.BATCH_GRAPH, reps=2)
    check_ragged(meta, inputs, pv[0])
    for o in tu:
        check_ragged(meta, inputs, o)


def test_ragged_empty_and_zero_length():
    c = mg.setup(8380417, 32)
    b = mg.Batch([c], [(0, mg.OP_MUL, "classic", 0, 0)])
    x = torch.zeros(16, dtype=torch.uint32, device="cuda")
    b.run(mg.pools([None, x, None], [None, x, None], [None, x, None]))
    sync()
    assert b.info()["ntiles"] == 0
    b.close()


# -------------------------------------------------------------------- CRT


def words_to_ints(w):
    return [sum(int(x) << (64 * j) for j, x in enumerate(row)) for row in w]


@pytest.mark.parametrize("k", [1, 2, 3, 8, 11, 16])
@pytest.mark.parametrize("kind", ["primes60", "primes62", "primes64", "mixed"])
def test_crt_parity(k, kind):
    g = inp.rng(94, k)
    if kind == "primes60":
        mods = inp.random_primes(g, 60, k)          # within a factor 2 and below 2^61: three-product quotients
    elif kind == "primes62":
        mods = inp.random_primes(g, 62, k)          # in [2^61, 2^62): exact Shoup quotients
    elif kind == "primes64":
        mods = inp.random_primes(g, 64, k)          # within a factor 2, above 2^63: one-subtraction path
    else:
        pool = [3, 5, 7, 65537, 1000000007, (1 << 61) - 1, (1 << 62) - 57, (1 << 64) - 59, 998244353,
                4294967291, 2147483647, 18446744073709551557 - 2 * 0, 1099511627791, 127, 8191, 131071]
        pool = sorted(set(p for p in pool if inp.is_prime(p)))
        mods = [pool[(i * 5) % len(pool)] for i in range(len(pool))][:k]
        mods = list(dict.fromkeys(mods))
        while len(mods) < k:
            q = inp.odd_modulus(g, 40)
            if inp.is_prime(q) and q not in mods:
                mods.append(q)
    n = 5003
    ld = 5008
    res = np.zeros((k, ld), np.uint64)
    for j, m in enumerate(mods):
        res[j, :n] = g.integers(0, m, size=n, dtype=np.uint64)
        res[j, :3] = [0, m - 1, 1]
    ctxs = [mg.setup(m, 64) for m in mods]
    got = mg.crt(ctxs, dev(res), n=n).cpu().numpy()
    want = orc.crt([[int(x) for x in res[j, :n]] for j in range(k)], mods)
    assert words_to_ints(got) == want


@pytest.mark.parametrize("k", [1, 3, 8])
def test_crt_small_and_edge_counts(k):
    """Element counts around one workgroup (the output leaves through LDS in
    16-byte chunks of the workgroup's words; an odd word count ends with one
    8-byte store), for each form: 60- and 62-bit primes (Shoup steps), 64-bit primes,
    moduli of mixed sizes."""
    g = inp.rng(94, 200 + k)
    for mods in (inp.random_primes(g, 60, k), inp.random_primes(g, 62, k), inp.random_primes(g, 64, k),
                 [3, 65537, (1 << 61) - 1, 1000000007, 127, 8191, 131071, (1 << 64) - 59][:k]):
        ctxs = [mg.setup(m, 64) for m in mods]
        for n in (1, 2, 255, 256, 257):
            res = np.stack([g.integers(0, m, size=n, dtype=np.uint64) for m in mods])
            got = mg.crt(ctxs, dev(res)).cpu().numpy()
            want = orc.crt([[int(x) for x in res[j]] for j in range(k)], mods)
            assert words_to_ints(got) == want, (mods[0], n)


def test_crt_rejects_common_factor():
    ctxs = [mg.setup(15, 64), mg.setup(21, 64)]
    res = torch.zeros((2, 16), dtype=torch.uint64, device="cuda")
    with pytest.raises(mg.MontError) as e:
        mg.crt(ctxs, res)
    assert e.value.code == -2


def test_crt_of_rns_product():
    """RNS product followed by reconstruction equals a b R^{-1} mod N_j in every row, i.e. the CRT
    of the per-row Montgomery products."""
    wl = inp.RNS64Workload(n=20_000)
    a, b = wl.operands(n=wl.n)
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    prod = mg.mul_rns(ctxs, dev(a), dev(b))
    X = words_to_ints(mg.crt(ctxs, prod).cpu().numpy())
    rows = [orc.mul("classic", 64, N, a[j], b[j]) for j, N in enumerate(wl.moduli)]
    assert X == orc.crt([[int(x) for x in r] for r in rows], wl.moduli)


def test_tune_mul_and_cache(tmp_path, monkeypatch):
    """The streaming tuner picks a candidate shape, keeps results exact and appends to the JSON cache."""
    import json
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MONT_TUNE_CACHE", str(cache))
    N, w = 8380417, 32
    c = mg.setup(N, w)
    saved = mg.get_launch(mg.OP_MUL, w, "plantard")
    try:
        a, b = operands("plantard", w, N, 1 << 22, inp.rng(92, 1))
        da, db = dev(a), dev(b)
        out = torch.empty_like(da)
        best = mg.tune_mul(c, da, db, out, variant="plantard")
        assert best["unroll"] in (1, 2, 4) and best["nontemporal"] in (0, 1) and best["blocks_per_cu"] in (0, 4, 8, 16)
        assert best["block"] in (64, 256)
        assert mg.get_launch(mg.OP_MUL, w, "plantard") == best
        got = host(mg.mul(c, da, db, variant="plantard"))
        assert np.array_equal(got, orc.mul("plantard", w, N, a, b))
        rec = [json.loads(l) for l in cache.read_text().splitlines()]
        assert ":mul:w32:v2:log2n22" in rec[-1]["key"] and rec[-1]["unroll"] == best["unroll"]
    finally:
        mg.set_launch(mg.OP_MUL, w, "plantard", **saved)
