"""Batched transforms on the GPU against the DFT definition (oracle)."""
import numpy as np
import pytest

import oracle as orc
import paper_2402_00675_amd as mg
from paper_2402_00675_amd import inputs as inp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDILOCKS = (1 << 64) - (1 << 32) + 1   # prime, 2^32 | N - 1, N > 2^63


def root(N, n):
    for g in range(2, 10000):
        w = pow(g, (N - 1) // n, N)
        if pow(w, n // 2, N) == N - 1:
            return w
    raise ValueError("no root")


def prime_1_mod(bits, log2n, seed):
    g = np.random.default_rng(seed)
    while True:
        k = int(g.integers(1 << (bits - 1 - log2n), 1 << (bits - log2n), dtype=np.uint64))
        p = k * (1 << log2n) + 1
        if p < (1 << bits) and inp.is_prime(p):
            return p


CASES = [
    (16, 12289, [1, 3, 4, 8, 9, 10, 12]),               # below 2^14: lazy butterflies (so is 3329)
    (16, 3329, [2, 5, 8]),
    (16, 18433, [1, 3, 6, 8, 10, 11]),                   # 2^14 < N < 2^15: reduced sums, smaller-modulus product
    (16, 36097, [3, 6, 8]),                      # above 2^15: wrap-checked modular add/subtract (both twiddle forms)
    (16, 40961, [4, 7, 8, 9, 10, 11, 12]),                 # above 2^16/phi: classic only
    (32, 8380417, [1, 4, 6, 7, 8, 9, 10, 12]),           # (2 log2n + 1) N < 2^32: no reduction between stages
    (32, 1073692673, [1, 2, 3, 8, 9, 10, 11, 12]),       # below 2^30, 5N > 2^32: lazy, one subtraction per stage
    (32, 2013265921, [5, 6, 8, 9, 10, 11, 12]),          # 2^30 < N < 2^31: reduced sums, smaller-modulus product
    (32, 3221225473, [4, 5, 7, 8, 9, 10, 11, 12]),        # above 2^31: the general classic product
    (64, prime_1_mod(62, 12, 1), [2, 4, 6, 8, 9, 10, 11, 12]),  # 2^61 < N < 2^62: reduced sums, smaller-modulus product
    (64, prime_1_mod(60, 12, 1), [3, 5, 7, 8, 9, 10, 11, 12]),  # below 2^61: lazy butterflies (8380417 takes them at w = 32)
    (64, GOLDILOCKS, [3, 4, 6, 8, 9, 10, 11, 12]),
    (64, 1125899906826241, [2, 6, 9, 10, 12]),          # 50-bit: no reduction between stages
]
DT = {16: np.uint16, 32: np.uint32, 64: np.uint64}


@pytest.mark.parametrize("w,N,logs", CASES, ids=["w%d-N%d" % (c[0], c[1]) for c in CASES])
def test_ntt_parity(w, N, logs):
    c = mg.setup(N, w)
    variants = ["classic"] + (["plantard"] if c.valid("plantard") else [])
    g = inp.rng(93, w + N % 97)
    for log2n in logs:
        n = 1 << log2n
        batch = 3 if log2n >= 11 else 17
        wr = root(N, n)
        x = g.integers(0, N, size=(batch, n), dtype=np.uint64).astype(DT[w])
        x[0, :] = 0
        x[1, :] = (N - 1)
        want_f = np.stack([orc.dft(w, N, x[i], wr) for i in range(batch)])
        for v in variants:
            d = torch.from_numpy(x.copy()).cuda()
            mg.ntt(c, d, wr, variant=v)
            got = d.cpu().numpy()
            assert np.array_equal(got, want_f), (v, log2n)
            mg.ntt(c, d, wr, inverse=True, variant=v)     # round trip
            assert np.array_equal(d.cpu().numpy(), x), (v, log2n)
        want_i = np.stack([orc.dft(w, N, x[i], wr, inverse=True) for i in range(min(batch, 3))])
        d = torch.from_numpy(x[:want_i.shape[0]].copy()).cuda()
        mg.ntt(c, d, wr, inverse=True, variant=variants[-1])
        assert np.array_equal(d.cpu().numpy(), want_i)


def test_ntt_rejects_bad_root_and_variant():
    c = mg.setup(12289, 16)
    d = torch.zeros((2, 16), dtype=torch.uint16, device="cuda")
    with pytest.raises(mg.MontError) as e:
        mg.ntt(c, d, 1)                        # 1^(n/2) != -1
    assert e.value.code == -2
    with pytest.raises(mg.MontError) as e:
        mg.ntt(c, d, root(12289, 16), variant="signed")
    assert e.value.code == -3


@pytest.mark.parametrize("w,N", [(16, 12289), (32, 8380417), (64, prime_1_mod(62, 12, 1))])
def test_ntt_unaligned_rows(w, N):
    """Rows that do not start on a 16-byte boundary take the element-wise path
    (at w = 16 both the 16-bit arithmetic, lengths 4 and 8, and the 32-bit
    arithmetic on 16-bit words, from 16 on)."""
    c = mg.setup(N, w)
    g = inp.rng(93, 500 + w)
    for n, batch in ((4, 5), (8, 9), (16, 7), (64, 5), (256, 6), (512, 3), (1024, 3), (2048, 3), (4096, 2)):
        wr = root(N, n)
        x = g.integers(0, N, size=(batch, n), dtype=np.uint64).astype(DT[w])
        want = np.stack([orc.dft(w, N, x[i], wr) for i in range(batch)])
        flat = torch.zeros(batch * n + 1, dtype=torch.from_numpy(x).dtype, device="cuda")
        view = flat[1:].view(batch, n)                 # one element in: misaligned for every width
        view.copy_(torch.from_numpy(x).cuda())
        for v in ["classic"] + (["plantard"] if c.valid("plantard") else []):
            dv = flat.clone()[1:].view(batch, n)
            assert dv.data_ptr() % 16 != 0
            mg.ntt(c, dv, wr, variant=v)
            assert np.array_equal(dv.cpu().numpy(), want), (v, n)


@pytest.mark.parametrize("w,N", [(16, 3329), (16, 12289), (16, 18433), (16, 40961), (32, 8380417), (32, 1073692673),
                                 (32, 2013265921), (32, 3221225473), (64, prime_1_mod(62, 12, 1)),
                                 (64, prime_1_mod(60, 12, 1)), (64, GOLDILOCKS), (64, 1125899906826241)])
def test_ntt_many_per_wave(w, N):
    """Batches of lengths 2 to 4096 larger than the resident waves or
    workgroups (up to 1024 each wave takes several units of max(n, 256)
    coefficients, with the next one's loads in flight, and below 256 the last
    unit is partial; at 2048 and 4096 each workgroup of four waves takes
    several polynomials): 40 seeded rows and the last against the DFT, the
    whole batch through the round trip."""
    c = mg.setup(N, w)
    g = inp.rng(93, 700 + w + N % 89)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for n in (2, 8, 16, 64, 128, 256, 512, 1024, 2048, 4096):
        if (N - 1) % n:
            continue
        # the one-wave kernel launches 32 workgroups of four waves per CU up to
        # length 256 and 8 at 512 and 1024: give every wave two units or more
        waves = cus * (32 if n <= 256 else 8) * 4
        batch = (2 * waves + 5) * 256 // n + (3 if n < 256 else 0) if n <= 1024 else 2 * 8192 + 5
        wr = root(N, n)
        x = g.integers(0, N, size=(batch, n), dtype=np.uint64).astype(DT[w])
        rows = sorted(set(g.choice(batch, size=40, replace=False).tolist()) | {batch - 1})
        want = {r: orc.dft(w, N, x[r], wr) for r in rows}
        for v in ["classic"] + (["plantard"] if c.valid("plantard") else []):
            d = torch.from_numpy(x.copy()).cuda()
            mg.ntt(c, d, wr, variant=v)
            got = d.cpu().numpy()
            for r in rows:
                assert np.array_equal(got[r], want[r]), (v, n, r)
            mg.ntt(c, d, wr, inverse=True, variant=v)
            assert np.array_equal(d.cpu().numpy(), x), (v, n)
