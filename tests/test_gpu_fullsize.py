"""Parity at the workloads' full sizes, in the launch shapes the benchmark
times (the library defaults), every output compared with the oracle.

The oracle runs on host threads over chunks; at ~10 ns per element the
largest case (2^28 products) takes well under a second of host time.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle as orc
import paper_2402_00675_amd as mg
from paper_2402_00675_amd import inputs as inp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WORKERS = min(16, len(os.sched_getaffinity(0)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def chunked_equal(got, fn, n, step=1 << 22):
    """True when got[s:e] == fn(s, e) for every chunk."""
    def chk(s):
        e = min(s + step, n)
        return bool(np.array_equal(got[s:e], fn(s, e)))
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        return all(ex.map(chk, range(0, n, step)))


def test_r16_workload():
    wl = inp.R16Workload()
    a, b = wl.operands()
    c = mg.setup(wl.N, 16)
    got = mg.mul(c, dev(a), dev(b)).cpu().numpy()
    assert np.array_equal(got, orc.mul("classic", 16, wl.N, a, b))


@pytest.mark.parametrize("variant", ["classic", "plantard", "signed", "signed_plantard", "signed_plantard_alpha"])
def test_r32_workload(variant):
    wl = inp.R32Workload()
    signed = variant.startswith("signed")
    a, b = wl.operands(signed)
    c = mg.setup(wl.N, 32)
    got = mg.mul(c, dev(a), dev(b), variant=variant).cpu().numpy()
    assert chunked_equal(got, lambda s, e: orc.mul(variant, 32, wl.N, a[s:e], b[s:e], alpha=1), wl.n)


def test_rns64_workload():
    wl = inp.RNS64Workload()
    a, b = wl.operands()
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    got = mg.mul_rns(ctxs, dev(a), dev(b)).cpu().numpy()
    for i, N in enumerate(wl.moduli):
        assert chunked_equal(got[i], lambda s, e, i=i, N=N: orc.mul("classic", 64, N, a[i, s:e], b[i, s:e]), wl.n), i


@pytest.mark.parametrize("flags,shape", [(mg.BATCH_GRAPH, None), (mg.BATCH_GRAPH | mg.BATCH_TUNE, None),
                                         (mg.BATCH_GRAPH, (8192, 2, 1)), (mg.BATCH_GRAPH, (4096, 2, 8))],
                         ids=["default", "tuned", "dynamic-1-counter", "dynamic-8-counters"])
def test_ragged_workload(flags, shape):
    """The 4096-vector batch of the benchmark, every element against the oracle: the default
    shape, the tuned one, and the persistent dynamic grids with one and with eight tile counters."""
    wl = inp.RaggedWorkload()
    lens, wide, mods = wl.segments()
    offs, (a32, b32), (a64, b64) = wl.operands(lens, wide, mods)
    ctxs = [mg.setup(N, 64 if wd else 32) for N, wd in zip(mods, wide)]
    segs = [(i, mg.OP_MUL, "classic", int(n), int(o), int(o)) for i, (n, o) in enumerate(zip(lens, offs))]
    d = [dev(x) for x in (a32, b32, a64, b64)]
    o32 = torch.zeros_like(d[0])
    o64 = torch.zeros_like(d[2])
    P = mg.pools([None, d[0], d[2]], [None, d[1], d[3]], [None, o32, o64])
    bt = mg.Batch(ctxs, segs, flags=flags)
    if shape is not None:
        bt.set_shape(tile_elems=shape[0], blocks_per_cu=shape[1], dynamic=shape[2])
    bt.run(P)
    bt.run(P)           # a replay
    torch.cuda.synchronize()
    g32, g64 = o32.cpu().numpy(), o64.cpu().numpy()
    bt.close()

    def seg_ok(i):
        n, o, wd, N = int(lens[i]), int(offs[i]), wide[i], mods[i]
        if wd:
            return np.array_equal(g64[o:o + n], orc.mul("classic", 64, N, a64[o:o + n], b64[o:o + n]))
        return np.array_equal(g32[o:o + n], orc.mul("classic", 32, N, a32[o:o + n], b32[o:o + n]))

    with cf.ThreadPoolExecutor(WORKERS) as ex:
        assert all(ex.map(seg_ok, range(len(lens))))


def test_pow_bench_shape_sampled():
    """Exponentiation at the benchmark's size (2^22), every 61st element checked."""
    g = inp.rng(inp.W_SERVE, 7)
    for bits, w in ((31, 32), (62, 64)):
        N = inp.odd_modulus(g, bits)
        n = 1 << 22
        dt = np.uint32 if w == 32 else np.uint64
        x = inp.uniform_residues(g, N, n, dt)
        e = inp.u64_uniform(g, n)
        got = mg.pow(mg.setup(N, w), dev(x), dev(e)).cpu().numpy()
        idx = np.arange(0, n, 61)
        assert np.array_equal(got[idx], orc.pow(w, N, x[idx], e[idx]))


def test_serving_stream_every_job():
    """The 10^5-job serving stream (60 % products, 40 % exponentiations with
    uniform 64-bit exponents, lengths log-uniform in [2^8, 2^18], odd 31- and
    62-bit moduli) through the server configuration the benchmark times, all
    jobs submitted at once, replayed five times: each pass gives a different
    fifth of the jobs outputs of their own (the rest write a shared sink), so
    every job is checked once: products in full, exponentiations on their first
    and last element and 256 seeded ones."""
    from paper_2402_00675_amd import serve
    njobs, passes = 100_000, 5
    checked = {0: 0, 1: 0}
    for c in range(passes):
        stream = serve.JobStream(torch, njobs, distinct_outputs=range(c, njobs, passes))
        srv = mg.Server(hbm_budget_bytes=8 << 30, streams=3, max_batch_jobs=512)
        stream.declare(srv)
        try:
            done = serve.replay(srv, stream, np.zeros(njobs))
            st = srv.stats()
        finally:
            srv.close()
        assert len(done) == njobs and all(d[1] == 0 for d in done)
        # one resident-constant upload per modulus seen, more moduli than the table holds
        # (entries are reused), a hit for every other job
        assert st["ctx_uploads"] + st["ctx_hits"] == njobs and st["ctx_uploads"] >= len(set(stream.mods))

        def job_ok(i):
            got = stream.outs[i].numpy()
            x, y = stream.inputs_of(i)
            w, N, n = (64 if stream.wide[i] else 32), int(stream.mods[i]), len(x)
            if stream.ops[i] == 0:
                return bool(np.array_equal(got, orc.mul("classic", w, N, x, y)))
            pick = np.random.default_rng(i).integers(0, n, size=256)
            idx = np.unique(np.concatenate([[0, n - 1], pick]))
            return bool(np.array_equal(got[idx], orc.pow(w, N, x[idx], y[idx])))

        sample = sorted(stream.outs)
        with cf.ThreadPoolExecutor(WORKERS) as ex:
            ok = list(ex.map(job_ok, sample))
        bad = [i for i, v in zip(sample, ok) if not v]
        assert not bad, (c, bad[:10])
        for i in sample:
            checked[int(stream.ops[i])] += 1
        print("pass %d: %d jobs checked" % (c, len(sample)), flush=True)
        del stream
    assert checked[0] + checked[1] == njobs
    assert checked[0] > 55_000 and checked[1] > 35_000    # both kinds are well represented


def test_crt_bench_shape_sampled():
    """CRT reconstruction at the benchmark's shape (2^25 integers from the 8 rows
    of the 64-bit RNS workload), every 8191st element and the last one checked."""
    wl = inp.RNS64Workload()
    a, _ = wl.operands()
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    got = mg.crt(ctxs, dev(a)).cpu().numpy().view(np.uint64)
    idx = list(range(0, wl.n, 8191)) + [wl.n - 1]
    want = orc.crt([[int(x) for x in a[j, idx]] for j in range(wl.k)], wl.moduli)
    have = [sum(int(x) << (64 * w) for w, x in enumerate(got[i])) for i in idx]
    assert have == want


@pytest.mark.parametrize("variant", ["classic", "plantard"])
def test_ntt_bench_shape_sampled(variant):
    """NTTs at the benchmark's shape (2^18 transforms of length 256 over
    N = 8380417), forward and back; 64 seeded transforms checked against the DFT
    by its definition, and the round trip checked in full."""
    N, n, batch = 8380417, 256, 1 << 18
    c = mg.setup(N, 32)
    root = next(w for w in (pow(q, (N - 1) // n, N) for q in range(2, 100)) if pow(w, n // 2, N) == N - 1)
    x = inp.uniform_residues(inp.rng(inp.W_R32, 9), N, batch * n, np.uint32).reshape(batch, n)
    d = dev(x)
    mg.ntt(c, d, root, variant=variant)
    got = d.cpu().numpy()
    rows = np.random.default_rng(5).choice(batch, size=64, replace=False)
    for r in rows:
        assert np.array_equal(got[r], orc.dft(32, N, x[r], root)), r
    mg.ntt(c, d, root, inverse=True, variant=variant)
    assert np.array_equal(d.cpu().numpy(), x)


@pytest.mark.parametrize("variant", ["classic", "plantard"])
@pytest.mark.parametrize("log2n", [4, 8, 12])
def test_ntt16_full_size_sampled(variant, log2n):
    """2^26 16-bit coefficients mod 12289 (the size of the benchmark's length
    sweep), at lengths where the 16-bit transform computes in 32-bit words:
    16 seeded transforms checked against the DFT by its definition, and the
    round trip checked in full."""
    N, n = 12289, 1 << log2n
    batch = (1 << 26) // n
    c = mg.setup(N, 16)
    root = next(w for w in (pow(q, (N - 1) // n, N) for q in range(2, 100)) if pow(w, n // 2, N) == N - 1)
    x = inp.uniform_residues(inp.rng(inp.W_R16, 11 + log2n), N, batch * n, np.uint16).reshape(batch, n)
    d = dev(x)
    mg.ntt(c, d, root, variant=variant)
    got = d.cpu().numpy()
    rows = np.random.default_rng(log2n).choice(batch, size=16, replace=False)
    for r in rows:
        assert np.array_equal(got[r], orc.dft(16, N, x[r], root)), r
    mg.ntt(c, d, root, inverse=True, variant=variant)
    assert np.array_equal(d.cpu().numpy(), x)
