"""The serving loop on the GPU: every job's result is the same alone and in
the mix (bit for bit), equals the oracle, and admission respects the device
budget."""
import numpy as np
import pytest

import oracle as orc
import paper_2402_00675_amd as mg
from paper_2402_00675_amd import serve

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def oracle_of(stream, i):
    w = 64 if stream.wide[i] else 32
    x, y = stream.inputs_of(i)
    N = int(stream.mods[i])
    if stream.ops[i] == 0:
        return orc.mul("classic", w, N, x, y)
    return orc.pow(w, N, x, y)


@pytest.mark.parametrize("staging", ["kernel", "dma"])
def test_alone_vs_mix_and_oracle(staging):
    stream = serve.JobStream(torch, njobs=400, seed_rep=3, distinct_outputs=True, hi=1 << 14)
    srv = mg.Server(hbm_budget_bytes=256 << 20, streams=3, max_batch_jobs=64)
    if staging == "kernel":
        stream.declare(srv)      # copies by the gather/scatter kernels
    try:
        done = serve.replay(srv, stream, stream.gaps_unit / 20000.0)   # Poisson, 20k jobs/s
        assert len(done) == stream.njobs and all(d[1] == 0 for d in done)
        st = srv.stats()
        assert st["completed"] == stream.njobs and st["jobs_launched"] == stream.njobs
        assert st["launches"] < stream.njobs          # jobs were fused into batches
        mix = {i: stream.outs[i].numpy().copy() for i in range(stream.njobs)}
        for i in range(stream.njobs):
            assert np.array_equal(mix[i], oracle_of(stream, i)), i
        for i in range(stream.njobs):                 # each job alone
            stream.outs[i].zero_()
            srv.submit_struct(stream.jobs[i])
            srv.drain(60_000)
            got = srv.poll(16)
            assert [g[0] for g in got] == [i] and got[0][1] == 0
            assert np.array_equal(stream.outs[i].numpy(), mix[i]), i
    finally:
        srv.close()


def test_budget_bounds_admission():
    stream = serve.JobStream(torch, njobs=300, seed_rep=4, distinct_outputs=True, hi=1 << 14)
    budget = 8 << 20
    srv = mg.Server(hbm_budget_bytes=budget, streams=2, max_batch_jobs=32)
    stream.declare(srv)
    try:
        done = serve.replay(srv, stream, np.zeros(stream.njobs))       # everything at once
        assert all(d[1] == 0 for d in done)
        st = srv.stats()
        assert 0 < st["peak_bytes_in_use"] <= budget and st["bytes_in_use"] == 0
        for i in range(0, stream.njobs, 7):
            assert np.array_equal(stream.outs[i].numpy(), oracle_of(stream, i)), i
        # a job larger than the whole budget is refused at submission
        big = np.zeros(1 << 20, np.uint32)
        with pytest.raises(mg.MontError) as e:
            srv.submit(10**6, 8380417, 32, mg.OP_MUL, big, big, big)
        assert e.value.code == -2
        with pytest.raises(mg.MontError) as e:
            srv.submit(10**6 + 1, 8380418, 32, mg.OP_MUL, big[:8], big[:8], big[:8])
        assert e.value.code == -1
    finally:
        srv.close()


def test_host_region_checks():
    srv = mg.Server(hbm_budget_bytes=16 << 20, streams=1)
    try:
        pinned = torch.empty(1 << 12, dtype=torch.uint32, pin_memory=True)
        srv.host_region(pinned)
        srv.host_region(pinned[16:64])            # inside a declared region: accepted
        pageable = torch.empty(1 << 12, dtype=torch.uint32)
        with pytest.raises(mg.MontError) as e:
            srv.host_region(pageable)             # not pinned: refused, DMA path stays
        assert e.value.code == -1
        dev = torch.empty(1 << 12, dtype=torch.uint32, device="cuda")
        with pytest.raises(mg.MontError):
            srv._keep = {}
            import ctypes
            from paper_2402_00675_amd import _lib
            _lib.check(_lib._serve_lib().mont_serve_host_region(srv.h, ctypes.c_void_p(dev.data_ptr()), 4096))
        # a job mixing a declared input and undeclared buffers still completes correctly
        x = pinned[:256]
        x.numpy()[:] = np.arange(256, dtype=np.uint32)
        y = torch.empty(256, dtype=torch.uint32, pin_memory=True)
        y.numpy()[:] = 7
        o = torch.empty(256, dtype=torch.uint32)
        srv.submit(1, 8380417, 32, mg.OP_MUL, x, y, o)
        srv.drain(60_000)
        assert srv.poll(4)[0][1] == 0
        want = orc.mul("classic", 32, 8380417, x.numpy().copy(), y.numpy().copy())
        assert np.array_equal(o.numpy(), want)
    finally:
        srv.close()
