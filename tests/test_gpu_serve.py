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


def test_server_is_a_context_manager():
    x = torch.from_numpy(np.arange(512, dtype=np.uint32))
    y = torch.from_numpy(np.full(512, 5, dtype=np.uint32))
    o = torch.from_numpy(np.zeros(512, dtype=np.uint32))
    with mg.Server(hbm_budget_bytes=16 << 20, streams=1) as srv:
        srv.submit(3, 8380417, 32, mg.OP_MUL, x, y, o)
        srv.drain(60_000)
        assert srv.poll(4)[0][1] == 0
    assert not srv.h
    assert np.array_equal(o.numpy(), orc.mul("classic", 32, 8380417, x.numpy(), y.numpy()))


def test_resident_constants_are_reused():
    """Jobs that share a modulus reuse its resident constants: one upload per distinct modulus."""
    stream = serve.JobStream(torch, njobs=200, seed_rep=5, distinct_outputs=True, hi=1 << 12)
    mods = [int(m) for m in stream.mods]
    shared = 0
    for i in range(0, 200, 2):
        # job i + 1 takes job i's modulus where its operands (drawn below its own bucket's
        # floor) stay below that modulus
        w = 64 if stream.wide[i] else 32
        if bool(stream.wide[i]) == bool(stream.wide[i + 1]) and serve.bucket_floor(stream.bucket[i + 1], w) <= mods[i]:
            mods[i + 1] = mods[i]
            stream.jobs[i + 1].N = mods[i]
            shared += 1
    assert shared >= 10
    stream.mods = mods
    srv = mg.Server(hbm_budget_bytes=64 << 20, streams=2, max_batch_jobs=16)
    stream.declare(srv)
    try:
        done = serve.replay(srv, stream, np.zeros(stream.njobs))
        assert all(d[1] == 0 for d in done)
        st = srv.stats()
        distinct = len({(m, bool(w)) for m, w in zip(mods, stream.wide)})
        assert st["ctx_uploads"] == distinct and st["ctx_uploads"] + st["ctx_hits"] == stream.njobs
        for i in range(stream.njobs):
            assert np.array_equal(stream.outs[i].numpy(), oracle_of(stream, i)), i
        # the same stream again: every modulus is resident already
        for i in range(stream.njobs):
            stream.outs[i].zero_()
        done = serve.replay(srv, stream, np.zeros(stream.njobs))
        assert all(d[1] == 0 for d in done)
        st2 = srv.stats()
        assert st2["ctx_uploads"] == distinct and st2["ctx_hits"] == st["ctx_hits"] + stream.njobs
        for i in range(0, stream.njobs, 3):
            assert np.array_equal(stream.outs[i].numpy(), oracle_of(stream, i)), i
    finally:
        srv.close()


def test_cancel_waiting_jobs():
    """Jobs cancelled before their launch complete with MONT_E_CANCELED and leave their out
    buffers untouched; the others complete exactly; memory returns to zero."""
    stream = serve.JobStream(torch, njobs=240, seed_rep=6, distinct_outputs=True, hi=1 << 16)
    for i in range(stream.njobs):
        stream.outs[i].fill_(0x5A)          # every element 90, never a result here
    srv = mg.Server(hbm_budget_bytes=32 << 20, streams=1, max_batch_jobs=8)
    stream.declare(srv)
    try:
        for i in range(stream.njobs):
            srv.submit_struct(stream.jobs[i])
        rcs = {i: srv.cancel(i) for i in range(stream.njobs - 1, 0, -3)}
        assert all(rc in (0, mg.E_BUSY, mg.E_INVAL) for rc in rcs.values())
        canceled = {i for i, rc in rcs.items() if rc == 0}
        assert len(canceled) > 20                   # most late jobs were still waiting
        srv.drain(120_000)
        got = {}
        while len(got) < stream.njobs:
            for d in srv.poll(4096, 100):
                assert d[0] not in got
                got[d[0]] = d[1]
        for i in range(stream.njobs):
            if i in canceled:
                assert got[i] == mg.E_CANCELED
                assert np.all(stream.outs[i].numpy() == 0x5A), i
            else:
                assert got[i] == 0
                assert np.array_equal(stream.outs[i].numpy(), oracle_of(stream, i)), i
        st = srv.stats()
        assert st["canceled"] == len(canceled) and st["bytes_in_use"] == 0
        assert srv.cancel(0) == mg.E_INVAL           # finished long ago
    finally:
        srv.close()


def test_batch_deadline_gives_up_and_recovers_memory():
    """With a 1 microsecond deadline nearly every batch is given up at its first poll: its jobs
    complete with MONT_E_DEVICE, the stream is replaced, and the batch's memory stays reserved
    until the abandoned work (which runs to its normal end here) is seen to finish.  Jobs that
    did complete are exact."""
    import time
    stream = serve.JobStream(torch, njobs=120, seed_rep=7, distinct_outputs=True, hi=1 << 16)
    srv = mg.Server(hbm_budget_bytes=64 << 20, streams=2, max_batch_jobs=8, deadline_us=1)
    stream.declare(srv)
    try:
        done = serve.replay(srv, stream, np.zeros(stream.njobs))
        status = {d[0]: d[1] for d in done}
        assert set(status.values()) <= {0, mg.E_DEVICE}
        st = srv.stats()
        assert st["timed_out"] > 0 and st["timed_out"] == sum(v == mg.E_DEVICE for v in status.values())
        for i, v in status.items():
            if v == 0:
                assert np.array_equal(stream.outs[i].numpy(), oracle_of(stream, i)), i
        t0 = time.time()
        while srv.stats()["quarantined_bytes"] and time.time() - t0 < 30:
            time.sleep(0.01)
        st = srv.stats()
        assert st["quarantined_bytes"] == 0 and st["bytes_in_use"] == 0 and st["dead_streams"] == 0
        # the abandoned batches ran to their end: their outputs are exact too
        for i, v in status.items():
            if v != 0:
                assert np.array_equal(stream.outs[i].numpy(), oracle_of(stream, i)), i
    finally:
        srv.close()
