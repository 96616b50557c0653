"""mont_batch_run_noalloc (needs a GPU): the allocation-free ragged batch against
mont_batch_create + mont_batch_run on the same inputs, element by element, on
two calls in a row (the second smaller), and against the oracle."""
import numpy as np
import pytest

import paper_2402_00675_amd as mg

from test_gpu_parity import check_ragged, dev, host, ragged_buffers, ragged_case, sync

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _pools(meta, cur0, cur1, seed):
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, seed)
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    d1 = {w: dev(in1[w]) for w in (16, 32, 64)}
    outs = [{w: torch.zeros(cur0[w] + 16, dtype=d0[w].dtype, device="cuda") for w in (16, 32, 64)}
            for _ in range(2)]
    P = [mg.pools([d0[16], d0[32], d0[64]], [d1[16], d1[32], d1[64]], [o[16], o[32], o[64]]) for o in outs]
    return inputs, outs, P, (d0, d1)


@pytest.mark.parametrize("tile", [0, 1024])
def test_noalloc_matches_batch_run_twice(tile):
    for seed, nseg, maxlen, ops in ((61, 400, 30_000, [mg.OP_MUL, mg.OP_MUL, mg.OP_POW]),
                                    (62, 90, 5_000, [mg.OP_MUL, mg.OP_POW])):   # second call: smaller
        ctxs, segs, meta, cur0, cur1 = ragged_case(seed, nseg, maxlen, ops)
        inputs, outs, P, keep = _pools(meta, cur0, cur1, seed)
        bt = mg.Batch(ctxs, segs)
        bt.run(P[0])
        mg.batch_run_noalloc(ctxs, segs, P[1], tile_elems=tile)
        sync()
        bt.close()
        ref = {w: host(outs[0][w]) for w in outs[0]}
        got = {w: host(outs[1][w]) for w in outs[1]}
        for w in ref:
            assert np.array_equal(got[w], ref[w]), (seed, w)
        check_ragged(meta, inputs, got)


def test_noalloc_reductions():
    ctxs, segs, meta, cur0, cur1 = ragged_case(63, 120, 8_000, [mg.OP_REDC])
    inputs, outs, P, keep = _pools(meta, cur0, cur1, 63)
    bt = mg.Batch(ctxs, segs)
    bt.run(P[0])
    mg.batch_run_noalloc(ctxs, segs, P[1])
    sync()
    bt.close()
    for w in outs[0]:
        assert np.array_equal(host(outs[1][w]), host(outs[0][w])), w
    check_ragged(meta, inputs, {w: host(outs[1][w]) for w in outs[1]})


def test_noalloc_rejects_tables_beyond_the_scratch_array():
    c = mg.setup(8380417, 32)
    x = torch.zeros(16, dtype=torch.uint32, device="cuda")
    P = mg.pools([None, x, None], [None, x, None], [None, x, None])
    with pytest.raises(mg.MontError) as e:
        mg.batch_run_noalloc([c], [(0, mg.OP_MUL, "classic", 1 << 30, 0)], P, tile_elems=256)
    assert e.value.code == -1 and "scratch" in str(e.value)
