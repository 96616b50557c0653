"""In-place calls (out == an input of the same width) against the CPU oracle (needs a GPU).

The interface allows every call to write its result over one of its inputs.
Each case copies the inputs to the device, calls the library with the output
pointer equal to an input pointer, and compares every element with the oracle
evaluated on the original inputs: a call that read an element after writing it,
or ran twice over the same buffer, would not match.
"""
import numpy as np
import pytest

import oracle as orc
import paper_2402_00675_amd as mg
from paper_2402_00675_amd import inputs as inp

from test_gpu_parity import ALL_VARIANTS, NP_E, SIGNED, check_ragged, dev, host, operands, ragged_buffers, \
    ragged_case, sync

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WIDTH_N = {16: 3329, 32: 8380417, 64: (1 << 62) - 57}


@pytest.mark.parametrize("w", [16, 32, 64])
@pytest.mark.parametrize("variant", ["classic", "signed", "plantard", "signed_plantard"])
@pytest.mark.parametrize("which", ["a", "b"])
@pytest.mark.parametrize("offset", [0, 1])
def test_mul_in_place(w, variant, which, offset):
    """mont_mul with out == a or out == b; offset 1 takes the element-wise path (not 16-byte aligned)."""
    N = WIDTH_N[w]
    c = mg.setup(N, w)
    n = 50_021
    a, b = operands(variant, w, N, n + offset, inp.rng(90, w + len(variant) + offset))
    want = orc.mul(variant, w, N, a[offset:], b[offset:])
    da, db = dev(a), dev(b)
    x, y = da[offset:], db[offset:]
    out = x if which == "a" else y
    mg.mul(c, x, y, out=out, variant=variant)
    got = host(out)
    assert np.array_equal(got, want)
    # the other operand is untouched
    other = host(y if which == "a" else x)
    assert np.array_equal(other, (b if which == "a" else a)[offset:])


@pytest.mark.parametrize("w", [16, 32, 64])
def test_mul_const_in_place(w):
    N = WIDTH_N[w]
    c = mg.setup(N, w)
    n = 40_009
    for variant in ["classic", "signed", "plantard", "signed_plantard"]:
        a, bs = operands(variant, w, N, n, inp.rng(89, w))
        b = int(bs[3])
        want = orc.mul(variant, w, N, a, np.full(n, b, dtype=a.dtype))
        da = dev(a)
        mg.mul_const(c, da, b, out=da, variant=variant)
        assert np.array_equal(host(da), want), variant


def test_mul_rns_in_place():
    wl = inp.RNS64Workload(n=30_011)
    a, b = wl.operands(n=wl.n)
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    da, db = dev(a), dev(b)
    mg.mul_rns(ctxs, da, db, out=db)
    got = host(db)
    for i, N in enumerate(wl.moduli):
        assert np.array_equal(got[i], orc.mul("classic", 64, N, a[i], b[i])), i
    assert np.array_equal(host(da), a)


@pytest.mark.parametrize("w", [16, 32, 64])
def test_pow_in_place(w):
    g = inp.rng(88, w)
    dt = NP_E[w][0]
    for N in {16: [3329, 65521], 32: [8380417, 4294967291], 64: [(1 << 62) - 57, (1 << 64) - 59]}[w]:
        n = 9_001
        x = g.integers(0, N, size=n, dtype=np.uint64).astype(dt)
        e = inp.u64_uniform(g, n)
        want = orc.pow(w, N, x, e)
        dx = dev(x)
        mg.pow(mg.setup(N, w), dx, dev(e), out=dx)
        assert np.array_equal(host(dx), want), N


def test_tune_mul_in_place(tmp_path, monkeypatch):
    """The tuner's candidate runs never write the caller's buffers: out == a gets one product."""
    monkeypatch.setenv("MONT_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    N, w = 8380417, 32
    c = mg.setup(N, w)
    saved = mg.get_launch(mg.OP_MUL, w, "signed")
    try:
        a, b = operands("signed", w, N, 1 << 20, inp.rng(87, 1))
        da, db = dev(a), dev(b)
        mg.tune_mul(c, da, db, da, variant="signed")
        assert np.array_equal(host(da), orc.mul("signed", w, N, a, b))
        assert np.array_equal(host(db), b)
    finally:
        mg.set_launch(mg.OP_MUL, w, "signed", **saved)


def _ragged_in_place(seed, flags, shape=None):
    """A mixed product/exponentiation batch whose output pools are its in0 pools."""
    ctxs, segs, meta, cur0, cur1 = ragged_case(seed, 150, 20_000, [mg.OP_MUL, mg.OP_MUL, mg.OP_POW])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, seed)
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    d1 = {w: dev(in1[w]) for w in (16, 32, 64)}
    P = mg.pools([d0[16], d0[32], d0[64]], [d1[16], d1[32], d1[64]], [d0[16], d0[32], d0[64]])
    bt = mg.Batch(ctxs, segs, flags=flags)
    if shape is not None:
        bt.set_shape(**shape)
    bt.run(P)
    sync()
    out = {w: host(d0[w]) for w in d0}
    info = bt.info()
    bt.close()
    check_ragged(meta, inputs, out)
    return info


@pytest.mark.parametrize("flags", [0, mg.BATCH_GRAPH, mg.BATCH_DYNAMIC, mg.BATCH_TUNE,
                                   mg.BATCH_TUNE | mg.BATCH_GRAPH])
def test_ragged_in_place(flags, tmp_path, monkeypatch):
    # a cache file of its own: the tuner must really time its candidates here
    monkeypatch.setenv("MONT_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    _ragged_in_place(21 + flags, flags)


def test_ragged_in_place_persistent():
    info = _ragged_in_place(31, mg.BATCH_GRAPH, dict(tile_elems=256, blocks_per_cu=1, dynamic=True))
    assert info["blocks_per_cu"] == 1 and info["grid"] < info["ntiles"]


# ------------------------------------------------------ ragged launch shapes

SHAPES = [(bpc, dyn, tile, bs) for bpc in (0, 4, 16) for dyn in (False, True) for tile in (1024, 8192)
          for bs in (64, 256)]


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("bpc,dyn,tile,bs", SHAPES)
def test_ragged_shapes(bpc, dyn, tile, bs, graph):
    """One-pass and persistent grids, static and dynamic schedules, against the oracle on every
    replay (the dynamic schedule's counter must reset itself between runs)."""
    ctxs, segs, meta, cur0, cur1 = ragged_case(41, 300, 20_000, [mg.OP_MUL, mg.OP_MUL, mg.OP_POW])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, 41)
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    d1 = {w: dev(in1[w]) for w in (16, 32, 64)}
    do = {w: torch.zeros(cur0[w] + 16, dtype=d0[w].dtype, device="cuda") for w in (16, 32, 64)}
    P = mg.pools([d0[16], d0[32], d0[64]], [d1[16], d1[32], d1[64]], [do[16], do[32], do[64]])
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_GRAPH if graph else 0)
    bt.set_shape(tile_elems=tile, blocks_per_cu=bpc, dynamic=dyn, block=bs)
    info = bt.info()
    assert info["blocks_per_cu"] == bpc and info["tile_elems"] == tile and info["block"] == bs
    assert bool(info["flags"] & mg.BATCH_DYNAMIC) == dyn
    if bpc:
        assert info["grid"] <= info["ntiles"] and info["grid"] <= bpc * torch.cuda.get_device_properties(0).multi_processor_count
    else:
        assert info["grid"] == info["ntiles"]
    for _ in range(3):
        for w in do:
            do[w].zero_()
        bt.run(P)
        sync()
        check_ragged(meta, inputs, {w: host(do[w]) for w in do})
    bt.close()


@pytest.mark.parametrize("bpc,dyn", [(0, False), (4, False), (16, True)])
def test_ragged_redc_shapes(bpc, dyn):
    ctxs, segs, meta, cur0, cur1 = ragged_case(42, 150, 10_000, [mg.OP_REDC])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, 42)
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    do = {w: torch.zeros(cur0[w] + 16, dtype=d0[w].dtype, device="cuda") for w in (16, 32, 64)}
    P = mg.pools([d0[16], d0[32], d0[64]], [None, None, None], [do[16], do[32], do[64]])
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_GRAPH)
    bt.set_shape(tile_elems=2048, blocks_per_cu=bpc, dynamic=dyn, block=64 if dyn else 256)
    for _ in range(2):
        bt.run(P)
        sync()
        check_ragged(meta, inputs, {w: host(do[w]) for w in do})
    bt.close()


def _ragged_out_case(seed):
    ctxs, segs, meta, cur0, cur1 = ragged_case(seed, 300, 20_000, [mg.OP_MUL, mg.OP_MUL, mg.OP_POW])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, seed)
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    d1 = {w: dev(in1[w]) for w in (16, 32, 64)}
    do = {w: torch.zeros(cur0[w] + 16, dtype=d0[w].dtype, device="cuda") for w in (16, 32, 64)}
    P = mg.pools([d0[16], d0[32], d0[64]], [d1[16], d1[32], d1[64]], [do[16], do[32], do[64]])
    return ctxs, segs, meta, inputs, do, P


def _run_check(bt, P, do, meta, inputs):
    for w in do:
        do[w].zero_()
    bt.run(P)
    sync()
    check_ragged(meta, inputs, {w: host(do[w]) for w in do})


def test_ragged_graph_follows_shape_changes():
    """A captured batch whose kernel changes (workgroup size, non-temporal
    access) or whose grid changes between runs: every run matches the oracle."""
    ctxs, segs, meta, inputs, do, P = _ragged_out_case(43)
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_GRAPH)
    steps = [dict(tile_elems=4096, block=256), dict(tile_elems=4096, block=64),
             dict(tile_elems=4096, block=64, nontemporal=False), dict(tile_elems=2048, block=256),
             dict(tile_elems=2048, blocks_per_cu=2, dynamic=True, block=256),
             dict(tile_elems=2048, blocks_per_cu=2, dynamic=True, block=64),
             dict(tile_elems=2048, blocks_per_cu=2, dynamic=False, block=64, nontemporal=False)]
    for shape in steps:
        bt.set_shape(**shape)
        info = bt.info()
        assert info["block"] == shape["block"] and info["tile_elems"] == shape["tile_elems"]
        for _ in range(2):
            _run_check(bt, P, do, meta, inputs)
    bt.close()


@pytest.mark.parametrize("counters", [1, 8])
def test_ragged_dynamic_counter_shards(counters):
    """Dynamic schedules with one tile counter, and with one per XCD on grids
    whose size is a multiple of 8 (including workgroups that move on to other
    XCDs' counters) and on grids that are not; each replayed so the counters'
    self-reset is exercised."""
    ctxs, segs, meta, inputs, do, P = _ragged_out_case(44)
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_GRAPH)
    sharded = set()
    for tile in (256, 1024, 2048, 4096, 8192):
        for bpc in (1, 64):
            bt.set_shape(tile_elems=tile, blocks_per_cu=bpc, dynamic=counters)
            info = bt.info()
            assert info["counters"] == counters and info["flags"] & mg.BATCH_DYNAMIC
            sharded.add(info["grid"] % 8 == 0)
            for _ in range(3):
                _run_check(bt, P, do, meta, inputs)
    bt.set_shape(tile_elems=4096)
    assert bt.info()["counters"] == 0
    bt.close()
    assert sharded == {True, False}


def test_batch_is_a_context_manager():
    c = mg.setup(8380417, 32)
    x = torch.zeros(4096, dtype=torch.uint32, device="cuda")
    with mg.Batch([c], [(0, mg.OP_MUL, "classic", 4000, 0)]) as bt:
        bt.run(mg.pools([None, x, None], [None, x, None], [None, x, None]))
        sync()
        assert bt.info()["ntiles"] >= 1
    assert not bt.h


@pytest.mark.parametrize("tiles", [8, 9, 16, 24])
def test_ragged_dynamic_few_tiles(tiles):
    """A dynamic grid of one workgroup per tile (grid = tile count): eight counters of one tile
    each (8), of two or three (16, 24), and one counter (9, not a multiple of 8); replayed."""
    N = 8380417
    c = mg.setup(N, 32)
    n = tiles * 256 - 5
    g = inp.rng(71, tiles)
    a = g.integers(0, N, size=n + 3, dtype=np.uint64).astype(np.uint32)
    b = g.integers(0, N, size=n + 3, dtype=np.uint64).astype(np.uint32)
    da, db = dev(a), dev(b)
    do = torch.zeros(n + 8, dtype=torch.uint32, device="cuda")
    bt = mg.Batch([c], [(0, mg.OP_MUL, "classic", n, 0)], flags=mg.BATCH_GRAPH)
    bt.set_shape(tile_elems=256, blocks_per_cu=64, dynamic=8)
    info = bt.info()
    assert info["ntiles"] == tiles and info["grid"] == tiles and info["counters"] == 8
    want = orc.mul("classic", 32, N, a[:n], b[:n])
    P = mg.pools([None, da, None], [None, db, None], [None, do, None])
    for _ in range(3):
        do.zero_()
        bt.run(P)
        sync()
        assert np.array_equal(host(do)[:n], want)
        assert not host(do)[n:].any()
    bt.close()


def test_ragged_shape_rejects_bad_values():
    c = mg.setup(8380417, 32)
    bt = mg.Batch([c], [(0, mg.OP_MUL, "classic", 100, 0)])
    for kw in (dict(tile_elems=1000), dict(tile_elems=128), dict(blocks_per_cu=65), dict(tile_elems=1 << 21),
               dict(blocks_per_cu=2, dynamic=2), dict(blocks_per_cu=2, dynamic=4)):
        with pytest.raises(mg.MontError) as e:
            bt.set_shape(**kw)
        assert e.value.code == -1
    bt.close()


# ----------------------------------------------------------- tuner cache


def test_tune_cache_is_read_back(tmp_path, monkeypatch):
    """A shape recorded in $MONT_TUNE_CACHE for this device, library version, width, variant and
    size class is applied without timing; a record for another library version is ignored."""
    import json
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MONT_TUNE_CACHE", str(cache))
    N, w = 8380417, 32
    c = mg.setup(N, w)
    saved = mg.get_launch(mg.OP_MUL, w, "plantard")
    try:
        a, b = operands("plantard", w, N, 1 << 21, inp.rng(86, 1))
        da, db = dev(a), dev(b)
        out = torch.empty_like(da)
        mg.tune_mul(c, da, db, out, variant="plantard")
        recs = [json.loads(l) for l in cache.read_text().splitlines()]
        assert len(recs) == 1
        key = recs[0]["key"]
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        assert key.startswith("%s:v%d:mul:w32:v2:log2n21" % (arch, mg.version()))
        # plant a distinctive shape for the same key, and one for another library version
        planted = {"unroll": 4, "nontemporal": 0, "blocks_per_cu": 8, "block": 256}
        if {k: recs[0][k] for k in planted} == planted:
            planted = {"unroll": 2, "nontemporal": 0, "blocks_per_cu": 16, "block": 64}
        other = key.replace(":v%d:" % mg.version(), ":v%d:" % (mg.version() + 1))
        with open(cache, "a") as f:
            f.write(json.dumps(dict(key=key, ms=0.001, **planted)) + "\n")
            f.write(json.dumps(dict(key=other, ms=0.001, unroll=1, nontemporal=1, blocks_per_cu=4, block=64)) + "\n")
        out.zero_()
        best = mg.tune_mul(c, da, db, out, variant="plantard")
        assert best == planted
        assert mg.get_launch(mg.OP_MUL, w, "plantard") == planted
        assert len(cache.read_text().splitlines()) == 3      # nothing timed, nothing appended
        assert np.array_equal(host(out), orc.mul("plantard", w, N, a, b))
    finally:
        mg.set_launch(mg.OP_MUL, w, "plantard", **saved)


def test_ragged_tune_cache_is_read_back(tmp_path, monkeypatch):
    import json
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MONT_TUNE_CACHE", str(cache))
    ctxs, segs, meta, cur0, cur1 = ragged_case(51, 64, 30_000, [mg.OP_MUL])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, 51)
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    d1 = {w: dev(in1[w]) for w in (16, 32, 64)}
    do = {w: torch.zeros(cur0[w] + 16, dtype=d0[w].dtype, device="cuda") for w in (16, 32, 64)}
    P = mg.pools([d0[16], d0[32], d0[64]], [d1[16], d1[32], d1[64]], [do[16], do[32], do[64]])
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_TUNE)
    bt.run(P)
    sync()
    check_ragged(meta, inputs, {w: host(do[w]) for w in do})
    bt.close()
    recs = [json.loads(l) for l in cache.read_text().splitlines()]
    assert len(recs) == 1 and ":ragged:" in recs[0]["key"]
    planted = {"tile_elems": 2048, "blocks_per_cu": 8, "dynamic": 1, "nontemporal": 0, "block": 64}
    if all(recs[0][k] == v for k, v in planted.items()):
        planted["tile_elems"] = 4096
    with open(cache, "a") as f:
        f.write(json.dumps(dict(key=recs[0]["key"], ms=0.001, **planted)) + "\n")
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_TUNE)
    for w in do:
        do[w].zero_()
    bt.run(P)
    sync()
    info = bt.info()
    bt.close()
    assert info["tile_elems"] == planted["tile_elems"] and info["blocks_per_cu"] == 8 and info["block"] == 64
    assert info["flags"] & mg.BATCH_DYNAMIC and not info["flags"] & mg.BATCH_NONTEMPORAL
    assert info["counters"] == 1
    assert len(cache.read_text().splitlines()) == 2
    check_ragged(meta, inputs, {w: host(do[w]) for w in do})


# ------------------------------------------------------------- environment


def _small_ragged(seed):
    ctxs, segs, meta, cur0, cur1 = ragged_case(seed, 64, 30_000, [mg.OP_MUL])
    in0, in1, inputs = ragged_buffers(meta, cur0, cur1, seed)
    d0 = {w: dev(in0[w]) for w in (16, 32, 64)}
    d1 = {w: dev(in1[w]) for w in (16, 32, 64)}
    do = {w: torch.zeros(cur0[w] + 16, dtype=d0[w].dtype, device="cuda") for w in (16, 32, 64)}
    P = mg.pools([d0[16], d0[32], d0[64]], [d1[16], d1[32], d1[64]], [do[16], do[32], do[64]])
    return ctxs, segs, meta, inputs, do, P


def test_tune_env_off_and_on(tmp_path, monkeypatch, capfd):
    """MONT_TUNE=0 ignores MONT_BATCH_TUNE and mont_tune_mul's sweep; MONT_TUNE=1 tunes a batch
    without the flag; MONT_LOG=info reports the decisions.  Results match the oracle throughout."""
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MONT_TUNE_CACHE", str(cache))
    monkeypatch.setenv("MONT_LOG", "info")
    ctxs, segs, meta, inputs, do, P = _small_ragged(61)
    monkeypatch.setenv("MONT_TUNE", "0")
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_TUNE)
    before = bt.info()
    _run_check(bt, P, do, meta, inputs)
    assert bt.info() == before
    bt.close()
    assert not cache.exists() or cache.read_text() == ""
    # mont_tune_mul keeps the current shape
    N, w = 8380417, 32
    c = mg.setup(N, w)
    saved = mg.get_launch(mg.OP_MUL, w, "classic")
    try:
        a, b = operands("classic", w, N, 1 << 20, inp.rng(62, 1))
        da, db = dev(a), dev(b)
        out = torch.zeros_like(da)
        got = mg.tune_mul(c, da, db, out, variant="classic")
        assert got == saved and mg.get_launch(mg.OP_MUL, w, "classic") == saved
        assert np.array_equal(host(out), orc.mul("classic", w, N, a, b))
        assert not cache.exists() or cache.read_text() == ""
        assert "MONT_TUNE=0" in capfd.readouterr().err
        # switched on: a batch without the flag is tuned, and the decision logged and cached
        monkeypatch.setenv("MONT_TUNE", "1")
        bt = mg.Batch(ctxs, segs, flags=0)
        _run_check(bt, P, do, meta, inputs)
        bt.close()
        assert len(cache.read_text().splitlines()) == 1
        assert "[mont info] ragged tune:" in capfd.readouterr().err
    finally:
        mg.set_launch(mg.OP_MUL, w, "classic", **saved)
