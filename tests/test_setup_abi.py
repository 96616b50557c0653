"""CPU tests of the C ABI: exported symbols, host-side setup, argument errors.

mont_setup is host code (no device use), so its constants are compared with
the oracle here.  No compute kernel is called.
"""
import ctypes

import numpy as np
import pytest

import oracle as orc
import paper_2402_00675_amd as mg
from paper_2402_00675_amd import _lib

VARS = ["classic", "signed", "plantard", "signed_plantard"]


def test_every_declared_symbol_is_exported():
    lib = mg.load()
    names = mg.header_functions()
    assert "mont_setup" in names and "mont_mul" in names and "mont_batch_run" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_debug_build_exports_the_same_interface():
    """libmont_debug.so (MONT_DEBUG) is a drop-in build of the same header."""
    with mg.library() as dbg:
        missing = [n for n in mg.header_functions() if not hasattr(dbg, n)]
        assert not missing, missing
        assert dbg.mont_version() == _lib._open(_lib.LIB_PATH).mont_version()
    assert mg.load() is not dbg


def test_release_build_has_no_violation_counter():
    with pytest.raises(mg.MontError) as e:
        mg.debug_violations()
    assert e.value.code == -3


def sample_moduli(w, k=60, seed=0):
    g = np.random.default_rng(seed + w)
    top = (1 << w) - 1
    Ns = {3, 5, 7, top if top % 2 else top - 1, (1 << (w - 1)) - 1, (1 << (w - 1)) + 1,
          (1 << (w - 2)) - 1, (1 << (w - 2)) + 1}
    if w == 16:
        Ns |= {3329, 7681, 12289, 40503, 40505}
    if w == 32:
        Ns |= {8380417, 2654435761 | 1}
    hi = min(1 << w, 1 << 63)
    Ns |= {int(x) | 1 for x in g.integers(3, hi, size=k, dtype=np.uint64)}
    return sorted(N for N in Ns if 3 <= N < (1 << w))


@pytest.mark.parametrize("w", [16, 32, 64])
def test_setup_matches_oracle_constants(w):
    for N in sample_moduli(w):
        c = mg.setup(N, w)
        o = orc.constants(N, w)
        s = c.s
        assert s.N == N and s.w == w
        assert s.ninv == o["ninv"]
        assert s.nprime == o["nprime"] % (1 << w)
        assert s.ninv2_lo == o["ninv2"] & (2**64 - 1)
        assert s.ninv2_hi == o["ninv2"] >> 64
        assert s.r_mod_n == o["r_mod_n"] and s.r2_mod_n == o["r2_mod_n"]
        for v in VARS:
            assert c.valid(v) == (v in o["valid"]), (N, w, v)
        # Algorithm 4 defaults to alpha = 1 where N < 2^(w-2)
        assert c.valid("signed_plantard_alpha") == (N < 1 << (w - 2))
        assert s.alpha == (1 if N < 1 << (w - 2) else 0)


def test_setup_rejects_bad_moduli():
    for N, w in [(4, 16), (1, 16), (0, 32), (65537, 16), (1 << 32 | 1, 32), (3329, 8), (3329, 24)]:
        with pytest.raises(mg.MontError) as e:
            mg.setup(N, w)
        assert e.value.code == -1


def test_set_alpha():
    c = mg.setup(1001, 16)
    with pytest.raises(mg.MontError) as e:
        c.set_alpha(0)                     # Example 3.1: alpha = 0 is wrong
    assert e.value.code == -2
    c.set_alpha(4)                         # 1001 < 2^(16-4-1)
    assert c.s.alpha == 4
    c.set_alpha(5)                         # 1001 < 2^10
    with pytest.raises(mg.MontError):
        c.set_alpha(6)                     # 1001 >= 2^9


def test_argument_errors_need_no_device():
    lib = mg.load()
    c = mg.setup(3329, 16)
    # n == 0: nothing launched
    assert lib.mont_mul(ctypes.byref(c.s), None, None, None, 0, 0, None) == 0
    # invalid variant for the modulus (65521 >= 2^16 / phi: Plantard invalid)
    c2 = mg.setup(65521, 16)
    assert lib.mont_mul(ctypes.byref(c2.s), None, None, None, 1, _lib.PLANTARD, None) == -2
    assert lib.mont_mul(ctypes.byref(c.s), None, None, None, 1, 9, None) == -1
    # null pointers with n > 0
    assert lib.mont_mul(ctypes.byref(c.s), None, None, None, 5, 0, None) == -1
    assert b"null" in lib.mont_last_error()
    # uninitialised context
    bad = _lib.CtxStruct()
    assert lib.mont_redc(ctypes.byref(bad), None, None, 4, 0, None) == -1
    # range beyond R N
    assert lib.mont_redc_range(ctypes.byref(c.s), 3329 * 65536 - 5, None, 10, 0, None) == -2
    # RNS row limits
    arr = (_lib.CtxStruct * 1)(c.s)
    assert lib.mont_mul_rns(arr, 0, None, None, None, 1, 1, 0, None) == -1
    assert lib.mont_mul_rns(arr, 1, None, None, None, 5, 4, 0, None) == -1


def test_batch_validation_errors():
    c32 = mg.setup(8380417, 32)
    big = mg.setup((1 << 32) - 5, 32)       # only classic is valid
    with pytest.raises(mg.MontError) as e:
        mg.Batch([c32], [(1, mg.OP_MUL, "classic", 10, 0)])    # bad ctx index
    assert e.value.code == -1
    with pytest.raises(mg.MontError) as e:
        mg.Batch([big], [(0, mg.OP_MUL, "signed", 10, 0)])     # 2N >= R
    assert e.value.code == -2
    with pytest.raises(mg.MontError) as e:
        mg.Batch([c32], [(0, mg.OP_POW, "signed", 10, 0)])     # pow is classic only
    assert e.value.code == -3


def test_noalloc_rejects_oversized_tables_before_device_use():
    """mont_batch_run_noalloc refuses tables larger than its fixed device array with
    MONT_E_INVAL before any device call (the pool addresses are never touched)."""
    c = mg.setup(8380417, 32)
    p = _lib.PoolsStruct()
    for i in range(3):
        p.in0[i] = p.in1[i] = p.out[i] = 0x10000 * (i + 1)
    with pytest.raises(mg.MontError) as e:
        mg.batch_run_noalloc([c], [(0, mg.OP_MUL, "classic", 1 << 30, 0)], p, tile_elems=256)
    assert e.value.code == -1 and "scratch" in str(e.value)
    with pytest.raises(mg.MontError) as e:
        mg.batch_run_noalloc([c], [(0, mg.OP_MUL, "classic", 10, 0)], p, tile_elems=1000)
    assert e.value.code == -1


def test_log_env_reports_errors(monkeypatch, capfd):
    """$MONT_LOG: silent when unset; from level 1 ("error") every returned error's message on stderr."""
    lib = mg.load()
    c = mg.setup(3329, 16)
    monkeypatch.delenv("MONT_LOG", raising=False)
    assert lib.mont_mul(ctypes.byref(c.s), None, None, None, 5, 0, None) == -1
    assert "[mont" not in capfd.readouterr().err
    for level in ("1", "error", "info", "3"):
        monkeypatch.setenv("MONT_LOG", level)
        assert lib.mont_mul(ctypes.byref(c.s), None, None, None, 5, 0, None) == -1
        err = capfd.readouterr().err
        assert "[mont error] error -1:" in err and "null" in err, (level, err)
    monkeypatch.setenv("MONT_LOG", "0")
    assert lib.mont_setup(4, 16, ctypes.byref(_lib.CtxStruct())) == -1
    assert "[mont" not in capfd.readouterr().err
