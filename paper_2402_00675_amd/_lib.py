"""ctypes binding of libmont.so (argument marshalling only).

Every operation runs in the library's HIP kernels; this module checks tensor
shapes and dtypes, passes device pointers and the current HIP stream, and
turns status codes into exceptions.  Torch supplies device memory and
streams, nothing else.  If the library has not been built the import fails
loudly: there is no fallback.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmont.so")
LIB_DEBUG_PATH = os.path.join(_HERE, "libmont_debug.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mont.h")

CLASSIC, SIGNED, PLANTARD, SIGNED_PLANTARD, SIGNED_PLANTARD_ALPHA = range(5)
VARIANTS = {"classic": CLASSIC, "signed": SIGNED, "plantard": PLANTARD,
            "signed_plantard": SIGNED_PLANTARD, "signed_plantard_alpha": SIGNED_PLANTARD_ALPHA}
SIGNED_VARIANTS = {SIGNED, SIGNED_PLANTARD, SIGNED_PLANTARD_ALPHA}
OP_MUL, OP_REDC, OP_POW = 0, 1, 2
BATCH_GRAPH, BATCH_DYNAMIC, BATCH_TUNE, BATCH_NONTEMPORAL = 1, 2, 4, 8

STATUS = {0: "MONT_OK", -1: "MONT_E_INVAL", -2: "MONT_E_DOMAIN", -3: "MONT_E_UNSUPPORTED",
          -4: "MONT_E_NOMEM", -5: "MONT_E_DEVICE", -6: "MONT_E_BUSY", -7: "MONT_E_CANCELED"}
E_INVAL, E_DEVICE, E_BUSY, E_CANCELED = -1, -5, -6, -7


class MontError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class CtxStruct(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint64), ("w", ctypes.c_uint32), ("valid", ctypes.c_uint32),
                ("nprime", ctypes.c_uint64), ("ninv", ctypes.c_uint64), ("ninv2_lo", ctypes.c_uint64),
                ("ninv2_hi", ctypes.c_uint64), ("r_mod_n", ctypes.c_uint64), ("r2_mod_n", ctypes.c_uint64),
                ("alpha", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class SegStruct(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_uint32), ("op", ctypes.c_uint16), ("variant", ctypes.c_uint16),
                ("n", ctypes.c_uint64), ("off", ctypes.c_uint64), ("off1", ctypes.c_uint64)]


class PoolsStruct(ctypes.Structure):
    _fields_ = [("in0", ctypes.c_void_p * 3), ("in1", ctypes.c_void_p * 3), ("out", ctypes.c_void_p * 3)]


class BatchInfoStruct(ctypes.Structure):
    _fields_ = [("ntiles", ctypes.c_uint64), ("elements", ctypes.c_uint64), ("tile_elems", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("block", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("pow_tile", ctypes.c_uint32), ("counters", ctypes.c_uint32)]


class BatchShapeStruct(ctypes.Structure):
    _fields_ = [("tile_elems", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32), ("dynamic", ctypes.c_uint32),
                ("nontemporal", ctypes.c_uint32), ("block", ctypes.c_uint32)]


class LaunchStruct(ctypes.Structure):
    _fields_ = [("unroll", ctypes.c_uint32), ("nontemporal", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("block", ctypes.c_uint32)]


_lib = None


_opened = {}


def load():
    """The library every call of this module goes to: libmont.so (built by
    paper_2402_00675_amd.build), or the file named by $MONT_LIBRARY; raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    _lib = _open(os.environ.get("MONT_LIBRARY") or LIB_PATH)
    return _lib


@contextlib.contextmanager
def library(path: str = None):
    """Routes this module's calls to another build of the library inside the
    block, by default libmont_debug.so (MONT_DEBUG precondition counters)."""
    global _lib
    prev = _lib
    _lib = _open(path or LIB_DEBUG_PATH)
    try:
        yield _lib
    finally:
        _lib = prev


def debug_violations(reset: bool = False) -> int:
    """Precondition violations counted by the MONT_DEBUG build since the last reset."""
    c = ctypes.c_uint64(0)
    check(load().mont_debug_violations(ctypes.byref(c), 1 if reset else 0))
    return c.value


def _open(path: str):
    if path in _opened:
        return _opened[path]
    if not os.path.exists(path):
        raise ImportError("%s is not built; run `python -m paper_2402_00675_amd.build`" % path)
    lib = ctypes.CDLL(path)
    vp, u64, u32, i32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "mont_setup": (i32, [u64, u32, P(CtxStruct)]),
        "mont_set_alpha": (i32, [P(CtxStruct), u32]),
        "mont_redc": (i32, [P(CtxStruct), vp, vp, sz, i32, vp]),
        "mont_mul": (i32, [P(CtxStruct), vp, vp, vp, sz, i32, vp]),
        "mont_mul_rns": (i32, [P(CtxStruct), u32, vp, vp, vp, sz, sz, i32, vp]),
        "mont_mul_const": (i32, [P(CtxStruct), vp, u64, vp, sz, i32, vp]),
        "mont_crt": (i32, [P(CtxStruct), u32, vp, sz, sz, vp, vp]),
        "mont_ntt": (i32, [P(CtxStruct), vp, sz, u32, u64, i32, i32, vp]),
        "mont_pow": (i32, [P(CtxStruct), vp, vp, vp, sz, vp]),
        "mont_redc_range": (i32, [P(CtxStruct), u64, vp, sz, i32, vp]),
        "mont_batch_create": (i32, [P(CtxStruct), u32, P(SegStruct), u32, u32, P(vp), vp]),
        "mont_batch_run": (i32, [vp, P(PoolsStruct), vp]),
        "mont_batch_run_pervector": (i32, [vp, P(PoolsStruct), vp]),
        "mont_mul_ragged": (i32, [vp, P(PoolsStruct), vp]),
        "mont_redc_ragged": (i32, [vp, P(PoolsStruct), vp]),
        "mont_pow_ragged": (i32, [vp, P(PoolsStruct), vp]),
        "mont_batch_info": (i32, [vp, P(BatchInfoStruct)]),
        "mont_batch_set_shape": (i32, [vp, P(BatchShapeStruct), vp]),
        "mont_batch_destroy": (None, [vp]),
        "mont_batch_run_noalloc": (i32, [P(CtxStruct), u32, P(SegStruct), u32, P(PoolsStruct), u32, vp]),
        "mont_tune_mul": (i32, [P(CtxStruct), vp, vp, vp, sz, i32, P(LaunchStruct), vp]),
        "mont_set_launch": (i32, [u32, u32, i32, P(LaunchStruct)]),
        "mont_get_launch": (i32, [u32, u32, i32, P(LaunchStruct)]),
        "mont_stream_ref": (i32, [vp, vp, vp, sz, vp]),
        "mont_valu_ref": (i32, [u32, u32, u32, vp, vp]),
        "mont_debug_violations": (i32, [P(u64), i32]),
        "mont_last_error": (ctypes.c_char_p, []),
        "mont_version": (u32, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _opened[path] = lib
    return lib


def version() -> int:
    """mont_version(): the library version (ABI revision in the low 16 bits)."""
    return int(load().mont_version())


def header_functions(path: str = HEADER) -> list:
    """Names of the functions include/mont.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mont_[a-z0-9_]+)\s*\(", text)))


def check(rc: int):
    if rc != 0:
        raise MontError(rc, load().mont_last_error().decode(errors="replace"))


def variant_id(v) -> int:
    return VARIANTS[v] if isinstance(v, str) else int(v)


# ------------------------------------------------------------------ contexts


class Ctx:
    """Per-modulus constants (mont_setup)."""

    def __init__(self, N: int, w: int):
        self.s = CtxStruct()
        check(load().mont_setup(N, w, ctypes.byref(self.s)))

    @property
    def N(self):
        return int(self.s.N)

    @property
    def w(self):
        return int(self.s.w)

    def valid(self, variant) -> bool:
        return bool(self.s.valid >> variant_id(variant) & 1)

    def set_alpha(self, alpha: int):
        check(load().mont_set_alpha(ctypes.byref(self.s), alpha))
        return self

    def as_dict(self):
        return {f: getattr(self.s, f) for f, _ in CtxStruct._fields_}


def setup(N: int, w: int) -> Ctx:
    return Ctx(N, w)


# ------------------------------------------------------------------ tensors

_ELEM_BYTES = {16: 2, 32: 4, 64: 8}


def _torch():
    import torch
    return torch


def _stream(stream):
    """The hipStream_t to enqueue on: the given torch stream, else torch's current one."""
    if stream is None:
        torch = _torch()
        if not torch.cuda.is_available():
            return ctypes.c_void_p(None)  # the library reports the missing device itself
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, what, nbytes_per, n):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() * t.element_size() < nbytes_per * n:
        raise ValueError("%s holds fewer than %d elements" % (what, n))
    return ctypes.c_void_p(t.data_ptr())


def elem_dtype(w: int, variant=CLASSIC):
    torch = _torch()
    s = variant_id(variant) in SIGNED_VARIANTS
    return {16: torch.int16 if s else torch.uint16, 32: torch.int32 if s else torch.uint32,
            64: torch.int64 if s else torch.uint64}[w]


def mul(ctx: Ctx, a, b, out=None, variant="classic", stream=None):
    n = a.numel()
    eb = _ELEM_BYTES[ctx.w]
    if out is None:
        out = _torch().empty(n, dtype=elem_dtype(ctx.w, variant), device=a.device)
    check(load().mont_mul(ctypes.byref(ctx.s), _dev(a, "a", eb, n), _dev(b, "b", eb, n), _dev(out, "out", eb, n),
                          n, variant_id(variant), _stream(stream)))
    return out


def mul_const(ctx: Ctx, a, b: int, out=None, variant="classic", stream=None):
    """out[i] = REDC(a[i] * b) for a fixed operand b (a Python int, negative allowed for signed variants)."""
    n = a.numel()
    eb = _ELEM_BYTES[ctx.w]
    if out is None:
        out = _torch().empty(n, dtype=elem_dtype(ctx.w, variant), device=a.device)
    check(load().mont_mul_const(ctypes.byref(ctx.s), _dev(a, "a", eb, n), b & (2**64 - 1),
                                _dev(out, "out", eb, n), n, variant_id(variant), _stream(stream)))
    return out


def redc(ctx: Ctx, T, n: int | None = None, out=None, variant="classic", stream=None):
    eb = _ELEM_BYTES[ctx.w]
    if n is None:
        n = T.numel() * T.element_size() // (2 * eb)
    if out is None:
        out = _torch().empty(n, dtype=elem_dtype(ctx.w, variant), device=T.device)
    check(load().mont_redc(ctypes.byref(ctx.s), _dev(T, "T", 2 * eb, n), _dev(out, "out", eb, n), n,
                           variant_id(variant), _stream(stream)))
    return out


def mul_rns(ctxs, a, b, out=None, n: int | None = None, variant="classic", stream=None):
    k, ld = a.shape
    n = ld if n is None else n
    eb = _ELEM_BYTES[ctxs[0].w]
    arr = (CtxStruct * k)(*[c.s for c in ctxs])
    if out is None:
        out = _torch().empty_like(a)
    check(load().mont_mul_rns(arr, k, _dev(a, "a", eb, k * ld), _dev(b, "b", eb, k * ld),
                              _dev(out, "out", eb, k * ld), n, ld, variant_id(variant), _stream(stream)))
    return out


def crt(ctxs, res, out=None, n: int | None = None, stream=None):
    """Integers X (k little-endian uint64 words each) from residue rows res[k][ld]."""
    k, ld = res.shape
    n = ld if n is None else n
    arr = (CtxStruct * k)(*[c.s for c in ctxs])
    if out is None:
        out = _torch().empty((n, k), dtype=_torch().uint64, device=res.device)
    check(load().mont_crt(arr, k, _dev(res, "res", 8, k * ld), n, ld, _dev(out, "out", 8 * k, n), _stream(stream)))
    return out


def ntt(ctx: Ctx, data, root: int, inverse=False, variant="classic", stream=None):
    """In-place transform of every row of data [batch][n] (n a power of two, <= 4096)."""
    batch, n = data.shape
    log2n = n.bit_length() - 1
    if 1 << log2n != n:
        raise ValueError("row length must be a power of two")
    check(load().mont_ntt(ctypes.byref(ctx.s), _dev(data, "data", _ELEM_BYTES[ctx.w], batch * n), batch, log2n,
                          root, 1 if inverse else 0, variant_id(variant), _stream(stream)))
    return data


def pow(ctx: Ctx, x, e, out=None, stream=None):  # noqa: A001
    n = x.numel()
    eb = _ELEM_BYTES[ctx.w]
    if out is None:
        out = _torch().empty_like(x)
    check(load().mont_pow(ctypes.byref(ctx.s), _dev(x, "x", eb, n), _dev(e, "e", 8, n), _dev(out, "out", eb, n),
                          n, _stream(stream)))
    return out


def redc_range(ctx: Ctx, T0: int, n: int, out=None, variant="classic", stream=None):
    eb = _ELEM_BYTES[ctx.w]
    if out is None:
        out = _torch().empty(n, dtype=elem_dtype(ctx.w, variant), device="cuda")
    check(load().mont_redc_range(ctypes.byref(ctx.s), T0, _dev(out, "out", eb, n), n, variant_id(variant),
                                 _stream(stream)))
    return out


def stream_ref(a, b, out, stream=None):
    """out = a XOR b (reference 2-read/1-write stream, no arithmetic)."""
    nbytes = a.numel() * a.element_size()
    check(load().mont_stream_ref(_dev(a, "a", 1, nbytes), _dev(b, "b", 1, nbytes), _dev(out, "out", 1, nbytes),
                                 nbytes, _stream(stream)))
    return out


VALU_KINDS = ("v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mul_u32_u24", "v_add_u32",
              "v_lshl_add_u64", "v_cndmask_b32", "v_cmp_le_u64", "v_lshrrev_b64", "v_sub_u32", "v_min_u32",
              "v_mov_b32", "v_and_or_b32", "v_add3_u32", "v_add_co_u32", "v_addc_co_u32", "v_or_b32", "v_and_b32",
              "v_lshlrev_b32", "v_alignbit_b32", "v_cmp_ne_u32", "v_mad_i64_i32")


def valu_ref(kind: int, iters: int, blocks: int, out, stream=None):
    """Issue-rate reference kernel: blocks x 256 lanes x iters x 32 instances of VALU_KINDS[kind]."""
    check(load().mont_valu_ref(kind, iters, blocks, _dev(out, "out", 8, blocks * 256), _stream(stream)))


def set_launch(op: int, w: int, variant, unroll=1, nontemporal=1, blocks_per_cu=0, block=64):
    L = LaunchStruct(unroll, nontemporal, blocks_per_cu, block)
    check(load().mont_set_launch(op, w, variant_id(variant), ctypes.byref(L)))


def get_launch(op: int, w: int, variant="classic"):
    L = LaunchStruct()
    check(load().mont_get_launch(op, w, variant_id(variant), ctypes.byref(L)))
    return {"unroll": L.unroll, "nontemporal": L.nontemporal, "blocks_per_cu": L.blocks_per_cu, "block": L.block}


def tune_mul(ctx: Ctx, a, b, out, variant="classic", stream=None):
    n = a.numel()
    eb = _ELEM_BYTES[ctx.w]
    L = LaunchStruct()
    check(load().mont_tune_mul(ctypes.byref(ctx.s), _dev(a, "a", eb, n), _dev(b, "b", eb, n),
                               _dev(out, "out", eb, n), n, variant_id(variant), ctypes.byref(L), _stream(stream)))
    return {"unroll": L.unroll, "nontemporal": L.nontemporal, "blocks_per_cu": L.blocks_per_cu, "block": L.block}


# ------------------------------------------------------------------- batches


def pools(in0=(None, None, None), in1=(None, None, None), out=(None, None, None)) -> PoolsStruct:
    """Pools by word-size class [16, 32, 64]; entries are CUDA tensors or None."""
    p = PoolsStruct()
    for i in range(3):
        p.in0[i] = in0[i].data_ptr() if in0[i] is not None else None
        p.in1[i] = in1[i].data_ptr() if in1[i] is not None else None
        p.out[i] = out[i].data_ptr() if out[i] is not None else None
    return p


class Batch:
    """A ragged batch (mont_batch_create).

    segs: tuples (ctx index, op, variant, n, off[, off1]); off1 defaults to off.
    """

    def __init__(self, ctxs, segs, flags=0, stream=None):
        arr = (CtxStruct * max(len(ctxs), 1))(*[c.s for c in ctxs])
        sa = (SegStruct * max(len(segs), 1))()
        for i, sg in enumerate(segs):
            ci, op, var, n, off = sg[:5]
            off1 = sg[5] if len(sg) > 5 else off
            sa[i].ctx, sa[i].op, sa[i].variant, sa[i].n, sa[i].off, sa[i].off1 = ci, op, variant_id(var), n, off, off1
        self.h = ctypes.c_void_p()
        check(load().mont_batch_create(arr, len(ctxs), sa, len(segs), flags, ctypes.byref(self.h),
                                       _stream(stream)))

    def run(self, p: PoolsStruct, stream=None):
        check(load().mont_batch_run(self.h, ctypes.byref(p), _stream(stream)))

    def run_pervector(self, p: PoolsStruct, stream=None):
        check(load().mont_batch_run_pervector(self.h, ctypes.byref(p), _stream(stream)))

    def run_op(self, op: int, p: PoolsStruct, stream=None):
        f = {OP_MUL: load().mont_mul_ragged, OP_REDC: load().mont_redc_ragged, OP_POW: load().mont_pow_ragged}[op]
        check(f(self.h, ctypes.byref(p), _stream(stream)))

    def set_shape(self, tile_elems=4096, blocks_per_cu=0, dynamic=False, nontemporal=True, block=256, stream=None):
        """Fixes the launch shape (mont_batch_set_shape): one pass (blocks_per_cu = 0) or a persistent grid.
        dynamic: False (static), True or 8 (a tile counter per XCD), 1 (one tile counter)."""
        dyn = 8 if dynamic is True else int(dynamic)
        sh = BatchShapeStruct(tile_elems, blocks_per_cu, dyn, 1 if nontemporal else 0, block)
        check(load().mont_batch_set_shape(self.h, ctypes.byref(sh), _stream(stream)))

    def info(self):
        i = BatchInfoStruct()
        check(load().mont_batch_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in BatchInfoStruct._fields_}

    def close(self):
        if self.h:
            load().mont_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _seg_array(segs):
    sa = (SegStruct * max(len(segs), 1))()
    for i, sg in enumerate(segs):
        ci, op, var, n, off = sg[:5]
        off1 = sg[5] if len(sg) > 5 else off
        sa[i].ctx, sa[i].op, sa[i].variant, sa[i].n, sa[i].off, sa[i].off1 = ci, op, variant_id(var), n, off, off1
    return sa


def batch_run_noalloc(ctxs, segs, p: PoolsStruct, tile_elems=0, stream=None):
    """mont_batch_run_noalloc: one ragged launch over segs (tuples as for Batch) with no device
    allocation (the tables go to the library's fixed device array)."""
    arr = (CtxStruct * max(len(ctxs), 1))(*[c.s for c in ctxs])
    check(load().mont_batch_run_noalloc(arr, len(ctxs), _seg_array(segs), len(segs), ctypes.byref(p), tile_elems,
                                        _stream(stream)))


def as_numpy_u64(t) -> np.ndarray:
    """Copies a CUDA tensor to host numpy, keeping unsigned dtypes."""
    return t.cpu().numpy()


# ------------------------------------------------------------------- serving


class ServerCfgStruct(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_jobs_in_flight", ctypes.c_uint32),
                ("streams", ctypes.c_uint32), ("max_batch_jobs", ctypes.c_uint32), ("tile_elems", ctypes.c_uint32),
                ("deadline_us", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class JobStruct(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("N", ctypes.c_uint64), ("w", ctypes.c_uint32), ("op", ctypes.c_uint32),
                ("n", ctypes.c_uint64), ("in0", ctypes.c_void_p), ("in1", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class CompletionStruct(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServerStatsStruct(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("submitted", "completed", "rejected", "launches", "jobs_launched",
                                                 "queued", "staged", "in_flight", "bytes_in_use",
                                                 "peak_bytes_in_use", "enqueue_ns", "canceled", "timed_out",
                                                 "quarantined_bytes", "dead_streams", "ctx_uploads", "ctx_hits")]


_SERVE_SIG = {
    "mont_serve_create": (ctypes.c_int32, [ctypes.POINTER(ServerCfgStruct), ctypes.POINTER(ctypes.c_void_p)]),
    "mont_serve_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(JobStruct)]),
    "mont_serve_submit_timed": (ctypes.c_int64, [ctypes.c_void_p, ctypes.POINTER(JobStruct),
                                                 ctypes.POINTER(ctypes.c_double), ctypes.c_uint64]),
    "mont_serve_poll": (ctypes.c_int64, [ctypes.c_void_p, ctypes.POINTER(CompletionStruct), ctypes.c_uint32,
                                         ctypes.c_int32]),
    "mont_serve_drain": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "mont_serve_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ServerStatsStruct)]),
    "mont_serve_now": (ctypes.c_double, []),
    "mont_serve_host_region": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "mont_serve_destroy": (None, [ctypes.c_void_p]),
    "mont_serve_cancel": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64]),
}


def _serve_lib():
    lib = load()
    if not getattr(lib, "_serve_sig_done", False):
        for name, (res, args) in _SERVE_SIG.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        lib._serve_sig_done = True
    return lib


def host_ptr(x) -> int:
    """Address of a host buffer: a numpy array or a CPU (ideally pinned) torch tensor."""
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("host buffers must be contiguous")
        return x.ctypes.data
    if getattr(x, "device", None) is not None and x.device.type == "cpu":
        return x.data_ptr()
    raise TypeError("serving jobs take host buffers (numpy arrays or CPU tensors)")


class Server:
    """The continuous-batching request loop (mont_serve_*)."""

    def __init__(self, hbm_budget_bytes=8 << 30, max_jobs_in_flight=4096, streams=3, max_batch_jobs=512,
                 tile_elems=0, deadline_us=0):
        lib = _serve_lib()
        cfg = ServerCfgStruct(hbm_budget_bytes, max_jobs_in_flight, streams, max_batch_jobs, tile_elems,
                              deadline_us, 0)
        self.h = ctypes.c_void_p()
        check(lib.mont_serve_create(ctypes.byref(cfg), ctypes.byref(self.h)))
        self._keep = {}

    @staticmethod
    def job(id_, N, w, op, n, in0, in1, out) -> JobStruct:
        return JobStruct(id_, N, w, op, n, host_ptr(in0), host_ptr(in1), host_ptr(out))

    def submit(self, id_, N, w, op, in0, in1, out):
        n = len(in0)
        j = self.job(id_, N, w, op, n, in0, in1, out)
        self._keep[id_] = (in0, in1, out)
        check(_serve_lib().mont_serve_submit(self.h, ctypes.byref(j)))

    def host_region(self, t):
        """Declares a pinned CPU tensor's storage as device-mapped host memory for staging kernels."""
        check(_serve_lib().mont_serve_host_region(self.h, ctypes.c_void_p(host_ptr(t)),
                                                  t.numel() * t.element_size()))

    def submit_struct(self, j: JobStruct):
        """Queues a prepared JobStruct (its host buffers are the caller's to keep alive)."""
        check(_serve_lib().mont_serve_submit(self.h, ctypes.byref(j)))

    def submit_timed(self, jobs: "ctypes.Array", arrival_s: np.ndarray) -> int:
        """Blocking: submits jobs[i] at arrival_s[i] seconds from now (call it from a thread)."""
        t = np.ascontiguousarray(arrival_s, dtype=np.float64)
        k = _serve_lib().mont_serve_submit_timed(self.h, jobs, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 len(t))
        if k < 0:
            check(int(k))
        return int(k)

    def poll(self, max_n=4096, wait_ms=0):
        buf = (CompletionStruct * max_n)()
        k = _serve_lib().mont_serve_poll(self.h, buf, max_n, wait_ms)
        if k < 0:
            check(int(k))
        out = []
        for i in range(k):
            c = buf[i]
            self._keep.pop(c.id, None)
            out.append((c.id, c.status, c.t_submit, c.t_admit, c.t_launch, c.t_done))
        return out

    def cancel(self, id_) -> int:
        """mont_serve_cancel: 0 (cancelled), E_BUSY (already launched) or E_INVAL (not waiting)."""
        rc = int(_serve_lib().mont_serve_cancel(self.h, id_))
        if rc not in (0, E_BUSY, E_INVAL):
            check(rc)
        return rc

    def drain(self, timeout_ms=-1):
        check(_serve_lib().mont_serve_drain(self.h, timeout_ms))

    def stats(self):
        s = ServerStatsStruct()
        check(_serve_lib().mont_serve_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStatsStruct._fields_}

    @staticmethod
    def now() -> float:
        return _serve_lib().mont_serve_now()

    def close(self):
        if self.h:
            _serve_lib().mont_serve_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
