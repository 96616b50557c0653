"""Benchmark of the Montgomery-type modular arithmetic library on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

A step is one Montgomery product (classic REDC, R = 2^64) over the
residue-number-system workload: eight distinct random 60-bit primes, uint64
operands of shape [8][2^25] (limb-major), row i uniform in [0, N_i).  The
headline value is Gmodmul/s with inputs resident in HBM.  The JSON line also
carries the roofline of the product kernel (algorithmic bytes per launch over
its HIP-event duration, against 8 TB/s), the CPU oracle timed on the host
cores, and secondary measurements: the 32-bit variants, the 16-bit workload,
exponentiation, and the ragged batch (one persistent launch vs one launch
per vector).  Everything runs in libmont.so's kernels; the oracle is used only
for the cpu_baseline figure and a sampled correctness check.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--quick", action="store_true", help="headline only (no secondary measurements)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--sections", default=None,
                   help="comma list of secondary measurements to run (default: all unless --quick): "
                        "copy,ceiling,r32,const,offsets,crt,ntt,r16,valu,pow,ragged,serving; opt-in: ntt_lengths "
                        "(every transform length at each width), ragged_fixed (the ragged batch at --ragged-shape)")
    p.add_argument("--ragged-segments", type=int, default=4096)
    p.add_argument("--ragged-shape", default="4096,2,8",
                   help="tile_elems,blocks_per_cu,dynamic of the opt-in ragged_fixed section")
    p.add_argument("--serve-jobs", type=int, default=100_000)
    return p.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("mont_arith.hpp", "mont_kernels.hpp", "mont_dispatch.hpp", "mont_k64.hip"):
        h.update(open(os.path.join(ROOT, "paper_2402_00675_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(launch_units: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if current."""
    path = os.path.join(ROOT, "profiles", "rns64_mul_pmc.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != source_hash() or d.get("units_per_launch") != launch_units:
        return None
    return d.get("hbm_bytes_per_launch")


def timed(fn, torch, steps, warmup):
    """Runs fn warmup + steps times; returns (wall s, HIP-event ms per call)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / steps


# Montgomery products per exponentiation, REDCs in and out included: 4-bit windows
# at w = 32 (14 table + 15 windows x 5 + 2), 2-bit windows at w = 64 (2 + 31 x 3 + 2)
POW_PRODUCTS = {32: 91, 64: 97}


def timed_sec(fn, torch, min_steps=10, warm_ms=30.0, span_ms=20.0):
    """Secondary measurements: calls fn for warm_ms of wall time first (clocks
    ramp up under load; a few calls of a 0.1 ms kernel are not enough), then
    times enough calls to span at least span_ms; returns (None, HIP-event ms per call)."""
    t0 = time.perf_counter()
    k = 0
    while True:
        fn()
        k += 1
        if k % 4 == 0:
            torch.cuda.synchronize()
            if (time.perf_counter() - t0) * 1e3 >= warm_ms:
                break
    per_ms = (time.perf_counter() - t0) * 1e3 / k
    steps = max(min_steps, int(span_ms / max(per_ms, 1e-3)) + 1)
    return None, timed(fn, torch, steps, 0)[1]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(each shard of the work would be independent); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2402_00675_amd as mg
    from paper_2402_00675_amd import inputs as inp

    mg.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    result = {}

    # ------------------------------------------------------------ headline
    wl = inp.RNS64Workload()
    log("generating RNS workload: %d x %d uint64, moduli %s" % (wl.k, wl.n, [hex(m) for m in wl.moduli]))
    a_h, b_h = wl.operands()
    a = torch.from_numpy(a_h).to(dev)
    b = torch.from_numpy(b_h).to(dev)
    out = torch.empty_like(a)
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    units = wl.k * wl.n

    def step():
        mg.mul_rns(ctxs, a, b, out=out)

    wall, ms_launch = timed(step, torch, args.steps, args.warmup)
    ms_step = wall * 1e3 / args.steps
    value = units / (ms_step * 1e-3) / 1e9
    algo_bytes = 24 * units
    achieved = algo_bytes / (ms_launch * 1e-3) / 1e9
    log("rns64 mul: %.3f ms/step (wall), %.3f ms/launch (events), %.1f Gmodmul/s, %.0f GB/s"
        % (ms_step, ms_launch, value, achieved))

    # sampled correctness check of the timed output against the oracle
    out_h = out.cpu().numpy()
    g = np.random.default_rng(1)
    idx = g.integers(0, wl.n, size=4096)
    import oracle as orc
    for i, N in enumerate(wl.moduli):
        want = orc.mul("classic", 64, N, a_h[i, idx], b_h[i, idx])
        if not np.array_equal(out_h[i, idx], want):
            raise SystemExit("bench: output mismatch against the oracle on row %d" % i)

    # per-launch median over 21 launches, each bracketed by its own events (after the timed region)
    per = []
    for _ in range(21):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        e1.record()
        per.append((e0, e1))
    torch.cuda.synchronize()
    ms_median = float(np.median([x.elapsed_time(y) for x, y in per[1:]]))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(units),
                "kernel": "k_map<64,classic,mul> (mont_mul_rns)", "launch": mg.get_launch(mg.OP_MUL, 64, "classic"),
                "bytes_per_unit": 24,
                "units_per_launch": units, "ms_per_launch": round(ms_launch, 4),
                "ms_per_launch_median": round(ms_median, 4)}

    # -------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu:
        import concurrent.futures as cf
        # every core this process may run on, within the CPU share the host grants one GPU's
        # job ($OMP_NUM_THREADS where it is set): both counts are reported
        avail = len(os.sched_getaffinity(0))
        share = int(os.environ.get("OMP_NUM_THREADS") or avail)
        cores = max(1, min(avail, share))
        chunks = [(i, s, min(s + (1 << 22), wl.n)) for i in range(wl.k) for s in range(0, wl.n, 1 << 22)]

        def work(c):
            i, s, e = c
            orc.mul("classic", 64, wl.moduli[i], a_h[i, s:e], b_h[i, s:e])

        # the whole headline workload, five passes (a pass takes well under a second on 16
        # threads); the median pass is reported
        passes = []
        with cf.ThreadPoolExecutor(cores) as ex:
            for _ in range(5):
                t0 = time.perf_counter()
                list(ex.map(work, chunks))
                passes.append(time.perf_counter() - t0)
        dt = float(np.median(passes))
        # one thread over one chunk (2^22 products of row 0)
        t1 = time.perf_counter()
        work(chunks[0])
        dt1 = time.perf_counter() - t1
        n1 = chunks[0][2] - chunks[0][1]
        cpu = {"value": round(units / dt / 1e9, 4), "unit": "Gmodmul/s", "cores": cores, "kind": "oracle",
               "cores_available": avail, "cpu_share": share,
               "sample": "the whole headline workload (8 x 2^25 classic 64-bit products), "
                         "128-bit '%%' oracle, %d threads, median of 5 passes: %.3f s" % (cores, dt),
               "single_thread_value": round(n1 / dt1 / 1e9, 4),
               "single_thread_sample": "2^22 products of row 0, %.3f s" % dt1}
        log("cpu oracle: %.3f Gmodmul/s on %d threads (%.2f s), %.3f Gmodmul/s on one thread"
            % (units / dt / 1e9, cores, dt, n1 / dt1 / 1e9))
    del a, b, out
    torch.cuda.empty_cache()

    if args.sections is not None:
        sections = [x for x in args.sections.split(",") if x]
    else:
        sections = [] if args.quick else list(SECTIONS)
    extra = secondary(torch, mg, inp, args, sections) if sections else {}

    line = {
        "metric": "Gmodmul/s & % HBM peak (64-bit REDC mul); ragged-batch vs per-call speedup",
        "value": round(value, 2),
        "unit": "Gmodmul/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded numpy PCG64)",
        "config": {"workload": "RNS mont_mul: 8 random 60-bit primes, uint64 [8][2^25], classic REDC R=2^64",
                   "elements": units},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if extra:
        line["extra"] = extra
    print(json.dumps(line), flush=True)


def copy_ceiling(torch):
    """Plain streams of known size over 2 GiB arrays: torch's device copy (the
    counter-scaling reference) and the library's 2-read/1-write reference
    kernel (the product kernels' access pattern with no arithmetic)."""
    import paper_2402_00675_amd as mg

    src = torch.empty(1 << 28, dtype=torch.int64, device="cuda:0")
    dst = torch.empty_like(src)
    _, ms = timed_sec(lambda: dst.copy_(src), torch)
    copy = round(2 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1)
    src2 = torch.empty_like(src)
    _, ms = timed_sec(lambda: mg.stream_ref(src, src2, dst), torch)
    ref = round(3 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1)
    log("copy: %.0f GB/s, 2-read/1-write reference: %.0f GB/s" % (copy, ref))
    return {"torch_copy_GBs": copy, "ref_2r1w_GBs": ref}


SECTIONS = ("copy", "ceiling", "r32", "const", "offsets", "crt", "ntt", "r16", "valu", "pow", "ragged", "serving")


def ceiling(torch, mg, inp):
    """The 2-read/1-write stream at equal bytes per launch, 2^24 to 2^29 64-bit RNS products
    (0.4 to 12.9 GB): the XOR reference kernel, the 32-bit classic product over twice as many
    elements and the 64-bit RNS product (8 rows), each timed with HIP events after warm-up.
    Working sets from 0.4 GB (partly held by the 256 MB last-level cache) to 12.9 GB (not)."""
    dev = torch.device("cuda:0")
    wl = inp.RNS64Workload()
    ctxs = [mg.setup(N, 64) for N in wl.moduli]
    c32 = mg.setup(8380417, 32)
    res = {}
    for lg in range(24, 30):
        E = 1 << lg
        row = {"bytes_per_launch": 24 * E}
        # 64-bit RNS product: 8 rows of E/8 residues below 2^59 (every modulus exceeds 2^59)
        a = torch.randint(0, 1 << 59, (8, E // 8), dtype=torch.int64, device=dev).view(torch.uint64)
        b = torch.randint(0, 1 << 59, (8, E // 8), dtype=torch.int64, device=dev).view(torch.uint64)
        o = torch.empty_like(a)
        _, ms = timed_sec(lambda: mg.mul_rns(ctxs, a, b, out=o), torch)
        row["rns64_GB_s"] = round(24 * E / (ms * 1e-3) / 1e9, 1)
        # the XOR reference over the same three buffers
        _, ms = timed_sec(lambda: mg.stream_ref(a, b, o), torch)
        row["xor_ref_GB_s"] = round(24 * E / (ms * 1e-3) / 1e9, 1)
        del a, b, o
        # 32-bit classic product over 2E residues below N = 8380417
        a = torch.randint(0, 8380417, (2 * E,), dtype=torch.int32, device=dev).view(torch.uint32)
        b = torch.randint(0, 8380417, (2 * E,), dtype=torch.int32, device=dev).view(torch.uint32)
        o = torch.empty_like(a)
        _, ms = timed_sec(lambda: mg.mul(c32, a, b, out=o), torch)
        row["r32_classic_GB_s"] = round(24 * E / (ms * 1e-3) / 1e9, 1)
        del a, b, o
        torch.cuda.empty_cache()
        res["E2^%d" % lg] = row
        log("ceiling 2^%d: %s" % (lg, row))
    return res


def secondary(torch, mg, inp, args, sections):
    dev = torch.device("cuda:0")
    ex = {}
    if "copy" in sections:
        ex["hbm_ceiling"] = copy_ceiling(torch)
    if "ceiling" in sections:
        ex["stream_by_size"] = ceiling(torch, mg, inp)

    if "r32" in sections:
        # 32-bit workload: N = 8380417, 2^26 residues, the variants at R = 2^32 (Plantard family 2^64)
        w2 = inp.R32Workload()
        c32 = mg.setup(w2.N, 32)
        r32 = {}
        # every variant runs on the same three buffers (the signed operands are
        # copied into them): where the buffers sit moves the rate by ~4 %
        a32, b32, o32 = (torch.empty(w2.n, dtype=torch.uint32, device=dev) for _ in range(3))
        for signed in (False, True):
            ah, bh = w2.operands(signed)
            dt = torch.int32 if signed else torch.uint32
            a, b, o = a32.view(dt), b32.view(dt), o32.view(dt)
            a32.view(torch.int32).copy_(torch.from_numpy(ah.view(np.int32)))
            b32.view(torch.int32).copy_(torch.from_numpy(bh.view(np.int32)))
            for v in (["signed", "signed_plantard", "signed_plantard_alpha"] if signed else ["classic", "plantard"]):
                _, ms = timed_sec(lambda: mg.mul(c32, a, b, out=o, variant=v), torch)
                gms = w2.n / (ms * 1e-3) / 1e9
                r32[v] = {"Gmodmul_s": round(gms, 1), "GB_s": round(12 * gms, 1),
                          "frac_hbm": round(12 * gms / HBM_PEAK_GBS, 4)}
                log("r32 %s: %.1f Gmodmul/s" % (v, gms))
        del a, b, o, a32, b32, o32
        ex["r32_mul"] = r32

    if "const" in sections:
        # product by a fixed operand (precomputed b N^-1): 32-bit workload, one read + one write per product
        w2 = inp.R32Workload()
        c32 = mg.setup(w2.N, 32)
        cst = {}
        a32, o32 = (torch.empty(w2.n, dtype=torch.uint32, device=dev) for _ in range(2))  # shared, as above
        for signed in (False, True):
            ah, _ = w2.operands(signed)
            dt = torch.int32 if signed else torch.uint32
            a, o = a32.view(dt), o32.view(dt)
            a32.view(torch.int32).copy_(torch.from_numpy(ah.view(np.int32)))
            b = int(ah[12345])
            for v in (["signed", "signed_plantard"] if signed else ["classic", "plantard"]):
                _, ms = timed_sec(lambda: mg.mul_const(c32, a, b, out=o, variant=v), torch)
                gms = w2.n / (ms * 1e-3) / 1e9
                cst[v] = {"Gmodmul_s": round(gms, 1), "GB_s": round(8 * gms, 1),
                          "frac_hbm": round(8 * gms / HBM_PEAK_GBS, 4)}
                log("r32 const %s: %.1f Gmodmul/s" % (v, gms))
        del a, o, a32, o32
        ex["r32_mul_const"] = cst

    if "offsets" in sections:
        # the 32-bit product on slices at element offsets: all aligned, all at one offset
        # (element-wise head, then the 16-byte body), and at different offsets (element-wise)
        w2 = inp.R32Workload()
        c32 = mg.setup(w2.N, 32)
        ah, bh = w2.operands(False)
        n = w2.n - 8
        A = torch.from_numpy(ah[:n]).to(dev)
        B = torch.from_numpy(bh[:n]).to(dev)
        bufs = [torch.zeros(w2.n + 8, dtype=torch.uint32, device=dev) for _ in range(3)]
        want = None
        offs = {}
        for name, (ka, kb, ko) in (("aligned", (0, 0, 0)), ("equal_offset_1", (1, 1, 1)),
                                   ("equal_offset_3", (3, 3, 3)), ("offsets_1_2_3", (1, 2, 3))):
            a, b, o = bufs[0][ka:ka + n], bufs[1][kb:kb + n], bufs[2][ko:ko + n]
            a.copy_(A)
            b.copy_(B)
            _, ms = timed_sec(lambda: mg.mul(c32, a, b, out=o), torch)
            got = o.cpu()
            if want is None:
                want = got
            elif not torch.equal(got, want):
                raise SystemExit("bench: offsets %s results differ from the aligned call" % name)
            gms = n / (ms * 1e-3) / 1e9
            offs[name] = {"Gmodmul_s": round(gms, 1), "GB_s": round(12 * gms, 1),
                          "frac_hbm": round(12 * gms / HBM_PEAK_GBS, 4)}
            log("r32 classic %s: %.1f Gmodmul/s" % (name, gms))
        del bufs, A, B
        ex["r32_mul_offsets"] = offs

    if "crt" in sections:
        # integers from the 64-bit RNS rows: 2^25 elements of 8 residues -> 8-word integers
        wl = inp.RNS64Workload()
        ah, _ = wl.operands()
        r = torch.from_numpy(ah).to(dev)
        ctxs = [mg.setup(N, 64) for N in wl.moduli]
        o = torch.empty((wl.n, wl.k), dtype=torch.uint64, device=dev)
        _, ms = timed_sec(lambda: mg.crt(ctxs, r, out=o), torch)
        ex["crt"] = {"k": wl.k, "elements": wl.n, "ms": round(ms, 3),
                     "Gelem_s": round(wl.n / (ms * 1e-3) / 1e9, 3),
                     "GB_s": round(2 * 8 * wl.k * wl.n / (ms * 1e-3) / 1e9, 1)}
        log("crt: %s" % ex["crt"])
        del r, o

    if "ntt" in sections:
        # 2^18 transforms of length 256 over N = 8380417 (2^26 coefficients, the 32-bit workload's size)
        N, log2n, batch = 8380417, 8, 1 << 18
        n = 1 << log2n
        c32 = mg.setup(N, 32)
        root = next(w for w in (pow(g, (N - 1) // n, N) for g in range(2, 100)) if pow(w, n // 2, N) == N - 1)
        d = torch.from_numpy(inp.uniform_residues(inp.rng(inp.W_R32, 9), N, batch * n, np.uint32)).to(dev)
        d = d.view(batch, n)
        res = {"N": N, "n": n, "batch": batch}
        for v in ("classic", "plantard"):
            _, ms = timed_sec(lambda: mg.ntt(c32, d, root, variant=v), torch)
            res[v] = {"ms": round(ms, 3), "Gcoef_s": round(batch * n / (ms * 1e-3) / 1e9, 1),
                      "Gbutterfly_s": round(batch * n // 2 * log2n / (ms * 1e-3) / 1e9, 1),
                      "GB_s": round(8 * batch * n / (ms * 1e-3) / 1e9, 1)}
            log("ntt %s: %s" % (v, res[v]))
        # the same coefficient count in 2^16 transforms of length 1024 and 2^14 of length 4096
        for lg in (10, 12):
            nl = 1 << lg
            rl = next(w for w in (pow(g, (N - 1) // nl, N) for g in range(2, 100)) if pow(w, nl // 2, N) == N - 1)
            dl = d.view(batch * n // nl, nl)
            for v in ("classic", "plantard"):
                _, ms = timed_sec(lambda: mg.ntt(c32, dl, rl, variant=v), torch)
                res["n%d_%s" % (nl, v)] = {"ms": round(ms, 3), "batch": batch * n // nl,
                                           "Gcoef_s": round(batch * n / (ms * 1e-3) / 1e9, 1),
                                           "GB_s": round(8 * batch * n / (ms * 1e-3) / 1e9, 1)}
                log("ntt n=%d %s: %s" % (nl, v, res["n%d_%s" % (nl, v)]))
        # the same shape over the 16-bit modulus N = 3329 (2^18 transforms of length 256)
        N16 = 3329
        c16 = mg.setup(N16, 16)
        root16 = next(w for w in (pow(g, (N16 - 1) // n, N16) for g in range(2, 100)) if pow(w, n // 2, N16) == N16 - 1)
        d16 = torch.from_numpy(inp.uniform_residues(inp.rng(inp.W_R16, 9), N16, batch * n, np.uint16)).to(dev)
        d16 = d16.view(batch, n)
        for v in ("classic", "plantard"):
            _, ms = timed_sec(lambda: mg.ntt(c16, d16, root16, variant=v), torch)
            res["w16_N3329_" + v] = {"ms": round(ms, 3), "Gcoef_s": round(batch * n / (ms * 1e-3) / 1e9, 1),
                                      "GB_s": round(4 * batch * n / (ms * 1e-3) / 1e9, 1)}
            log("ntt w16 N=3329 %s: %s" % (v, res["w16_N3329_" + v]))
        ex["ntt"] = res
        del d, d16

    if "ntt_lengths" in sections:
        # every transform length over 2^26 coefficients (2^25 at w = 64), both twiddle forms:
        # w = 32 mod 8380417, w = 16 mod 12289, w = 64 mod a 50-bit and a 62-bit prime
        res = {}
        for w, N, logs in ((32, 8380417, range(1, 13)), (16, 12289, range(1, 13)),
                           (64, 1125899906826241, (4, 8, 10, 11, 12)), (64, 4611686018326724609, (8, 10, 12))):
            c = mg.setup(N, w)
            dt = {16: np.uint16, 32: np.uint32, 64: np.uint64}[w]
            count = 1 << (26 if w < 64 else 25)
            d = torch.from_numpy(inp.uniform_residues(inp.rng(inp.W_R32, 11), N, count, dt)).to(dev)
            row = {}
            for lg in logs:
                nl = 1 << lg
                rl = next(r for r in (pow(g, (N - 1) // nl, N) for g in range(2, 1000)) if pow(r, nl // 2, N) == N - 1)
                dl = d.view(count // nl, nl)
                row["n%d" % nl] = {}
                for v in ("classic", "plantard"):
                    _, ms = timed_sec(lambda: mg.ntt(c, dl, rl, variant=v), torch)
                    row["n%d" % nl][v] = {"ms": round(ms, 4), "GB_s": round(2 * count * w / 8 / (ms * 1e-3) / 1e9, 1)}
                log("ntt w=%d N=%d n=%d: %s" % (w, N, nl, row["n%d" % nl]))
            res["w%d_N%d" % (w, N)] = row
            del d
        ex["ntt_lengths"] = res

    if "r16" in sections:
        # 16-bit workload: N = 3329, 2^20 residues + the exhaustive REDC sweep
        w1 = inp.R16Workload()
        c16 = mg.setup(w1.N, 16)
        ah, bh = w1.operands()
        a = torch.from_numpy(ah).to(dev)
        b = torch.from_numpy(bh).to(dev)
        o = torch.empty_like(a)
        _, ms = timed_sec(lambda: mg.mul(c16, a, b, out=o), torch)
        ex["r16_mul"] = {"us": round(ms * 1e3, 2), "Gmodmul_s": round(w1.n / (ms * 1e-3) / 1e9, 1)}
        # per-launch medians, warm and cold (a 512 MB write between launches evicts the
        # 6 MiB working set from every cache level, the 256 MB last-level cache included)
        flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        for name, cold in (("warm", False), ("cold", True)):
            t = []
            for r in range(21):
                if cold:
                    flush.fill_(r + 1)
                torch.cuda._sleep(100_000)   # GPU busy while the host enqueues: the events bracket the kernel only
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                mg.mul(c16, a, b, out=o)
                e1.record()
                torch.cuda.synchronize()
                t.append(e0.elapsed_time(e1))
            ex["r16_mul"][name + "_us_median"] = round(float(np.median(t[1:])) * 1e3, 2)
        # launch floor: the same call over 64 residues (one workgroup), timed the same way
        t = []
        for r in range(21):
            torch.cuda._sleep(100_000)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mg.mul(c16, a[:64], b[:64], out=o[:64])
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        ex["r16_mul"]["floor_64_elements_us_median"] = round(float(np.median(t[1:])) * 1e3, 2)
        del flush
        total = w1.N << 16
        ro = torch.empty(total, dtype=torch.uint16, device=dev)
        _, ms = timed_sec(lambda: mg.redc_range(c16, 0, total, out=ro), torch)
        ex["r16_exhaustive_redc"] = {"T": total, "us": round(ms * 1e3, 1),
                                     "GB_s_written": round(2 * total / (ms * 1e-3) / 1e9, 1)}
        log("r16: mul %s, exhaustive %s" % (ex["r16_mul"], ex["r16_exhaustive_redc"]))
        del a, b, o, ro

    if "valu" in sections:
        # measured issue rates of the integer instructions the reductions are built from
        from paper_2402_00675_amd._lib import VALU_KINDS
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        blocks, iters = cus * 8, 2048
        o = torch.empty(blocks * 256, dtype=torch.int64, device=dev)
        vr = {}
        for kind, name in enumerate(VALU_KINDS):
            _, ms = timed_sec(lambda: mg.valu_ref(kind, iters, blocks, o), torch)
            winst = blocks * 4 * iters * 32          # wave64 instructions
            rate = winst / (ms * 1e-3)
            vr[name] = {"G_wave_instr_s": round(rate / 1e9, 1), "T_lane_ops_s": round(rate * 64 / 1e12, 2),
                        "cycles_per_instr_per_simd_at_2p4GHz": round(cus * 4 * 2.4e9 / rate, 2)}
            log("valu %s: %s" % (name, vr[name]))
        ex["valu_issue"] = vr
        del o

    if "pow" in sections:
        # exponentiation: 2^22 elements, 31- and 62-bit odd moduli, uniform 64-bit exponents
        g = inp.rng(inp.W_SERVE, 7)
        pw = {}
        for bits, w in ((31, 32), (62, 64)):
            N = inp.odd_modulus(g, bits)
            n = 1 << 22
            dt = np.uint32 if w == 32 else np.uint64
            x = torch.from_numpy(inp.uniform_residues(g, N, n, dt)).to(dev)
            e = torch.from_numpy(inp.u64_uniform(g, n)).to(dev)
            o = torch.empty_like(x)
            c = mg.setup(N, w)
            _, ms = timed_sec(lambda: mg.pow(c, x, e, out=o), torch)
            rate = n / (ms * 1e-3) / 1e9
            pw["w%d" % w] = {"Gpow_s": round(rate, 3), "ms": round(ms, 3),
                             "Gmontmul_s": round(rate * POW_PRODUCTS[w], 1)}
            log("pow w%d: %.3f Gpow/s" % (w, rate))
        # the 32-bit workload's modulus N = 8380417 (the same signed ladder as 31-bit moduli)
        N = 8380417
        x = torch.from_numpy(inp.uniform_residues(g, N, n, np.uint32)).to(dev)
        e = torch.from_numpy(inp.u64_uniform(g, n)).to(dev)
        o = torch.empty_like(x)
        c = mg.setup(N, 32)
        _, ms = timed_sec(lambda: mg.pow(c, x, e, out=o), torch)
        rate = n / (ms * 1e-3) / 1e9
        pw["w32_N8380417"] = {"Gpow_s": round(rate, 3), "ms": round(ms, 3), "Gmontmul_s": round(rate * POW_PRODUCTS[32], 1)}
        log("pow w32, N = 8380417: %.3f Gpow/s" % rate)
        ex["pow"] = pw

    if "ragged_fixed" in sections:
        ex["ragged_fixed"] = ragged_fixed(torch, mg, inp, args.ragged_segments,
                                          tuple(int(x) for x in args.ragged_shape.split(",")))
    if "ragged" in sections:
        ex["ragged"] = ragged(torch, mg, inp, args.ragged_segments)
    if "serving" in sections and args.serve_jobs:
        ex["serving"] = serving(torch, mg, args.serve_jobs)
    return ex


def serving(torch, mg, njobs):
    """Poisson stream of jobs through the continuous-batching loop."""
    from paper_2402_00675_amd import serve

    stream = serve.JobStream(torch, njobs)
    nel = stream.elements()
    log("serving: %d jobs, %d elements" % (njobs, nel))
    res_dma = {}
    srv = mg.Server(hbm_budget_bytes=8 << 30, streams=3, max_batch_jobs=512)
    try:
        # staging by DMA copies (buffers not declared): saturation only, for comparison
        res_dma = serve.summarize(serve.replay(srv, stream, np.zeros(njobs)), nel)
        log("serving saturation, DMA staging: %s" % res_dma)
    finally:
        srv.close()
    srv = mg.Server(hbm_budget_bytes=8 << 30, streams=3, max_batch_jobs=512)
    stream.declare(srv)
    try:
        sat = serve.summarize(serve.replay(srv, stream, np.zeros(njobs)), nel)
        log("serving saturation: %s" % sat)
        res = {"jobs": njobs, "elements": nel, "mix": "60% mul / 40% pow (uniform 64-bit e), lengths "
               "log-uniform [2^8, 2^18], odd 31/62-bit moduli", "staging": "copy kernels (declared pinned host "
               "buffers)", "saturation": sat, "saturation_dma_staging": res_dma}
        for f in (0.5, 0.8, 0.95):
            rate = f * sat["jobs_per_s"]
            r = serve.summarize(serve.replay(srv, stream, stream.gaps_unit / rate), nel)
            r["offered_jobs_per_s"] = round(rate, 1)
            res["load_%.2f" % f] = r
            log("serving at %.2f x saturation: %s" % (f, r))
        res["server"] = srv.stats()
    finally:
        srv.close()
    return res


def _mismatch(o32, e32, o64, e64):
    """Count of elements differing from the expected pools, with the first differing index of each."""
    r = {"count": 0}
    for name, o, e in (("w32", o32, e32), ("w64", o64, e64)):
        d = np.flatnonzero(o.cpu().numpy() != e)
        r["count"] += int(d.size)
        if d.size:
            r[name] = {"count": int(d.size), "first": int(d[0]), "last": int(d[-1])}
    return r


def ragged_fixed(torch, mg, inp, nseg, shape):
    """The ragged product batch at one explicit launch shape (tile_elems, blocks_per_cu,
    dynamic), checked once against one launch per vector, then 20 graph-replayed runs: the
    run the ragged kernel's rocprofv3 summaries are taken from."""
    dev = torch.device("cuda:0")
    wl = inp.RaggedWorkload(nseg=nseg)
    lens, wide, mods = wl.segments()
    offs, (a32, b32), (a64, b64) = wl.operands(lens, wide, mods)
    ctxs = [mg.setup(N, 64 if wd else 32) for N, wd in zip(mods, wide)]
    segs = [(i, mg.OP_MUL, "classic", int(n), int(o), int(o)) for i, (n, o) in enumerate(zip(lens, offs))]
    d = {k: torch.from_numpy(v).to(dev) for k, v in (("a32", a32), ("b32", b32), ("a64", a64), ("b64", b64))}
    o32 = torch.zeros_like(d["a32"])
    o64 = torch.zeros_like(d["a64"])
    P = mg.pools([None, d["a32"], d["a64"]], [None, d["b32"], d["b64"]], [None, o32, o64])
    nbytes = 12 * int(sum(n for n, wd in zip(lens, wide) if not wd)) + 24 * int(sum(n for n, wd in zip(lens, wide) if wd))
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_GRAPH)
    bt.run_pervector(P)
    torch.cuda.synchronize()
    o32h, o64h = o32.cpu().numpy(), o64.cpu().numpy()
    o32.zero_()
    o64.zero_()
    tile, bpc, dyn = shape
    bt.set_shape(tile_elems=tile, blocks_per_cu=bpc, dynamic=dyn)
    bt.run(P)
    torch.cuda.synchronize()
    bad = _mismatch(o32, o32h, o64, o64h)
    if bad["count"]:
        raise SystemExit("bench: ragged shape %s results differ from the per-vector launches: %s" % (shape, bad))
    _, ms = timed(lambda: bt.run(P), torch, 20, 5)
    info = bt.info()
    bt.close()
    r = {"shape": {"tile_elems": tile, "blocks_per_cu": bpc, "dynamic": dyn}, "grid": info["grid"],
         "ntiles": info["ntiles"], "bytes": nbytes, "ms": round(ms, 4), "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1)}
    log("ragged fixed shape: %s" % r)
    return r


def ragged(torch, mg, inp, nseg):
    """The ragged batch in one launch, by grid kind, against one launch per vector.

    Every launch shape's output pools are compared in full with those of the
    per-vector launches (themselves checked against the oracle by the tests)."""
    dev = torch.device("cuda:0")
    wl = inp.RaggedWorkload(nseg=nseg)
    lens, wide, mods = wl.segments()
    offs, (a32, b32), (a64, b64) = wl.operands(lens, wide, mods)
    log("ragged: %d segments, %d elements" % (nseg, int(lens.sum())))
    ctxs = [mg.setup(N, 64 if wd else 32) for N, wd in zip(mods, wide)]
    segs = [(i, mg.OP_MUL, "classic", int(n), int(o), int(o)) for i, (n, o) in enumerate(zip(lens, offs))]
    d = {k: torch.from_numpy(v).to(dev) for k, v in (("a32", a32), ("b32", b32), ("a64", a64), ("b64", b64))}
    # zeroed: the padding between vectors is never written, and the pools are compared whole
    o32 = torch.zeros_like(d["a32"])
    o64 = torch.zeros_like(d["a64"])
    P = mg.pools([None, d["a32"], d["a64"]], [None, d["b32"], d["b64"]], [None, o32, o64])
    nbytes = 12 * int(sum(n for n, wd in zip(lens, wide) if not wd)) + 24 * int(sum(n for n, wd in zip(lens, wide) if wd))
    res = {"segments": nseg, "elements": int(lens.sum()), "bytes": nbytes}

    # one launch per vector: the reference results and the baseline time
    bt = mg.Batch(ctxs, segs, flags=mg.BATCH_GRAPH)
    bt.run_pervector(P)
    torch.cuda.synchronize()
    o32h, o64h = o32.cpu().numpy(), o64.cpu().numpy()
    _, ms_pv = timed_sec(lambda: bt.run_pervector(P), torch)
    res["per_vector_launches"] = {"ms": round(ms_pv, 3), "launches": len(segs)}

    def shape_run(name, flags, shape):
        b2 = mg.Batch(ctxs, segs, flags=flags)
        if shape is not None:
            b2.set_shape(**shape)
        o32.zero_()
        o64.zero_()
        b2.run(P)  # the first run tunes when asked
        torch.cuda.synchronize()
        bad = _mismatch(o32, o32h, o64, o64h)
        if bad["count"]:
            raise SystemExit("bench: ragged %s results differ from the per-vector launches: %s" % (name, bad))
        _, ms = timed_sec(lambda: b2.run(P), torch)
        info = b2.info()
        b2.close()
        kind = "one_pass" if not info["blocks_per_cu"] else "persistent_%s" % (
            "dynamic%d" % info["counters"] if info["flags"] & mg.BATCH_DYNAMIC else "static")
        r = {"ms": round(ms, 3), "GB_s": round(nbytes / (ms * 1e-3) / 1e9, 1), "grid_kind": kind,
             "speedup_vs_per_vector": round(ms_pv / ms, 2), "info": info}
        log("ragged %s: %s" % (name, r))
        return r

    # the tuned launch (the tuner picks tile size x grid kind x schedule), then each grid kind
    # at a fixed shape, all replayed from a hipGraph
    res["tuned_graph"] = shape_run("tuned_graph", mg.BATCH_GRAPH | mg.BATCH_TUNE, None)
    for tile, bs in ((2048, 256), (2048, 64), (4096, 256)):
        nm = "one_pass_tile%d_block%d_graph" % (tile, bs)
        res[nm] = shape_run(nm, mg.BATCH_GRAPH, dict(tile_elems=tile, blocks_per_cu=0, dynamic=False, block=bs))
    # persistent grids: static round-robin, and dynamic with one tile counter or one per XCD
    for bpc, tile, dyn in ((2, 8192, 0), (2, 4096, 1), (2, 4096, 8), (2, 8192, 1), (2, 8192, 8), (4, 2048, 8)):
        nm = "persistent_%s_bpc%d_tile%d_block256_graph" % ("dynamic%d" % dyn if dyn else "static", bpc, tile)
        res[nm] = shape_run(nm, mg.BATCH_GRAPH, dict(tile_elems=tile, blocks_per_cu=bpc, dynamic=dyn, block=256))
    res["speedup_vs_per_vector"] = res["tuned_graph"]["speedup_vs_per_vector"]

    # the same per-vector launches replayed from one captured graph (no host launch cost)
    o32.zero_()
    o64.zero_()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run_pervector(P)              # warm, outside the capture
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            bt.run_pervector(P, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    # every replay is checked against the eager results, with eager work between replays
    for _ in range(3):
        o32.zero_()
        o64.zero_()
        g.replay()
        torch.cuda.synchronize()
        bad = _mismatch(o32, o32h, o64, o64h)
        if bad["count"]:
            raise SystemExit("bench: graph-replayed per-vector results differ: %s" % bad)
    _, ms_pg = timed_sec(lambda: g.replay(), torch)
    bad = _mismatch(o32, o32h, o64, o64h)
    if bad["count"]:
        raise SystemExit("bench: graph-replayed per-vector results differ after timing: %s" % bad)
    res["per_vector_graph_replay"] = {"ms": round(ms_pg, 3), "nodes": len(segs)}
    res["speedup_vs_per_vector_graph"] = round(ms_pg / res["tuned_graph"]["ms"], 2)
    del g
    bt.close()
    log("ragged: %s" % {k: v for k, v in res.items() if not isinstance(v, dict)})
    return res


if __name__ == "__main__":
    main()
