"""Driver of the continuous-batching request loop (mont_serve_* in libmont.so).

The loop itself is native (a service thread in the library).  This module
builds a job stream (Poisson arrivals, mixed products and exponentiations,
log-uniform lengths, each job with its own odd 31- or 62-bit modulus),
replays it against a Server with native-clock arrivals, and summarises the
completions as latency percentiles and throughput.

Host staging: jobs read their operands from pinned host pools at a seeded
offset per job, and write results into pinned result buffers.  Each word-size
class splits its modulus range into POOL_BUCKETS equal intervals (31-bit
moduli: [2^30, 2^31) in steps of 2^24; 62-bit: [2^61, 2^62) in steps of 2^55),
and bucket k has its own operand pools drawn uniform in [0, L_k), L_k the
bucket's lower end: every operand of a job is below its modulus N, and the
operands cover [0, N) except its top N - L_k < 2^24 (2^55) values, i.e. more
than 98 % of the residue range, top half included.  Exponents are uniform
over 64 bits.  With ``distinct_outputs=False`` all jobs of a class share one
result buffer (a sink), which keeps host memory bounded for 10^5-job streams
while still copying every result back.
"""
from __future__ import annotations

import threading

import numpy as np

from . import _lib
from . import inputs as inp

POOL_SLACK = 1 << 16
POOL_BUCKETS = 64
CLASS_BITS = {32: 31, 64: 62}


def bucket_of(N: int, w: int, buckets: int = POOL_BUCKETS) -> int:
    """The operand-pool bucket of a modulus of the 31-bit (w = 32) or 62-bit (w = 64) class."""
    b = CLASS_BITS[w]
    return (N - (1 << (b - 1))) >> (b - 1 - (buckets.bit_length() - 1))


def bucket_floor(k: int, w: int, buckets: int = POOL_BUCKETS) -> int:
    """L_k: the lower end of bucket k's modulus interval, the bound of its operand pools."""
    b = CLASS_BITS[w]
    return (1 << (b - 1)) + (k << (b - 1 - (buckets.bit_length() - 1)))


def _pinned(torch, n, dtype):
    return torch.empty(n, dtype=dtype, pin_memory=True)


class JobStream:
    """Jobs of one stream with their host buffers (kept alive here)."""

    def __init__(self, torch, njobs, seed_rep=0, distinct_outputs=False, hi=None, buckets=POOL_BUCKETS):
        """distinct_outputs: True (every job), False (all jobs write one sink buffer per
        word size) or a collection of job indices that get their own output buffers.
        buckets: operand pools per class (a power of two; 1 = one pool below the class's
        smallest modulus)."""
        wl = inp.ServeWorkload()
        if hi is not None:
            wl.hi = hi
        t, ops, lens, wide, mods, seeds = wl.jobs(rate_per_s=1.0, rep=seed_rep, njobs=njobs)
        self.gaps_unit = t            # arrival times for rate 1 job/s
        self.ops, self.lens, self.wide, self.mods = ops, lens, wide, mods
        self.njobs = njobs
        g = inp.rng(inp.W_SERVE, 100 + seed_rep)
        P = int(wl.hi) + POOL_SLACK
        # pool[w][k] = (a, b): operands of the jobs whose modulus lies in bucket k, uniform below L_k
        self.buckets = buckets
        self.bucket = [bucket_of(int(N), 64 if wd else 32, buckets) for N, wd in zip(mods, wide)]
        self.pool = {}
        for w, tdt, ndt in ((32, torch.uint32, np.uint32), (64, torch.uint64, np.uint64)):
            self.pool[w] = []
            for k in range(buckets):
                L = bucket_floor(k, w, buckets)
                pair = (_pinned(torch, P, tdt), _pinned(torch, P, tdt))
                for t in pair:
                    t.numpy()[:] = g.integers(0, L, size=P, dtype=np.uint64).astype(ndt)
                self.pool[w].append(pair)
        self.exps = _pinned(torch, P, torch.uint64)
        self.exps.numpy()[:] = inp.u64_uniform(g, P)
        offs = (seeds % POOL_SLACK).astype(np.int64)
        self.offs = offs
        self.jobs = (_lib.JobStruct * njobs)()
        self.outs = {}
        own = set(range(njobs)) if distinct_outputs is True else set(distinct_outputs or ())
        if len(own) < njobs:
            self.sink = {32: _pinned(torch, P, torch.uint32), 64: _pinned(torch, P, torch.uint64)}
        # the jobs' own outputs are slices of one pinned arena per word size (64-element aligned)
        own_len = {32: 0, 64: 0}
        for i in own:
            own_len[64 if wide[i] else 32] += (int(lens[i]) + 63) // 64 * 64
        self.arena = {w: _pinned(torch, max(own_len[w], 1), torch.uint32 if w == 32 else torch.uint64)
                      for w in (32, 64)}
        arena_at = {32: 0, 64: 0}
        esz = {32: 4, 64: 8}
        for i in range(njobs):
            w = 64 if wide[i] else 32
            n = int(lens[i])
            o = int(offs[i])
            x, b = self.pool[w][self.bucket[i]]
            in0 = x.data_ptr() + o * esz[w]
            if ops[i] == 0:
                op, in1 = _lib.OP_MUL, b.data_ptr() + o * esz[w]
            else:
                op, in1 = _lib.OP_POW, self.exps.data_ptr() + o * 8
            if i in own:
                out_t = self.arena[w][arena_at[w]:arena_at[w] + n]
                arena_at[w] += (n + 63) // 64 * 64
                self.outs[i] = out_t
                out = out_t.data_ptr()
            else:
                out = self.sink[w].data_ptr()
            j = self.jobs[i]
            j.id, j.N, j.w, j.op, j.n, j.in0, j.in1, j.out = i, mods[i], w, op, n, in0, in1, out

    def pinned_buffers(self):
        """Every pinned host buffer the stream's jobs read or write."""
        bufs = [t for pairs in self.pool.values() for pair in pairs for t in pair] + [self.exps]
        bufs += list(getattr(self, "sink", {}).values()) + list(self.arena.values())
        return bufs

    def declare(self, server):
        """Declares the stream's pinned buffers to the server (kernel staging)."""
        for t in self.pinned_buffers():
            server.host_region(t)

    def elements(self) -> int:
        return int(self.lens.sum())

    def inputs_of(self, i):
        """Host copies of job i's operands (for checking)."""
        w = 64 if self.wide[i] else 32
        n, o = int(self.lens[i]), int(self.offs[i])
        a, b = self.pool[w][self.bucket[i]]
        x = a.numpy()[o:o + n].copy()
        if self.ops[i] == 0:
            return x, b.numpy()[o:o + n].copy()
        return x, self.exps.numpy()[o:o + n].copy()


def replay(server: "_lib.Server", stream: JobStream, arrivals: np.ndarray, poll_ms=20, timeout_s=600.0):
    """Submits the stream at the given arrival times; returns completions (id order)."""
    done = []
    res = {}

    def feeder():
        try:
            res["accepted"] = server.submit_timed(stream.jobs, arrivals)
        except Exception as e:  # reported below
            res["error"] = e

    th = threading.Thread(target=feeder)
    t0 = server.now()
    th.start()
    while True:
        done.extend(server.poll(8192, poll_ms))
        if "error" in res:
            break
        if not th.is_alive() and len(done) >= res.get("accepted", stream.njobs):
            break
        if server.now() - t0 > timeout_s:
            raise TimeoutError("serving replay did not finish in %.0f s" % timeout_s)
    th.join()
    if "error" in res:
        raise res["error"]
    done.sort()
    return done


def summarize(done, nelems: int):
    c = np.array([(d[2], d[3], d[4], d[5]) for d in done])
    status = np.array([d[1] for d in done])
    lat = (c[:, 3] - c[:, 0]) * 1e3
    span = c[:, 3].max() - c[:, 0].min()
    return {
        "jobs": len(done),
        "failed": int(np.count_nonzero(status)),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "p999_ms": round(float(np.percentile(lat, 99.9)), 3),
        "max_ms": round(float(lat.max()), 3),
        "queue_p50_ms": round(float(np.percentile((c[:, 1] - c[:, 0]) * 1e3, 50)), 3),
        "jobs_per_s": round(len(done) / span, 1),
        "Gelem_per_s": round(nelems / span / 1e9, 3),
        "span_s": round(float(span), 3),
    }
