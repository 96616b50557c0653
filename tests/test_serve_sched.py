"""The serving scheduler core on the CPU, driven through a recording backend.

The harness (tests/native/sched_sim.cpp) compiles the same header the
library uses (mont_sched.hpp) with g++; the test decides when each launch
slot finishes, so admission order, the device-memory budget, continuous
batching across slots and failure handling are checked deterministically.
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_sim.cpp")
HDR = os.path.join(ROOT, "paper_2402_00675_amd", "csrc", "mont_sched.hpp")
LIB = os.path.join(ROOT, "_build", "libsched_sim_ubsan.so")

OK, E_INVAL, E_DOMAIN, E_DEVICE, E_BUSY, E_CANCELED = 0, -1, -2, -5, -6, -7
MUL, POW = 0, 2
ALIGN = 64


def build(lib_path, sanitize):
    os.makedirs(os.path.dirname(lib_path), exist_ok=True)
    if not os.path.exists(lib_path) or os.path.getmtime(lib_path) < max(os.path.getmtime(SRC),
                                                                          os.path.getmtime(HDR)):
        subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-Wall", "-fno-sanitize-recover=all",
                        "-fsanitize=" + sanitize, "-shared", "-fPIC", "-o", lib_path, SRC], check=True)
    return lib_path


def bind(L):
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.sim_create.restype = vp
    L.sim_create.argtypes = [u64, u64, u32, u32, i32, ctypes.c_double]
    L.sim_advance.argtypes = [vp, ctypes.c_double]
    L.sim_cancel.argtypes = [vp, u64]
    L.sim_fail_next_retire.argtypes = [vp]
    L.sim_finish_retired.argtypes = [vp, i32, i32]
    L.sim_retire_count.argtypes = [vp, i32]
    L.sim_idle.argtypes = [vp]
    L.sim_submit.argtypes = [vp, u64, u64, u32, u32, u64]
    L.sim_step.argtypes = [vp]
    L.sim_finish_slot.argtypes = [vp, i32, i32]
    L.sim_fail_next_launch.argtypes = [vp]
    L.sim_take.restype = ctypes.c_int64
    L.sim_take.argtypes = [vp, vp, vp, u64]
    L.sim_slot_jobs.restype = ctypes.c_int64
    L.sim_slot_jobs.argtypes = [vp, i32, vp, vp, u64]
    L.sim_stats.argtypes = [vp, vp]
    L.sim_destroy.argtypes = [vp]
    return L


@pytest.fixture(scope="module")
def lib():
    return bind(ctypes.CDLL(build(LIB, "undefined")))


class Sim:
    KEYS = ["submitted", "completed", "rejected", "launches", "jobs_launched", "used32", "used64", "peak32",
            "peak64", "queued", "staged", "in_flight", "canceled", "timed_out", "quarantined32", "quarantined64",
            "dead_slots"]

    def __init__(self, L, cap32=4096, cap64=4096, max_in_flight=1000, max_batch=100, slots=2, deadline=0.0):
        self.L = L
        self.h = L.sim_create(cap32, cap64, max_in_flight, max_batch, slots, deadline)

    def submit(self, id_, n, w=32, op=MUL, N=8380417):
        return self.L.sim_submit(self.h, id_, N, w, op, n)

    def step(self):
        return self.L.sim_step(self.h)

    def finish(self, slot, status=1):
        self.L.sim_finish_slot(self.h, slot, status)

    def take(self):
        ids = np.zeros(10000, np.uint64)
        st = np.zeros(10000, np.int32)
        k = self.L.sim_take(self.h, ids.ctypes.data, st.ctypes.data, 10000)
        return dict(zip(ids[:k].tolist(), st[:k].tolist()))

    def slot(self, s):
        ids = np.zeros(10000, np.uint64)
        offs = np.zeros(10000, np.uint64)
        k = self.L.sim_slot_jobs(self.h, s, ids.ctypes.data, offs.ctypes.data, 10000)
        return ids[:k].tolist(), offs[:k].tolist()

    def advance(self, dt):
        self.L.sim_advance(self.h, dt)

    def cancel(self, id_):
        return self.L.sim_cancel(self.h, id_)

    def stats(self):
        v = np.zeros(len(self.KEYS), np.uint64)
        self.L.sim_stats(self.h, v.ctypes.data)
        return dict(zip(self.KEYS, v.tolist()))

    def close(self):
        self.L.sim_destroy(self.h)


def test_fifo_admission_by_budget(lib):
    s = Sim(lib, cap32=1024, slots=1)
    assert s.submit(1, 600) == OK
    assert s.submit(2, 600) == OK      # 640 + 640 slots > 1024: waits
    assert s.submit(3, 10) == OK       # fits, but FIFO keeps it behind job 2
    s.step()
    assert s.slot(0)[0] == [1]
    st = s.stats()
    assert st["used32"] == 640 and st["queued"] == 2 and st["in_flight"] == 1
    s.step()
    assert s.slot(0)[0] == [1] and s.take() == {}   # still running
    s.finish(0)
    s.step()                            # reaps job 1, admits 2 and 3, launches both
    assert s.take() == {1: OK}
    assert s.slot(0)[0] == [2, 3]
    assert s.stats()["used32"] == 640 + 64
    s.finish(0)
    s.step()
    assert s.take() == {2: OK, 3: OK}
    st = s.stats()
    assert st["used32"] == 0 and st["peak32"] == 704 and st["completed"] == 3 and st["launches"] == 2
    s.close()


def test_continuous_batching_across_slots(lib):
    s = Sim(lib, cap32=1 << 20, slots=2)
    for i in range(3):
        s.submit(i, 1000)
    s.step()
    assert s.slot(0)[0] == [0, 1, 2]
    # arrivals while slot 0 runs go to slot 1 at once
    s.submit(10, 500)
    s.submit(11, 500, w=64, N=(1 << 61) - 1)
    s.step()
    assert s.slot(1)[0] == [10, 11]
    # both slots busy: new work waits, admitted (memory reserved) but not launched
    s.submit(20, 100)
    s.step()
    st = s.stats()
    assert st["staged"] == 1 and st["in_flight"] == 6
    s.finish(1)
    s.step()
    assert s.take() == {10: OK, 11: OK}
    assert s.slot(1)[0] == [20]
    s.finish(0)
    s.finish(1)
    s.step()
    assert s.take() == {0: OK, 1: OK, 2: OK, 20: OK}
    s.close()


def test_batch_and_in_flight_limits(lib):
    s = Sim(lib, cap32=1 << 20, max_in_flight=5, max_batch=3, slots=2)
    for i in range(8):
        s.submit(i, 10)
    s.step()
    assert s.slot(0)[0] == [0, 1, 2]
    s.step()
    assert s.slot(1)[0] == [3, 4]           # only 5 may be in flight
    assert s.stats()["queued"] == 3
    s.finish(0)
    s.step()
    assert s.slot(0)[0] == [5, 6, 7]
    s.close()


def test_offsets_disjoint_and_aligned(lib):
    s = Sim(lib, cap32=1 << 16, slots=1, max_batch=1000)
    rng = np.random.default_rng(3)
    lens = rng.integers(1, 2000, size=25)
    for i, n in enumerate(lens):
        s.submit(i, int(n))
    s.step()
    ids, offs = s.slot(0)
    assert ids == list(range(25))
    spans = sorted((o, o + ((int(lens[i]) + ALIGN - 1) // ALIGN) * ALIGN) for i, o in zip(ids, offs))
    assert all(o % ALIGN == 0 for o, _ in spans)
    assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
    s.close()


def test_fragmented_arena_coalesces(lib):
    s = Sim(lib, cap32=64 * 10, slots=1, max_batch=1)
    for i in range(10):
        s.submit(i, 64)
    for k in range(10):
        s.step()
        s.finish(0)
    s.step()
    assert len(s.take()) == 10
    assert s.submit(99, 640) == OK          # needs the whole arena: free blocks merged back
    s.step()
    assert s.slot(0)[0] == [99]
    s.close()


def test_rejections(lib):
    s = Sim(lib, cap32=1024, cap64=128)
    assert s.submit(1, 10, N=100) == E_INVAL                 # even modulus
    assert s.submit(2, 10, N=1) == E_INVAL
    assert s.submit(3, 10, w=16) == E_INVAL                  # the loop serves 32/64-bit words
    assert s.submit(4, 10, op=1) == E_INVAL                  # products and powers only
    assert s.submit(5, 10, w=32, N=(1 << 32) + 1) == E_INVAL
    assert s.submit(6, 2000) == E_DOMAIN                     # larger than the whole budget
    assert s.submit(7, 129, w=64, N=(1 << 61) - 1) == E_DOMAIN
    assert s.submit(8, 0) == OK                              # empty job completes at once
    done = s.take()
    assert done == {1: E_INVAL, 2: E_INVAL, 3: E_INVAL, 4: E_INVAL, 5: E_INVAL, 6: E_DOMAIN, 7: E_DOMAIN, 8: OK}
    st = s.stats()
    assert st["rejected"] == 7 and st["completed"] == 1
    s.close()


def test_launch_and_device_failures_release_memory(lib):
    s = Sim(lib, cap32=4096, slots=1)
    s.submit(1, 100)
    lib.sim_fail_next_launch(s.h)
    s.step()
    assert s.take() == {1: E_DEVICE}
    assert s.stats()["used32"] == 0
    s.submit(2, 100, op=POW)
    s.step()
    s.finish(0, -1)                          # the batch's completion event reported an error
    s.step()
    assert s.take() == {2: E_DEVICE}
    st = s.stats()
    assert st["used32"] == 0 and st["in_flight"] == 0
    s.submit(3, 100)                         # the loop keeps serving
    s.step()
    s.finish(0)
    s.step()
    assert s.take() == {3: OK}
    s.close()


def test_random_workload_accounting(lib):
    """Random arrivals and completions: every job finishes once, memory returns to zero."""
    rng = np.random.default_rng(7)
    s = Sim(lib, cap32=1 << 18, cap64=1 << 17, max_in_flight=64, max_batch=16, slots=3)
    nxt, seen = 0, {}
    for _ in range(3000):
        for _ in range(int(rng.poisson(2))):
            w = 64 if rng.uniform() < 0.5 else 32
            N = (1 << 61) - 1 if w == 64 else 8380417
            s.submit(nxt, int(rng.integers(1, 20000)), w=w, N=N, op=MUL if rng.uniform() < 0.6 else POW)
            nxt += 1
        s.step()
        for sl in range(3):
            if rng.uniform() < 0.3:
                s.finish(sl)
        for k, v in s.take().items():
            assert k not in seen
            seen[k] = v
        st = s.stats()
        assert st["used32"] <= 1 << 18 and st["used64"] <= 1 << 17 and st["in_flight"] <= 64
    for _ in range(10000):
        for sl in range(3):
            s.finish(sl)
        s.step()
        seen.update(s.take())
        if len(seen) == nxt:
            break
    assert len(seen) == nxt and all(v == OK for v in seen.values())
    st = s.stats()
    assert st["used32"] == 0 and st["used64"] == 0 and st["completed"] == nxt
    s.close()


def test_deadline_quarantines_memory_until_the_retired_batch_ends(lib):
    """A batch past its deadline fails at once with E_DEVICE; its slot is renewed; its memory is
    released only when the retired work is seen to end, so no new job is placed under it."""
    s = Sim(lib, cap32=1024, slots=1, deadline=5.0)
    s.submit(1, 512)
    s.step()
    assert s.slot(0)[0] == [1]
    s.advance(3.0)
    s.step()
    assert s.take() == {}                     # within the deadline
    s.advance(3.0)
    s.step()
    assert s.take() == {1: E_DEVICE}
    st = s.stats()
    assert st["timed_out"] == 1 and st["quarantined32"] == 512 and st["used32"] == 512 and st["in_flight"] == 0
    assert lib.sim_retire_count(s.h, 0) == 1
    # the renewed slot serves new work, placed beside the quarantined span
    s.submit(2, 512)
    s.step()
    ids, offs = s.slot(0)
    assert ids == [2] and offs == [512]
    s.submit(3, 100)                          # no room until the retired batch ends
    s.step()
    assert s.stats()["queued"] == 1
    assert lib.sim_finish_retired(s.h, 0, 1) == 0
    s.step()                                  # releases the quarantined span, admits job 3
    st = s.stats()
    assert st["quarantined32"] == 0 and st["used32"] == 512 + 128 and st["staged"] == 1
    s.finish(0)
    s.step()
    s.finish(0)
    s.step()
    assert s.take() == {2: OK, 3: OK}
    assert s.stats()["used32"] == 0
    s.close()


def test_failed_retired_batch_also_releases_memory(lib):
    s = Sim(lib, cap32=4096, slots=2, deadline=1.0)
    s.submit(1, 100)
    s.step()
    s.advance(2.0)
    s.step()
    assert s.take() == {1: E_DEVICE}
    lib.sim_finish_retired(s.h, 0, -1)
    s.step()
    st = s.stats()
    assert st["used32"] == 0 and st["quarantined32"] == 0
    s.close()


def test_slot_that_cannot_be_renewed_leaves_service(lib):
    s = Sim(lib, cap32=4096, slots=2, deadline=1.0)
    s.submit(1, 100)
    s.step()
    lib.sim_fail_next_retire(s.h)
    s.advance(2.0)
    s.step()
    assert s.take() == {1: E_DEVICE} and s.stats()["dead_slots"] == 1
    s.submit(2, 100)                          # served by the other slot
    s.step()
    assert s.slot(1)[0] == [2] and s.slot(0)[0] == [1]
    s.finish(1)
    s.step()
    assert s.take() == {2: OK}
    s.submit(3, 100)
    s.step()
    lib.sim_fail_next_retire(s.h)
    s.advance(2.0)
    s.step()                                  # the last slot dies too
    assert s.take() == {3: E_DEVICE} and s.stats()["dead_slots"] == 2
    assert s.submit(4, 100) == OK
    s.step()
    assert s.take() == {4: E_DEVICE}          # nothing can run any more
    assert s.stats()["used32"] == 256         # the dead slots' memory (two 128-slot spans) stays reserved
    s.close()


def test_cancel_queued_staged_and_launched(lib):
    s = Sim(lib, cap32=1024, slots=1, max_batch=1)
    s.submit(1, 512)
    s.submit(2, 256)
    s.submit(3, 512)                          # does not fit: stays queued
    s.step()                                  # 1 launched, 2 admitted (staged), 3 queued
    st = s.stats()
    assert st["staged"] == 1 and st["queued"] == 1
    assert s.cancel(1) == E_BUSY
    assert s.cancel(3) == OK
    assert s.cancel(2) == OK
    assert s.cancel(2) == E_INVAL and s.cancel(99) == E_INVAL
    assert s.take() == {3: E_CANCELED, 2: E_CANCELED}
    st = s.stats()
    assert st["canceled"] == 2 and st["used32"] == 512 and st["queued"] == 0 and st["staged"] == 0
    s.finish(0)
    s.step()
    assert s.take() == {1: OK}
    assert s.stats()["used32"] == 0 and s.stats()["completed"] == 3
    s.close()


def test_random_workload_with_deadlines_and_cancels(lib):
    """Random arrivals, completions, expiries, retired-batch ends and cancels: every job
    finishes exactly once, and memory (quarantined included) returns to zero."""
    rng = np.random.default_rng(11)
    s = Sim(lib, cap32=1 << 17, cap64=1 << 16, max_in_flight=64, max_batch=16, slots=3, deadline=4.0)
    nxt, seen, tickets = 0, {}, 0
    for _ in range(3000):
        for _ in range(int(rng.poisson(2))):
            w = 64 if rng.uniform() < 0.5 else 32
            s.submit(nxt, int(rng.integers(1, 20000)), w=w, N=(1 << 61) - 1 if w == 64 else 8380417)
            nxt += 1
        if nxt and rng.uniform() < 0.2:
            s.cancel(int(rng.integers(0, nxt)))
        s.advance(1.0)
        s.step()
        for sl in range(3):
            if rng.uniform() < 0.2:
                s.finish(sl)
        for t in range(tickets + 8):
            if rng.uniform() < 0.3:
                lib.sim_finish_retired(s.h, t, 1)
        tickets = int(s.stats()["timed_out"]) + 8
        for k, v in s.take().items():
            assert k not in seen
            seen[k] = v
    for _ in range(10000):
        for sl in range(3):
            s.finish(sl)
        for t in range(tickets + 3000):
            lib.sim_finish_retired(s.h, t, 1)
        s.advance(0.5)
        s.step()
        seen.update(s.take())
        if len(seen) == nxt and s.stats()["quarantined32"] == 0 and s.stats()["quarantined64"] == 0:
            break
    st = s.stats()
    assert len(seen) == nxt and set(seen.values()) <= {OK, E_DEVICE, E_CANCELED}
    assert st["timed_out"] > 0 and st["canceled"] > 0
    assert st["used32"] == 0 and st["used64"] == 0 and st["completed"] == nxt
    s.close()


ASAN_SCRIPT = """
import ctypes, sys
sys.path.insert(0, %r)
import test_serve_sched as t
L = t.bind(ctypes.CDLL(%r))
t.test_random_workload_accounting(L)
t.test_fragmented_arena_coalesces(L)
t.test_launch_and_device_failures_release_memory(L)
t.test_random_workload_with_deadlines_and_cancels(L)
t.test_deadline_quarantines_memory_until_the_retired_batch_ends(L)
t.test_cancel_queued_staged_and_launched(L)
print("asan-ok")
"""


def test_scheduler_under_address_sanitizer():
    """The random workload again, with the core built under AddressSanitizer (host code)."""
    path = build(os.path.join(ROOT, "_build", "libsched_sim_asan.so"), "address,undefined")
    rt = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt):
        pytest.skip("libasan runtime not found")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([sys.executable, "-c", ASAN_SCRIPT % (os.path.join(ROOT, "tests"), path)],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "asan-ok" in r.stdout, r.stderr[-3000:]
