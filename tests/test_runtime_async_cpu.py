"""The one-call host runtime (runtime.cpp, through its C-ABI) on the CPU
against a fake HIP runtime (helpers/fakehip: every stream is a queue run by
a thread of its own, device memory is host memory).  The trace "kernel"
(helpers/trace_harness.cpp) records the tables its parameter block points
at when it runs.

mrt_trace copies the rocking-curve table and the spectrum to the device
through pinned staging that the stream releases, so with host tables and no
counters requested it returns while its stream is still held shut, the
caller may overwrite its arrays at once, and every kernel reads its own
call's tables (two calls in flight use two staging buffers).  With
counters requested it waits, as the header states."""
import ctypes as C
import os
import subprocess
import threading

import numpy as np
import pytest

from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2503_16955_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("runtime") / "libtrace_harness.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-pthread", "-shared", "-fPIC",
                           "-I", os.path.join(HERE, "helpers", "fakehip"),
                           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                           os.path.join(CSRC, "runtime.cpp"), os.path.join(CSRC, "params.cpp"),
                           os.path.join(HERE, "helpers", "trace_harness.cpp"), "-o", str(out)])
    L = mrt._declare_trace(C.CDLL(str(out)))
    L.harness_stream.restype = C.c_void_p
    L.harness_hold.argtypes = [C.c_void_p]
    L.harness_sync.argtypes = [C.c_void_p]
    L.harness_counts.argtypes = [C.POINTER(C.c_long)] * 3
    L.harness_seen.argtypes = [C.c_int, C.c_void_p, C.c_int]
    L.harness_init()
    return L


def _counts(L):
    v = [C.c_long() for _ in range(3)]
    L.harness_counts(*[C.byref(x) for x in v])
    return [x.value for x in v]


def _small_stress(n_table=4096):
    w = W.get("flat_stress")
    w["detector"] = dict(w["detector"], nx=64, ny=48)
    if n_table != len(w["rocking_curve"]["table"]):
        w["rocking_curve"] = dict(w["rocking_curve"], table=W.darwin_prins_table(n=n_table)[0].tolist())
    return w


class Call:
    """One mrt_trace call's structs and host images (fake device memory)."""

    def __init__(self, w, n=1000, seed=3):
        self.w, self.n, self.seed = w, n, seed
        self.S = mrt.Structs(w)
        px = w["detector"]["nx"] * w["detector"]["ny"]
        self.counts = np.zeros(px, np.uint32)
        self.energy = np.zeros(px, np.uint64)
        self.lut = np.array(w["rocking_curve"]["table"], np.float64)

    def run(self, L, stream, counters=None, entry="mrt_trace"):
        opt = mrt.MrtOptions(precision=1)
        return getattr(L, entry)(*self.S.refs(), 0, self.n, self.seed, C.byref(opt),
                                 self.counts.ctypes.data, self.energy.ctypes.data, None, 0,
                                 C.byref(counters) if counters is not None else None,
                                 C.c_void_p(stream))

    def scribble(self):
        # the caller reuses its arrays as soon as the call has returned
        self.S._table[:] = -1.0


def _call_in_thread(fn, timeout=10.0):
    box = {}
    t = threading.Thread(target=lambda: box.setdefault("rc", fn()), daemon=True)
    t.start()
    t.join(timeout)
    return box.get("rc"), t.is_alive()


def _seen(L, i):
    buf = np.zeros(1 << 14, np.float64)
    k = L.harness_seen(i, buf.ctypes.data, buf.size)
    return buf[:k]


def test_host_tables_do_not_make_the_call_wait(lib):
    L = lib
    s = L.harness_stream()
    runs0 = L.harness_runs()
    a, b = Call(_small_stress()), Call(_small_stress(n_table=1500), n=700)
    waits0, dev0, pinned0 = _counts(L)
    L.harness_hold(s)
    rc, stuck = _call_in_thread(lambda: a.run(L, s))
    if stuck:
        L.harness_open()
    assert not stuck, "mrt_trace waited for its stream"
    assert rc == 0, L.mrt_last_error()
    a.scribble()
    # a second call in flight needs a staging buffer of its own
    rc, stuck = _call_in_thread(lambda: b.run(L, s))
    if stuck:
        L.harness_open()
    assert not stuck and rc == 0
    b.scribble()
    waits1, dev1, pinned1 = _counts(L)
    assert waits1 == waits0, "a host wait happened"
    assert L.harness_runs() == runs0          # nothing ran: the stream is held
    L.harness_open()
    L.harness_sync(s)
    assert L.harness_runs() == runs0 + 2
    for i, c in ((runs0, a), (runs0 + 1, b)):
        seen = _seen(L, i)
        n_lut = len(c.lut)
        assert np.array_equal(seen[:n_lut], c.lut)
        cdf = seen[n_lut:]
        assert len(cdf) == len(c.w["source"]["bin_weights"]) + 1 and cdf[0] == 0.0 and cdf[-1] == 1.0
        assert np.all(np.diff(cdf) >= 0)
    assert pinned1 - pinned0 <= 2   # staging buffers, kept for later calls


def test_staging_is_reused_once_released(lib):
    L = lib
    s = L.harness_stream()
    c = Call(_small_stress())
    assert c.run(L, s) == 0
    L.harness_sync(s)
    _, _, pinned0 = _counts(L)
    for _ in range(5):
        assert c.run(L, s) == 0
        L.harness_sync(s)
    assert _counts(L)[2] == pinned0


def test_counters_make_the_call_wait(lib):
    L = lib
    s = L.harness_stream()
    c = Call(_small_stress(), n=1234)
    cnt = mrt.MrtCounters()
    waits0 = _counts(L)[0]
    assert c.run(L, s, cnt) == 0
    assert _counts(L)[0] > waits0
    # the fake kernel adds n to `events` and the table size to `detected`
    assert cnt.events == 1234 and cnt.detected == len(c.lut) + len(c.w["source"]["bin_weights"]) + 1
    assert cnt.emitted == 1234


def test_noalloc_entry_allocates_nothing(lib):
    """mrt_trace_noalloc takes its counters, cursor and tables from the
    static scratch array: no device or pinned allocation in any call, the
    same scratch for every call, and each kernel reads its own call's
    tables (the second call's smaller table over the first's)."""
    L = lib
    s = L.harness_stream()
    big, small = Call(_small_stress(), n=2000), Call(_small_stress(n_table=900), n=500)
    runs0 = L.harness_runs()
    _, dev0, pinned0 = _counts(L)
    for c in (big, small):
        cnt = mrt.MrtCounters()
        assert c.run(L, s, cnt, entry="mrt_trace_noalloc") == 0, L.mrt_last_error()
        n_tab = len(c.lut) + len(c.w["source"]["bin_weights"]) + 1
        # counters start from zero in each call (the scratch keeps the last)
        assert cnt.events == c.n and cnt.detected == n_tab and cnt.kernel_ms == 0.0
        c.scribble()
    # and without counters: no wait, nothing allocated either (the call's
    # host images stay alive until the stream has run)
    last = Call(_small_stress(n_table=900), n=300)
    assert last.run(L, s, None, entry="mrt_trace_noalloc") == 0
    L.harness_sync(s)
    del last
    _, dev1, pinned1 = _counts(L)
    assert (dev1, pinned1) == (dev0, pinned0)
    assert L.harness_runs() == runs0 + 3
    for i, c in ((runs0, big), (runs0 + 1, small)):
        assert np.array_equal(_seen(L, i)[:len(c.lut)], c.lut)
