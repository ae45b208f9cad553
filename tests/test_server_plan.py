"""The request server's scheduling policy on the CPU: strict FIFO admission
by slots and device-memory budget, fair-share rounds in whole chunks,
completion, cancellation, failure and release, plus randomized invariants."""
import ctypes as C
import os
import subprocess

import pytest
from hypothesis import given, settings, strategies as st

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "helpers", "libplan_harness.so")
QUEUED, RUNNING, DONE, FAILED, CANCELED = range(5)


@pytest.fixture(scope="module")
def lib():
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-Wall",
                           "-I", os.path.join(ROOT, "paper_2503_16955_amd", "csrc"),
                           os.path.join(HERE, "helpers", "plan_harness.cpp"), "-o", LIB])
    L = C.CDLL(LIB)
    L.plan_new.restype = C.c_void_p
    L.plan_new.argtypes = [C.c_uint64, C.c_int, C.c_uint64, C.c_uint32]
    L.plan_free.argtypes = [C.c_void_p]
    L.plan_submit.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_double]
    L.plan_admit.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_uint64), C.c_int]
    L.plan_round.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_int),
                             C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.c_int]
    L.plan_complete.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_uint64), C.c_int]
    L.plan_fail.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.c_double]
    L.plan_cancel.argtypes = [C.c_void_p, C.c_uint64, C.c_double]
    L.plan_release.restype = C.c_longlong
    L.plan_release.argtypes = [C.c_void_p, C.c_uint64]
    L.plan_query.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_int),
                             C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                             C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.plan_used.restype = C.c_uint64
    for f in ("plan_used", "plan_free_slots", "plan_queued", "plan_running"):
        getattr(L, f).argtypes = [C.c_void_p]
    return L


class P:
    def __init__(self, L, budget, slots, round_rays, chunk):
        self.L, self.h = L, L.plan_new(budget, slots, round_rays, chunk)
        self.t = 0.0

    def tick(self):
        self.t += 1.0
        return self.t

    def submit(self, ticket, n, bytes_):
        return bool(self.L.plan_submit(self.h, ticket, n, bytes_, self.tick()))

    def admit(self):
        out = (C.c_uint64 * 4096)()
        n = self.L.plan_admit(self.h, self.tick(), out, 4096)
        return list(out[:n])

    def round(self):
        cap = 65536
        t, s = (C.c_uint64 * cap)(), (C.c_int * cap)()
        f, c = (C.c_uint64 * cap)(), (C.c_uint32 * cap)()
        n = self.L.plan_round(self.h, t, s, f, c, cap)
        return [(t[i], s[i], f[i], c[i]) for i in range(n)]

    def complete(self):
        out = (C.c_uint64 * 4096)()
        n = self.L.plan_complete(self.h, self.tick(), out, 4096)
        return list(out[:n])

    def query(self, ticket):
        st_, sl = C.c_int(), C.c_int()
        sc, co = C.c_uint64(), C.c_uint64()
        ta, td = C.c_double(), C.c_double()
        if not self.L.plan_query(self.h, ticket, C.byref(st_), C.byref(sl), C.byref(sc),
                                 C.byref(co), C.byref(ta), C.byref(td)):
            return None
        return dict(state=st_.value, slot=sl.value, scheduled=sc.value, completed=co.value,
                    t_admit=ta.value, t_done=td.value)

    def run_to_idle(self, limit=100000):
        done = []
        for _ in range(limit):
            self.admit()
            items = self.round()
            if not items:
                return done
            done += self.complete()
        raise AssertionError("did not drain")

    def __del__(self):
        self.L.plan_free(self.h)


def test_fifo_admission_by_budget_and_release(lib):
    p = P(lib, budget=100, slots=8, round_rays=1000, chunk=100)
    for t in (1, 2, 3):
        assert p.submit(t, 300, 40)
    assert p.admit() == [1, 2]               # 40 + 40 fit, the third waits for memory
    assert p.query(3)["state"] == QUEUED
    done = p.run_to_idle()
    assert sorted(done) == [1, 2]
    assert p.admit() == []                   # images of 1 and 2 still held
    assert lib.plan_used(p.h) == 80
    assert lib.plan_release(p.h, 1) == 40
    assert p.admit() == [3]
    assert p.run_to_idle() == [3]


def test_head_of_line_blocks_later_requests(lib):
    p = P(lib, budget=100, slots=8, round_rays=1000, chunk=100)
    assert p.submit(1, 100, 70)
    assert p.submit(2, 100, 60)              # does not fit next to 1
    assert p.submit(3, 100, 10)              # would fit, but is behind 2
    assert p.admit() == [1]
    assert p.admit() == []
    p.run_to_idle()
    lib.plan_release(p.h, 1)
    assert p.admit() == [2, 3]


def test_slot_limit(lib):
    p = P(lib, budget=10**9, slots=2, round_rays=1000, chunk=100)
    for t in range(1, 6):
        p.submit(t, 100, 1)
    assert p.admit() == [1, 2]
    assert lib.plan_free_slots(p.h) == 0
    assert sorted(p.run_to_idle()) == [1, 2, 3, 4, 5]
    assert lib.plan_free_slots(p.h) == 2


def test_fair_share_rounds_in_whole_chunks(lib):
    p = P(lib, budget=10**9, slots=8, round_rays=1000, chunk=100)
    for t, n in ((1, 5000), (2, 150), (3, 10000)):
        p.submit(t, n, 1)
    p.admit()
    items = p.round()
    per = {}
    for t, s, f, c in items:
        assert 0 < c <= 100
        per.setdefault(t, []).append((f, c))
    # share 1000 / 3 = 333 rounded up to 400; request 2 only has 150
    assert sum(c for _, c in per[1]) == 400 and sum(c for _, c in per[3]) == 400
    assert sum(c for _, c in per[2]) == 150
    for t, pieces in per.items():
        pos = 0
        for f, c in pieces:
            assert f == pos
            pos += c
    assert p.complete() == [2]               # the small request is done after one round


def test_ray_ranges_tile_exactly(lib):
    p = P(lib, budget=10**9, slots=4, round_rays=777, chunk=64)
    sizes = {1: 1, 2: 63, 3: 64, 4: 65, 5: 5000, 6: 12345}
    for t, n in sizes.items():
        p.submit(t, n, 1)
    seen = {t: [] for t in sizes}
    for _ in range(10000):
        p.admit()
        items = p.round()
        if not items:
            break
        for t, s, f, c in items:
            seen[t].append((f, c))
        p.complete()
    for t, n in sizes.items():
        cover = sorted(seen[t])
        pos = 0
        for f, c in cover:
            assert f == pos
            pos += c
        assert pos == n
        assert p.query(t)["state"] == DONE


def test_cancel_and_fail(lib):
    p = P(lib, budget=100, slots=1, round_rays=100, chunk=100)
    p.submit(1, 1000, 10)
    p.submit(2, 1000, 10)
    assert p.admit() == [1]
    assert lib.plan_cancel(p.h, 2, 0.0) == 1          # queued: cancelled at once
    assert p.query(2)["state"] == CANCELED
    items = p.round()
    assert lib.plan_cancel(p.h, 1, 0.0) == 1          # running: after the round in flight
    assert p.query(1)["state"] == RUNNING
    assert p.complete() == [1]
    q = p.query(1)
    assert q["state"] == CANCELED and q["completed"] == sum(c for *_, c in items)
    assert p.round() == []
    assert lib.plan_cancel(p.h, 1, 0.0) == 0          # already finished
    assert lib.plan_release(p.h, 1) == 10
    p.submit(3, 10, 50)
    assert p.admit() == [3]
    lib.plan_fail(p.h, 3, 2, 0.0)                     # e.g. allocation failed
    assert p.query(3)["state"] == FAILED
    assert lib.plan_used(p.h) == 0 and lib.plan_free_slots(p.h) == 1


def test_oversized_request_rejected(lib):
    p = P(lib, budget=100, slots=1, round_rays=100, chunk=100)
    assert not p.submit(1, 10, 101)
    assert not p.submit(2, 0, 1)
    assert p.query(1) is None


def test_release_rules(lib):
    p = P(lib, budget=100, slots=1, round_rays=100, chunk=100)
    p.submit(1, 100, 10)
    assert lib.plan_release(p.h, 1) == -1             # queued
    p.admit()
    assert lib.plan_release(p.h, 1) == -1             # running
    p.run_to_idle()
    assert lib.plan_release(p.h, 1) == 10
    assert lib.plan_release(p.h, 1) == -1             # forgotten


@settings(max_examples=60, deadline=None)
@given(st.lists(st.tuples(st.integers(1, 3000), st.integers(1, 60), st.booleans()),
                min_size=1, max_size=25),
       st.integers(1, 4), st.integers(64, 2000))
def test_random_workloads_keep_invariants(lib, reqs, slots, round_rays):
    budget = 100
    p = P(lib, budget=budget, slots=slots, round_rays=round_rays, chunk=64)
    admitted_order = []
    tickets = []
    for i, (n, b, cancel) in enumerate(reqs, start=1):
        assert p.submit(i, n, b)
        tickets.append((i, n, cancel))
    for _ in range(100000):
        admitted_order += p.admit()
        assert lib.plan_used(p.h) <= budget
        assert lib.plan_running(p.h) <= slots
        for t, n, cancel in tickets:
            q = p.query(t)
            if cancel and q and q["state"] == RUNNING and q["completed"] > 0:
                lib.plan_cancel(p.h, t, 0.0)
        items = p.round()
        for t, s, f, c in items:
            q = p.query(t)
            assert q["state"] == RUNNING and q["slot"] == s and c <= 64
        done = p.complete()
        for t in done:
            lib.plan_release(p.h, t)
        if not items and lib.plan_queued(p.h) == 0 and lib.plan_running(p.h) == 0:
            break
    assert admitted_order == sorted(admitted_order)   # strict FIFO
    assert lib.plan_used(p.h) == 0 and lib.plan_free_slots(p.h) == slots
