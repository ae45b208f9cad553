"""The kernels' device code run on the CPU: the serving kernel's body and the
one-call trace loop (runtime kinds) execute under a SIMT emulator
(helpers/simt_emu.cpp: 64 coroutines per wave that meet at every ballot and
readfirstlane), so their wave-level control flow (lane refill, chunk claims,
drain, counter flushes) runs as written, without a GPU.

Checks: every emulated wave terminates with its lanes in lockstep at each
wave operation; the serving loop, fed a round of items that interleaves ray
ranges of the whole request mix, gives each request exactly the images and
counters of the same request traced alone; the counters balance (every emitted ray
ends in exactly one way).

What the emulation cannot show is how the compiler maps this control flow to
the hardware's exec masks; that is checked on the GPU."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2503_16955_amd import mosaicrt as mrt
from serving_mix import mix

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2503_16955_amd", "csrc")
N_COUNTERS = 10            # device counter words per request (kNumCounters)
SCALE = 0.002              # ray counts of the mix scaled down for the emulator
WAVES = 4
MAX_MEETINGS = 10 ** 9

# The one inline-asm statement of the device math (a v_fma_f64 with a scalar
# operand) becomes the equivalent fused multiply-add on the host.
ASM_FMA = 'asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(z), "s"(c));'


def build_emu(d, extra_flags=()):
    """Compile the emulator with the device sources copied into directory d;
    returns the library's path."""
    for f in ("trace_impl.h", "trace_params.h", "device_math.h", "math_tables.h", "params.h",
              "params.cpp"):
        shutil.copy(os.path.join(CSRC, f), d / f)
    shutil.copy(os.path.join(CSRC, "trace_mwg.hip"), d / "trace_mwg.h")
    dm = (d / "device_math.h").read_text()
    assert dm.count(ASM_FMA) == 1, "device_math.h: the inline asm this test replaces has changed"
    (d / "device_math.h").write_text(dm.replace(ASM_FMA, "r = __builtin_fma(p, z, c);"))
    lib = d / "libsimt_emu.so"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", *extra_flags,
                           "-I", os.path.join(HERE, "helpers", "fakedev"), "-I", str(d),
                           "-I", os.path.join(ROOT, "include"),
                           os.path.join(HERE, "helpers", "simt_emu.cpp"), str(d / "params.cpp"),
                           "-o", str(lib)])
    return lib


def declare(L):
    """Signatures of the emulator's entry points."""
    L.emu_build_params.argtypes = [C.c_void_p] * 7 + [C.c_int, C.c_void_p]
    L.emu_set_run.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32]
    L.emu_trace.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_longlong]
    L.emu_serve.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_int, C.c_int, C.c_longlong]
    L.emu_serve_ext.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_int, C.c_int, C.c_longlong]
    L.emu_serve_defer.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_int, C.c_int,
                                  C.c_longlong, C.c_int]
    L.emu_build_mwg.argtypes = [C.c_void_p] * 3 + [C.c_int] * 3 + [C.c_void_p, C.c_void_p, C.c_int,
                                                                   C.c_int]
    L.emu_trace_mwg.argtypes = [C.c_void_p, C.c_int, C.c_longlong]
    L.emu_set_records.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64]
    return L


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    return declare(C.CDLL(str(build_emu(tmp_path_factory.mktemp("simt")))))


class Job:
    """One request: its parameter block, tables, images and counters in host
    memory (the emulated kernels use them in place)."""

    def __init__(self, L, w, n, seed, rays=None):
        self.S = mrt.Structs(w)
        # user ray arrays: host memory, read in place by the emulated kernel
        self.rays = {k: np.ascontiguousarray(v, np.float64) for k, v in (rays or {}).items()}
        for k, v in self.rays.items():
            setattr(self.S.source, k, v.ctypes.data)
        self.P = (C.c_char * L.emu_params_size())()
        self.tab = np.zeros(1 << 16, np.float64)
        nt = C.c_int()
        r = L.emu_build_params(*[C.cast(x, C.c_void_p) for x in self.S.refs()], C.byref(self.P),
                               self.tab.ctypes.data, len(self.tab), C.byref(nt))
        assert r == 0, r
        self.n_tables = nt.value
        px = w["detector"]["nx"] * w["detector"]["ny"]
        self.counts = np.zeros(px, np.uint32)
        self.energy = np.zeros(px, np.uint64)
        self.cnt = np.zeros(N_COUNTERS + 8, np.uint64)
        L.emu_set_run(self.P, 0, n, seed, 0, self.counts.ctypes.data, self.energy.ctypes.data,
                      self.cnt.ctypes.data, 64, 16)
        self.n = n

    def counters(self):
        names = ("missed", "absorbed", "exit_reflected", "exit_transmitted", "truncated",
                 "detected", "events", "reflections", "records", "refined")
        return dict(zip(names, (int(x) for x in self.cnt[:N_COUNTERS])))


def _jobs():
    out = []
    for w, n, s in mix():
        out.append((w, n if n < 5000 else max(1, int(n * SCALE)), s))
    return out


def _round(served, ragged=False):
    """Slots and items of a round: each request split into two ray ranges,
    the halves of all requests interleaved (the kernel takes any items; the
    server sends one per request).  ragged: chunks that are not multiples of
    the 64-ray batch."""
    ps = len(served[0].P)
    slots = (C.c_char * (ps * len(served)))()
    for i, j in enumerate(served):
        C.memmove(C.addressof(slots) + i * ps, j.P, ps)
    items = [(0, j.n // 2, i) for i, j in enumerate(served)]
    items += [(j.n // 2, j.n - j.n // 2, i) for i, j in enumerate(served)]
    items = [x for x in items if x[1] > 0]
    it = np.zeros(len(items), dtype=[("first", "<u8"), ("count", "<u8"), ("start", "<u8"),
                                     ("slot", "<i4"), ("chunk", "<u4")])
    start = 0
    for k, (f, c, i) in enumerate(items):
        it[k] = (f, c, start, i, (37 + 29 * k) if ragged else 64 * (1 + k % 4))
        start += c
    return slots, it


def served_with_deferral(L, precision, ragged, ext, limit=None):
    """The serving loop with the one-call kernels' deferral of the ended
    rays' detector work (off in the device's serving kernels) over a round
    of the mix (ext: the extended requests) equals each request's one-call
    trace; every index the loop computes is checked on the way."""
    prec = mrt.PRECISION[precision]
    jobs = _ext_jobs() if ext else [(w, n, s, None) for w, n, s in _jobs()]
    jobs = jobs[:limit]
    alone = []
    for w, n, s, r in jobs:
        j = Job(L, w, n, s, rays=r)
        assert L.emu_trace(j.P, WAVES, prec, MAX_MEETINGS) == 0, w["name"]
        alone.append(j)
    served = [Job(L, w, n, s, rays=r) for w, n, s, r in jobs]
    slots, it = _round(served, ragged)
    assert L.emu_serve_defer(slots, it.ctypes.data, len(it), 3 * WAVES, prec, MAX_MEETINGS,
                             1 if ext else 0) == 0
    for a, b, (w, n, s, r) in zip(alone, served, jobs):
        assert np.array_equal(a.counts, b.counts), (w["name"], n)
        assert np.array_equal(a.energy, b.energy), (w["name"], n)
        assert a.counters() == b.counters(), (w["name"], n)
    return alone


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
@pytest.mark.parametrize("ragged", [False, True])
@pytest.mark.parametrize("ext", [False, True])
def test_served_mix_with_deferred_detector_work(emu, precision, ragged, ext):
    """Every wave stays in lockstep, every index is in bounds, and each
    request equals its one-call trace, over requests with different
    detector sizes, also with ragged chunks."""
    alone = served_with_deferral(emu, precision, ragged, ext)
    assert ext or len({j.counts.size for j in alone}) > 1


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_served_mix_equals_requests_alone(emu, precision):
    prec = mrt.PRECISION[precision]
    jobs = _jobs()
    alone = []
    for w, n, s in jobs:
        j = Job(emu, w, n, s)
        assert emu.emu_trace(j.P, WAVES, prec, MAX_MEETINGS) == 0, w["name"]
        c = j.counters()
        ended = (c["missed"] + c["absorbed"] + c["exit_reflected"] + c["exit_transmitted"]
                 + c["truncated"])
        assert ended == n, (w["name"], c)
        assert c["detected"] <= c["exit_reflected"] + c["exit_transmitted"]
        alone.append(j)

    served = [Job(emu, w, n, s) for w, n, s in jobs]
    ps = len(served[0].P)
    slots = (C.c_char * (ps * len(served)))()
    for i, j in enumerate(served):
        C.memmove(C.addressof(slots) + i * ps, j.P, ps)
    # a round of items: each request split into two ray ranges, the halves
    # of all requests interleaved (the kernel takes any items; the server
    # sends one per request)
    items = []
    for i, j in enumerate(served):
        items.append((0, j.n // 2, i))
    for i, j in enumerate(served):
        items.append((j.n // 2, j.n - j.n // 2, i))
    items = [x for x in items if x[1] > 0]
    it = np.zeros(len(items), dtype=[("first", "<u8"), ("count", "<u8"), ("start", "<u8"),
                                     ("slot", "<i4"), ("chunk", "<u4")])
    start = 0
    for k, (f, c, i) in enumerate(items):
        it[k] = (f, c, start, i, 64 * (1 + k % 4))
        start += c
    assert emu.emu_serve(slots, it.ctypes.data, len(it), 3 * WAVES, prec, MAX_MEETINGS) == 0

    for a, b, (w, n, s) in zip(alone, served, jobs):
        assert np.array_equal(a.counts, b.counts), (w["name"], n)
        assert np.array_equal(a.energy, b.energy), (w["name"], n)
        assert a.counters() == b.counters(), (w["name"], n)


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_schedule_does_not_change_results(emu, precision):
    """The wave's schedule (idle lanes that trigger a refill, chunk size,
    number of waves) decides which lanes and which batches of candidate rays
    carry each ray, never its result: images and counters are identical for
    refill thresholds 1..64 and chunks that are not multiples of the 64-ray
    batch (ragged batches at every chunk end)."""
    prec = mrt.PRECISION[precision]
    for w, n, s in _jobs()[:6]:
        ref = None
        for chunk, refill, waves in ((64, 16, WAVES), (100, 1, 3), (37, 4, 5), (2048, 64, 2),
                                     (130, 63, WAVES)):
            j = Job(emu, w, n, s)
            emu.emu_set_run(j.P, 0, n, s, 0, j.counts.ctypes.data, j.energy.ctypes.data,
                            j.cnt.ctypes.data, chunk, refill)
            assert emu.emu_trace(j.P, waves, prec, MAX_MEETINGS) == 0, (w["name"], chunk, refill)
            got = (j.counts.copy(), j.energy.copy(), j.counters())
            if ref is None:
                ref = got
                continue
            assert np.array_equal(ref[0], got[0]), (w["name"], chunk, refill)
            assert np.array_equal(ref[1], got[1]), (w["name"], chunk, refill)
            assert ref[2] == got[2], (w["name"], chunk, refill)


@pytest.mark.parametrize("name,n,burn", [("flat_hopg", 4000, 300), ("von_hamos_hapg", 6000, 200),
                                          ("flat_stress", 1500, 100)])
def test_mwg_loop_matches_the_oracle_ray_for_ray(emu, name, n, burn):
    """The paper's event model: the device loop (event step with the psi
    quadrature, parked lanes and batched sampler, queue refill) run under the
    emulator gives every ray the oracle's status, event and reflection
    counts and pixel, and its end point and direction within 1e-12."""
    import oracle
    from paper_2503_16955_amd import workloads as W
    w = W.get(name)
    w["event_model"] = {"kind": "mwg", "burn_in": burn, "psi_nodes": 256}
    seed = w["seed"]
    j = Job(emu, w, n, seed)
    refs = [C.cast(x, C.c_void_p) for x in j.S.refs()]
    assert emu.emu_build_mwg(refs[1], refs[2], refs[3], burn, 256, 16, C.byref(j.P),
                             j.tab.ctypes.data, len(j.tab), j.n_tables) == 0
    rec = np.zeros(n, mrt.RECORD_DTYPE)
    emu.emu_set_records(j.P, rec.ctypes.data, n)
    assert emu.emu_trace_mwg(j.P, WAVES, MAX_MEETINGS) == 0
    o = oracle.trace(w, n=n, seed=seed, records=True)
    orec = o["records"]
    for f in ("ray_id", "status", "n_events", "n_refl", "detected", "pix_i", "pix_j"):
        assert np.array_equal(rec[f], orec[f]), f
    for f in ("energy", "end", "dir"):
        a, b = rec[f], orec[f]
        ok = np.isnan(a) & np.isnan(b) | (np.abs(a - b) <= 1e-12 * np.maximum(np.maximum(np.abs(a), np.abs(b)), 1.0))
        assert ok.all(), f
    assert np.array_equal(j.counts, o["counts"].ravel())
    c = j.counters()
    assert c["reflections"] == int(orec["n_refl"].sum()) > 0
    assert c["events"] == int(orec["n_events"].sum())


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_energy_dependent_rocking_curve_loop(emu, precision):
    """The kernel for rocking curves whose shift and width depend on the
    photon energy, run under the emulator: in FP64 every ray matches the
    oracle; in FP32-mixed with constant tables (shift as given, scale 1) the
    images and counters equal those of the plain kernel."""
    import copy
    import oracle
    from paper_2503_16955_amd import workloads as W
    w = W.get("flat_hopg")
    w["rocking_curve"]["energy_dependence"] = [(7.9, -20e-6, 0.7), (8.0, 5e-6, 1.3), (8.1, 30e-6, 2.0)]
    n, seed = 6000, 3
    j = Job(emu, w, n, seed)
    prec = mrt.PRECISION[precision]
    if precision == "fp64":
        rec = np.zeros(n, mrt.RECORD_DTYPE)
        emu.emu_set_records(j.P, rec.ctypes.data, n)
        assert emu.emu_trace(j.P, WAVES, prec, MAX_MEETINGS) == 0
        o = oracle.trace(w, n=n, seed=seed, records=True)["records"]
        for f in ("ray_id", "status", "n_events", "n_refl", "detected", "pix_i", "pix_j"):
            assert np.array_equal(rec[f], o[f]), f
        assert int(rec["n_refl"].sum()) > 20
    else:
        w0 = copy.deepcopy(w)
        w0["rocking_curve"]["energy_dependence"] = [(7.0, w["rocking_curve"]["shift"], 1.0),
                                                    (9.0, w["rocking_curve"]["shift"], 1.0)]
        w0["rocking_curve"].pop("energy_dependence_", None)
        a = Job(emu, w0, n, seed)
        assert emu.emu_trace(a.P, WAVES, prec, MAX_MEETINGS) == 0
        plain = copy.deepcopy(w)
        plain["rocking_curve"].pop("energy_dependence")
        b = Job(emu, plain, n, seed)
        assert emu.emu_trace(b.P, WAVES, prec, MAX_MEETINGS) == 0
        assert np.array_equal(a.counts, b.counts) and a.counters() == b.counters()


def _assert_records_match(rec, o):
    for f in ("ray_id", "status", "n_events", "n_refl", "detected", "pix_i", "pix_j"):
        assert np.array_equal(rec[f], o[f]), f
    for f in ("energy", "entry", "end", "dir"):
        a, b = rec[f], o[f]
        ok = np.isnan(a) & np.isnan(b) | (np.abs(a - b) <= 1e-12 * np.maximum(np.maximum(np.abs(a), np.abs(b)), 1.0))
        assert ok.all(), f


def _user_rays(w, n, seed):
    """Origins scattered about the source point, directions of the oracle's
    own cone tilted a little, energies over the spectrum's range."""
    import oracle
    rng = np.random.default_rng(seed)
    _, k, _ = oracle.source_sample(w, np.arange(n))
    o = np.array(w["source"]["origin"]) + rng.normal(0, 0.02, (n, 3))
    k = k + rng.normal(0, 1e-3, (n, 3))
    k /= np.linalg.norm(k, axis=1)[:, None]
    e = rng.uniform(w["source"]["e_min"], w["source"]["e_max"], n)
    return dict(origins=o, directions=k, energies=e)


@pytest.mark.parametrize("case", ["gaussian_spot", "disk_spot", "user_rays", "user_energies",
                                  "mwg_spot", "mwg_user_rays", "mwg_polarised",
                                  "mwg_polarised_oblique", "mwg_planes", "mwg_planes_polarised",
                                  "mwg_energy_dependent"])
def test_source_spot_and_user_ray_loops(emu, case):
    """The extended-input kernels (FP64) run under the emulator with a source
    spot or user ray arrays: every ray matches the oracle's record; the
    paper's event model takes the same source."""
    import copy
    import oracle
    from paper_2503_16955_amd import workloads as W
    w = W.get("von_hamos_hapg")
    n, seed = 4000, 9
    rays = None
    if case in ("gaussian_spot", "mwg_spot"):
        w["source"]["spot"] = dict(kind="gaussian", u=[0.0, 1.0, 0.0], v=[0.0, 0.0, 1.0],
                                   sigma=[0.02, 0.05])
    elif case == "disk_spot":
        w["source"]["spot"] = dict(kind="disk", u=[0.0, 1.0, 0.0], v=[0.0, 0.0, 1.0], sigma=[0.04])
    elif case == "user_energies":
        rays = {"energies": _user_rays(w, n, seed)["energies"]}
    elif case == "mwg_polarised":
        _, k, _ = oracle.source_sample(w, np.arange(n), seed=seed)
        rays = {"polarisations": _random_polarisations(k, 2)}
    elif case == "mwg_energy_dependent":
        w["rocking_curve"]["energy_dependence"] = [(7.9, -20e-6, 0.7), (8.05, 5e-6, 1.6)]
    elif case in ("mwg_planes", "mwg_planes_polarised"):
        # H-bar at 0.6 and a second order, with a line at twice the energy
        w["crystal"]["planes"] = {"hbar_ratio": 0.6,
                                  "extra": [(w["crystal"]["two_d"] / 2, 0.7, 1.4, 4e-6)]}
        w["source"]["lines"] = list(w["source"]["lines"]) + [(2 * 8.048, 0.004, 0.4)]
        if case == "mwg_planes_polarised":
            _, k, _ = oracle.source_sample(w, np.arange(n), seed=seed)
            rays = {"polarisations": _random_polarisations(k, 4)}
    elif case == "mwg_polarised_oblique":
        # unit vectors with a component along k: only the normal part counts
        a = np.random.default_rng(3).normal(size=(n, 3))
        rays = {"polarisations": a / np.linalg.norm(a, axis=1)[:, None]}
    else:
        rays = _user_rays(w, n, seed)
    mwg = case.startswith("mwg")
    j = Job(emu, w, n, seed, rays=rays)
    if mwg:
        w = copy.deepcopy(w)
        w["event_model"] = {"kind": "mwg", "burn_in": 50, "psi_nodes": 64}
        refs = [C.cast(x, C.c_void_p) for x in j.S.refs()]
        assert emu.emu_build_mwg(refs[1], refs[2], refs[3], 50, 64, 32, C.byref(j.P),
                                 j.tab.ctypes.data, len(j.tab), j.n_tables) == 0
    rec = np.zeros(n, mrt.RECORD_DTYPE)
    emu.emu_set_records(j.P, rec.ctypes.data, n)
    if mwg:
        assert emu.emu_trace_mwg(j.P, WAVES, MAX_MEETINGS) == 0
    else:
        assert emu.emu_trace(j.P, WAVES, mrt.PRECISION["fp64"], MAX_MEETINGS) == 0
    o = oracle.trace(w, n=n, seed=seed, records=True, rays=rays)
    _assert_records_match(rec, o["records"])
    assert np.array_equal(j.counts, o["counts"].ravel())
    assert int(rec["n_refl"].sum()) > 20


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_reflecting_planes_loop(emu, precision):
    """The extended-input kernel with an antiparallel-plane ratio and a second
    order, under the emulator: in FP64 every ray matches the oracle; in
    FP32-mixed (every plane decision in FP64) the counters agree with FP64
    within counting statistics."""
    import oracle
    from paper_2503_16955_amd import workloads as W
    w = W.get("von_hamos_hapg")
    td = w["crystal"]["two_d"]
    w["crystal"]["planes"] = {"hbar_ratio": 0.4, "extra": [(td / 2, 0.6, 1.5, 5e-6)]}
    # a line at twice the Cu K-alpha-like energy, which the second order
    # reflects onto the same detector region
    w["source"]["lines"] = list(w["source"]["lines"]) + [(2 * 8.048, 0.004, 0.4)]
    n, seed = 5000, 4
    j = Job(emu, w, n, seed)
    if precision == "fp64":
        rec = np.zeros(n, mrt.RECORD_DTYPE)
        emu.emu_set_records(j.P, rec.ctypes.data, n)
        assert emu.emu_trace(j.P, WAVES, mrt.PRECISION["fp64"], MAX_MEETINGS) == 0
        o = oracle.trace(w, n=n, seed=seed, records=True)
        _assert_records_match(rec, o["records"])
        assert np.array_equal(j.counts, o["counts"].ravel())
        assert int(rec["n_refl"].sum()) > 20
    else:
        assert emu.emu_trace(j.P, WAVES, mrt.PRECISION["fp32_mixed"], MAX_MEETINGS) == 0
        o = oracle.trace(w, n=n, seed=seed)["counters"]
        c = j.counters()
        for f in ("reflections", "absorbed"):
            assert abs(c[f] - o[f]) < 5 * np.sqrt(c[f] + o[f]) + 5, (f, c[f], o[f])


def _random_polarisations(k, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=k.shape)
    a -= np.sum(a * k, axis=1)[:, None] * k
    return a / np.linalg.norm(a, axis=1)[:, None]


@pytest.mark.parametrize("case", ["von_hamos", "flat_planes", "box", "energy_dependent", "table",
                                  "fp32_mixed"])
def test_polarisation_loop(emu, case):
    """The extended-input kernel with user polarisations (and, on the flat
    crystal, further planes), under the emulator: in FP64 every ray matches
    the oracle; in FP32-mixed the counters agree within statistics."""
    import oracle
    from paper_2503_16955_amd import workloads as W
    w = W.get("flat_hopg" if case == "flat_planes" else "von_hamos_hapg")
    if case == "flat_planes":
        w["crystal"]["max_refl"] = 4
        w["crystal"]["planes"] = {"hbar_ratio": 0.7, "extra": [(w["crystal"]["two_d"] / 2, 0.5, 1.0, 0.0)]}
    elif case == "box":
        w["rocking_curve"] = dict(kind="box", peak=0.5, shift=0.0, fwhm=80e-6)
    elif case == "energy_dependent":
        w["rocking_curve"]["energy_dependence"] = [(7.9, -20e-6, 0.7), (8.05, 5e-6, 1.6)]
    elif case == "table":
        w = W.get("flat_stress", precision="fp64")
    n, seed = 5000, 6
    _, k, _ = oracle.source_sample(w, np.arange(n), seed=seed)
    rays = {"polarisations": _random_polarisations(k, 1)}
    j = Job(emu, w, n, seed, rays=rays)
    if case != "fp32_mixed":
        rec = np.zeros(n, mrt.RECORD_DTYPE)
        emu.emu_set_records(j.P, rec.ctypes.data, n)
        assert emu.emu_trace(j.P, WAVES, mrt.PRECISION["fp64"], MAX_MEETINGS) == 0
        o = oracle.trace(w, n=n, seed=seed, records=True, rays=rays)
        _assert_records_match(rec, o["records"])
        assert np.array_equal(j.counts, o["counts"].ravel())
        assert int(rec["n_refl"].sum()) > 20
    else:
        assert emu.emu_trace(j.P, WAVES, mrt.PRECISION["fp32_mixed"], MAX_MEETINGS) == 0
        o = oracle.trace(w, n=n, seed=seed, rays=rays)["counters"]
        c = j.counters()
        for f in ("reflections", "absorbed"):
            assert abs(c[f] - o[f]) < 5 * np.sqrt(c[f] + o[f]) + 5, (f, c[f], o[f])


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_served_extended_requests_equal_requests_alone(emu, precision):
    """The extended serving loop (a spot, an energy-dependent curve, further
    planes, user polarisations) over a round of interleaved half ranges
    gives each request the images and counters of its one-call trace."""
    prec = mrt.PRECISION[precision]
    jobs = _ext_jobs()
    alone = []
    for w, n, s, r in jobs:
        j = Job(emu, w, n, s, rays=r)
        assert emu.emu_trace(j.P, WAVES, prec, MAX_MEETINGS) == 0, w["name"]
        alone.append(j)
    served = [Job(emu, w, n, s, rays=r) for w, n, s, r in jobs]
    slots, it = _round(served)
    assert emu.emu_serve_ext(slots, it.ctypes.data, len(it), 3 * WAVES, prec, MAX_MEETINGS) == 0
    for a, b, (w, n, s, r) in zip(alone, served, jobs):
        assert np.array_equal(a.counts, b.counts), (w["name"], n)
        assert np.array_equal(a.energy, b.energy), (w["name"], n)
        assert a.counters() == b.counters(), (w["name"], n)
        assert a.counters()["reflections"] > 0, w["name"]


def _ext_jobs():
    """Requests with a spot, an energy-dependent curve, further planes and
    user polarisations."""
    import copy
    import oracle
    from paper_2503_16955_amd import workloads as W
    vh = W.get("von_hamos_hapg")
    dep = copy.deepcopy(vh)
    dep["rocking_curve"]["energy_dependence"] = [(7.8, -30e-6, 0.6), (8.2, 45e-6, 2.2)]
    planes = copy.deepcopy(vh)
    planes["crystal"]["planes"] = {"hbar_ratio": 0.5,
                                   "extra": [(vh["crystal"]["two_d"] / 2, 0.6, 1.5, 5e-6)]}
    n_pol = 2500
    _, k, _ = oracle.source_sample(vh, np.arange(n_pol))
    a = np.random.default_rng(3).normal(size=k.shape)
    a -= np.sum(a * k, axis=1)[:, None] * k
    pol = {"polarisations": a / np.linalg.norm(a, axis=1)[:, None]}
    return [(W.with_spot(vh), 3000, 5, None), (dep, 2500, 6, None), (planes, 3000, 7, None),
            (vh, n_pol, 8, pol)]
