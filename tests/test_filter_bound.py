"""The FP32 acceptance filter (the first test of every crystallite
encounter's decision u < r(Delta - Delta_M) / R_max, sec. 2.2.1), pinned
on the CPU.

The device code of the filter (Tracer::sin_delta_f32, asin_small_f32,
x_bounds, filter) runs compiled for the host (helpers/simt_emu.cpp).  FP32
arithmetic is IEEE on both sides; the hardware's v_sqrt_f32, v_rcp_f32 and
v_exp_f32 are within 1 ulp and not correctly rounded, so every case runs
three times with those results moved one float down, not at all, and one
float up.  Against Delta computed in long double from the same c = |k.n|
and sin(alpha_B):

  * the FP32 estimate of x = Delta - shift (before its error band) is
    within ERR_STATED of the reference (the stated worst case; measured
    3.1e-7 at alpha_B = 84 deg and sqrt(1 - c^2) = 0.1, a fifth of the
    filter's 2e-6 band);
  * the bounds always contain the reference x and |x|;
  * a decision the filter takes (accept or reject) is the exact one of
    both precisions: u < r(x) / R_max evaluated as the FP32-mixed path and
    as the FP64 path evaluate it.

Cases: Bragg angles from 1 to 84 deg, deviations over +-0.3 rad and dense
around the curve's centre, the steepest case the filter still bounds (c near
0.995, where sqrt(1 - c^2) = 0.1 multiplies c's rounding by ~10), c at the
largest rounding error of its conversion to float, curve shifts up to 1e-2
rad and width scales 0.6 and 2.2 (the energy-dependent curve), and u at
relative distances 1e-6 to 1e-2 from r(x) on both sides.  Every curve kind:
Gaussian, pseudo-Voigt, Lorentzian, box and the Darwin-Prins table."""
import ctypes as C

import numpy as np
import pytest

from paper_2503_16955_amd import workloads as W

import test_simt_emulation as T

ERR_STATED = 4.0e-7          # worst case of the FP32 estimate, stated in trace_impl.h


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    L = T.declare(C.CDLL(str(T.build_emu(tmp_path_factory.mktemp("filter")))))
    f, d, i = C.c_float, C.c_double, C.c_int
    P = C.POINTER
    L.emu_filter_cases.argtypes = [C.c_void_p, C.c_void_p, i, P(d), P(d), P(d), d, d, i,
                                   P(f), P(d), P(f), P(i), P(i), P(i), P(i), P(d)]
    L.emu_filter_cases.restype = None
    return L


IRCS = {
    "gaussian": dict(kind="gaussian", peak=0.5, shift=0.0, fwhm=50e-6),
    "gaussian_shifted": dict(kind="gaussian", peak=0.8, shift=30e-6, fwhm=80e-6),
    "pseudo_voigt": dict(kind="pseudo_voigt", peak=0.5, shift=-10e-6, fwhm_g=50e-6, fwhm_l=8e-6),
    "lorentzian": dict(kind="lorentzian", peak=0.4, shift=0.0, fwhm=60e-6),
    "box": dict(kind="box", peak=0.3, shift=5e-6, fwhm=100e-6),
    "table": None,
}


def _workload(kind):
    if kind == "table":
        return W.get("flat_stress")
    w = W.get("flat_hopg")
    w["rocking_curve"] = dict(IRCS[kind])
    return w


def _cases(rng, shift, n_rand=20000):
    """(c, s) pairs: Bragg angles 1-84 deg, deviations random over +-0.3 rad,
    dense near the curve's centre, at the steep cutoff, and c at the
    largest rounding error of its float conversion."""
    a = rng.uniform(np.radians(1.0), np.radians(84.0), n_rand)
    dev = np.concatenate([rng.uniform(-0.3, 0.3, n_rand // 4),
                          shift + rng.normal(0.0, 2e-4, n_rand // 2),
                          shift + rng.normal(0.0, 2e-5, n_rand // 4)])
    c = np.abs(np.sin(a + dev))
    s = np.sin(a)
    # the steepest bounded case: sqrt(1 - c^2) just above 0.1
    cw = rng.uniform(0.1, 0.1003, 4000)
    c2 = np.sqrt(1.0 - cw * cw)
    s2 = np.sin(np.arcsin(c2) - shift - rng.normal(0.0, 3e-5, cw.size))
    # c half a float ulp off a float (the largest conversion error)
    cf = np.abs(np.sin(a[:4000] + dev[:4000])).astype(np.float32)
    half = (np.nextafter(cf, np.float32(2.0)) - cf).astype(np.float64) * 0.4999
    c3 = np.clip(cf.astype(np.float64) + np.where(rng.random(4000) < 0.5, half, -half), 0.0, 1.0)
    s3 = s[:4000]
    c = np.concatenate([c, c2, c3])
    s = np.concatenate([s, s2, s3])
    keep = (s > 0.0) & (s < 1.0) & (c <= 1.0)
    return c[keep], s[keep]


def _run(L, P, lut, c, s, u, shift, scale, bias):
    n = len(c)
    f = lambda k, t: np.zeros(k, t)
    x_est, x_ref, b = f(n, np.float32), f(n, np.float64), f(4 * n, np.float32)
    has, dec, d32, d64 = (f(n, np.int32) for _ in range(4))
    ratio = f(n, np.float64)
    D = lambda a: np.ascontiguousarray(a, np.float64).ctypes.data_as(C.POINTER(C.c_double))
    Pf = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
    Pi = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
    cc, ss, uu = (np.ascontiguousarray(v, np.float64) for v in (c, s, u))
    L.emu_filter_cases(P, lut, n, D(cc), D(ss), D(uu), shift, scale, bias, Pf(x_est),
                       x_ref.ctypes.data_as(C.POINTER(C.c_double)), Pf(b), Pi(has), Pi(dec),
                       Pi(d32), Pi(d64), ratio.ctypes.data_as(C.POINTER(C.c_double)))
    return x_est, x_ref, b.reshape(n, 4), has.astype(bool), dec, d32, d64, ratio


@pytest.mark.parametrize("kind", sorted(IRCS))
def test_filter_bounds_and_decisions(emu, kind):
    w = _workload(kind)
    job = T.Job(emu, w, 64, 0)
    lut = job.tab.ctypes.data if kind == "table" else None
    base = float(w["rocking_curve"].get("shift", 0.0))
    rng = np.random.default_rng(2025)
    worst = 0.0
    n_decided = 0
    for shift, scale in ((base, 1.0), (base + 3e-5, 0.6), (base - 1e-2, 2.2), (1e-3, 1.0)):
        c, s = _cases(rng, shift)
        # u near the decision threshold r(x) / R_max (as the FP64 path
        # evaluates it), on both sides, or anywhere
        r = _run(emu, job.P, lut, c, s, np.full(len(c), 0.5), shift, scale, 0)[-1]
        rel = rng.choice([-1e-2, -1e-4, -2e-5, -1e-6, 1e-6, 2e-5, 1e-4, 1e-2], len(c))
        u = np.where(rng.random(len(c)) < 0.7, r * (1.0 + rel), rng.random(len(c)))
        u = np.clip(u, 2.0 ** -25, 1.0 - 2.0 ** -25)
        for bias in (-1, 0, 1):
            xe, xr, b, has, dec, d32, d64, _ = _run(emu, job.P, lut, c, s, u, shift, scale, bias)
            lo, hi, slo, shi = b.T.astype(np.float64)
            # the bounds hold the reference
            assert np.all(slo[has] <= xr[has]) and np.all(xr[has] <= shi[has])
            ax = np.abs(xr)
            assert np.all(lo[has] <= ax[has]) and np.all(ax[has] <= hi[has])
            # the FP32 estimate's own error (in x before the 1/scale)
            ok = np.isfinite(xe)
            err = np.abs(xe[ok].astype(np.float64) - xr[ok] * scale)
            worst = max(worst, float(err.max()))
            # every decision the filter takes is the exact one in both paths
            taken = dec >= 0
            assert np.array_equal(dec[taken], d32[taken]), kind
            assert np.array_equal(dec[taken], d64[taken]), kind
            n_decided += int(taken.sum())
    assert worst <= ERR_STATED, worst
    assert n_decided > 100_000


def test_table_envelope_bounds_the_curve(emu):
    """The table curve's envelope (the minimum and maximum node of each
    bucket, rounded outward to float): over random x intervals of the
    filter's width, around the peak, in the tails and across the table's
    ends, the bounds hold the exact FP64 ratio at every sampled x; the
    buckets are sized so that such an interval reaches at most two."""
    w = _workload("table")
    job = T.Job(emu, w, 64, 0)
    f, i = C.c_float, C.c_int
    emu.emu_table_bounds.argtypes = [C.c_void_p, f, f, C.POINTER(f), C.POINTER(f), i,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i)]
    emu.emu_table_bounds.restype = i
    rc = w["rocking_curve"]
    x0, x1 = rc["x_min"], rc["x_max"]
    rng = np.random.default_rng(77)
    m = 33
    xs, rs = np.zeros(m), np.zeros(m)
    lo, hi, sh = f(), f(), i()
    taken = 0
    centres = np.concatenate([rng.uniform(x0 - 2e-5, x1 + 2e-5, 3000),
                              rng.normal(0.0, 3e-5, 3000), [x0, x1, x0 + 1e-7, x1 - 1e-7]])
    for c in centres:
        half = rng.choice([2e-6, 2e-6 / 0.6, 5e-7])
        slo, shi = np.float32(c - half), np.float32(c + half)
        ok = emu.emu_table_bounds(job.P, slo, shi, C.byref(lo), C.byref(hi), m,
                                  xs.ctypes.data_as(C.POINTER(C.c_double)),
                                  rs.ctypes.data_as(C.POINTER(C.c_double)), C.byref(sh))
        if not ok:
            # only intervals beyond the table's ends go without bounds
            assert shi < x0 or slo > x1 or half > 2.1e-6 or c < x0 + 1e-5 or c > x1 - 1e-5, c
            continue
        taken += 1
        assert np.all(rs <= hi.value) and np.all(rs >= lo.value), (c, half, lo.value, hi.value)
    assert taken > 5000
    assert 3 <= sh.value <= 12
