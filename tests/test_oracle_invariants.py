"""Invariants and closed-form special cases of the oracle's transport:
photon conservation, integer images consistent with per-ray records,
determinism under threading and range splits, Beer-Lambert absorption
(sec. 2.2.3), specular reflection for a zero-width mosaic (sec. 2.2.4) and
Bragg's-law line positions of a zero-mosaic von Hamos spectrometer."""
import copy
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2503_16955_amd import workloads as W

HC = 6.62607015e-34 * 299792458.0 / 1.602176634e-19 * 1e7   # keV A


def _small(name, n):
    w = W.get(name)
    w["n_rays"] = n
    return w


@pytest.mark.parametrize("name,n", [("flat_hopg", 100000), ("von_hamos_hapg", 200000),
                                    ("flat_stress", 60000)])
def test_conservation_and_image_consistency(name, n):
    w = _small(name, n)
    r = oracle.trace(w, records=True)
    c, rec = r["counters"], r["records"]
    assert c["emitted"] == n
    assert c["emitted"] == (c["missed"] + c["absorbed"] + c["exit_reflected"]
                            + c["exit_transmitted"] + c["truncated"])
    assert c["detected"] <= c["exit_reflected"] + c["exit_transmitted"]
    st = rec["status"]
    for key, code in (("missed", oracle.MISS), ("absorbed", oracle.ABSORBED),
                      ("exit_reflected", oracle.EXIT_REFLECTED),
                      ("exit_transmitted", oracle.EXIT_TRANSMITTED), ("truncated", oracle.TRUNCATED)):
        assert c[key] == int((st == code).sum())
    assert c["events"] == int(rec["n_events"].sum())
    assert c["reflections"] == int(rec["n_refl"].sum())
    det = rec["detected"] == 1
    assert c["detected"] == int(det.sum())
    nx, ny = w["detector"]["nx"], w["detector"]["ny"]
    flat = rec["pix_j"][det].astype(np.int64) * nx + rec["pix_i"][det]
    assert np.array_equal(np.bincount(flat, minlength=nx * ny).reshape(ny, nx), r["counts"])
    quanta = np.rint(rec["energy"][det] * 1e6).astype(np.uint64)
    emap = np.zeros(nx * ny, np.uint64)
    np.add.at(emap, flat, quanta)
    assert np.array_equal(emap.reshape(ny, nx), r["energy_mev"])
    assert np.all((st == oracle.EXIT_REFLECTED) == ((rec["n_refl"] > 0) & (st != oracle.ABSORBED)
                                                    & (st != oracle.TRUNCATED) & (st != oracle.MISS)))
    assert np.all(rec["n_refl"] <= w["crystal"]["max_refl"])
    assert np.allclose(np.linalg.norm(rec["dir"], axis=1), 1.0, atol=1e-14)
    assert np.all(rec["ray_id"] == np.arange(n))


def test_threads_and_range_splits_are_bit_identical():
    w = _small("von_hamos_hapg", 60000)
    a = oracle.trace(w, threads=1, records=True)
    b = oracle.trace(w, threads=7, records=True)
    assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["energy_mev"], b["energy_mev"])
    assert a["records"].tobytes() == b["records"].tobytes()
    h1 = oracle.trace(w, first=0, n=25000)
    h2 = oracle.trace(w, first=25000, n=35000)
    assert np.array_equal(h1["counts"] + h2["counts"], a["counts"])
    assert np.array_equal(h1["energy_mev"] + h2["energy_mev"], a["energy_mev"])
    ids = np.array([5, 59999, 123, 40000], np.uint64)
    rec, _ = oracle.trace_ids(w, ids)
    assert rec.tobytes() == a["records"][ids.astype(int)].tobytes()


def test_truncation_at_event_cap():
    w = _small("flat_hopg", 20000)
    r = oracle.trace(w, max_events=3, records=True)
    rec = r["records"]
    tr = rec["status"] == oracle.TRUNCATED
    assert tr.sum() > 0 and r["counters"]["truncated"] == tr.sum()
    assert np.all(rec["n_events"][tr] == 3) and np.all(rec["n_events"] <= 3)
    assert np.all(rec["detected"][tr] == 0)


def pencil(alpha, energy, thickness=0.040, n=200000, seed=9):
    """Flat crystal (60 x 60 mm), pencil beam at glancing angle alpha onto
    its centre, monochromatic energy, single reflection."""
    w = W.get("flat_hopg")
    ca, sa = math.cos(alpha), math.sin(alpha)
    w["source"].update(origin=[-200 * ca, 0.0, 200 * sa], axis=[ca, 0.0, -sa], half_angle=0.0,
                       spectrum="uniform", e_min=energy, e_max=energy)
    w["crystal"].update(thickness=thickness, length=60.0, width=60.0)
    w["detector"].update(centre=[200 * ca, 0.0, 200 * sa], normal=[-ca, 0.0, -sa], u=[-sa, 0.0, ca])
    w.update(n_rays=n, seed=seed)
    return w


def test_beer_lambert_absorption():
    # no reflection (R_peak = 0): absorbed fraction 1 - exp(-mu0 T / sin a)
    # and absorption depth exponential with rate mu0 / sin a, cut at T
    alpha = 0.3
    w = pencil(alpha, 8.0, thickness=0.5, n=100000)
    w["rocking_curve"]["peak"] = 0.0
    r = oracle.trace(w, records=True, images=False)
    rec = r["records"]
    mu0, T = w["crystal"]["mu0"], 0.5
    p = 1 - math.exp(-mu0 * T / math.sin(alpha))
    frac = r["counters"]["absorbed"] / r["counters"]["emitted"]
    assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / 100000)
    assert r["counters"]["reflections"] == 0 and r["counters"]["missed"] == 0
    ab = rec["status"] == oracle.ABSORBED
    depth = -rec["end"][ab][:, 2]
    lam = mu0 / math.sin(alpha)
    cdf = lambda z: (1 - np.exp(-lam * z)) / (1 - math.exp(-lam * T))
    assert stats.kstest(depth, cdf).pvalue > 1e-3
    # every entered ray meets exactly one event (absorption) unless it exits
    assert np.all(rec["n_events"][ab] == 1)


def test_zero_mosaic_reflection_is_specular():
    w = _small("flat_hopg", 100000)
    w["mosaic"]["fwhm"] = 0.0
    r = oracle.trace(w, records=True, images=False)
    rec = r["records"]
    refl = rec["n_refl"] == 1
    assert refl.sum() > 20
    ids = rec["ray_id"][refl]
    _, k0, e = oracle.source_sample(w, ids)
    N = np.array([0.0, 0.0, 1.0])
    spec = k0 - 2 * (k0 @ N)[:, None] * N
    assert np.abs(rec["dir"][refl] - spec).max() < 1e-14
    # only rays within a few rocking-curve widths of the Bragg angle reflect
    alpha = np.arcsin(-(k0 @ N))
    alpha_b = np.arcsin(HC / (6.708 * e))
    assert np.abs(alpha - alpha_b).max() < 8 * 50e-6


@pytest.mark.parametrize("energy,column", [(8.028, 49.8), (8.048, 85.4)])
def test_von_hamos_zero_mosaic_line_position(energy, column):
    # a zero-mosaic cylinder reflects the on-axis point source back onto the
    # axis at z = 2 rho / tan(alpha), rho the reflection radius in [R, R + T]
    # and alpha within a few rocking-curve widths of alpha_B(E) (Eq. BraggLaw)
    w = _small("von_hamos_hapg", 200000)
    w["source"].update(spectrum="uniform", e_min=energy, e_max=energy)
    w["mosaic"]["fwhm"] = 0.0
    w["crystal"]["max_refl"] = 1
    w["rocking_curve"] = dict(kind="gaussian", peak=0.5, shift=0.0, fwhm=50e-6)
    r = oracle.trace(w, records=True, images=False)
    rec = r["records"]
    det = rec["detected"] == 1
    assert det.sum() > 50
    h = rec["end"][det]
    assert np.abs(h[:, 0]).max() < 1e-9 and np.abs(h[:, 1]).max() < 1e-9
    ab = math.asin(HC / (6.708 * energy))
    R, T, lam = 80.0, 0.040, 50e-6
    lo, hi = 2 * R / math.tan(ab + 8 * lam), 2 * (R + T) / math.tan(ab - 8 * lam)
    assert h[:, 2].min() >= lo and h[:, 2].max() <= hi
    # the line sits at the expected detector column (centre 2 z_c)
    zc = w["crystal"]["z_c"]
    col = (2 * R / math.tan(ab) - 2 * zc) / 0.05
    assert col == pytest.approx(column, abs=0.15)
    got = np.median((h[:, 2] - 2 * zc) / 0.05)
    assert col - 0.5 < got < col + 2 * T / math.tan(ab) / 0.05 + 0.5


def test_below_bragg_cutoff_never_reflects():
    w = _small("flat_hopg", 20000)
    e = 0.9 * HC / 6.708
    w["source"].update(e_min=e, e_max=e)
    r = oracle.trace(w, images=False)
    assert r["counters"]["reflections"] == 0
