"""Pins of the oracle's detector outputs (sec. 2.3, sec. 3): the energy image
weighted by the detector's quantum efficiency, and the calibration map of a
uniform-energy run.

The QE weight is checked against numpy's linear interpolation applied to the
oracle's own per-ray records; the calibration map against Bragg's law for
the von Hamos geometry (an on-axis source is focused back onto the axis at
z = 2 rho / tan(alpha_B(E)), rho between the front radius R and R + T)."""
import copy
import math

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import workloads as W

HC = 12.398419843320026


def _image_from_records(rec, nx, ny, weight):
    det = rec["detected"] == 1
    px = rec["pix_j"][det].astype(np.int64) * nx + rec["pix_i"][det]
    e = np.rint(rec["energy"][det] * weight(rec["energy"][det]) * 1e6).astype(np.uint64)
    out = np.zeros(nx * ny, np.uint64)
    np.add.at(out, px, e)
    return out.reshape(ny, nx)


@pytest.mark.parametrize("table", [
    [(7.9, 0.2), (7.95, 0.9), (8.02, 0.5), (8.1, 0.7)],
    [(7.0, 0.3), (7.96, 0.8), (8.04, 0.6), (9.0, 1.0)],   # nodes past the spectrum's ends
    [(8.0, 0.75)],                                        # one node: a constant
])
def test_energy_image_is_weighted_by_the_interpolated_qe(table):
    w = W.get("flat_hopg")
    n = 60000
    plain = oracle.trace(w, n=n, records=True)
    wq = copy.deepcopy(w)
    wq["detector"]["qe"] = table
    q = oracle.trace(wq, n=n, records=True)
    # the counts image and the rays are unchanged
    assert np.array_equal(q["counts"], plain["counts"])
    assert q["records"].tobytes() == plain["records"].tobytes()
    e, v = np.array(table).T
    want = _image_from_records(q["records"], w["detector"]["nx"], w["detector"]["ny"],
                               lambda E: np.interp(E, e, v))
    assert np.array_equal(q["energy_mev"], want)
    assert q["energy_mev"].sum() < plain["energy_mev"].sum()


def test_unit_qe_leaves_the_energy_image_unchanged():
    w = W.get("flat_hopg")
    a = oracle.trace(w, n=30000)
    w["detector"]["qe"] = [(7.0, 1.0), (9.0, 1.0)]
    b = oracle.trace(w, n=30000)
    assert np.array_equal(a["energy_mev"], b["energy_mev"])


def test_qe_table_must_increase():
    w = W.get("flat_hopg")
    w["detector"]["qe"] = [(8.0, 0.5), (8.0, 0.6)]
    with pytest.raises(ValueError):
        oracle.trace(w, n=10)


def test_calibration_map_is_the_mean_energy_per_pixel():
    w = W.calibration_workload(W.get("flat_hopg"), 7.9, 8.1)
    o = oracle.trace(w, n=50000, records=True)
    m = oracle.calibration_map(o["counts"], o["energy_mev"])
    rec = o["records"]
    det = rec["detected"] == 1
    assert det.sum() > 100
    nx = w["detector"]["nx"]
    px = rec["pix_j"][det].astype(np.int64) * nx + rec["pix_i"][det]
    for p in np.unique(px)[:200]:
        sel = rec["energy"][det][px == p]
        want = np.rint(sel * 1e6).sum() / len(sel) * 1e-6
        assert m.ravel()[p] == pytest.approx(want, rel=1e-15)
    assert np.isnan(m[o["counts"] == 0]).all()
    # uniform energies in the window
    assert 7.9 <= np.nanmin(m) and np.nanmax(m) <= 8.1


def test_calibration_map_follows_braggs_law_on_the_von_hamos():
    # mean energy per detector column of a uniform 8.00-8.06 keV run: between
    # the energies focused at that column from the front face (rho = R) and
    # from the back (rho = R + T), increasing along the dispersion axis
    w = W.calibration_workload(W.get("von_hamos_hapg"), 8.00, 8.06)
    o = oracle.trace(w, n=3_000_000)
    cnt = o["counts"].sum(0)
    en = o["energy_mev"].sum(0).astype(np.float64)
    cols = np.nonzero(cnt > 100)[0]
    assert len(cols) > 60
    inner = cols[5:-5]   # the window's ends are cut by the band limits
    zc, R, T, pitch, nx = w["crystal"]["z_c"], 80.0, 0.040, 0.05, w["detector"]["nx"]
    mean = en[inner] / cnt[inner] * 1e-6
    z = 2 * zc + (inner + 0.5 - nx / 2) * pitch
    e_front = HC / (6.708 * np.sin(np.arctan(2 * R / z)))
    e_back = HC / (6.708 * np.sin(np.arctan(2 * (R + T) / z)))
    assert np.all(mean <= e_front + 0.5e-3) and np.all(mean >= e_back - 0.5e-3)
    assert np.all(np.diff(mean) > -0.5e-3) and mean[-1] - mean[0] > 0.04
