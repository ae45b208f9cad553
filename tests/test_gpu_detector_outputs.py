"""The detector outputs on the GPU (sec. 2.3, sec. 3), through the C-ABI: the
energy image weighted by the detector's quantum efficiency (FP64 parity with
the oracle; the FP32-mixed kernels and the request server apply the same
weight), and the calibration map of a uniform-energy run (bit-exact against
its definition applied to the same images, and the run itself in parity with
the oracle)."""
import copy

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu

QE = [(7.8, 0.35), (7.95, 0.9), (8.03, 0.55), (8.2, 0.8)]


def _with_qe(name, table=QE, **kw):
    w = W.get(name, **kw)
    w["detector"]["qe"] = table
    return w


def test_qe_parity_flat():
    g, o = assert_parity(_with_qe("flat_hopg"), 100_000)
    plain = oracle.trace(W.get("flat_hopg"), n=100_000)
    assert np.array_equal(o["counts"], plain["counts"])
    assert o["energy_mev"].sum() < plain["energy_mev"].sum()


def test_qe_parity_von_hamos_and_paper_model():
    assert_parity(_with_qe("von_hamos_hapg"), 300_000)
    w = _with_qe("von_hamos_hapg")
    w["event_model"] = {"kind": "mwg", "burn_in": 100, "psi_nodes": 256}
    assert_parity(w, 100_000)


def _energy_from_records(rec, nx, ny, table):
    e, v = np.array(table).T
    det = rec["detected"] == 1
    px = rec["pix_j"][det].astype(np.int64) * nx + rec["pix_i"][det]
    E = rec["energy"][det]
    out = np.zeros(nx * ny, np.uint64)
    np.add.at(out, px, np.rint(E * np.interp(E, e, v) * 1e6).astype(np.uint64))
    return out.reshape(ny, nx)


def test_qe_fp32_mixed_weights_each_detected_photon():
    w = _with_qe("von_hamos_hapg")
    n = 500_000
    g = mrt.trace(w, n_rays=n, precision="fp32_mixed", records="all")
    gc, ge = mrt.image_to_numpy(g["counts"], g["energy"])
    rec = mrt.records_to_numpy(g["records"])
    assert np.array_equal(ge, _energy_from_records(rec, w["detector"]["nx"], w["detector"]["ny"], QE))
    p = mrt.trace(W.get("von_hamos_hapg"), n_rays=n, precision="fp32_mixed")
    assert np.array_equal(gc, mrt.image_to_numpy(p["counts"])[0])


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_qe_in_a_served_request(precision):
    w = _with_qe("von_hamos_hapg")
    n = 400_000
    with mrt.Server(hbm_budget_bytes=1 << 30, max_slots=4, precision=precision) as srv:
        t = srv.submit(w, n_rays=n, seed=5)
        r = srv.wait(t, timeout_ms=60000)
        print(f"[qe-serve] {precision} done", flush=True)
        assert r["state"] == "done"
        sc, se = mrt.image_to_numpy(r["counts"], r["energy"])
        a = mrt.trace(w, n_rays=n, seed=5, precision=precision)
        ac, ae = mrt.image_to_numpy(a["counts"], a["energy"])
        assert np.array_equal(sc, ac) and np.array_equal(se, ae)
        srv.release(t)


def test_calibration_run_and_map():
    w = W.get("von_hamos_hapg")
    cal = W.calibration_workload(w, 8.00, 8.06)
    assert_parity(cal, 200_000)
    counts, energy, m = mrt.calibrate(w, 8.00, 8.06, n_rays=20_000_000)
    gc, ge = mrt.image_to_numpy(counts, energy)
    want = oracle.calibration_map(gc, ge)
    got = m.cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.array_equal(got[~np.isnan(got)], want[~np.isnan(want)])
    assert (gc > 0).sum() > 10_000
    assert 8.0 <= np.nanmin(got) and np.nanmax(got) <= 8.06
