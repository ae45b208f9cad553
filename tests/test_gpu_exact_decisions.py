"""The FP32 acceptance bound never changes a decision, checked on the device.

Every crystallite encounter's decision u_acc < r(Delta - Delta_M) / R_max
(sec. 2.2.1) is normally settled by an FP32 interval bound of Delta and the
curve, and only re-taken by the FP64 evaluation when u_acc falls inside the
bound's band.  With ``exact_decisions`` every decision is the FP64
evaluation.  Both runs must give the same images and counters bit for bit
(only the `refined` diagnostic differs), in both precisions, for every
curve kind and with the extended decisions (energy-dependent curve,
polarisation, plane sums).  The exact runs take the run-time-kind kernel and
the default ones the kernel specialised for the kinds, so the FP32-mixed
cases also show that two instances round the FP32 geometry alike."""
import copy

import numpy as np
import pytest
import torch

from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("missed", "absorbed", "exit_reflected", "exit_transmitted", "truncated", "detected",
          "events", "reflections")


def _check_same(w, n, precision, rays=None):
    a = mrt.trace(w, n_rays=n, precision=precision, rays=rays)
    b = mrt.trace(w, n_rays=n, precision=precision, rays=rays, exact_decisions=True)
    ca, ea = mrt.image_to_numpy(a["counts"], a["energy"])
    cb, eb = mrt.image_to_numpy(b["counts"], b["energy"])
    print(f"[exact] {w['name']} {precision} n={n} refined {a['counters']['refined']} -> "
          f"{b['counters']['refined']}, detected {a['counters']['detected']}", flush=True)
    for f in FIELDS:
        assert a["counters"][f] == b["counters"][f], (f, a["counters"][f], b["counters"][f])
    assert np.array_equal(ca, cb) and np.array_equal(ea, eb)
    # the exact run evaluated far more decisions than the bound left over
    assert b["counters"]["refined"] > 10 * max(a["counters"]["refined"], 1)
    assert a["counters"]["reflections"] > 100
    return a, b


def _flat(irc):
    w = W.get("flat_hopg")
    w["rocking_curve"] = dict(W.get("flat_hopg")["rocking_curve"], **irc)
    w["name"] = f"flat_hopg/{irc['kind']}"
    return w


IRCS = {
    "gaussian": {"kind": "gaussian"},
    "pseudo_voigt": {"kind": "pseudo_voigt", "fwhm_g": 50e-6, "fwhm_l": 8e-6},
    "lorentzian": {"kind": "lorentzian", "fwhm": 50e-6},
    "box": {"kind": "box", "fwhm": 50e-6},
}


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_von_hamos_bound_changes_nothing(precision):
    _check_same(W.get("von_hamos_hapg"), 1_000_000, precision)


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
@pytest.mark.parametrize("kind", sorted(IRCS))
def test_every_analytic_curve(kind, precision):
    _check_same(_flat(IRCS[kind]), 200_000, precision)


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_table_curve_stress(precision):
    # the Darwin-Prins table: the bound only rejects outside the table
    w = W.get("flat_stress")
    a, _ = _check_same(w, 300_000, precision)
    assert a["counters"]["refined"] > 0


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_extended_decisions(precision):
    # energy-dependent curve, polarisation and plane sums: their own bounds
    vh = W.get("von_hamos_hapg")
    dep = copy.deepcopy(vh)
    dep["name"] = "von_hamos/dep"
    dep["rocking_curve"]["energy_dependence"] = [(7.8, -3e-6, 0.8), (8.0, 2e-6, 1.0),
                                                 (8.2, 6e-6, 1.3)]
    _check_same(dep, 500_000, precision)

    planes = copy.deepcopy(vh)
    planes["name"] = "von_hamos/planes"
    td = planes["crystal"]["two_d"]
    planes["source"]["lines"] = list(planes["source"]["lines"]) + [(2 * 8.048, 0.004, 0.4)]
    planes["crystal"]["planes"] = {"hbar_ratio": 0.7, "extra": [(td / 2, 0.6, 1.5, 5e-6)]}
    _check_same(planes, 500_000, precision)

    n = 400_000
    g = np.random.default_rng(31)
    k_axis = np.asarray(vh["source"]["axis"], np.float64)
    a = g.normal(size=(n, 3))
    a -= (a @ k_axis)[:, None] * k_axis
    a /= np.linalg.norm(a, axis=1)[:, None]
    # polarisations normal to the cone axis (not exactly to each ray: only
    # their use in G and the update matters here)
    pol = torch.as_tensor(a, device="cuda").contiguous()
    polar = copy.deepcopy(vh)
    polar["name"] = "von_hamos/polarised"
    _check_same(polar, n, precision, rays={"polarisations": pol})
