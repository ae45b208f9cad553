"""Rocking curves whose shift and width depend on the photon energy (sec.
2.2.1) on the GPU, through the C-ABI: FP64 parity with the oracle on both
geometries and every curve kind; the FP32-mixed kernel equals the plain one
with constant tables and agrees with FP64 statistically otherwise; the
request server serves such curves (its tests sit with the server's)."""
import copy

import numpy as np
import pytest

from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

from test_gpu_parity import _flat_variant, assert_parity

pytestmark = pytest.mark.gpu

DEP = [(7.8, -30e-6, 0.6), (7.95, 5e-6, 1.0), (8.05, 20e-6, 1.5), (8.2, 45e-6, 2.2)]


def _dep(w, table=DEP):
    w = copy.deepcopy(w)
    w["rocking_curve"]["energy_dependence"] = table
    return w


def test_parity_flat_and_von_hamos():
    g, o = assert_parity(_dep(W.get("flat_hopg")), 100_000)
    assert o["counters"]["reflections"] > 500
    assert_parity(_dep(W.get("von_hamos_hapg")), 300_000)


IRCS = {
    "gaussian": dict(kind="gaussian", peak=0.5, shift=0.0, fwhm=50e-6),
    "pseudo_voigt": dict(kind="pseudo_voigt", peak=0.5, shift=0.0, fwhm_g=50e-6, fwhm_l=8e-6),
    "lorentzian": dict(kind="lorentzian", peak=0.4, shift=0.0, fwhm=30e-6),
    "box": dict(kind="box", peak=0.3, shift=0.0, fwhm=60e-6),
    "table": dict(kind="table", peak=0.0, shift=0.0, x_min=-200e-6, x_max=200e-6,
                  table=list(0.5 * np.exp(-np.linspace(-5, 5, 129) ** 2))),
}


@pytest.mark.parametrize("kind", sorted(IRCS))
def test_every_curve_kind(kind):
    g, o = assert_parity(_dep(_flat_variant(irc=IRCS[kind])), 30_000)
    assert o["counters"]["reflections"] > 50


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_constant_tables_take_the_plain_kernels_decisions(precision):
    """With the curve's own shift and scale 1 the kernel takes every decision
    the plain kernel takes (identical counters, refined ones included) and
    gives identical images, in both precisions: the two instances round
    their FP32 arithmetic alike (multiply-adds are fused only inside a
    source expression)."""
    w = W.get("von_hamos_hapg")
    n = 1_000_000
    const = _dep(w, [(7.0, w["rocking_curve"]["shift"], 1.0), (9.0, w["rocking_curve"]["shift"], 1.0)])
    a = mrt.trace(const, n_rays=n, precision=precision)
    b = mrt.trace(w, n_rays=n, precision=precision)
    for f in ("absorbed", "exit_reflected", "exit_transmitted", "detected", "events",
              "reflections", "refined"):
        assert a["counters"][f] == b["counters"][f], f
    ca, ea = mrt.image_to_numpy(a["counts"], a["energy"])
    cb, eb = mrt.image_to_numpy(b["counts"], b["energy"])
    assert np.array_equal(ca, cb) and np.array_equal(ea, eb)


def test_fp32_mixed_agrees_with_fp64():
    w = _dep(W.get("von_hamos_hapg"))
    n = 20_000_000
    a = mrt.trace(w, n_rays=n, precision="fp32_mixed")["counters"]
    b = mrt.trace(w, n_rays=n, precision="fp64")["counters"]
    for f in ("reflections", "detected", "exit_reflected"):
        assert abs(a[f] - b[f]) < 5 * np.sqrt(a[f] + b[f]) + 1e-3 * b[f], (f, a[f], b[f])
    assert a["refined"] < 0.01 * a["events"]


def test_papers_model_parity():
    # the paper's event model with the energy-dependent curve (sec. 2.2.1):
    # per photon beta = alpha_B + Delta_M(E) and strength s(E) int r / h
    for name, n in (("von_hamos_hapg", 100_000), ("flat_hopg", 60_000)):
        w = _dep(W.get(name))
        w["event_model"] = {"kind": "mwg", "burn_in": 200, "psi_nodes": 256}
        g, o = assert_parity(w, n)
        assert o["counters"]["reflections"] > 300
