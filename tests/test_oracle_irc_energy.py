"""Pins of the oracle's energy-dependent rocking curve (sec. 2.2.1): the
curve of a photon of energy E is r((Delta - Delta_M(E)) / s(E)), Delta_M and
the width scale s interpolated from the user's tables.

Exact equivalences: constant tables equal to the curve's own shift and a
scale of 1 change nothing; a constant scale of 2 is the Gaussian curve of
twice the FWHM.  Statistics: the accepted Bragg deviations of a pencil beam
centre on Delta_M(E) and spread as s(E) times the curve's width, slice by
slice in energy."""
import copy
import math

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import workloads as W
from test_oracle_invariants import HC, pencil


def _records(w, n):
    return oracle.trace(w, n=n, records=True, images=False)["records"]


def test_constant_tables_change_nothing():
    w = W.get("flat_hopg")
    w["rocking_curve"]["shift"] = 7e-6
    base = _records(w, 40000)
    d = copy.deepcopy(w)
    d["rocking_curve"]["energy_dependence"] = [(7.0, 7e-6, 1.0), (8.0, 7e-6, 1.0), (9.0, 7e-6, 1.0)]
    assert _records(d, 40000).tobytes() == base.tobytes()


def test_scale_two_is_the_gaussian_of_twice_the_width():
    w = W.get("flat_hopg")
    d = copy.deepcopy(w)
    d["rocking_curve"]["energy_dependence"] = [(7.5, 0.0, 2.0)]
    wide = copy.deepcopy(w)
    wide["rocking_curve"]["fwhm"] = 2 * w["rocking_curve"]["fwhm"]
    a, b = _records(d, 40000), _records(wide, 40000)
    assert a.tobytes() == b.tobytes()
    assert b["n_refl"].sum() > _records(w, 40000)["n_refl"].sum()


def test_deviations_follow_the_energy_dependent_curve():
    # pencil beam onto a flat slab, energies 7.9-8.1 keV, single reflection:
    # per energy slice, the accepted Delta = asin|k.n| - alpha_B(E) has mean
    # Delta_M(E) and standard deviation s(E) sigma of the Gaussian curve
    alpha = math.asin(HC / (6.708 * 8.0))
    w = pencil(alpha, 8.0, n=1_500_000)
    w["source"].update(e_min=7.9, e_max=8.1)
    w["mosaic"] = dict(kind="gaussian_vmf", fwhm=1.0 * math.pi / 180, eta=0.0)
    table = [(7.9, -40e-6, 0.6), (8.0, 10e-6, 1.0), (8.1, 60e-6, 1.8)]
    w["rocking_curve"] = dict(kind="gaussian", peak=0.5, shift=0.0, fwhm=50e-6,
                              energy_dependence=table)
    rec = _records(w, w["n_rays"])
    refl = rec["n_refl"] == 1
    assert refl.sum() > 3000
    k0 = np.array(w["source"]["axis"])
    n = rec["dir"][refl] - k0
    n /= np.linalg.norm(n, axis=1)[:, None]
    E = rec["energy"][refl]
    delta = np.arcsin(np.abs(n @ k0)) - np.arcsin(HC / (6.708 * E))
    e, sh, sc = np.array(table).T
    sigma = 50e-6 / (2 * math.sqrt(2 * math.log(2)))
    for lo, hi in [(7.9, 7.95), (7.975, 8.025), (8.05, 8.1)]:
        m = (E >= lo) & (E < hi)
        assert m.sum() > 400
        want_mean = np.interp(E[m], e, sh).mean()
        want_sd = np.sqrt(np.mean((np.interp(E[m], e, sc) * sigma) ** 2))
        got = delta[m]
        assert abs(got.mean() - want_mean) < 5 * got.std() / math.sqrt(m.sum())
        # the spread about each photon's own Delta_M(E)
        resid = got - np.interp(E[m], e, sh)
        assert resid.std() == pytest.approx(want_sd, rel=0.08)


def test_energy_dependence_needs_increasing_energies_and_positive_scales():
    for table in ([(8.0, 0.0, 1.0), (8.0, 0.0, 1.0)], [(8.0, 0.0, 0.0)], [(8.0, 0.0, -1.0)]):
        w = W.get("flat_hopg")
        w["rocking_curve"]["energy_dependence"] = table
        with pytest.raises(ValueError):
            oracle.trace(w, n=10)


# ---- the paper's event model ---------------------------------------------------

def _mwg(w, burn_in=100):
    w = copy.deepcopy(w)
    w["event_model"] = {"kind": "mwg", "burn_in": burn_in, "psi_nodes": 128}
    return w


def _rec_m(w, n):
    return oracle.trace(w, n=n, records=True, margins=True, images=False)


def test_papers_model_constant_tables_take_the_plain_decisions():
    import parity
    w = _mwg(W.get("von_hamos_hapg"))
    w["rocking_curve"]["shift"] = 6e-6
    d = copy.deepcopy(w)
    d["rocking_curve"]["energy_dependence"] = [(7.0, 6e-6, 1.0), (9.0, 6e-6, 1.0)]
    A, B = _rec_m(w, 30000), _rec_m(d, 30000)
    n_ties, bad, _ = parity.compare(A["records"], B["records"], np.minimum(A["margins"], B["margins"]))
    assert len(bad) == 0 and n_ties <= 2
    assert A["records"]["n_refl"].sum() > 200


def test_papers_model_scale_two_is_the_gaussian_of_twice_the_width():
    import parity
    w = _mwg(W.get("flat_hopg"))
    d = copy.deepcopy(w)
    d["rocking_curve"]["energy_dependence"] = [(7.5, 0.0, 2.0)]
    wide = copy.deepcopy(w)
    wide["rocking_curve"]["fwhm"] = 2 * w["rocking_curve"]["fwhm"]
    A, B = _rec_m(d, 40000), _rec_m(wide, 40000)
    n_ties, bad, _ = parity.compare(A["records"], B["records"], np.minimum(A["margins"], B["margins"]))
    assert len(bad) == 0 and n_ties <= 2
    assert B["records"]["n_refl"].sum() > _rec_m(w, 40000)["records"]["n_refl"].sum()
