"""Pins of the oracle's rocking curves (sec. 2.2.1) and Bragg's law
(Eq. BraggLaw) against numbers the paper prints and closed forms."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("case", GOLD["pseudo_voigt_width"])
def test_pseudo_voigt_width_matches_paper(case):
    f, eta = oracle.pvoigt_params(case["fwhm_g"], case["fwhm_l"])
    assert abs(f - case["fwhm"]) <= case["tol"], case["cite"]
    assert 0 < eta < 1


def test_pseudo_voigt_limits():
    # pure Gaussian and pure Lorentzian components
    f, eta = oracle.pvoigt_params(50e-6, 0.0)
    assert f == pytest.approx(50e-6, rel=1e-15) and eta == 0.0
    f, eta = oracle.pvoigt_params(0.0, 20e-6)
    assert f == pytest.approx(20e-6, rel=1e-15)
    assert eta == pytest.approx(1.36603 - 0.47719 + 0.11116, rel=1e-15)


@pytest.mark.parametrize("curve", [
    dict(kind="gaussian", peak=0.5, fwhm=50e-6),
    dict(kind="lorentzian", peak=0.3, fwhm=110.8e-6),
    dict(kind="pseudo_voigt", peak=0.5, fwhm_g=50e-6, fwhm_l=8e-6),
    dict(kind="pseudo_voigt", peak=0.7, fwhm_g=100e-6, fwhm_l=20e-6),
])
def test_peak_and_half_maximum(curve):
    # r(0) = peak; r(+-FWHM/2) = peak / 2 (holds for the pseudo-Voigt sum as
    # both parts share the width Lambda)
    if curve["kind"] == "pseudo_voigt":
        lam, _ = oracle.pvoigt_params(curve["fwhm_g"], curve["fwhm_l"])
    else:
        lam = curve["fwhm"]
    r = oracle.irc_value(dict(curve, shift=0.0), [0.0, lam / 2, -lam / 2, 3 * lam])
    assert r[0] == pytest.approx(curve["peak"], rel=1e-15)
    assert r[1] == pytest.approx(curve["peak"] / 2, rel=1e-13)
    assert r[2] == pytest.approx(curve["peak"] / 2, rel=1e-13)
    assert r[3] < curve["peak"] / 2


def test_unit_area_forms():
    # Eq. Gaussian and Eq. Lorentz are unit-area: integral of r / r(0) is
    # 1 / G(0) and 1 / L(0) respectively
    lam = 50e-6
    g = lambda x: oracle.irc_value(dict(kind="gaussian", peak=1.0, fwhm=lam), [x])[0]
    area, _ = integrate.quad(g, -20 * lam, 20 * lam, epsabs=1e-16, limit=200)
    assert area == pytest.approx(1.0 / math.sqrt(4 * math.log(2) / (math.pi * lam * lam)), rel=1e-9)
    l = lambda x: oracle.irc_value(dict(kind="lorentzian", peak=1.0, fwhm=lam), [x])[0]
    area, _ = integrate.quad(l, -np.inf, np.inf, epsabs=1e-16, limit=400)
    assert area == pytest.approx(math.pi * lam / 2, rel=1e-7)


def test_pseudo_voigt_area():
    lam, eta = oracle.pvoigt_params(50e-6, 8e-6)
    r = lambda x: oracle.irc_value(dict(kind="pseudo_voigt", peak=1.0, fwhm_g=50e-6, fwhm_l=8e-6), [x])[0]
    a = 2000 * lam
    core, _ = integrate.quad(r, -a, a, points=[0.0], epsabs=1e-16, limit=1000)
    r0 = eta * 2 / (math.pi * lam) + (1 - eta) * math.sqrt(4 * math.log(2) / math.pi) / lam
    # Lorentzian tails beyond +-a in closed form (the Gaussian part is zero there)
    tails = eta / r0 * 2 * (0.5 - math.atan(2 * a / lam) / math.pi)
    assert core + tails == pytest.approx(1 / r0, rel=1e-8)


def test_box():
    r = oracle.irc_value(dict(kind="box", peak=0.4, fwhm=100e-6), [0, 49.9e-6, 50e-6, 50.1e-6, -60e-6])
    assert list(r) == [0.4, 0.4, 0.4, 0.0, 0.0]


def test_table_interpolation():
    tab = np.array([0.0, 0.2, 0.5, 0.1, 0.3])
    c = dict(kind="table", table=tab.tolist(), x_min=-2e-4, x_max=2e-4, peak=0.5)
    nodes = np.linspace(-2e-4, 2e-4, 5)
    assert np.array_equal(oracle.irc_value(c, nodes), tab)
    mid = (nodes[:-1] + nodes[1:]) / 2
    assert np.allclose(oracle.irc_value(c, mid), (tab[:-1] + tab[1:]) / 2, rtol=1e-12, atol=1e-15)
    q = nodes[1] + 0.25 * (nodes[2] - nodes[1])
    assert oracle.irc_value(c, [q])[0] == pytest.approx(0.75 * 0.2 + 0.25 * 0.5, rel=1e-12)
    assert list(oracle.irc_value(c, [-2.0001e-4, 2.0001e-4])) == [0.0, 0.0]


def test_shift_is_applied_by_caller():
    # r is a function of x = Delta - Delta_M; the curve value does not read shift
    c = dict(kind="gaussian", peak=0.5, fwhm=50e-6, shift=1e-5)
    assert oracle.irc_value(c, [0.0])[0] == 0.5


@pytest.mark.parametrize("case", [c for c in GOLD["bragg_angle"] if "alpha_b" in c])
def test_bragg_angle_matches_paper(case):
    a = oracle.bragg_angle(case["energy_kev"], case["two_d"])
    assert abs(a - case["alpha_b"]) <= case["tol"], case["cite"]


@pytest.mark.parametrize("case", [c for c in GOLD["bragg_angle"] if "alpha_b_deg" in c])
def test_bragg_angle_degrees_matches_paper(case):
    a = math.degrees(oracle.bragg_angle(case["energy_kev"], case["two_d"]))
    assert abs(a - case["alpha_b_deg"]) <= case["tol_deg"], case["cite"]


def test_bragg_law_identity_and_cutoff():
    # hc / E = 2 d sin(alpha_B) with hc = 12.398419843320026 keV A; below the
    # cut-off energy hc / 2d there is no Bragg angle
    hc = 6.62607015e-34 * 299792458.0 / 1.602176634e-19 * 1e7   # keV A from SI constants
    for e in (2.0, 7.06, 8.0, 8.5, 20.0):
        a = oracle.bragg_angle(e, 6.708)
        assert 6.708 * math.sin(a) == pytest.approx(hc / e, rel=1e-14)   # 6.708 A is 2d
    assert oracle.bragg_angle(hc / 6.708 * 0.999, 6.708) == -1.0


@pytest.mark.parametrize("case", GOLD["von_hamos_placement"])
def test_von_hamos_placement_matches_paper(case):
    a = oracle.bragg_angle(case["energy_kev"], case["two_d"])
    z = case["radius"] / math.tan(a)
    assert z == pytest.approx(case["crystal_mm"], rel=case["rel_tol"]), case["cite"]
    assert 2 * z == pytest.approx(case["detector_mm"], rel=case["rel_tol"]), case["cite"]
