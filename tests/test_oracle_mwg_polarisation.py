"""Pins of the oracle's polarisation in the paper's own event model
(sec. 2.2.3 Eqs. G_pol, SimpleReflXsectionPol, ReflXsectionPol; sec. 2.2.4).

The angle form G(Delta, phi - psi) = 1 - sin^2(2 b) sin^2(phi - psi), with
phi from the oracle's polarisation angle, equals the vector form
1 - (p.k_s)^2 for the crystallite the oracle builds at (psi, b); the
polarised psi integral averages over phi to G_unpol times the unpolarised
one exactly, and agrees with a dense independent quadrature of W G; the
sampler's psi distribution for a wide mosaic follows W G (moments of
2 psi); and random polarisations reproduce the unpolarised model whose
peak carries G_unpol."""
import copy
import math

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import workloads as W


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("alpha,b", [(0.23, 0.231), (0.25, 0.22), (0.6, 0.58), (1.1, 1.0)])
def test_angle_form_equals_vector_form(alpha, b):
    rng = np.random.default_rng(int(alpha * 100))
    for _ in range(20):
        N = _unit(rng.normal(size=3))
        t = _unit(np.cross(N, rng.normal(size=3)))
        k = -math.sin(alpha) * N + math.cos(alpha) * t
        q = _unit(np.cross(k, rng.normal(size=3)))      # a polarisation normal to k
        phi = oracle.polarisation_angle(q, N, k, alpha)
        for psi in np.linspace(-math.pi, math.pi, 9):
            n = oracle.crystallite(N, k, alpha, b, psi)
            assert np.dot(k, n) == pytest.approx(-math.sin(b), abs=1e-13)
            ks = k - 2 * np.dot(k, n) * n
            g_vec = 1 - np.dot(q, ks) ** 2
            g_ang = 1 - math.sin(2 * b) ** 2 * math.sin(phi - psi) ** 2
            assert g_ang == pytest.approx(g_vec, abs=1e-12)
        # the paper's definition of cos(phi)
        assert math.cos(phi) == pytest.approx(np.dot(q, np.cross(N, k)) / math.cos(alpha), abs=1e-12)


MOSAICS = [dict(kind="gaussian_vmf", fwhm=0.02, eta=0.0),
           dict(kind="wrapped_lorentzian", fwhm=0.01, eta=0.0),
           dict(kind="pseudo_voigt", fwhm=0.015, eta=0.4)]


@pytest.mark.parametrize("mosaic", MOSAICS, ids=[m["kind"] for m in MOSAICS])
def test_phi_average_is_the_unpolarised_factor(mosaic):
    alpha, beta = 0.24, 0.233
    S = math.sin(2 * beta) ** 2
    unpol = oracle.psi_integral(mosaic, alpha, beta, 256)
    phis = np.arange(12) * (2 * math.pi / 12)
    pol = np.mean([oracle.psi_integral_pol(mosaic, alpha, beta, f, 256) for f in phis])
    assert pol == pytest.approx((1 - S / 2) * unpol, rel=1e-13)


@pytest.mark.parametrize("phi", [0.0, 0.7, 1.5708, 2.4])
def test_polarised_integral_against_a_dense_quadrature(phi):
    mosaic = MOSAICS[0]
    alpha, beta = 0.25, 0.233
    # independent: a dense uniform grid in psi, Eq. ThetaPsi and Eq. G_pol written here
    psi = np.linspace(-math.pi, math.pi, 400001)
    v = 2 * math.sin((alpha - beta) / 2) ** 2 + 2 * math.cos(alpha) * math.cos(beta) * np.sin(psi / 2) ** 2
    Wv = oracle.mdf_density(mosaic, v)
    G = 1 - math.sin(2 * beta) ** 2 * np.sin(phi - psi) ** 2
    y = Wv * G
    dense = float(np.sum((y[1:] + y[:-1]) / 2 * np.diff(psi)))
    assert oracle.psi_integral_pol(mosaic, alpha, beta, phi, 2048) == pytest.approx(dense, rel=2e-5)
    assert oracle.psi_integral_pol(mosaic, alpha, beta, phi, 256) == pytest.approx(dense, rel=5e-3)


def test_sampler_follows_the_polarised_integrand():
    # a wide mosaic, so that G's modulation over psi shows in the samples
    mosaic = dict(kind="gaussian_vmf", fwhm=1.0, eta=0.0)
    irc = dict(kind="gaussian", peak=0.5, shift=0.0, fwhm=50e-6)
    alpha, ab, phi = 0.30, 0.25, 0.6
    w_psi = 1.0 / math.cos(ab)
    s = oracle.mwg_sample_pol(mosaic, irc, w_psi, 50e-6, 7, np.arange(6000), 3, 400, alpha, ab, phi)
    psi = s[:, 0]
    grid = np.linspace(-math.pi, math.pi, 20001)
    v = 2 * math.sin((alpha - ab) / 2) ** 2 + 2 * math.cos(alpha) * math.cos(ab) * np.sin(grid / 2) ** 2
    f = oracle.mdf_density(mosaic, v) * (1 - math.sin(2 * ab) ** 2 * np.sin(phi - grid) ** 2)
    f /= f.sum()
    for fn in (lambda x: np.sin(2 * x), lambda x: np.cos(2 * x)):
        want = float(np.sum(f * fn(grid)))
        vals = fn(psi)
        assert abs(vals.mean() - want) < 4 * vals.std() / math.sqrt(len(vals)) + 2e-3, (vals.mean(), want)
    # the asymmetry that G introduces is resolved
    assert abs(float(np.sum(f * np.sin(2 * grid)))) > 5 * np.sin(2 * psi).std() / math.sqrt(len(psi))


def test_random_polarisations_match_the_unpolarised_factor():
    w = W.get("flat_hopg")
    w["event_model"] = {"kind": "mwg", "burn_in": 50, "psi_nodes": 128}
    n = 400000
    _, k, _ = oracle.source_sample(w, np.arange(n))
    a = np.random.default_rng(9).normal(size=(n, 3))
    a -= np.sum(a * k, axis=1)[:, None] * k
    p = a / np.linalg.norm(a, axis=1)[:, None]
    pol = oracle.trace(w, n=n, rays={"polarisations": p})["counters"]["reflections"]
    ab = math.asin(12.398419843320026 / (w["crystal"]["two_d"] * 8.0))
    g = (1 + math.cos(2 * ab) ** 2) / 2
    w2 = copy.deepcopy(w)
    w2["rocking_curve"]["peak"] *= g
    unp = oracle.trace(w2, n=n)["counters"]["reflections"]
    assert pol > 2000
    assert abs(pol - unp) < 4 * math.sqrt(pol + unp), (pol, unp)
    plain = oracle.trace(w, n=n)["counters"]["reflections"]
    assert plain - pol > 4 * math.sqrt(pol + plain)
