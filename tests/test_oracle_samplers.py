"""Pins of the oracle's samplers: mosaic distributions on the unit sphere
(sec. 2.2.2), the point source and the spectra (sec. 2.1).

Every expected distribution is computed here from the paper's densities by
numerical integration or from a textbook distribution in scipy, never by
re-typing the oracle's inverse-CDF formulas."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from paper_2503_16955_amd import workloads as W

DEG = math.pi / 180


# ---- the paper's mosaic densities per unit solid angle ----------------------

def w_mf(theta, gamma):
    """Eq. MF with its normalisation; s from Gamma = 2 s sqrt(2 ln 2)."""
    s = gamma / (2 * math.sqrt(2 * math.log(2)))
    return math.exp((math.cos(theta) - 1) / s**2) / (2 * math.pi * s**2 * (1 - math.exp(-2 / s**2)))


def w_wl(theta, gamma):
    """Eq. WL with its normalisation."""
    return 1.0 / (math.pi * math.log(1 + (4 / gamma) ** 2)) / ((gamma / 2) ** 2 + 2 - 2 * math.cos(theta))


def w_swl(theta, gamma):
    """Eq. SWL with its normalisation."""
    return math.sinh(gamma / 2) ** 2 / (4 * math.pi) / (math.cosh(gamma / 2) - math.cos(theta)) ** 2


def radial_cdf(density, theta, gamma):
    """P(angle to N <= theta) for an isotropic density on the sphere."""
    f = lambda t: 2 * math.pi * math.sin(t) * density(t, gamma)
    pts = [p for p in (gamma, 3 * gamma, 10 * gamma) if p < theta]
    val, _ = integrate.quad(f, 0.0, theta, points=pts or None, limit=400, epsabs=1e-13, epsrel=1e-11)
    return val


@pytest.mark.parametrize("density,gamma", [(w_mf, 0.4 * DEG), (w_mf, 5 * DEG), (w_mf, 60 * DEG),
                                           (w_wl, 0.063 * DEG), (w_wl, 0.8 * DEG),
                                           (w_swl, 0.1 * DEG), (w_swl, 20 * DEG)])
def test_paper_densities_are_normalised(density, gamma):
    assert radial_cdf(density, math.pi, gamma) == pytest.approx(1.0, abs=1e-8)


def _thetas(kind, gamma, u2, eta=0.0):
    n = oracle.mdf_sample(dict(kind=kind, fwhm=gamma, eta=eta), u2, np.full(len(u2), 0.25))
    return np.arccos(np.clip(n[:, 2], -1, 1)), n


@pytest.mark.parametrize("gamma", [0.4 * DEG, 5 * DEG, 60 * DEG])
def test_vmf_quantiles(gamma):
    u = np.linspace(0.01, 0.99, 25)
    th, n = _thetas("gaussian_vmf", gamma, u)
    assert np.allclose(np.linalg.norm(n, axis=1), 1, atol=1e-14)
    for ui, ti in zip(u, th):
        # the sampler maps u to a tilt exceeded with probability u
        assert radial_cdf(w_mf, ti, gamma) == pytest.approx(1 - ui, abs=2e-8)


@pytest.mark.parametrize("gamma", [0.063 * DEG, 0.8 * DEG])
def test_wrapped_lorentzian_quantiles(gamma):
    u = np.linspace(0.01, 0.99, 25)
    th, _ = _thetas("wrapped_lorentzian", gamma, u)
    for ui, ti in zip(u, th):
        assert radial_cdf(w_wl, ti, gamma) == pytest.approx(ui, abs=1e-8)


@pytest.mark.parametrize("gamma", [0.1 * DEG, 20 * DEG])
def test_spherical_wrapped_lorentzian_quantiles(gamma):
    u = np.linspace(0.01, 0.99, 25)
    th, _ = _thetas("spherical_wrapped_lorentzian", gamma, u)
    for ui, ti in zip(u, th):
        assert radial_cdf(w_swl, ti, gamma) == pytest.approx(ui, abs=1e-8)


def test_azimuth_is_two_pi_u3():
    u3 = np.linspace(0.001, 0.999, 50)
    n = oracle.mdf_sample(dict(kind="gaussian_vmf", fwhm=3 * DEG), np.full(50, 0.3), u3)
    xi = np.mod(np.arctan2(n[:, 1], n[:, 0]), 2 * math.pi)
    assert np.allclose(xi, 2 * math.pi * u3, atol=1e-12)


def test_zero_mosaic_gives_surface_normal():
    for kind in ("gaussian_vmf", "lorentzian", "pseudo_voigt", "wrapped_lorentzian",
                 "spherical_wrapped_lorentzian"):
        n = oracle.mdf_sample(dict(kind=kind, fwhm=0.0, eta=0.5), [0.3, 0.9], [0.1, 0.7])
        assert np.array_equal(n, np.array([[0, 0, 1.0], [0, 0, 1.0]]))


def _random_tilts(kind, gamma, eta=0.0, n=40000, seed=1):
    rng = np.random.default_rng(seed)
    u2 = (rng.integers(0, 2**32, n) + 0.5) / 2**32
    u3 = (rng.integers(0, 2**32, n) + 0.5) / 2**32
    return oracle.mdf_sample(dict(kind=kind, fwhm=gamma, eta=eta), u2, u3)


@pytest.mark.parametrize("gamma", [0.1 * DEG, 0.8 * DEG, 10 * DEG])
def test_lorentzian_marginal_is_eq_lorentz(gamma):
    # reading of the Lorentzian mosaic: each one-dimensional tilt marginal is
    # the Lorentzian of Eq. Lorentz with FWHM Gamma (tangent-plane coordinate)
    n = _random_tilts("lorentzian", gamma)
    for axis in (0, 1):
        x = n[:, axis] / n[:, 2]
        assert stats.kstest(x, stats.cauchy(scale=gamma / 2).cdf).pvalue > 1e-3


def test_vmf_small_angle_marginal_is_gaussian_of_width_gamma():
    # sec. 2.2.2: for narrow widths the von Mises-Fisher tilt looks like the
    # Gaussian of Eq. Gaussian with Lambda -> Gamma = 2 s sqrt(2 ln 2)
    gamma = 0.4 * DEG
    n = _random_tilts("gaussian_vmf", gamma)
    s = gamma / (2 * math.sqrt(2 * math.log(2)))
    for axis in (0, 1):
        x = n[:, axis] / n[:, 2]
        assert stats.kstest(x, stats.norm(scale=s).cdf).pvalue > 1e-3


def test_pseudo_voigt_mixture():
    gamma, eta = 0.1 * DEG, 0.3
    n = _random_tilts("pseudo_voigt", gamma, eta=eta, n=60000)
    T = np.sqrt(n[:, 0] ** 2 + n[:, 1] ** 2) / n[:, 2]      # tan(theta), all tilts < 90 deg here
    s = gamma / (2 * math.sqrt(2 * math.log(2)))
    g = gamma / 2

    def cdf(t):   # eta * bivariate Cauchy + (1 - eta) * bivariate normal (small angle)
        return eta * (1 - g / np.sqrt(g * g + t * t)) + (1 - eta) * (1 - np.exp(-t * t / (2 * s * s)))
    assert stats.kstest(T, cdf).pvalue > 1e-3


# ---- source ------------------------------------------------------------------

def test_cone_directions_uniform_in_solid_angle():
    w = W.get("von_hamos_hapg")
    o, k, _ = oracle.source_sample(w, np.arange(20000))
    axis = np.array(w["source"]["axis"])
    b1 = np.array(w["source"]["b1"])
    b2 = np.cross(axis, b1)
    th_max = w["source"]["half_angle"]
    assert np.allclose(np.linalg.norm(k, axis=1), 1, atol=1e-14)
    assert np.all(o == np.array(w["source"]["origin"]))
    one_minus_cos = 1 - k @ axis
    assert one_minus_cos.max() <= 1 - math.cos(th_max) + 1e-15
    assert stats.kstest(one_minus_cos, stats.uniform(0, 1 - math.cos(th_max)).cdf).pvalue > 1e-3
    phi = np.arctan2(k @ b2, k @ b1)
    assert stats.kstest(phi, stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > 1e-3


def test_uniform_spectrum():
    w = W.get("flat_hopg")
    _, _, e = oracle.source_sample(w, np.arange(20000))
    assert stats.kstest(e, stats.uniform(7.9, 0.2).cdf).pvalue > 1e-3


def test_lines_plus_flat_spectrum():
    w = W.get("von_hamos_hapg")
    s = w["source"]
    _, _, e = oracle.source_sample(w, np.arange(40000))
    tot = sum(l[2] for l in s["lines"]) + s["background_w"]

    def cdf(x):
        c = s["background_w"] / tot * np.clip((x - s["e_min"]) / (s["e_max"] - s["e_min"]), 0, 1)
        for (mu, sig, wt) in s["lines"]:
            c = c + wt / tot * stats.norm(mu, sig).cdf(x)
        return c
    assert stats.kstest(e, cdf).pvalue > 1e-3


def test_tabulated_spectrum():
    w = W.get("flat_stress")
    s = w["source"]
    wts = np.array(s["bin_weights"])
    nb = len(wts)
    _, _, e = oracle.source_sample(w, np.arange(300000))
    pos = (e - s["e_min"]) / (s["e_max"] - s["e_min"]) * nb
    b = np.floor(pos).astype(int)
    assert b.min() >= 0 and b.max() < nb
    obs = np.bincount(b, minlength=nb).reshape(-1, 8).sum(1)
    exp = wts.reshape(-1, 8).sum(1) / wts.sum() * len(e)
    assert stats.chisquare(obs, exp).pvalue > 1e-3
    assert stats.kstest(pos - b, stats.uniform(0, 1).cdf).pvalue > 1e-3
