"""Pins of the oracle's regular Gaussian mosaic distribution (sec. 2.2.2,
"a common form for the MDF is a Gaussian"; Eq. Gaussian with Delta -> theta
and Lambda -> Gamma), read as an isotropic tilt on the sphere: a bivariate
normal in the tangent plane at N, mapped by tan(theta) = |T|.

* Each tangent-plane coordinate of the sampled normals, (n.e1)/(n.N) and
  (n.e2)/(n.N), is normal with standard deviation Gamma / (2 sqrt(2 ln 2))
  (Kolmogorov-Smirnov against scipy's normal), and the two are independent;
  so every one-dimensional marginal of the tilt is Eq. Gaussian of FWHM
  Gamma.
* The density per steradian is normalised over the sphere (quadrature), the
  sampled polar angles follow it (KS), and for small angles it is the
  two-dimensional Gaussian exp(-theta^2 / (2 s^2)) / (2 pi s^2).
* Fig. MF_vs_G(a): at Gamma = 1 deg its shape in theta is that of the von
  Mises-Fisher distribution of Eq. MF, to within a percent of the peak over
  +-2 Gamma (both normalised to their peaks)."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle

DEG = math.pi / 180
K = 2 * math.sqrt(2 * math.log(2))     # FWHM / sigma of a normal


def _sample(gamma, n, seed):
    rng = np.random.default_rng(seed)
    u2 = rng.uniform(0.0, 1.0, n)
    u3 = rng.uniform(0.0, 1.0, n)
    nrm = oracle.mdf_sample(dict(kind="gaussian", fwhm=gamma), u2, u3)
    return nrm


@pytest.mark.parametrize("gamma", [0.1 * DEG, 1.0 * DEG, 10.0 * DEG])
def test_tangent_plane_marginals_are_eq_gaussian(gamma):
    n = _sample(gamma, 40_000, 7)
    t1 = n[:, 0] / n[:, 2]
    t2 = n[:, 1] / n[:, 2]
    sigma = gamma / K
    for t in (t1, t2):
        assert stats.kstest(t / sigma, "norm").pvalue > 1e-3
    # a wrong width is rejected: sigma taken as the FWHM, or 5 % off
    assert stats.kstest(t1 / gamma, "norm").pvalue < 1e-6
    assert stats.kstest(t1 / (1.05 * sigma), "norm").pvalue < 1e-3
    # independent coordinates (a bivariate normal with isotropic covariance)
    assert abs(np.corrcoef(t1, t2)[0, 1]) < 0.03
    assert abs(np.corrcoef(t1 * t1, t2 * t2)[0, 1]) < 0.03
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0, atol=1e-14)


def _w(gamma, theta):
    c = math.cos(theta)
    return float(oracle.mdf_density(dict(kind="gaussian", fwhm=gamma), 1.0 - c)[0])


@pytest.mark.parametrize("gamma", [0.1 * DEG, 1.0 * DEG, 10.0 * DEG])
def test_density_normalised_and_followed_by_the_sampler(gamma):
    f = lambda t: 2 * math.pi * math.sin(t) * _w(gamma, t)
    pts = [gamma, 3 * gamma, 10 * gamma]
    total, _ = integrate.quad(f, 0.0, math.pi / 2, points=pts, limit=400, epsabs=1e-12)
    assert total == pytest.approx(1.0, abs=1e-7)
    # nothing on the far hemisphere
    assert _w(gamma, 0.6 * math.pi) == 0.0
    n = _sample(gamma, 20_000, 11)
    theta = np.arccos(np.clip(n[:, 2], -1, 1))
    grid = np.linspace(0.0, min(12 * gamma, math.pi / 2), 400)
    cdf = np.concatenate([[0.0], np.cumsum([integrate.quad(f, a, b)[0]
                                            for a, b in zip(grid[:-1], grid[1:])])])
    assert stats.kstest(theta, lambda x: np.interp(x, grid, cdf)).pvalue > 1e-3


def test_small_angle_limit_is_the_planar_gaussian():
    gamma = 0.1 * DEG
    s = gamma / K
    for theta in np.linspace(0.0, 2.5 * s, 11):
        planar = math.exp(-theta * theta / (2 * s * s)) / (2 * math.pi * s * s)
        assert _w(gamma, theta) == pytest.approx(planar, rel=1e-5)


def test_shape_of_the_von_mises_fisher_at_one_degree():
    gamma = 1.0 * DEG
    th = np.linspace(0.0, 2 * gamma, 41)
    g = np.array([_w(gamma, t) for t in th])
    vmf = oracle.mdf_density(dict(kind="gaussian_vmf", fwhm=gamma), 1.0 - np.cos(th))
    g, vmf = g / g[0], vmf / vmf[0]
    assert np.max(np.abs(g - vmf)) < 0.01
