"""The core physics pin: the oracle's depth stepping reflects at the rate of
the paper's mosaic cross-section, Eq. ReflXsection (sec. 2.2.3, unpolarised
with G folded into the peak), evaluated here by direct quadrature over the
rocking-curve angle Delta and the crystallite azimuth psi with theta(psi)
from Eq. ThetaPsi; and the reflecting crystallites are distributed in psi as
W(theta(psi)) (appendix A, method II), with no gap at psi = 0.

With a pencil beam at glancing angle alpha on a flat slab and a single
reflection allowed, null-collision stepping with majorant rate
lambda_c = R_max / h gives reflection rate rho = lambda_c * A(alpha), A the
per-encounter acceptance = Eq. ReflXsection / Q with r normalised to its
maximum.  Competing with absorption mu0 over the path L = T / sin(alpha):
P(reflect) = rho / (mu0 + rho) * (1 - exp(-(mu0 + rho) L)).
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
from test_oracle_invariants import HC, pencil

DEG = math.pi / 180


# ---- mosaic densities per unit solid angle, as functions of v = 1 - cos(theta)

def dens_vmf(v, gamma):          # Eq. MF
    s = gamma / (2 * math.sqrt(2 * math.log(2)))
    return np.exp(-v / s**2) / (2 * math.pi * s**2 * (1 - math.exp(-2 / s**2)))


def dens_wl(v, gamma):           # Eq. WL
    return 1.0 / (math.pi * math.log(1 + (4 / gamma) ** 2)) / ((gamma / 2) ** 2 + 2 * v)


def dens_swl(v, gamma):          # Eq. SWL; cosh(G/2) - 1 = 2 sinh^2(G/4) avoids cancellation
    return math.sinh(gamma / 2) ** 2 / (4 * math.pi) / (2 * math.sinh(gamma / 4) ** 2 + v) ** 2


def dens_lorentz(v, gamma):
    # sphere density of the isotropic tilt with Lorentzian marginals of FWHM
    # Gamma (bivariate Cauchy in the tangent plane, tan(theta) = T)
    g = gamma / 2
    out = g / (2 * math.pi) / (v * (2 - v) + g * g * (1 - v) ** 2) ** 1.5
    return np.where(v < 1, out, 0.0)


DENS = {"gaussian_vmf": dens_vmf, "wrapped_lorentzian": dens_wl,
        "spherical_wrapped_lorentzian": dens_swl, "lorentzian": dens_lorentz}


def mosaic_density(mosaic):
    if mosaic["kind"] == "pseudo_voigt":
        e, g = mosaic["eta"], mosaic["fwhm"]
        return lambda v: e * dens_lorentz(v, g) + (1 - e) * dens_vmf(v, g)
    return lambda v: DENS[mosaic["kind"]](v, mosaic["fwhm"])


def rhat(curve):
    """Rocking curve normalised to its maximum, via the oracle's curve
    (pinned separately against the paper's widths and closed forms)."""
    peak = oracle.irc_value(curve, [0.0])[0]
    return lambda d: oracle.irc_value(curve, d) / peak


def v_of(alpha, psi, at):
    # 1 - cos(theta) with cos(theta) from Eq. ThetaPsi, written without
    # cancellation: 2 sin^2((alpha - at)/2) + 2 cos(alpha) cos(at) sin^2(psi/2)
    return 2 * np.sin((alpha - at) / 2) ** 2 + 2 * np.cos(alpha) * np.cos(at) * np.sin(psi / 2) ** 2


def psi_grid(width):
    a = np.linspace(0.0, 60 * width, 6001)
    b = np.geomspace(60 * width, math.pi, 3000)[1:]
    return np.concatenate([a, b])


def acceptance(alpha, alpha_b, mosaic, curve, lam, span=40, n_delta=801):
    """Eq. ReflXsection / Q: integral over Delta of rhat(Delta - Delta_M)
    cos(alpha_B + Delta) times the integral over psi of W(theta)."""
    W = mosaic_density(mosaic)
    shift = curve.get("shift", 0.0)
    d = np.linspace(shift - span * lam, shift + span * lam, n_delta)
    rh = rhat(curve)(d - shift)
    psi = psi_grid(mosaic["fwhm"] / math.cos(alpha) + 1e-12)
    inner = np.empty(len(d))
    for i, D in enumerate(d):
        at = alpha_b + D
        f = W(v_of(alpha, psi, at))
        inner[i] = 2 * integrate.trapezoid(f, psi)
    core = integrate.simpson(rh * np.cos(alpha_b + d) * inner, x=d)
    return core


def p_reflect(A, w, alpha):
    lam_c = w["rocking_curve"].get("peak", 0.5) / w["crystal"]["mfp"]
    if w["rocking_curve"]["kind"] == "table":
        lam_c = max(w["rocking_curve"]["table"]) / w["crystal"]["mfp"]
    rho = lam_c * A
    mu0 = w["crystal"]["mu0"]
    L = w["crystal"]["thickness"] / math.sin(alpha)
    return rho / (mu0 + rho) * (1 - math.exp(-(mu0 + rho) * L))


PV_IRC = dict(kind="pseudo_voigt", peak=0.5, shift=0.0, fwhm_g=50e-6, fwhm_l=8e-6)
G_IRC = dict(kind="gaussian", peak=0.5, shift=0.0, fwhm=50e-6)

CASES = [
    # mosaic, rocking curve, alpha - alpha_B
    (dict(kind="gaussian_vmf", fwhm=0.4 * DEG), G_IRC, 0.0),
    (dict(kind="gaussian_vmf", fwhm=0.4 * DEG), G_IRC, 0.2 * DEG),
    (dict(kind="gaussian_vmf", fwhm=0.4 * DEG), dict(G_IRC, shift=30e-6), -0.3 * DEG),
    (dict(kind="lorentzian", fwhm=0.1 * DEG), PV_IRC, 0.0),
    (dict(kind="lorentzian", fwhm=0.1 * DEG), PV_IRC, 0.05 * DEG),
    (dict(kind="pseudo_voigt", fwhm=0.1 * DEG, eta=0.3), PV_IRC, 0.03 * DEG),
    (dict(kind="wrapped_lorentzian", fwhm=0.1 * DEG), G_IRC, 0.0),
    (dict(kind="wrapped_lorentzian", fwhm=0.1 * DEG), G_IRC, 0.5 * DEG),
    (dict(kind="spherical_wrapped_lorentzian", fwhm=0.2 * DEG), PV_IRC, 0.1 * DEG),
]


@pytest.mark.parametrize("mosaic,curve,offset", CASES)
def test_reflection_rate_matches_eq_reflxsection(mosaic, curve, offset):
    energy = 8.0
    alpha_b = math.asin(HC / (6.708 * energy))
    alpha = alpha_b + offset
    lam = curve.get("fwhm") or oracle.pvoigt_params(curve["fwhm_g"], curve["fwhm_l"])[0]
    A = acceptance(alpha, alpha_b, mosaic, curve, lam)
    n = 400000
    w = pencil(alpha, energy, n=n)
    w["mosaic"] = dict(mosaic, eta=mosaic.get("eta", 0.0))
    w["rocking_curve"] = curve
    r = oracle.trace(w, images=False)
    assert r["counters"]["missed"] == 0
    got = r["counters"]["reflections"] / n
    p = p_reflect(A, w, alpha)
    assert abs(got - p) < 5 * math.sqrt(p * (1 - p) / n) + 1e-4 * p, (got, p, A)


def test_small_angle_limit_recovers_planar_gaussian():
    # sec. 2.2.3: for Lambda << Gamma and the von Mises-Fisher MDF, the psi
    # integral of Eq. SimpleReflXsection recovers Eq. SimpleZachXsection:
    # A(alpha) ~ (integral of rhat) * G(alpha - alpha_B; Gamma), Eq. Gaussian
    gamma = 0.4 * DEG
    alpha_b = math.asin(HC / (6.708 * 8.0))
    area = integrate.quad(lambda d: math.exp(-4 * math.log(2) * d * d / 50e-6**2), -1e-3, 1e-3)[0]
    for off in (0.0, 0.1 * DEG, 0.25 * DEG):
        A = acceptance(alpha_b + off, alpha_b, dict(kind="gaussian_vmf", fwhm=gamma), G_IRC, 50e-6)
        planar = math.sqrt(4 * math.log(2) / (math.pi * gamma**2)) * math.exp(-4 * math.log(2) * off**2 / gamma**2)
        assert A == pytest.approx(area * planar, rel=2e-3)


def _reflected_normals(w, alpha):
    r = oracle.trace(w, records=True, images=False)
    rec = r["records"]
    refl = rec["n_refl"] == 1
    k0 = np.array(w["source"]["axis"])
    k1 = rec["dir"][refl]
    n = k1 - k0
    n /= np.linalg.norm(n, axis=1)[:, None]
    return k0, n


def test_crystallite_azimuth_follows_method_two():
    # appendix A: the azimuth psi of the reflecting crystallite about the ray
    # is distributed as W(theta(psi)) integrated against the rocking curve
    # (method II), peaked at psi = 0; sampling theta first (method I) would
    # empty the psi = 0 bins
    energy, gamma, off = 8.0, 0.4 * DEG, 0.3 * DEG
    alpha_b = math.asin(HC / (6.708 * energy))
    alpha = alpha_b + off
    w = pencil(alpha, energy, n=1500000)
    w["mosaic"] = dict(kind="gaussian_vmf", fwhm=gamma, eta=0.0)
    k0, n = _reflected_normals(w, alpha)
    N = np.array([0.0, 0.0, 1.0])
    a = N - (N @ k0) * k0
    a /= np.linalg.norm(a)
    b = np.cross(k0, a)
    psi = np.arctan2(n @ b, n @ a)
    edges = np.linspace(-4 * gamma, 4 * gamma, 41)
    obs, _ = np.histogram(psi, edges)
    # predicted density: integral over Delta of rhat cos(alpha_B + Delta) W(theta(psi))
    d = np.linspace(-8 * 50e-6, 8 * 50e-6, 161)
    rh = np.exp(-4 * math.log(2) * d**2 / 50e-6**2) * np.cos(alpha_b + d)
    fine = np.linspace(edges[0], edges[-1], 40 * 200 + 1)
    dens = np.array([integrate.simpson(rh * dens_vmf(v_of(alpha, p, alpha_b + d), gamma), x=d)
                     for p in fine])
    cum = np.concatenate([[0], np.cumsum((dens[1:] + dens[:-1]) / 2 * np.diff(fine))])
    prob = np.diff(np.interp(edges, fine, cum))
    exp = prob / prob.sum() * obs.sum()
    keep = exp > 5
    o, e = obs[keep], exp[keep]
    assert stats.chisquare(o, e * o.sum() / e.sum()).pvalue > 1e-3
    mid = len(obs) // 2
    assert obs[mid - 1:mid + 1].min() > 0.9 * obs.max()


def test_rocking_angle_of_reflections_follows_the_curve_with_shift():
    # the accepted Delta = asin|k.n| - alpha_B follows the rocking curve
    # about its maximum Delta_M (the mosaic is flat on this scale)
    energy, gamma = 8.0, 0.4 * DEG
    alpha_b = math.asin(HC / (6.708 * energy))
    w = pencil(alpha_b, energy, n=600000)
    w["mosaic"] = dict(kind="gaussian_vmf", fwhm=gamma, eta=0.0)
    w["rocking_curve"] = dict(G_IRC, shift=20e-6)
    k0, n = _reflected_normals(w, alpha_b)
    delta = np.arcsin(np.abs(n @ k0)) - alpha_b
    s = 50e-6 / (2 * math.sqrt(2 * math.log(2)))
    assert stats.kstest(delta, stats.norm(20e-6, s).cdf).pvalue > 1e-3
