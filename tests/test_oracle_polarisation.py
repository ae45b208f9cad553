"""Pins of the oracle's polarisation tracking (sec. 2.1, 2.2.3, 2.2.4).

Closed forms: G = 1 - (p.k_s)^2 equals the paper's 1 - sin^2(2 theta)
sin^2(phi) for a polarisation at angle phi from n x k; averaged over phi it
is the paper's unpolarised factor (1 + cos^2(2 theta)) / 2; the polarisation
after a reflection is unit, normal to k_s and in the plane of p and k_s, and
a sigma polarisation (normal to the plane of incidence) is unchanged.
Whole traces: with no mosaic spread, sigma-polarised rays trace bit for bit
like unpolarised ones (G = 1 on every reflection), and pi-polarised rays
reflect (single reflection) only where the sigma-polarised ones do.
Statistics: polarisations uniform about the ray give the reflection count of
the unpolarised model whose peak carries G_unpol."""
import copy
import math

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import workloads as W


def _frame(theta, rng):
    """Unit k, crystallite normal n with k.n = -sin(theta), and the sigma
    and pi directions e1 = n x k / |n x k|, e2 = k x e1."""
    a = rng.normal(size=3)
    n = a / np.linalg.norm(a)
    t = np.cross(n, rng.normal(size=3))
    t /= np.linalg.norm(t)
    k = -math.sin(theta) * n + math.cos(theta) * t
    e1 = np.cross(n, k)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(k, e1)
    return k, n, e1, e2


@pytest.mark.parametrize("theta", [0.05, 0.2319, 0.6, 1.2])
def test_factor_and_update_closed_forms(theta):
    rng = np.random.default_rng(int(theta * 1000))
    for phi in np.linspace(0, 2 * math.pi, 13):
        k, n, e1, e2 = _frame(theta, rng)
        p = math.cos(phi) * e1 + math.sin(phi) * e2
        ks = k - 2 * np.dot(k, n) * n
        G, q = oracle.polarisation_reflect(p, ks)
        assert G == pytest.approx(1 - math.sin(2 * theta) ** 2 * math.sin(phi) ** 2, abs=1e-14)
        assert np.linalg.norm(q) == pytest.approx(1.0, abs=1e-14)
        assert abs(np.dot(q, ks)) < 1e-14
        assert abs(np.linalg.det(np.stack([q, p, ks]))) < 1e-14
    # sigma: unchanged
    k, n, e1, _ = _frame(theta, rng)
    G, q = oracle.polarisation_reflect(e1, k - 2 * np.dot(k, n) * n)
    assert G == pytest.approx(1.0, abs=1e-15) and np.allclose(q, e1, atol=1e-15)


@pytest.mark.parametrize("theta", [0.1, 0.2319, 0.7])
def test_average_over_phi_is_the_unpolarised_factor(theta):
    rng = np.random.default_rng(5)
    k, n, e1, e2 = _frame(theta, rng)
    ks = k - 2 * np.dot(k, n) * n
    phis = (np.arange(720) + 0.5) * (2 * math.pi / 720)
    g = [oracle.polarisation_reflect(math.cos(f) * e1 + math.sin(f) * e2, ks)[0] for f in phis]
    assert np.mean(g) == pytest.approx((1 + math.cos(2 * theta) ** 2) / 2, abs=1e-13)


def _flat_no_mosaic(max_refl):
    w = W.get("flat_hopg")
    w["mosaic"] = dict(kind="gaussian_vmf", fwhm=0.0, eta=0.0)
    w["crystal"]["max_refl"] = max_refl
    return w


def _sigma_pi(w, n):
    _, k, _ = oracle.source_sample(w, np.arange(n))
    N = np.array(w["crystal"]["normal"])
    s = np.cross(N, k)
    s /= np.linalg.norm(s, axis=1)[:, None]
    p = np.cross(k, s)
    return s, p


def test_sigma_polarisation_without_mosaic_is_unpolarised():
    w = _flat_no_mosaic(4)
    w["source"]["half_angle"] = 0.5 * W.DEG
    n = 200000
    sigma, _ = _sigma_pi(w, n)
    a = oracle.trace(w, n=n, records=True)["records"]
    b = oracle.trace(w, n=n, records=True, rays={"polarisations": sigma})["records"]
    assert a.tobytes() == b.tobytes()
    assert a["n_refl"].sum() > 100


def test_pi_reflections_are_a_subset_of_sigma_reflections():
    w = _flat_no_mosaic(1)
    w["source"]["half_angle"] = 0.5 * W.DEG
    n = 200000
    sigma, pi = _sigma_pi(w, n)
    s = oracle.trace(w, n=n, records=True, rays={"polarisations": sigma})["records"]
    p = oracle.trace(w, n=n, records=True, rays={"polarisations": pi})["records"]
    rs, rp = s["n_refl"] == 1, p["n_refl"] == 1
    assert rs.sum() > 200
    assert np.all(rs[rp])               # pi reflects only where sigma does
    assert 0.5 * rs.sum() < rp.sum() < rs.sum()


def test_random_polarisations_match_the_unpolarised_factor():
    w = W.get("flat_hopg")
    n = 600000
    _, k, e = oracle.source_sample(w, np.arange(n))
    rng = np.random.default_rng(8)
    a = rng.normal(size=(n, 3))
    a -= np.sum(a * k, axis=1)[:, None] * k
    p = a / np.linalg.norm(a, axis=1)[:, None]
    pol = oracle.trace(w, n=n, rays={"polarisations": p})["counters"]["reflections"]
    # the unpolarised model with the peak times G_unpol at the mean energy
    ab = math.asin(12.398419843320026 / (w["crystal"]["two_d"] * 8.0))
    g = (1 + math.cos(2 * ab) ** 2) / 2
    w2 = copy.deepcopy(w)
    w2["rocking_curve"]["peak"] *= g
    unp = oracle.trace(w2, n=n)["counters"]["reflections"]
    assert pol > 2000
    assert abs(pol - unp) < 4 * math.sqrt(pol + unp), (pol, unp)
    plain = oracle.trace(w, n=n)["counters"]["reflections"]
    assert plain - pol > 4 * math.sqrt(pol + plain)
