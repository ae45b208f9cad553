"""Pins of the oracle's source extensions (sec. 2.1, sec. 4.2): the finite
source spot and the user ray arrays.

Spots: the origin offsets of a Gaussian spot are two independent normals of
the stated standard deviations in the spot plane (Kolmogorov-Smirnov against
the normal CDF, zero correlation, nothing out of the plane); a disk spot has
r^2 / R^2 and the polar angle uniform and nothing past the rim; a spot
changes neither directions nor energies, and a spot of size zero is the point
source exactly.  User arrays: feeding back the oracle's own sampled origins,
directions and energies (at an offset first ray id) reproduces every record
bit for bit; a user ray that cannot reflect crosses a flat slab along the
straight line computed by hand here."""
import copy
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2503_16955_amd import workloads as W

U = np.array([0.6, 0.8, 0.0])
V = np.array([0.0, 0.0, 1.0])


def _spot(w, kind, sigma, u=U, v=V):
    w = copy.deepcopy(w)
    w["source"]["spot"] = dict(kind=kind, u=list(u), v=list(v), sigma=sigma)
    return w


def _offsets(w, n=40000, seed=None):
    o, k, e = oracle.source_sample(w, np.arange(n), seed=seed)
    d = o - np.array(w["source"]["origin"])
    return d, k, e


def test_gaussian_spot_offsets_are_independent_normals():
    w = _spot(W.get("von_hamos_hapg"), "gaussian", [0.010, 0.004])
    d, _, _ = _offsets(w)
    x, y = d @ U, d @ V
    normal = np.cross(U, V)
    assert np.abs(d @ normal).max() < 1e-15
    assert stats.kstest(x / 0.010, "norm").pvalue > 1e-3
    assert stats.kstest(y / 0.004, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(x, y)[0, 1]) < 0.02
    # |(x/sx, y/sy)|^2 is chi-square with two degrees of freedom
    assert stats.kstest((x / 0.010) ** 2 + (y / 0.004) ** 2, "chi2", args=(2,)).pvalue > 1e-3


def test_disk_spot_is_uniform_over_the_disk():
    R = 0.005
    w = _spot(W.get("flat_hopg"), "disk", [R, 0.0])
    d, _, _ = _offsets(w)
    x, y = d @ U, d @ V
    r2 = (x * x + y * y) / (R * R)
    assert r2.max() <= 1.0 + 1e-12
    assert stats.kstest(r2, "uniform").pvalue > 1e-3
    phi = np.mod(np.arctan2(y, x), 2 * math.pi) / (2 * math.pi)
    assert stats.kstest(phi, "uniform").pvalue > 1e-3
    # equal areas: the quadrants hold a quarter each
    q = np.histogram(phi, bins=4, range=(0, 1))[0] / len(phi)
    assert np.allclose(q, 0.25, atol=0.01)


@pytest.mark.parametrize("kind", ["gaussian", "disk"])
def test_spot_keeps_directions_and_energies(kind):
    base = W.get("von_hamos_hapg")
    o0, k0, e0 = oracle.source_sample(base, np.arange(3000))
    o1, k1, e1 = oracle.source_sample(_spot(base, kind, [0.01, 0.01]), np.arange(3000))
    assert np.array_equal(k0, k1) and np.array_equal(e0, e1)
    assert not np.array_equal(o0, o1)


@pytest.mark.parametrize("kind", ["gaussian", "disk"])
def test_spot_of_size_zero_is_the_point_source(kind):
    base = W.get("flat_hopg")
    a = oracle.trace(base, n=20000, records=True)
    b = oracle.trace(_spot(base, kind, [0.0, 0.0]), n=20000, records=True)
    assert a["records"].tobytes() == b["records"].tobytes()


@pytest.mark.parametrize("name,spot", [("von_hamos_hapg", None),
                                       ("von_hamos_hapg", ("gaussian", [0.01, 0.02])),
                                       ("flat_stress", ("disk", [0.05, 0.0]))])
def test_user_arrays_reproduce_the_sampled_rays(name, spot):
    w = W.get(name)
    if spot:
        w = _spot(w, *spot)
    first, n = 12345, 30000
    want = oracle.trace(w, first=first, n=n, records=True)
    o, k, e = oracle.source_sample(w, np.arange(first, first + n))
    # each array alone, then all three: the point-source workload with the
    # sampled fields supplied reproduces the same records
    plain = copy.deepcopy(w)
    plain["source"].pop("spot", None)
    for rays in (dict(origins=o), dict(directions=k, origins=o), dict(energies=e, origins=o),
                 dict(origins=o, directions=k, energies=e)):
        got = oracle.trace(plain, first=first, n=n, records=True, rays=rays)
        assert got["records"].tobytes() == want["records"].tobytes(), sorted(rays)
        assert np.array_equal(got["counts"], want["counts"])
    # ids looked up one by one use the same rows
    ids = np.array([first, first + 7, first + n - 1])
    rec, _ = oracle.trace_ids(plain, ids, rays=dict(origins=o, directions=k, energies=e),
                              first=first, n_rows=n)
    assert rec.tobytes() == want["records"][ids - first].tobytes()
    with pytest.raises(ValueError):
        oracle.trace_ids(plain, [first + n], rays=dict(energies=e), first=first, n_rows=n)


def test_user_ray_crosses_a_slab_along_the_hand_computed_line():
    # flat slab, no absorption, energies below the Bragg cutoff: a user ray
    # enters the front face and leaves through the back face on a straight line
    w = W.get("flat_hopg")
    c = w["crystal"]
    c["mu0"] = 0.0
    N, e1 = np.array(c["normal"]), np.array(c["e1"])
    e2 = np.cross(N, e1)
    C0 = np.array(c["centre"])
    rng = np.random.default_rng(3)
    n = 200
    # aim at points of the front face from 10 mm above it
    a = rng.uniform(-0.3, 0.3, n) * c["length"]
    b = rng.uniform(-0.3, 0.3, n) * c["width"]
    target = C0 + a[:, None] * e1 + b[:, None] * e2
    tilt = rng.uniform(0.2, 1.2, n)
    az = rng.uniform(0, 2 * math.pi, n)
    k = -np.cos(tilt)[:, None] * N + np.sin(tilt)[:, None] * (np.cos(az)[:, None] * e1
                                                               + np.sin(az)[:, None] * e2)
    o = target - 10.0 / np.cos(tilt)[:, None] * k
    E = np.full(n, 1.0)    # 2d sin(alpha) < hc / E: no Bragg angle
    rec = oracle.trace(w, n=n, records=True, rays=dict(origins=o, directions=k, energies=E))["records"]
    assert np.all(rec["status"] == oracle.EXIT_TRANSMITTED)
    assert np.allclose(rec["entry"], target, atol=1e-9)
    back = target + (c["thickness"] / np.cos(tilt))[:, None] * k
    inside = np.all(np.abs((back - C0) @ np.stack([e1, e2]).T) <= [c["length"] / 2, c["width"] / 2],
                    axis=1)
    assert inside.sum() > 150
    assert np.allclose(rec["end"][inside], back[inside], atol=1e-9)
    assert np.array_equal(rec["dir"], k) and np.array_equal(rec["energy"], E)
