"""Pins of the oracle's crystal geometry (sec. 2.2: FlatCrystal and
CylinderCrystal entry and inside tests; sec. 2.3 detector) by brute force:
an independent inside predicate, bisection along rays, and a direct
ray-surface search."""
import math

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import workloads as W


def inside(c, p):
    """Independent point-in-crystal predicate written from the geometry."""
    p = np.asarray(p, float)
    if c["geometry"] == "flat":
        N, e1 = np.array(c["normal"]), np.array(c["e1"])
        e2 = np.cross(N, e1)
        d = p - np.array(c["centre"])
        return (-c["thickness"] <= d @ N <= 0 and abs(d @ e1) <= c["length"] / 2
                and abs(d @ e2) <= c["width"] / 2)
    a = np.array(c["axis_dir"])
    b1 = np.array(c["ref_dir"])
    b2 = np.cross(a, b1)
    d = p - np.array(c["axis_pt"])
    z = d @ a
    rho = d - z * a
    r = np.linalg.norm(rho)
    phi = math.atan2(rho @ b2, rho @ b1)
    dphi = (phi - c["phi_c"] + math.pi) % (2 * math.pi) - math.pi
    return (c["radius"] <= r <= c["radius"] + c["thickness"] and abs(z - c["z_c"]) <= c["length"] / 2
            and abs(dphi) <= c["width"] / (2 * c["radius"]))


def random_inside(c, rng):
    if c["geometry"] == "flat":
        N, e1 = np.array(c["normal"]), np.array(c["e1"])
        e2 = np.cross(N, e1)
        return (np.array(c["centre"]) - rng.uniform(0, c["thickness"]) * N
                + rng.uniform(-0.5, 0.5) * c["length"] * e1 + rng.uniform(-0.5, 0.5) * c["width"] * e2)
    a = np.array(c["axis_dir"])
    b1 = np.array(c["ref_dir"])
    b2 = np.cross(a, b1)
    r = c["radius"] + rng.uniform(0, c["thickness"])
    phi = c["phi_c"] + rng.uniform(-0.5, 0.5) * c["width"] / c["radius"]
    z = c["z_c"] + rng.uniform(-0.5, 0.5) * c["length"]
    return np.array(c["axis_pt"]) + z * a + r * (math.cos(phi) * b1 + math.sin(phi) * b2)


def random_dir(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("name", ["flat_hopg", "von_hamos_hapg"])
def test_exit_distance_by_bisection(name):
    w = W.get(name)
    c = w["crystal"]
    rng = np.random.default_rng(3)
    for _ in range(400):
        p = random_inside(c, rng)
        if not inside(c, p):
            continue
        k = random_dir(rng)
        d = oracle.exit_distance(w, p, k)
        eps = 1e-9
        assert inside(c, p + max(d - eps, 0) * k)
        assert not inside(c, p + (d + eps) * k)
        # the segment before the exit stays inside (sampled)
        for f in (0.25, 0.5, 0.9):
            assert inside(c, p + f * d * k)


def inside_many(c, P):
    """Vectorised form of `inside` for an (n, 3) array of points."""
    if c["geometry"] == "flat":
        N, e1 = np.array(c["normal"]), np.array(c["e1"])
        e2 = np.cross(N, e1)
        d = P - np.array(c["centre"])
        z = d @ N
        return ((z >= -c["thickness"]) & (z <= 0) & (np.abs(d @ e1) <= c["length"] / 2)
                & (np.abs(d @ e2) <= c["width"] / 2))
    a = np.array(c["axis_dir"])
    b1 = np.array(c["ref_dir"])
    b2 = np.cross(a, b1)
    d = P - np.array(c["axis_pt"])
    z = d @ a
    rho = d - z[:, None] * a
    r = np.linalg.norm(rho, axis=1)
    phi = np.arctan2(rho @ b2, rho @ b1)
    dphi = (phi - c["phi_c"] + math.pi) % (2 * math.pi) - math.pi
    return ((r >= c["radius"]) & (r <= c["radius"] + c["thickness"])
            & (np.abs(z - c["z_c"]) <= c["length"] / 2) & (np.abs(dphi) <= c["width"] / (2 * c["radius"])))


def _first_crossing(w, o, k):
    """Brute-force search along the ray for the first point inside the
    crystal, refined by bisection; None if the ray never enters."""
    c = w["crystal"]
    ts = np.linspace(0.0, 600.0, 300001)
    ins = inside_many(c, o + ts[:, None] * k)
    if not ins.any():
        return None
    i = int(np.argmax(ins))
    lo, hi = ts[i - 1], ts[i]
    for _ in range(60):
        m = 0.5 * (lo + hi)
        if inside(c, o + m * k):
            hi = m
        else:
            lo = m
    return hi


def _on_front_face(c, p, tol=1e-6):
    if c["geometry"] == "flat":
        return abs((p - np.array(c["centre"])) @ np.array(c["normal"])) < tol
    d = p - np.array(c["axis_pt"])
    rho = d - (d @ np.array(c["axis_dir"])) * np.array(c["axis_dir"])
    return abs(np.linalg.norm(rho) - c["radius"]) < tol


@pytest.mark.parametrize("name", ["flat_hopg", "von_hamos_hapg"])
def test_entry_decision_brute_force(name):
    # the oracle's hit / miss decision and entry distance against a direct
    # march along the ray with the independent inside predicate
    w = W.get(name)
    ids = np.arange(200)
    o, k, _ = oracle.source_sample(w, ids)
    rec, _ = oracle.trace_ids(w, ids)
    c = w["crystal"]
    for i in range(len(ids)):
        t = _first_crossing(w, o[i], k[i])
        if t is not None and not _on_front_face(c, o[i] + t * k[i]):
            t = None      # entry through a side face is not modelled: a miss
        if rec["status"][i] == oracle.MISS:
            assert t is None
        else:
            assert t is not None
            t_or = np.linalg.norm(rec["entry"][i] - o[i])
            assert abs(t - t_or) < 1e-8


@pytest.mark.parametrize("name,frac", [("flat_hopg", 0.608), ("von_hamos_hapg", 0.513)])
def test_hit_fraction_is_solid_angle_fraction(name, frac):
    # fraction of the cone subtended by the crystal front face, by a plain
    # numpy Monte Carlo over directions with the independent geometry
    w = W.get(name)
    c = w["crystal"]
    s = w["source"]
    rng = np.random.default_rng(5)
    n = 40000
    th_max = s["half_angle"]
    ct = 1 - rng.uniform(0, 1 - math.cos(th_max), n)
    st = np.sqrt(1 - ct * ct)
    ph = rng.uniform(0, 2 * math.pi, n)
    a, b1 = np.array(s["axis"]), np.array(s["b1"])
    b2 = np.cross(a, b1)
    k = ct[:, None] * a + st[:, None] * (np.cos(ph)[:, None] * b1 + np.sin(ph)[:, None] * b2)
    o = np.array(s["origin"])
    if c["geometry"] == "flat":
        N = np.array(c["normal"])
        t = -((o - c["centre"]) @ N) / (k @ N)
        h = o + t[:, None] * k - c["centre"]
        e2 = np.cross(N, c["e1"])
        hit = (t > 0) & (np.abs(h @ c["e1"]) <= c["length"] / 2) & (np.abs(h @ e2) <= c["width"] / 2)
    else:
        ax = np.array(c["axis_dir"])
        kp = k - np.outer(k @ ax, ax)
        t = c["radius"] / np.linalg.norm(kp, axis=1)    # source on the axis
        h = o + t[:, None] * k
        z = h @ ax
        phi = np.arctan2(h @ np.cross(ax, c["ref_dir"]), h @ np.array(c["ref_dir"]))
        hit = (np.abs(z - c["z_c"]) <= c["length"] / 2) & (np.abs(phi - c["phi_c"]) <= c["width"] / (2 * c["radius"]))
    expect = hit.mean()
    r = oracle.trace(w, n=40000, images=False)
    got = 1 - r["counters"]["missed"] / r["counters"]["emitted"]
    sig = math.sqrt(2 * expect * (1 - expect) / n)
    assert abs(got - expect) < 5 * sig
    assert abs(expect - frac) < 0.01


def test_detector_pixel_mapping():
    # a ray through a known point of the detector plane lands in the pixel
    # of floor(coordinate / pitch + n / 2); the lower pixel edge belongs to it
    w = W.get("flat_hopg")
    d = w["detector"]
    P, u, v, n = (np.array(d[x]) for x in ("centre", "u", "v", "normal"))
    r = oracle.trace(w, n=30000, records=True, images=True)
    rec = r["records"]
    det = rec["detected"] == 1
    assert det.sum() > 100
    h = rec["end"][det]
    assert np.abs((h - P) @ n).max() < 1e-9
    i = np.floor((h - P) @ u / d["pitch"] + d["nx"] / 2).astype(int)
    j = np.floor((h - P) @ v / d["pitch"] + d["ny"] / 2).astype(int)
    assert np.array_equal(i, rec["pix_i"][det]) and np.array_equal(j, rec["pix_j"][det])
    assert np.all(rec["pix_i"][~det] == -1)


@pytest.mark.parametrize("name", ["flat_hopg", "von_hamos_hapg"])
def test_entry_points_on_front_face(name):
    w = W.get(name)
    r = oracle.trace(w, n=20000, records=True, images=False)
    rec = r["records"]
    c = w["crystal"]
    hit = rec["status"] != oracle.MISS
    e = rec["entry"][hit]
    if c["geometry"] == "flat":
        zeta = (e - np.array(c["centre"])) @ np.array(c["normal"])
        assert np.abs(zeta).max() < 1e-12
    else:
        d = e - np.array(c["axis_pt"])
        rho = d - np.outer(d @ np.array(c["axis_dir"]), c["axis_dir"])
        assert np.abs(np.linalg.norm(rho, axis=1) - c["radius"]).max() < 1e-11
    assert np.all(np.isnan(rec["entry"][~hit]))
