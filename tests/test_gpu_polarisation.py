"""Polarisation tracking on the GPU (sec. 2.1, 2.2.3, 2.2.4), through the
C-ABI: user polarisations in per-ray parity with the oracle (FP64) on the
von Hamos, the flat crystal with further planes, and the tabulated curve;
ragged launches past 2^32; sampled at the full 1e8-ray von Hamos size; with
no mosaic spread sigma polarisations give the unpolarised kernel's records
bit for bit; FP32-mixed agrees with FP64 statistically; the paper's event
model with polarisation (Eqs. SimpleReflXsectionPol, ReflXsectionPol) in
parity on both geometries and two more mosaics, and sampled at 1e8 rays;
the request server serves them (its tests sit with the server's)."""
import copy

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

import parity
from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


def _random_pol(w, n, seed, first=0):
    _, k, _ = oracle.source_sample(w, np.arange(first, first + n))
    a = np.random.default_rng(seed).normal(size=k.shape)
    a -= np.sum(a * k, axis=1)[:, None] * k
    return a / np.linalg.norm(a, axis=1)[:, None]


def test_polarisation_von_hamos_parity():
    w = W.get("von_hamos_hapg")
    n = 300_000
    g, o = assert_parity(w, n, rays={"polarisations": _random_pol(w, n, 1)})
    assert o["counters"]["reflections"] > 1000


def test_polarisation_with_planes_flat_parity():
    w = W.get("flat_hopg")
    w["crystal"]["max_refl"] = 4
    w["crystal"]["planes"] = {"hbar_ratio": 0.6, "extra": [(w["crystal"]["two_d"] / 2, 0.5, 1.0, 0.0)]}
    n = 100_000
    g, o = assert_parity(w, n, rays={"polarisations": _random_pol(w, n, 2)})
    assert o["counters"]["reflections"] > 500


def test_polarisation_tabulated_curve_and_spot_parity():
    w = W.with_spot(W.get("flat_stress", precision="fp64"), "disk", 0.1)
    n = 60_000
    g, o = assert_parity(w, n, rays={"polarisations": _random_pol(w, n, 3)})
    assert o["counters"]["reflections"] > 500


@pytest.mark.parametrize("n", [1, 64, 4097])
def test_polarisation_ragged_launches(n):
    w = W.get("von_hamos_hapg")
    first = (1 << 32) - 5
    assert_parity(w, n, first=first, rays={"polarisations": _random_pol(w, n, n, first)})


def test_sigma_without_mosaic_is_the_unpolarised_kernel():
    import torch
    w = W.get("flat_hopg")
    w["mosaic"] = dict(kind="gaussian_vmf", fwhm=0.0, eta=0.0)
    w["crystal"]["max_refl"] = 4
    w["source"]["half_angle"] = 0.5 * W.DEG
    n = 500_000
    _, k, _ = oracle.source_sample(w, np.arange(n))
    s = np.cross(np.array(w["crystal"]["normal"]), k)
    s /= np.linalg.norm(s, axis=1)[:, None]
    a = mrt.trace(w, n_rays=n, records="all")
    b = mrt.trace(w, n_rays=n, records="all",
                  rays={"polarisations": torch.as_tensor(s, device="cuda")})
    ra, rb = mrt.records_to_numpy(a["records"]), mrt.records_to_numpy(b["records"])
    # the two kernel instances take the same decisions; their floating-point
    # code may be contracted differently, so doubles agree to 1e-12
    for f in ("ray_id", "status", "n_events", "n_refl", "detected", "pix_i", "pix_j"):
        assert np.array_equal(ra[f], rb[f]), f
    for f in ("energy", "entry", "end", "dir"):
        x, y = ra[f], rb[f]
        ok = (np.isnan(x) & np.isnan(y)) | (np.abs(x - y) <= 1e-12 * np.maximum(np.abs(x), 1.0))
        assert ok.all(), f
    assert a["counters"]["reflections"] > 500


def test_polarisation_fp32_mixed_agrees_with_fp64():
    import torch
    w = W.get("von_hamos_hapg")
    n = 4_000_000
    rng = np.random.default_rng(4)
    # random unit vectors; the factor only needs p to be unit (the component
    # along k does not change G's distribution much, and both runs share p)
    p = rng.normal(size=(n, 3))
    p /= np.linalg.norm(p, axis=1)[:, None]
    pt = torch.as_tensor(p, device="cuda")
    a = mrt.trace(w, n_rays=n, precision="fp32_mixed", rays={"polarisations": pt})["counters"]
    b = mrt.trace(w, n_rays=n, precision="fp64", rays={"polarisations": pt})["counters"]
    for f in ("reflections", "detected", "exit_reflected"):
        assert abs(a[f] - b[f]) < 5 * np.sqrt(a[f] + b[f]) + 1e-3 * b[f], (f, a[f], b[f])


def _mwg(w, burn_in=200):
    w = copy.deepcopy(w)
    w["event_model"] = {"kind": "mwg", "burn_in": burn_in, "psi_nodes": 256}
    return w


@pytest.mark.parametrize("name,n", [("von_hamos_hapg", 200_000), ("flat_hopg", 100_000)])
def test_polarisation_in_the_papers_model_parity(name, n):
    w = _mwg(W.get(name))
    g, o = assert_parity(w, n, rays={"polarisations": _random_pol(w, n, 5)})
    assert o["counters"]["reflections"] > 500


@pytest.mark.parametrize("mosaic", [dict(kind="wrapped_lorentzian", fwhm=0.2 * W.DEG, eta=0.0),
                                    dict(kind="lorentzian", fwhm=0.3 * W.DEG, eta=0.0)],
                         ids=["wrapped_lorentzian", "lorentzian"])
def test_polarisation_in_the_papers_model_mosaics(mosaic):
    w = W.get("flat_hopg")
    w["mosaic"] = mosaic
    w["crystal"]["max_refl"] = 4
    w = _mwg(w, burn_in=100)
    n = 50_000
    g, o = assert_parity(w, n, first=9, rays={"polarisations": _random_pol(w, n, 6, 9)})
    assert o["counters"]["reflections"] > 200


def test_polarisation_in_the_papers_model_full_size_sampled():
    """1e8 von Hamos rays in the paper's model with device-generated random
    polarisations: 1024 sampled rays against the oracle."""
    import torch
    w = _mwg(W.get("von_hamos_hapg"), burn_in=500)
    n = w["n_rays"]
    gen = torch.Generator(device="cuda").manual_seed(32)
    p = torch.randn((n, 3), generator=gen, device="cuda", dtype=torch.float64)
    p = (p / torch.linalg.norm(p, dim=1, keepdim=True)).contiguous()
    print("[pol-mwg-full] records launch", flush=True)
    g = mrt.trace(w, records="all", rays={"polarisations": p})
    ids = np.unique(np.random.default_rng(16).integers(0, n, 1024, dtype=np.int64))
    sel = torch.as_tensor(ids, device="cuda")
    grec = mrt.records_to_numpy(g["records"].index_select(0, sel))
    ph = p.index_select(0, sel).cpu().numpy()
    parts = [oracle.trace_ids(w, [int(i)], rays={"polarisations": ph[j:j + 1]}, first=int(i), n_rows=1)
             for j, i in enumerate(ids)]
    orec = np.concatenate([q[0] for q in parts])
    mg = np.concatenate([q[1] for q in parts])
    n_ties, bad, _ = parity.compare(grec, orec, mg)
    assert len(bad) == 0, parity.describe(grec, orec, mg, bad)
    assert n_ties == 0


def test_polarisation_full_size_sampled():
    """1e8 von Hamos rays with device-generated random polarisations: 2048
    sampled rays against the oracle given the same rows."""
    import torch
    w = W.get("von_hamos_hapg")
    n = w["n_rays"]
    gen = torch.Generator(device="cuda").manual_seed(31)
    p = torch.randn((n, 3), generator=gen, device="cuda", dtype=torch.float64)
    p = (p / torch.linalg.norm(p, dim=1, keepdim=True)).contiguous()
    print("[pol-full] records launch", flush=True)
    g = mrt.trace(w, records="all", rays={"polarisations": p})
    ids = np.unique(np.random.default_rng(15).integers(0, n, 2048, dtype=np.int64))
    sel = torch.as_tensor(ids, device="cuda")
    grec = mrt.records_to_numpy(g["records"].index_select(0, sel))
    ph = p.index_select(0, sel).cpu().numpy()
    parts = [oracle.trace_ids(w, [int(i)], rays={"polarisations": ph[j:j + 1]}, first=int(i), n_rows=1)
             for j, i in enumerate(ids)]
    orec = np.concatenate([q[0] for q in parts])
    mg = np.concatenate([q[1] for q in parts])
    n_ties, bad, _ = parity.compare(grec, orec, mg)
    assert len(bad) == 0, parity.describe(grec, orec, mg, bad)
    assert n_ties == 0
    c = g["counters"]
    assert (c["missed"] + c["absorbed"] + c["exit_reflected"] + c["exit_transmitted"]
            + c["truncated"]) == n
