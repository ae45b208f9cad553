"""Parity of the HIP kernel of the paper's own event model (sec. 2.2.3,
2.2.4; FP64) with the oracle's, through the C-ABI: per-ray records exact
(status, events, reflections, pixel; doubles within 1e-12 relative) and
images bit-exact except counted ties, on every mosaic distribution and
rocking curve, both geometries, the sampler's and quadrature's extreme
settings, the edge cases of the method, and a sampled check at the full
1e8-ray von Hamos size; the wave schedule (sampler batch, refill) does not
change any result.
"""
import copy

import numpy as np
import pytest

import oracle
from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

import parity
from test_gpu_parity import _flat_variant, assert_parity

pytestmark = pytest.mark.gpu

DEG = np.pi / 180


def mwg(w, burn_in=300, psi_nodes=256):
    w = copy.deepcopy(w)
    w["event_model"] = {"kind": "mwg", "burn_in": burn_in, "psi_nodes": psi_nodes}
    return w


def test_mwg_flat_hopg_full_config():
    g, o = assert_parity(mwg(W.get("flat_hopg"), burn_in=500), 100_000)
    assert o["counters"]["reflections"] > 1000


def test_mwg_von_hamos():
    g, o = assert_parity(mwg(W.get("von_hamos_hapg"), burn_in=500), 300_000)
    assert o["counters"]["reflections"] > 3000


def test_mwg_flat_stress():
    # Lorentzian mosaic, tabulated rocking curve, up to 8 reflections
    g, o = assert_parity(mwg(W.get("flat_stress", precision="fp64"), burn_in=200), 60_000)
    assert o["counters"]["reflections"] > 500


MOSAICS = {
    "gaussian_vmf": dict(kind="gaussian_vmf", fwhm=0.4 * DEG, eta=0.0),
    "lorentzian": dict(kind="lorentzian", fwhm=0.2 * DEG, eta=0.0),
    "pseudo_voigt": dict(kind="pseudo_voigt", fwhm=0.3 * DEG, eta=0.4),
    "wrapped_lorentzian": dict(kind="wrapped_lorentzian", fwhm=0.2 * DEG, eta=0.0),
    "spherical_wrapped_lorentzian": dict(kind="spherical_wrapped_lorentzian", fwhm=0.3 * DEG, eta=0.0),
    "gaussian": dict(kind="gaussian", fwhm=0.3 * DEG, eta=0.0),
}
IRCS = {
    "gaussian": dict(kind="gaussian", peak=0.5, shift=10e-6, fwhm=50e-6),
    "pseudo_voigt": dict(kind="pseudo_voigt", peak=0.5, shift=-5e-6, fwhm_g=50e-6, fwhm_l=8e-6),
    "lorentzian": dict(kind="lorentzian", peak=0.4, shift=0.0, fwhm=30e-6),
    "box": dict(kind="box", peak=0.3, shift=0.0, fwhm=60e-6),
    "table": dict(kind="table", peak=0.0, shift=0.0, x_min=-200e-6, x_max=200e-6,
                  table=list(0.5 * np.exp(-np.linspace(-5, 5, 129) ** 2))),
}


@pytest.mark.parametrize("kind", sorted(MOSAICS))
def test_mwg_mosaic_kinds(kind):
    g, o = assert_parity(mwg(_flat_variant(mosaic=MOSAICS[kind]), burn_in=200), 30_000)
    assert o["counters"]["reflections"] > 50


@pytest.mark.parametrize("kind", sorted(IRCS))
def test_mwg_rocking_curve_kinds(kind):
    g, o = assert_parity(mwg(_flat_variant(irc=IRCS[kind]), burn_in=200), 30_000)
    assert o["counters"]["reflections"] > 50


@pytest.mark.parametrize("burn_in,psi_nodes", [(0, 256), (1, 1), (50, 2048), (1000, 64)])
def test_mwg_sampler_and_quadrature_settings(burn_in, psi_nodes):
    # no burn-in (the sampler's start), a single psi interval, the largest
    # grid, and a long chain
    w = mwg(W.get("von_hamos_hapg"), burn_in=burn_in, psi_nodes=psi_nodes)
    # A chain that ends at its start psi = 0 (always without burn-in, often
    # after one sweep) puts the crystallite in the plane of the ray and the
    # surface normal, which holds the cylinder axis and the on-axis source:
    # the reflected ray lands exactly on the detector's central row edge (a
    # pixel-edge tie).  Half a pixel of detector offset moves that line to
    # mid-row.
    d = w["detector"]
    d["centre"] = [c + 0.5 * d["pitch"] * v for c, v in zip(d["centre"], d["v"])]
    g, o = assert_parity(w, 20_000)
    if burn_in == 0:
        rec = o["records"]
        refl = rec[(rec["n_refl"] > 0) & (rec["detected"] == 1)]
        assert len(refl) > 20 and np.all(refl["pix_j"] == w["detector"]["ny"] // 2 - 1)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1000, 4097])
def test_mwg_tiny_and_ragged_launches(n):
    assert_parity(mwg(W.get("von_hamos_hapg"), burn_in=100), n, first=777)


def test_mwg_edge_cases():
    # truncation, no reflection budget, no Bragg angle, no attenuation, rays
    # past 2^32, all misses
    w = mwg(W.get("flat_hopg"), burn_in=100)
    g, o = assert_parity(w, 20_000, max_events=1)
    assert o["counters"]["truncated"] > 100
    g, o = assert_parity(mwg(_flat_variant(max_refl=0), burn_in=100), 20_000)
    assert o["counters"]["reflections"] == 0
    w2 = copy.deepcopy(w)
    w2["source"].update(e_min=1.0, e_max=1.5)
    g, o = assert_parity(w2, 20_000)
    assert o["counters"]["reflections"] == 0 and o["counters"]["absorbed"] > 0
    g, o = assert_parity(mwg(_flat_variant(mu0=0.0), burn_in=100), 20_000)
    assert o["counters"]["absorbed"] == 0
    assert_parity(w, 5000, first=(1 << 32) - 2500, seed=(1 << 63) + 5)
    w3 = copy.deepcopy(w)
    w3["source"]["axis"] = [-a for a in w3["source"]["axis"]]
    g, o = assert_parity(w3, 5000)
    assert o["counters"]["missed"] == 5000


def test_mwg_schedule_does_not_change_results():
    """Images and records do not depend on the sampler batch, the refill
    threshold or the launch shape."""
    w = mwg(W.get("von_hamos_hapg"), burn_in=200)
    n = 200_000
    ref = mrt.trace(w, n_rays=n, records="all")
    rc, re = mrt.image_to_numpy(ref["counts"], ref["energy"])
    rr = mrt.records_to_numpy(ref["records"])
    for batch, refill, grid, block in [(1, 0, 0, 0), (64, 0, 0, 0), (5, 1, 0, 0), (32, 64, 7, 128),
                                       (17, 3, 1, 64)]:
        print(f"[mwg-shape] batch={batch} refill={refill} grid={grid} block={block}", flush=True)
        g = mrt.trace(w, n_rays=n, records="all", mwg_batch=batch, refill_idle=refill,
                      grid_blocks=grid, block_threads=block)
        gc, ge = mrt.image_to_numpy(g["counts"], g["energy"])
        assert np.array_equal(gc, rc) and np.array_equal(ge, re)
        assert mrt.records_to_numpy(g["records"]).tobytes() == rr.tobytes()


def test_mwg_von_hamos_full_size_sampled():
    """1e8 von Hamos rays in the paper's model with 500 sweeps per
    reflection: 4096 sampled ray ids against the oracle, the benchmark's
    no-records kernel gives the image the records imply, photons conserved."""
    import torch
    w = mwg(W.get("von_hamos_hapg"), burn_in=500)
    n = w["n_rays"]
    nx, ny = w["detector"]["nx"], w["detector"]["ny"]
    print("[mwg-full] records launch", flush=True)
    g = mrt.trace(w, records="all")
    c = g["counters"]
    assert c["emitted"] == n
    assert (c["missed"] + c["absorbed"] + c["exit_reflected"] + c["exit_transmitted"]
            + c["truncated"]) == n
    rng = np.random.default_rng(11)
    ids = np.unique(rng.integers(0, n, 4096, dtype=np.int64))
    rec_dev = g["records"]
    sample = rec_dev.index_select(0, torch.as_tensor(ids, device=rec_dev.device))
    grec = mrt.records_to_numpy(sample)
    orec, mg = oracle.trace_ids(w, ids)
    n_ties, bad, _ = parity.compare(grec, orec, mg)
    assert len(bad) == 0, parity.describe(grec, orec, mg, bad)
    assert n_ties == 0
    as_i32 = rec_dev.view(torch.int32)
    det = rec_dev[:, 103] == 1
    img = torch.bincount(as_i32[:, 23][det].long() * nx + as_i32[:, 22][det].long(),
                         minlength=nx * ny).view(ny, nx)
    del as_i32, det, g, rec_dev
    print("[mwg-full] no-records launch (benchmark kernel)", flush=True)
    b = mrt.trace(w)
    assert torch.equal(b["counts"].long(), img)
    assert b["counters"]["events"] == c["events"]
    assert b["counters"]["reflections"] == c["reflections"]


def test_mwg_irc_disabled():
    # sec. 2.2.1: the IRC disabled, every reflection at Delta_M (psi moves only)
    w = mwg(W.get("von_hamos_hapg"), burn_in=300)
    w["event_model"]["irc_off"] = True
    w["rocking_curve"]["shift"] = 8e-6
    g, o = assert_parity(w, 200_000)
    assert o["counters"]["reflections"] > 1000
