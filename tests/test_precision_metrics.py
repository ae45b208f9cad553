"""The image precision metrics against closed forms and simple statistics."""
import math

import numpy as np

import oracle
from paper_2503_16955_amd import precision as pr
from paper_2503_16955_amd import workloads as W


def _gauss_image(centre, sigma, nx=200, ny=4, amp=1e4):
    x = np.arange(nx) + 0.5
    row = amp * np.exp(-0.5 * ((x - centre) / sigma) ** 2)
    return np.tile(row, (ny, 1))


def test_centroid_and_fwhm_of_a_gaussian_line():
    img = _gauss_image(100.0, 3.0)
    prof = pr.dispersive_profile(img)
    # pixel centres at i + 0.5 and columns counted from 0: centroid = centre - 0.5
    # (the +-15 px window is half a pixel off-centre: a bias of a few 1e-6 px)
    assert abs(pr.centroid(prof, 99.5, half=15) - 99.5) < 1e-4
    # linear interpolation of a sampled sigma = 3 px Gaussian: ~1 % wide; the
    # metric compares two images of one line, where this bias cancels
    assert abs(pr.fwhm(prof, 99.5, half=15) / (2.0 * math.sqrt(2.0 * math.log(2.0)) * 3.0) - 1) < 0.02


def test_centroid_shift_is_recovered():
    a = pr.dispersive_profile(_gauss_image(100.0, 3.0))
    b = pr.dispersive_profile(_gauss_image(100.3, 3.0))
    assert abs((pr.centroid(b, 99.5) - pr.centroid(a, 99.5)) - 0.3) < 1e-3


def test_chi2_identical_and_poisson():
    rng = np.random.default_rng(1)
    lam = rng.uniform(5, 50, (64, 64))
    a, b = rng.poisson(lam), rng.poisson(lam)
    assert pr.chi2_per_pixel(a, a) == 0.0
    c = pr.chi2_per_pixel(a, b)
    assert 0.85 < c < 1.15          # two independent Poisson draws of one mean: E = 1
    # scaled reference: b has twice the rays
    b2 = rng.poisson(2 * lam)
    assert 0.85 < pr.chi2_per_pixel(a, b2, scale=0.5) < 1.15


def test_von_hamos_focus_columns_match_the_oracle_zero_mosaic_lines():
    """The focus column formula against the oracle's own zero-mosaic image of a
    monochromatic on-axis source (lines at the Bragg focus)."""
    for e in (8.028, 8.048):
        w = W.get("von_hamos_hapg")
        w["source"].update(spectrum="uniform", e_min=e, e_max=e)
        w["mosaic"] = dict(kind="gaussian_vmf", fwhm=0.0, eta=0.0)
        w["rocking_curve"] = dict(kind="gaussian", peak=1.0, shift=0.0, fwhm=2e-3)
        w["crystal"]["max_refl"] = 1
        r = oracle.trace(w, n=200_000)
        prof = pr.dispersive_profile(r["counts"])
        col = pr.von_hamos_line_column(w, e)
        assert prof.sum() > 100
        # the depth of the reflection point shifts the focus by < 1 px
        assert abs(pr.centroid(prof, col, half=6) - col) < 1.0
