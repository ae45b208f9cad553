"""Precision of a spectrometer image against a reference image of the same
rays: per spectral line, the centroid and the full width at half maximum
of the dispersive profile, and the chi-square per pixel of the two images.

The dispersive profile is the image summed over rows (the detector's v
axis); a line's centroid is the count-weighted mean column within
``half`` pixels of its zero-mosaic focus column, and its FWHM comes from
linear interpolation of the two half-maximum crossings around the peak.
Poisson weights follow the paper's error bars, sigma^2 = N (+1 for empty
pixels, which are skipped here).
"""
from __future__ import annotations

import math

import numpy as np

HC_KEV_ANGSTROM = 12.398419843320026


def dispersive_profile(counts):
    """Counts per column (sum over rows)."""
    return np.asarray(counts, np.float64).sum(axis=0)


def centroid(profile, centre_col, half=15):
    lo = max(0, int(round(centre_col)) - half)
    hi = min(len(profile), int(round(centre_col)) + half + 1)
    cols = np.arange(lo, hi, dtype=np.float64)
    w = profile[lo:hi]
    s = w.sum()
    return float((cols * w).sum() / s) if s > 0 else float("nan")


def fwhm(profile, centre_col, half=15):
    """Full width at half maximum of the peak within `half` pixels of
    centre_col (linear interpolation of the half-maximum crossings)."""
    lo = max(0, int(round(centre_col)) - half)
    hi = min(len(profile), int(round(centre_col)) + half + 1)
    seg = np.asarray(profile[lo:hi], np.float64)
    if seg.max() <= 0:
        return float("nan")
    m = int(np.argmax(seg))
    hm = seg[m] / 2.0
    i = m
    while i > 0 and seg[i] > hm:
        i -= 1
    left = i + (hm - seg[i]) / (seg[i + 1] - seg[i]) if seg[i + 1] != seg[i] else float(i)
    j = m
    while j < len(seg) - 1 and seg[j] > hm:
        j += 1
    right = (j - 1) + (seg[j - 1] - hm) / (seg[j - 1] - seg[j]) if seg[j - 1] != seg[j] else float(j)
    return float(right - left)


def chi2_per_pixel(a, b, scale=1.0):
    """(1 / N) sum over pixels with a + b > 0 of (a - s b)^2 / (a + s^2 b):
    the Poisson chi-square of image a against image b scaled by s (the ratio
    of their ray counts), per contributing pixel."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    m = (a + b) > 0
    d = a[m] - scale * b[m]
    return float((d * d / (a[m] + scale * scale * b[m])).sum() / max(1, int(m.sum())))


def von_hamos_line_column(workload, e_kev):
    """Zero-mosaic focus column of an energy on the von Hamos detector: a
    ray from a source on the cylinder axis reflected specularly focuses back
    on the axis at z = 2 R / tan(alpha_B) (alpha_B from Bragg's law)."""
    c, d = workload["crystal"], workload["detector"]
    a = math.asin(HC_KEV_ANGSTROM / (c["two_d"] * e_kev))
    z = 2.0 * c["radius"] / math.tan(a)
    return (z - d["centre"][2]) / d["pitch"] + d["nx"] / 2.0


def compare_images(workload, test_counts, ref_counts, lines_kev, scale=1.0, half=15):
    """Per-line centroid shift and FWHM change of `test` against `ref`, and the
    chi-square per pixel.  Returns a JSON-ready dict."""
    pt, pr = dispersive_profile(test_counts), dispersive_profile(ref_counts)
    out = {"lines": [], "chi2_per_px": round(chi2_per_pixel(test_counts, ref_counts, scale), 5)}
    for e in lines_kev:
        col = von_hamos_line_column(workload, e)
        ct, cr = centroid(pt, col, half), centroid(pr, col, half)
        ft, fr = fwhm(pt, col, half), fwhm(pr, col, half)
        out["lines"].append({"e_kev": e, "focus_col": round(col, 3), "centroid_ref": round(cr, 4),
                             "centroid_test": round(ct, 4), "centroid_shift_px": round(ct - cr, 5),
                             "fwhm_ref_px": round(fr, 4), "fwhm_test_px": round(ft, 4),
                             "fwhm_change": round((ft - fr) / fr, 6) if fr else None})
    return out
