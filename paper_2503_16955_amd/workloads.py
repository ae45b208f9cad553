"""Seeded synthetic workloads: spectrometer geometries, spectra, mosaic and
rocking-curve settings, detectors, ray counts and seeds.

This module only *describes inputs*.  It holds no step of the transport
itself and is the one module shared by the GPU path and the CPU oracle.  All
values are plain numbers in the library's units: mm, rad, keV, Angstrom, 1/mm.

Geometry follows the spectrometer types the paper simulates (sec. 4.1 flat
crystal and von Hamos images, sec. 4.2 the 80 mm HAPG von Hamos at 8 keV):

* ``flat_hopg``        flat HOPG(002) at 200 mm, uniform 7.9-8.1 keV, 1e5 rays
* ``von_hamos_hapg``   cylindrical HAPG(002), R = 80 mm, Cu K-alpha-like doublet
                       on a flat background, 1e8 rays
* ``von_hamos_precision`` the same set-up at 1e9 rays (mixed precision study)
* ``flat_stress``      100 um HOPG, Lorentzian mosaic 0.8 deg, tabulated
                       Darwin-Prins-shaped rocking curve, 1024-bin spectrum,
                       4096^2 detector, 2e9 rays
* ``serving_requests`` 256 von Hamos design requests for the serving loop

The placement angle below is the Bragg angle of 8.0 keV on 2d = 6.708 A,
written as a literal: it only positions the crystal, source and detector.
"""
from __future__ import annotations

import copy
import math

import numpy as np

DEG = math.pi / 180.0

# Placement angle: 8.0 keV on graphite (002), 2d = 6.708 A.
PLACEMENT_ANGLE = 0.23314434736170897
TWO_D_GRAPHITE = 6.708           # Angstrom, (002)
MU0_GRAPHITE = 1.04              # 1/mm  (10.4 /cm)
MEAN_FREE_PATH = 0.002           # mm between crystallite encounters (2 um)

SPEC_UNIFORM, SPEC_LINES, SPEC_TABLE = "uniform", "lines", "table"


def _flat_geometry(distance=200.0, thickness=0.040, nx=512, ny=512, pitch=0.05,
                   angle=PLACEMENT_ANGLE, half_angle=2.0 * DEG):
    """Flat crystal at the origin (surface normal +z, length axis +x); point
    source and detector symmetric about the surface normal at `distance`."""
    ca, sa = math.cos(angle), math.sin(angle)
    source = dict(origin=[-distance * ca, 0.0, distance * sa],
                  axis=[ca, 0.0, -sa], b1=[0.0, 1.0, 0.0], half_angle=half_angle)
    crystal = dict(geometry="flat", centre=[0.0, 0.0, 0.0], normal=[0.0, 0.0, 1.0],
                   e1=[1.0, 0.0, 0.0], length=30.0, width=30.0, thickness=thickness,
                   two_d=TWO_D_GRAPHITE, mu0=MU0_GRAPHITE, mfp=MEAN_FREE_PATH)
    detector = dict(centre=[distance * ca, 0.0, distance * sa],
                    normal=[-ca, 0.0, -sa], u=[-sa, 0.0, ca], v=[0.0, 1.0, 0.0],
                    nx=nx, ny=ny, pitch=pitch)
    return source, crystal, detector


def _von_hamos_geometry(radius=80.0, length=100.0, width=30.0, thickness=0.040,
                        angle=PLACEMENT_ANGLE, half_angle=3.5 * DEG,
                        nx=2048, ny=512, pitch=0.05):
    """Von Hamos: cylinder axis +z through the source; crystal patch centred at
    azimuth -90 deg (the -y side) and axial position z_c = R / tan(angle);
    detector in the plane y = 0 centred on the axis at 2 z_c."""
    ca, sa = math.cos(angle), math.sin(angle)
    z_c = radius * ca / sa
    source = dict(origin=[0.0, 0.0, 0.0], axis=[0.0, -sa, ca], b1=[1.0, 0.0, 0.0],
                  half_angle=half_angle)
    crystal = dict(geometry="cylinder", axis_pt=[0.0, 0.0, 0.0], axis_dir=[0.0, 0.0, 1.0],
                   ref_dir=[1.0, 0.0, 0.0], radius=radius, phi_c=-math.pi / 2.0, z_c=z_c,
                   length=length, width=width, thickness=thickness,
                   two_d=TWO_D_GRAPHITE, mu0=MU0_GRAPHITE, mfp=MEAN_FREE_PATH)
    detector = dict(centre=[0.0, 0.0, 2.0 * z_c], normal=[0.0, -1.0, 0.0],
                    u=[0.0, 0.0, 1.0], v=[1.0, 0.0, 0.0], nx=nx, ny=ny, pitch=pitch)
    return source, crystal, detector


def darwin_prins_table(n=4096, half_range=500e-6, w_d=23.3e-6, g=0.1, kappa=0.02,
                       peak=0.5):
    """Tabulated rocking curve of Darwin-Prins shape (absorbing perfect
    crystal): y = x / w_D, eta = (y + i g) / (1 + i kappa), reflectivity
    min |eta -+ sqrt(eta^2 - 1)|^2, scaled so that the maximum is `peak`.
    Returns (table, x_min, x_max)."""
    x = np.linspace(-half_range, half_range, n)
    y = x / w_d
    eta = (y + 1j * g) / (1.0 + 1j * kappa)
    root = np.sqrt(eta * eta - 1.0 + 0j)
    r = np.minimum(np.abs(eta - root) ** 2, np.abs(eta + root) ** 2)
    r = r * (peak / r.max())
    return r.astype(np.float64), -half_range, half_range


def exponential_spectrum(n=1024, e_min=7.9, e_max=8.1, scale=0.05):
    """Bin weights at bin centres decaying as exp(-(E - e_min) / scale)."""
    centres = e_min + (np.arange(n) + 0.5) * (e_max - e_min) / n
    return np.exp(-(centres - e_min) / scale)


def flat_hopg():
    src, cr, det = _flat_geometry()
    src.update(spectrum=SPEC_UNIFORM, e_min=7.9, e_max=8.1)
    cr.update(max_refl=1)
    return dict(name="flat_hopg", source=src, crystal=cr,
                mosaic=dict(kind="gaussian_vmf", fwhm=0.4 * DEG, eta=0.0),
                rocking_curve=dict(kind="gaussian", peak=0.5, shift=0.0, fwhm=50e-6),
                detector=det, n_rays=100_000, seed=0, precision="fp64")


def von_hamos_hapg():
    src, cr, det = _von_hamos_geometry()
    src.update(spectrum=SPEC_LINES, e_min=7.8, e_max=8.2,
               lines=[(8.048, 0.002, 0.6), (8.028, 0.002, 0.3)], background_w=0.1)
    cr.update(max_refl=4)
    return dict(name="von_hamos_hapg", source=src, crystal=cr,
                mosaic=dict(kind="pseudo_voigt", fwhm=0.1 * DEG, eta=0.3),
                rocking_curve=dict(kind="pseudo_voigt", peak=0.5, shift=0.0,
                                   fwhm_g=50e-6, fwhm_l=8e-6),
                detector=det, n_rays=100_000_000, seed=1, precision="fp64")


def von_hamos_burn_in():
    """The instrument-function study of the paper's burn-in figure (sec.
    2.2.4, Fig. BurnIn): a point source of 8.5 keV photons on a von Hamos
    spectrometer whose central energy is 8.5 keV; graphite with a Lorentzian
    mosaic of 0.14 deg and a Voigt rocking curve of 50.7 / 10.0 urad
    Gaussian / Lorentzian FWHM (peak 0.5), up to 4 reflections.  The radius
    (80 mm), crystal size and detector are the von Hamos workload's, which
    the figure does not give."""
    src, cr, det = _von_hamos_geometry(angle=placement_angle(8.5))
    src.update(spectrum=SPEC_UNIFORM, e_min=8.5, e_max=8.5)
    cr.update(max_refl=4)
    return dict(name="von_hamos_burn_in", source=src, crystal=cr,
                mosaic=dict(kind="lorentzian", fwhm=0.14 * DEG, eta=0.0),
                rocking_curve=dict(kind="pseudo_voigt", peak=0.5, shift=0.0,
                                   fwhm_g=50.7e-6, fwhm_l=10.0e-6),
                detector=det, n_rays=10_000_000, seed=21, precision="fp64")


def von_hamos_precision():
    w = von_hamos_hapg()
    w.update(name="von_hamos_precision", n_rays=1_000_000_000, precision="fp32_mixed")
    return w


def flat_stress():
    src, cr, det = _flat_geometry(thickness=0.100, nx=4096, ny=4096, pitch=0.025)
    bins = exponential_spectrum()
    src.update(spectrum=SPEC_TABLE, e_min=7.9, e_max=8.1, bin_weights=bins.tolist())
    cr.update(max_refl=8)
    table, x0, x1 = darwin_prins_table()
    return dict(name="flat_stress", source=src, crystal=cr,
                mosaic=dict(kind="lorentzian", fwhm=0.8 * DEG, eta=0.0),
                rocking_curve=dict(kind="table", peak=float(table.max()), shift=0.0,
                                   table=table.tolist(), x_min=x0, x_max=x1),
                detector=det, n_rays=2_000_000_000, seed=3, precision="fp32_mixed")


WORKLOADS = {
    "flat_hopg": flat_hopg,
    "von_hamos_hapg": von_hamos_hapg,
    "von_hamos_precision": von_hamos_precision,
    "flat_stress": flat_stress,
    "von_hamos_burn_in": von_hamos_burn_in,
}


def get(name: str, **overrides):
    """A fresh copy of a named workload with top-level keys overridden."""
    w = copy.deepcopy(WORKLOADS[name]())
    w.update(overrides)
    return w


def serving_requests(n=256, seed=4):
    """Design requests for the serving loop: von Hamos crystals of radius
    60-120 mm, mosaic FWHM 0.05-0.8 deg (log-uniform), thickness 20-100 um,
    a flat energy window (centre 7.5-8.5 keV, width 0.1-0.4 keV), mosaic kind
    cycling Gaussian / Lorentzian / pseudo-Voigt, ray counts log-uniform in
    [1e5, 1e8].  Each crystal is aimed at its window centre with
    `placement_angle`, a literal table interpolated linearly."""
    rng = np.random.default_rng(seed)
    kinds = ["gaussian_vmf", "lorentzian", "pseudo_voigt"]
    reqs = []
    for i in range(n):
        radius = float(rng.uniform(60.0, 120.0))
        fwhm = float(math.exp(rng.uniform(math.log(0.05), math.log(0.8)))) * DEG
        thick = float(rng.uniform(0.020, 0.100))
        centre = float(rng.uniform(7.5, 8.5))
        width = float(rng.uniform(0.1, 0.4))
        n_rays = int(round(math.exp(rng.uniform(math.log(1e5), math.log(1e8)))))
        angle = placement_angle(centre)
        src, cr, det = _von_hamos_geometry(radius=radius, thickness=thick, angle=angle)
        src.update(spectrum=SPEC_UNIFORM, e_min=centre - width / 2, e_max=centre + width / 2)
        cr.update(max_refl=4)
        kind = kinds[i % 3]
        reqs.append(dict(name=f"request_{i}", source=src, crystal=cr,
                         mosaic=dict(kind=kind, fwhm=fwhm, eta=0.3 if kind == "pseudo_voigt" else 0.0),
                         rocking_curve=dict(kind="pseudo_voigt", peak=0.5, shift=0.0,
                                            fwhm_g=50e-6, fwhm_l=8e-6),
                         detector=det, n_rays=n_rays, seed=1000 + i, precision="fp32_mixed"))
    return reqs


# Placement angles (rad) of graphite (002) at whole-tenth keV energies, used
# only to aim a crystal at an energy window.  Interpolated linearly.
_PLACEMENT_TABLE_KEV = [7.4, 7.5, 7.6, 7.7, 7.8, 7.9, 8.0, 8.1, 8.2, 8.3, 8.4, 8.5, 8.6]
_PLACEMENT_TABLE_RAD = [0.25244, 0.24901, 0.24566, 0.24241, 0.23924, 0.23615, 0.23314,
                        0.23021, 0.22736, 0.22457, 0.22185, 0.21920, 0.21661]


def placement_angle(energy_kev: float) -> float:
    return float(np.interp(energy_kev, _PLACEMENT_TABLE_KEV, _PLACEMENT_TABLE_RAD))


def calibration_workload(w, e_min, e_max):
    """The paper's calibration run (sec. 3): the same spectrometer with photon
    energies uniform over [e_min, e_max] keV and no detector efficiency."""
    c = copy.deepcopy(w)
    c["source"] = dict(c["source"], spectrum="uniform", e_min=float(e_min), e_max=float(e_max))
    c["source"].pop("lines", None)
    c["detector"] = dict(c["detector"])
    c["detector"].pop("qe", None)
    c["name"] = w["name"] + "_calibration"
    return c


def with_spot(w, kind="gaussian", fwhm=0.010):
    """`w` with a finite source spot in the plane normal to the source axis
    (sec. 4.2: a nominal 10 um Gaussian XFEL spot on the target).  Gaussian:
    `fwhm` (mm) in both directions; disk: diameter `fwhm`."""
    c = copy.deepcopy(w)
    s = c["source"]
    b2 = np.cross(s["axis"], s["b1"])
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0))) if kind == "gaussian" else fwhm / 2.0
    s["spot"] = dict(kind=kind, u=list(s["b1"]), v=[float(x) for x in b2],
                     sigma=[sigma, sigma] if kind == "gaussian" else [sigma, 0.0])
    c["name"] = w["name"] + "_" + kind + "_spot"
    return c
