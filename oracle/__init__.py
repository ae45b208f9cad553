"""ctypes binding of the FP64 CPU oracle (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import this package.  It turns a workload description (plain
dicts from ``paper_2503_16955_amd.workloads``) into the oracle's own C
structs and returns numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))

MISS, ABSORBED, EXIT_REFLECTED, EXIT_TRANSMITTED, TRUNCATED = range(5)

_SPEC = {"uniform": 0, "lines": 1, "table": 2}
_GEOM = {"flat": 0, "cylinder": 1}
_MDF = {"gaussian_vmf": 0, "lorentzian": 1, "pseudo_voigt": 2, "wrapped_lorentzian": 3,
        "spherical_wrapped_lorentzian": 4, "gaussian": 5}
_IRC = {"gaussian": 0, "pseudo_voigt": 1, "table": 2, "lorentzian": 3, "box": 4}
_MODEL = {"stepping": 0, "mwg": 1}
_SPOT = {"point": 0, "gaussian": 1, "disk": 2}

D3 = C.c_double * 3
D8 = C.c_double * 8


class Source(C.Structure):
    _fields_ = [("origin", D3), ("axis", D3), ("b1", D3), ("half_angle", C.c_double),
                ("spectrum", C.c_int32), ("n_lines", C.c_int32),
                ("e_min", C.c_double), ("e_max", C.c_double),
                ("line_e", D8), ("line_sigma", D8), ("line_w", D8),
                ("background_w", C.c_double), ("n_bins", C.c_int32), ("spot_kind", C.c_int32),
                ("bin_w", C.POINTER(C.c_double)),
                ("spot_u", D3), ("spot_v", D3), ("spot_sigma", C.c_double * 2),
                ("user_o", C.c_void_p), ("user_k", C.c_void_p), ("user_e", C.c_void_p),
                ("user_first", C.c_uint64), ("user_p", C.c_void_p)]


class Planes(C.Structure):
    _fields_ = [("hbar_ratio", C.c_double), ("n_extra", C.c_int32), ("pad_", C.c_int32),
                ("two_d", D3), ("strength", D3), ("width_scale", D3), ("shift", D3)]


class Crystal(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("max_refl", C.c_int32),
                ("centre", D3), ("normal", D3), ("e1", D3),
                ("axis_pt", D3), ("axis_dir", D3), ("ref_dir", D3),
                ("radius", C.c_double), ("phi_c", C.c_double), ("z_c", C.c_double),
                ("length", C.c_double), ("width", C.c_double), ("thickness", C.c_double),
                ("two_d", C.c_double), ("mu0", C.c_double), ("mfp", C.c_double),
                ("planes", C.POINTER(Planes))]


class Mosaic(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("fwhm", C.c_double),
                ("eta", C.c_double)]


class Irc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_table", C.c_int32), ("peak", C.c_double),
                ("shift", C.c_double), ("fwhm", C.c_double), ("fwhm_g", C.c_double),
                ("fwhm_l", C.c_double), ("x_min", C.c_double), ("x_max", C.c_double),
                ("table", C.POINTER(C.c_double)), ("n_dep", C.c_int32), ("pad_", C.c_int32),
                ("dep_kev", C.POINTER(C.c_double)), ("dep_shift", C.POINTER(C.c_double)),
                ("dep_scale", C.POINTER(C.c_double))]


class Model(C.Structure):
    _fields_ = [("kind", C.c_int32), ("burn_in", C.c_int32), ("psi_nodes", C.c_int32),
                ("irc_off", C.c_int32)]


def model_of(w):
    """The event model of a workload: w["event_model"] = {"kind": "mwg",
    "burn_in": B, "psi_nodes": M, "irc_off": False}, or absent (null-collision
    stepping)."""
    e = w.get("event_model") or {"kind": "stepping"}
    return Model(kind=_MODEL[e["kind"]], burn_in=int(e.get("burn_in", 500)),
                 psi_nodes=int(e.get("psi_nodes", 256)), irc_off=1 if e.get("irc_off") else 0)


class Detector(C.Structure):
    _fields_ = [("centre", D3), ("normal", D3), ("u", D3), ("v", D3),
                ("nx", C.c_int32), ("ny", C.c_int32), ("pitch", C.c_double),
                ("n_qe", C.c_int32), ("pad_", C.c_int32), ("qe_kev", C.POINTER(C.c_double)),
                ("qe", C.POINTER(C.c_double))]


class Counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("emitted", "missed", "absorbed", "exit_reflected",
                                          "exit_transmitted", "truncated", "detected",
                                          "events", "reflections")]


RECORD_DTYPE = np.dtype([("ray_id", "<u8"), ("energy", "<f8"), ("entry", "<f8", 3),
                         ("end", "<f8", 3), ("dir", "<f8", 3), ("pix_i", "<i4"),
                         ("pix_j", "<i4"), ("n_events", "<u4"), ("n_refl", "<u2"),
                         ("status", "u1"), ("detected", "u1")])
assert RECORD_DTYPE.itemsize == 104

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER
        L.orc_philox4x32.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_philox4x64.argtypes = [P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
        L.orc_polarisation_angle.restype = C.c_double
        L.orc_polarisation_angle.argtypes = [P(C.c_double), P(C.c_double), P(C.c_double), C.c_double]
        L.orc_psi_integral_pol.restype = C.c_double
        L.orc_psi_integral_pol.argtypes = [P(Mosaic), C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_mwg_sample_pol.argtypes = [P(Mosaic), P(Irc), C.c_double, C.c_double, C.c_uint64,
                                         C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_double,
                                         C.c_double, P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_polarisation_reflect.restype = C.c_double
        L.orc_polarisation_reflect.argtypes = [P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_bragg_angle.restype = C.c_double
        L.orc_bragg_angle.argtypes = [C.c_double, C.c_double]
        L.orc_pvoigt_params.argtypes = [C.c_double, C.c_double, P(C.c_double), P(C.c_double)]
        L.orc_irc_value.restype = C.c_double
        L.orc_irc_value.argtypes = [P(Irc), C.c_double]
        L.orc_mdf_sample.argtypes = [P(Mosaic), C.c_double, C.c_double, P(C.c_double),
                                     P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_source_sample.argtypes = [P(Source), C.c_uint64, C.c_uint64, P(C.c_double),
                                        P(C.c_double), P(C.c_double)]
        L.orc_exit_distance.restype = C.c_double
        L.orc_exit_distance.argtypes = [P(Crystal), P(C.c_double), P(C.c_double)]
        L.orc_trace.restype = C.c_int
        L.orc_trace.argtypes = [P(Source), P(Crystal), P(Mosaic), P(Irc), P(Detector),
                                C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                C.c_void_p, C.c_void_p, C.c_void_p, P(Counters), C.c_void_p,
                                C.c_int]
        L.orc_trace_model.restype = C.c_int
        L.orc_trace_model.argtypes = [P(Source), P(Crystal), P(Mosaic), P(Irc), P(Detector),
                                      P(Model), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, P(Counters),
                                      C.c_void_p, C.c_int]
        L.orc_trace_ids_model.restype = C.c_int
        L.orc_trace_ids_model.argtypes = [P(Source), P(Crystal), P(Mosaic), P(Irc),
                                          P(Detector), P(Model), C.c_void_p, C.c_uint64,
                                          C.c_uint64, C.c_uint32, C.c_void_p, C.c_void_p,
                                          C.c_int]
        L.orc_mdf_density.restype = C.c_double
        L.orc_mdf_density.argtypes = [P(Mosaic), C.c_double]
        L.orc_psi_integral.restype = C.c_double
        L.orc_psi_integral.argtypes = [P(Mosaic), C.c_double, C.c_double, C.c_int]
        L.orc_irc_integral.restype = C.c_double
        L.orc_irc_integral.argtypes = [P(Irc)]
        L.orc_irc_width.restype = C.c_double
        L.orc_irc_width.argtypes = [P(Irc)]
        L.orc_mwg_sample.argtypes = [P(Mosaic), P(Irc), C.c_double, C.c_double, C.c_uint64,
                                     C.c_uint64, C.c_uint32, C.c_int, C.c_double, C.c_double,
                                     P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_crystallite.argtypes = [P(C.c_double), P(C.c_double), C.c_double, C.c_double,
                                      C.c_double, P(C.c_double)]
        L.orc_trace_ids.restype = C.c_int
        L.orc_trace_ids.argtypes = [P(Source), P(Crystal), P(Mosaic), P(Irc), P(Detector),
                                    C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint32,
                                    C.c_void_p, C.c_void_p, C.c_int]
        _lib = L
    return _lib


def _d3(v):
    return D3(*[float(x) for x in v])


class Structs:
    """The oracle's C structs for one workload (keeps table buffers alive)."""

    def __init__(self, w):
        s, c, m, r, d = (w["source"], w["crystal"], w["mosaic"], w["rocking_curve"],
                         w["detector"])
        self.src = Source()
        self.src.origin, self.src.axis, self.src.b1 = _d3(s["origin"]), _d3(s["axis"]), _d3(s["b1"])
        self.src.half_angle = s["half_angle"]
        self.src.spectrum = _SPEC[s["spectrum"]]
        self.src.e_min, self.src.e_max = s.get("e_min", 0.0), s.get("e_max", 0.0)
        lines = s.get("lines", [])
        self.src.n_lines = len(lines)
        for j, (e, sig, wt) in enumerate(lines):
            self.src.line_e[j], self.src.line_sigma[j], self.src.line_w[j] = e, sig, wt
        self.src.background_w = s.get("background_w", 0.0)
        self._bins = np.ascontiguousarray(s.get("bin_weights", [1.0]), dtype=np.float64)
        self.src.n_bins = len(self._bins) if s["spectrum"] == "table" else 0
        self.src.bin_w = self._bins.ctypes.data_as(C.POINTER(C.c_double))
        spot = s.get("spot")
        if spot:
            self.src.spot_kind = _SPOT[spot["kind"]]
            self.src.spot_u, self.src.spot_v = _d3(spot["u"]), _d3(spot["v"])
            sig = list(spot["sigma"]) if np.ndim(spot["sigma"]) else [spot["sigma"]]
            self.src.spot_sigma = (C.c_double * 2)(*(float(x) for x in (sig + [0.0])[:2]))
        self._rays = []

        self.cr = Crystal()
        self.cr.geometry = _GEOM[c["geometry"]]
        self.cr.max_refl = c["max_refl"]
        for key in ("centre", "normal", "e1", "axis_pt", "axis_dir", "ref_dir"):
            if key in c:
                setattr(self.cr, key, _d3(c[key]))
        for key in ("radius", "phi_c", "z_c", "length", "width", "thickness", "two_d",
                    "mu0", "mfp"):
            if key in c:
                setattr(self.cr, key, float(c[key]))
        if c.get("planes") is not None:
            pl = c["planes"]
            extra = list(pl.get("extra", []))
            self._planes = Planes(hbar_ratio=float(pl.get("hbar_ratio", 1.0)), n_extra=len(extra))
            for j, (p_d, p_a, p_sc, p_sh) in enumerate(extra[:3]):
                self._planes.two_d[j], self._planes.strength[j] = p_d, p_a
                self._planes.width_scale[j], self._planes.shift[j] = p_sc, p_sh
            self.cr.planes = C.pointer(self._planes)

        self.mo = Mosaic(kind=_MDF[m["kind"]], fwhm=m["fwhm"], eta=m.get("eta", 0.0))

        self.irc = Irc(kind=_IRC[r["kind"]], peak=r.get("peak", 0.0), shift=r.get("shift", 0.0),
                       fwhm=r.get("fwhm", 0.0), fwhm_g=r.get("fwhm_g", 0.0),
                       fwhm_l=r.get("fwhm_l", 0.0), x_min=r.get("x_min", 0.0),
                       x_max=r.get("x_max", 0.0))
        self._table = np.ascontiguousarray(r.get("table", [0.0]), dtype=np.float64)
        self.irc.n_table = len(self._table) if r["kind"] == "table" else 0
        self.irc.table = self._table.ctypes.data_as(C.POINTER(C.c_double))
        dep = np.ascontiguousarray(r.get("energy_dependence") or [(0.0, 0.0, 1.0)],
                                   dtype=np.float64).reshape(-1, 3)
        self._dep = [np.ascontiguousarray(dep[:, i]) for i in range(3)]
        self.irc.n_dep = len(dep) if r.get("energy_dependence") else 0
        P_ = C.POINTER(C.c_double)
        self.irc.dep_kev, self.irc.dep_shift, self.irc.dep_scale = (a.ctypes.data_as(P_) for a in self._dep)

        self.det = Detector(centre=_d3(d["centre"]), normal=_d3(d["normal"]), u=_d3(d["u"]),
                            v=_d3(d["v"]), nx=d["nx"], ny=d["ny"], pitch=d["pitch"])
        qe = np.ascontiguousarray(d.get("qe") or [(0.0, 1.0)], dtype=np.float64).reshape(-1, 2)
        self._qe_e, self._qe_v = np.ascontiguousarray(qe[:, 0]), np.ascontiguousarray(qe[:, 1])
        self.det.n_qe = len(qe) if d.get("qe") else 0
        self.det.qe_kev = self._qe_e.ctypes.data_as(C.POINTER(C.c_double))
        self.det.qe = self._qe_v.ctypes.data_as(C.POINTER(C.c_double))

    def set_rays(self, rays, first, n_rows):
        """Point the source at user ray arrays (host numpy float64): rows
        for ray ids first .. first + n_rows - 1."""
        for key, field, shape in (("origins", "user_o", (n_rows, 3)),
                                  ("directions", "user_k", (n_rows, 3)),
                                  ("energies", "user_e", (n_rows,)),
                                  ("polarisations", "user_p", (n_rows, 3))):
            a = (rays or {}).get(key)
            if a is None:
                continue
            a = np.ascontiguousarray(a, dtype=np.float64)
            if a.shape != shape:
                raise ValueError(f"rays[{key!r}] must have shape {shape}")
            self._rays.append(a)
            setattr(self.src, field, a.ctypes.data)
        self.src.user_first = first

    def args(self):
        return (C.byref(self.src), C.byref(self.cr), C.byref(self.mo), C.byref(self.irc),
                C.byref(self.det))


def trace(w, first=0, n=None, seed=None, max_events=0, images=True, records=False,
          margins=False, threads=0, rays=None):
    """Trace rays [first, first + n) of workload `w` on the CPU.

    rays: optional user ray arrays (numpy, row i for ray first + i):
    ``origins`` (n, 3), ``directions`` (n, 3), ``energies`` (n,).

    Returns a dict with ``counts`` (ny, nx) uint32, ``energy_mev`` (ny, nx)
    uint64, ``counters`` (dict), and on request ``records`` (structured array)
    and ``margins`` (float64)."""
    n = int(w["n_rays"] if n is None else n)
    seed = int(w["seed"] if seed is None else seed)
    S = Structs(w)
    S.set_rays(rays, first, n)
    nx, ny = w["detector"]["nx"], w["detector"]["ny"]
    out = {}
    counts = np.zeros((ny, nx), np.uint32) if images else None
    energy = np.zeros((ny, nx), np.uint64) if images else None
    recs = np.zeros(n, RECORD_DTYPE) if records else None
    mg = np.zeros(n, np.float64) if margins else None
    cnt = Counters()
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    model = model_of(w)
    rc = lib().orc_trace_model(*S.args(), C.byref(model), first, n, seed, max_events,
                               ptr(counts), ptr(energy), ptr(recs), C.byref(cnt), ptr(mg),
                               threads)
    if rc != 0:
        raise ValueError(f"oracle rejected the workload (code {rc})")
    out["counters"] = {f: getattr(cnt, f) for f, _ in Counters._fields_}
    if images:
        out["counts"], out["energy_mev"] = counts, energy
    if records:
        out["records"] = recs
    if margins:
        out["margins"] = mg
    return out


def trace_ids(w, ids, seed=None, max_events=0, threads=0, rays=None, first=0, n_rows=None):
    """Records and decision margins for an arbitrary list of ray ids (user
    ray arrays, if any, hold the n_rows rays from id `first` on)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    seed = int(w["seed"] if seed is None else seed)
    S = Structs(w)
    if rays:
        if n_rows is None or np.any(ids < first) or np.any(ids >= first + n_rows):
            raise ValueError("ray ids outside the user arrays")
        S.set_rays(rays, first, n_rows)
    recs = np.zeros(len(ids), RECORD_DTYPE)
    mg = np.zeros(len(ids), np.float64)
    model = model_of(w)
    rc = lib().orc_trace_ids_model(*S.args(), C.byref(model), ids.ctypes.data_as(C.c_void_p),
                                   len(ids), seed, max_events, recs.ctypes.data_as(C.c_void_p),
                                   mg.ctypes.data_as(C.c_void_p), threads)
    if rc != 0:
        raise ValueError(f"oracle rejected the workload (code {rc})")
    return recs, mg


# ---- single-function access for unit pins ---------------------------------

def philox4x32(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32(c, k, o)
    return list(o)


def philox4x64(ctr, key):
    c = (C.c_uint64 * 4)(*ctr)
    k = (C.c_uint64 * 2)(*key)
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64(c, k, o)
    return list(o)


def polarisation_angle(p, N, k, alpha):
    """The angle phi of polarisation p about k for planes of normal N."""
    return lib().orc_polarisation_angle(_d3(p), _d3(N), _d3(k), float(alpha))


def psi_integral_pol(mosaic, alpha, beta, phi, nodes=256):
    """The psi integral of W G (Eq. SimpleReflXsectionPol)."""
    return lib().orc_psi_integral_pol(C.byref(_mosaic(mosaic)), float(alpha), float(beta),
                                      float(phi), int(nodes))


def mwg_sample_pol(mosaic, rocking_curve, w_psi, w_delta, seed, rays, event, burn_in, alpha, ab,
                   phi):
    """(psi, Delta) drawn by the polarised sampler (polarisation angle phi)
    for each ray id in `rays`."""
    m = _mosaic(mosaic)
    irc, _tab = _irc(rocking_curve)
    rays = np.atleast_1d(np.asarray(rays, np.uint64))
    out = np.zeros((len(rays), 2))
    ps, de = C.c_double(), C.c_double()
    for i, r in enumerate(rays):
        lib().orc_mwg_sample_pol(C.byref(m), C.byref(irc), float(w_psi), float(w_delta), int(seed),
                                 int(r), int(event), int(burn_in), float(alpha), float(ab),
                                 float(phi), C.byref(ps), C.byref(de), None)
        out[i] = ps.value, de.value
    return out


def polarisation_reflect(p, ks):
    """(G, new polarisation) for polarisation p and reflected direction ks."""
    out = D3()
    g = lib().orc_polarisation_reflect(_d3(p), _d3(ks), out)
    return g, np.array(list(out))


def bragg_angle(energy_kev, two_d):
    return lib().orc_bragg_angle(energy_kev, two_d)


def pvoigt_params(fwhm_g, fwhm_l):
    f, e = C.c_double(), C.c_double()
    lib().orc_pvoigt_params(fwhm_g, fwhm_l, C.byref(f), C.byref(e))
    return f.value, e.value


def irc_value(rocking_curve, x):
    w = {"source": {"origin": [0, 0, 0], "axis": [0, 0, 1], "b1": [1, 0, 0], "half_angle": 0,
                    "spectrum": "uniform"},
         "crystal": {"geometry": "flat", "max_refl": 0}, "mosaic": {"kind": "gaussian_vmf", "fwhm": 0},
         "rocking_curve": rocking_curve,
         "detector": {"centre": [0, 0, 0], "normal": [0, 0, 1], "u": [1, 0, 0], "v": [0, 1, 0],
                      "nx": 1, "ny": 1, "pitch": 1}}
    S = Structs(w)
    xs = np.atleast_1d(np.asarray(x, dtype=np.float64))
    return np.array([lib().orc_irc_value(C.byref(S.irc), float(v)) for v in xs])


def mdf_sample(mosaic, u2, u3, N=(0, 0, 1), e1=(1, 0, 0), e2=(0, 1, 0)):
    m = Mosaic(kind=_MDF[mosaic["kind"]], fwhm=mosaic["fwhm"], eta=mosaic.get("eta", 0.0))
    u2 = np.atleast_1d(np.asarray(u2, np.float64))
    u3 = np.atleast_1d(np.asarray(u3, np.float64))
    out = np.zeros((len(u2), 3))
    n = D3()
    a, b, c = _d3(N), _d3(e1), _d3(e2)
    for i in range(len(u2)):
        lib().orc_mdf_sample(C.byref(m), float(u2[i]), float(u3[i]), a, b, c, n)
        out[i] = list(n)
    return out


def source_sample(w, ray_ids, seed=None):
    seed = int(w["seed"] if seed is None else seed)
    S = Structs(w)
    ids = np.atleast_1d(np.asarray(ray_ids, np.uint64))
    o = np.zeros((len(ids), 3))
    k = np.zeros((len(ids), 3))
    e = np.zeros(len(ids))
    oo, kk, ee = D3(), D3(), C.c_double()
    for i, r in enumerate(ids):
        lib().orc_source_sample(C.byref(S.src), seed, int(r), oo, kk, C.byref(ee))
        o[i], k[i], e[i] = list(oo), list(kk), ee.value
    return o, k, e


def exit_distance(w, p, k):
    S = Structs(w)
    return lib().orc_exit_distance(C.byref(S.cr), _d3(p), _d3(k))


# ---- the paper's event model: pieces for unit pins -------------------------

def _mosaic(mosaic):
    return Mosaic(kind=_MDF[mosaic["kind"]], fwhm=mosaic["fwhm"], eta=mosaic.get("eta", 0.0))


def _irc(rocking_curve):
    r = rocking_curve
    tab = np.ascontiguousarray(r.get("table", [0.0]), dtype=np.float64)
    irc = Irc(kind=_IRC[r["kind"]], peak=r.get("peak", 0.0), shift=r.get("shift", 0.0),
              fwhm=r.get("fwhm", 0.0), fwhm_g=r.get("fwhm_g", 0.0), fwhm_l=r.get("fwhm_l", 0.0),
              x_min=r.get("x_min", 0.0), x_max=r.get("x_max", 0.0))
    irc.n_table = len(tab) if r["kind"] == "table" else 0
    irc.table = tab.ctypes.data_as(C.POINTER(C.c_double))
    return irc, tab


def mdf_density(mosaic, v):
    """Mosaic density per steradian at v = 1 - cos(theta)."""
    m = _mosaic(mosaic)
    vs = np.atleast_1d(np.asarray(v, np.float64))
    return np.array([lib().orc_mdf_density(C.byref(m), float(x)) for x in vs])


def psi_integral(mosaic, alpha, beta, nodes=256):
    m = _mosaic(mosaic)
    return lib().orc_psi_integral(C.byref(m), float(alpha), float(beta), int(nodes))


def irc_integral(rocking_curve):
    irc, _tab = _irc(rocking_curve)
    return lib().orc_irc_integral(C.byref(irc))


def irc_width(rocking_curve):
    irc, _tab = _irc(rocking_curve)
    return lib().orc_irc_width(C.byref(irc))


def mwg_sample(mosaic, rocking_curve, w_psi, w_delta, seed, rays, event, burn_in, alpha, ab):
    """(psi, Delta) drawn by the sampler for each ray id in `rays`."""
    m = _mosaic(mosaic)
    irc, _tab = _irc(rocking_curve)
    rays = np.atleast_1d(np.asarray(rays, np.uint64))
    out = np.zeros((len(rays), 2))
    ps, de = C.c_double(), C.c_double()
    for i, r in enumerate(rays):
        lib().orc_mwg_sample(C.byref(m), C.byref(irc), float(w_psi), float(w_delta), int(seed),
                             int(r), int(event), int(burn_in), float(alpha), float(ab),
                             C.byref(ps), C.byref(de), None)
        out[i] = ps.value, de.value
    return out


def crystallite(N, k, alpha, b, psi):
    n = D3()
    lib().orc_crystallite(_d3(N), _d3(k), float(alpha), float(b), float(psi), n)
    return np.array(list(n))


def calibration_map(counts, energy_mev):
    """Mean photon energy per pixel in keV, NaN where no photon landed
    (sec. 3, the calibration map): (energy / counts) * 1e-6."""
    c = np.asarray(counts).astype(np.float64)
    e = np.asarray(energy_mev).astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        m = (e / c) * 1e-6
    m[np.asarray(counts) == 0] = np.nan
    return m
