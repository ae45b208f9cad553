"""The C-ABI boundary without a GPU: the library loads, exports every function
``include/*.h`` declares, and its host-side validation turns every invalid
argument into a status code and a message before touching a device."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(mrt_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = mrt.load()
    names = declared_functions()
    assert {"mrt_trace", "mrt_last_error", "mrt_version", "mrt_get_device_info"} <= names
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(mrt.EXPORTS) <= names


def test_version_matches_header():
    text = open(os.path.join(ROOT, "include", "mosaicrt.h")).read()
    v = int(re.search(r"#define\s+MRT_VERSION\s+(\d+)", text).group(1))
    assert mrt.load().mrt_version() == v


def test_struct_sizes_match_header():
    # sizes the header's layout implies (x86-64 / amdgcn, natural alignment)
    assert C.sizeof(mrt.MrtSource) == 416
    assert C.sizeof(mrt.MrtCrystal) == 232
    assert C.sizeof(mrt.MrtPlanes) == 112
    assert C.sizeof(mrt.MrtMosaic) == 24
    assert C.sizeof(mrt.MrtRockingCurve) == 104
    assert C.sizeof(mrt.MrtDetector) == 136
    assert C.sizeof(mrt.MrtOptions) == 56
    assert C.sizeof(mrt.MrtCounters) == 96
    assert mrt.RECORD_DTYPE.itemsize == 104


LAYOUT_STRUCTS = [("mrt_source", "MrtSource"), ("mrt_crystal", "MrtCrystal"), ("mrt_planes", "MrtPlanes"),
                  ("mrt_mosaic", "MrtMosaic"), ("mrt_rocking_curve", "MrtRockingCurve"),
                  ("mrt_detector", "MrtDetector"), ("mrt_options", "MrtOptions"),
                  ("mrt_counters", "MrtCounters"), ("mrt_server_config", "MrtServerConfig"),
                  ("mrt_request", "MrtRequest"), ("mrt_request_result", "MrtRequestResult")]


def test_binding_layout_matches_the_compiled_header(tmp_path):
    """Every field offset and struct size of the Python binding equals what
    a C compiler makes of include/mosaicrt.h."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mosaicrt.h"',
             'int main(void) {']
    want = []
    for cname, pyname in LAYOUT_STRUCTS:
        cls = getattr(mrt, pyname)
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        want.append(C.sizeof(cls))
        for f in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f[0]}));')
            want.append(getattr(cls, f[0]).offset)
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want


def _call(w, n=1000, first=0, opts=None, counts=1, energy=0, records=None, cap=0,
          counters=False):
    """mrt_trace with fake (never dereferenced) device pointers: validation
    runs first and returns before any device call."""
    L = mrt.load()
    S = mrt.Structs(w)
    o = opts or mrt.MrtOptions()
    cnt = mrt.MrtCounters()
    return L.mrt_trace(*S.refs(), first, n, 0, C.byref(o),
                       C.c_void_p(counts) if counts else None,
                       C.c_void_p(energy) if energy else None,
                       C.c_void_p(records) if records else None, cap,
                       C.byref(cnt) if counters else None, None)


def _mut(path, value, base="flat_hopg"):
    w = W.get(base)
    d = w
    for k in path[:-1]:
        d = d[k]
    d[path[-1]] = value
    return w


INVALID = [
    ("source axis not unit", ("source", "axis"), [1.0, 0.0, 0.1]),
    ("source b1 not orthogonal", ("source", "b1"), [0.97294474, 0.0, -0.23103794]),
    ("negative half angle", ("source", "half_angle"), -0.1),
    ("zero e_min", ("source", "e_min"), 0.0),
    ("e_max below e_min", ("source", "e_max"), 7.0),
    ("crystal normal not unit", ("crystal", "normal"), [0.0, 0.0, 2.0]),
    ("zero thickness", ("crystal", "thickness"), 0.0),
    ("negative mu0", ("crystal", "mu0"), -1.0),
    ("zero mfp", ("crystal", "mfp"), 0.0),
    ("negative max_refl", ("crystal", "max_refl"), -1),
    ("zero 2d", ("crystal", "two_d"), 0.0),
    ("negative mosaic fwhm", ("mosaic", "fwhm"), -1e-3),
    ("eta above 1", ("mosaic", "eta"), 1.5),
    ("zero rocking-curve width", ("rocking_curve", "fwhm"), 0.0),
    ("peak above 1", ("rocking_curve", "peak"), 1.5),
    ("detector axes not orthogonal", ("detector", "u"), [0.0, 1.0, 0.0]),
    ("zero pitch", ("detector", "pitch"), 0.0),
    ("zero columns", ("detector", "nx"), 0),
    ("image of 2^31 pixels", ("detector", "nx"), 1 << 16),
]


@pytest.mark.parametrize("label,path,value", INVALID, ids=[x[0] for x in INVALID])
def test_invalid_arguments_rejected(label, path, value):
    w = _mut(path, value)
    if label == "image of 2^31 pixels":
        w["detector"]["ny"] = 1 << 15
    assert _call(w) == mrt.EINVAL
    assert mrt.last_error() != ""


def test_invalid_spectra_and_tables():
    w = W.get("von_hamos_hapg")
    w["source"]["lines"] = [(8.0, -0.001, 1.0)]
    assert _call(w) == mrt.EINVAL
    w = W.get("von_hamos_hapg")
    w["source"]["lines"], w["source"]["background_w"] = [(8.0, 0.001, 0.0)], 0.0
    assert _call(w) == mrt.EINVAL and "zero" in mrt.last_error()
    w = W.get("flat_stress")
    w["rocking_curve"]["table"] = [0.1]
    assert _call(w) == mrt.EINVAL
    w = W.get("flat_stress")
    w["rocking_curve"]["table"] = [0.1, 1.5, 0.2]
    assert _call(w) == mrt.EINVAL
    w = W.get("flat_stress")
    w["rocking_curve"]["x_max"] = w["rocking_curve"]["x_min"]
    assert _call(w) == mrt.EINVAL
    w = W.get("flat_stress")
    w["source"]["bin_weights"] = [0.0] * 8
    assert _call(w) == mrt.EINVAL
    w = W.get("von_hamos_hapg")
    w["crystal"]["width"] = 4.0 * w["crystal"]["radius"]
    assert _call(w) == mrt.EINVAL


SPOT = dict(kind="gaussian", u=[1.0, 0.0, 0.0], v=[0.0, 1.0, 0.0], sigma=[0.01, 0.02])


@pytest.mark.parametrize("change", [
    dict(kind="gaussian", sigma=[-0.01, 0.01]), dict(kind="gaussian", sigma=[0.01, float("nan")]),
    dict(kind="disk", sigma=[float("inf"), 0.0]), dict(u=[1.0, 0.0, 0.1]),
    dict(v=[0.6, 0.8, 0.0]),
])
def test_invalid_source_spots(change):
    w = W.get("flat_hopg")
    w["source"]["spot"] = dict(SPOT, **change)
    assert _call(w) == mrt.EINVAL and "spot" in mrt.last_error()


def test_unknown_spot_kind_and_valid_spots():
    import torch
    w = W.get("flat_hopg")
    w["source"]["spot"] = SPOT
    S = mrt.Structs(w)
    S.source.spot_kind = 3
    L = mrt.load()
    o, cnt = mrt.MrtOptions(), mrt.MrtCounters()
    assert L.mrt_trace(*S.refs(), 0, 10, 0, C.byref(o), C.c_void_p(1), None, None, 0, None,
                       None) == mrt.EINVAL
    if torch.cuda.is_available():
        return
    # a disk ignores spot_sigma[1]; a valid spot gets past validation
    for spot in (SPOT, dict(SPOT, kind="disk", sigma=[0.01, -5.0])):
        w["source"]["spot"] = spot
        assert _call(w) == mrt.EDEVICE, mrt.last_error()


@pytest.mark.parametrize("planes", [
    dict(hbar_ratio=-0.5), dict(hbar_ratio=float("inf")), dict(extra=[(7.0, 1.0, 1.0, 0.0)]),
    dict(extra=[(3.354, 0.0, 1.0, 0.0)]), dict(extra=[(3.354, 1.0, -1.0, 0.0)]),
    dict(extra=[(3.354, 1.0, 1.0, float("nan"))]), dict(extra=[(0.0, 1.0, 1.0, 0.0)]),
])
def test_invalid_planes(planes):
    w = W.get("flat_hopg")
    w["crystal"]["planes"] = planes
    assert _call(w) == mrt.EINVAL and "planes" in mrt.last_error()


def test_planes_exclusions_and_count():
    import torch
    w = W.get("flat_hopg")
    w["crystal"]["planes"] = dict(extra=[(3.354, 1.0, 1.0, 0.0)])
    S = mrt.Structs(w)
    S._planes.n_extra = 4
    L = mrt.load()
    o = mrt.MrtOptions()
    assert L.mrt_trace(*S.refs(), 0, 10, 0, C.byref(o), C.c_void_p(1), None, None, 0, None,
                       None) == mrt.EINVAL
    w["rocking_curve"]["energy_dependence"] = [(8.0, 0.0, 1.0)]
    assert _call(w) == mrt.EINVAL and "planes" in mrt.last_error()
    if not torch.cuda.is_available():
        w["rocking_curve"].pop("energy_dependence")
        assert _call(w) == mrt.EDEVICE, mrt.last_error()
        # the paper's model takes plane sets too
        assert _call(w, opts=mrt.MrtOptions(event_model=mrt.MODEL["mwg"])) == mrt.EDEVICE, mrt.last_error()


def test_user_ray_arrays_are_checked_by_the_binding():
    import torch
    w = W.get("flat_hopg")
    bad = [dict(energies=torch.ones(10, dtype=torch.float64)),                # host tensor
           dict(origins=torch.zeros((10, 3), dtype=torch.float32)),
           dict(directions=torch.zeros((3, 10), dtype=torch.float64).t()),
           dict(speeds=torch.zeros(10, dtype=torch.float64))]
    for rays in bad:
        with pytest.raises(ValueError):
            mrt._user_rays(rays, 10, torch.device("cuda", 0))
    assert mrt._user_rays(None, 10, torch.device("cpu")) == dict(origins=None, directions=None,
                                                                 energies=None, polarisations=None)


def test_invalid_run_arguments():
    w = W.get("flat_hopg")
    assert _call(w, n=0) == mrt.EINVAL
    assert _call(w, n=10, first=(1 << 64) - 5) == mrt.EINVAL
    assert _call(w, counts=0) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(precision=7)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(records_mode=1)) == mrt.EINVAL   # no buffer
    assert _call(w, opts=mrt.MrtOptions(records_mode=1), records=0x1000, cap=10,
                 n=1000) == mrt.ECAPACITY
    assert _call(w, opts=mrt.MrtOptions(block_threads=96)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(grid_blocks=-1)) == mrt.EINVAL


def test_invalid_qe_tables_and_calibration_arguments():
    # QE: energies strictly increasing, values in [0, 1], at most 1024 nodes;
    # the calibration map needs its three device pointers
    for table in ([(8.0, 0.5), (8.0, 0.6)], [(8.1, 0.5), (8.0, 0.6)], [(8.0, 1.5)],
                  [(8.0, -0.1)], [(float("nan"), 0.5)], [(7.0 + i * 1e-3, 0.5) for i in range(1025)]):
        w = W.get("flat_hopg")
        w["detector"]["qe"] = table
        assert _call(w) == mrt.EINVAL, table
    w = W.get("flat_hopg")
    w["detector"]["qe"] = [(7.0, 0.5), (9.0, 0.6)]
    assert _call(w) != mrt.EINVAL      # valid: fails later, at the device
    L = mrt.load()
    assert L.mrt_calibration_map(None, C.c_void_p(8), 10, C.c_void_p(8), None) == mrt.EINVAL
    assert L.mrt_calibration_map(C.c_void_p(8), None, 10, C.c_void_p(8), None) == mrt.EINVAL
    assert L.mrt_calibration_map(C.c_void_p(8), C.c_void_p(8), 10, None, None) == mrt.EINVAL


def test_invalid_energy_dependence_tables():
    for table in ([(8.0, 0.0, 1.0), (8.0, 0.0, 1.0)], [(8.1, 0.0, 1.0), (8.0, 0.0, 1.0)],
                  [(8.0, 0.0, 0.0)], [(8.0, float("inf"), 1.0)],
                  [(7.0 + i * 1e-3, 0.0, 1.0) for i in range(1025)]):
        w = W.get("flat_hopg")
        w["rocking_curve"]["energy_dependence"] = table
        assert _call(w) == mrt.EINVAL, table
    w = W.get("flat_hopg")
    w["rocking_curve"]["energy_dependence"] = [(8.0, 1e-5, 1.2)]
    assert _call(w) != mrt.EINVAL
    # the paper's model takes it too
    assert _call(w, opts=mrt.MrtOptions(event_model=mrt.MODEL["mwg"])) != mrt.EINVAL, mrt.last_error()


def test_invalid_event_model_options():
    # the paper's event model: FP64 only, a mosaic density (fwhm > 0), burn-in
    # >= -1, at most 2048 psi intervals, batch within a wave, and event
    # indices that fit the sampler's counter word
    w = W.get("flat_hopg")
    M = dict(event_model=mrt.MODEL["mwg"])
    assert _call(w, opts=mrt.MrtOptions(event_model=5)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(precision=1, **M)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(mwg_burn_in=-2, **M)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(psi_nodes=2049, **M)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(psi_nodes=-1, **M)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(mwg_batch=65, **M)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(max_events=1 << 31, **M)) == mrt.EINVAL
    assert _call(w, opts=mrt.MrtOptions(mwg_irc_off=1)) == mrt.EINVAL      # needs the MWG model
    assert _call(w, opts=mrt.MrtOptions(mwg_irc_off=2, **M)) == mrt.EINVAL
    w["mosaic"]["fwhm"] = 0.0
    assert _call(w, opts=mrt.MrtOptions(**M)) == mrt.EINVAL
    assert "fwhm" in mrt.last_error()


def test_valid_call_without_gpu_fails_loudly():
    """A valid call on a machine without a GPU reports EDEVICE; there is no
    CPU fallback."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st = _call(W.get("flat_hopg"))
    assert st == mrt.EDEVICE, (st, mrt.last_error())
    with pytest.raises(Exception):
        mrt.trace(W.get("flat_hopg"))


def test_server_config_validation_and_no_gpu():
    """Server configuration errors are EINVAL before any device call; a valid
    configuration without a GPU is EDEVICE."""
    import torch
    L = mrt._load_server(mrt.load())
    h = C.c_void_p()
    bad = [dict(hbm_budget_bytes=0), dict(max_slots=0), dict(max_slots=5000), dict(precision=9),
           dict(chunk=100), dict(refill_idle=65)]
    for b in bad:
        cfg = dict(hbm_budget_bytes=1 << 30, max_slots=8, precision=1, round_rays=0, chunk=0,
                   refill_idle=0)
        cfg.update(b)
        assert L.mrt_server_create(C.byref(mrt.MrtServerConfig(**cfg)), C.byref(h)) == mrt.EINVAL, b
    assert L.mrt_server_create(None, C.byref(h)) == mrt.EINVAL
    if not torch.cuda.is_available():
        cfg = mrt.MrtServerConfig(hbm_budget_bytes=1 << 30, max_slots=8, precision=1)
        assert L.mrt_server_create(C.byref(cfg), C.byref(h)) == mrt.EDEVICE


def test_server_struct_sizes():
    assert C.sizeof(mrt.MrtServerConfig) == 40
    assert C.sizeof(mrt.MrtRequest) == 64
    assert C.sizeof(mrt.MrtRequestResult) == 160
    assert C.sizeof(mrt.MrtServerStats) == 88
