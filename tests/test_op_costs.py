"""The instruction prices of the ALU roofline are the ones the compiled
probe kernels show (gfx950 cross-compile on the CPU)."""
import os
import shutil

import pytest

from paper_2503_16955_amd import op_costs


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc") or not shutil.which("true"),
                    reason="needs hipcc")
def test_op_cost_table_matches_probe_kernels():
    assert op_costs.derive() == op_costs.OP_COSTS


def test_mix_is_positive_and_monotone():
    for prec in ("fp64", "fp32_mixed"):
        for geom in ("flat", "cylinder"):
            for mdf in ("gaussian_vmf", "lorentzian", "pseudo_voigt", "wrapped_lorentzian",
                        "spherical_wrapped_lorentzian"):
                for irc in ("gaussian", "pseudo_voigt", "table", "lorentzian", "box"):
                    m = op_costs.mix(prec, geom, mdf, irc, "lines", 0.3)
                    assert all(v > 0 for v in m.values())
    w = {"crystal": {"geometry": "flat"}, "mosaic": {"kind": "gaussian_vmf", "eta": 0.0},
         "rocking_curve": {"kind": "gaussian"}, "source": {"spectrum": "uniform"}}
    c = dict(emitted=10, missed=4, absorbed=2, exit_reflected=1, exit_transmitted=3, truncated=0,
             detected=1, events=100, reflections=2)
    a = op_costs.algorithmic_ops(w, "fp64", c)
    c2 = dict(c, events=200)
    assert op_costs.algorithmic_ops(w, "fp64", c2) > a > 0


def test_extended_pricing_adds_the_spot_and_polarisation_work():
    from paper_2503_16955_amd import workloads as W
    w = W.get("von_hamos_hapg")
    c = dict(emitted=1000, missed=400, absorbed=50, exit_reflected=20, exit_transmitted=530,
             truncated=0, detected=15, events=12000, reflections=30, refined=2)
    for prec in ("fp64", "fp32_mixed"):
        base = op_costs.algorithmic_ops(w, prec, c)
        assert op_costs.algorithmic_ops_ext(w, prec, c) == base
        s = op_costs.algorithmic_ops_ext(w, prec, c, spot=True)
        p = op_costs.algorithmic_ops_ext(w, prec, c, pol=True)
        both = op_costs.algorithmic_ops_ext(w, prec, c, spot=True, pol=True)
        assert base < s and base < p
        assert both == pytest.approx(s + p - base)
        # the spot is per emitted ray, polarisation per tilt and reflection
        c2 = dict(c, events=2 * c["events"])
        assert op_costs.algorithmic_ops_ext(w, prec, c2, spot=True) - op_costs.algorithmic_ops(w, prec, c2) \
            == pytest.approx(s - base)


def test_extended_pricing_adds_the_plane_bounds():
    from paper_2503_16955_amd import workloads as W
    w = W.get("von_hamos_hapg")
    c = dict(emitted=1000, missed=400, absorbed=50, exit_reflected=20, exit_transmitted=530,
             truncated=0, detected=15, events=12000, reflections=30, refined=2)
    one = op_costs.algorithmic_ops_ext(w, "fp64", c, planes=1)
    two = op_costs.algorithmic_ops_ext(w, "fp64", c, planes=2)
    base = op_costs.algorithmic_ops(w, "fp64", c)
    assert base < one < two
    assert (two - one) < (one - base)   # the sums and the comparison are paid once


def test_polarised_model_pricing_adds_work_per_event_and_sweep():
    a = op_costs.mix_mwg("cylinder", "pseudo_voigt", "pseudo_voigt", "lines", 256, 500)
    b = op_costs.mix_mwg("cylinder", "pseudo_voigt", "pseudo_voigt", "lines", 256, 500, pol=True)
    assert b["event"] > a["event"] and b["sweep"] > a["sweep"]
    assert b["reflection"] - a["reflection"] > 500 * (b["sweep"] - a["sweep"])
    assert b["ray"] == a["ray"] and b["detected"] == a["detected"]


def test_vmf_live_share_of_the_quadrature():
    """The share of psi nodes whose vMF exponential is priced grows with the
    mosaic width and stays in (0, 1]; past it exp(-kappa b) is exactly zero
    (pinned in test_device_math)."""
    import math
    deg = math.pi / 180.0
    shares = [op_costs.vmf_live_fraction(f * deg, 256) for f in (0.02, 0.1, 0.4, 0.8, 5.0, 60.0)]
    assert all(0.0 < x <= 1.0 for x in shares)
    assert shares == sorted(shares) and shares[0] < shares[-1] == 1.0
    # fewer priced exponentials price the quadrature lower
    a = op_costs.mix_mwg("cylinder", "pseudo_voigt", "pseudo_voigt", "lines", 256, 500, vmf_live=0.2)
    b = op_costs.mix_mwg("cylinder", "pseudo_voigt", "pseudo_voigt", "lines", 256, 500, vmf_live=1.0)
    assert a["quadrature"] < b["quadrature"]
