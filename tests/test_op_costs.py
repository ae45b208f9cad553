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
