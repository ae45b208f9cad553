"""The VALU issue-rate microbenchmark (csrc/valu_rates.hip) measures what
its table says: compiled for gfx950, the timed loop of each kernel holds
only the named instruction class (32 per loop trip: 8 chains x 4 steps;
64 for the two-instruction classes)."""
import collections
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "paper_2503_16955_amd", "csrc", "valu_rates.hip")
HIPCC = "/opt/rocm/bin/hipcc"

WANT = {0: {"v_xor_b32_e32": 32, "v_add_u32_e32": 32}, 1: {"v_fma_f32": 32},
        2: {"v_fma_f64": 32}, 3: {"v_mul_lo_u32": 32}, 4: {"v_mad_u64_u32": 32},
        5: {"v_log_f32_e32": 32, "v_exp_f32_e32": 32}, 6: {"v_rcp_f32_e32": 32},
        7: {"v_sqrt_f32_e32": 32}, 8: {"v_rcp_f64_e32": 32},
        9: {"v_mul_f32_e32": 32, "v_add_f32_e32": 32}, 10: {"v_mul_hi_u32": 32},
        11: {"v_xor_b32_e32": 32, "v_cvt_f32_u32_e32": 32, "v_cvt_u32_f32_e32": 32},
        12: {"v_cmp_lt_u32_e32": 32, "v_cndmask_b32_e32": 32}, 13: {"v_bitop3_b32": 32}}


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_timed_loops_hold_one_instruction_class(tmp_path):
    out = tmp_path / "vr.s"
    subprocess.check_call([HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950",
                           "-ffp-contract=off", "-Xclang",
                           "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
                           "-S", "-x", "hip", SRC, "-o", str(out)], stderr=subprocess.DEVNULL)
    lines = out.read_text().split("\n")
    found = {}
    cur = None
    i = 0
    while i < len(lines):
        m = re.match(r"^_Z\w*rate_kernelILi(\d+)E\w*:", lines[i])
        if m:
            cur = int(m.group(1))
        m = re.match(r"^(\.LBB\d+_\d+):\s*;\s*=>This Inner Loop Header", lines[i])
        if m:
            ops, j = [], i + 1
            while not re.search(r"s_cbranch_\w+\s+" + re.escape(m.group(1)) + r"\b", lines[j]):
                mm = re.match(r"^\s+(v_\w+)", lines[j])
                if mm:
                    ops.append(mm.group(1))
                j += 1
            found[cur] = dict(collections.Counter(ops))
            i = j
        i += 1
    assert found == WANT
