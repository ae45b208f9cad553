"""VALU instruction cost of the operations on the transport's per-event path,
as the library's kernels compile them for gfx950, and the algorithmic
operation count of a trace.

``OP_COSTS`` was counted by ``derive()``: each probe kernel in
``csrc/op_cost_probe.hip`` applies one operation; its VALU instruction count
in the gfx950 disassembly minus that of the matching copy kernel is the
operation's cost.  Plain arithmetic (add, mul, fma, compare, select,
convert) costs one instruction.  The algorithmic work of a trace is the
method's operation mix per unit (per emitted ray, per entering ray, per event,
per drawn crystallite tilt, per reflection, per detected ray), each operation
priced by this table, times the unit counts the trace reports.  It does not
depend on how the kernel is written: a faster kernel does the same
algorithmic work in less time.
"""
from __future__ import annotations

import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))

# VALU instructions per operation in steady state (gfx950, -O3, packed FP32
# disabled), as counted by derive().
OP_COSTS = {
    "f64": {"log": 36, "exp": 22, "expm1": 31, "sqrt": 14, "rsqrt": 8, "rcp": 5, "div": 11,
            "sincos": 40},
    "f32": {"log": 2, "exp": 2, "expm1": 23, "sqrt": 1, "rsqrt": 1, "rcp": 1, "div": 11,
            "sincos": 2},
    "filter": {"gaussian": 37, "pseudo_voigt": 45, "table": 25, "lorentzian": 37, "box": 27},
    "philox": 53,
}

PROBES = {
    ("f64", "log"): ("log_f64", "glue_f64"), ("f64", "exp"): ("exp_f64", "glue_f64"),
    ("f64", "expm1"): ("expm1_f64", "glue_f64"), ("f64", "sqrt"): ("sqrt_f64", "glue_f64"),
    ("f64", "rsqrt"): ("rsqrt_f64", "glue_f64"), ("f64", "rcp"): ("rcp_f64", "glue_f64"),
    ("f64", "div"): ("div_ieee_f64", "glue_f64"), ("f64", "sincos"): ("sincos_f64", "glue2_f64"),
    ("f32", "log"): ("log_f32", "glue_f32"), ("f32", "exp"): ("exp_f32", "glue_f32"),
    ("f32", "expm1"): ("expm1_f32", "glue_f32"), ("f32", "sqrt"): ("sqrt_f32", "glue_f32"),
    ("f32", "rsqrt"): ("rsqrt_f32", "glue_f32"), ("f32", "rcp"): ("rcp_f32", "glue_f32"),
    ("f32", "div"): ("div_ieee_f32", "glue_f32"), ("f32", "sincos"): ("sincos_f32", "glue2_f32"),
    ("philox",): ("philox", "glue_u32"),
    ("filter", "gaussian"): ("filter_gaussian", "glue_filter"),
    ("filter", "pseudo_voigt"): ("filter_pseudo_voigt", "glue_filter"),
    ("filter", "table"): ("filter_table", "glue_filter"),
    ("filter", "lorentzian"): ("filter_lorentzian", "glue_filter"),
    ("filter", "box"): ("filter_box", "glue_filter"),
}


def _loop_valu(lines):
    """VALU instructions inside the loop of one probe kernel: from the target
    of its backward branch to the branch."""
    labels, ins = {}, []
    for line in lines:
        t = line.strip()
        m = re.match(r"^[0-9a-f]+ <(L\d+)>:", t)
        if m:
            labels[m.group(1)] = len(ins)
            continue
        if t:
            ins.append(t.split("//")[0].strip())
    best = None
    for i, x in enumerate(ins):
        m = re.match(r"s_(?:cbranch_\w+|branch)\s+(L\d+)", x)
        if m and labels.get(m.group(1), len(ins)) < i:
            a = labels[m.group(1)]
            if best is None or i - a > best[1] - best[0]:
                best = (a, i)
    if best is None:
        return 0
    return sum(1 for x in ins[best[0]:best[1] + 1] if x.startswith("v_"))


def derive(hipcc="/opt/rocm/bin/hipcc", objdump="/opt/rocm/llvm/bin/llvm-objdump", tmp="/tmp"):
    """Recount OP_COSTS from the probe kernels' gfx950 code."""
    src = os.path.join(HERE, "csrc", "op_cost_probe.hip")
    obj = os.path.join(tmp, "mosaicrt_op_cost_probe.co")
    subprocess.check_call([hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang",
                           "-target-feature", "-Xclang", "-packed-fp32-ops", "-I",
                           os.path.join(HERE, "csrc"), "-I", os.path.join(os.path.dirname(HERE), "include"),
                           "--cuda-device-only", "--no-gpu-bundle-output", "-c", src, "-o", obj],
                          stderr=subprocess.DEVNULL)
    dis = subprocess.check_output([objdump, "-d", "--no-show-raw-insn", "--symbolize-operands",
                                   obj], text=True).splitlines()
    funcs, cur = {}, None
    for line in dis:
        m = re.match(r"^[0-9a-f]+ <probe_(\w+)>:", line)
        if m:
            cur = m.group(1)
            funcs[cur] = []
            continue
        if re.match(r"^[0-9a-f]+ <[^L]", line):
            cur = None
        if cur:
            funcs[cur].append(line)
    counts = {k: _loop_valu(v) for k, v in funcs.items()}
    out = {"f64": {}, "f32": {}, "filter": {}}
    for key, (probe, base) in PROBES.items():
        c = counts[probe] - counts[base]
        if key == ("philox",):
            out["philox"] = c
        else:
            out[key[0]][key[1]] = c
    return out


def mix(precision, geometry, mosaic, irc, spectrum, mosaic_eta=0.0):
    """Operation mix per unit, in VALU instructions, from OP_COSTS.

    Units: 'ray' (every emitted ray: cone direction and front-face entry
    test), 'entered' (energy, Bragg angle, first exit distance), 'event' (one
    draw of the event uniforms, free path, move, absorption test), 'tilt'
    (local frame, crystallite normal, k.n in FP64, acceptance decision),
    'reflection' (reflected direction and new exit distance) and 'detected'
    (detector plane, pixel, two integer atomics).  Plain arithmetic, compares
    and selects count one each."""
    D = OP_COSTS["f64"]
    R = OP_COSTS["f64"] if precision == "fp64" else OP_COSTS["f32"]
    ph = OP_COSTS["philox"]
    U = 2 if precision == "fp64" else 3          # word -> uniform
    cyl = geometry == "cylinder"
    if cyl:
        exit_d = 2 * R["sqrt"] + 6 * R["div"] + 45
        entry = R["sqrt"] + R["div"] + 30
        frame = R["rsqrt"] + 18
    else:
        exit_d = 6 * R["div"] + 30
        entry = R["div"] + 20
        frame = 0
    ray = ph + 2 * U + R["sqrt"] + R["sincos"] + 18 + entry
    if spectrum == "lines":
        energy = 8 + ph + D["sincos"] + D["log"] + D["sqrt"] + 6
    elif spectrum == "table":
        energy = 10 * 4 + 6
    else:
        energy = 2
    entered = energy + D["div"] + D["sqrt"] + 5 + exit_d
    event = ph + 4 * U + R["log"] + 8
    vmf = R["log"] + R["sqrt"] + 8
    lor = R["rsqrt"] + R["sqrt"] + 8
    if mosaic == "gaussian_vmf":
        mdf = vmf
    elif mosaic == "lorentzian":
        mdf = lor
    elif mosaic == "pseudo_voigt":
        mdf = 3 + mosaic_eta * (R["rsqrt"] + 7) + (1.0 - mosaic_eta) * (R["log"] + 7) + R["sqrt"] + 1
    elif mosaic == "wrapped_lorentzian":
        mdf = R["expm1"] + R["sqrt"] + 7
    else:
        mdf = R["div"] + R["sqrt"] + 7
    kn = 3 if precision == "fp64" else 9
    tilt = 2 + frame + mdf + R["sincos"] + 12 + kn + 2 + OP_COSTS["filter"][irc] + 2
    reflection = 7 + R["rsqrt"] + 3 + exit_d
    detected = 3 * R["div"] + 36
    return {"ray": ray, "entered": entered, "event": event, "tilt": tilt,
            "reflection": reflection, "detected": detected}


def algorithmic_ops(workload, precision, counters):
    """VALU lane-operations the method needs for a trace with these counters."""
    m = workload["mosaic"]
    M = mix(precision, workload["crystal"]["geometry"], m["kind"],
            workload["rocking_curve"]["kind"], workload["source"]["spectrum"],
            m.get("eta", 0.0))
    c = counters
    entered = c["emitted"] - c["missed"]
    ended = c["absorbed"] + c["exit_reflected"] + c["exit_transmitted"]
    tilts = max(0, c["events"] - ended)
    return (c["emitted"] * M["ray"] + entered * M["entered"] + c["events"] * M["event"]
            + tilts * M["tilt"] + c["reflections"] * M["reflection"]
            + c["detected"] * M["detected"])


if __name__ == "__main__":
    print(derive())
