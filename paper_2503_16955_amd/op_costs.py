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

# VALU instructions per operation (gfx950, -O3, packed FP32 disabled).
OP_COSTS = {
    "f64": {"log": 97, "exp": 41, "asin": 99, "sqrt": 21, "rcp": 11, "expm1": 52,
            "sincos": 153},
    "f32": {"log": 13, "exp": 2, "sqrt": 6, "rcp": 11, "expm1": 26, "sincos": 3},
    "philox": 80,
}

PROBES = {
    ("f64", "log"): ("log_f64", "copy_f64"), ("f64", "exp"): ("exp_f64", "copy_f64"),
    ("f64", "asin"): ("asin_f64", "copy_f64"), ("f64", "sqrt"): ("sqrt_f64", "copy_f64"),
    ("f64", "rcp"): ("rcp_f64", "copy_f64"), ("f64", "expm1"): ("expm1_f64", "copy_f64"),
    ("f64", "sincos"): ("sincos_f64", "copy2_f64"),
    ("f32", "log"): ("log_f32", "copy_f32"), ("f32", "exp"): ("exp_f32", "copy_f32"),
    ("f32", "sqrt"): ("sqrt_f32", "copy_f32"), ("f32", "rcp"): ("rcp_f32", "copy_f32"),
    ("f32", "expm1"): ("expm1_f32", "copy_f32"), ("f32", "sincos"): ("sincos_f32", "copy2_f32"),
    ("philox",): ("philox", "copy4_u32"),
}


def derive(hipcc="/opt/rocm/bin/hipcc", objdump="/opt/rocm/llvm/bin/llvm-objdump", tmp="/tmp"):
    """Recount OP_COSTS from the probe kernels' gfx950 code."""
    src = os.path.join(HERE, "csrc", "op_cost_probe.hip")
    obj = os.path.join(tmp, "mosaicrt_op_cost_probe.co")
    subprocess.check_call([hipcc, "-O3", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                           "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
                           "--no-gpu-bundle-output", "-c", src, "-o", obj],
                          stderr=subprocess.DEVNULL)
    dis = subprocess.check_output([objdump, "-d", "--no-show-raw-insn", obj], text=True)
    counts, cur = {}, None
    for line in dis.splitlines():
        m = re.match(r"^[0-9a-f]+ <probe_(\w+)>:", line)
        if m:
            cur = m.group(1)
            counts[cur] = 0
            continue
        t = line.strip().split()
        if cur and t and t[0].startswith("v_"):
            counts[cur] += 1
    out = {"f64": {}, "f32": {}}
    for key, (probe, base) in PROBES.items():
        c = counts[probe] - counts[base]
        if key == ("philox",):
            out["philox"] = c
        else:
            out[key[0]][key[1]] = c
    return out


def mix(precision, geometry, mosaic, irc, spectrum, mosaic_eta=0.0):
    """Operation mix per unit, in VALU instructions, from OP_COSTS.

    Units: 'ray' (every emitted ray: source draws and front-face entry test),
    'entered' (Bragg angle and first exit distance), 'event' (one draw of the
    event uniforms, free path, move, absorption test), 'tilt' (local frame,
    crystallite normal, Bragg deviation in FP64, rocking-curve value,
    acceptance test), 'reflection' (reflected direction and new exit distance)
    and 'detected' (detector plane, pixel, two integer atomics)."""
    D = OP_COSTS["f64"]
    R = OP_COSTS["f64"] if precision == "fp64" else OP_COSTS["f32"]
    ph = OP_COSTS["philox"]
    cyl = geometry == "cylinder"
    # exit distance: flat = 6 face tests with one reciprocal each;
    # cylinder = 2 quadratic roots (sqrt + rcp) + 2 end planes + 2 edge planes
    exit_d = (6 * R["rcp"] + 30) if not cyl else (2 * (R["sqrt"] + R["rcp"]) + 4 * R["rcp"] + 45)
    entry = (R["rcp"] + 20) if not cyl else (R["sqrt"] + R["rcp"] + 40)
    source = 2 * ph + 8 + R["sqrt"] + R["sincos"] + 20 + entry
    if spectrum == "lines":
        source += D["log"] + D["sqrt"] + D["sincos"] + 12
    elif spectrum == "table":
        source += 10 * 4 + 6
    else:
        source += 2
    entered = D["rcp"] + D["asin"] + 4 + exit_d + 6
    event = ph + 8 + R["log"] + 10
    frame = 0 if not cyl else (6 + R["sqrt"] + R["rcp"] + 3 + 6)
    vmf = R["log"] + 4 + R["sqrt"] + 3
    lor = 3 + 2 * R["sqrt"] + 2 * R["rcp"] + 3
    if mosaic == "gaussian_vmf":
        tilt_mdf = vmf
    elif mosaic == "lorentzian":
        tilt_mdf = lor
    elif mosaic == "pseudo_voigt":
        tilt_mdf = 3 + mosaic_eta * lor + (1.0 - mosaic_eta) * vmf
    elif mosaic == "wrapped_lorentzian":
        tilt_mdf = R["expm1"] + 3 + R["sqrt"] + 3
    else:
        tilt_mdf = R["rcp"] + 4 + R["sqrt"] + 3
    irc_cost = {"gaussian": D["exp"] + 3, "pseudo_voigt": D["exp"] + D["rcp"] + 8,
                "table": 20, "lorentzian": D["rcp"] + 3, "box": 3}[irc]
    if precision != "fp64" and irc in ("gaussian", "pseudo_voigt"):
        irc_cost = irc_cost - D["exp"] + R["exp"] + 2
    tilt = frame + tilt_mdf + 1 + R["sincos"] + 12 + 6 + D["asin"] + 3 + irc_cost + 2
    reflection = 9 + 3 + R["sqrt"] + 3 * R["rcp"] + exit_d
    detected = 12 + R["rcp"] + 14 + 4
    return {"ray": source, "entered": entered, "event": event, "tilt": tilt,
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
