"""Issue cost of the operations on the transport's per-event path, as the
library's kernels compile them for gfx950, and the algorithmic work of a
trace in VALU issue slots.

gfx950 issues VALU instructions at different rates by class.  The rates
come from the throughput microbenchmark ``csrc/valu_rates.hip`` (its tables
are in profiles/valu_issue_rates_gfx950.md): measured on MI355X, FP32
arithmetic (fma, mul, add) runs at about twice the FP64 FMA's lane rate,
32-bit integer, logic, compare, select, conversion and three-input bitwise
instructions and the 32-bit integer multiplies at about 1.1 times it,
v_mad_u64_u32 at 1.05 times, FP32 transcendentals at 0.55 times and
v_rcp_f64 at 0.28 times.  One
issue slot is one FP64 FMA lane, so the peak is 256 CUs x 64 x 2.4 GHz =
39.32 T slots/s (the published 78.6 TFLOP/s FP64 peak over 2 flops) and an
instruction costs SLOT_WEIGHT of its class: the FP64 FMA's measured rate
over its class's.

``OP_COSTS`` was counted by ``derive()``: each probe kernel in
``csrc/op_cost_probe.hip`` applies one operation inside a loop (constants
placed as in the trace kernel); the slot-weighted VALU instructions of its
loop body, minus those of the glue-only loop, are the operation's cost.
The algorithmic work of a trace is the method's operation mix per unit
(per emitted ray, per entering ray, per event, per drawn crystallite tilt,
per reflection, per detected ray), each operation priced by this table,
times the unit counts the trace reports.
"""
from __future__ import annotations

import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))

# Issue slots per VALU instruction class on gfx950 (see the module doc):
# the measured FP64 FMA rate over the class's, averaged over three runs of
# the microbenchmark and rounded to 0.05 (per run: fp32 0.46-0.53, alu32
# 0.88-0.91 (integer, logic, compare, select, conversion, bitop3), mul32
# 0.87-0.89, mad64 0.94-0.95, trans32 1.76-1.81, trans64 3.53-3.62).  64-bit
# integer instructions other than v_mad_u64_u32 are not measured and are
# priced like FP64.
SLOT_WEIGHT = {"fp32": 0.5, "alu32": 0.9, "mul32": 0.9, "alu64": 1.0, "mad64": 0.95,
               "trans32": 1.8, "trans64": 3.6}
_TRANS32 = ("v_exp_f32", "v_log_f32", "v_sqrt_f32", "v_rsq_f32", "v_rcp_f32", "v_sin_f32",
            "v_cos_f32")
_TRANS64 = ("v_rcp_f64", "v_rsq_f64", "v_sqrt_f64")
_FP32_ARITH = re.compile(r"^v_(fma|fmac|mac|mad|mul|add|sub|subrev|max|min|med3|ldexp|fmamk|"
                         r"fmaak)_f32$")


def slot_class(op):
    """Class of a VALU mnemonic (without its encoding suffix)."""
    op = re.sub(r"_e(32|64)$", "", op)
    if op.startswith(_TRANS32):
        return "trans32"
    if op.startswith(_TRANS64):
        return "trans64"
    if op.startswith(("v_mad_u64_u32", "v_mad_i64_i32")):
        return "mad64"
    if op.startswith(("v_mul_hi_u32", "v_mul_lo_u32", "v_mul_hi_i32")):
        return "mul32"
    if "f64" in op or "b64" in op or "u64" in op or "i64" in op:
        return "alu64"
    if _FP32_ARITH.match(op):
        return "fp32"
    return "alu32"


# Issue slots per operation in the trace kernels' code, as counted by derive().
OP_COSTS = {'f64': {'log': 23.2, 'exp': 19.5, 'expm1': 47.4, 'sqrt': 16.4, 'rsqrt': 8.6, 'rcp': 7.6, 'div': 13.6, 'sincos': 23.6, 'sin': 143.1, 'cos': 143.1, 'asin': 100.9}, 'f32': {'log': 2.3, 'exp': 2.3, 'expm1': 17.8, 'sqrt': 1.8, 'rsqrt': 1.8, 'rcp': 1.8, 'div': 8.4, 'sincos': 3.6}, 'filter': {'gaussian': 32.0, 'pseudo_voigt': 38.6, 'table': 23.4, 'lorentzian': 32.0, 'box': 22.6}, 'philox': 30.7}

PROBES = {
    ("f64", "log"): ("log_f64", "glue_f64"), ("f64", "exp"): ("exp_f64", "glue_f64"),
    ("f64", "expm1"): ("expm1_f64", "glue_f64"), ("f64", "sqrt"): ("sqrt_f64", "glue_f64"),
    ("f64", "rsqrt"): ("rsqrt_f64", "glue_f64"), ("f64", "rcp"): ("rcp_f64", "glue_f64"),
    ("f64", "div"): ("div_ieee_f64", "glue_f64"), ("f64", "sincos"): ("sincos_f64", "glue2_f64"),
    ("f64", "sin"): ("sin_f64", "glue_f64"), ("f64", "cos"): ("cos_f64", "glue_f64"),
    ("f64", "asin"): ("asin_f64", "glue_f64"),
    ("f32", "log"): ("log_f32", "glue_f32"), ("f32", "exp"): ("exp_f32", "glue_f32"),
    ("f32", "expm1"): ("expm1_f32", "glue_f32"), ("f32", "sqrt"): ("sqrt_f32", "glue_f32"),
    ("f32", "rsqrt"): ("rsqrt_f32", "glue_f32"), ("f32", "rcp"): ("rcp_f32", "glue_f32"),
    ("f32", "div"): ("div_ieee_f32", "glue_f32"), ("f32", "sincos"): ("sincos_f32", "glue2_f32"),
    ("philox",): ("philox", "glue_u32"),
    ("filter", "gaussian"): ("filter_gaussian", "glue_filter"),
    ("filter", "pseudo_voigt"): ("filter_pseudo_voigt", "glue_filter"),
    ("filter", "table"): ("filter_table_range", "glue_filter"),
    ("filter", "lorentzian"): ("filter_lorentzian", "glue_filter"),
    ("filter", "box"): ("filter_box", "glue_filter"),
}


def _loop_valu(lines):
    """Slot-weighted VALU instructions inside the loop of one probe kernel:
    from the target of its backward branch to the branch."""
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
        return 0.0
    return sum(SLOT_WEIGHT[slot_class(x.split()[0])] for x in ins[best[0]:best[1] + 1]
               if x.startswith("v_"))


def derive(hipcc="/opt/rocm/bin/hipcc", objdump="/opt/rocm/llvm/bin/llvm-objdump", tmp="/tmp"):
    """Recount OP_COSTS from the probe kernels' gfx950 code."""
    src = os.path.join(HERE, "csrc", "op_cost_probe.hip")
    obj = os.path.join(tmp, "mosaicrt_op_cost_probe.co")
    from . import build as _build
    flags = [f for f in _build.FLAGS if f != "-fPIC"]
    subprocess.check_call([hipcc, *flags, "--cuda-device-only", "--no-gpu-bundle-output", "-c",
                           src, "-o", obj], stderr=subprocess.DEVNULL)
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
        c = round(counts[probe] - counts[base], 2)
        if key == ("philox",):
            out["philox"] = c
        else:
            out[key[0]][key[1]] = c
    return out


def mix(precision, geometry, mosaic, irc, spectrum, mosaic_eta=0.0):
    """Operation mix per unit, in issue slots, from OP_COSTS.

    Units: 'ray' (every emitted ray: cone direction and front-face entry
    test), 'entered' (energy, Bragg angle, first exit distance), 'event' (one
    draw of the event uniforms, free path, move, absorption test), 'tilt'
    (local frame, crystallite normal, k.n in FP64, acceptance decision),
    'reflection' (reflected direction and new exit distance) and 'detected'
    (detector plane, pixel, two integer atomics).  Plain arithmetic, compares
    and selects count one instruction each, in the precision of the path
    (FP64 1 slot, FP32 0.5), except the FP64 energy and k.n of both paths.
    A word becomes an FP64 uniform in a conversion and an FMA, an FP32 one
    in a shift, a conversion and an FMA."""
    D = OP_COSTS["f64"]
    R = OP_COSTS["f64"] if precision == "fp64" else OP_COSTS["f32"]
    a = SLOT_WEIGHT["alu64"] if precision == "fp64" else SLOT_WEIGHT["fp32"]
    d = SLOT_WEIGHT["alu64"]
    ph = OP_COSTS["philox"]
    U = 2 * d if precision == "fp64" else 2 * SLOT_WEIGHT["alu32"] + SLOT_WEIGHT["fp32"]
    cyl = geometry == "cylinder"
    if cyl:
        exit_d = 2 * R["sqrt"] + 6 * R["div"] + 45 * a
        entry = R["sqrt"] + R["div"] + 30 * a
        frame = R["rsqrt"] + 18 * a
    else:
        exit_d = 6 * R["div"] + 30 * a
        entry = R["div"] + 20 * a
        frame = 0
    ray = ph + 2 * U + R["sqrt"] + R["sincos"] + 18 * a + entry
    if spectrum == "lines":
        energy = 8 * d + ph + D["sincos"] + D["log"] + D["sqrt"] + 6 * d
    elif spectrum == "table":
        energy = 46 * d
    else:
        energy = 2 * d
    entered = energy + D["div"] + D["sqrt"] + 5 * d + exit_d
    event = ph + 4 * U + R["log"] + 8 * a
    vmf = R["log"] + R["sqrt"] + 8 * a
    lor = R["rsqrt"] + R["sqrt"] + 8 * a
    if mosaic == "gaussian_vmf":
        mdf = vmf
    elif mosaic == "lorentzian":
        mdf = lor
    elif mosaic == "pseudo_voigt":
        mdf = (3 * a + mosaic_eta * (R["rsqrt"] + 7 * a) + (1.0 - mosaic_eta) * (R["log"] + 7 * a)
               + R["sqrt"] + a)
    elif mosaic == "wrapped_lorentzian":
        mdf = R["expm1"] + R["sqrt"] + 7 * a
    elif mosaic == "gaussian":
        mdf = R["log"] + R["rsqrt"] + R["sqrt"] + 4 * a
    else:
        mdf = R["div"] + R["sqrt"] + 7 * a
    kn = 3 * d if precision == "fp64" else 9 * d
    tilt = 2 * a + frame + mdf + R["sincos"] + 12 * a + kn + 2 * d + OP_COSTS["filter"][irc] + 2 * a
    reflection = 7 * a + R["rsqrt"] + 3 * a + exit_d
    detected = 3 * R["div"] + 36 * a
    return {"ray": ray, "entered": entered, "event": event, "tilt": tilt,
            "reflection": reflection, "detected": detected}


def algorithmic_ops(workload, precision, counters):
    """Issue slots the method needs for a trace with these counters."""
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


# ---- the paper's event model (FP64) ------------------------------------------

def _density_cost(mosaic):
    """Issue slots of one mosaic density value per steradian."""
    D, a = OP_COSTS["f64"], SLOT_WEIGHT["alu64"]
    vmf = D["exp"] + 2 * a
    cau = D["rsqrt"] + 10 * a
    return {"gaussian_vmf": vmf, "lorentzian": cau, "pseudo_voigt": vmf + cau + 3 * a,
            "wrapped_lorentzian": D["div"] + 2 * a,
            "spherical_wrapped_lorentzian": D["div"] + 3 * a,
            "gaussian": D["rcp"] + D["exp"] + 9 * a}[mosaic]


def vmf_live_fraction(fwhm, psi_nodes):
    """Share of the quadrature's nodes psi_j = pi (j/M)^3 at which the vMF
    factor exp(-kappa b), b = cc sin^2(psi_j / 2), can be nonzero (kappa b <=
    746), taken at the largest cc = 2 cos(alpha) cos(beta), 2: the fewest
    nodes, so the exponentials are never over-priced."""
    import math
    sv = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    kappa = 1.0 / (sv * sv)
    live = sum(1 for j in range(1, psi_nodes + 1)
               if kappa * 2.0 * math.sin(math.pi * (j / psi_nodes) ** 3 / 2.0) ** 2 <= 746.0)
    return live / psi_nodes


def _node_cost(mosaic, live=1.0):
    """Issue slots of one node of the psi quadrature: the density at v0 + b
    for the H and the anti-H planes.  The vMF density splits as exp(-kappa
    v0) exp(-kappa b), so one exponential and two products serve both sides
    (for the pseudo-Voigt mosaic's vMF part too); past kappa b = 746 the
    exponential is exactly zero and skipped (`live`: the share of nodes
    before that).  The Lorentzian's q is a quadratic in the node's
    sin^2(psi/2) (two FMAs), then q^(-3/2) from one reciprocal square root
    and three products, the range test and its select."""
    D, a = OP_COSTS["f64"], SLOT_WEIGHT["alu64"]
    vmf = live * D["exp"] + 4 * a
    lor = D["rsqrt"] + 8 * a
    if mosaic == "gaussian_vmf":
        return vmf
    if mosaic == "lorentzian":
        return 2 * lor
    if mosaic == "pseudo_voigt":
        return vmf + 2 * (lor + a)
    return 2 * (a + _density_cost(mosaic))


def _irc_cost(irc):
    D, a = OP_COSTS["f64"], SLOT_WEIGHT["alu64"]
    return {"gaussian": D["exp"] + 3 * a, "pseudo_voigt": D["div"] + D["exp"] + 8 * a,
            "lorentzian": D["div"] + 3 * a, "box": 2 * a, "table": 15 * a}[irc]


def mix_mwg(geometry, mosaic, irc, spectrum, psi_nodes, burn_in, pol=False, vmf_live=1.0):
    """Operation mix per unit of the paper's event model, in issue slots.

    Units: 'ray' and 'entered' as in mix() (FP64); 'event' (one free path:
    Philox, exit distance, frame, glancing angle, the psi quadrature of Eq.
    SimpleReflXsection on psi_nodes intervals for the H and anti-H planes,
    free path, absorption and plane choice); 'reflection' (burn_in sweeps of
    the sampler, each one Philox, a psi move and a Delta move re-evaluating
    only the factors they change, then the crystallite's orientation and the
    reflection); 'detected' as in mix().  Sines and cosines are priced as
    the table-driven sin/cos of turns; `vmf_live`: the share of quadrature
    nodes whose vMF exponential can be nonzero (vmf_live_fraction)."""
    D, a = OP_COSTS["f64"], SLOT_WEIGHT["alu64"]
    base = mix("fp64", geometry, "gaussian_vmf", "gaussian", spectrum)
    cyl = geometry == "cylinder"
    exit_d = (2 * D["sqrt"] + 6 * D["div"] + 45 * a) if cyl else (6 * D["div"] + 30 * a)
    frame = (D["rsqrt"] + 18 * a) if cyl else 0.0
    W = _density_cost(mosaic)
    sc = D["sincos"]
    # per node: b = 2 cos(a) cos(beta) sin^2(psi_j / 2), the densities, and
    # the weighted sums (two FMAs)
    quad = (2 * D["asin"] + 4 * sc + 10 * a + 2 * W
            + psi_nodes * (_node_cost(mosaic, vmf_live) + 3 * a) + sc + 3 * a)
    event = (OP_COSTS["philox"] + 3 * 2 * a + exit_d + frame + 5 * a + quad
             + D["log"] + 2 * D["div"] + 14 * a)
    R = _irc_cost(irc)
    # a Delta move takes cos(b) from the half angle's sin/cos (one sincos
    # and five operations)
    sweep = (OP_COSTS["philox"] + 4 * 2 * a + 9 * a + sc + (W + 8 * a) + 3 * a
             + 7 * a + R + sc + 9 * a + (W + 8 * a) + 3 * a)
    orient = 2 * sc + 3 * D["div"] + 15 * a + 9 * a + 5 * a + 15 * a + 11 * a + D["sqrt"] + 3 * D["div"]
    reflection = (D["asin"] + sc + D["div"] + sc + R + sc + 5 * a + 3 * a + W + burn_in * sweep
                  + orient)
    if pol:
        # Eq. SimpleReflXsectionPol: the sum of W cos(2 psi) beside the plain
        # one on every node (an FMA per side with the weighted table), the
        # polarisation's frame (u, k x u, two dots, their normalisation) and
        # sin^2(2 beta) per event; Eq. ReflXsectionPol: the frame once per
        # reflection and, per sweep, G in both target evaluations and
        # sin^2(2 b) in the Delta move; the polarisation's update after the
        # reflection
        frame_p = 6 * D["div"] + 30 * a + D["sqrt"] + D["div"] + 4 * a
        event += psi_nodes * 2 * a + frame_p + sc + 8 * a
        # (the polarised Delta move keeps the sin/cos of b beside the half
        # angle's sine)
        sweep_extra = 2 * 6 * a + 3 * a + sc - 5 * a
        sweep += sweep_extra
        reflection += (frame_p + sc - 5 * a + burn_in * sweep_extra + 14 * a + D["sqrt"]
                       + 3 * D["div"])
    return {"ray": base["ray"], "entered": base["entered"], "event": event,
            "reflection": reflection, "detected": base["detected"], "sweep": sweep,
            "quadrature": quad}


def algorithmic_ops_mwg(workload, counters, psi_nodes, burn_in, pol=False):
    """Issue slots the paper's model needs for a trace with these counters
    (every event priced with the quadrature; events past a ray's reflection
    cap skip it, which over-prices them slightly); `pol`: with polarisation."""
    m = workload["mosaic"]
    M = mix_mwg(workload["crystal"]["geometry"], m["kind"], workload["rocking_curve"]["kind"],
                workload["source"]["spectrum"], psi_nodes, burn_in, pol,
                vmf_live_fraction(m["fwhm"], psi_nodes))
    c = counters
    entered = c["emitted"] - c["missed"]
    return (c["emitted"] * M["ray"] + entered * M["entered"] + c["events"] * M["event"]
            + c["reflections"] * M["reflection"] + c["detected"] * M["detected"])


# ---- the extended source and polarisation (stepping model) -------------------

def algorithmic_ops_ext(workload, precision, counters, spot=False, pol=False, planes=0):
    """Issue slots of a stepping-model trace with a source spot,
    polarisations and/or `planes` further plane sets: the plain mix plus,
    per emitted ray with a spot, the second source draw, the Box-Muller
    offset (FP64 log, sqrt, sin/cos) and the move in the spot plane; with
    polarisations, per tilt the reflected direction (needed before the
    decision), G = 1 - (p.k_s)^2 and u / G, and per reflection the
    projection and renormalisation of p; with further sets, per tilt and set
    its sin(alpha_B) (one FP64 product), cos(alpha_B) (FP32 sqrt) and the
    FP32 bounds of its curve, and the weighted sums and the FP64 comparison.
    The counters already hold the events of the summed majorant."""
    base = algorithmic_ops(workload, precision, counters)
    D = OP_COSTS["f64"]
    R = OP_COSTS["f64"] if precision == "fp64" else OP_COSTS["f32"]
    a = SLOT_WEIGHT["alu64"] if precision == "fp64" else SLOT_WEIGHT["fp32"]
    d = SLOT_WEIGHT["alu64"]
    c = counters
    extra = 0.0
    if spot:
        extra += c["emitted"] * (OP_COSTS["philox"] + 4 * d + D["log"] + D["sqrt"] + D["sincos"]
                                 + 12 * d)
    if pol:
        ended = c["absorbed"] + c["exit_reflected"] + c["exit_transmitted"]
        tilts = max(0, c["events"] - ended)
        extra += tilts * (10 * a + R["rsqrt"] + 6 * d + D["div"])
        extra += c["reflections"] * (6 * a + R["rsqrt"])
    if planes:
        ended = c["absorbed"] + c["exit_reflected"] + c["exit_transmitted"]
        tilts = max(0, c["events"] - ended)
        F = OP_COSTS["f32"]
        f = SLOT_WEIGHT["fp32"]
        irc = workload["rocking_curve"]["kind"]
        per_set = d + 2 * d + F["sqrt"] + 2 * f + OP_COSTS["filter"][irc] + 4 * f
        extra += tilts * (planes * per_set + 4 * f + 6 * d)
    return base + extra
