#!/usr/bin/env python3
"""Throughput of the per-ray mosaic-crystal transport on one MI355X.

One step traces one batch of rays of the von Hamos HAPG(002) spectrometer
(R = 80 mm, 100 x 30 mm, 40 um, pseudo-Voigt mosaic 0.1 deg with eta = 0.3,
pseudo-Voigt rocking curve 50/8 urad, two lines at 8.048 / 8.028 keV on a flat
7.8-8.2 keV background, up to 4 reflections, 2048 x 512 detector at 50 um):
1e8 rays in FP64, images resident in HBM and accumulated step after step
(step s traces ray ids [s N, (s + 1) N), so K steps are one K N-ray
simulation).  The same steps are then run in FP32-mixed precision.

Then the request server serves 256 spectrometer-design requests (varied
crystal radius, mosaic, thickness, energy window; ray counts log-uniform in
1e5-1e8) in each precision: once all queued at once (saturated rays/s), once
with Poisson arrivals at 0.7 times that rate (p50/p99 latency from submission
to completion, rays/s).

The same workload is also traced in the paper's own event model (free paths
at mu0 + gamma0 sigma(alpha) with sigma from the psi quadrature of Eq.
SimpleReflXsection, reflecting crystallites from Metropolis-within-Gibbs with
500 sweeps), FP64, with its own roofline and oracle rate ("mwg_model").

Each timed region enqueues its K traces back to back on one stream (the
host does not wait between them); the same rays are then traced again with
counters, whose unit counts and per-kernel HIP-event durations give the
rooflines.

Printed: one JSON line with rays/s (FP64 is `value`), events/s, the ALU
roofline of the trace kernel (algorithmic VALU lane-operations per launch over
the kernel's HIP-event duration on its stream, against 256 CUs x 64 lanes x
2.4 GHz), the serving figures, and the FP64 CPU oracle timed on a bounded
sample of the same workload on the host's cores.
"""
import argparse
import copy
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/sec traced (FP32-mixed vs FP64) at matched image; serving p50/p99 latency"
PEAK_CLOCK_HZ = 2.4e9            # MI355X peak engine clock
LANES_PER_CU_PER_CLK = 64        # issue slots per CU and clock: the FP64 FMA lane rate


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_precision(mrt, w, precision, steps, warmup, n, counts, energy, refill=0, rays=None):
    """Warm up, then time `steps` traces of n rays enqueued back to back on
    one stream (no host wait between them), then trace the same rays again
    with counters (unit counts and each kernel's own duration, for the
    roofline).  Returns (per-step counters, timed GPU ms, timed wall s)."""
    import torch
    first_base = 1 << 40          # warm-up rays come from a separate id range
    for s in range(warmup):
        mrt.trace(w, n_rays=n, first=first_base + s * n, precision=precision, counts=counts,
                  energy=energy, refill_idle=refill, rays=rays)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for s in range(steps):
        mrt.trace(w, n_rays=n, first=s * n, precision=precision, counts=counts, energy=energy,
                  accumulate=s > 0, stream=stream, refill_idle=refill, rays=rays, sync=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    per_step = []
    for s in range(steps):
        out = mrt.trace(w, n_rays=n, first=s * n, precision=precision, counts=counts,
                        energy=energy, accumulate=s > 0, stream=stream, refill_idle=refill,
                        rays=rays)
        per_step.append(out["counters"])
        log(f"{precision} step {s}: kernel {out['counters']['kernel_ms']:.2f} ms")
    return per_step, gpu_ms, wall


KIND = {"geometry": {"flat": 0, "cylinder": 1},
        "mosaic": {"gaussian_vmf": 0, "lorentzian": 1, "pseudo_voigt": 2, "wrapped_lorentzian": 3,
                   "spherical_wrapped_lorentzian": 4},
        "irc": {"gaussian": 0, "pseudo_voigt": 1, "table": 2, "lorentzian": 3, "box": 4}}


def kernel_name(w, precision, records=False):
    """The trace-kernel instance a workload runs (as profilers name it)."""
    r = "double" if precision == "fp64" else "float"
    g = KIND["geometry"][w["crystal"]["geometry"]]
    m = KIND["mosaic"][w["mosaic"]["kind"]]
    i = KIND["irc"][w["rocking_curve"]["kind"]]
    return (f"void mrt::tk::trace_kernel<{r}, {g}, {m}, {i}, {'true' if records else 'false'}>"
            "(mrt::TraceParams)")


def roofline(op_costs, profiling, w, precision, per_step, cus):
    ops = [op_costs.algorithmic_ops(w, precision, c) for c in per_step]
    ms = [c["kernel_ms"] for c in per_step]
    achieved = sum(o / (m * 1e-3) for o, m in zip(ops, ms)) / len(ops) / 1e12
    peak = cus * LANES_PER_CU_PER_CLK * PEAK_CLOCK_HZ / 1e12
    name = kernel_name(w, precision)
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": round(peak, 4),
            "unit": "TOP/s", "frac": round(achieved / peak, 4),
            "traffic": profiling.traffic_per_launch(name),
            "kernel": name, "op": "VALU issue slot (one FP64-FMA lane; measured relative costs, FP32 arithmetic 0.5)",
            "ops_per_launch": int(sum(ops) / len(ops)),
            "kernel_ms_avg": round(sum(ms) / len(ms), 4),
            "issue": profiling.issue_ratios(name, sum(ops) / len(ops), sum(ms) / len(ms), cus)}


def mwg_kernel_name(w, records=False, polarised=False, planes=False):
    g = KIND["geometry"][w["crystal"]["geometry"]]
    b = lambda x: "true" if x else "false"
    return (f"void mrt::tk::mwg_kernel<{g}, {b(records)}, {b(polarised)}, {b(planes)}>"
            "(mrt::TraceParams)")


def roofline_mwg(op_costs, profiling, w, per_step, cus, psi_nodes, burn_in):
    ops = [op_costs.algorithmic_ops_mwg(w, c, psi_nodes, burn_in) for c in per_step]
    ms = [c["kernel_ms"] for c in per_step]
    achieved = sum(o / (m * 1e-3) for o, m in zip(ops, ms)) / len(ops) / 1e12
    peak = cus * LANES_PER_CU_PER_CLK * PEAK_CLOCK_HZ / 1e12
    name = mwg_kernel_name(w)
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": round(peak, 4),
            "unit": "TOP/s", "frac": round(achieved / peak, 4),
            "traffic": profiling.traffic_per_launch(name),
            "kernel": name, "op": "VALU issue slot (one FP64-FMA lane; measured relative costs, FP32 arithmetic 0.5)",
            "ops_per_launch": int(sum(ops) / len(ops)),
            "kernel_ms_avg": round(sum(ms) / len(ms), 4),
            "issue": profiling.issue_ratios(name, sum(ops) / len(ops), sum(ms) / len(ms), cus)}


def mwg_model(mrt, op_costs, profiling, w, n, steps, warmup, burn_in, psi_nodes, cus, cpu_rays,
              stepping_value):
    """The paper's event model on the same workload and ray ids (FP64)."""
    import copy
    wm = copy.deepcopy(w)
    wm["event_model"] = {"kind": "mwg", "burn_in": burn_in, "psi_nodes": psi_nodes}
    counts, energy = mrt.alloc_images(wm)
    per, gms, wall = run_precision(mrt, wm, "fp64", steps, warmup, n, counts, energy)
    rays = n * steps
    refl = sum(c["reflections"] for c in per)
    out = {"value": round(rays / (gms * 1e-3), 1), "unit": "rays/s", "steps": steps,
           "ms_per_step": round(gms / steps, 4), "burn_in": burn_in, "psi_nodes": psi_nodes,
           "events_per_s": round(sum(c["events"] for c in per) / (gms * 1e-3), 1),
           "reflections_per_s": round(refl / (gms * 1e-3), 1),
           "sweeps_per_s": round(refl * burn_in / (gms * 1e-3), 1),
           "vs_stepping": round(rays / (gms * 1e-3) / stepping_value, 4),
           "roofline": roofline_mwg(op_costs, profiling, wm, per, cus, psi_nodes, burn_in),
           "counters_last_step": {k: v for k, v in per[-1].items() if k != "kernel_ms"}}
    # with every ray polarised along the source's b1 (Eqs.
    # SimpleReflXsectionPol, ReflXsectionPol), on the same rays
    import torch
    b1 = torch.as_tensor(w["source"]["b1"], dtype=torch.float64, device="cuda")
    pol = {"polarisations": b1.expand(n, 3).contiguous()}
    pp, pms, _ = run_precision(mrt, wm, "fp64", steps, warmup, n, counts, energy, rays=pol)
    del pol
    ops = [op_costs.algorithmic_ops_mwg(wm, c, psi_nodes, burn_in, pol=True) for c in pp]
    ach = sum(o / (c["kernel_ms"] * 1e-3) for o, c in zip(ops, pp)) / len(pp) / 1e12
    peak = cus * LANES_PER_CU_PER_CLK * PEAK_CLOCK_HZ / 1e12
    out["polarised"] = {"value": round(rays / (pms * 1e-3), 1), "unit": "rays/s",
                        "ms_per_step": round(pms / steps, 4),
                        "vs_unpolarised": round(gms / pms, 4),
                        "roofline": {"bound": "alu", "achieved": round(ach, 4),
                                     "peak": round(peak, 4), "unit": "TOP/s",
                                     "frac": round(ach / peak, 4),
                                     "traffic": profiling.traffic_per_launch(
                                         mwg_kernel_name(wm, polarised=True)),
                                     "kernel": mwg_kernel_name(wm, polarised=True)}}
    log(f"paper's model, polarised: {out['polarised']['value']:.3e} rays/s")
    if cpu_rays:
        import oracle
        threads = min(16, len(os.sched_getaffinity(0)))
        log(f"oracle, paper's model: {cpu_rays} rays on {threads} threads")
        t0 = time.perf_counter()
        oracle.trace(wm, first=0, n=cpu_rays, threads=threads, images=True)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(cpu_rays / dt, 1), "unit": "rays/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"ray ids [0, {cpu_rays}) of the same workload in the "
                                         f"paper's model, FP64, images on, {dt:.2f} s"}
    return out


def stress(mrt, W, op_costs, profiling, precision, cus, rays_per_step, steps):
    """The stress workload (100 um HOPG, Lorentzian 0.8 deg mosaic,
    Darwin-Prins table curve, 1024-bin spectrum, up to 8 reflections, 4096^2
    detector): ray ids [0, steps x rays_per_step) in both precisions, their
    rooflines, FP32-mixed against FP64 (chi^2 per pixel of the images; the
    fraction of detected rays on another pixel, from records of 1e7 rays)."""
    import torch
    w = W.get("flat_stress")
    out = {"workload": "flat_stress: flat HOPG(002) 100 um, Lorentzian mosaic 0.8 deg, "
                       "Darwin-Prins table rocking curve, 1024-bin spectrum, max 8 reflections, "
                       "4096x4096 px", "rays": rays_per_step * steps}
    imgs = {}
    for prec in ("fp64", "fp32_mixed"):
        c, e = mrt.alloc_images(w)
        ps, gms, _ = run_precision(mrt, w, prec, steps, 1, rays_per_step, c, e)
        out[prec] = {"value": round(rays_per_step * steps / (gms * 1e-3), 1), "unit": "rays/s",
                     "ms_per_step": round(gms / steps, 4),
                     "events_per_s": round(sum(x["events"] for x in ps) / (gms * 1e-3), 1),
                     "roofline": roofline(op_costs, profiling, w, prec, ps, cus)}
        imgs[prec] = mrt.image_to_numpy(c)[0]
        del c, e
    # the same seed's images share their noise: their chi-square per pixel
    # measures the difference only; FP32-mixed at an independent seed against
    # FP64 is the test (expectation 1 per pixel with counts)
    out["fp32_vs_fp64_chi2_per_px_same_seed"] = round(
        precision.chi2_per_pixel(imgs["fp32_mixed"], imgs["fp64"]), 5)
    out["fp32_vs_fp64_chi2_per_px"] = round(precision.chi2_per_pixel(
        independent_image(mrt, w, "fp32_mixed", rays_per_step, steps), imgs["fp64"]), 5)
    n = 10_000_000
    r64 = mrt.trace(w, n_rays=n, precision="fp64", records="all")["records"]
    r32 = mrt.trace(w, n_rays=n, precision="fp32_mixed", records="all")["records"]
    i64, i32 = r64.view(torch.int32), r32.view(torch.int32)
    d64, d32 = r64[:, 103] == 1, r32[:, 103] == 1
    moved = (d64 != d32) | (d64 & ((i64[:, 22] != i32[:, 22]) | (i64[:, 23] != i32[:, 23])))
    out["detected_rays_moved_fraction"] = float(moved.sum().item()) / max(1, int(d64.sum().item()))
    del r64, r32, i64, i32
    log(f"stress: fp64 {out['fp64']['value']:.3e}, fp32_mixed {out['fp32_mixed']['value']:.3e} rays/s")
    return out


def independent_image(mrt, w, precision, n, steps, offset=1000):
    """Counts image of ray ids [0, steps n) at seed + offset (noise
    independent of the workload's own seed)."""
    c, e = mrt.alloc_images(w, energy=False)
    for s in range(steps):
        mrt.trace(w, n_rays=n, first=s * n, seed=w["seed"] + offset, precision=precision,
                  counts=c, energy=e, accumulate=s > 0, want_energy=False, sync=False)
    img = mrt.image_to_numpy(c)[0]
    del c
    return img


def extended_inputs(mrt, W, op_costs, w, n, steps, warmup, cus, plain):
    """The extended inputs on the benchmark workload: the paper's 10 um
    Gaussian XFEL spot (sec. 4.2), which runs in the kernels specialised
    for the kinds; the spot with every ray polarised along the source's b1
    (normal to the cone axis; a 2.4 GB device array) and the spot with the
    antiparallel planes at 0.8 and the (004) order at 0.3, which run in
    the extended kernels (trace_kernel_ext).  `plain` maps precision
    to the tuned kernel's rays/s on the plain workload."""
    import torch
    spot = W.with_spot(w)
    b1 = torch.as_tensor(w["source"]["b1"], dtype=torch.float64, device="cuda")
    pol = {"polarisations": b1.expand(n, 3).contiguous()}
    planes = copy.deepcopy(spot)
    planes["crystal"]["planes"] = {"hbar_ratio": 0.8,
                                   "extra": [(w["crystal"]["two_d"] / 2, 0.3, 1.0, 0.0)]}
    peak = cus * LANES_PER_CU_PER_CLK * PEAK_CLOCK_HZ / 1e12
    counts, energy = mrt.alloc_images(w)      # images of its own
    out = {"note": "the benchmark workload with a spot (tuned kernels), and with polarisations "
                   "or plane sets (trace_kernel_ext)"}
    for label, wl, rays, priced in (("xfel_spot", spot, None, dict(spot=True)),
                                    ("xfel_spot_polarised", spot, pol, dict(spot=True, pol=True)),
                                    ("xfel_spot_planes", planes, None, dict(spot=True, planes=1))):
        entry = {}
        for prec in ("fp64", "fp32_mixed"):
            ps, gms, _ = run_precision(mrt, wl, prec, steps, warmup, n, counts, energy, rays=rays)
            v = n * steps / (gms * 1e-3)
            e = {"value": round(v, 1), "unit": "rays/s", "ms_per_step": round(gms / steps, 4),
                 "vs_tuned_kernel": round(v / plain[prec], 3) if plain.get(prec) else None,
                 "refined_per_event": round(sum(c["refined"] for c in ps) / max(1, sum(c["events"] for c in ps)), 5)}
            if priced is not None:
                ops = [op_costs.algorithmic_ops_ext(wl, prec, c, **priced) for c in ps]
                ach = sum(o / (c["kernel_ms"] * 1e-3) for o, c in zip(ops, ps)) / len(ps) / 1e12
                e["roofline"] = {"bound": "alu", "achieved": round(ach, 4), "peak": round(peak, 4),
                                 "unit": "TOP/s", "frac": round(ach / peak, 4)}
            entry[prec] = e
        out[label] = entry
        log(f"extended {label}: fp64 {entry['fp64']['value']:.3e} rays/s")
    del pol
    return out


def burn_in_study(mrt, W, precision, n, burn_ins=(0, 100, 500, 1500), half=40):
    """The paper's burn-in figure (sec. 2.2.4, Fig. BurnIn): the instrument
    function of an 8.5 keV point source on a von Hamos spectrometer aimed at
    8.5 keV (Lorentzian mosaic 0.14 deg, Voigt curve 50.7 / 10.0 urad), in
    the stepping model (exact at any burn-in: it draws each crystallite
    directly) and in the paper's event model at several burn-ins of its
    Metropolis-within-Gibbs sampler, n rays each at independent seeds, FP64.
    Per run: the line's centroid and FWHM over +-half pixels of the focus
    and the chi-square per pixel against the stepping image (1 for
    independent images of one mean; the stepping model at another seed is
    the control), with the kernel time."""
    import copy
    w = W.get("von_hamos_burn_in")
    col = precision.von_hamos_line_column(w, 8.5)

    def run(wl, seed):
        r = mrt.trace(wl, n_rays=n, seed=seed, precision="fp64", want_energy=False)
        img = mrt.image_to_numpy(r["counts"])[0]
        del r["counts"]
        return img, r["counters"]["kernel_ms"]

    ref, ms_ref = run(w, 100)
    pref = precision.dispersive_profile(ref)

    def summary(img, ms):
        p = precision.dispersive_profile(img)
        c, f = precision.centroid(p, col, half), precision.fwhm(p, col, half)
        return {"kernel_ms": round(ms, 3), "centroid_px": round(c, 4),
                "centroid_shift_px": round(c - precision.centroid(pref, col, half), 4),
                "fwhm_px": round(f, 4),
                "fwhm_change": round(f / precision.fwhm(pref, col, half) - 1.0, 5),
                "chi2_per_px": round(precision.chi2_per_pixel(img, ref), 4)}

    out = {"workload": "von_hamos_burn_in: 8.5 keV point source, von Hamos R=80 mm aimed at "
                       "8.5 keV, Lorentzian mosaic 0.14 deg, Voigt curve 50.7/10.0 urad, FP64",
           "rays": n, "focus_col": round(col, 3),
           "stepping": {"kernel_ms": round(ms_ref, 3),
                        "centroid_px": round(precision.centroid(pref, col, half), 4),
                        "fwhm_px": round(precision.fwhm(pref, col, half), 4)}}
    out["stepping_control"] = summary(*run(w, 101))
    for b in burn_ins:
        wm = copy.deepcopy(w)
        wm["event_model"] = {"kind": "mwg", "burn_in": b, "psi_nodes": 256}
        out[f"mwg_burn_in_{b}"] = summary(*run(wm, 200 + b))
        log(f"burn-in {b}: {out[f'mwg_burn_in_{b}']}")
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# The GPU host grants the process of one GPU a share of 16 cores, whatever
# the number of CPUs it can see; the oracle runs one thread per core of it.
CPU_SHARE = 16


def cpu_baseline(w, n):
    import oracle
    visible = len(os.sched_getaffinity(0))
    threads = min(CPU_SHARE, visible)
    log(f"oracle: {n} rays on {threads} threads ({visible} CPUs visible, {cpu_model()})")
    t0 = time.perf_counter()
    r = oracle.trace(w, first=0, n=n, threads=threads)
    dt = time.perf_counter() - t0
    # and on one core, over a tenth of the sample
    n1 = max(1, n // 10)
    t1 = time.perf_counter()
    oracle.trace(w, first=0, n=n1, threads=1)
    dt1 = time.perf_counter() - t1
    log(f"oracle: {n1} rays on 1 thread")
    return {"value": round(n / dt, 1), "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"ray ids [0, {n}) of the same workload, FP64, images on, {dt:.2f} s",
            "cpu_model": cpu_model(), "cpus_visible": visible,
            "cores_note": f"one thread per core of the {CPU_SHARE}-core share the host grants "
                          "one GPU's process",
            "events": r["counters"]["events"],
            "one_core": {"value": round(n1 / dt1, 1), "unit": "rays/s",
                         "sample": f"ray ids [0, {n1}), {dt1:.2f} s"}}, r


def precision_report(mrt, precision, w, c64, c32, n, steps, oracle_result, n_oracle, detected):
    """FP32-mixed against FP64 at the same rays (centroid and FWHM per line:
    shared noise shows small differences; their chi-square per pixel is a
    difference measure), FP32-mixed at an independent seed against FP64
    (the chi-square test, expectation 1 per pixel with counts, beside FP64
    against FP64), and both against the oracle."""
    import numpy as np
    import torch
    lines = [e for e, _, _ in w["source"].get("lines", [])]
    a64, _ = mrt.image_to_numpy(c64)
    a32, _ = mrt.image_to_numpy(c32)
    rays = n * steps
    # the images must be the ones the timed steps made (nothing traced into
    # them since): each holds exactly the detected rays of its steps
    for img, det, name in ((a64, detected[0], "fp64"), (a32, detected[1], "fp32_mixed")):
        if int(img.sum(dtype=np.uint64)) != det:
            raise RuntimeError(f"precision report: the {name} image holds {int(img.sum())} "
                               f"counts, its steps detected {det}")
    cmp = precision.compare_images(w, a32, a64, lines)
    cmp["chi2_per_px_same_seed"] = cmp.pop("chi2_per_px")
    i32 = independent_image(mrt, w, "fp32_mixed", n, steps)
    i64 = independent_image(mrt, w, "fp64", n, steps)
    cmp["chi2_per_px"] = round(precision.chi2_per_pixel(i32, a64), 5)
    cmp["chi2_per_px_fp64_control"] = round(precision.chi2_per_pixel(i64, a64), 5)
    cmp["chi2_note"] = (f"chi2_per_px: fp32_mixed at seed {w['seed'] + 1000} against fp64 at seed "
                        f"{w['seed']} over the same {rays} ray ids (independent noise, expectation "
                        f"1); the fp64 control is fp64 at seed {w['seed'] + 1000}")
    del i32, i64
    rep = {"rays": rays, "fp32_vs_fp64": cmp}
    # per-ray pixel changes on a sample, from device records of both paths
    n = min(n_oracle, 10_000_000)
    r64 = mrt.trace(w, n_rays=n, precision="fp64", records="all")["records"]
    r32 = mrt.trace(w, n_rays=n, precision="fp32_mixed", records="all")["records"]
    i64, i32 = r64.view(torch.int32), r32.view(torch.int32)
    d64, d32 = r64[:, 103] == 1, r32[:, 103] == 1
    moved = (d64 != d32) | (d64 & ((i64[:, 22] != i32[:, 22]) | (i64[:, 23] != i32[:, 23])))
    rep["sample_rays"] = n
    rep["detected_rays_moved_fraction"] = float(moved.sum().item()) / max(1, int(d64.sum().item()))
    del r64, r32, i64, i32
    if oracle_result is not None:
        g64 = mrt.trace(w, n_rays=n_oracle, precision="fp64")
        g32 = mrt.trace(w, n_rays=n_oracle, precision="fp32_mixed")
        o, _ = oracle_result["counts"], None
        b64, e64 = mrt.image_to_numpy(g64["counts"], g64["energy"])
        b32, _ = mrt.image_to_numpy(g32["counts"])
        rep["oracle_rays"] = n_oracle
        rep["fp64_vs_oracle_bit_exact"] = bool(np.array_equal(b64, o) and
                                               np.array_equal(e64, oracle_result["energy_mev"]))
        rep["fp64_vs_oracle_pixels_differing"] = int(np.count_nonzero(b64 != o))
        cmp_o = precision.compare_images(w, b32, o, lines)
        cmp_o["chi2_per_px_same_seed"] = cmp_o.pop("chi2_per_px")   # shared noise
        rep["fp32_vs_oracle"] = cmp_o
    return rep


def serving_run(mrt, reqs, precision, budget, max_slots, gaps_s=None, round_rays=0):
    """Serve the requests: submitted all at once (gaps_s None) or with the
    given inter-arrival gaps; a consumer thread takes each finished request
    from the completion queue and releases it at once.  Returns per-request
    latencies (ms, server clock), rays, the span from first submission to last
    completion (s), the server's stats and (workload, counters) of every
    request."""
    import threading
    n = len(reqs)
    done = []
    by_ticket = {}
    srv = mrt.Server(hbm_budget_bytes=budget, max_slots=max_slots, precision=precision,
                     round_rays=round_rays)

    def consume():
        for _ in range(n):
            t, r = srv.wait_any(views=False)
            if r["state"] != "done":
                raise RuntimeError(f"request {t} ended {r['state']} (status {r['status']})")
            r["ticket"] = t
            done.append(r)
            srv.release(t)

    th = threading.Thread(target=consume)
    th.start()
    try:
        for i, w in enumerate(reqs):
            if gaps_s is not None and i:
                time.sleep(gaps_s[i])
            by_ticket[srv.submit(w)] = w
        th.join()
        st = srv.stats()
    finally:
        srv.close()
    if len(done) != n:
        raise RuntimeError("serving: not every request finished")
    lat = [r["done_ms"] - r["submit_ms"] for r in done]
    span = (max(r["done_ms"] for r in done) - min(r["submit_ms"] for r in done)) * 1e-3
    return lat, span, st, [(by_ticket[r["ticket"]], r["counters"]) for r in done]


def sequential_run(mrt, reqs, precision):
    """The same requests traced one mrt_trace call after another on one
    stream (each with the kernel specialised for its kinds), as the reference
    point for the server.  Returns (seconds, events)."""
    import torch
    counts, energy = mrt.alloc_images(reqs[0])
    stream = torch.cuda.current_stream()
    mrt.trace(reqs[0], n_rays=1 << 16, precision=precision, counts=counts, energy=energy)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    events = 0
    for w in reqs:
        out = mrt.trace(w, precision=precision, counts=counts, energy=energy, stream=stream)
        events += out["counters"]["events"]
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) * 1e-3, events


def serving(mrt, W, op_costs, cus, n_requests, budget, max_slots, load, seed=4, round_rays=0):
    """The serving workload (design requests of varied geometry and ray
    count): for each precision, the saturated throughput (all requests queued
    at once), then Poisson arrivals at `load` times that throughput with
    p50/p99 latency."""
    import numpy as np
    reqs = W.serving_requests(n=n_requests, seed=seed)
    rays = sum(w["n_rays"] for w in reqs)
    out = {"requests": n_requests, "total_rays": rays, "hbm_budget_bytes": budget,
           "max_slots": max_slots, "load": load,
           "mix": "von Hamos R 60-120 mm, mosaic FWHM 0.05-0.8 deg (von Mises-Fisher / Lorentzian / "
                  "pseudo-Voigt), 20-100 um, 0.1-0.4 keV windows at 7.5-8.5 keV, "
                  "rays log-uniform 1e5-1e8"}
    for prec in ("fp32_mixed", "fp64"):
        for w in reqs:
            w["precision"] = prec
        seq_s, seq_events = sequential_run(mrt, reqs, prec)
        lat0, span0, st0, per_req = serving_run(mrt, reqs, prec, budget, max_slots,
                                                round_rays=round_rays)
        sat = rays / span0
        rate = load * sat / (rays / n_requests)           # requests per second
        gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, n_requests)
        lat, span, st, _ = serving_run(mrt, reqs, prec, budget, max_slots, gaps, round_rays)
        # the serving kernel's ALU roofline: the priced work of every
        # request (its own counters and kinds) over the time the device was
        # tracing rounds (the union of the rounds' HIP-event intervals), and
        # over the whole saturated run
        ops = sum(op_costs.algorithmic_ops(w, prec, c) for w, c in per_req)
        peak = cus * LANES_PER_CU_PER_CLK * PEAK_CLOCK_HZ / 1e12
        busy = st0["busy_ms"] * 1e-3
        serve_roof = {"bound": "alu", "achieved": round(ops / busy / 1e12, 4), "peak": round(peak, 4),
                      "unit": "TOP/s", "frac": round(ops / busy / 1e12 / peak, 4),
                      "frac_whole_run": round(ops / span0 / 1e12 / peak, 4),
                      "kernel": f"serve_kernel<{'double' if prec == 'fp64' else 'float'}>",
                      "ops": round(ops, 1), "busy_s": round(busy, 4)}
        out[prec] = {
            "one_call_per_request_rays_per_s": round(rays / seq_s, 1),
            "events_per_ray": round(seq_events / rays, 3),
            "saturated_rays_per_s": round(sat, 1),
            "saturated_gpu_busy": round(st0["busy_ms"] * 1e-3 / span0, 3),
            "arrival_rate_per_s": round(rate, 2),
            "rays_per_s": round(rays / span, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "max_ms": round(float(np.max(lat)), 2),
            "rounds": int(st["rounds"]),
            "roofline": serve_roof,
        }
        log(f"serving {prec}: saturated {sat:.3e} rays/s, Poisson {rate:.1f}/s: "
            f"p50 {out[prec]['p50_ms']} ms p99 {out[prec]['p99_ms']} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="von_hamos_hapg")
    ap.add_argument("--rays", type=int, default=0, help="rays per step (0 = the workload's)")
    ap.add_argument("--cpu-rays", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--refill", type=int, default=0, help="lanes idle before a wave refills (0 = default)")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-budget-mib", type=int, default=4096)
    ap.add_argument("--serving-load", type=float, default=0.7)
    ap.add_argument("--serving-round-rays", type=int, default=0, help="rays per round (0 = the server's default)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--mwg-steps", type=int, default=3, help="steps of the paper's event model")
    ap.add_argument("--mwg-burn-in", type=int, default=500)
    ap.add_argument("--mwg-psi-nodes", type=int, default=256)
    ap.add_argument("--mwg-cpu-rays", type=int, default=20_000_000)
    ap.add_argument("--no-mwg", action="store_true")
    ap.add_argument("--no-burn-in", action="store_true",
                    help="skip the burn-in study (stepping vs the paper's model, Fig. BurnIn)")
    ap.add_argument("--burn-in-rays", type=int, default=100_000_000)
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the stress workload (2e9 rays per precision)")
    ap.add_argument("--no-extended", action="store_true",
                    help="skip the extended-input kernels (spot, polarisation, planes)")
    ap.add_argument("--shard-of", type=int, default=8,
                    help="also time one GPU's share of the launch split over this many GPUs "
                         "(0 = skip)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the transport shards by ray-id ranges with one "
              "integer image reduce, but this build runs and reports a single MI355X only.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_16955_amd import mosaicrt as mrt
    from paper_2503_16955_amd import op_costs, profiling
    from paper_2503_16955_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2503_16955_amd import precision

    w = W.get(a.workload)
    n = a.rays or w["n_rays"]
    info = mrt.device_info()
    log(f"device {info['name']} {info['arch']} CUs {info['compute_units']}")
    counts, energy = mrt.alloc_images(w)
    counts32, energy32 = mrt.alloc_images(w)

    per64, gpu_ms64, wall64 = run_precision(mrt, w, "fp64", a.steps, a.warmup, n, counts, energy,
                                            a.refill)
    rays = n * a.steps
    value = rays / (gpu_ms64 * 1e-3)
    events64 = sum(c["events"] for c in per64)
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "rays/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(gpu_ms64 / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: von Hamos HAPG(002) R=80 mm, PV mosaic 0.1 deg "
                               "eta=0.3, PV rocking curve 50/8 urad, 2 lines + flat, "
                               "max 4 reflections, 2048x512 px",
                   "rays_per_step": n, "seed": w["seed"], "precision": "fp64",
                   "parallelism": "1 GPU"},
        "events_per_s": round(events64 / (gpu_ms64 * 1e-3), 1),
        "wall_s": round(wall64, 3),
        "roofline": roofline(op_costs, profiling, w, "fp64", per64, info["compute_units"]),
        "counters_last_step": {k: v for k, v in per64[-1].items() if k != "kernel_ms"},
    }
    if not a.no_mixed:
        pm, gms, wl = run_precision(mrt, w, "fp32_mixed", a.steps, a.warmup, n, counts32,
                                    energy32, a.refill)
        res["fp32_mixed"] = {
            "value": round(rays / (gms * 1e-3), 1), "unit": "rays/s",
            "ms_per_step": round(gms / a.steps, 4),
            "events_per_s": round(sum(c["events"] for c in pm) / (gms * 1e-3), 1),
            "speedup_vs_fp64": round(gpu_ms64 / gms, 3),
            "roofline": roofline(op_costs, profiling, w, "fp32_mixed", pm, info["compute_units"]),
        }
    if not a.no_stress and not a.no_mixed:
        res["stress"] = stress(mrt, W, op_costs, profiling, precision, info["compute_units"],
                               1_000_000_000, 2)
    if not a.no_extended and not a.no_mixed:
        res["extended"] = extended_inputs(
            mrt, W, op_costs, w, n, a.steps, a.warmup, info["compute_units"],
            {"fp64": value, "fp32_mixed": res["fp32_mixed"]["value"]})
    if a.shard_of > 1:
        # one GPU's ray-id range when the launch is split over shard_of GPUs:
        # the shard kernel at its real shape (the integer image reduce that
        # would follow is not run on one GPU)
        ns = -(-n // a.shard_of)
        sh = {"gpus_modelled": a.shard_of, "rays_per_step": ns,
              "note": "ray ids [0, n/G) of the same workload on this GPU; no image reduce"}
        for prec in ("fp64", "fp32_mixed"):
            if prec == "fp32_mixed" and a.no_mixed:
                continue
            # images of its own: the precision report below compares the
            # full-size FP64 and FP32-mixed images
            c_, e_ = mrt.alloc_images(w)
            ps, gms, _ = run_precision(mrt, w, prec, a.steps, a.warmup, ns, c_, e_, a.refill)
            del c_, e_
            sh[prec] = {"value": round(ns * a.steps / (gms * 1e-3), 1), "unit": "rays/s",
                        "ms_per_step": round(gms / a.steps, 4)}
        res["shard"] = sh
        log(f"shard 1/{a.shard_of}: fp64 {sh['fp64']['value']:.3e} rays/s")
    if not a.no_mwg:
        res["mwg_model"] = mwg_model(mrt, op_costs, profiling, w, n, a.mwg_steps, 1, a.mwg_burn_in,
                                     a.mwg_psi_nodes, info["compute_units"],
                                     0 if a.no_cpu_baseline else a.mwg_cpu_rays, value)
        log(f"paper's model: {res['mwg_model']['value']:.3e} rays/s, "
            f"{res['mwg_model']['ms_per_step']} ms per step")
    if not a.no_burn_in and not a.no_mwg:
        res["burn_in_study"] = burn_in_study(mrt, W, precision, a.burn_in_rays)
    res["serving"] = None if a.no_serving else serving(
        mrt, W, op_costs, info["compute_units"], a.serving_requests, a.serving_budget_mib << 20, 64,
        a.serving_load, round_rays=a.serving_round_rays)
    orc = None
    if not a.no_cpu_baseline:
        res["cpu_baseline"], orc = cpu_baseline(w, a.cpu_rays)
    if not a.no_mixed and w["source"]["spectrum"] == "lines" and w["crystal"]["geometry"] == "cylinder":
        res["precision"] = precision_report(
            mrt, precision, w, counts, counts32, n, a.steps, orc, a.cpu_rays,
            (sum(c["detected"] for c in per64), sum(c["detected"] for c in pm)))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
