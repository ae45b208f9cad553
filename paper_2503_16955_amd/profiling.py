"""Profile bookkeeping for the trace kernels.

* ``python -m paper_2503_16955_amd.profiling copy [--mib M]`` runs one plain
  device-to-device copy of M MiB: the reference that scales the HBM byte
  counters (FETCH_SIZE, WRITE_SIZE) of the same box.
* ``python -m paper_2503_16955_amd.profiling summarize ...`` turns rocprofv3
  CSV outputs (kernel trace with stats, and one ``--pmc`` pass per counter
  group) into a short markdown summary and ``hbm_traffic.json`` (HBM bytes
  per launch of each trace kernel, scaled by the copy reference, and the
  VALU-issue, lane-activity and atomic counters per launch).
* ``sources_sha256()`` fingerprints the kernel sources and build flags;
  ``hbm_traffic.json`` records it, and a reader treats the traffic as
  unknown once the kernels have changed since the counters were taken.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def sources_sha256():
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*.h")) +
                   glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                   glob.glob(os.path.join(HERE, "csrc", "*.cpp")) +
                   [os.path.join(ROOT, "include", "mosaicrt.h"), os.path.join(HERE, "build.py")])
    for f in files:
        if os.path.basename(f) == "op_cost_probe.hip":
            continue
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_per_launch(kernel_name):
    """HBM bytes per launch of a kernel from hbm_traffic.json, or None when the
    file is missing, lacks the kernel, or predates the current sources."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_sha256():
        return None
    k = t.get("kernels", {}).get(kernel_name)
    return None if k is None else k["hbm_bytes_per_launch"]


# SQ and L2 counters kept per kernel beside the traffic (means per dispatch)
ISSUE_COUNTERS = ("SQ_INSTS_VALU", "SQ_THREAD_CYCLES_VALU", "TCC_ATOMIC_sum")


def counters_per_launch(kernel_name):
    """{counter: mean per dispatch} of ISSUE_COUNTERS for a kernel from
    hbm_traffic.json, or None when missing or taken from other sources."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_sha256():
        return None
    k = t.get("kernels", {}).get(kernel_name)
    if k is None or not all(c in k.get("counters", {}) for c in ISSUE_COUNTERS):
        return None
    return k["counters"]


def issue_ratios(kernel_name, useful_lane_ops, kernel_ms, cus):
    """The survey's reported ratios for one launch from the profiled
    counters: VALU instructions per CU and clock at 2.4 GHz = SQ_INSTS_VALU
    / (t x CUs x 2.4 GHz) (FP64 and integer instructions issue at most one
    wave64 instruction per CU and clock, FP32 arithmetic up to two, so this
    is a rate rather than a fraction), lane efficiency = the priced
    lane-slots / (SQ_INSTS_VALU x 64), active lanes per VALU instruction =
    SQ_THREAD_CYCLES_VALU / SQ_INSTS_VALU, and L2 atomics per second.  None
    when the counters are missing or stale."""
    c = counters_per_launch(kernel_name)
    if c is None or not c["SQ_INSTS_VALU"]:
        return None
    t = kernel_ms * 1e-3
    v = c["SQ_INSTS_VALU"]
    return {"valu_insts_per_cu_clock": round(v / (t * cus * 2.4e9), 4),
            "lane_efficiency": round(useful_lane_ops / (v * 64.0), 4),
            "lanes_per_valu_inst": round(c["SQ_THREAD_CYCLES_VALU"] / v, 2),
            "atomics_per_s": round(c["TCC_ATOMIC_sum"] / t, 1),
            "source": "rocprofv3 counters of profiles/trace_kernel_von_hamos_1e8.md"}


def copy_reference(mib):
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n * 4} bytes", flush=True)


def _rows(d):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def _per_kernel(rows):
    """{(kernel, counter): [value per dispatch]}"""
    agg = collections.defaultdict(list)
    for r in rows:
        agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return agg


def _copy_kib(d, counter):
    vals = [v for (k, c), vs in _per_kernel(_rows(d)).items() if c == counter and "copyBuffer" in k
            for v in vs]
    return max(vals) if vals else None


def dispatch_stats(trace_dir, skip_first=1):
    """Per kernel, from the dispatch records of a rocprofv3 kernel trace:
    (calls kept, average, min, max duration in ns) after dropping each
    kernel's first `skip_first` dispatches (the warm-up launches, which run
    on a cold device and would bias the average)."""
    files = glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True)
    per = collections.defaultdict(list)
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                per[r["Kernel_Name"]].append((int(r["Start_Timestamp"]),
                                              int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = {}
    for k, v in per.items():
        v.sort()
        d = [x for _, x in v[skip_first:]] or [x for _, x in v]
        out[k] = (len(d), sum(d) / len(d), min(d), max(d), len(v))
    return out


def summarize(trace_dir, pmc_dirs, copy_fetch, copy_write, copy_mib, command, out_md, label,
              skip_first=1):
    lines = [f"# rocprofv3: {label}", "", "Commands (from /tmp on one MI355X, gfx950):", "", "```"]
    lines += command.strip().splitlines()
    lines += ["```", ""]
    # kernel trace statistics, without each kernel's warm-up dispatches
    stats = dispatch_stats(trace_dir, skip_first)
    if stats:
        lines += [f"Kernel trace (durations in microseconds; each kernel's first {skip_first} "
                  "dispatch(es), the warm-up, left out):", "",
                  "| kernel | dispatches | kept | average us | min us | max us |",
                  "|---|---|---|---|---|---|"]
        for k, (n, avg, lo, hi, total) in sorted(stats.items(), key=lambda kv: -kv[1][1] * kv[1][0]):
            lines.append(f"| `{k[:90]}` | {total} | {n} | {avg / 1e3:.1f} | {lo / 1e3:.1f} | "
                         f"{hi / 1e3:.1f} |")
        lines.append("")
    # counters
    agg = collections.defaultdict(list)
    for d in pmc_dirs:
        for k, v in _per_kernel(_rows(d)).items():
            agg[k] += v
    kernels = sorted({k for k, _ in agg if "trace_kernel" in k or "mwg_kernel" in k})
    counters = sorted({c for _, c in agg})
    if kernels:
        lines += ["Counters per dispatch (mean over dispatches of each trace kernel):", "",
                  "| counter | " + " | ".join(f"`{k[:60]}`" for k in kernels) + " |",
                  "|---|" + "---|" * len(kernels)]
        for c in counters:
            vals = [agg.get((k, c)) for k in kernels]
            lines.append(f"| {c} | " + " | ".join(f"{sum(v) / len(v):.4g}" if v else "-" for v in vals)
                         + " |")
        lines.append("")
    cf, cw = _copy_kib(copy_fetch, "FETCH_SIZE"), _copy_kib(copy_write, "WRITE_SIZE")
    traffic = {"sources_sha256": sources_sha256(), "kernels": {}}
    if cf and cw:
        ref_kib = copy_mib * 1024.0
        sf, sw = ref_kib / cf, ref_kib / cw
        lines += [f"Copy reference ({copy_mib} MiB read and written): FETCH_SIZE {cf:.0f} KiB, "
                  f"WRITE_SIZE {cw:.0f} KiB per dispatch, so the scale factors are {sf:.3f} (fetch) "
                  f"and {sw:.3f} (write).", ""]
        for k in kernels:
            f, w = agg.get((k, "FETCH_SIZE")), agg.get((k, "WRITE_SIZE"))
            if f and w:
                b = (sum(f) / len(f) * sf + sum(w) / len(w) * sw) * 1024.0
                traffic["kernels"][k] = {"fetch_kib": sum(f) / len(f), "write_kib": sum(w) / len(w),
                                         "fetch_scale": sf, "write_scale": sw,
                                         "hbm_bytes_per_launch": b}
                cs = {c: sum(agg[(k, c)]) / len(agg[(k, c)]) for c in ISSUE_COUNTERS
                      if agg.get((k, c))}
                if cs:
                    traffic["kernels"][k]["counters"] = cs
                lines.append(f"HBM traffic of `{k[:90]}`: {b / 1e6:.2f} MB per launch.")
        lines.append("")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines))
    return traffic


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=256)
    s = sub.add_parser("summarize")
    s.add_argument("--trace", required=True)
    s.add_argument("--pmc", nargs="*", default=[])
    s.add_argument("--copy-fetch", required=True)
    s.add_argument("--copy-write", required=True)
    s.add_argument("--copy-mib", type=int, default=256)
    s.add_argument("--command-file", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--label", required=True)
    s.add_argument("--traffic-json", default=None)
    s.add_argument("--skip-first", type=int, default=1,
                   help="warm-up dispatches of each kernel left out of its statistics")
    a = ap.parse_args()
    if a.cmd == "copy":
        copy_reference(a.mib)
        return
    with open(a.command_file) as fh:
        command = fh.read()
    t = summarize(a.trace, a.pmc, a.copy_fetch, a.copy_write, a.copy_mib, command, a.out, a.label,
                  a.skip_first)
    if a.traffic_json:
        with open(a.traffic_json, "w") as fh:
            json.dump(t, fh, indent=1)


if __name__ == "__main__":
    main()
