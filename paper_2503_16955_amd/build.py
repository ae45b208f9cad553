"""Builds libmosaicrt.so (HIP for gfx950) in-tree.  The trace-kernel instance
translation units compile in parallel."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmosaicrt.so")
# VALU issue-rate microbenchmark behind the roofline's slot weights (a
# program of its own, run by the profiling scripts)
RATES_EXE = os.path.join(HERE, "valu_rates")
SOURCES = ["trace_f64_flat.hip", "trace_f64_cyl.hip", "trace_f32_flat.hip", "trace_f32_cyl.hip",
           "trace_ext_f64_flat.hip", "trace_ext_f64_cyl.hip", "trace_ext_f32_flat.hip",
           "trace_ext_f32_cyl.hip", "trace_mwg.hip", "serve_f64.hip", "serve_f32.hip", "launch.hip",
           "params.cpp", "runtime.cpp", "server.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # multiply-adds fuse only within one source expression, never
         # across statements: every kernel instance that inlines the same
         # code then rounds it the same way, so FP32-mixed results do not
         # depend on which instance (one-call, extended, serving) traced them
         "-ffp-contract=on",
         # no packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # keep loop-invariant constants out of registers: hoisting them out
         # of the persistent ray loop costs ~100 VGPRs and halves occupancy,
         # and the trace kernels are latency-bound at two waves per SIMD
         "-mllvm", "-disable-machine-licm",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src, extra_flags, verbose):
    obj = os.path.join(CSRC, src.rsplit(".", 1)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra_flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose=False, extra_flags=(), jobs=None):
    jobs = jobs or min(len(SOURCES), max(1, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra_flags, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    build_rates(verbose)
    return LIB


def build_rates(verbose=False):
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(CSRC, "valu_rates.hip"), "-o", RATES_EXE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(RATES_EXE + ".tmp", RATES_EXE)
    return RATES_EXE


if __name__ == "__main__":
    print(build(verbose=True, extra_flags=sys.argv[1:]))
