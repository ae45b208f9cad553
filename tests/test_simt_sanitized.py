"""The emulated serving loops with deferred detector work, built with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only: the device
code compiled for the CPU).  A sanitized library needs the ASan runtime
loaded first, so the check runs in a child Python process that preloads
it; any report ends that process with an error."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

DRIVER = r"""
import ctypes as C, sys
sys.path[:0] = [{tests!r}, {root!r}]
import test_simt_emulation as T
L = T.declare(C.CDLL({lib!r}))
# the FP32-mixed loops (the case whose device run failed), plain requests
# with ragged chunks and the extended requests
for ext, ragged in ((False, True), (True, False)):
    T.served_with_deferral(L, "fp32_mixed", ragged, ext, limit={limit})
    print("ok", ext, ragged, flush=True)
"""


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_deferred_serving_loop_under_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no ASan runtime")
    sys.path.insert(0, HERE)
    import test_simt_emulation as T
    lib = T.build_emu(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                 "-fno-omit-frame-pointer", "-g"])
    env = dict(os.environ, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:detect_stack_use_after_return=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = DRIVER.format(tests=HERE, root=ROOT, lib=str(lib), limit=6)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=1800)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.count("ok") == 2
