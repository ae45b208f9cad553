"""The library binds to the HIP runtime that torch loaded (one runtime per
process), whatever the import order of the caller."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_shares_torchs_hip_runtime():
    from paper_2503_16955_amd import mosaicrt
    if not os.path.exists(mosaicrt.LIB_PATH):
        pytest.skip("library not built")
    # a fresh interpreter that loads the library before anything imports torch
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2503_16955_amd import mosaicrt\n"
        "mosaicrt.load()\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "hip = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
        "print('\\n'.join(hip))\n" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    libs = [l for l in out.stdout.splitlines() if l.strip()]
    assert len(libs) == 1, libs
