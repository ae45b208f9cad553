"""mrt_trace_noalloc on the device, through the C-ABI: its images and
counters equal mrt_trace's bit for bit on two calls in a row, the second
with a smaller input (fewer rays, a smaller table), so that nothing of the
first call's scratch contents (counters, chunk cursor, tables) leaks into
the second.  Also for the FP64 and FP32-mixed stepping kernels without
tables and for the paper's event model, whose psi table sits in the same
scratch."""
import copy

import numpy as np
import pytest
import torch

from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("emitted", "missed", "absorbed", "exit_reflected", "exit_transmitted", "truncated",
          "detected", "events", "reflections", "records", "refined")


def _stress(nx, n_table):
    w = W.get("flat_stress")
    w["detector"] = dict(w["detector"], nx=nx, ny=nx, pitch=0.025 * 4096 / nx)
    if n_table:
        t, x0, x1 = W.darwin_prins_table(n=n_table)
        w["rocking_curve"].update(table=t.tolist(), x_min=x0, x_max=x1, peak=float(t.max()))
    return w


def _same(w, n, precision, first=0):
    print(f"[noalloc] {w['name']} {precision} n={n} first={first}", flush=True)
    ref = mrt.trace(w, n_rays=n, first=first, precision=precision)
    out = mrt.trace(w, n_rays=n, first=first, precision=precision, noalloc=True)
    for f in FIELDS:
        assert out["counters"][f] == ref["counters"][f], (f, out["counters"][f], ref["counters"][f])
    assert out["counters"]["kernel_ms"] == 0.0
    a = mrt.image_to_numpy(ref["counts"], ref["energy"])
    b = mrt.image_to_numpy(out["counts"], out["energy"])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert ref["counters"]["detected"] > 0


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_two_calls_second_smaller(precision):
    # the table curve and the 1024-bin spectrum in the scratch, then a
    # smaller table over them
    _same(_stress(2048, 0), 400_000, precision)
    _same(_stress(512, 700), 60_000, precision, first=123_456)


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_without_tables(precision):
    _same(W.get("von_hamos_hapg"), 2_000_000, precision)
    _same(W.get("flat_hopg"), 1000, precision)


def test_papers_model_psi_table():
    w = copy.deepcopy(W.get("von_hamos_hapg"))
    w["event_model"] = {"kind": "mwg", "burn_in": 200, "psi_nodes": 512}
    _same(w, 200_000, "fp64")
    w["event_model"] = {"kind": "mwg", "burn_in": 100, "psi_nodes": 64}
    _same(w, 30_000, "fp64")


def test_async_on_a_stream_without_counters():
    # calls without counters on one stream are ordered through the scratch
    w = W.get("flat_hopg")
    s = torch.cuda.Stream()
    refs = [mrt.trace(w, n_rays=50_000, first=k * 50_000) for k in range(3)]
    outs = []
    with torch.cuda.stream(s):
        for k in range(3):
            outs.append(mrt.trace(w, n_rays=50_000, first=k * 50_000, stream=s, sync=False,
                                  noalloc=True))
    s.synchronize()
    for r, o in zip(refs, outs):
        assert np.array_equal(mrt.image_to_numpy(r["counts"])[0], mrt.image_to_numpy(o["counts"])[0])
