"""The request server on the GPU: every request traced in a mix of
concurrently running requests (shared rounds of one persistent launch)
gives exactly the images and counters of the same request traced alone;
admission respects the memory budget in arrival order; cancellation and
release return memory."""
import copy
import math
import time

import numpy as np
import pytest

from paper_2503_16955_amd import mosaicrt as mrt
from paper_2503_16955_amd import workloads as W
from serving_mix import mix as _mix

pytestmark = pytest.mark.gpu

WAIT_MS = 60_000.0    # a request of these tests finishes in well under a second


def _alone(w, n, seed, precision):
    r = mrt.trace(w, n_rays=n, seed=seed, precision=precision)
    c, e = mrt.image_to_numpy(r["counts"], r["energy"])
    return c, e, r["counters"]


def _check_equal(res, w, n, seed, precision):
    assert res["state"] == "done", res["state"]
    c = res["counts"].cpu().numpy().view(np.uint32)
    e = res["energy"].cpu().numpy().view(np.uint64)
    ac, ae, acnt = _alone(w, n, seed, precision)
    assert np.array_equal(c, ac) and np.array_equal(e, ae)
    for f in ("emitted", "missed", "absorbed", "exit_reflected", "exit_transmitted", "truncated",
              "detected", "events", "reflections", "refined"):
        assert res["counters"][f] == acnt[f], f


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_mix_equals_alone(precision):
    reqs = _mix()
    with mrt.Server(hbm_budget_bytes=1 << 30, max_slots=16, precision=precision,
                    round_rays=1 << 19, chunk=2048) as srv:
        tickets = [srv.submit(w, n_rays=n, seed=s) for w, n, s in reqs]
        results = []
        for t, (w, n, _) in zip(tickets, reqs):
            results.append(srv.wait(t, timeout_ms=WAIT_MS))
            print(f"[serve] {precision} ticket {t} {w['name']} n={n} done", flush=True)
        st = srv.stats()
        assert st["rounds"] > 3            # the requests shared several rounds
        assert st["rays_traced"] == sum(n for _, n, _ in reqs)
        for (w, n, s), r in zip(reqs, results):
            print(f"[serve] {precision} {w['name']} n={n} rounds={st['rounds']}", flush=True)
            _check_equal(r, w, n, s, precision)
        for t in tickets:
            srv.release(t)
        assert srv.stats()["used_bytes"] == 0


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_design_requests_served_equal_alone(precision):
    """The benchmark's own spectrometer-design requests (varied radius,
    mosaic kind and width, thickness and energy window, each with its own
    seed), the first 48 with their ray counts scaled by 1/100 (1e3-1e6,
    ragged): served together through 16 slots, each equals its one-call
    trace bit for bit."""
    reqs = [(w, max(1, w["n_rays"] // 100), w["seed"]) for w in W.serving_requests()[:48]]
    with mrt.Server(hbm_budget_bytes=1 << 30, max_slots=16, precision=precision,
                    round_rays=1 << 20) as srv:
        tickets = [srv.submit(w, n_rays=n, seed=s) for w, n, s in reqs]
        results = [srv.wait(t, timeout_ms=WAIT_MS) for t in tickets]
        st = srv.stats()
        print(f"[serve-design] {precision}: {len(reqs)} requests, "
              f"{sum(n for _, n, _ in reqs)} rays, {st['rounds']} rounds", flush=True)
        assert st["rounds"] > 3
        for (w, n, s), r in zip(reqs, results):
            _check_equal(r, w, n, s, precision)
        for t in tickets:
            srv.release(t)
        assert srv.stats()["used_bytes"] == 0


def test_budget_admission_in_arrival_order():
    w = W.get("von_hamos_hapg")
    per = 2048 * 512 * 12
    with mrt.Server(hbm_budget_bytes=2 * per + 1000, max_slots=8, precision="fp32_mixed",
                    round_rays=1 << 20) as srv:
        tickets = [srv.submit(w, n_rays=1_000_000 + i, seed=10 + i) for i in range(6)]
        done = []
        # release each request as soon as it is done, so the next ones fit
        pending = list(tickets)
        while pending:
            t = pending.pop(0)
            r = srv.wait(t, timeout_ms=WAIT_MS)
            done.append(r)
            _check_equal(r, w, 1_000_000 + tickets.index(t), 10 + tickets.index(t), "fp32_mixed")
            srv.release(t)
        admits = [r["admit_ms"] for r in done]
        assert admits == sorted(admits)
        # at most two requests' images fit: the third waited for a release
        assert done[2]["admit_ms"] >= min(done[0]["done_ms"], done[1]["done_ms"])


def test_oversized_request_is_rejected():
    w = W.get("flat_stress")                # 4096^2 images: 192 MiB
    with mrt.Server(hbm_budget_bytes=64 << 20, max_slots=4) as srv:
        with pytest.raises(mrt.MosaicRTError) as e:
            srv.submit(w, n_rays=1000)
        assert e.value.status == mrt.ENOMEM


def test_cancel_and_release():
    w = W.get("von_hamos_hapg")
    with mrt.Server(hbm_budget_bytes=1 << 30, max_slots=4, precision="fp32_mixed",
                    round_rays=1 << 20) as srv:
        big = srv.submit(w, n_rays=2_000_000_000)
        small = srv.submit(w, n_rays=100_000, seed=7)
        time.sleep(0.05)
        srv.cancel(big)
        r = srv.wait(big, timeout_ms=WAIT_MS)
        assert r["state"] == "canceled" and 0 < r["rays_done"] < 2_000_000_000
        _check_equal(srv.wait(small, timeout_ms=WAIT_MS), w, 100_000, 7, "fp32_mixed")
        srv.release(big)
        srv.release(small)
        assert srv.stats()["used_bytes"] == 0
        with pytest.raises(mrt.MosaicRTError):
            srv.release(big)


def test_poisson_arrivals_latency_recorded():
    """Requests arrive while others run; a consumer takes each from the
    completion queue as it finishes and releases it."""
    reqs = W.serving_requests(n=24, seed=4)
    rng = np.random.default_rng(5)
    with mrt.Server(hbm_budget_bytes=1 << 30, max_slots=16, precision="fp32_mixed") as srv:
        tickets = set()
        for w in reqs:
            w = copy.deepcopy(w)
            w["n_rays"] = min(w["n_rays"], 2_000_000)
            time.sleep(rng.exponential(0.002))
            tickets.add(srv.submit(w))
        lat, order = [], []
        for _ in reqs:
            t, r = srv.wait_any(timeout_ms=WAIT_MS, views=False)
            assert r["state"] == "done" and t in tickets
            lat.append(r["done_ms"] - r["submit_ms"])
            order.append(r["done_ms"])
            srv.release(t)
        assert order == sorted(order)
        assert all(x > 0 for x in lat)
        assert srv.stats()["used_bytes"] == 0
        print(f"[serve] p50 {np.percentile(lat, 50):.2f} ms p99 {np.percentile(lat, 99):.2f} ms",
              flush=True)


def _served_extended_mix():
    """Plain requests among requests with a Gaussian spot, an energy-dependent
    curve, further planes and user polarisations (with user energies)."""
    import torch
    vh = W.get("von_hamos_hapg")
    spot = W.with_spot(vh)
    dep = copy.deepcopy(vh)
    dep["rocking_curve"]["energy_dependence"] = [(7.8, -30e-6, 0.6), (8.05, 20e-6, 1.5),
                                                 (8.2, 45e-6, 2.2)]
    planes = copy.deepcopy(vh)
    planes["source"]["lines"] = list(planes["source"]["lines"]) + [(2 * 8.048, 0.004, 0.4)]
    planes["crystal"]["planes"] = {"hbar_ratio": 0.5,
                                   "extra": [(vh["crystal"]["two_d"] / 2, 0.6, 1.5, 5e-6)]}
    n_pol = 300_000
    import oracle
    _, k, _ = oracle.source_sample(vh, np.arange(n_pol))
    a = np.random.default_rng(21).normal(size=k.shape)
    a -= np.sum(a * k, axis=1)[:, None] * k
    pol = torch.as_tensor(a / np.linalg.norm(a, axis=1)[:, None], device="cuda").contiguous()
    en = torch.as_tensor(np.random.default_rng(22).uniform(7.95, 8.15, n_pol), device="cuda")
    torch.cuda.synchronize()
    return [(vh, 700_000, 3, None), (spot, 900_000, 4, None), (dep, 500_000, 5, None),
            (W.get("flat_hopg"), 400_000, 6, None), (planes, 800_000, 7, None),
            (vh, n_pol, 8, {"polarisations": pol, "energies": en}), (spot, 1_100_000, 9, None)]


@pytest.mark.parametrize("precision", ["fp32_mixed", "fp64"])
def test_extended_inputs_served_equal_alone(precision):
    """Requests with extended inputs run in the same rounds as plain ones
    (one launch per group and round).  Each gives exactly the images and
    counters of the same request traced alone, in both precisions: the
    serving and one-call kernels are separate compilations of the same
    loop, and with multiply-adds fused only inside a source expression they
    round every FP32 operation alike."""
    reqs = _served_extended_mix()
    fields = ("emitted", "missed", "absorbed", "exit_reflected", "exit_transmitted",
              "truncated", "detected", "events", "reflections", "refined")
    with mrt.Server(hbm_budget_bytes=1 << 30, max_slots=16, precision=precision,
                    round_rays=1 << 18, chunk=2048) as srv:
        tickets = [srv.submit(w, n_rays=n, seed=s, rays=r) for w, n, s, r in reqs]
        results = [srv.wait(t, timeout_ms=WAIT_MS) for t in tickets]
        st = srv.stats()
        assert st["rounds"] > 3 and st["rays_traced"] == sum(n for _, n, _, _ in reqs)
        for (w, n, s, rays), res in zip(reqs, results):
            assert res["state"] == "done", res["state"]
            alone = mrt.trace(w, n_rays=n, seed=s, precision=precision, rays=rays)
            ac, ae = mrt.image_to_numpy(alone["counts"], alone["energy"])
            c = res["counts"].cpu().numpy().view(np.uint32)
            e = res["energy"].cpu().numpy().view(np.uint64)
            n_px = int(np.sum((c != ac) | (e != ae)))
            print(f"[serve-ext] {precision} {w['name']} n={n} rays={bool(rays)} "
                  f"pixels apart {n_px}", flush=True)
            assert n_px == 0
            for f in fields:
                assert res["counters"][f] == alone["counters"][f], (f, res["counters"][f],
                                                                    alone["counters"][f])
            assert alone["counters"]["reflections"] > 100
        for t in tickets:
            srv.release(t)
        assert srv.stats()["used_bytes"] == 0
