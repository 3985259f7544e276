"""Continuous-batching server (tc_server_*): requests from pads of different
sizes arrive while others run, join the running batch between its ticks
(a Newton iteration in lockstep, a round of the staged schedule), and give
the same result as the same step run alone (bitwise:
the per-pad arithmetic does not depend on the batch).  Admission by HBM
footprint: with a budget that holds only a few pads' step scratch, every
request still completes, with the same results."""
from __future__ import annotations

import time

import numpy as np
import pytest

from gpu_util import gpu_pad, log, tc
from workloads import scenes

pytestmark = pytest.mark.gpu

MM = scenes.MM
N_STEPS = 4


def _episodes():
    rng = np.random.default_rng(11)
    eps = [scenes.config1()]
    shapes = [scenes.SPHERE, scenes.TEXTURE, scenes.TORUS, scenes.BOX, scenes.CYLINDER, scenes.SPHERE, scenes.TEXTURE]
    dims = [(7, 5, 3), (12, 10, 4), (16, 12, 4), (9, 8, 3), (20, 16, 5), (10, 10, 3), (14, 11, 3)]
    for shape, (nx, ny, nz) in zip(shapes, dims):
        p = scenes.box_pad(0.018, 0.014, 0.004, nx, ny, nz) if nz != 3 else \
            scenes.dome_pad(0.019, 0.016, 0.003, nx, ny, nz)
        ind = scenes.place_indenter(p, shape, (0.5 * p.dims[0], 0.45 * p.dims[1]), 1e-4, sphere_radius=3 * MM)
        eps.append(scenes.Episode(p, ind, float(rng.uniform(0.2, 0.6)) * MM, N_STEPS, scenes.Params()))
    return eps


def _alone(eps):
    ctx = tc.Context(0)
    out = []
    for e in eps:
        g = gpu_pad(ctx, e.pad, "mixed")
        st = [g.step([e.pose(s)]) for s in range(1, N_STEPS + 1)]
        out.append((g.read("positions"), g.read("sigma"), [(x.newton_iters, x.cg_iters) for x in st]))
        g.close()
    ctx.close()
    return out


def _served(eps, budget=0, max_slots=4, staged=True):
    ctx = tc.Context(0, hbm_budget=budget)
    ctx.set_schedule(staged)
    pads = [gpu_pad(ctx, e.pad, "mixed") for e in eps]
    srv = tc.Server(ctx, max_slots)
    order = [(k, s) for s in range(1, N_STEPS + 1) for k in range(len(eps))]
    rng = np.random.default_rng(5)
    results = []
    i = 0
    while i < len(order):
        # bursts of 1-4 requests, each pad's steps in order
        burst = int(rng.integers(1, 5))
        for k, s in order[i:i + burst]:
            srv.submit(pads[k], [eps[k].pose(s)], tag=k * 100 + s)
        i += burst
        time.sleep(float(rng.uniform(0.0, 0.004)))
        results += srv.poll()
    t0 = time.perf_counter()
    while len(results) < len(order):
        results += srv.poll(wait_us=2000)
        assert time.perf_counter() - t0 < 60, "server did not finish"
    stats = srv.stats()
    srv.close()
    final = [(g.read("positions"), g.read("sigma")) for g in pads]
    for g in pads:
        g.close()
    ctx.close()
    return results, final, stats


def _check(eps, alone, results, final, stats, label):
    assert all(r["status"] == 0 for r in results), [r for r in results if r["status"]]
    for r in results:
        assert r["t_arrive_ms"] <= r["t_admit_ms"] <= r["t_done_ms"]
        k, s = divmod(r["tag"], 100)
        assert (r["stats"].newton_iters, r["stats"].cg_iters) == alone[k][2][s - 1], (label, k, s)
    for k, ((xa, sa, _), (xb, sb)) in enumerate(zip(alone, final)):
        assert np.array_equal(xa, xb) and np.array_equal(sa, sb), (label, k)
    lat = np.array([r["t_done_ms"] - r["t_arrive_ms"] for r in results])
    log(f"{label}: {len(results)} requests, max running {stats['max_running_seen']}, batched iterations "
        f"{stats['ticks']}, latency p50 {np.percentile(lat, 50):.1f} ms p99 {np.percentile(lat, 99):.1f} ms")


@pytest.mark.parametrize("staged", [True, False])
def test_server_results_equal_alone_bitwise(staged):
    eps = _episodes()
    alone = _alone(eps)
    results, final, stats = _served(eps, staged=staged)
    _check(eps, alone, results, final, stats, "server, " + ("staged" if staged else "lockstep"))
    assert stats["max_running_seen"] > 1      # requests did overlap on the device


def test_server_admission_by_memory_budget():
    eps = _episodes()
    alone = _alone(eps)
    # probe the pads' footprints, then allow the resident data plus room for
    # the step scratch of about two of the largest pads
    ctx = tc.Context(0)
    pads = [gpu_pad(ctx, e.pad, "mixed") for e in eps]
    resident = sum(g.info["resident_bytes"] for g in pads)
    scratch = max(g.info["scratch_bytes"] for g in pads)
    ctx.close()
    budget = resident + int(2.2 * scratch) + (8 << 20)
    results, final, stats = _served(eps, budget=budget, max_slots=6)
    _check(eps, alone, results, final, stats, f"server, budget {budget / 2**20:.1f} MiB")


def test_server_evicts_idle_scratch():
    """A pad that has finished its requests keeps its step scratch until
    memory is needed: with room for about one large pad's scratch, requests
    of the other pads arriving afterwards still complete (the idle scratch
    is released), with the same results as alone."""
    eps = _episodes()
    alone = _alone(eps)
    ctx = tc.Context(0)
    probe = [gpu_pad(ctx, e.pad, "mixed") for e in eps]
    resident = sum(g.info["resident_bytes"] for g in probe)
    scratch = max(g.info["scratch_bytes"] for g in probe)
    total = sum(g.info["scratch_bytes"] for g in probe)
    ctx.close()
    room = int(1.3 * scratch) + (1 << 20)      # 1 MiB for plans and state slots
    assert total > room + (1 << 20)            # not every pad's scratch fits at once
    budget = resident + room
    ctx = tc.Context(0, hbm_budget=budget)
    pads = [gpu_pad(ctx, e.pad, "mixed") for e in eps]
    srv = tc.Server(ctx, 4)
    results = []
    big = max(range(len(eps)), key=lambda k: pads[k].info["scratch_bytes"])
    order = [big] + [k for k in range(len(eps)) if k != big]
    t0 = time.perf_counter()
    for k in order:
        # one pad at a time: each finishes (and idles, holding its scratch)
        # before the next pad's requests arrive
        for s in range(1, N_STEPS + 1):
            srv.submit(pads[k], [eps[k].pose(s)], tag=k * 100 + s)
        while sum(1 for r in results if r["tag"] // 100 == k) < N_STEPS:
            results += srv.poll(wait_us=2000)
            assert time.perf_counter() - t0 < 60, "server did not finish"
    stats = srv.stats()
    srv.close()
    final = [(g.read("positions"), g.read("sigma")) for g in pads]
    ctx.close()
    _check(eps, alone, results, final, stats, f"server, budget {budget / 2**20:.1f} MiB, one pad at a time")
    assert stats["evictions"] > 0


def test_server_plan_rebuilt_after_pad_recreated():
    """A pad destroyed between two requests of a live server and a new pad
    created in its place (on the host often at the same address, with the
    same arena scratch): the server must not replay the old pad's batch
    plan.  The new pad's steps equal the same steps run alone, bitwise."""
    eps = _episodes()
    a, b = eps[1], eps[3]
    alone_b = _alone([b])[0]
    ctx = tc.Context(0)
    srv = tc.Server(ctx, 2)

    def serve(g, ep, steps):
        out = []
        for s in steps:
            srv.submit(g, [ep.pose(s)], tag=s)
            t0 = time.perf_counter()
            while not out or out[-1]["tag"] != s:
                out += srv.poll(wait_us=2000)
                assert time.perf_counter() - t0 < 60, "server did not finish"
        return out

    ga = gpu_pad(ctx, a.pad, "mixed")
    assert all(r["status"] == 0 for r in serve(ga, a, [1, 2]))
    ga.close()
    gb = gpu_pad(ctx, b.pad, "mixed")
    res = serve(gb, b, range(1, N_STEPS + 1))
    assert [(r["stats"].newton_iters, r["stats"].cg_iters) for r in res] == alone_b[2]
    assert np.array_equal(gb.read("positions"), alone_b[0]) and np.array_equal(gb.read("sigma"), alone_b[1])
    log(f"recreated pad: {len(res)} requests equal the pad alone")
    srv.close()
    gb.close()
    ctx.close()
