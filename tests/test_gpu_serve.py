"""Served form: continuous batching under the HBM budget.  Every request's
result must be the same alone and in the mix (normwise 1e-5), and the
scheduler must actually mix (groups of several requests, overlapping groups)."""
import numpy as np
import pytest
import torch

from paper_2304_01841_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_01841_amd import serve, wcsim
    return serve, wcsim


def normwise(got, ref):
    ref = np.asarray(ref, np.float64)
    return np.abs(np.asarray(got, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-300)


def _requests(n, seed=11, nticks=1500):
    reqs = W.serve_requests(seed=seed, nreq=n, lo=3.0, hi=4.3, nticks=nticks)
    for r in reqs:  # keep the test small: at most 300 wires per plane
        for pl in r["planes"]:
            pl["nwires"] = min(pl["nwires"], 300)
        rng = np.random.default_rng(r["event_id"])
        box = (W.BOX_X * nticks / 6000.0, W.BOX_Y, max(p["nwires"] for p in r["planes"]) * W.PITCH)
        r["depos"] = W.clipped_track_depos(rng, r["depos"].shape[0], box)
    return reqs


def _alone(wcsim, server, r):
    outs = []
    for d, R in zip(r["planes"], r["responses"]):
        p = server.plane(d, R)
        outs.append(wcsim.simulate_event(p, torch.from_numpy(r["depos"]).cuda(),
                                         r["event_id"]).cpu().numpy())
    return outs


def test_serve_mix_equals_alone(mods):
    serve, wcsim = mods
    print("case: serve mix", flush=True)
    reqs = _requests(24)
    srv = serve.Server(W.physics(True), slots=3, max_batch=6)
    arr = W.poisson_arrivals(3, len(reqs), qps=4000.0)
    res = srv.serve(reqs, arr)
    assert all(r.error is None for r in res)
    assert srv.stats["max_group"] >= 2
    assert srv.stats["max_inflight_groups"] >= 2
    for r, q in zip(res, reqs):
        alone = _alone(wcsim, srv, q)
        assert len(r.outputs) == len(alone)
        for got, ref in zip(r.outputs, alone):
            assert normwise(got, ref) <= 1e-5
    s = serve.latency_summary(res)
    assert s["requests"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0


def test_serve_budget_serialises_and_rejects(mods):
    serve, wcsim = mods
    print("case: serve budget", flush=True)
    reqs = _requests(6, seed=21)
    probe = serve.Server(W.physics(True))
    need = [probe.request_bytes([probe.plane(d, R) for d, R in zip(q["planes"], q["responses"])],
                                q["depos"].shape[0]) for q in reqs]
    # a budget below any two requests together: admission serialises, and
    # requests larger than the budget are rejected instead of run
    two = sorted(need)
    budget = two[0] + two[1] - 1
    srv = serve.Server(W.physics(True), hbm_budget=budget, slots=4, max_batch=4)
    res = srv.serve(reqs)
    assert srv.stats["max_group"] == 1
    assert srv.stats["max_inflight_groups"] == 1
    assert srv.stats["max_inflight_bytes"] <= budget
    for r, q, nb in zip(res, reqs, need):
        if nb > budget:
            assert r.error is not None and not r.outputs
            continue
        assert r.error is None
        for got, ref in zip(r.outputs, _alone(wcsim, srv, q)):
            assert normwise(got, ref) <= 1e-5
    # a request larger than the whole budget is rejected, not run
    tiny = serve.Server(W.physics(True), hbm_budget=min(need) // 2)
    res = tiny.serve(reqs[:2])
    assert all(r.error is not None for r in res)


def test_serve_isolates_invalid_requests_and_cancellations(mods):
    """Failure injection: a request with a non-finite depo, one with a depo
    behind its plane and one over the budget fail alone; a request cancelled
    while queued and one cancelled while its group runs return no output; all
    other requests equal their results alone."""
    serve, wcsim = mods
    print("case: serve failure injection", flush=True)
    reqs = _requests(10, seed=21)
    reqs[2]["depos"] = reqs[2]["depos"].copy()
    reqs[2]["depos"][5, 1] = np.nan
    reqs[6]["depos"] = reqs[6]["depos"].copy()
    reqs[6]["depos"][0, 0] = -10.0
    big = _requests(1, seed=5)[0]
    rng = np.random.default_rng(3)
    big["depos"] = W.clipped_track_depos(rng, 400_000, (W.BOX_X / 4, W.BOX_Y, 1500.0))
    big["event_id"] = 99
    reqs = [big] + reqs
    srv = serve.Server(W.physics(True), slots=1, max_batch=1, depth=1)
    # request 0 (large) runs first and is cancelled 1 ms in, while it runs;
    # request 4 is cancelled while still queued behind it
    res = srv.serve(reqs, None, cancel_at={0: 1e-3, 4: 0.0})
    assert res[3].error is not None and "non-finite" in res[3].error
    assert res[7].error is not None and "behind" in res[7].error
    assert res[0].error == "cancelled" and not res[0].outputs
    assert res[4].error == "cancelled" and not res[4].outputs
    for k in (1, 2, 5, 6, 8, 9, 10):
        assert res[k].error is None
        for got, ref in zip(res[k].outputs, _alone(wcsim, srv, reqs[k])):
            assert normwise(got, ref) <= 1e-5


def test_serve_plain_baseline_matches(mods):
    """The per-request baseline on the same stream gives the same results."""
    serve, wcsim = mods
    print("case: serve plain baseline", flush=True)
    reqs = _requests(6, seed=31)
    srv = serve.Server(W.physics(True), slots=2, max_batch=4)
    res = srv.serve_plain(reqs)
    for r, q in zip(res, reqs):
        assert r.error is None
        for got, ref in zip(r.outputs, _alone(wcsim, srv, q)):
            assert normwise(got, ref) <= 1e-5


def test_served_requests_against_oracle(mods):
    """Three requests of the serving workload's own mix (one of three planes),
    served inside the whole 64-request mix: sampled wire waveforms of every
    plane against the oracle.  For each sampled wire (the two strongest, two
    at random) the oracle takes every depo whose window can reach that wire's
    response reach (a superset by mean pitch bin), keyed by its index in the
    request, and evaluates the defining convolution sum at every 7th tick."""
    from oracle import oracle as O

    serve, wcsim = mods
    print("case: served requests against the oracle", flush=True)
    reqs = W.serve_requests(nreq=64)
    phys = W.physics(True)
    srv = serve.Server(phys, slots=4, max_batch=8)
    res = srv.serve(reqs)
    assert all(r.error is None for r in res)
    sizes = [r["depos"].shape[0] for r in reqs]
    three = [k for k, r in enumerate(reqs) if len(r["planes"]) == 3 and sizes[k] < 600_000]
    others = [k for k, r in enumerate(reqs) if len(r["planes"]) < 3 and sizes[k] < 600_000]
    picks = [max(three, key=lambda k: sizes[k])] + sorted(others, key=lambda k: -sizes[k])[:2]
    rng = np.random.default_rng(41)
    for k in picks:
        r = reqs[k]
        dep = r["depos"]
        print("  request %d: %d planes, %d depos" % (k, len(r["planes"]), dep.shape[0]),
              flush=True)
        for pl, R, out in zip(r["planes"], r["responses"], res[k].outputs):
            Rp, r0, nimp = R.shape[0], R.shape[0] // 2, pl["nimpact"]
            dp = pl["pitch"] / nimp
            mu = ((dep[:, 1] * pl["dir_y"] + dep[:, 2] * pl["dir_z"]) - pl["pitch_origin"]) / dp
            scale = np.abs(out).max()
            assert scale > 0
            wires = list(np.argsort(-np.abs(out).max(axis=1))[:2])
            wires += list(rng.integers(0, pl["nwires"], 2))
            ticks = np.arange(0, pl["nticks"], 7)
            for wi in wires:
                p = int(wi) * nimp + nimp // 2
                lo, hi = p + r0 - (Rp - 1), p + r0
                idx = np.nonzero((mu >= lo - 40) & (mu <= hi + 40))[0]
                G = O.grid(dep[idx], phys, pl, r["event_id"], ids=idx)
                pts = np.stack([np.full(ticks.shape, p), ticks], axis=1)
                ref = O.convolve_points(G, R.astype(np.float64), r0, pts)
                assert np.abs(out[int(wi), ticks] - ref).max() / scale <= 1e-4, (k, int(wi))
